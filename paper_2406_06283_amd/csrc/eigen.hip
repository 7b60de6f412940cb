// Local H_k-GenEO eigenproblems (Def. 2.14) on the GPU, batched over subdomains.
//
// The pencil (B~, X D~ X) on ovdof(D) has |Gamma| infinite eigenvalues (its right-hand side vanishes
// on Gamma); the finite ones are those of the symmetric-definite pencil S p = lambda C_II p with
// S = B_II - B_IG B~_GG^{-1} B_GI (Lemma 2.6 gives real eigenvalues and C-orthonormal vectors).  The
// host driver forms S and the factor C_II = L L^T; the kernels here take the standard symmetric
// matrix L^{-1} S L^{-T} through:
//   1. Householder reduction to tridiagonal form T = Q^T (L^{-1} S L^{-T}) Q,
//   2. Sturm-sequence counts on T: the number of eigenvalues below tau / below 0 and bisection for
//      the smallest ones, with the selection of Def. 2.15 (lambda_{m+1} > 0, clusters kept whole),
//   3. inverse iteration on T for the selected eigenvalues (re-orthogonalised inside clusters),
//   4. back-transformation by Q (and by L^{-T} on the host side), the sign convention (largest
//      entry positive), and the partition-of-unity scaling X that gives the coarse basis
//      Z_i = X_I P_i (Def. 2.15),
// and finally the blocks of the coarse matrix B_0 = Z^T B Z (eq. (2.23)).
#include "internal.hpp"
#include "kernels.hpp"
#include "tile.hpp"
#include "wave.hpp"

namespace hkg {

// sum over the 64 lanes of a wave (all lanes active); every lane gets the result
__device__ __forceinline__ double wave_sum(double v) { return wave_sum64(v); }

// block-wide sum; every thread gets the result. red must hold one double per wave.
__device__ __forceinline__ double block_sum(double v, double *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += red[i];
    return t;
}

// ------------------------------------------------------------------------------------------------
// 1. Blocked Householder tridiagonalisation of the symmetric nI x nI matrix T of each subdomain,
//    stored at offM with the padded leading dimension ldM (every column starts on a 256-byte
//    boundary; with V and W in LDS only the lower triangle is kept up to date, otherwise both).  Reflector j is stored in column j below the diagonal
//    (its first entry, 1, explicitly), with tau[j]; d and e receive the diagonal and sub-diagonal.
//    Within a panel of SY_NB columns starting at j0 the
//     trailing matrix A0 is left as it was at the panel start; with V (reflectors) and W (their
//     images) of the panel's earlier columns the current matrix is A0 - V W^T - W V^T, so column j
//     is corrected before its reflector is formed and the product A v needs only one pass over A0
//     plus corrections with V and W.  After the panel one rank-2 SY_NB update (a batched GEMM over
//     many blocks) brings the trailing matrix up to date.  Per subdomain the workspace VWV holds
//     [V | W | V] (n x 3 SY_NB, column-major), so that the update is one GEMM with K = 2 SY_NB.
// ------------------------------------------------------------------------------------------------
constexpr int SY_NB = 32;           // panel width when V and W stay in global memory
constexpr int SY_NB_LDS = 16;       // panel width when V and W of the panel fit in LDS
constexpr int SY_THREADS = 1024;
constexpr int SY_RT = 256;          // row-pair threads of the product A0 v
constexpr int SY_G = SY_THREADS / SY_RT;   // column groups of the product

// part[g (n + 1) + r] = sum over the columns c = j + 1 + g (mod SY_G) of A0[r][c] v[c], rows j+1..n-1:
// row pairs (16-byte loads: ld and the pair's first row are even) times SY_G column groups, eight
// column loads in flight per thread (indices clamped into range, the surplus terms masked), summed in
// column order
__device__ __forceinline__ void sytrd_product_parts(const double *__restrict__ A, int ld, int n, int j,
                                                    const double *v, double *part, int tid) {
    const int rt = tid & (SY_RT - 1), g = tid / SY_RT;
    const int rp0 = (j + 1) & ~1;
    for (int r = rp0 + 2 * rt; r < n; r += 2 * SY_RT) {
        double s0 = 0.0, s1 = 0.0;
        for (int c0 = j + 1 + g; c0 < n; c0 += 8 * SY_G) {
            double2 a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                a[u] = *reinterpret_cast<const double2 *>(A + r + (int64_t)min(c0 + SY_G * u, n - 1) * ld);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const double vc = c0 + SY_G * u < n ? v[min(c0 + SY_G * u, n - 1)] : 0.0;
                s0 = fma(a[u].x, vc, s0);
                s1 = fma(a[u].y, vc, s1);
            }
        }
        part[g * (n + 1) + r] = s0;
        part[g * (n + 1) + r + 1] = s1;
    }
}

// block-wide sum with a single barrier; `red` holds one slot per wave.  The slots may be written
// again only after a later barrier that every reader of this call has passed, so callers alternate
// between two slot sets with other barriers between their uses.
__device__ __forceinline__ double block_sum_once(double v, double *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += red[i];
    return t;
}

// NB: panel width; V and W of the panel in the global workspace
template <int NB>
__global__ __launch_bounds__(SY_THREADS) void k_sytrd_panel(const SubDev *__restrict__ subs, double *__restrict__ Sq,
                                                            double *__restrict__ VWVb, double *__restrict__ dout,
                                                            double *__restrict__ eout, double *__restrict__ tout,
                                                            int j0) {
    extern __shared__ double sh[];
    const SubDev sd = subs[blockIdx.x];
    const int n = sd.nI;
    double *A = Sq + sd.offM;
    const int ld = sd.ldM;
    double *d = dout + sd.offI, *e = eout + sd.offI, *tau = tout + sd.offI;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (j0 >= n - 1) return;
    const int jb = min(NB, n - 1 - j0);
    double *Vg = VWVb + 3 * NB * sd.offI;      // n x 3 NB per subdomain (offI runs over sum n_I)
    double *v = sh;                  // n
    double *p = sh + n;              // n (first the corrected column, then A v)
    double *part = sh + 2 * n;       // SY_G (n + 1): partial products per column group
    double *t12 = part + SY_G * (n + 1);   // 2 NB
    double *vw = t12 + 2 * NB;       // 2 NB: W[j, :], V[j, :]
    double *red = vw + 2 * NB;       // 32
    double *V = Vg;                  // V and W of the panel (column q at q n)
    double *W = V + (int64_t)NB * n;
    double *V2 = Vg + (int64_t)2 * NB * n;
    double dmine = 0.0, emine = 0.0, tmine = 0.0;   // column tid's d, e, tau (tid < jb)
    // zero the panel's columns of V, W (and V2 in global memory; rows not written stay zero)
    for (int64_t q = tid; q < (int64_t)3 * NB * n; q += SY_THREADS) V[q] = 0.0;
    __syncthreads();
    for (int kk = 0; kk < jb; ++kk) {
        const int j = j0 + kk;
        const int L = n - j - 1;
        // W[j, q], V[j, q] for q < kk
        if (tid < kk) vw[tid] = W[j + (int64_t)tid * n];
        else if (tid >= 64 && tid - 64 < kk) vw[NB + tid - 64] = V[j + (int64_t)(tid - 64) * n];
        __syncthreads();
        // 1. corrected column j, rows j..n-1
        for (int r = j + tid; r < n; r += SY_THREADS) {
            double s = A[r + (int64_t)j * ld];
            for (int q0 = 0; q0 < kk; q0 += 8) {
                double a[8], b[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int q = min(q0 + u, kk - 1);
                    a[u] = V[r + (int64_t)q * n];
                    b[u] = W[r + (int64_t)q * n];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (q0 + u < kk) s -= a[u] * vw[q0 + u] + b[u] * vw[NB + q0 + u];
            }
            p[r] = s;
        }
        __syncthreads();
        // 2. reflector from x = p[j+1 .. n-1]
        const double alpha = p[j + 1];
        double acc = 0.0;
        for (int r = j + 2 + tid; r < n; r += SY_THREADS) acc += p[r] * p[r];
        const double xn2 = block_sum(acc, red);
        double t = 0.0, beta = alpha, scal = 0.0;
        if (xn2 != 0.0) {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            t = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        for (int r = j + 1 + tid; r < n; r += SY_THREADS) {
            const double vr = (r == j + 1) ? 1.0 : (xn2 != 0.0 ? p[r] * scal : 0.0);
            v[r] = vr;
            A[r + (int64_t)j * ld] = vr;
            V[r + (int64_t)kk * n] = vr;
            V2[r + (int64_t)kk * n] = vr;
        }
        if (tid == kk) {            // stored after the panel (a store per column stalls its wave)
            dmine = p[j];
            emine = beta;
            tmine = t;
        }
        __syncthreads();
        if (t == 0.0) continue;          // H_j = I: W column stays zero
        // 3. p = t (A0 v - V (W^T v) - W (V^T v)) on rows j+1..n-1
        sytrd_product_parts(A, ld, n, j, v, part, tid);
        for (int q2 = wv; q2 < 2 * kk; q2 += SY_THREADS / 64) {
            const double *col = (q2 < kk) ? W + (int64_t)q2 * n : V + (int64_t)(q2 - kk) * n;
            double s = 0.0;
            for (int r = j + 1 + lane; r < n; r += 64) s = fma(col[r], v[r], s);
            s = wave_sum(s);
            if (lane == 0) t12[q2] = s;      // t12[q] = W_q . v, t12[kk + q] = V_q . v
        }
        __syncthreads();
        for (int r = j + 1 + tid; r < n; r += SY_THREADS) {
            double s = (part[r] + part[(n + 1) + r]) + (part[2 * (n + 1) + r] + part[3 * (n + 1) + r]);
            for (int q0 = 0; q0 < kk; q0 += 8) {
                double a[8], b[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int q = min(q0 + u, kk - 1);
                    a[u] = V[r + (int64_t)q * n];
                    b[u] = W[r + (int64_t)q * n];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (q0 + u < kk) s -= a[u] * t12[q0 + u] + b[u] * t12[kk + q0 + u];
            }
            p[r] = t * s;
        }
        __syncthreads();
        // 4. w = p - (t/2)(p . v) v
        acc = 0.0;
        for (int r = j + 1 + tid; r < n; r += SY_THREADS) acc += p[r] * v[r];
        const double K = 0.5 * t * block_sum(acc, red);
        for (int r = j + 1 + tid; r < n; r += SY_THREADS) W[r + (int64_t)kk * n] = p[r] - K * v[r];
        __syncthreads();
    }
    if (tid < jb) {
        d[j0 + tid] = dmine;
        e[j0 + tid] = emine;
        tau[j0 + tid] = tmine;
    }
}


// The product A0 v of the panel with V and W in LDS, from the lower triangle of A0 only (the update
// after such a panel keeps only the lower triangle current).  Rows are cut into blocks of SYM_RB
// (a wave covers one block, two rows per lane, 16-byte loads) and columns into chunks of SYM_CH.
// An entry (r, c) with c < r adds A0[r][c] v[c] to row r (summed in the lane) and A0[r][c] v[r] to
// row c (summed over the wave's 64 lanes); a diagonal entry adds to its row only.  v is zero outside
// rows j+1 .. n-1, so entries outside the trailing block add nothing; entries above the diagonal,
// and the row past n that a 16-byte load reads when n is odd, are masked by selects.
//
// The active row blocks share the 16 waves in proportion to their active chunk counts (one wave at
// least, the remainder to the last block); the waves of a block take its chunks in turn.  Outputs:
// rowpart[w][0 .. SYM_RB) the row sums of wave w, colpart[b npad + c] the column sums of row block b,
// share[2 b], share[2 b + 1] the first wave of block b and the number of its waves with chunks.
constexpr int SYM_RB = 128;
constexpr int SYM_CH = 8;
constexpr int SYM_CPB = SYM_RB / SYM_CH;
constexpr int SYM_NW = SY_THREADS / 64;

// sum of p's and q's values over the two 32-lane halves: the lower half gets p's sums, the upper q's
__device__ __forceinline__ double fold32(double p, double q) {
    const long long pb = __double_as_longlong(p), qb = __double_as_longlong(q);
    const auto lo = __builtin_amdgcn_permlane32_swap((int)pb, (int)qb, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((int)(pb >> 32), (int)(qb >> 32), false, false);
    const double p2 = __longlong_as_double(((long long)(int)hi[0] << 32) | (unsigned int)lo[0]);
    const double q2 = __longlong_as_double(((long long)(int)hi[1] << 32) | (unsigned int)lo[1]);
    return p2 + q2;
}

// the same over pairs of 16-lane rows (0, 1) and (2, 3): rows 0 and 2 get p's sums, rows 1 and 3 q's
__device__ __forceinline__ double fold16(double p, double q) {
    const long long pb = __double_as_longlong(p), qb = __double_as_longlong(q);
    const auto lo = __builtin_amdgcn_permlane16_swap((int)pb, (int)qb, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((int)(pb >> 32), (int)(qb >> 32), false, false);
    const double p2 = __longlong_as_double(((long long)(int)hi[0] << 32) | (unsigned int)lo[0]);
    const double q2 = __longlong_as_double(((long long)(int)hi[1] << 32) | (unsigned int)lo[1]);
    return p2 + q2;
}

// x[u] summed over the 64 lanes; lane l returns the sum of x[l >> 3]
__device__ __forceinline__ double wave_sum_cols8(double x[SYM_CH], int lane) {
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = fold32(x[k], x[k + 4]);
#pragma unroll
    for (int k = 0; k < 2; ++k) x[k] = fold16(x[k], x[k + 2]);
    const bool up = lane & 8;          // partner lane 15 - l of the row has the other value of bit 3
    const double snd = up ? x[0] : x[1];
    double s = (up ? x[1] : x[0]) + dpp_f64<DPP_ROW_MIRROR>(snd);
    s += dpp_f64<DPP_QUAD_XOR1>(s);
    s += dpp_f64<DPP_QUAD_XOR2>(s);
    s += dpp_f64<DPP_ROW_HALF_MIRROR>(s);
    return s;
}

__device__ __forceinline__ void sytrd_product_sym(const double *__restrict__ A, int ld, int n, int npad, int j,
                                                  const double *v, double *rowpart, double *colpart, int *share,
                                                  int tid) {
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nblk = npad / SYM_RB, bmin = (j + 1) / SYM_RB, nb = nblk - bmin;
    const int cmin = (j + 1) / SYM_CH, clast = (n - 1) / SYM_CH;
    int K = 0;
    for (int q = bmin; q < nblk; ++q) K += min(SYM_CPB * q + SYM_CPB - 1, clast) - cmin + 1;
    const float scale = (float)(SYM_NW - nb) / (float)K;
    int B = bmin, i = 0, wb = 1, acc = 0;
    for (int q = bmin; q < nblk; ++q) {
        const int kq = min(SYM_CPB * q + SYM_CPB - 1, clast) - cmin + 1;
        const int wq = (q == nblk - 1) ? SYM_NW - acc : 1 + (int)(scale * (float)kq);
        if (w >= acc && w < acc + wq) {
            B = q;
            i = w - acc;
            wb = min(wq, kq);
            if (i == 0 && lane == 0) {
                share[2 * q] = acc;
                share[2 * q + 1] = wb;
            }
        }
        acc += wq;
    }
    if (i >= wb) return;
    const int r0 = SYM_RB * B + 2 * lane, r1 = r0 + 1;
    const bool rin = r0 < n && r1 > j;
    const double2 vr = *reinterpret_cast<const double2 *>(v + r0);
    double s0 = 0.0, s1 = 0.0;
    const int cmax = min(SYM_CPB * B + SYM_CPB - 1, clast);
    for (int C = cmin + i; C <= cmax; C += wb) {
        const int c0 = C * SYM_CH;
        const bool need = rin && r1 >= c0;
        double2 a[SYM_CH];
#pragma unroll
        for (int u = 0; u < SYM_CH; ++u) a[u] = make_double2(0.0, 0.0);
        if (need) {
#pragma unroll
            for (int u = 0; u < SYM_CH; ++u)
                a[u] = *reinterpret_cast<const double2 *>(A + r0 + (int64_t)min(c0 + u, n - 1) * ld);
        }
        double x[SYM_CH];
#pragma unroll
        for (int u = 0; u < SYM_CH; ++u) {
            const int c = c0 + u;
            const double vc = v[c];
            const double a0 = c <= r0 ? a[u].x : 0.0;
            const double a1 = (c <= r1 && r1 < n) ? a[u].y : 0.0;
            s0 = fma(a0, vc, s0);
            s1 = fma(a1, vc, s1);
            x[u] = fma(c < r0 ? a0 : 0.0, vr.x, (c < r1 ? a1 : 0.0) * vr.y);
        }
        const double cs = wave_sum_cols8(x, lane);
        if ((lane & 7) == 0) colpart[B * npad + c0 + (lane >> 3)] = cs;
    }
    *reinterpret_cast<double2 *>(rowpart + w * SYM_RB + 2 * lane) = make_double2(s0, s1);
}

// The panel with V and W in LDS (every access of the corrections and of W^T v, V^T v is an LDS
// access; copied to the global [V | W | V] at the end), n <= SY_THREADS: thread t owns row j + t in
// the column phases and keeps its values in registers, so a column takes five barriers; the product
// A0 v reads the lower triangle only (sytrd_product_sym).  A0 is not
// modified within the panel except for the reflector written into column j while column j is
// processed, so the next column's entry of each row is loaded one column ahead.
template <int NB>
__global__ __launch_bounds__(SY_THREADS) void k_sytrd_panel_lds(const SubDev *__restrict__ subs,
                                                                double *__restrict__ Sq, double *__restrict__ VWVb,
                                                                double *__restrict__ dout, double *__restrict__ eout,
                                                                double *__restrict__ tout, int j0) {
    extern __shared__ double sh[];
    const SubDev sd = subs[blockIdx.x];
    const int n = sd.nI;
    double *A = Sq + sd.offM;
    const int ld = sd.ldM;
    double *d = dout + sd.offI, *e = eout + sd.offI, *tau = tout + sd.offI;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (j0 >= n - 1) return;
    const int jb = min(NB, n - 1 - j0);
    double *Vg = VWVb + 3 * NB * sd.offI;
    const int npad = (n + SYM_RB - 1) / SYM_RB * SYM_RB;
    double *v = sh;                  // npad: the reflector on rows j+1 .. n-1, zero elsewhere
    double *p = sh + npad;           // n: the corrected column
    double *rowpart = p + npad;      // SYM_NW x SYM_RB
    double *colpart = rowpart + SYM_NW * SYM_RB;   // (npad / SYM_RB) x npad
    int *share = reinterpret_cast<int *>(colpart + (npad / SYM_RB) * npad);   // 16 ints
    double *t12 = colpart + (npad / SYM_RB) * npad + 8;   // 2 NB
    double *red = t12 + 4 * NB;      // two sets of 16 slots
    double *det = red + 32;          // 3 NB: d, e, tau of the panel's columns
    double *V = det + 3 * NB;        // NB x n
    double *W = V + (int64_t)NB * n; // NB x n
    for (int64_t q = tid; q < (int64_t)2 * NB * n; q += SY_THREADS) V[q] = 0.0;
    for (int q = tid; q < npad; q += SY_THREADS) v[q] = 0.0;
    double anext = j0 + tid < n ? A[(j0 + tid) + (int64_t)j0 * ld] : 0.0;
    __syncthreads();
    for (int kk = 0; kk < jb; ++kk) {
        const int j = j0 + kk;
        const int r = j + tid;
        const bool own = r < n;
        // 1. corrected column j (rows j..n-1) and the squared norm of its part below j + 1
        double s = anext;
        anext = (r + 1 < n && kk + 1 < jb) ? A[(r + 1) + (int64_t)(j + 1) * ld] : 0.0;
        if (own) {
            for (int q = 0; q < kk; ++q)
                s -= V[r + (int64_t)q * n] * W[j + (int64_t)q * n] + W[r + (int64_t)q * n] * V[j + (int64_t)q * n];
            p[r] = s;
        }
        const double xn2 = block_sum_once(own && r >= j + 2 ? s * s : 0.0, red);
        // 2. reflector from x = p[j+1 .. n-1]
        const double alpha = p[j + 1];
        double t = 0.0, beta = alpha, scal = 0.0;
        if (xn2 != 0.0) {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            t = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        const bool below = own && r >= j + 1;
        if (below) {
            const double vr = (r == j + 1) ? 1.0 : (xn2 != 0.0 ? s * scal : 0.0);
            v[r] = vr;
            A[r + (int64_t)j * ld] = vr;
            V[r + (int64_t)kk * n] = vr;
        } else if (tid == 0) {
            v[j] = 0.0;                  // row j leaves the trailing block
        }
        if (tid == 0) {              // stored after the panel (a global store per column stalls its wave)
            det[kk] = p[j];
            det[NB + kk] = beta;
            det[2 * NB + kk] = t;
        }
        __syncthreads();
        if (t == 0.0) continue;          // H_j = I: W column stays zero
        // 3. A0 v in column-group parts, and t12[q] = W_q . v, t12[kk + q] = V_q . v
        sytrd_product_sym(A, ld, n, npad, j, v, rowpart, colpart, share, tid);
        for (int q2 = wv; q2 < 2 * kk; q2 += SY_THREADS / 64) {
            const double *col = (q2 < kk) ? W + (int64_t)q2 * n : V + (int64_t)(q2 - kk) * n;
            double sq = 0.0;
            for (int rr = j + 1 + lane; rr < n; rr += 64) sq = fma(col[rr], v[rr], sq);
            sq = wave_sum(sq);
            if (lane == 0) t12[q2] = sq;
        }
        __syncthreads();
        // 4. p = t (A0 v - V (W^T v) - W (V^T v)); w = p - (t/2)(p . v) v
        double pr = 0.0, vr = 0.0;
        if (below) {
            const int b = r / SYM_RB, w0 = share[2 * b], nw = share[2 * b + 1];
            double y = 0.0;
            for (int q = 0; q < nw; ++q) y += rowpart[(w0 + q) * SYM_RB + (r & (SYM_RB - 1))];
            for (int q = b; q < npad / SYM_RB; ++q) y += colpart[q * npad + r];
            for (int q = 0; q < kk; ++q) y -= V[r + (int64_t)q * n] * t12[q] + W[r + (int64_t)q * n] * t12[kk + q];
            pr = t * y;
            vr = v[r];
        }
        const double K = 0.5 * t * block_sum_once(pr * vr, red + 16);
        if (below) W[r + (int64_t)kk * n] = pr - K * vr;
        __syncthreads();
    }
    __syncthreads();
    if (tid < jb) {
        d[j0 + tid] = det[tid];
        e[j0 + tid] = det[NB + tid];
        tau[j0 + tid] = det[2 * NB + tid];
    }
    for (int64_t q = tid; q < (int64_t)NB * n; q += SY_THREADS) {
        const double x = V[q], y = W[q];
        Vg[q] = x;
        Vg[q + (int64_t)NB * n] = y;
        Vg[q + (int64_t)2 * NB * n] = x;
    }
}

// trailing update after the panel at j0: A[j1:, j1:] -= [V W] [W V]^T (rank 2 NB), j1 = j0 + jb
template <int NB>
__global__ __launch_bounds__(256) void k_sytrd_update(const SubDev *__restrict__ subs, double *__restrict__ Sq,
                                                      const double *__restrict__ VWVb, int j0, int tiles_max) {
    const SubDev sd = subs[blockIdx.y];
    const int n = sd.nI;
    if (j0 >= n - 1) return;
    const int jb = min(NB, n - 1 - j0);
    const int j1 = j0 + jb;
    const int L1 = n - j1;
    const int tm = blockIdx.x % tiles_max, tn = blockIdx.x / tiles_max;
    if (tm * 64 >= L1 || tn * 64 >= L1) return;
    const double *V = VWVb + 3 * NB * sd.offI;
    double *A = Sq + sd.offM;
    const int ld = sd.ldM;
    gemm_tile<double>(L1, L1, 2 * NB, V + j1, n, false, V + (int64_t)NB * n + j1, n, true, A + j1 + (int64_t)j1 * ld, ld,
                      -1.0, 1.0, tm, tn);
}

// the same update on the lower 64 x 64 tiles only (tile index t = tm (tm + 1) / 2 + tn, tn <= tm), for
// the panel that reads the lower triangle only.  K = 2 NB is short, so a block stages the whole
// 64 x K slices of [V W] and [W V] in LDS at once and loads its 64 x 64 tile of A in the same round
// of loads: one barrier, then K FMAs per output (k in increasing order), then A - acc is stored.
template <int NB>
__global__ __launch_bounds__(256) void k_sytrd_update_lower(const SubDev *__restrict__ subs, double *__restrict__ Sq,
                                                            const double *__restrict__ VWVb, int j0) {
    constexpr int K = 2 * NB;
    __shared__ double sA[K][GT + 1];
    __shared__ double sB[K][GT + 1];
    const SubDev sd = subs[blockIdx.y];
    const int n = sd.nI;
    if (j0 >= n - 1) return;
    const int jb = min(NB, n - 1 - j0);
    const int j1 = j0 + jb;
    const int L1 = n - j1;
    const int t = blockIdx.x;
    int tm = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((tm + 1) * (tm + 2) / 2 <= t) ++tm;
    while (tm * (tm + 1) / 2 > t) --tm;
    const int tn = t - tm * (tm + 1) / 2;
    if (tm * GT >= L1) return;
    const double *VW = VWVb + 3 * NB * sd.offI + j1;          // [V W], column q at q n
    const double *WV = VWVb + 3 * NB * sd.offI + (int64_t)NB * n + j1;   // [W V]
    double *A = Sq + sd.offM + j1 + (int64_t)j1 * sd.ldM;
    const int ld = sd.ldM;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int i0 = tm * GT, c0 = tn * GT;
    // the tile of A (rows i0 + tx + 16 r, columns c0 + ty + 16 c) and the two K-slices, all in flight
    double cv[4][4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int gi = i0 + tx + 16 * r, gj = c0 + ty + 16 * c;
            cv[r][c] = (gi < L1 && gj < L1) ? A[gi + (int64_t)gj * ld] : 0.0;
        }
    double ra[K * GT / 256], rb[K * GT / 256];
#pragma unroll
    for (int u = 0; u < K * GT / 256; ++u) {
        const int e = tid + 256 * u, ii = e % GT, kk = e / GT;
        ra[u] = i0 + ii < L1 ? VW[(i0 + ii) + (int64_t)kk * n] : 0.0;
        rb[u] = c0 + ii < L1 ? WV[(c0 + ii) + (int64_t)kk * n] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < K * GT / 256; ++u) {
        const int e = tid + 256 * u, ii = e % GT, kk = e / GT;
        sA[kk][ii] = ra[u];
        sB[kk][ii] = rb[u];
    }
    __syncthreads();
    double acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
#pragma unroll 8
    for (int kk = 0; kk < K; ++kk) {
        double a[4], b[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = sA[kk][tx + 16 * r];
#pragma unroll
        for (int c = 0; c < 4; ++c) b[c] = sB[kk][ty + 16 * c];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] = fma(a[r], b[c], acc[r][c]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int gi = i0 + tx + 16 * r, gj = c0 + ty + 16 * c;
            if (gi < L1 && gj < L1) A[gi + (int64_t)gj * ld] = cv[r][c] - acc[r][c];
        }
}

// The trailing block of at most SY_TAIL rows.  Once the blocked panels have reduced the columns
// before J, the lower triangle of A[J:, J:] is copied into LDS (packed by rows: entry (r, c), c <= r,
// at r (r + 1) / 2 + c) and its columns are reduced there one at a time, each reflector's two-sided
// update A -= v w^T + w v^T applied at once.  Four threads (a quad) share row r, taking the columns
// c = q (mod 4), eight LDS reads in flight.  Per column: the squared norm of the column below the
// subdiagonal (block sum), the reflector (stored in its column of A in global memory, as the panels
// store theirs, with d, e, tau), p = tau A v from the lower triangle (row r's entries for c <= r,
// column r's for c > r; the quad's sums added by DPP moves), K = tau/2 p.v (block sum), w = p - K v,
// and the update of row r.  The last diagonal entry is written back to A for the final step.
constexpr int SY_TAIL = 192;
constexpr int SY_TAIL_THREADS = 4 * SY_TAIL;

__global__ __launch_bounds__(SY_TAIL_THREADS) void k_sytrd_tail(const SubDev *__restrict__ subs, double *__restrict__ Sq,
                                                                double *__restrict__ dout, double *__restrict__ eout,
                                                                double *__restrict__ tout, int J) {
    extern __shared__ double sh[];
    const SubDev sd = subs[blockIdx.x];
    const int n = sd.nI, m = n - J;
    if (m < 2) return;
    double *A = Sq + sd.offM;
    const int ld = sd.ldM;
    double *d = dout + sd.offI + J, *e = eout + sd.offI + J, *tau = tout + sd.offI + J;
    double *L = sh;                          // m (m + 1) / 2
    double *v = L + m * (m + 1) / 2;         // m
    double *w = v + m;                       // m
    double *red = w + m;                     // two sets of 16 slots
    const int r = threadIdx.x >> 2, q = threadIdx.x & 3;
    const bool own = r < m;
    const int Tr = r * (r + 1) / 2;
    const double *Aj = A + J + (int64_t)J * ld;
    if (own) {
        for (int c0 = q; c0 <= r; c0 += 32) {
            double x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = Aj[r + (int64_t)min(c0 + 4 * u, r) * ld];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (c0 + 4 * u <= r) L[Tr + c0 + 4 * u] = x[u];
        }
    }
    __syncthreads();
    for (int jj = 0; jj < m - 1; ++jj) {
        const bool below = own && r > jj;
        const double x = below ? L[Tr + jj] : 0.0;
        const double xn2 = block_sum_once(q == 0 && below && r >= jj + 2 ? x * x : 0.0, red);
        const double alpha = L[(jj + 1) * (jj + 2) / 2 + jj];
        double t = 0.0, beta = alpha, scal = 0.0;
        if (xn2 != 0.0) {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            t = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        double vr = 0.0;
        if (below) {
            vr = (r == jj + 1) ? 1.0 : (xn2 != 0.0 ? x * scal : 0.0);
            if (q == 0) {
                v[r] = vr;
                A[(J + r) + (int64_t)(J + jj) * ld] = vr;
            }
        }
        if (threadIdx.x == 0) {
            d[jj] = L[jj * (jj + 1) / 2 + jj];
            e[jj] = beta;
            tau[jj] = t;
        }
        __syncthreads();
        if (t == 0.0) continue;          // H = I: nothing to update
        double y0 = 0.0, y1 = 0.0;
        if (below) {
            for (int c0 = jj + 1 + q; c0 < m; c0 += 32) {
                double a[8], vc[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int c = min(c0 + 4 * u, m - 1);
                    a[u] = L[c <= r ? Tr + c : c * (c + 1) / 2 + r];
                    vc[u] = v[c];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) vc[u] = c0 + 4 * u < m ? vc[u] : 0.0;
#pragma unroll
                for (int u = 0; u < 8; u += 2) {
                    y0 = fma(a[u], vc[u], y0);
                    y1 = fma(a[u + 1], vc[u + 1], y1);
                }
            }
        }
        double y = y0 + y1;
        y += dpp_f64<DPP_QUAD_XOR1>(y);
        y += dpp_f64<DPP_QUAD_XOR2>(y);
        const double pr = t * y;
        const double K = 0.5 * t * block_sum_once(q == 0 ? pr * vr : 0.0, red + 16);
        const double wr = pr - K * vr;
        if (below && q == 0) w[r] = wr;
        __syncthreads();
        if (below) {
            for (int c0 = jj + 1 + q; c0 <= r; c0 += 32) {
                double a[8], wc[8], vc[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int c = min(c0 + 4 * u, r);
                    a[u] = L[Tr + c];
                    wc[u] = w[c];
                    vc[u] = v[c];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int c = c0 + 4 * u;
                    if (c <= r) L[Tr + c] = a[u] - (vr * wc[u] + wr * vc[u]);
                }
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) A[(n - 1) + (int64_t)(n - 1) * ld] = L[(m - 1) * m / 2 + (m - 1)];
}

// the last diagonal entry, after the final trailing update
__global__ void k_sytrd_last(const SubDev *__restrict__ subs, const double *__restrict__ Sq, double *__restrict__ dout) {
    const SubDev sd = subs[blockIdx.x];
    if (threadIdx.x == 0) dout[sd.offI + sd.nI - 1] = Sq[sd.offM + (int64_t)(sd.nI - 1) * (sd.ldM + 1)];
}

int32_t tridiagonalize_blocked(const SubDev *d_sub, int nsub, int maxnI, double *Sq, double *VWV, double *d, double *e,
                               double *tau, hipStream_t s) {
    const int tiles = (maxnI + 63) / 64;
    const size_t base = (size_t)(2 * maxnI + SY_G * (maxnI + 1) + 32);
    const size_t npad = (size_t)(maxnI + SYM_RB - 1) / SYM_RB * SYM_RB;
    const size_t shm_lds = (2 * npad + SYM_NW * SYM_RB + (npad / SYM_RB) * npad + 8 + 4 * SY_NB_LDS + 32 +
                            3 * SY_NB_LDS + (size_t)2 * SY_NB_LDS * maxnI) * sizeof(double);
    // the columns from J on (at most SY_TAIL rows left) are reduced in LDS by k_sytrd_tail
    const bool lds_panels = shm_lds <= (size_t)156 * 1024 && maxnI <= SY_THREADS;
    const int nb = lds_panels ? SY_NB_LDS : SY_NB;
    const int J = maxnI > SY_TAIL ? (maxnI - SY_TAIL + nb - 1) / nb * nb : 0;
    if (lds_panels) {
        for (int j0 = 0; j0 < J; j0 += SY_NB_LDS) {
            hipLaunchKernelGGL(k_sytrd_panel_lds<SY_NB_LDS>, dim3(nsub), dim3(SY_THREADS), shm_lds, s, d_sub, Sq, VWV,
                               d, e, tau, j0);
            hipLaunchKernelGGL(k_sytrd_update_lower<SY_NB_LDS>, dim3(tiles * (tiles + 1) / 2, nsub), dim3(256), 0, s,
                               d_sub, Sq, VWV, j0);
        }
    } else {
        const size_t shm = (base + 4 * SY_NB) * sizeof(double);
        for (int j0 = 0; j0 < J; j0 += SY_NB) {
            hipLaunchKernelGGL(k_sytrd_panel<SY_NB>, dim3(nsub), dim3(SY_THREADS), shm, s, d_sub, Sq, VWV, d, e,
                               tau, j0);
            hipLaunchKernelGGL(k_sytrd_update<SY_NB>, dim3(tiles * tiles, nsub), dim3(256), 0, s, d_sub, Sq, VWV, j0,
                               tiles);
        }
    }
    const size_t mt = (size_t)std::min(maxnI - J, SY_TAIL);
    const size_t shm_tail = (mt * (mt + 1) / 2 + 2 * mt + 32) * sizeof(double);
    if (mt >= 2)
        hipLaunchKernelGGL(k_sytrd_tail, dim3(nsub), dim3(SY_TAIL_THREADS), shm_tail, s, d_sub, Sq, d, e, tau, J);
    hipLaunchKernelGGL(k_sytrd_last, dim3(nsub), dim3(64), 0, s, d_sub, Sq, d);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// ------------------------------------------------------------------------------------------------
// 2. Sturm counts and selection.
// ------------------------------------------------------------------------------------------------
// number of eigenvalues of T (diagonal d, squared off-diagonal e2) strictly below sigma
__device__ int sturm_count(const double *__restrict__ d, const double *__restrict__ e2, int n, double sigma,
                           double pivmin) {
    int cnt = 0;
    double q = d[0] - sigma;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0);
    for (int i = 1; i < n; ++i) {
        q = d[i] - sigma - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += (q < 0.0);
    }
    return cnt;
}

// Sturm count with the quotient e^2 / q from the hardware reciprocal estimate refined by two
// Newton-Raphson steps (r <- r (2 - q r)); |q| >= pivmin keeps every operand finite, and the
// refined quotient is within a few ulps, inside the rounding model of the recurrence.  Used by the
// multisection, whose cost is the instruction count of this loop.
__device__ __forceinline__ double quot_nr(double e2, double q) {
    double r = __builtin_amdgcn_rcp(q);
    r = fma(fma(-q, r, 1.0), r, r);
    r = fma(fma(-q, r, 1.0), r, r);
    return e2 * r;
}

__device__ int sturm_count_nr(const double *__restrict__ d, const double *__restrict__ e2, int n, double sigma,
                              double pivmin) {
    int cnt = 0;
    double q = d[0] - sigma;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0);
    for (int i = 1; i < n; ++i) {
        q = (d[i] - sigma) - quot_nr(e2[i - 1], q);
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += (q < 0.0);
    }
    return cnt;
}

// k-th smallest eigenvalue (0-based) by bisection in (lo, hi]
__device__ double bisect_kth(const double *d, const double *e2, int n, int k, double lo, double hi, double pivmin) {
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(d, e2, n, mid, pivmin) <= k) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

// Selection runs in three launches.  (1) One wave per subdomain: Gershgorin interval, pivot floor of
// the Sturm recurrence and m from the counts at tau (or nev) and at 0.  (2) One wave per (subdomain,
// eigenvalue k <= m, eight to a wave): the k-th smallest eigenvalue by multisection, the 8 lanes
// of a group testing 8 interior shifts of its bracket at once (the Sturm counts are the cost: 8
// shifts give 3.2 bits per round for 8 counts, 64 gave 6 bits for 64).  (3) One wave per
// subdomain: the cluster at the cut is
// closed (Def. 2.15 keeps lambda_{m+1} away from lambda_m), extending m by serial bisection when
// needed.

// T staged in LDS as (d, e^2) by the whole wave; returns the Gershgorin interval, widened, and pivmin
__device__ void stage_tridiagonal(const double *__restrict__ dg, const double *__restrict__ eg, int n, double *d,
                                  double *e2, double *lo_out, double *hi_out, double *piv_out) {
    const int lane = threadIdx.x & 63;
    double lo = 1e300, hi = -1e300, emax2 = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double r = (i > 0 ? fabs(eg[i - 1]) : 0.0) + (i + 1 < n ? fabs(eg[i]) : 0.0);
        lo = fmin(lo, dg[i] - r);
        hi = fmax(hi, dg[i] + r);
        d[i] = dg[i];
        if (i + 1 < n) {
            e2[i] = eg[i] * eg[i];
            emax2 = fmax(emax2, e2[i]);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, o, 64));
        hi = fmax(hi, __shfl_xor(hi, o, 64));
        emax2 = fmax(emax2, __shfl_xor(emax2, o, 64));
    }
    __syncthreads();
    const double tnorm = fmax(fabs(lo), fabs(hi));
    const double pivmin = fmax(2.2250738585072014e-308, 2.2204460492503131e-16 * 2.2204460492503131e-16 * emax2);
    *lo_out = lo - (2.2204460492503131e-16 * tnorm * n + pivmin);
    *hi_out = hi + (2.2204460492503131e-16 * tnorm * n + pivmin);
    *piv_out = pivmin;
}

// per subdomain: Gershgorin bounds, pivot floor, count below tau, count below 0
constexpr int IV_SLOTS = 5;

__global__ __launch_bounds__(64) void k_select_count(const SubDev *__restrict__ subs, const double *__restrict__ dbuf,
                                                     const double *__restrict__ ebuf, int mode, double tau, int nev,
                                                     int mmax, int32_t *__restrict__ m_out, int32_t *__restrict__ flag,
                                                     double *__restrict__ iv) {
    extern __shared__ double sh[];
    const SubDev sd = subs[blockIdx.x];
    const int n = sd.nI;
    double *d = sh, *e2 = sh + n;
    double lo, hi, pivmin;
    stage_tridiagonal(dbuf + sd.offI, ebuf + sd.offI, n, d, e2, &lo, &hi, &pivmin);
    const int lane = threadIdx.x;
    // lane 0 counts below tau, lane 1 below 0 (the rest idle)
    int c = 0;
    if (lane == 0) c = (mode == HKG_EIG_THRESHOLD) ? sturm_count(d, e2, n, tau, pivmin) : nev;
    else if (lane == 1) c = sturm_count(d, e2, n, 0.0, pivmin);
    const int c0 = __shfl(c, 0, 64), c1 = __shfl(c, 1, 64);
    const int m = min(max(c0, c1), n);     // every lambda <= 0 joins (Def. 2.15: lambda_{m+1} > 0)
    if (lane == 0) {
        m_out[blockIdx.x] = m;
        flag[blockIdx.x] = m > mmax ? 1 : 0;
        iv[IV_SLOTS * blockIdx.x] = lo;
        iv[IV_SLOTS * blockIdx.x + 1] = hi;
        iv[IV_SLOTS * blockIdx.x + 2] = pivmin;
        // the counts below tau (threshold mode) and below 0: eigenvalue k < count lies below that
        // shift, which bounds its bracket from above
        iv[IV_SLOTS * blockIdx.x + 3] = mode == HKG_EIG_THRESHOLD ? (double)c0 : 0.0;
        iv[IV_SLOTS * blockIdx.x + 4] = (double)c1;
    }
}

// wave (subdomain, eight eigenvalues): 8-lane group r of the wave takes eigenvalue k = 8 y + r, with
// lambda_k in (a, b] and count(a) <= k < count(b), and narrows the bracket 9-fold per round (8
// interior shifts, one per lane; the group's new bracket by DPP max / min inside the group)
__device__ __forceinline__ double group_max8(double v) {
    v = fmax(v, dpp_f64<DPP_QUAD_XOR1>(v));
    v = fmax(v, dpp_f64<DPP_QUAD_XOR2>(v));
    return fmax(v, dpp_f64<DPP_ROW_HALF_MIRROR>(v));
}

__device__ __forceinline__ double group_min8(double v) {
    v = fmin(v, dpp_f64<DPP_QUAD_XOR1>(v));
    v = fmin(v, dpp_f64<DPP_QUAD_XOR2>(v));
    return fmin(v, dpp_f64<DPP_ROW_HALF_MIRROR>(v));
}

__global__ __launch_bounds__(64) void k_select_refine(const SubDev *__restrict__ subs, const double *__restrict__ dbuf,
                                                      const double *__restrict__ ebuf, int mmax, double tau,
                                                      const int32_t *__restrict__ m_in, const int32_t *__restrict__ flag,
                                                      const double *__restrict__ iv, double *__restrict__ lam_out) {
    extern __shared__ double sh[];
    const int sub = blockIdx.x, lane = threadIdx.x, t = lane & 7;
    const int k = 8 * blockIdx.y + (lane >> 3);
    const SubDev sd = subs[sub];
    const int n = sd.nI;
    const int kend = min(n, m_in[sub] + 1);
    if (flag[sub] || 8 * (int)blockIdx.y >= kend) return;
    double *d = sh, *e2 = sh + n;
    double lo0, hi0, pv0;
    stage_tridiagonal(dbuf + sd.offI, ebuf + sd.offI, n, d, e2, &lo0, &hi0, &pv0);
    const double pivmin = iv[IV_SLOTS * sub + 2];
    double a = iv[IV_SLOTS * sub], b = iv[IV_SLOTS * sub + 1];
    // count(tau) > k or count(0) > k: the bracket (a, b] may end at that shift
    if (k < (int)iv[IV_SLOTS * sub + 3]) b = fmin(b, tau);
    if (k < (int)iv[IV_SLOTS * sub + 4]) b = fmin(b, 0.0);
    bool done = k >= kend;               // rows past the last eigenvalue take part without a result
    for (int it = 0; it < 120; ++it) {
        const double sig = a + (b - a) * ((double)(t + 1) / 9.0);
        const bool inside = !done && sig > a && sig < b;
        const int cnt = sturm_count_nr(d, e2, n, sig, pivmin);
        const double na = group_max8((inside && cnt <= k) ? sig : a);
        const double nb = group_min8((inside && cnt > k) ? sig : b);
        if (na == a && nb == b) done = true;     // the bracket cannot be split further
        a = na;
        b = nb;
        if (__all(done)) break;
    }
    if (t == 0 && k < kend) lam_out[(int64_t)sub * (mmax + 2) + k] = 0.5 * (a + b);
}

// close a cluster at the cut: lambda_{m+1} - lambda_m <= rtol max(1, |lambda_m|) moves the cut up
__global__ __launch_bounds__(64) void k_select_close(const SubDev *__restrict__ subs, const double *__restrict__ dbuf,
                                                     const double *__restrict__ ebuf, double rtol, int mmax,
                                                     int32_t *__restrict__ m_io, int32_t *__restrict__ flag,
                                                     const double *__restrict__ iv, double *__restrict__ lam_out) {
    extern __shared__ double sh[];
    const int sub = blockIdx.x;
    const SubDev sd = subs[sub];
    const int n = sd.nI;
    if (flag[sub]) return;
    double *d = sh, *e2 = sh + n;
    double lo, hi, pivmin;
    stage_tridiagonal(dbuf + sd.offI, ebuf + sd.offI, n, d, e2, &lo, &hi, &pivmin);
    if (threadIdx.x != 0) return;
    double *lam = lam_out + (int64_t)sub * (mmax + 2);
    int m = m_io[sub];
    while (m > 0 && m < n && lam[m] - lam[m - 1] <= rtol * fmax(1.0, fabs(lam[m - 1]))) {
        ++m;
        if (m > mmax) break;
        if (m < n) lam[m] = bisect_kth(d, e2, n, m, iv[IV_SLOTS * sub], iv[IV_SLOTS * sub + 1], pivmin);
    }
    flag[sub] = (m > mmax) ? 1 : 0;
    m_io[sub] = m;
}

int32_t select_eigs(const SubDev *d_sub, int nsub, int maxnI, const double *d, const double *e, int mode, double tau,
                    int nev, double rtol, int mmax, int32_t *m_out, double *lam_out, int32_t *flag, double *iv,
                    hipStream_t s) {
    const size_t shm = (size_t)2 * maxnI * sizeof(double);
    hipLaunchKernelGGL(k_select_count, dim3(nsub), dim3(64), shm, s, d_sub, d, e, mode, tau, nev, mmax, m_out, flag, iv);
    hipLaunchKernelGGL(k_select_refine, dim3(nsub, (mmax + 1 + 7) / 8), dim3(64), shm, s, d_sub, d, e, mmax, tau, m_out, flag,
                       iv, lam_out);
    hipLaunchKernelGGL(k_select_close, dim3(nsub), dim3(64), shm, s, d_sub, d, e, rtol, mmax, m_out, flag, iv, lam_out);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// ------------------------------------------------------------------------------------------------
// 3. inverse iteration on T for each selected eigenvalue, one lane per eigenvalue: (T - lambda I) y = b
//    by Gaussian elimination with partial pivoting on the tridiagonal (a serial recurrence per lane),
//    then, by the whole wave, Gram-Schmidt against the earlier vectors whose eigenvalues lie within
//    1e-3 ||T|| and normalisation.  Three sweeps from a fixed pseudo-random start vector.
//    Per-lane work arrays live in a global scratch area, interleaved (entry i of lane k at i m + k)
//    so that the lanes' accesses coalesce.
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ double start_value(int i, int k) {
    uint32_t h = (uint32_t)i * 2654435761u ^ ((uint32_t)k * 40503u + 0x9e3779b9u);
    h ^= h >> 15; h *= 2246822519u; h ^= h >> 13; h *= 3266489917u; h ^= h >> 16;
    return ((double)(h & 0xffffff) / 16777216.0) * 2.0 - 1.0;
}

// The iterates live in LDS when n m doubles fit (LDSB), else in the global scratch; the factors of
// T - lambda I stay in the global scratch (read-only in the sweeps).  Running values of the
// recurrences are carried in registers, the reciprocal pivots are stored, and the loads of four
// steps are issued before their arithmetic.
// rows per group of the substitution sweeps: the group's loads are issued together, so a sweep
// waits on memory once per IU rows
constexpr int IU = 16;

// NBI: rows per lane of a vector held in registers during the orthogonalisation (n <= 64 NBI)
template <bool LDSB, int NBI>
__global__ __launch_bounds__(64) void k_inverse_iteration(const SubDev *__restrict__ subs, const double *__restrict__ dbuf,
                                                          const double *__restrict__ ebuf, const double *__restrict__ lam_all,
                                                          int mmax, double *__restrict__ Zb, double *__restrict__ scratch,
                                                          unsigned char *__restrict__ swp_all) {
    extern __shared__ double sb[];
    const SubDev sd = subs[blockIdx.x];
    const int n = sd.nI, m = sd.m;
    if (m == 0) return;
    const double *d = dbuf + sd.offI, *e = ebuf + sd.offI;
    const double *lam = lam_all + (int64_t)blockIdx.x * (mmax + 2);
    const int64_t nm = (int64_t)n * m;
    double *__restrict__ rdd = scratch + 5 * sd.offZ;
    double *__restrict__ du = rdd + nm;
    double *__restrict__ du2 = du + nm;
    double *__restrict__ fac = du2 + nm;
    double *__restrict__ b = LDSB ? sb : fac + nm;
    __shared__ double scl[64];            // per vector: the scale of the last substitution
    const unsigned char *__restrict__ swp = swp_all + sd.offZ;
    unsigned char *__restrict__ swpw = swp_all + sd.offZ;
    double *Z = Zb + sd.offZ;
    const int lane = threadIdx.x;
    double tnorm = 0.0;
    for (int i = lane; i < n; i += 64)
        tnorm = fmax(tnorm, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0));
    for (int o = 32; o > 0; o >>= 1) tnorm = fmax(tnorm, __shfl_xor(tnorm, o, 64));
    const double pert = 2.2204460492503131e-16 * fmax(tnorm, 1e-300);
    const double orth_tol = 1e-3 * tnorm;
    // factor T - lambda_k I = P L U for every selected k (lane k), U with two super-diagonals
    for (int k = lane; k < m; k += 64) {
        const double lk = lam[k];
        double ddi = d[0] - lk;                       // running diagonal entry of row i
        double dui = n > 1 ? e[0] : 0.0;              // running entry (i, i+1)
        for (int i = 0; i + 1 < n; ++i) {
            const double sub = e[i];
            const double dnext = d[i + 1] - lk;
            const double unext = (i + 2 < n) ? e[i + 1] : 0.0;
            const int64_t q = (int64_t)i * m + k;
            if (fabs(ddi) >= fabs(sub)) {
                if (ddi == 0.0) ddi = pert;
                const double f = sub / ddi;
                swpw[q] = 0;
                fac[q] = f;
                rdd[q] = 1.0 / ddi;
                du[q] = dui;
                du2[q] = 0.0;
                ddi = dnext - f * dui;
                dui = unext;
            } else {
                const double f = ddi / sub;
                swpw[q] = 1;
                fac[q] = f;
                rdd[q] = 1.0 / sub;
                du[q] = dnext;
                du2[q] = unext;
                ddi = dui - f * dnext;
                dui = -f * unext;
            }
        }
        if (ddi == 0.0) ddi = pert;
        rdd[(int64_t)(n - 1) * m + k] = 1.0 / ddi;
        for (int i = 0; i < n; ++i) b[(int64_t)i * m + k] = start_value(i, k);
    }
    __syncthreads();
    for (int sweep = 0; sweep < 3; ++sweep) {
        for (int k = lane; k < m; k += 64) {
            // forward elimination with the row exchanges; cur = running entry of row i
            double cur = b[k];
            for (int i0 = 0; i0 + 1 < n; i0 += IU) {
                double bn[IU], f[IU];
                int sw[IU];
#pragma unroll
                for (int u = 0; u < IU; ++u) {
                    const int i = min(i0 + u, n - 2);
                    const int64_t q = (int64_t)i * m + k;
                    bn[u] = b[q + m];
                    f[u] = fac[q];
                    sw[u] = swp[q];
                }
#pragma unroll
                for (int u = 0; u < IU; ++u) {
                    if (i0 + u + 1 < n) {
                        const double out = sw[u] ? bn[u] : cur;
                        cur = sw[u] ? cur - f[u] * bn[u] : bn[u] - f[u] * cur;
                        b[(int64_t)(i0 + u) * m + k] = out;
                    }
                }
            }
            b[(int64_t)(n - 1) * m + k] = cur;
            // back substitution with U (diagonal, two super-diagonals); x1 = x_{i+1}, x2 = x_{i+2}
            double x1 = 0.0, x2 = 0.0, mx = 0.0;
            for (int i0 = n - 1; i0 >= 0; i0 -= IU) {
                double bv[IU], u1[IU], u2[IU], r[IU];
#pragma unroll
                for (int u = 0; u < IU; ++u) {
                    const int i = max(i0 - u, 0);
                    const int64_t q = (int64_t)i * m + k;
                    bv[u] = b[q];
                    u1[u] = du[q];
                    u2[u] = du2[q];
                    r[u] = rdd[q];
                }
#pragma unroll
                for (int u = 0; u < IU; ++u) {
                    const int i = i0 - u;
                    if (i >= 0) {
                        double v = bv[u];
                        if (i + 1 < n) v -= u1[u] * x1;
                        if (i + 2 < n) v -= u2[u] * x2;
                        v *= r[u];
                        b[(int64_t)i * m + k] = v;
                        x2 = x1;
                        x1 = v;
                        mx = fmax(mx, fabs(v));
                    }
                }
            }
            scl[k] = mx > 0.0 ? 1.0 / mx : 1.0;      // applied as the vector is loaded below
        }
        __syncthreads();
        // modified Gram-Schmidt inside clusters, then normalisation: the whole wave per vector, the
        // vector in registers (row lane + 64 j in slot j) from its scaled load to its store
        for (int k = 0; k < m; ++k) {
            const double sk = scl[k];
            double bk[NBI];
#pragma unroll
            for (int j = 0; j < NBI; ++j) {
                const int i = lane + 64 * j;
                bk[j] = i < n ? b[(int64_t)i * m + k] * sk : 0.0;
            }
            for (int q = 0; q < k; ++q) {
                if (fabs(lam[q] - lam[k]) > orth_tol) continue;
                double bq[NBI], s = 0.0;
#pragma unroll
                for (int j = 0; j < NBI; ++j) {
                    const int i = lane + 64 * j;
                    bq[j] = i < n ? b[(int64_t)i * m + q] : 0.0;
                }
#pragma unroll
                for (int j = 0; j < NBI; ++j) s += bq[j] * bk[j];
                s = wave_sum(s);
#pragma unroll
                for (int j = 0; j < NBI; ++j) bk[j] -= s * bq[j];
            }
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < NBI; ++j) s += bk[j] * bk[j];
            s = wave_sum(s);
            const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
#pragma unroll
            for (int j = 0; j < NBI; ++j) {
                const int i = lane + 64 * j;
                if (i < n) b[(int64_t)i * m + k] = bk[j] * inv;
            }
            __syncthreads();
        }
    }
    for (int k = 0; k < m; ++k)
        for (int i = lane; i < n; i += 64) Z[(int64_t)k * n + i] = b[(int64_t)i * m + k];
}

constexpr size_t II_LDS_MAX = 150 * 1024;

int32_t tridiag_vectors_n(const SubDev *d_sub, int nsub, int maxnI, int64_t max_nm, const double *d, const double *e,
                          const double *lam, int mmax, double *Z, double *scratch, unsigned char *swp, hipStream_t s) {
    if (maxnI > 24 * 64) {
        set_last_error("inverse iteration supports at most 1536 unknowns per subdomain");
        return HKG_EINVAL;
    }
    const size_t shm = (size_t)max_nm * sizeof(double);
    const bool lds = shm <= II_LDS_MAX, narrow = maxnI <= 8 * 64;
    if (lds && narrow)
        hipLaunchKernelGGL((k_inverse_iteration<true, 8>), dim3(nsub), dim3(64), shm, s, d_sub, d, e, lam, mmax, Z,
                           scratch, swp);
    else if (lds)
        hipLaunchKernelGGL((k_inverse_iteration<true, 24>), dim3(nsub), dim3(64), shm, s, d_sub, d, e, lam, mmax, Z,
                           scratch, swp);
    else if (narrow)
        hipLaunchKernelGGL((k_inverse_iteration<false, 8>), dim3(nsub), dim3(64), 0, s, d_sub, d, e, lam, mmax, Z,
                           scratch, swp);
    else
        hipLaunchKernelGGL((k_inverse_iteration<false, 24>), dim3(nsub), dim3(64), 0, s, d_sub, d, e, lam, mmax, Z,
                           scratch, swp);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// ------------------------------------------------------------------------------------------------
// 4. back-transformation y <- Q y with Q = H_0 H_1 ... H_{n-2} (reflectors applied last-first), one
//    wave per eigenvector with the vector staged in LDS.  The reflectors are read three steps ahead
//    into a queue of registers (a step is a dot product, a wave sum and an update, shorter than a
//    memory round trip, so one step of look-ahead left every step waiting on its loads).
//    NB = ceil(n / 64) registers per lane hold a reflector.
// ------------------------------------------------------------------------------------------------
template <int NB>
__global__ __launch_bounds__(64) void k_back_transform(const SubDev *__restrict__ subs, const double *__restrict__ Sq,
                                                       const double *__restrict__ taub, double *__restrict__ Zb) {
    extern __shared__ double zs[];
    const SubDev sd = subs[blockIdx.x];
    const int c = blockIdx.y;
    if (c >= sd.m) return;
    const int n = sd.nI, lane = threadIdx.x;
    const double *A = Sq + sd.offM;
    const int ld = sd.ldM;
    const double *tau = taub + sd.offI;
    double *z = Zb + sd.offZ + (int64_t)c * n;
    for (int i = lane; i < n; i += 64) zs[i] = z[i];
    __syncthreads();
    if (n < 2) {
        for (int i = lane; i < n; i += 64) z[i] = zs[i];
        return;
    }
    // reflector j: v = A[j+1 .. n-1, j]; entry i of it (i < L = n - j - 1) in lane i % 64, slot i / 64.
    // Indices below 0 are clamped to reflector 0 (loaded, never applied).
    double v0[NB], v1[NB], v2[NB];
    auto load = [&](int j, double *dst) {
        j = max(j, 0);
        const int L = n - j - 1;
        const double *v = A + (j + 1) + (int64_t)j * ld;
#pragma unroll
        for (int q = 0; q < NB; ++q) dst[q] = v[min(lane + 64 * q, L - 1)];
    };
    load(n - 2, v0);
    load(n - 3, v1);
    load(n - 4, v2);
    double t0 = tau[n - 2], t1 = tau[max(n - 3, 0)], t2 = tau[max(n - 4, 0)];
    for (int j = n - 2; j >= 0; --j) {
        double v3[NB];
        load(j - 3, v3);
        const double t3 = tau[max(j - 3, 0)];
        if (t0 != 0.0) {
            const int L = n - j - 1;
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int i = lane + 64 * q;
                if (i < L) s = fma(v0[q], zs[j + 1 + i], s);
            }
            s = t0 * wave_sum(s);
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int i = lane + 64 * q;
                if (i < L) zs[j + 1 + i] -= s * v0[q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            v0[q] = v1[q];
            v1[q] = v2[q];
            v2[q] = v3[q];
        }
        t0 = t1;
        t1 = t2;
        t2 = t3;
    }
    for (int i = lane; i < n; i += 64) z[i] = zs[i];
}

// The same with one workgroup per subdomain: the subdomain's eigenvectors stay in registers (wave w
// holds eigenvectors w, w + BT_WAVES, ...; lane l rows l + 64 k), and the reflectors are staged in
// LDS a panel of BT_PB at a time (reflector q of a panel in row q, zero outside rows j+1 .. n-1), the
// next panel's loads in flight while the current panel is applied: one global round trip per panel
// instead of one per reflector.  E = eigenvectors per wave at most; n <= 64 NB.
constexpr int BT_PB = 8;
constexpr int BT_WAVES = 16;

template <int NB, int E>
__global__ __launch_bounds__(64 * BT_WAVES) void k_back_transform_panel(const SubDev *__restrict__ subs,
                                                                        const double *__restrict__ Sq,
                                                                        const double *__restrict__ taub,
                                                                        double *__restrict__ Zb) {
    constexpr int NP = 64 * NB;                    // panel row stride
    constexpr int NT = 64 * BT_WAVES;
    constexpr int PER = BT_PB * NP / NT;           // panel entries staged per thread
    __shared__ double pv[2][BT_PB * NP];
    __shared__ double pt[2][BT_PB];
    const SubDev sd = subs[blockIdx.x];
    const int n = sd.nI, m = sd.m;
    if (m == 0 || n < 2) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const double *A = Sq + sd.offM;
    const int ld = sd.ldM;
    const double *tau = taub + sd.offI;
    double *Z = Zb + sd.offZ;
    double z[E][NB];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int c = w + BT_WAVES * e;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const int r = lane + 64 * k;
            z[e][k] = (c < m && r < n) ? Z[(int64_t)c * n + r] : 0.0;
        }
    }
    // panel p: reflectors j = n - 2 - p BT_PB - q, q < BT_PB (the order of application)
    const int npanel = (n - 1 + BT_PB - 1) / BT_PB;
    double reg[PER], treg = 0.0;
    auto load_panel = [&](int p) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + NT * u, q = e / NP, r = e % NP, j = n - 2 - p * BT_PB - q;
            const bool ok = j >= 0 && r > j && r < n;
            reg[u] = ok ? A[r + (int64_t)max(j, 0) * ld] : 0.0;
        }
        if (tid < BT_PB) {
            const int j = n - 2 - p * BT_PB - tid;
            treg = j >= 0 ? tau[j] : 0.0;
        }
    };
    auto store_panel = [&](int b) {
#pragma unroll
        for (int u = 0; u < PER; ++u) pv[b][tid + NT * u] = reg[u];
        if (tid < BT_PB) pt[b][tid] = treg;
    };
    load_panel(0);
    store_panel(0);
    __syncthreads();
    for (int p = 0; p < npanel; ++p) {
        const int b = p & 1;
        if (p + 1 < npanel) load_panel(p + 1);
        for (int q = 0; q < BT_PB; ++q) {
            const double t = pt[b][q];
            if (t == 0.0) continue;        // H = I (also the slots past reflector 0)
            double v[NB];
#pragma unroll
            for (int k = 0; k < NB; ++k) v[k] = pv[b][q * NP + lane + 64 * k];
            double sdot[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                double a = 0.0;
#pragma unroll
                for (int k = 0; k < NB; ++k) a = fma(v[k], z[e][k], a);
                sdot[e] = wave_sum(a);
            }
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double f = t * sdot[e];
#pragma unroll
                for (int k = 0; k < NB; ++k) z[e][k] = fma(-f, v[k], z[e][k]);
            }
        }
        if (p + 1 < npanel) store_panel(b ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int c = w + BT_WAVES * e;
        if (c < m)
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const int r = lane + 64 * k;
                if (r < n) Z[(int64_t)c * n + r] = z[e][k];
            }
    }
}

int32_t back_transform_n(const SubDev *d_sub, int nsub, int maxnI, int max_m, const double *Sq, const double *tau,
                         double *Z, hipStream_t s) {
    if (max_m == 0) return HKG_OK;
    if (maxnI <= 8 * 64 && max_m <= 4 * BT_WAVES) {
        const dim3 g(nsub), t(64 * BT_WAVES);
        if (max_m <= BT_WAVES) hipLaunchKernelGGL((k_back_transform_panel<8, 1>), g, t, 0, s, d_sub, Sq, tau, Z);
        else if (max_m <= 2 * BT_WAVES) hipLaunchKernelGGL((k_back_transform_panel<8, 2>), g, t, 0, s, d_sub, Sq, tau, Z);
        else hipLaunchKernelGGL((k_back_transform_panel<8, 4>), g, t, 0, s, d_sub, Sq, tau, Z);
        HKG_HIP(hipGetLastError());
        return HKG_OK;
    }
    const size_t shm = (size_t)maxnI * sizeof(double);
    if (maxnI <= 8 * 64)
        hipLaunchKernelGGL(k_back_transform<8>, dim3(nsub, max_m), dim3(64), shm, s, d_sub, Sq, tau, Z);
    else if (maxnI <= 24 * 64)
        hipLaunchKernelGGL(k_back_transform<24>, dim3(nsub, max_m), dim3(64), shm, s, d_sub, Sq, tau, Z);
    else {
        set_last_error("back-transformation supports at most 1536 unknowns per subdomain");
        return HKG_EINVAL;
    }
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// Z[i, :] /= sqrt(U_ii) with U the upper factor of C_II = L U (no row exchanges)
__global__ __launch_bounds__(256) void k_scale_rows(const SubDev *__restrict__ subs, const double *__restrict__ C,
                                                    double *__restrict__ Zb) {
    const SubDev sd = subs[blockIdx.x];
    const int n = sd.nI;
    for (int64_t q = threadIdx.x; q < (int64_t)n * sd.m; q += 256) {
        int i = (int)(q % n);
        Zb[sd.offZ + q] /= sqrt(C[sd.offSq + i + (int64_t)i * n]);
    }
}

int32_t scale_rows_invsqrt_diag(const SubDev *d_sub, int nsub, const double *C, double *Z, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_rows, dim3(nsub), dim3(256), 0, s, d_sub, C, Z);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// sign convention (entry of largest magnitude positive, first on ties) then Z = X_I P
__global__ __launch_bounds__(256) void k_finish_basis(const SubDev *__restrict__ subs, const int32_t *__restrict__ I_idx,
                                                      const double *__restrict__ winv, double *__restrict__ Zb) {
    const SubDev sd = subs[blockIdx.x];
    const int n = sd.nI, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int c = wv; c < sd.m; c += 4) {
        double *z = Zb + sd.offZ + (int64_t)c * n;
        double best = -1.0;
        int bi = n;
        for (int i = lane; i < n; i += 64) {
            double a = fabs(z[i]);
            if (a > best) { best = a; bi = i; }
        }
        for (int o = 32; o > 0; o >>= 1) {
            double ob = __shfl_xor(best, o, 64);
            int oi = __shfl_xor(bi, o, 64);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        const double sgn = (bi < n && z[bi] < 0.0) ? -1.0 : 1.0;
        for (int i = lane; i < n; i += 64) z[i] = sgn * z[i] * winv[I_idx[sd.offI + i]];
    }
}

int32_t finish_basis(const SubDev *d_sub, int nsub, const int32_t *I_idx, const double *winv, double *Z,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_finish_basis, dim3(nsub), dim3(256), 0, s, d_sub, I_idx, winv, Z);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// ------------------------------------------------------------------------------------------------
// coarse matrix blocks: B_0[(j, b), (i, a)] = sum over q in ovdof(D_i) and dof(D_j) of
//   Z_j[q, b] (B Z_i)[q, a],  with (B Z_i)[q, a] = Y_i[a, q] and Y_i = Z_i^T [B_II | B_IG]  (B symmetric)
// ------------------------------------------------------------------------------------------------
// the shared dofs of a pair in chunks of CP_CH staged in LDS (rows of Z_j from its row-major copy,
// columns of Y_i, both contiguous), each thread then summing its entries over the chunk in the
// same order as the direct form below
constexpr int CP_CH = 64;
constexpr int CP_MMAX = 32;

__global__ __launch_bounds__(256) void k_coarse_pairs(const int32_t *__restrict__ pi, const int32_t *__restrict__ pj,
                                                      const int32_t *__restrict__ ptr, const int32_t *__restrict__ qi,
                                                      const int32_t *__restrict__ qj, const SubDev *__restrict__ subs,
                                                      const double *__restrict__ Y, const double *__restrict__ Zr,
                                                      double *__restrict__ B0, int m0) {
    __shared__ double ys[CP_CH][CP_MMAX + 1];      // ys[u][a] = Y_i[a, qi[u]]
    __shared__ double zs[CP_CH][CP_MMAX + 1];      // zs[u][b] = Z_j[qj[u], b]
    const int t = blockIdx.x;
    const SubDev si = subs[pi[t]], sj = subs[pj[t]];
    const int mi = si.m, mj = sj.m;
    if (mi == 0 || mj == 0) return;
    const int beg = ptr[t], end = ptr[t + 1];
    const int tid = threadIdx.x;
    constexpr int PER = CP_MMAX * CP_MMAX / 256;   // entries per thread
    double acc[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) acc[k] = 0.0;
    for (int u0 = beg; u0 < end; u0 += CP_CH) {
        const int cnt = min(CP_CH, end - u0);
        __syncthreads();
        for (int e = tid; e < cnt * mi; e += 256) {
            const int u = e / mi, a = e % mi;
            ys[u][a] = Y[si.offY + a + (int64_t)qi[u0 + u] * mi];
        }
        for (int e = tid; e < cnt * mj; e += 256) {
            const int u = e / mj, b = e % mj;
            zs[u][b] = Zr[sj.offZ + (int64_t)qj[u0 + u] * mj + b];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int q = tid + 256 * k;
            if (q < mi * mj) {
                const int b = q % mj, a = q / mj;
                double sacc = acc[k];
                for (int u = 0; u < cnt; ++u) sacc += zs[u][b] * ys[u][a];
                acc[k] = sacc;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int q = tid + 256 * k;
        if (q < mi * mj) {
            const int b = q % mj, a = q / mj;
            B0[(int64_t)(sj.offm + b) + (int64_t)(si.offm + a) * m0] = acc[k];
        }
    }
}

// direct form: every thread gathers its terms from global memory (subdomains with m > CP_MMAX)
__global__ __launch_bounds__(256) void k_coarse_pairs_direct(const int32_t *__restrict__ pi,
                                                             const int32_t *__restrict__ pj,
                                                             const int32_t *__restrict__ ptr,
                                                             const int32_t *__restrict__ qi,
                                                             const int32_t *__restrict__ qj,
                                                             const SubDev *__restrict__ subs,
                                                             const double *__restrict__ Y,
                                                             const double *__restrict__ Zr,
                                                             double *__restrict__ B0, int m0) {
    const int t = blockIdx.x;
    const SubDev si = subs[pi[t]], sj = subs[pj[t]];
    const int mi = si.m, mj = sj.m;
    if (mi == 0 || mj == 0) return;
    const int beg = ptr[t], end = ptr[t + 1];
    for (int q = threadIdx.x; q < mi * mj; q += 256) {
        const int b = q % mj, a = q / mj;
        double s = 0.0;
        for (int u = beg; u < end; ++u)
            s += Zr[sj.offZ + (int64_t)qj[u] * mj + b] * Y[si.offY + a + (int64_t)qi[u] * mi];
        B0[(int64_t)(sj.offm + b) + (int64_t)(si.offm + a) * m0] = s;
    }
}

int32_t coarse_pairs(int npairs, const int32_t *pi, const int32_t *pj, const int32_t *ptr, const int32_t *qi,
                     const int32_t *qj, const SubDev *d_sub, int max_m, const double *Y, const double *Zr, double *B0,
                     int m0, hipStream_t s) {
    if (npairs == 0) return HKG_OK;
    if (max_m <= CP_MMAX)
        hipLaunchKernelGGL(k_coarse_pairs, dim3(npairs), dim3(256), 0, s, pi, pj, ptr, qi, qj, d_sub, Y, Zr, B0, m0);
    else
        hipLaunchKernelGGL(k_coarse_pairs_direct, dim3(npairs), dim3(256), 0, s, pi, pj, ptr, qi, qj, d_sub, Y, Zr, B0,
                           m0);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

}  // namespace hkg
