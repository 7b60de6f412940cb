// Batched kernels of one FGMRES iteration (and of the cycle start/end) over all problems of a batch.
//
// One application of the two-level preconditioner (eq. (2.23)) and one CGS2 Arnoldi step for every
// active (problem, rhs) pair; see batch.hpp for the descriptors.  The numerical content of each kernel
// is the single-problem one: local solves with the resident inverses (the coarse restriction fused
// into the same pass over r_D), split coarse product with a fixed-order reduction, Z_i y_i added per
// subdomain, the transpose-map sum, the CSR product, CGS2 with wave-parallel fixed-order reductions,
// Givens rotations on the device.  No atomics: results do not depend on how the batch is composed,
// so a problem solved alone or in a mix gives bitwise the same iterates.
#include "batch.hpp"
#include "internal.hpp"
#include "wave.hpp"

namespace hkg {

constexpr int LS_ROWS = 64;
constexpr int NPART = 16;        // partial sums per local-solve row (a multiple of every wave count)

// sum over the 64 lanes of a wave (DPP moves within 16-lane rows, then the four row sums in order)
__device__ __forceinline__ double bwsum(double v) { return wave_sum64(v); }

// Loads in the loops below are never guarded by a wave-uniform branch: a branch around a load makes the
// wave wait for it before the next one issues.  Indices are clamped into range instead and only the
// arithmetic is masked, so every load of an unrolled group is in flight at once.

// sum over the nonzeros of row i of val[t] x[col[t]], eight at a time, in index order
__device__ __forceinline__ double csr_row_dot(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                              const double *__restrict__ val, const double *__restrict__ x, int i) {
    const int t0 = rowptr[i], t1 = rowptr[i + 1];
    double s = 0.0;
    for (int t = t0; t < t1; t += 8) {
        int c[8];
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int tt = min(t + k, t1 - 1);
            c[k] = col[tt];
            v[k] = t + k < t1 ? val[tt] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) s = fma(v[k], x[c[k]], s);
    }
    return s;
}

__device__ __forceinline__ bool inactive(const ProbDev &P, int rhs, int mode) {
    return rhs >= P.nrhs || (mode == 1 && P.active[rhs] != PS_ITER);
}

// Arnoldi index of a pair, double-buffered: iteration graphs alternate the parity `par`; an iteration
// reads jcur[2 rhs + par] and its last kernel writes jcur[2 rhs + 1 - par]
__device__ __forceinline__ int jget(const ProbDev &P, int rhs, int par) { return P.jcur[2 * rhs + par]; }

__device__ __forceinline__ const double *vcol(const ProbDev &P, int rhs, int j) {
    return P.V + (int64_t)rhs * P.n * (P.restart + 1) + (int64_t)j * P.n;
}

__device__ __forceinline__ double *vcol_w(const ProbDev &P, int rhs, int j) {
    return P.V + (int64_t)rhs * P.n * (P.restart + 1) + (int64_t)j * P.n;
}

__device__ __forceinline__ double *zcol(const ProbDev &P, int rhs, int j) {
    return P.Zk + (int64_t)rhs * P.n * P.restart + (int64_t)j * P.n;
}

// ------------------------------------------------------------------------------------------------
// local solves (+ restriction tile), T = storage precision of the local inverses
// ------------------------------------------------------------------------------------------------
// The column sums of the product with the inverse are split into NPART partial sums (partial q takes
// the columns congruent to q modulo NPART, in increasing order) and the partials are added in order
// q = 0, 1, ...: the rounding does not depend on how many waves share the columns, so every launch
// shape the autotuner may pick gives the same bits.  A tile is LTILE rows; each lane owns two
// consecutive rows and reads them with one aligned 2-element vector load (the inverses' leading
// dimension is padded to a multiple of 32 entries, rows past n_I are padding and discarded).
template <typename T>
struct Pair2;
template <>
struct Pair2<float> {
    using type = float2;
};
template <>
struct Pair2<double> {
    using type = double2;
};

template <typename T, int WAVES>
__device__ __forceinline__ void local_body(const ProbDev &P, const SubDev &sd, const double *__restrict__ r, int rhs,
                                           double *sh) {
    using V2 = typename Pair2<T>::type;
    constexpr int PW = NPART / WAVES;                 // partials per wave
    constexpr int UNR = PW >= 4 ? 1 : 4 / PW;         // vector loads in flight per thread: PW * UNR
    const int n = sd.nI;
    const int tiles = (n + LTILE - 1) / LTILE;
    const bool coarse = P.two_level && P.m0 > 0;
    const bool restrict_tile = (int)blockIdx.x == tiles;
    double *xd = sh;
    T *xt = reinterpret_cast<T *>(sh + n);
    double *part = sh + n + (n * sizeof(T) + 7) / 8;  // NPART x LTILE
    const int32_t *I = P.I_idx + sd.offI;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // the row tile's first UNR column groups are loaded before the gather of r, so that their
    // latency overlaps the gather's two dependent loads (same summation order as the loop below)
    const int row0 = blockIdx.x * LTILE + 2 * lane;
    const T *M = reinterpret_cast<const T *>(P.Minv) + sd.offM + row0;
    const int64_t ldm = sd.ldM;
    const bool rows_ok = !restrict_tile && row0 < n;
    V2 pre[UNR][PW];
#pragma unroll
    for (int g = 0; g < UNR; ++g)
#pragma unroll
        for (int k = 0; k < PW; ++k) {
            const int col = min(g * NPART + wv + k * WAVES, n - 1);
            pre[g][k] = rows_ok ? *reinterpret_cast<const V2 *>(M + col * ldm) : V2{};
        }
    for (int i = threadIdx.x; i < n; i += LS_ROWS * WAVES) {
        const double v = r[I[i]];
        xd[i] = v;
        xt[i] = (T)v;
    }
    __syncthreads();
    if (restrict_tile) {
        // c_i = Z_i^T r on dof(D_i), same partial-sum order
        const int m = sd.m;
        const double *Zt = P.Zr + sd.offZ;
        for (int q = wv; q < NPART; q += WAVES) {
            double acc = 0.0;
            if (lane < m)
                for (int p = q; p < n; p += NPART) acc = fma(Zt[lane + (int64_t)p * m], xd[p], acc);
            part[q * LTILE + lane] = acc;
        }
        __syncthreads();
        if (wv == 0 && lane < m && coarse) {
            double s = 0.0;
            for (int q = 0; q < NPART; ++q) s += part[q * LTILE + lane];
            P.c[(int64_t)rhs * P.m0 + sd.offm + lane] = s;
        }
        return;
    }
    T acc[PW][2];
#pragma unroll
    for (int k = 0; k < PW; ++k) acc[k][0] = acc[k][1] = T(0);
    if (row0 < n) {
        int c0 = 0;
        if (UNR * NPART <= n) {
#pragma unroll
            for (int g = 0; g < UNR; ++g)
#pragma unroll
                for (int k = 0; k < PW; ++k) {
                    const int col = g * NPART + wv + k * WAVES;
                    acc[k][0] = fma(pre[g][k].x, xt[col], acc[k][0]);
                    acc[k][1] = fma(pre[g][k].y, xt[col], acc[k][1]);
                }
            c0 = UNR * NPART;
        }
#pragma unroll UNR
        for (; c0 + NPART <= n; c0 += NPART) {
#pragma unroll
            for (int k = 0; k < PW; ++k) {
                const int col = c0 + wv + k * WAVES;
                const V2 v = *reinterpret_cast<const V2 *>(M + col * ldm);
                acc[k][0] = fma(v.x, xt[col], acc[k][0]);
                acc[k][1] = fma(v.y, xt[col], acc[k][1]);
            }
        }
#pragma unroll
        for (int k = 0; k < PW; ++k) {
            const int col = c0 + wv + k * WAVES;
            if (col < n) {
                const V2 v = *reinterpret_cast<const V2 *>(M + col * ldm);
                acc[k][0] = fma(v.x, xt[col], acc[k][0]);
                acc[k][1] = fma(v.y, xt[col], acc[k][1]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < PW; ++k) {
        part[(wv + k * WAVES) * LTILE + 2 * lane] = (double)acc[k][0];
        part[(wv + k * WAVES) * LTILE + 2 * lane + 1] = (double)acc[k][1];
    }
    __syncthreads();
    const int t = threadIdx.x, row = blockIdx.x * LTILE + t;
    if (t < LTILE && row < n) {
        T s = T(0);
        for (int q = 0; q < NPART; ++q) s += (T)part[q * LTILE + t];
        P.u[(int64_t)rhs * P.sum_nI + sd.offI + row] = P.wloc[sd.offI + row] * (double)s;
    }
}

template <int WAVES>
__global__ __launch_bounds__(LS_ROWS *WAVES) void k_b_local(const ProbDev *__restrict__ probs,
                                                            const WorkItem *__restrict__ items, int mode, int par) {
    extern __shared__ double sh[];
    const WorkItem it = items[blockIdx.y];
    const ProbDev &P = probs[it.p];
    const int rhs = blockIdx.z;
    if (inactive(P, rhs, mode)) return;
    const SubDev sd = P.subs[it.s];
    const int tiles = (sd.nI + LTILE - 1) / LTILE;
    const bool coarse = P.two_level && P.m0 > 0;
    if ((int)blockIdx.x > tiles || ((int)blockIdx.x == tiles && (!coarse || sd.m == 0))) return;
    const double *r = (mode == 0) ? P.xin + (int64_t)rhs * P.ldin : vcol(P, rhs, jget(P, rhs, par));
    if (P.local_f32) local_body<float, WAVES>(P, sd, r, rhs, sh);
    else local_body<double, WAVES>(P, sd, r, rhs, sh);
}

// Coarse solve y = B_0^{-1} c: CG_WPR waves per coarse row r, one block per row.  B_0 is symmetric
// (B_0 = Z^T B Z), so row r of its inverse is read as column r of the stored column-major inverse:
// contiguous, coalesced.  Wave w takes the w-th of CG_WPR contiguous column ranges (a multiple of 64
// loads each); with m_0 even (the column then starts 16-byte aligned) a lane reads column pairs
// (16-byte loads: 8-byte ones reach about 3.5 TB/s on this row length, 16-byte ones 4.8) and sums the
// pairs l, l + 64, ... of its wave's range in increasing order, both entries of a pair in turn; with
// m_0 odd it reads single entries in the same pattern.  Each wave's sum is reduced in fixed order and
// the CG_WPR wave sums are added in wave order: the final y (no split partial sums), whatever the
// batch composition.  y is stored in the ypart region.
constexpr int CG_RPB = 4;        // rows per work item (the host lists items of four rows)
constexpr int CG_WPR = 4;        // waves per row
constexpr int CG_U = 5;          // loads in flight per lane

__global__ __launch_bounds__(64 * CG_WPR) void k_b_coarse_gemv(const ProbDev *__restrict__ probs,
                                                               const WorkItem *__restrict__ cblk, int mode) {
    __shared__ double wsum[CG_WPR];
    const WorkItem it = cblk[blockIdx.x / CG_RPB];
    const ProbDev &P = probs[it.p];
    const int rhs = blockIdx.z;
    if (inactive(P, rhs, mode) || !P.two_level) return;
    const int m0 = P.m0, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = it.s * CG_RPB + (int)(blockIdx.x % CG_RPB);
    if (r >= m0) return;
    const double *col = P.B0inv + (int64_t)r * m0;
    const double *c = P.c + (int64_t)rhs * m0;
    const bool pairs = (m0 & 1) == 0 && (((uintptr_t)P.B0inv | (uintptr_t)P.c) & 15) == 0;
    double acc = 0.0;
    if (pairs) {
        const int np = m0 / 2;
        const int span = ((np + CG_WPR - 1) / CG_WPR + 63) / 64 * 64;
        const int k1 = min(wv * span, np), k2 = min(k1 + span, np);
        const double2 *b2 = reinterpret_cast<const double2 *>(col);
        const double2 *c2 = reinterpret_cast<const double2 *>(c);
        for (int k0 = k1 + lane; k0 < k2; k0 += 64 * CG_U) {
            double2 b[CG_U], x[CG_U];
#pragma unroll
            for (int k = 0; k < CG_U; ++k) {
                const int q = min(k0 + 64 * k, k2 - 1);
                b[k] = b2[q];
                x[k] = c2[q];
            }
#pragma unroll
            for (int k = 0; k < CG_U; ++k) {
                const bool in = k0 + 64 * k < k2;
                acc = fma(b[k].x, in ? x[k].x : 0.0, acc);
                acc = fma(b[k].y, in ? x[k].y : 0.0, acc);
            }
        }
    } else {
        const int span = ((m0 + CG_WPR - 1) / CG_WPR + 63) / 64 * 64;
        const int k1 = min(wv * span, m0), k2 = min(k1 + span, m0);
        for (int k0 = k1 + lane; k0 < k2; k0 += 64 * 2 * CG_U) {
            double b[2 * CG_U], x[2 * CG_U];
#pragma unroll
            for (int k = 0; k < 2 * CG_U; ++k) {
                const int q = min(k0 + 64 * k, k2 - 1);
                b[k] = col[q];
                x[k] = c[q];
            }
#pragma unroll
            for (int k = 0; k < 2 * CG_U; ++k) acc = fma(b[k], k0 + 64 * k < k2 ? x[k] : 0.0, acc);
        }
    }
    acc = bwsum(acc);
    if (lane == 0) wsum[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double y = wsum[0];
#pragma unroll
        for (int w = 1; w < CG_WPR; ++w) y += wsum[w];
        P.ypart[(int64_t)rhs * m0 + r] = y;
    }
}

// z_l = sum over the positions t of dof l in the local vectors (transpose map, fixed order) of
// u[t] + (Z_i y_i)[a], t = (subdomain i, local index a): the coarse correction E_0 y = sum_i E_i Z_i y_i
// folded into the same pass.  Four lanes per dof: lane q takes the positions t0 + q, t0 + q + 4, ...
// (each carries its row of Z_i in the row-major copy and its slice of y; Z and y entries are loaded
// eight at a time), and the quad's sums are added in lane order, which for up to four positions is
// the sequential order over t.  (One lane per dof left a chain of dependent memory round trips per
// thread at four waves per CU.)
__global__ __launch_bounds__(4 * BROWS) void k_b_prolong(const ProbDev *__restrict__ probs,
                                                         const WorkItem *__restrict__ rblk, int mode, int par) {
    const WorkItem it = rblk[blockIdx.x];
    const ProbDev &P = probs[it.p];
    const int rhs = blockIdx.z;
    if (inactive(P, rhs, mode)) return;
    const int q = threadIdx.x & 3;
    const int l = it.s * BROWS + (threadIdx.x >> 2);
    if (l >= P.n) return;                  // whole quads leave together
    const double *uu = P.u + (int64_t)rhs * P.sum_nI;
    const double *y = P.ypart + (int64_t)rhs * P.m0;
    const int t1 = P.tp_ptr[l + 1];
    double v = 0.0;
    for (int t = P.tp_ptr[l] + q; t < t1; t += 4) {
        const double ut = uu[P.tp_pos[t]];     // issued before the coarse row's loads
        double c = 0.0;
        if (P.two_level) {
            const TpCoarse d = P.tpc[t];
            for (int b0 = 0; b0 < d.m; b0 += 8) {
                double zv[8], yv[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int kk = min(b0 + k, d.m - 1);
                    zv[k] = P.Zr[d.zoff + kk];
                    yv[k] = y[d.yoff + kk];
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) c = fma(zv[k], b0 + k < d.m ? yv[k] : 0.0, c);
            }
        }
        v += ut + c;
    }
    const double s = ((dpp_f64<0x00>(v) + dpp_f64<0x55>(v)) + dpp_f64<0xAA>(v)) + dpp_f64<0xFF>(v);
    if (q == 0) {
        double *z = (mode == 0) ? P.xout + (int64_t)rhs * P.ldout : zcol(P, rhs, jget(P, rhs, par));
        z[l] = s;
    }
}

int32_t batch_apply(const BatchGeom &g, const ProbDev *probs, const WorkItem *items, const WorkItem *rblk,
                    const WorkItem *cblk, int mode, int par, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    const dim3 gl(g.max_tiles + (g.any_coarse ? 1 : 0), g.nitems, g.max_nrhs);
    const size_t shm = (size_t)2 * g.max_nI * sizeof(double) + (size_t)NPART * LTILE * sizeof(double);
    if (ev0) HKG_HIP(hipEventRecord(ev0, s));
    switch (g.local_waves) {
        case 4:
            hipLaunchKernelGGL(k_b_local<4>, gl, dim3(LS_ROWS * 4), shm, s, probs, items,
                               mode, par);
            break;
        case 16:
            hipLaunchKernelGGL(k_b_local<16>, gl, dim3(LS_ROWS * 16), shm, s, probs, items, mode, par);
            break;
        default:
            hipLaunchKernelGGL(k_b_local<8>, gl, dim3(LS_ROWS * 8), shm, s, probs, items,
                               mode, par);
    }
    HKG_HIP(hipGetLastError());
    if (ev1) HKG_HIP(hipEventRecord(ev1, s));
    if (g.any_coarse)
        hipLaunchKernelGGL(k_b_coarse_gemv, dim3(g.ncblk * CG_RPB, 1, g.max_nrhs), dim3(64 * CG_WPR), 0, s, probs,
                           cblk, mode);
    hipLaunchKernelGGL(k_b_prolong, dim3(g.nrblk, 1, g.max_nrhs), dim3(4 * BROWS), 0, s, probs, rblk, mode, par);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// ------------------------------------------------------------------------------------------------
// Arnoldi step (CGS2) at the device-side index j = jcur
// ------------------------------------------------------------------------------------------------
// CGS2 kernels run CG_T = 4 BROWS threads per row block: thread t owns row r0 + (t mod BROWS) in
// column group t / BROWS for the update w -= V h, and the 16 waves share the slots of the partial
// sums, so that a CU keeps many independent loads of V in flight.
constexpr int CG_T = 4 * BROWS;
constexpr int CG_W = CG_T / 64;          // waves per block
constexpr int RED_U = 4;                 // row-block partials a lane loads at once when reducing them

// Partial sums of one row block (BROWS rows r0 .. r0 + BROWS): slot i <= j of x_i . w, slot j + 1 of
// w . w, written column by column (out[i * nb], the row blocks of one slot contiguous).  Wave wv takes
// the slots congruent to wv modulo CG_W; lane l holds rows r0 + l + 64 q (q < 4) of w in wl[q], so a
// slot costs 4 independent loads and one cross-lane sum, and four slots are in flight at once.
__device__ __forceinline__ void slot_partials(const double *__restrict__ V, int n, int r0, int j, const double wl[4],
                                              double *__restrict__ out, int nb) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i0 = wv; i0 <= j + 1; i0 += 4 * CG_W) {
        double a[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = i0 + CG_W * k;
            const double *x = V + (int64_t)min(i, j) * n;
            double d = 0.0, ww = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // wl[q] is 0 for rows past n
                d = fma(x[min(r0 + lane + 64 * q, n - 1)], wl[q], d);
                ww = fma(wl[q], wl[q], ww);
            }
            a[k] = i <= j ? d : (i == j + 1 ? ww : 0.0);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = i0 + CG_W * k;
            if (i <= j + 1) {
                const double t = bwsum(a[k]);
                if (lane == 0) out[(int64_t)i * nb] = t;
            }
        }
    }
}

// part region of a pair: two halves of S x nb (slot-major), the first also holding the residual
// norm partials in slot 0
__device__ __forceinline__ double *part_half(const ProbDev &P, int rhs, int half) {
    const int S = P.restart + 2;
    return P.part + ((int64_t)rhs * 2 + half) * S * P.nblk;
}

// w = V[:, j+1] = B Zk[:, j] for the block's rows, then the block's first-pass partials (they need
// only these rows of w)
__global__ __launch_bounds__(CG_T) void k_b_spmv_dots(const ProbDev *__restrict__ probs,
                                                      const WorkItem *__restrict__ rblk, int par) {
    __shared__ double wsh[BROWS];
    const WorkItem it = rblk[blockIdx.x];
    const ProbDev &P = probs[it.p];
    const int rhs = blockIdx.z;
    if (inactive(P, rhs, 1)) return;
    const int n = P.n, j = jget(P, rhs, par), r0 = it.s * BROWS, lane = threadIdx.x & 63;
    const double *x = zcol(P, rhs, j);
    double *V = vcol_w(P, rhs, 0);
    if (threadIdx.x < BROWS) {
        const int i = r0 + threadIdx.x;
        double s = 0.0;
        if (i < n) {
            s = csr_row_dot(P.rowptr, P.colidx, P.Bval, x, i);
            V[(int64_t)(j + 1) * n + i] = s;
        }
        wsh[threadIdx.x] = s;
    }
    __syncthreads();
    double wl[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) wl[q] = wsh[lane + 64 * q];
    slot_partials(V, n, r0, j, wl, part_half(P, rhs, 0) + it.s, P.nblk);
}

// reduce the pass's partials (one wave per slot, fixed order: lane-strided sums, then a butterfly),
// w -= V h (four column groups per row, added in group order), next partials
__global__ __launch_bounds__(CG_T) void k_b_update(const ProbDev *__restrict__ probs, const WorkItem *__restrict__ rblk,
                                                   int pass, int par) {
    extern __shared__ double sh[];
    const WorkItem it = rblk[blockIdx.x];
    const ProbDev &P = probs[it.p];
    const int rhs = blockIdx.z;
    if (inactive(P, rhs, 1)) return;
    const int n = P.n, m = P.restart, S = m + 2, nb = P.nblk, j = jget(P, rhs, par);
    double *V = vcol_w(P, rhs, 0);
    double *w = V + (int64_t)(j + 1) * n;
    const double *pin = part_half(P, rhs, pass == 1 ? 0 : 1);
    double *h = sh;              // S
    double *wsh = sh + S;        // BROWS
    double *gs = wsh + BROWS;    // 4 x BROWS column-group sums
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i0 = wv; i0 <= j + 1; i0 += 4 * CG_W) {
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        for (int b0 = lane; b0 < nb; b0 += 64 * RED_U) {
            double v[RED_U][4];
#pragma unroll
            for (int u = 0; u < RED_U; ++u)
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    v[u][k] = pin[(int64_t)min(i0 + CG_W * k, j + 1) * nb + min(b0 + 64 * u, nb - 1)];
#pragma unroll
            for (int u = 0; u < RED_U; ++u)
                if (b0 + 64 * u < nb)
#pragma unroll
                    for (int k = 0; k < 4; ++k) a[k] += v[u][k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = i0 + CG_W * k;
            if (i <= j + 1) {
                const double t = bwsum(a[k]);
                if (lane == 0) h[i] = t;
            }
        }
    }
    __syncthreads();
    if (it.s == 0) {
        double *hc = P.hcol + (int64_t)rhs * S;
        for (int i = threadIdx.x; i <= j; i += CG_T) hc[i] = (pass == 1) ? h[i] : hc[i] + h[i];
        if (pass == 1 && threadIdx.x == 0) hc[m + 1] = sqrt(h[j + 1]);
    }
    const int r0 = it.s * BROWS, lr = threadIdx.x & (BROWS - 1), grp = threadIdx.x / BROWS;
    const int row = min(r0 + lr, n - 1);
    {
        double acc = 0.0;
        for (int i0 = grp; i0 <= j; i0 += 4 * 8) {
            double x[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) x[k] = V[(int64_t)min(i0 + 4 * k, j) * n + row];
#pragma unroll
            for (int k = 0; k < 8; ++k) acc = fma(x[k], i0 + 4 * k <= j ? h[min(i0 + 4 * k, j)] : 0.0, acc);
        }
        gs[grp * BROWS + lr] = acc;
    }
    __syncthreads();
    double v = 0.0;
    if (grp == 0 && r0 + lr < n) {
        v = w[row] - (((gs[lr] + gs[BROWS + lr]) + gs[2 * BROWS + lr]) + gs[3 * BROWS + lr]);
        w[row] = v;
    }
    if (pass == 1) {
        if (grp == 0) wsh[lr] = v;
        __syncthreads();
        double wl[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) wl[q] = wsh[lane + 64 * q];
        slot_partials(V, n, r0, j, wl, part_half(P, rhs, 1) + it.s, nb);
    } else {
        const double s = bwsum(v * v);
        if (lane == 0 && wv < 4) wsh[wv] = s;
        __syncthreads();
        if (threadIdx.x == 0) part_half(P, rhs, 0)[it.s] = wsh[0] + wsh[1] + wsh[2] + wsh[3];
    }
}

// ||w||, v_{j+1} = w / ||w||; block 0: Hessenberg column, Givens rotations, stopping tests
__global__ __launch_bounds__(BROWS) void k_b_finish(const ProbDev *__restrict__ probs, const WorkItem *__restrict__ rblk,
                                                    int par) {
    extern __shared__ double fs[];       // hc[0..j+1], cs[0..j), sn[0..j)
    const WorkItem it = rblk[blockIdx.x];
    const ProbDev &P = probs[it.p];
    const int rhs = blockIdx.z;
    if (inactive(P, rhs, 1)) return;
    const int n = P.n, m = P.restart, S = m + 2, nb = P.nblk, j = jget(P, rhs, par);
    const double *pin = part_half(P, rhs, 0);
    double nrm2 = 0.0;
    for (int b0 = (threadIdx.x & 63); b0 < nb; b0 += 64 * RED_U) {
        double v[RED_U];
#pragma unroll
        for (int u = 0; u < RED_U; ++u) v[u] = pin[min(b0 + 64 * u, nb - 1)];
#pragma unroll
        for (int u = 0; u < RED_U; ++u)
            if (b0 + 64 * u < nb) nrm2 += v[u];
    }
    nrm2 = bwsum(nrm2);
    const double hn = sqrt(nrm2);
    double *w = vcol_w(P, rhs, j + 1);
    const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
    const int row = it.s * BROWS + threadIdx.x;
    if (row < n) w[row] *= inv;
    if (it.s != 0) return;
    const double *hc = P.hcol + (int64_t)rhs * S;
    double *H = P.H + (int64_t)rhs * (m + 1) * m + (int64_t)j * (m + 1);
    double *cs = P.cs + (int64_t)rhs * m, *sn = P.sn + (int64_t)rhs * m, *g = P.g + (int64_t)rhs * (m + 1);
    double *hs = fs, *css = fs + S, *sns = fs + S + m;
    for (int i = threadIdx.x; i <= j; i += BROWS) hs[i] = hc[i];
    for (int i = threadIdx.x; i < j; i += BROWS) {
        css[i] = cs[i];
        sns[i] = sn[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // the earlier rotations, four at a time with their operands read ahead of the chain (the
        // same operations in the same order as one at a time)
        double cur = hs[0];
        int i = 0;
        for (; i + 4 <= j; i += 4) {
            double nx[4], cc[4], ss[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                nx[u] = hs[i + 1 + u];
                cc[u] = css[i + u];
                ss[u] = sns[i + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                hs[i + u] = cc[u] * cur + ss[u] * nx[u];
                cur = -ss[u] * cur + cc[u] * nx[u];
            }
        }
        for (; i < j; ++i) {
            const double nx = hs[i + 1];
            hs[i] = css[i] * cur + sns[i] * nx;
            cur = -sns[i] * cur + css[i] * nx;
        }
        const double d = hypot(cur, hn);
        const double c = d > 0.0 ? cur / d : 1.0, s = d > 0.0 ? hn / d : 0.0;
        cs[j] = c;
        sn[j] = s;
        hs[j] = d;
        hs[j + 1] = 0.0;
        double *sc = P.scal + (int64_t)rhs * 8;
        g[j + 1] = -s * g[j];
        g[j] = c * g[j];
        sc[2] = fabs(g[j + 1]);
        const int conv = fabs(g[j + 1]) <= P.rtol * sc[1];
        const int brk = hn <= 1e-14 * hc[m + 1];
        const int sing = d == 0.0;
        const int itn = ++P.iters[rhs];
        // a singular rotated column (zero diagonal of R) is left out of the back substitution; the
        // restart phase then retires the pair (sc[5])
        sc[3] = (double)(sing ? j : j + 1);
        if (conv || brk || sing || j + 1 == m || itn >= P.max_iter) {
            P.active[rhs] = PS_CYCLE_END;
            sc[4] = conv ? 1.0 : 0.0;
            sc[5] = sing ? 1.0 : 0.0;
        } else {
            P.jcur[2 * rhs + 1 - par] = j + 1;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j + 1; i += BROWS) H[i] = hs[i];
}

int32_t batch_arnoldi(const BatchGeom &g, const ProbDev *probs, const WorkItem *rblk, int par, hipStream_t s) {
    const dim3 grid(g.nrblk, 1, g.max_nrhs);
    const size_t upd = (size_t)(g.restart + 2 + 5 * BROWS) * sizeof(double);
    const size_t fin = (size_t)(3 * g.restart + 2) * sizeof(double);
    hipLaunchKernelGGL(k_b_spmv_dots, grid, dim3(CG_T), 0, s, probs, rblk, par);
    hipLaunchKernelGGL(k_b_update, grid, dim3(CG_T), upd, s, probs, rblk, 1, par);
    hipLaunchKernelGGL(k_b_update, grid, dim3(CG_T), upd, s, probs, rblk, 2, par);
    hipLaunchKernelGGL(k_b_finish, grid, dim3(BROWS), fin, s, probs, rblk, par);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// ------------------------------------------------------------------------------------------------
// restart phase: pairs whose cycle ended (PS_CYCLE_END) or that just joined (PS_NEW)
// ------------------------------------------------------------------------------------------------
// y = R^{-1} g on the rotated Hessenberg of a pair whose cycle ended (one block per pair; column
// oriented back substitution, the next column's entries loaded while the current one is applied),
// stored in the pair's hcol (free once its cycle has ended)
constexpr int TS_Q = 4;         // restart <= TS_Q * BROWS

__global__ __launch_bounds__(BROWS) void k_r_solve_y(const ProbDev *__restrict__ probs, const int32_t *__restrict__ live,
                                                     int max_nrhs) {
    extern __shared__ double y[];        // restart
    const int t = blockIdx.x;
    const ProbDev &P = probs[live[t / max_nrhs]];
    const int rhs = t % max_nrhs;
    if (rhs >= P.nrhs || P.active[rhs] != PS_CYCLE_END) return;
    const int m = P.restart;
    const int jd = (int)P.scal[(int64_t)rhs * 8 + 3];
    if (jd <= 0) return;
    const double *H = P.H + (int64_t)rhs * (m + 1) * m;
    const double *g = P.g + (int64_t)rhs * (m + 1);
    for (int i = threadIdx.x; i < jd; i += BROWS) y[i] = g[i];
    double cur[TS_Q], nxt[TS_Q];
    int k = jd - 1;
#pragma unroll
    for (int q = 0; q < TS_Q; ++q) cur[q] = H[min((int)threadIdx.x + BROWS * q, k) + (int64_t)k * (m + 1)];
    double dcur = H[k + (int64_t)k * (m + 1)], dnxt = 0.0;
    __syncthreads();
    for (; k >= 0; --k) {
        const int kn = max(k - 1, 0);
#pragma unroll
        for (int q = 0; q < TS_Q; ++q) nxt[q] = H[min((int)threadIdx.x + BROWS * q, kn) + (int64_t)kn * (m + 1)];
        dnxt = H[kn + (int64_t)kn * (m + 1)];
        const double yk = y[k] / dcur;
        __syncthreads();
        if (threadIdx.x == 0) y[k] = yk;
#pragma unroll
        for (int q = 0; q < TS_Q; ++q) {
            const int i = threadIdx.x + BROWS * q;
            if (i < k) y[i] -= cur[q] * yk;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < TS_Q; ++q) cur[q] = nxt[q];
        dcur = dnxt;
    }
    for (int i = threadIdx.x; i < jd; i += BROWS) P.hcol[(int64_t)rhs * (m + 2) + i] = y[i];
}

// x += Z_k y (PS_CYCLE_END, y from k_r_solve_y), or x = 0 (PS_NEW)
__global__ __launch_bounds__(BROWS) void k_r_update_x(const ProbDev *__restrict__ probs,
                                                      const WorkItem *__restrict__ rblk) {
    extern __shared__ double ys[];       // restart
    const WorkItem it = rblk[blockIdx.x];
    const ProbDev &P = probs[it.p];
    const int rhs = blockIdx.z;
    if (rhs >= P.nrhs) return;
    const int st = P.active[rhs];
    const int r = it.s * BROWS + threadIdx.x;
    double *x = P.x + (int64_t)rhs * P.ldx;
    if (st == PS_NEW) {
        if (r < P.n) x[r] = 0.0;
        return;
    }
    if (st != PS_CYCLE_END) return;
    const int m = P.restart;
    const int jd = (int)P.scal[(int64_t)rhs * 8 + 3];
    if (jd <= 0) return;
    for (int i = threadIdx.x; i < jd; i += BROWS) ys[i] = P.hcol[(int64_t)rhs * (m + 2) + i];
    __syncthreads();
    if (r >= P.n) return;
    const double *Zk = zcol(P, rhs, 0);
    double s = x[r];
    for (int i0 = 0; i0 < jd; i0 += 4) {
        double zv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) zv[k] = Zk[(int64_t)min(i0 + k, jd - 1) * P.n + r];
#pragma unroll
        for (int k = 0; k < 4; ++k) s = fma(zv[k], i0 + k < jd ? ys[min(i0 + k, jd - 1)] : 0.0, s);
    }
    x[r] = s;
}

// V[:, 0] = f - B x (PS_NEW: x = 0, so V[:, 0] = f) and partial squared norms per row block
__global__ __launch_bounds__(BROWS) void k_r_residual(const ProbDev *__restrict__ probs,
                                                      const WorkItem *__restrict__ rblk) {
    __shared__ double red[BROWS / 64];
    const WorkItem it = rblk[blockIdx.x];
    const ProbDev &P = probs[it.p];
    const int rhs = blockIdx.z;
    if (rhs >= P.nrhs) return;
    const int st = P.active[rhs];
    if (st != PS_NEW && st != PS_CYCLE_END) return;
    const int i = it.s * BROWS + threadIdx.x;
    double v = 0.0;
    if (i < P.n) {
        v = P.f[(int64_t)rhs * P.ldf + i];
        if (st == PS_CYCLE_END) {
            v -= csr_row_dot(P.rowptr, P.colidx, P.Bval, P.x + (int64_t)rhs * P.ldx, i);
        }
        vcol_w(P, rhs, 0)[i] = v;
    }
    const double s = bwsum(v * v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < BROWS / 64; ++w) t += red[w];
        part_half(P, rhs, 0)[it.s] = t;
    }
}

// per pair: ||r|| (fixed order over row blocks); stop (converged, ||f|| = 0 or out of iterations) or
// start a new cycle: beta = ||r||, g = beta e_1, j = 0
__global__ void k_r_decide(const ProbDev *__restrict__ probs, const int32_t *__restrict__ live, int nlive,
                           int max_nrhs) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nlive * max_nrhs) return;
    const ProbDev &P = probs[live[t / max_nrhs]];
    const int rhs = t % max_nrhs;
    if (rhs >= P.nrhs) return;
    const int st = P.active[rhs];
    if (st != PS_NEW && st != PS_CYCLE_END) return;
    const double *pp = part_half(P, rhs, 0);
    double s = 0.0;
    for (int b = 0; b < P.nblk; ++b) s += pp[b];
    const double rn = sqrt(s);
    P.rnorm[rhs] = rn;
    double *sc = P.scal + (int64_t)rhs * 8;
    if (st == PS_NEW) {
        for (int k = 0; k < 8; ++k) sc[k] = 0.0;
        sc[1] = rn;
        sc[2] = rn;
        P.iters[rhs] = 0;
    }
    const double fn = sc[1];
    const bool sing = st == PS_CYCLE_END && sc[5] != 0.0;
    if (fn == 0.0 || !gmres_keeps_going(rn, fn, P.rtol) || sing || P.iters[rhs] >= P.max_iter) {
        P.active[rhs] = PS_DONE;
        return;
    }
    double *g = P.g + (int64_t)rhs * (P.restart + 1);
    for (int k = 0; k <= P.restart; ++k) g[k] = 0.0;
    g[0] = rn;
    sc[0] = rn;
    sc[2] = rn;
    sc[3] = 0.0;
    sc[4] = 0.0;
    sc[5] = 0.0;
    P.jcur[2 * rhs] = 0;
    P.jcur[2 * rhs + 1] = 0;
    P.active[rhs] = PS_START;
}

// v_0 = r / beta for the pairs starting a cycle
__global__ __launch_bounds__(BROWS) void k_r_start(const ProbDev *__restrict__ probs, const WorkItem *__restrict__ rblk) {
    const WorkItem it = rblk[blockIdx.x];
    const ProbDev &P = probs[it.p];
    const int rhs = blockIdx.z;
    if (rhs >= P.nrhs || P.active[rhs] != PS_START) return;
    const int i = it.s * BROWS + threadIdx.x;
    if (i < P.n) vcol_w(P, rhs, 0)[i] *= 1.0 / P.rnorm[rhs];
}

__global__ void k_r_activate(const ProbDev *__restrict__ probs, const int32_t *__restrict__ live, int nlive,
                             int max_nrhs) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nlive * max_nrhs) return;
    const ProbDev &P = probs[live[t / max_nrhs]];
    const int rhs = t % max_nrhs;
    if (rhs < P.nrhs && P.active[rhs] == PS_START) P.active[rhs] = PS_ITER;
}

int32_t batch_restart(const BatchGeom &g, const ProbDev *probs, const WorkItem *rblk, const int32_t *live,
                      hipStream_t s) {
    const dim3 grid(g.nrblk, 1, g.max_nrhs);
    const int pairs = g.nprob * g.max_nrhs;
    hipLaunchKernelGGL(k_r_solve_y, dim3(pairs), dim3(BROWS), (size_t)g.restart * sizeof(double), s, probs, live,
                       g.max_nrhs);
    hipLaunchKernelGGL(k_r_update_x, grid, dim3(BROWS), (size_t)g.restart * sizeof(double), s, probs, rblk);
    hipLaunchKernelGGL(k_r_residual, grid, dim3(BROWS), 0, s, probs, rblk);
    hipLaunchKernelGGL(k_r_decide, dim3((pairs + 255) / 256), dim3(256), 0, s, probs, live, g.nprob, g.max_nrhs);
    hipLaunchKernelGGL(k_r_start, grid, dim3(BROWS), 0, s, probs, rblk);
    hipLaunchKernelGGL(k_r_activate, dim3((pairs + 255) / 256), dim3(256), 0, s, probs, live, g.nprob, g.max_nrhs);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

}  // namespace hkg
