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

namespace hkg {

constexpr int LS_ROWS = 64;
constexpr int NPART = 16;        // partial sums per local-solve row (a multiple of every wave count)
constexpr int CG_ROWS = 64;
constexpr int CG_COLS = 64;

__device__ __forceinline__ double bwsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ bool inactive(const ProbDev &P, int rhs, int mode) {
    return rhs >= P.nrhs || (mode == 1 && P.active[rhs] != PS_ITER);
}

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
// shape the autotuner may pick gives the same bits.
template <typename T, int WAVES>
__device__ __forceinline__ void local_body(const ProbDev &P, const SubDev &sd, const double *__restrict__ r, int rhs,
                                           double *sh) {
    constexpr int PW = NPART / WAVES;                 // partials per wave
    constexpr int UNR = PW >= 4 ? 1 : 4 / PW;         // loads in flight per thread: PW * UNR
    const int n = sd.nI;
    const int tiles = (n + LS_ROWS - 1) / LS_ROWS;
    const bool coarse = P.two_level && P.m0 > 0;
    const bool restrict_tile = (int)blockIdx.x == tiles;
    double *xd = sh;
    T *xt = reinterpret_cast<T *>(sh + n);
    double *part = sh + n + (n * sizeof(T) + 7) / 8;  // NPART x LS_ROWS
    const int32_t *I = P.I_idx + sd.offI;
    for (int i = threadIdx.x; i < n; i += LS_ROWS * WAVES) {
        const double v = r[I[i]];
        xd[i] = v;
        xt[i] = (T)v;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (restrict_tile) {
        // c_i = Z_i^T r on dof(D_i), same partial-sum order
        const int m = sd.m;
        const double *Zt = P.Zr + sd.offZ;
        for (int q = wv; q < NPART; q += WAVES) {
            double acc = 0.0;
            if (lane < m)
                for (int p = q; p < n; p += NPART) acc = fma(Zt[lane + (int64_t)p * m], xd[p], acc);
            part[q * LS_ROWS + lane] = acc;
        }
        __syncthreads();
        if (wv == 0 && lane < m && coarse) {
            double s = 0.0;
            for (int q = 0; q < NPART; ++q) s += part[q * LS_ROWS + lane];
            P.c[(int64_t)rhs * P.m0 + sd.offm + lane] = s;
        }
        return;
    }
    const int row = blockIdx.x * LS_ROWS + lane;
    const T *M = reinterpret_cast<const T *>(P.Minv) + sd.offSq + row;
    T acc[PW];
#pragma unroll
    for (int k = 0; k < PW; ++k) acc[k] = T(0);
    if (row < n) {
        int c0 = 0;
#pragma unroll UNR
        for (; c0 + NPART <= n; c0 += NPART) {
#pragma unroll
            for (int k = 0; k < PW; ++k) {
                const int col = c0 + wv + k * WAVES;
                acc[k] = fma(M[(int64_t)col * n], xt[col], acc[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < PW; ++k) {
            const int col = c0 + wv + k * WAVES;
            if (col < n) acc[k] = fma(M[(int64_t)col * n], xt[col], acc[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < PW; ++k) part[(wv + k * WAVES) * LS_ROWS + lane] = (double)acc[k];
    __syncthreads();
    if (wv == 0 && row < n) {
        T s = T(0);
        for (int q = 0; q < NPART; ++q) s += (T)part[q * LS_ROWS + lane];
        P.u[(int64_t)rhs * P.sum_nI + sd.offI + row] = P.wloc[sd.offI + row] * (double)s;
    }
}

template <int WAVES>
__global__ __launch_bounds__(LS_ROWS *WAVES) void k_b_local(const ProbDev *__restrict__ probs,
                                                            const WorkItem *__restrict__ items, int mode) {
    extern __shared__ double sh[];
    const WorkItem it = items[blockIdx.y];
    const ProbDev &P = probs[it.p];
    const int rhs = blockIdx.z;
    if (inactive(P, rhs, mode)) return;
    const SubDev sd = P.subs[it.s];
    const int tiles = (sd.nI + LS_ROWS - 1) / LS_ROWS;
    const bool coarse = P.two_level && P.m0 > 0;
    if ((int)blockIdx.x > tiles || ((int)blockIdx.x == tiles && (!coarse || sd.m == 0))) return;
    const double *r = (mode == 0) ? P.xin + (int64_t)rhs * P.ldin : vcol(P, rhs, P.jcur[rhs]);
    if (P.local_f32) local_body<float, WAVES>(P, sd, r, rhs, sh);
    else local_body<double, WAVES>(P, sd, r, rhs, sh);
}

// partial coarse products: ypart[chunk][row] = sum over the chunk's columns of B_0^{-1}[row, col] c[col]
__global__ __launch_bounds__(256) void k_b_coarse_gemv(const ProbDev *__restrict__ probs,
                                                       const WorkItem *__restrict__ cblk, int mode) {
    __shared__ double cs[CG_COLS];
    __shared__ double part[4][CG_ROWS];
    const WorkItem it = cblk[blockIdx.x];
    const ProbDev &P = probs[it.p];
    const int rhs = blockIdx.z;
    if (inactive(P, rhs, mode) || !P.two_level || P.m0 == 0) return;
    const int m0 = P.m0;
    const int rt = it.s / P.nchunk, ch = it.s % P.nchunk;
    const int col0 = ch * CG_COLS;
    const int ncol = min(CG_COLS, m0 - col0);
    for (int i = threadIdx.x; i < ncol; i += 256) cs[i] = P.c[(int64_t)rhs * m0 + col0 + i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row = rt * CG_ROWS + lane;
    double acc = 0.0;
    if (row < m0) {
        const double *B = P.B0inv + row + (int64_t)col0 * m0;
#pragma unroll 4
        for (int k = wv; k < ncol; k += 4) acc = fma(B[(int64_t)k * m0], cs[k], acc);
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && row < m0)
        P.ypart[((int64_t)rhs * P.nchunk + ch) * m0 + row] = part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane];
}

// per subdomain: y_i = sum of the chunk partials (fixed order), u_D += Z_i y_i
__global__ __launch_bounds__(256) void k_b_coarse_add(const ProbDev *__restrict__ probs,
                                                      const WorkItem *__restrict__ items, int mode) {
    __shared__ double ys[64];
    const WorkItem it = items[blockIdx.y];
    const ProbDev &P = probs[it.p];
    const int rhs = blockIdx.z;
    if (inactive(P, rhs, mode) || !P.two_level || P.m0 == 0) return;
    const SubDev sd = P.subs[it.s];
    if (sd.m == 0 || (int)blockIdx.x * 256 >= sd.nI) return;
    if (threadIdx.x < sd.m) {
        double s = 0.0;
        for (int k = 0; k < P.nchunk; ++k) s += P.ypart[((int64_t)rhs * P.nchunk + k) * P.m0 + sd.offm + threadIdx.x];
        ys[threadIdx.x] = s;
    }
    __syncthreads();
    const int a = blockIdx.x * 256 + threadIdx.x;
    if (a >= sd.nI) return;
    const double *z = P.Z + sd.offZ + a;
    double s = 0.0;
    for (int b = 0; b < sd.m; ++b) s = fma(z[(int64_t)b * sd.nI], ys[b], s);
    P.u[(int64_t)rhs * P.sum_nI + sd.offI + a] += s;
}

// z_l = sum over the transpose map of u (fixed order)
__global__ __launch_bounds__(BROWS) void k_b_prolong(const ProbDev *__restrict__ probs,
                                                     const WorkItem *__restrict__ rblk, int mode) {
    const WorkItem it = rblk[blockIdx.x];
    const ProbDev &P = probs[it.p];
    const int rhs = blockIdx.z;
    if (inactive(P, rhs, mode)) return;
    const int l = it.s * BROWS + threadIdx.x;
    if (l >= P.n) return;
    const double *uu = P.u + (int64_t)rhs * P.sum_nI;
    double s = 0.0;
    for (int t = P.tp_ptr[l]; t < P.tp_ptr[l + 1]; ++t) s += uu[P.tp_pos[t]];
    double *z = (mode == 0) ? P.xout + (int64_t)rhs * P.ldout : zcol(P, rhs, P.jcur[rhs]);
    z[l] = s;
}

int32_t batch_apply(const BatchGeom &g, const ProbDev *probs, const WorkItem *items, const WorkItem *rblk,
                    const WorkItem *cblk, int mode, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    const dim3 gl(g.max_tiles + (g.any_coarse ? 1 : 0), g.nitems, g.max_nrhs);
    const size_t shm = (size_t)2 * g.max_nI * sizeof(double) + (size_t)NPART * LS_ROWS * sizeof(double);
    if (ev0) HKG_HIP(hipEventRecord(ev0, s));
    switch (g.local_waves) {
        case 4:
            hipLaunchKernelGGL(k_b_local<4>, gl, dim3(LS_ROWS * 4), shm, s, probs, items,
                               mode);
            break;
        case 16:
            hipLaunchKernelGGL(k_b_local<16>, gl, dim3(LS_ROWS * 16), shm, s, probs,
                               items, mode);
            break;
        default:
            hipLaunchKernelGGL(k_b_local<8>, gl, dim3(LS_ROWS * 8), shm, s, probs, items,
                               mode);
    }
    HKG_HIP(hipGetLastError());
    if (ev1) HKG_HIP(hipEventRecord(ev1, s));
    if (g.any_coarse) {
        hipLaunchKernelGGL(k_b_coarse_gemv, dim3(g.ncblk, 1, g.max_nrhs), dim3(256), 0, s, probs, cblk, mode);
        hipLaunchKernelGGL(k_b_coarse_add, dim3((g.max_nI + 255) / 256, g.nitems, g.max_nrhs), dim3(256), 0, s, probs,
                           items, mode);
    }
    hipLaunchKernelGGL(k_b_prolong, dim3(g.nrblk, 1, g.max_nrhs), dim3(BROWS), 0, s, probs, rblk, mode);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// ------------------------------------------------------------------------------------------------
// Arnoldi step (CGS2) at the device-side index j = jcur
// ------------------------------------------------------------------------------------------------
// w = V[:, j+1] = B Zk[:, j]
__global__ __launch_bounds__(BROWS) void k_b_spmv_next(const ProbDev *__restrict__ probs,
                                                       const WorkItem *__restrict__ rblk) {
    const WorkItem it = rblk[blockIdx.x];
    const ProbDev &P = probs[it.p];
    const int rhs = blockIdx.z;
    if (inactive(P, rhs, 1)) return;
    const int i = it.s * BROWS + threadIdx.x;
    if (i >= P.n) return;
    const int j = P.jcur[rhs];
    const double *x = zcol(P, rhs, j);
    double s = 0.0;
    for (int t = P.rowptr[i]; t < P.rowptr[i + 1]; ++t) s = fma(P.Bval[t], x[P.colidx[t]], s);
    vcol_w(P, rhs, j + 1)[i] = s;
}

// partial sums over the block's rows of x_i . w for i < ncol and of w . w (slot ncol)
__device__ __forceinline__ void bdots(const double *__restrict__ X, int n, int ncol, double wl, int row,
                                      double *__restrict__ out, double *red) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i = 0; i <= ncol; ++i) {
        double s = (i < ncol) ? ((row < n) ? X[(int64_t)i * n + row] * wl : 0.0) : wl * wl;
        s = bwsum(s);
        if (lane == 0) red[wv * (ncol + 1) + i] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= ncol; i += BROWS)
        out[i] = red[i] + red[(ncol + 1) + i] + red[2 * (ncol + 1) + i] + red[3 * (ncol + 1) + i];
}

__global__ __launch_bounds__(BROWS) void k_b_dots(const ProbDev *__restrict__ probs, const WorkItem *__restrict__ rblk) {
    extern __shared__ double red[];
    const WorkItem it = rblk[blockIdx.x];
    const ProbDev &P = probs[it.p];
    const int rhs = blockIdx.z;
    if (inactive(P, rhs, 1)) return;
    const int n = P.n, S = P.restart + 2, j = P.jcur[rhs];
    const double *V = vcol(P, rhs, 0);
    const int row = it.s * BROWS + threadIdx.x;
    const double wl = row < n ? V[(int64_t)(j + 1) * n + row] : 0.0;
    double *part = P.part + ((int64_t)rhs * 2 * P.nblk + it.s) * S;
    bdots(V, n, j + 1, wl, row, part, red);
}

// reduce the pass's partials (wave per entry, fixed order), w -= V h, next partials
__global__ __launch_bounds__(BROWS) void k_b_update(const ProbDev *__restrict__ probs, const WorkItem *__restrict__ rblk,
                                                    int pass) {
    extern __shared__ double sh[];
    const WorkItem it = rblk[blockIdx.x];
    const ProbDev &P = probs[it.p];
    const int rhs = blockIdx.z;
    if (inactive(P, rhs, 1)) return;
    const int n = P.n, m = P.restart, S = m + 2, nb = P.nblk, j = P.jcur[rhs];
    double *V = vcol_w(P, rhs, 0);
    double *w = V + (int64_t)(j + 1) * n;
    const double *pin = P.part + ((int64_t)rhs * 2 * nb + (pass == 1 ? 0 : nb)) * S;
    double *h = sh;
    double *red = sh + S;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i = wv; i <= j + 1; i += BROWS / 64) {
        double s = 0.0;
        for (int b = lane; b < nb; b += 64) s += pin[(int64_t)b * S + i];
        s = bwsum(s);
        if (lane == 0) h[i] = s;
    }
    __syncthreads();
    if (it.s == 0) {
        double *hc = P.hcol + (int64_t)rhs * S;
        for (int i = threadIdx.x; i <= j; i += BROWS) hc[i] = (pass == 1) ? h[i] : hc[i] + h[i];
        if (pass == 1 && threadIdx.x == 0) hc[m + 1] = sqrt(h[j + 1]);
    }
    const int row = it.s * BROWS + threadIdx.x;
    double v = 0.0;
    if (row < n) {
        v = w[row];
        for (int i = 0; i <= j; ++i) v = fma(-V[(int64_t)i * n + row], h[i], v);
        w[row] = v;
    }
    __syncthreads();
    double *pout = P.part + ((int64_t)rhs * 2 * nb + (pass == 1 ? nb : 0)) * S + (int64_t)it.s * S;
    if (pass == 1) {
        bdots(V, n, j + 1, v, row, pout, red);
    } else {
        double s = bwsum(v * v);
        if (lane == 0) red[wv] = s;
        __syncthreads();
        if (threadIdx.x == 0) pout[0] = red[0] + red[1] + red[2] + red[3];
    }
}

// ||w||, v_{j+1} = w / ||w||; block 0: Hessenberg column, Givens rotations, stopping tests
__global__ __launch_bounds__(BROWS) void k_b_finish(const ProbDev *__restrict__ probs, const WorkItem *__restrict__ rblk) {
    const WorkItem it = rblk[blockIdx.x];
    const ProbDev &P = probs[it.p];
    const int rhs = blockIdx.z;
    if (inactive(P, rhs, 1)) return;
    const int n = P.n, m = P.restart, S = m + 2, nb = P.nblk, j = P.jcur[rhs];
    const double *pin = P.part + (int64_t)rhs * 2 * nb * S;
    double nrm2 = 0.0;
    for (int b = (threadIdx.x & 63); b < nb; b += 64) nrm2 += pin[(int64_t)b * S];
    nrm2 = bwsum(nrm2);
    const double hn = sqrt(nrm2);
    double *w = vcol_w(P, rhs, j + 1);
    const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
    const int row = it.s * BROWS + threadIdx.x;
    if (row < n) w[row] *= inv;
    if (it.s == 0 && threadIdx.x == 0) {
        const double *hc = P.hcol + (int64_t)rhs * S;
        double *H = P.H + (int64_t)rhs * (m + 1) * m + (int64_t)j * (m + 1);
        double *cs = P.cs + (int64_t)rhs * m, *sn = P.sn + (int64_t)rhs * m, *g = P.g + (int64_t)rhs * (m + 1);
        double *sc = P.scal + (int64_t)rhs * 8;
        for (int i = 0; i <= j; ++i) H[i] = hc[i];
        H[j + 1] = hn;
        for (int i = 0; i < j; ++i) {
            double t = cs[i] * H[i] + sn[i] * H[i + 1];
            H[i + 1] = -sn[i] * H[i] + cs[i] * H[i + 1];
            H[i] = t;
        }
        const double d = hypot(H[j], H[j + 1]);
        const double c = d > 0.0 ? H[j] / d : 1.0, s = d > 0.0 ? H[j + 1] / d : 0.0;
        cs[j] = c;
        sn[j] = s;
        H[j] = d;
        H[j + 1] = 0.0;
        g[j + 1] = -s * g[j];
        g[j] = c * g[j];
        sc[2] = fabs(g[j + 1]);
        const int conv = fabs(g[j + 1]) <= P.rtol * sc[1];
        const int brk = hn <= 1e-14 * hc[m + 1];
        const int sing = d == 0.0;
        const int itn = ++P.iters[rhs];
        sc[3] = (double)(j + 1);
        if (conv || brk || sing || j + 1 == m || itn >= P.max_iter) {
            P.active[rhs] = PS_CYCLE_END;
            sc[4] = conv ? 1.0 : 0.0;
            sc[5] = sing ? 1.0 : 0.0;
        }
    }
}

// advance j of every active pair (a separate launch: no block of the step reads j after this)
__global__ void k_b_advance(const ProbDev *__restrict__ probs, const int32_t *__restrict__ live, int nlive,
                            int max_nrhs) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nlive * max_nrhs) return;
    const ProbDev &P = probs[live[t / max_nrhs]];
    const int rhs = t % max_nrhs;
    if (rhs < P.nrhs && P.active[rhs] == PS_ITER) P.jcur[rhs] += 1;
}

int32_t batch_arnoldi(const BatchGeom &g, const ProbDev *probs, const WorkItem *rblk, const int32_t *live,
                      hipStream_t s) {
    const dim3 grid(g.nrblk, 1, g.max_nrhs);
    // the restart length of every problem is the same (checked at batch creation)
    hipLaunchKernelGGL(k_b_spmv_next, grid, dim3(BROWS), 0, s, probs, rblk);
    const size_t red = (size_t)4 * (g.restart + 2) * sizeof(double), hbuf = (size_t)(g.restart + 2) * sizeof(double);
    hipLaunchKernelGGL(k_b_dots, grid, dim3(BROWS), red, s, probs, rblk);
    hipLaunchKernelGGL(k_b_update, grid, dim3(BROWS), hbuf + red, s, probs, rblk, 1);
    hipLaunchKernelGGL(k_b_update, grid, dim3(BROWS), hbuf + red, s, probs, rblk, 2);
    hipLaunchKernelGGL(k_b_finish, grid, dim3(BROWS), 0, s, probs, rblk);
    const int pairs = g.nprob * g.max_nrhs;
    hipLaunchKernelGGL(k_b_advance, dim3((pairs + 255) / 256), dim3(256), 0, s, probs, live, g.nprob, g.max_nrhs);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// ------------------------------------------------------------------------------------------------
// restart phase: pairs whose cycle ended (PS_CYCLE_END) or that just joined (PS_NEW)
// ------------------------------------------------------------------------------------------------
// x += Z_k y with y = R^{-1} g from the rotated Hessenberg (PS_CYCLE_END; each block solves the small
// triangle redundantly on one thread), or x = 0 (PS_NEW)
__global__ __launch_bounds__(BROWS) void k_r_update_x(const ProbDev *__restrict__ probs,
                                                      const WorkItem *__restrict__ rblk) {
    extern __shared__ double y[];
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
    if (threadIdx.x == 0) {
        const double *H = P.H + (int64_t)rhs * (m + 1) * m;
        const double *g = P.g + (int64_t)rhs * (m + 1);
        for (int i = jd - 1; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k < jd; ++k) s -= H[i + (int64_t)k * (m + 1)] * y[k];
            y[i] = s / H[i + (int64_t)i * (m + 1)];
        }
    }
    __syncthreads();
    if (r >= P.n) return;
    const double *Zk = zcol(P, rhs, 0);
    double s = x[r];
    for (int i = 0; i < jd; ++i) s = fma(Zk[(int64_t)i * P.n + r], y[i], s);
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
            const double *x = P.x + (int64_t)rhs * P.ldx;
            double s = 0.0;
            for (int t = P.rowptr[i]; t < P.rowptr[i + 1]; ++t) s = fma(P.Bval[t], x[P.colidx[t]], s);
            v -= s;
        }
        vcol_w(P, rhs, 0)[i] = v;
    }
    const double s = bwsum(v * v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < BROWS / 64; ++w) t += red[w];
        P.part[(int64_t)rhs * 2 * P.nblk * (P.restart + 2) + it.s] = t;
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
    const double *pp = P.part + (int64_t)rhs * 2 * P.nblk * (P.restart + 2);
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
    if (fn == 0.0 || rn <= P.rtol * fn || P.iters[rhs] >= P.max_iter) {
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
    P.jcur[rhs] = 0;
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
    hipLaunchKernelGGL(k_r_update_x, grid, dim3(BROWS), (size_t)g.restart * sizeof(double), s, probs, rblk);
    hipLaunchKernelGGL(k_r_residual, grid, dim3(BROWS), 0, s, probs, rblk);
    hipLaunchKernelGGL(k_r_decide, dim3((pairs + 255) / 256), dim3(256), 0, s, probs, live, g.nprob, g.max_nrhs);
    hipLaunchKernelGGL(k_r_start, grid, dim3(BROWS), 0, s, probs, rblk);
    hipLaunchKernelGGL(k_r_activate, dim3((pairs + 255) / 256), dim3(256), 0, s, probs, live, g.nprob, g.max_nrhs);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

}  // namespace hkg
