// Flexible GMRES kernels (right preconditioning, Euclidean inner product) and the CSR operator.
//
// Arnoldi uses classical Gram-Schmidt applied twice (CGS2): each pass needs one batch of dot
// products V_j^T w, which a block computes over its rows for all columns at once; the partial sums
// are then reduced by every block of the next kernel in the same fixed order, so all blocks agree
// bitwise and no atomics are used.  The Hessenberg column, the Givens rotations and the residual
// estimate |g_{j+1}| are updated on the device by one thread per right-hand side.
#include "internal.hpp"
#include "kernels.hpp"

namespace hkg {

constexpr int KB = 256;          // threads per block
constexpr int KR = 1;            // rows per thread
constexpr int ROWS_PER_BLOCK = KB * KR;

// y = B x  (f == nullptr)   or   y = f - B x ; CSR, one thread per row
__global__ __launch_bounds__(256) void k_spmv(int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                                              const double *__restrict__ val, const double *__restrict__ x, int ldx,
                                              double *__restrict__ y, int ldy, const double *__restrict__ f, int ldf,
                                              const int32_t *__restrict__ active) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int rhs = blockIdx.y;
    if (active && !active[rhs]) return;
    const double *xx = x + (int64_t)rhs * ldx;
    double s = 0.0;
    for (int t = rowptr[i]; t < rowptr[i + 1]; ++t) s = fma(val[t], xx[colidx[t]], s);
    if (f) s = f[(int64_t)rhs * ldf + i] - s;
    y[(int64_t)rhs * ldy + i] = s;
}

int32_t spmv(int n, int nrhs, const int32_t *rowptr, const int32_t *colidx, const double *val, const double *x,
             int ldx, double *y, int ldy, const double *f, int ldf, hipStream_t s, const int32_t *active) {
    hipLaunchKernelGGL(k_spmv, dim3((n + 255) / 256, nrhs), dim3(256), 0, s, n, rowptr, colidx, val, x, ldx, y, ldy, f,
                       ldf, active);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// partial sums over this block's rows of x_i . w for i < ncol (x_i = column i of X, ld n) and of
// w . w (slot ncol); written to part[blk * stride + i]
__device__ void block_dots(const double *__restrict__ X, int n, int ncol, const double *w, int row0,
                           double *__restrict__ out, double *red /* 4 x (ncol+1) */) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double wl[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        int r = row0 + threadIdx.x + k * KB;
        wl[k] = r < n ? w[r] : 0.0;
    }
    for (int i = 0; i <= ncol; ++i) {
        double s = 0.0;
        if (i < ncol) {
            const double *xi = X + (int64_t)i * n;
#pragma unroll
            for (int k = 0; k < KR; ++k) {
                int r = row0 + threadIdx.x + k * KB;
                if (r < n) s = fma(xi[r], wl[k], s);
            }
        } else {
#pragma unroll
            for (int k = 0; k < KR; ++k) s = fma(wl[k], wl[k], s);
        }
        s = wsum(s);
        if (lane == 0) red[wv * (ncol + 1) + i] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= ncol; i += KB)
        out[i] = red[i] + red[(ncol + 1) + i] + red[2 * (ncol + 1) + i] + red[3 * (ncol + 1) + i];
}

// first CGS pass dot products: part_a[blk][i] = V_i . w (i <= j), part_a[blk][j+1] = w . w
__global__ __launch_bounds__(KB) void k_cgs_dots(GmresDev G, int j) {
    extern __shared__ double red[];
    const int rhs = blockIdx.y;
    if (!G.active[rhs]) return;
    const int n = G.n, S = G.restart + 2;
    const double *V = G.V + (int64_t)rhs * n * (G.restart + 1);
    const double *w = V + (int64_t)(j + 1) * n;
    double *part = G.part + ((int64_t)rhs * 2 * G.nblk + blockIdx.x) * S;
    block_dots(G.VD + (int64_t)rhs * n * (G.restart + 1), n, j + 1, w, blockIdx.x * ROWS_PER_BLOCK, part, red);
}

// reduce pass-p partial sums (fixed order), w -= V h; pass 1 then forms the pass-2 dot products,
// pass 2 the partial squared norm.  Block 0 accumulates h into hcol.
__global__ __launch_bounds__(KB) void k_cgs_update(GmresDev G, int j, int pass) {
    extern __shared__ double sh[];
    const int rhs = blockIdx.y;
    if (!G.active[rhs]) return;
    const int n = G.n, S = G.restart + 2, nb = G.nblk;
    double *V = G.V + (int64_t)rhs * n * (G.restart + 1);
    double *w = V + (int64_t)(j + 1) * n;
    const double *pin = G.part + ((int64_t)rhs * 2 * nb + (pass == 1 ? 0 : nb)) * S;
    double *h = sh;                    // j + 2
    double *red = sh + (G.restart + 2);
    {
        // h[i] = sum over blocks of the partials: one wave per i, lanes over blocks, fixed shuffle tree
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        for (int i = wv; i <= j + 1; i += KB / 64) {
            double s = 0.0;
            for (int b = lane; b < nb; b += 64) s += pin[(int64_t)b * S + i];
            s = wsum(s);
            if (lane == 0) h[i] = s;
        }
    }
    __syncthreads();
    if (blockIdx.x == 0) {
        double *hc = G.hcol + (int64_t)rhs * (G.restart + 2);
        for (int i = threadIdx.x; i <= j; i += KB) hc[i] = (pass == 1) ? h[i] : hc[i] + h[i];
        if (pass == 1 && threadIdx.x == 0) hc[G.restart + 1] = sqrt(h[j + 1]);   // ||w|| before orthogonalisation
    }
    const int row0 = blockIdx.x * ROWS_PER_BLOCK;
    double wl[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        int r = row0 + threadIdx.x + k * KB;
        double v = 0.0;
        if (r < n) {
            v = w[r];
            for (int i = 0; i <= j; ++i) v = fma(-V[(int64_t)i * n + r], h[i], v);
            w[r] = v;
        }
        wl[k] = v;
    }
    __syncthreads();
    double *pout = G.part + ((int64_t)rhs * 2 * nb + (pass == 1 ? nb : 0)) * S + (int64_t)blockIdx.x * S;
    if (pass == 1) {
        block_dots(G.VD + (int64_t)rhs * n * (G.restart + 1), n, j + 1, w, row0, pout, red);
    } else {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < KR; ++k) s = fma(wl[k], wl[k], s);
        s = wsum(s);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) pout[0] = red[0] + red[1] + red[2] + red[3];
    }
}

// ||w||, v_{j+1} = w / ||w||, and (block 0, thread 0) the Hessenberg column with Givens rotations
__global__ __launch_bounds__(KB) void k_arnoldi_finish(GmresDev G, int j, double tol_abs_scale) {
    const int rhs = blockIdx.y;
    if (!G.active[rhs]) return;
    const int n = G.n, S = G.restart + 2, nb = G.nblk, m = G.restart;
    const double *pin = G.part + (int64_t)rhs * 2 * nb * S;
    double nrm2 = 0.0;
    for (int b = (threadIdx.x & 63); b < nb; b += 64) nrm2 += pin[(int64_t)b * S];
    nrm2 = wsum(nrm2);                 // the same fixed tree in every wave of every block
    const double hn = sqrt(nrm2);
    double *V = G.V + (int64_t)rhs * n * (m + 1);
    double *w = V + (int64_t)(j + 1) * n;
    const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
    const int row0 = blockIdx.x * ROWS_PER_BLOCK;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        int r = row0 + threadIdx.x + k * KB;
        if (r < n) {
            w[r] *= inv;
            if (G.dk) G.DV[(int64_t)rhs * n * (m + 1) + (int64_t)(j + 1) * n + r] *= inv;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const double *hc = G.hcol + (int64_t)rhs * (m + 2);
        // ||w|| before the orthogonalisation: measured for the Euclidean product; in the D_k product
        // the norm of its D_k-orthogonal decomposition (the h_i of this column and the new norm)
        double w0 = hc[m + 1];
        if (G.dk) {
            double q = hn * hn;
            for (int i = 0; i <= j; ++i) q = fma(hc[i], hc[i], q);
            w0 = sqrt(q);
        }
        double *H = G.H + (int64_t)rhs * (m + 1) * m + (int64_t)j * (m + 1);
        double *cs = G.cs + (int64_t)rhs * m, *sn = G.sn + (int64_t)rhs * m, *g = G.g + (int64_t)rhs * (m + 1);
        double *sc = G.scal + (int64_t)rhs * 8;
        for (int i = 0; i <= j; ++i) H[i] = hc[i];
        H[j + 1] = hn;
        for (int i = 0; i < j; ++i) {
            double t = cs[i] * H[i] + sn[i] * H[i + 1];
            H[i + 1] = -sn[i] * H[i] + cs[i] * H[i + 1];
            H[i] = t;
        }
        double d = hypot(H[j], H[j + 1]);
        double c = d > 0.0 ? H[j] / d : 1.0, s = d > 0.0 ? H[j + 1] / d : 0.0;
        cs[j] = c;
        sn[j] = s;
        H[j] = d;
        H[j + 1] = 0.0;
        g[j + 1] = -s * g[j];
        g[j] = c * g[j];
        sc[2] = fabs(g[j + 1]);
        const int conv = fabs(g[j + 1]) <= tol_abs_scale * sc[1];
        const int brk = hn <= 1e-14 * w0;
        const int sing = d == 0.0;
        const int it = ++G.iters[rhs];
        if (conv || brk || sing || j + 1 == m || it >= G.max_iter) {
            G.active[rhs] = 0;
            // columns used in this cycle; a singular rotated column (zero diagonal of R) is left
            // out of the back substitution, and the host stops the right-hand side (sc[5])
            sc[3] = (double)(sing ? j : j + 1);
            sc[4] = conv ? 1.0 : 0.0;
            sc[5] = sing ? 1.0 : 0.0;
        }
    }
}

__global__ void k_dk_norm(GmresDev G, int j, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                          const double *__restrict__ Aval, const double *__restrict__ Sval, double k2);

int32_t gmres_arnoldi_step(const GmresDev &G, int j, double rtol, hipStream_t s, const int32_t *rowptr,
                           const int32_t *colidx, const double *Aval, const double *Sval, double k2) {
    const dim3 grid(G.nblk, G.nrhs);
    const size_t red_bytes = (size_t)4 * (G.restart + 2) * sizeof(double);
    hipLaunchKernelGGL(k_cgs_dots, grid, dim3(KB), red_bytes, s, G, j);
    hipLaunchKernelGGL(k_cgs_update, grid, dim3(KB), red_bytes + (G.restart + 2) * sizeof(double), s, G, j, 1);
    hipLaunchKernelGGL(k_cgs_update, grid, dim3(KB), red_bytes + (G.restart + 2) * sizeof(double), s, G, j, 2);
    if (G.dk) hipLaunchKernelGGL(k_dk_norm, grid, dim3(KB), 0, s, G, j, rowptr, colidx, Aval, Sval, k2);
    hipLaunchKernelGGL(k_arnoldi_finish, grid, dim3(KB), 0, s, G, j, rtol);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// cycle start: beta = ||r||, v_0 = r / beta, g = beta e_1, active if beta > rtol ||f|| (per rhs).
// r is V[:, 0] already (the residual was written there); fnorm is scal[1].
__global__ __launch_bounds__(KB) void k_cycle_start(GmresDev G, const double *__restrict__ rnorm, double rtol,
                                                    const int32_t *__restrict__ want) {
    const int rhs = blockIdx.y;
    const int n = G.n, m = G.restart;
    const double beta = rnorm[rhs];
    double *sc = G.scal + (int64_t)rhs * 8;
    const int act = want[rhs] && gmres_keeps_going(beta, sc[1], rtol) && beta > 0.0;
    double *V = G.V + (int64_t)rhs * n * (m + 1);
    const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
    const int row0 = blockIdx.x * ROWS_PER_BLOCK;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        int r = row0 + threadIdx.x + k * KB;
        if (r < n) {
            V[r] *= inv;
            if (G.dk && want[rhs]) G.DV[(int64_t)rhs * n * (m + 1) + r] *= inv;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double *g = G.g + (int64_t)rhs * (m + 1);
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        sc[0] = beta;
        sc[2] = beta;
        sc[3] = 0.0;
        sc[4] = 0.0;
        sc[5] = 0.0;
        G.active[rhs] = act;
    }
}

int32_t gmres_cycle_start(const GmresDev &G, const double *rnorm, double rtol, const int32_t *want, hipStream_t s) {
    hipLaunchKernelGGL(k_cycle_start, dim3(G.nblk, G.nrhs), dim3(KB), 0, s, G, rnorm, rtol, want);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// y = R^{-1} g on the jd x jd rotated Hessenberg (one thread per rhs), then x += X y with X the
// preconditioned directions Zk (flexible, right preconditioning) or the basis V (left preconditioning)
__global__ __launch_bounds__(KB) void k_cycle_update(GmresDev G, double *__restrict__ x, int ldx,
                                                     const double *__restrict__ Xb, int64_t xstride) {
    extern __shared__ double y[];
    const int rhs = blockIdx.y;
    const int n = G.n, m = G.restart;
    const int jd = (int)G.scal[(int64_t)rhs * 8 + 3];
    if (jd <= 0) return;
    if (threadIdx.x == 0) {
        const double *H = G.H + (int64_t)rhs * (m + 1) * m;
        const double *g = G.g + (int64_t)rhs * (m + 1);
        for (int i = jd - 1; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k < jd; ++k) s -= H[i + (int64_t)k * (m + 1)] * y[k];
            y[i] = s / H[i + (int64_t)i * (m + 1)];
        }
    }
    __syncthreads();
    const double *Zk = Xb + (int64_t)rhs * xstride;
    const int row0 = blockIdx.x * ROWS_PER_BLOCK;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        int r = row0 + threadIdx.x + k * KB;
        if (r < n) {
            double s = x[(int64_t)rhs * ldx + r];
            for (int i = 0; i < jd; ++i) s = fma(Zk[(int64_t)i * n + r], y[i], s);
            x[(int64_t)rhs * ldx + r] = s;
        }
    }
}

int32_t gmres_cycle_update(const GmresDev &G, double *x, int ldx, hipStream_t s) {
    const double *X = G.dk ? G.V : G.Zk;
    const int64_t stride = (int64_t)G.n * (G.dk ? G.restart + 1 : G.restart);
    hipLaunchKernelGGL(k_cycle_update, dim3(G.nblk, G.nrhs), dim3(KB), (size_t)(G.restart + 1) * sizeof(double), s, G, x,
                       ldx, X, stride);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// D_k w for w = V[:, j+1] (D_k = A + k2 S, one thread per row, nonzeros in index order) into
// DV[:, j+1], and the block's partial sum of w . D_k w (slot 0 of the pass-2 partials)
__global__ __launch_bounds__(KB) void k_dk_norm(GmresDev G, int j, const int32_t *__restrict__ rowptr,
                                                const int32_t *__restrict__ colidx, const double *__restrict__ Aval,
                                                const double *__restrict__ Sval, double k2) {
    __shared__ double red[KB / 64];
    const int rhs = blockIdx.y;
    if (j >= 0 && !G.active[rhs]) return;
    const int n = G.n, m = G.restart, S = m + 2;
    const double *w = G.V + (int64_t)rhs * n * (m + 1) + (int64_t)(j + 1) * n;
    double *dw = G.DV + (int64_t)rhs * n * (m + 1) + (int64_t)(j + 1) * n;
    const int i = blockIdx.x * ROWS_PER_BLOCK + threadIdx.x;
    double s = 0.0;
    if (i < n) {
        double d = 0.0;
        for (int t = rowptr[i]; t < rowptr[i + 1]; ++t) d = fma(fma(k2, Sval[t], Aval[t]), w[colidx[t]], d);
        dw[i] = d;
        s = w[i] * d;
    }
    s = wsum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        G.part[((int64_t)rhs * 2 * G.nblk + blockIdx.x) * S] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_dk_reduce(GmresDev G, double *__restrict__ out) {
    const int rhs = blockIdx.x;
    if (threadIdx.x == 0) {
        const int S = G.restart + 2;
        const double *pin = G.part + (int64_t)rhs * 2 * G.nblk * S;
        double s = 0.0;
        for (int b = 0; b < G.nblk; ++b) s += pin[(int64_t)b * S];
        out[rhs] = sqrt(fmax(s, 0.0));
    }
}

int32_t gmres_dk_norm(const GmresDev &G, int j, const int32_t *rowptr, const int32_t *colidx, const double *Aval,
                      const double *Sval, double k2, hipStream_t s) {
    hipLaunchKernelGGL(k_dk_norm, dim3(G.nblk, G.nrhs), dim3(KB), 0, s, G, j, rowptr, colidx, Aval, Sval, k2);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

int32_t gmres_dk_reduce(const GmresDev &G, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_dk_reduce, dim3(G.nrhs), dim3(64), 0, s, G, out);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// out[rhs] = ||x_rhs||_2 via per-block partials reduced in a fixed order
__global__ __launch_bounds__(KB) void k_norm_part(int n, const double *__restrict__ x, int ldx, double *__restrict__ part) {
    __shared__ double red[4];
    const int rhs = blockIdx.y;
    const int row0 = blockIdx.x * ROWS_PER_BLOCK;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        int r = row0 + threadIdx.x + k * KB;
        if (r < n) {
            double v = x[(int64_t)rhs * ldx + r];
            s = fma(v, v, s);
        }
    }
    s = wsum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[(int64_t)rhs * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_norm_final(int nblk, const double *__restrict__ part, double *__restrict__ out) {
    const int rhs = blockIdx.x;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += part[(int64_t)rhs * nblk + b];
        out[rhs] = sqrt(s);
    }
}

int32_t vec_norms(int n, int nrhs, const double *x, int ldx, double *out, double *part, int nblk, hipStream_t s) {
    hipLaunchKernelGGL(k_norm_part, dim3(nblk, nrhs), dim3(KB), 0, s, n, x, ldx, part);
    hipLaunchKernelGGL(k_norm_final, dim3(nrhs), dim3(64), 0, s, nblk, part, out);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

int gmres_rows_per_block() { return ROWS_PER_BLOCK; }

}  // namespace hkg
