// One application z = M^{-1} r of the two-level additive Schwarz preconditioner (eq. (2.23)):
//
//   local:     u_D = W_D B_D^{-1} R_D r          (eq. (2.22); R_D gathers dof(D) from r)
//   restrict:  c_i = Z_i^T R_i r                 (R_0 = Z^T on nodal residuals)
//   coarse:    y = B_0^{-1} c
//   prolong:   u_D += Z_i y_i ; z_l = sum over the subdomains holding l of u_D[l]
//
// B_D^{-1} and B_0^{-1} are applied as products with the inverses formed at setup from the LU
// factors (the same bytes as reading L and U, with no sequential dependency).  The local kernel
// also forms the restriction from the same gathered residual (its last tile per subdomain reads
// Z_i^T); the coarse product is split over column chunks whose partial sums are reduced in a fixed
// order by the kernel that adds Z_i y_i; the final sum walks a transpose map (dof -> positions in
// the concatenated local vectors) in a fixed order.  No atomics: z is bitwise reproducible.
//
// Every kernel is HBM-bound; the local inverses dominate (sum n_D^2 words per application).
// Inside FGMRES every kernel first checks its right-hand side's active flag, so iterations issued
// after convergence cost only their launch.
#include "internal.hpp"
#include "kernels.hpp"

namespace hkg {

constexpr int LS_ROWS = 64;     // rows per block (one per lane)
constexpr int LS_WAVES = 8;     // waves splitting the columns
constexpr int CG_ROWS = 64;
constexpr int CG_COLS = 64;     // column chunk of the split coarse product

// Tiles 0..T-1 of subdomain D: u_D[rows] = w .* (B_D^{-1} r_D)[rows].  Tile T: c_i = Z_i^T r_D.
template <typename T>
__global__ __launch_bounds__(LS_ROWS * LS_WAVES) void k_local_solve(const SubDev *__restrict__ subs,
                                                                    const int32_t *__restrict__ I_idx,
                                                                    const double *__restrict__ wloc,
                                                                    const T *__restrict__ Minv,
                                                                    const double *__restrict__ Zr,
                                                                    const double *__restrict__ r, int ldr,
                                                                    double *__restrict__ u, int64_t ldu,
                                                                    double *__restrict__ c, int m0,
                                                                    const int32_t *__restrict__ active) {
    extern __shared__ double sh[];
    const int rhs = blockIdx.z;
    if (active && !active[rhs]) return;
    const SubDev sd = subs[blockIdx.y];
    const int n = sd.nI;
    const int tiles = (n + LS_ROWS - 1) / LS_ROWS;
    const bool restrict_tile = (int)blockIdx.x == tiles;
    if ((int)blockIdx.x > tiles || (restrict_tile && (sd.m == 0 || c == nullptr))) return;
    if (!restrict_tile && Minv == nullptr) {
        // coarse correction alone (the first-level solves of a nested decomposition run elsewhere):
        // the local vectors start at zero and receive Z_i y_i
        const int row = blockIdx.x * LS_ROWS + threadIdx.x;
        if (threadIdx.x < LS_ROWS && row < n) u[(int64_t)rhs * ldu + sd.offI + row] = 0.0;
        return;
    }
    double *xd = sh;                                  // r_D in double
    T *xt = reinterpret_cast<T *>(sh + n);            // r_D in T (aliases nothing when T = double)
    double *part = sh + n + (n * sizeof(T) + 7) / 8;
    const double *rr = r + (int64_t)rhs * ldr;
    const int32_t *I = I_idx + sd.offI;
    for (int i = threadIdx.x; i < n; i += LS_ROWS * LS_WAVES) {
        const double v = rr[I[i]];
        xd[i] = v;
        xt[i] = (T)v;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (restrict_tile) {
        // c_b = sum_p Z_i[p, b] r_D[p]; Zr holds Z_i row-major (p * m + b), i.e. Z_i^T column-major
        const int m = sd.m;
        const double *Zt = Zr + sd.offZ;
        double acc = 0.0;
        if (lane < m)
            for (int p = wv; p < n; p += LS_WAVES) acc = fma(Zt[lane + (int64_t)p * m], xd[p], acc);
        part[wv * LS_ROWS + lane] = acc;
        __syncthreads();
        if (wv == 0 && lane < m) {
            double s = 0.0;
            for (int w = 0; w < LS_WAVES; ++w) s += part[w * LS_ROWS + lane];
            c[(int64_t)rhs * m0 + sd.offm + lane] = s;
        }
        return;
    }
    const int row = blockIdx.x * LS_ROWS + lane;
    const T *M = Minv + sd.offM;
    const int ldm = sd.ldM;
    T acc = T(0);
    if (row < n) {
        int col = wv;
        for (; col + 3 * LS_WAVES < n; col += 4 * LS_WAVES) {
            T a0 = M[row + (int64_t)col * ldm];
            T a1 = M[row + (int64_t)(col + LS_WAVES) * ldm];
            T a2 = M[row + (int64_t)(col + 2 * LS_WAVES) * ldm];
            T a3 = M[row + (int64_t)(col + 3 * LS_WAVES) * ldm];
            acc = fma(a0, xt[col], acc);
            acc = fma(a1, xt[col + LS_WAVES], acc);
            acc = fma(a2, xt[col + 2 * LS_WAVES], acc);
            acc = fma(a3, xt[col + 3 * LS_WAVES], acc);
        }
        for (; col < n; col += LS_WAVES) acc = fma(M[row + (int64_t)col * ldm], xt[col], acc);
    }
    part[wv * LS_ROWS + lane] = (double)acc;
    __syncthreads();
    if (wv == 0 && row < n) {
        T s = T(0);
        for (int w = 0; w < LS_WAVES; ++w) s += (T)part[w * LS_ROWS + lane];
        u[(int64_t)rhs * ldu + sd.offI + row] = wloc[sd.offI + row] * (double)s;
    }
}

// partial coarse products: ypart[chunk][row] = sum over the chunk's columns of B_0^{-1}[row, col] c[col]
__global__ __launch_bounds__(256) void k_coarse_gemv(const double *__restrict__ Binv, int m0, const double *__restrict__ c,
                                                     double *__restrict__ ypart, const int32_t *__restrict__ active) {
    __shared__ double cs[CG_COLS];
    __shared__ double part[4][CG_ROWS];
    const int rhs = blockIdx.z;
    if (active && !active[rhs]) return;
    const int col0 = blockIdx.y * CG_COLS;
    const int ncol = min(CG_COLS, m0 - col0);
    for (int i = threadIdx.x; i < ncol; i += 256) cs[i] = c[(int64_t)rhs * m0 + col0 + i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row = blockIdx.x * CG_ROWS + lane;
    double acc = 0.0;
    if (row < m0) {
        const double *B = Binv + row + (int64_t)col0 * m0;
#pragma unroll 4
        for (int k = wv; k < ncol; k += 4) acc = fma(B[(int64_t)k * m0], cs[k], acc);
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && row < m0)
        ypart[((int64_t)rhs * gridDim.y + blockIdx.y) * m0 + row] = part[0][lane] + part[1][lane] + part[2][lane] +
                                                                    part[3][lane];
}

// per subdomain: y_i = sum of the chunk partials (fixed order), then u_D += Z_i y_i
__global__ __launch_bounds__(256) void k_coarse_add(const SubDev *__restrict__ subs, int m0, int nchunk,
                                                    const double *__restrict__ ypart, const double *__restrict__ Z,
                                                    double *__restrict__ u, int64_t ldu,
                                                    const int32_t *__restrict__ active) {
    __shared__ double ys[64];
    const int rhs = blockIdx.z;
    if (active && !active[rhs]) return;
    const SubDev sd = subs[blockIdx.y];
    if (sd.m == 0) return;
    if (threadIdx.x < sd.m) {
        double s = 0.0;
        for (int k = 0; k < nchunk; ++k) s += ypart[((int64_t)rhs * nchunk + k) * m0 + sd.offm + threadIdx.x];
        ys[threadIdx.x] = s;
    }
    __syncthreads();
    const int a = blockIdx.x * 256 + threadIdx.x;
    if (a >= sd.nI) return;
    const double *z = Z + sd.offZ + a;
    double s = 0.0;
    for (int b = 0; b < sd.m; ++b) s = fma(z[(int64_t)b * sd.nI], ys[b], s);
    u[(int64_t)rhs * ldu + sd.offI + a] += s;
}

// z_l = sum over the transpose map of u (fixed order); accumulate: z_l += that sum
__global__ __launch_bounds__(256) void k_prolong(int n, const int32_t *__restrict__ tp_ptr,
                                                 const int32_t *__restrict__ tp_pos, const double *__restrict__ u,
                                                 int64_t ldu, double *__restrict__ z, int ldz,
                                                 const int32_t *__restrict__ active, int accumulate) {
    const int rhs = blockIdx.y;
    if (active && !active[rhs]) return;
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= n) return;
    const double *uu = u + (int64_t)rhs * ldu;
    double s = 0.0;
    for (int t = tp_ptr[l]; t < tp_ptr[l + 1]; ++t) s += uu[tp_pos[t]];
    double *zz = z + (int64_t)rhs * ldz + l;
    *zz = accumulate ? *zz + s : s;
}

int32_t apply_two_level(const ApplyPlan &p, const double *r, int ldr, double *z, int ldz, hipStream_t s) {
    const int tiles = (p.maxnI + LS_ROWS - 1) / LS_ROWS;
    const int64_t ldu = p.sum_nI;
    const bool coarse = p.two_level && p.m0 > 0;
    if (p.ev0) HKG_HIP(hipEventRecord(p.ev0, s));
    const dim3 gl(tiles + (coarse ? 1 : 0), p.nsub, p.nrhs);
    if (p.local_f32) {
        size_t shm = (size_t)p.maxnI * sizeof(double) + ((p.maxnI * sizeof(float) + 7) / 8) * 8 +
                     LS_ROWS * LS_WAVES * sizeof(double);
        hipLaunchKernelGGL(k_local_solve<float>, gl, dim3(LS_ROWS * LS_WAVES), shm, s, p.d_sub, p.I_idx, p.winv_loc,
                           (const float *)p.Minv, p.Zr, r, ldr, p.u, ldu, coarse ? p.c : nullptr, p.m0, p.active);
    } else {
        size_t shm = (size_t)2 * p.maxnI * sizeof(double) + LS_ROWS * LS_WAVES * sizeof(double);
        hipLaunchKernelGGL(k_local_solve<double>, gl, dim3(LS_ROWS * LS_WAVES), shm, s, p.d_sub, p.I_idx, p.winv_loc,
                           (const double *)p.Minv, p.Zr, r, ldr, p.u, ldu, coarse ? p.c : nullptr, p.m0, p.active);
    }
    HKG_HIP(hipGetLastError());
    if (p.ev1) HKG_HIP(hipEventRecord(p.ev1, s));
    if (coarse) {
        const int nchunk = (p.m0 + CG_COLS - 1) / CG_COLS;
        hipLaunchKernelGGL(k_coarse_gemv, dim3((p.m0 + CG_ROWS - 1) / CG_ROWS, nchunk, p.nrhs), dim3(256), 0, s, p.B0inv,
                           p.m0, p.c, p.ypart, p.active);
        hipLaunchKernelGGL(k_coarse_add, dim3((p.maxnI + 255) / 256, p.nsub, p.nrhs), dim3(256), 0, s, p.d_sub, p.m0,
                           nchunk, p.ypart, p.Z, p.u, ldu, p.active);
        HKG_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_prolong, dim3((p.n_dof + 255) / 256, p.nrhs), dim3(256), 0, s, p.n_dof, p.tp_ptr, p.tp_pos,
                       p.u, ldu, z, ldz, p.active, p.accumulate);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

int apply_ypart_chunks(int m0) { return (m0 + CG_COLS - 1) / CG_COLS; }

// Zr = Z_i transposed per subdomain (row-major n_I x m_i)
__global__ __launch_bounds__(256) void k_transpose_basis(const SubDev *__restrict__ subs, const double *__restrict__ Z,
                                                         double *__restrict__ Zr) {
    const SubDev sd = subs[blockIdx.y];
    const int64_t nm = (int64_t)sd.nI * sd.m;
    for (int64_t q = blockIdx.x * 256 + threadIdx.x; q < nm; q += (int64_t)gridDim.x * 256) {
        const int b = (int)(q / sd.nI), a = (int)(q % sd.nI);
        Zr[sd.offZ + (int64_t)a * sd.m + b] = Z[sd.offZ + q];
    }
}

int32_t transpose_basis(const SubDev *d_sub, int nsub, const double *Z, double *Zr, hipStream_t s) {
    hipLaunchKernelGGL(k_transpose_basis, dim3(64, nsub), dim3(256), 0, s, d_sub, Z, Zr);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

__global__ __launch_bounds__(256) void k_tp_coarse(const SubDev *__restrict__ subs, const int32_t *__restrict__ tp_pos,
                                                   const int32_t *__restrict__ tp_sub, int64_t ntp,
                                                   TpCoarse *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= ntp) return;
    const SubDev &sd = subs[tp_sub[t]];
    // a subdomain without coarse vectors points at entry 0 (read, then masked, by the prolongation)
    if (sd.m > 0) out[t] = {sd.offZ + (int64_t)(tp_pos[t] - sd.offI) * sd.m, sd.offm, sd.m};
    else out[t] = {0, 0, 0};
}

int32_t tp_coarse(const SubDev *d_sub, const int32_t *tp_pos, const int32_t *tp_sub, int64_t ntp, TpCoarse *out,
                  hipStream_t s) {
    if (ntp == 0) return HKG_OK;
    hipLaunchKernelGGL(k_tp_coarse, dim3((unsigned)((ntp + 255) / 256)), dim3(256), 0, s, d_sub, tp_pos, tp_sub, ntp, out);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

}  // namespace hkg
