// One application z = M^{-1} r of the two-level additive Schwarz preconditioner (eq. (2.23)):
//
//   local:     u_D = W_D B_D^{-1} R_D r          (eq. (2.22); R_D gathers dof(D) from r)
//   restrict:  c_i = Z_i^T R_i r                 (R_0 = Z^T on nodal residuals)
//   coarse:    y = B_0^{-1} c
//   prolong:   t_D = u_D + Z_i y_i ; z_l = sum over the subdomains holding l of t_D[l]
//
// B_D^{-1} and B_0^{-1} are applied as products with the inverses formed at setup from the LU
// factors (the same bytes as reading L and U, with no sequential dependency).  The final sum walks
// a transpose map (dof -> positions in the concatenated local vectors) in a fixed order, so z is
// bitwise reproducible and needs no atomics.
//
// Every kernel is HBM-bound: the local inverses dominate (sum n_D^2 words per application).
#include "internal.hpp"
#include "kernels.hpp"

namespace hkg {

constexpr int LS_ROWS = 64;     // rows of B_D^{-1} per block (one per lane)
constexpr int LS_WAVES = 8;     // waves splitting the columns
constexpr int CG_ROWS = 64;

// u_D[rows of tile] = w .* (B_D^{-1} r_D)[rows], r_D gathered into LDS
template <typename T>
__global__ __launch_bounds__(LS_ROWS * LS_WAVES) void k_local_solve(const SubDev *__restrict__ subs,
                                                                    const int32_t *__restrict__ I_idx,
                                                                    const double *__restrict__ wloc,
                                                                    const T *__restrict__ Minv, const double *__restrict__ r,
                                                                    int ldr, double *__restrict__ u, int64_t ldu) {
    extern __shared__ double sh[];
    const SubDev sd = subs[blockIdx.y];
    const int n = sd.nI;
    const int row0 = blockIdx.x * LS_ROWS;
    if (row0 >= n) return;
    const int rhs = blockIdx.z;
    T *xs = reinterpret_cast<T *>(sh);
    double *part = sh + ((n * sizeof(T) + 7) / 8);
    const double *rr = r + (int64_t)rhs * ldr;
    const int32_t *I = I_idx + sd.offI;
    for (int i = threadIdx.x; i < n; i += LS_ROWS * LS_WAVES) xs[i] = (T)rr[I[i]];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row = row0 + lane;
    const T *M = Minv + sd.offSq;
    T acc = T(0);
    if (row < n) {
        int c = wv;
        for (; c + 3 * LS_WAVES < n; c += 4 * LS_WAVES) {
            T a0 = M[row + (int64_t)c * n];
            T a1 = M[row + (int64_t)(c + LS_WAVES) * n];
            T a2 = M[row + (int64_t)(c + 2 * LS_WAVES) * n];
            T a3 = M[row + (int64_t)(c + 3 * LS_WAVES) * n];
            acc = fma(a0, xs[c], acc);
            acc = fma(a1, xs[c + LS_WAVES], acc);
            acc = fma(a2, xs[c + 2 * LS_WAVES], acc);
            acc = fma(a3, xs[c + 3 * LS_WAVES], acc);
        }
        for (; c < n; c += LS_WAVES) acc = fma(M[row + (int64_t)c * n], xs[c], acc);
    }
    part[wv * LS_ROWS + lane] = (double)acc;
    __syncthreads();
    if (wv == 0 && row < n) {
        T s = T(0);
        for (int w = 0; w < LS_WAVES; ++w) s += (T)part[w * LS_ROWS + lane];
        u[(int64_t)rhs * ldu + sd.offI + row] = wloc[sd.offI + row] * (double)s;
    }
}

// c_i = Z_i^T r_D: one block per subdomain, one wave per coarse vector
__global__ __launch_bounds__(256) void k_restrict(const SubDev *__restrict__ subs, const int32_t *__restrict__ I_idx,
                                                  const double *__restrict__ Z, const double *__restrict__ r, int ldr,
                                                  double *__restrict__ c, int m0) {
    extern __shared__ double xs[];
    const SubDev sd = subs[blockIdx.x];
    if (sd.m == 0) return;
    const int n = sd.nI, rhs = blockIdx.y;
    const double *rr = r + (int64_t)rhs * ldr;
    for (int i = threadIdx.x; i < n; i += 256) xs[i] = rr[I_idx[sd.offI + i]];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int b = wv; b < sd.m; b += 4) {
        const double *z = Z + sd.offZ + (int64_t)b * n;
        double s = 0.0;
        for (int i = lane; i < n; i += 64) s = fma(z[i], xs[i], s);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) c[(int64_t)rhs * m0 + sd.offm + b] = s;
    }
}

// y = B_0^{-1} c, rows split over blocks, columns over the block's waves
__global__ __launch_bounds__(256) void k_coarse_gemv(const double *__restrict__ Binv, int m0, const double *__restrict__ c,
                                                     double *__restrict__ y) {
    extern __shared__ double sh[];
    const int rhs = blockIdx.y;
    const double *cc = c + (int64_t)rhs * m0;
    double *xs = sh;
    double *part = sh + m0;
    for (int i = threadIdx.x; i < m0; i += 256) xs[i] = cc[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row = blockIdx.x * CG_ROWS + lane;
    double acc = 0.0;
    if (row < m0) {
        int col = wv;
        for (; col + 12 < m0; col += 16) {
            double a0 = Binv[row + (int64_t)col * m0];
            double a1 = Binv[row + (int64_t)(col + 4) * m0];
            double a2 = Binv[row + (int64_t)(col + 8) * m0];
            double a3 = Binv[row + (int64_t)(col + 12) * m0];
            acc = fma(a0, xs[col], acc);
            acc = fma(a1, xs[col + 4], acc);
            acc = fma(a2, xs[col + 8], acc);
            acc = fma(a3, xs[col + 12], acc);
        }
        for (; col < m0; col += 4) acc = fma(Binv[row + (int64_t)col * m0], xs[col], acc);
    }
    part[wv * 64 + lane] = acc;
    __syncthreads();
    if (wv == 0 && row < m0) y[(int64_t)rhs * m0 + row] = part[lane] + part[64 + lane] + part[128 + lane] + part[192 + lane];
}

// t_D = u_D + Z_i y_i (in place in u)
__global__ __launch_bounds__(256) void k_add_coarse(const SubDev *__restrict__ subs, const double *__restrict__ Z,
                                                    const double *__restrict__ y, int m0, double *__restrict__ u,
                                                    int64_t ldu) {
    const SubDev sd = subs[blockIdx.y];
    const int a = blockIdx.x * 256 + threadIdx.x;
    if (a >= sd.nI || sd.m == 0) return;
    const int rhs = blockIdx.z;
    const double *yy = y + (int64_t)rhs * m0 + sd.offm;
    const double *z = Z + sd.offZ + a;
    double s = 0.0;
    for (int b = 0; b < sd.m; ++b) s = fma(z[(int64_t)b * sd.nI], yy[b], s);
    u[(int64_t)rhs * ldu + sd.offI + a] += s;
}

// z_l = sum over the transpose map of t (fixed order)
__global__ __launch_bounds__(256) void k_sum_local(int n, const int32_t *__restrict__ tp_ptr,
                                                   const int32_t *__restrict__ tp_pos, const double *__restrict__ u,
                                                   int64_t ldu, double *__restrict__ z, int ldz) {
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= n) return;
    const int rhs = blockIdx.y;
    const double *uu = u + (int64_t)rhs * ldu;
    double s = 0.0;
    for (int t = tp_ptr[l]; t < tp_ptr[l + 1]; ++t) s += uu[tp_pos[t]];
    z[(int64_t)rhs * ldz + l] = s;
}

int32_t apply_two_level(const ApplyPlan &p, const double *r, int ldr, double *z, int ldz, hipStream_t s) {
    const int tiles = (p.maxnI + LS_ROWS - 1) / LS_ROWS;
    const int64_t ldu = p.sum_nI;
    if (p.ev0) HKG_HIP(hipEventRecord(p.ev0, s));
    if (p.local_f32) {
        size_t shm = ((p.maxnI * sizeof(float) + 7) / 8) * 8 + LS_ROWS * LS_WAVES * sizeof(double);
        hipLaunchKernelGGL(k_local_solve<float>, dim3(tiles, p.nsub, p.nrhs), dim3(LS_ROWS * LS_WAVES), shm, s, p.d_sub,
                           p.I_idx, p.winv_loc, (const float *)p.Minv, r, ldr, p.u, ldu);
    } else {
        size_t shm = (size_t)p.maxnI * sizeof(double) + LS_ROWS * LS_WAVES * sizeof(double);
        hipLaunchKernelGGL(k_local_solve<double>, dim3(tiles, p.nsub, p.nrhs), dim3(LS_ROWS * LS_WAVES), shm, s,
                           p.d_sub, p.I_idx, p.winv_loc, (const double *)p.Minv, r, ldr, p.u, ldu);
    }
    HKG_HIP(hipGetLastError());
    if (p.ev1) HKG_HIP(hipEventRecord(p.ev1, s));
    if (p.two_level && p.m0 > 0) {
        hipLaunchKernelGGL(k_restrict, dim3(p.nsub, p.nrhs), dim3(256), (size_t)p.maxnI * sizeof(double), s, p.d_sub,
                           p.I_idx, p.Z, r, ldr, p.c, p.m0);
        size_t shm = (size_t)(p.m0 + 256) * sizeof(double);
        hipLaunchKernelGGL(k_coarse_gemv, dim3((p.m0 + CG_ROWS - 1) / CG_ROWS, p.nrhs), dim3(256), shm, s, p.B0inv, p.m0,
                           p.c, p.y);
        hipLaunchKernelGGL(k_add_coarse, dim3((p.maxnI + 255) / 256, p.nsub, p.nrhs), dim3(256), 0, s, p.d_sub, p.Z, p.y,
                           p.m0, p.u, ldu);
        HKG_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_sum_local, dim3((p.n_dof + 255) / 256, p.nrhs), dim3(256), 0, s, p.n_dof, p.tp_ptr, p.tp_pos,
                       p.u, ldu, z, ldz);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

}  // namespace hkg
