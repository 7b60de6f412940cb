// Setup kernels: the operator values and the dense local blocks of every subdomain.
//
//   B = A - k^2 S and D_k = A + k^2 S on the CSR pattern (Sec. 2.1; D_k of Prop. 2.11).
//   [B_II | B_IG]  rows dof(D), columns ovdof(D) = [dof(D), Gamma]: the Dirichlet matrix
//                  B_D = R_D B E_D of eq. (2.22) and the coupling to Gamma.  Internal dofs have
//                  their support inside closure(D), so these rows of the subdomain form b_D equal the
//                  global ones.
//   C_II = X D_k[I, I] X with X = diag(1/mu): the right-hand side (Xi p, Xi v)_{1,k,D} of Def. 2.14 on
//                  dof(D) (Xi vanishes on Gamma, Def. 2.13).
//   B~_GG          sum over the elements of D of (K_e - k^2 M_e) on Gamma x Gamma: the only block of
//                  the subdomain form b_D (eq. (2.18)) that differs from the global matrix.
#include "internal.hpp"
#include "kernels.hpp"

namespace hkg {

__global__ void k_form_operator(const double *__restrict__ A, const double *__restrict__ S, double k2,
                                double *__restrict__ B, double *__restrict__ Dk, int64_t nnz) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * blockDim.x) {
        B[i] = A[i] - k2 * S[i];
        Dk[i] = A[i] + k2 * S[i];
    }
}

int32_t form_operator(const double *A, const double *S, double k2, double *B, double *Dk, int64_t nnz, hipStream_t s) {
    int blocks = (int)std::min<int64_t>((nnz + 255) / 256, 8192);
    hipLaunchKernelGGL(k_form_operator, dim3(blocks), dim3(256), 0, s, A, S, k2, B, Dk, nnz);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// position of key in the ascending list a[0..n) or -1
__device__ __forceinline__ int find_sorted(const int32_t *__restrict__ a, int n, int key) {
    int lo = 0, hi = n - 1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        int v = a[mid];
        if (v == key) return mid;
        if (v < key) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

__global__ __launch_bounds__(256) void k_extract_blocks(const SubDev *__restrict__ subs, const int32_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ colidx, const double *__restrict__ Bval,
                                                        const double *__restrict__ Dval, const int32_t *__restrict__ I_idx,
                                                        const int32_t *__restrict__ G_idx, const double *__restrict__ winv,
                                                        double *__restrict__ BIO, double *__restrict__ CII) {
    const SubDev sd = subs[blockIdx.y];
    const int a = blockIdx.x * 256 + threadIdx.x;
    if (a >= sd.nI) return;
    const int32_t *I = I_idx + sd.offI;
    const int32_t *G = G_idx + sd.offG;
    const int g = I[a];
    const double wa = winv[g];
    for (int t = rowptr[g]; t < rowptr[g + 1]; ++t) {
        const int q = colidx[t];
        int c = find_sorted(I, sd.nI, q);
        if (c >= 0) {
            BIO[sd.offBIO + a + (int64_t)c * sd.nI] = Bval[t];
            CII[sd.offSq + a + (int64_t)c * sd.nI] = wa * winv[q] * Dval[t];
        } else {
            c = find_sorted(G, sd.nG, q);
            if (c >= 0) BIO[sd.offBIO + a + (int64_t)(sd.nI + c) * sd.nI] = Bval[t];
        }
    }
}

int32_t extract_blocks(const SubDev *d_sub, int nsub, int maxnI, const int32_t *rowptr, const int32_t *colidx,
                       const double *Bval, const double *Dval, const int32_t *I_idx, const int32_t *G_idx,
                       const double *winv, double *BIO, double *CII, hipStream_t s) {
    hipLaunchKernelGGL(k_extract_blocks, dim3((maxnI + 255) / 256, nsub), dim3(256), 0, s, d_sub, rowptr, colidx, Bval,
                       Dval, I_idx, G_idx, winv, BIO, CII);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// B~_GG: one block per subdomain walks its band elements in a fixed order; within one element the
// (a, c) vertex pairs hit distinct entries, so the sum needs no atomics and is deterministic.
__global__ __launch_bounds__(64) void k_assemble_gamma(const SubDev *__restrict__ subs, int npe,
                                                       const int32_t *__restrict__ band_loc,
                                                       const double *__restrict__ bandK, const double *__restrict__ bandM,
                                                       double k2, double *__restrict__ BGG) {
    const SubDev sd = subs[blockIdx.x];
    const int t = threadIdx.x;
    const int a = t / npe, c = t % npe;
    const int npe2 = npe * npe;
    for (int b = sd.bandBeg; b < sd.bandEnd; ++b) {
        if (t < npe2) {
            const int la = band_loc[(int64_t)b * npe + a], lc = band_loc[(int64_t)b * npe + c];
            if (la >= 0 && lc >= 0)
                BGG[sd.offGG + la + (int64_t)lc * sd.nG] +=
                    bandK[(int64_t)b * npe2 + a * npe + c] - k2 * bandM[(int64_t)b * npe2 + a * npe + c];
        }
        __syncthreads();
    }
}

// The same sums with the block in LDS: one wave adds the elements in the same order (a wave's LDS
// operations complete in order, and within one element the lanes hit distinct entries), the
// element data loaded eight elements ahead; the block is written out once.
constexpr int AG_AHEAD = 8;

__global__ __launch_bounds__(64) void k_assemble_gamma_lds(const SubDev *__restrict__ subs, int npe,
                                                           const int32_t *__restrict__ band_loc,
                                                           const double *__restrict__ bandK,
                                                           const double *__restrict__ bandM, double k2,
                                                           double *__restrict__ BGG) {
    extern __shared__ double G[];                     // nG x nG, ld nG
    const SubDev sd = subs[blockIdx.x];
    const int nG = sd.nG;
    const int t = threadIdx.x;
    for (int e = t; e < nG * nG; e += 64) G[e] = 0.0;
    const int npe2 = npe * npe;
    const int a = t / npe, c = t % npe;
    for (int b0 = sd.bandBeg; b0 < sd.bandEnd; b0 += AG_AHEAD) {
        double v[AG_AHEAD];
        int idx[AG_AHEAD];
#pragma unroll
        for (int u = 0; u < AG_AHEAD; ++u) {
            const int b = b0 + u;
            const bool ok = t < npe2 && b < sd.bandEnd;
            const int la = ok ? band_loc[(int64_t)b * npe + a] : -1;
            const int lc = ok ? band_loc[(int64_t)b * npe + c] : -1;
            idx[u] = (la >= 0 && lc >= 0) ? la + lc * nG : -1;
            v[u] = ok ? bandK[(int64_t)b * npe2 + t] - k2 * bandM[(int64_t)b * npe2 + t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < AG_AHEAD; ++u)
            if (idx[u] >= 0) G[idx[u]] += v[u];
    }
    for (int e = t; e < nG * nG; e += 64) BGG[sd.offGG + e] = G[e];
}

int32_t assemble_gamma(const SubDev *d_sub, int nsub, int maxnG, int npe, const int32_t *band_elem,
                       const int32_t *band_loc, const double *elemK, const double *elemM, double k2, double *BGG,
                       hipStream_t s) {
    (void)band_elem;
    const size_t shm = (size_t)maxnG * maxnG * sizeof(double);
    if (npe * npe <= 64 && shm <= (size_t)120 * 1024) {
        hipLaunchKernelGGL(k_assemble_gamma_lds, dim3(nsub), dim3(64), shm, s, d_sub, npe, band_loc, elemK, elemM, k2,
                           BGG);
        HKG_HIP(hipGetLastError());
        return HKG_OK;
    }
    hipLaunchKernelGGL(k_assemble_gamma, dim3(nsub), dim3(64), 0, s, d_sub, npe, band_loc, elemK, elemM, k2, BGG);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// GI = B_GI = (B_IG)^T, nG x nI with ld nG: 64 columns of GI per block through an LDS tile (reads
// along the rows of B_IG, writes along the columns of GI, both contiguous)
constexpr int GG_TILE = 64;

__global__ __launch_bounds__(256) void k_gather_gamma_rows(const SubDev *__restrict__ subs, const double *__restrict__ BIO,
                                                           double *__restrict__ GI) {
    extern __shared__ double tile[];                  // nG x (GG_TILE + 1)
    const SubDev sd = subs[blockIdx.y];
    const int a0 = blockIdx.x * GG_TILE;
    const int nI = sd.nI, nG = sd.nG;
    if (a0 >= nI || nG == 0) return;
    const int na = min(GG_TILE, nI - a0);
    const int tid = threadIdx.x;
    for (int q = tid; q < nG * GG_TILE; q += 256) {
        const int la = q % GG_TILE, g = q / GG_TILE;
        if (la < na) tile[g * (GG_TILE + 1) + la] = BIO[sd.offBIO + (a0 + la) + (int64_t)(nI + g) * nI];
    }
    __syncthreads();
    for (int q = tid; q < nG * GG_TILE; q += 256) {
        const int g = q % nG, la = q / nG;
        if (la < na) GI[sd.offGI + g + (int64_t)(a0 + la) * nG] = tile[g * (GG_TILE + 1) + la];
    }
}

// the same without the tile (Gamma blocks too tall for it)
__global__ __launch_bounds__(256) void k_gather_gamma_rows_direct(const SubDev *__restrict__ subs,
                                                                  const double *__restrict__ BIO,
                                                                  double *__restrict__ GI) {
    const SubDev sd = subs[blockIdx.y];
    const int a = blockIdx.x * 256 + threadIdx.x;
    if (a >= sd.nI) return;
    for (int g = 0; g < sd.nG; ++g)
        GI[sd.offGI + g + (int64_t)a * sd.nG] = BIO[sd.offBIO + a + (int64_t)(sd.nI + g) * sd.nI];
}

int32_t gather_gamma_rows(const SubDev *d_sub, int nsub, int maxnI, int maxnG, const double *BIO, double *GI,
                          hipStream_t s) {
    const size_t shm = (size_t)std::max(maxnG, 1) * (GG_TILE + 1) * sizeof(double);
    if (shm <= (size_t)64 * 1024)
        hipLaunchKernelGGL(k_gather_gamma_rows, dim3((maxnI + GG_TILE - 1) / GG_TILE, nsub), dim3(256), shm, s, d_sub,
                           BIO, GI);
    else
        hipLaunchKernelGGL(k_gather_gamma_rows_direct, dim3((maxnI + 255) / 256, nsub), dim3(256), 0, s, d_sub, BIO,
                           GI);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// X <- P X with the row exchanges of the LU of B~_GG (which == 0: X = GI, nG x nI)
template <typename T>
__global__ __launch_bounds__(256) void k_apply_pivots_rows(const SubDev *__restrict__ subs, const int32_t *__restrict__ piv,
                                                           T *__restrict__ X, int which) {
    const SubDev sd = subs[blockIdx.y];
    (void)which;
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= sd.nI) return;
    T *col = X + sd.offGI + (int64_t)c * sd.nG;
    const int32_t *pv = piv + sd.offPiv;
    for (int j = 0; j < sd.nG; ++j) {
        int p = pv[j];
        if (p != j) {
            T t = col[j];
            col[j] = col[p];
            col[p] = t;
        }
    }
}

template <typename T>
int32_t apply_pivots_rows(const SubDev *d_sub, int nsub, int maxcol, const int32_t *piv, T *X, int which,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_apply_pivots_rows<T>, dim3((maxcol + 255) / 256, nsub), dim3(256), 0, s, d_sub, piv, X, which);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}
template int32_t apply_pivots_rows<double>(const SubDev *, int, int, const int32_t *, double *, int, hipStream_t);

// copy B_II (the first nI columns of [B_II | B_IG]) into an nI x nI work matrix
template <typename TO>
__global__ __launch_bounds__(256) void k_copy_bii(const SubDev *__restrict__ subs, const double *__restrict__ BIO,
                                                  TO *__restrict__ out) {
    const SubDev sd = subs[blockIdx.y];
    const int64_t n2 = (int64_t)sd.nI * sd.nI;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n2; i += (int64_t)gridDim.x * 256)
        out[sd.offSq + i] = (TO)BIO[sd.offBIO + i];
}

int32_t copy_bii(const SubDev *d_sub, int nsub, int maxnI, const double *BIO, double *out, hipStream_t s) {
    int blocks = std::max(1, std::min(256, (maxnI * maxnI + 255) / 256));
    hipLaunchKernelGGL(k_copy_bii<double>, dim3(blocks, nsub), dim3(256), 0, s, d_sub, BIO, out);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}


// C_II = L U without row exchanges; it is SPD exactly when every pivot is positive
__global__ __launch_bounds__(256) void k_check_spd(const SubDev *__restrict__ subs, const double *__restrict__ C,
                                                   int32_t *__restrict__ flag) {
    const SubDev sd = subs[blockIdx.x];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < sd.nI; i += 256) {
        double d = C[sd.offSq + i + (int64_t)i * sd.nI];
        if (!(d > 0.0) || !isfinite(d)) bad = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) flag[blockIdx.x] = bad;
}

// C_II = L D L^T for every subdomain (C_II of Def 2.14 restricted to the interior dofs: symmetric
// positive definite, and banded, no entry farther than `band` from the diagonal), one workgroup per
// subdomain with the lower band in LDS.  Column j is one step: every entry (j+t, j+s),
// 1 <= s <= t <= band, of the trailing window takes its rank-1 term -l_t a_s (l_t = a_t / d_j) from
// the thread that owns the pair (s, t); one barrier per step.  Written back in the packed form of an
// LU without exchanges: unit L below the diagonal, D on it, D L^T above (only the band).
constexpr int LDL_THREADS = 256;
constexpr int LDL_PAIRS = 4;            // (s, t) pairs per thread: band <= 44

bool ldl_band_fits(int maxnI, int band) {
    return band >= 0 && band * (band + 1) / 2 <= LDL_THREADS * LDL_PAIRS &&
           (size_t)2 * maxnI * (band + 1) * sizeof(double) <= (size_t)156 * 1024;
}

__global__ __launch_bounds__(LDL_THREADS) void k_ldl_band(const SubDev *__restrict__ subs, double *__restrict__ C,
                                                          int band) {
    extern __shared__ double shl[];
    const SubDev sd = subs[blockIdx.x];
    const int n = sd.nI;
    if (n == 0) return;
    const int w = band + 1;
    double *Bd = shl;                          // Bd[j w + t]: current entry (j + t, j)
    double *Lo = shl + (int64_t)n * w;         // Lo[j w] = d_j, Lo[j w + t] = L[j + t][j]
    double *A = C + sd.offSq;                  // n x n, ld n
    const int tid = threadIdx.x;
    for (int e0 = tid; e0 < n * w; e0 += LDL_THREADS * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = min(e0 + u * LDL_THREADS, n * w - 1), j = e / w, t = e % w;
            v[u] = A[min(j + t, n - 1) + (int64_t)j * n];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * LDL_THREADS;
            if (e < n * w) Bd[e] = (e / w) + (e % w) < n ? v[u] : 0.0;
        }
    }
    // this thread's pairs (s, t), enumerated t = 1.., s = 1..t
    const int npair = band * (band + 1) / 2;
    int ps[LDL_PAIRS], pt[LDL_PAIRS];
#pragma unroll
    for (int u = 0; u < LDL_PAIRS; ++u) {
        const int q = tid + u * LDL_THREADS;
        int t = 1;
        while (t * (t + 1) / 2 <= q) ++t;
        pt[u] = q < npair ? t : n;          // t = n: never applied
        ps[u] = q < npair ? q - t * (t - 1) / 2 + 1 : 1;
    }
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        const double *col = Bd + (int64_t)j * w;
        const double d = col[0];
        const double rd = 1.0 / d;
#pragma unroll
        for (int u = 0; u < LDL_PAIRS; ++u) {
            const int s = ps[u], t = pt[u];
            if (j + t < n) Bd[(int64_t)(j + s) * w + (t - s)] -= (col[t] * rd) * col[s];
        }
        if (tid < w) Lo[(int64_t)j * w + tid] = tid == 0 ? d : (j + tid < n ? col[tid] * rd : 0.0);
        __syncthreads();
    }
    for (int e = tid; e < n * w; e += LDL_THREADS) {
        const int j = e / w, t = e % w;
        if (j + t >= n) continue;
        const double v = Lo[e];
        if (t == 0) {
            A[j + (int64_t)j * n] = v;
        } else {
            A[(j + t) + (int64_t)j * n] = v;
            A[j + (int64_t)(j + t) * n] = Lo[(int64_t)j * w] * v;
        }
    }
}

int32_t ldl_band(const SubDev *d_sub, int nsub, int maxnI, double *C, int band, hipStream_t s) {
    if (!ldl_band_fits(maxnI, band)) return HKG_EINVAL;
    const size_t shm = (size_t)2 * maxnI * (band + 1) * sizeof(double);
    hipLaunchKernelGGL(k_ldl_band, dim3(nsub), dim3(LDL_THREADS), shm, s, d_sub, C, band);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

int32_t check_spd_pivots(const SubDev *d_sub, int nsub, const double *C, int32_t *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_check_spd, dim3(nsub), dim3(256), 0, s, d_sub, C, flag);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// T = D^{-1/2} S D^{-1/2} with D = diag(U) of C_II = L U (so C_II = (L D^{1/2}) (L D^{1/2})^T); S has
// leading dimension nI at offSq, T the padded leading dimension ldM at offM
__global__ __launch_bounds__(256) void k_scale_sym(const SubDev *__restrict__ subs, const double *__restrict__ C,
                                                   const double *__restrict__ S, double *__restrict__ T) {
    const SubDev sd = subs[blockIdx.y];
    const int64_t n2 = (int64_t)sd.nI * sd.nI;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n2; i += (int64_t)gridDim.x * 256) {
        int r = (int)(i % sd.nI), c = (int)(i / sd.nI);
        double dr = C[sd.offSq + r + (int64_t)r * sd.nI], dc = C[sd.offSq + c + (int64_t)c * sd.nI];
        T[sd.offM + r + (int64_t)c * sd.ldM] = S[sd.offSq + i] / (sqrt(dr) * sqrt(dc));
    }
}

int32_t scale_sym(const SubDev *d_sub, int nsub, int maxnI, const double *C, const double *S, double *T, hipStream_t s) {
    int blocks = std::max(1, std::min(256, (maxnI * maxnI + 255) / 256));
    hipLaunchKernelGGL(k_scale_sym, dim3(blocks, nsub), dim3(256), 0, s, d_sub, C, S, T);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

}  // namespace hkg
