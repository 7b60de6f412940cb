// Batched dense linear algebra for uneven matrix sizes: tiled GEMM, blocked LU with partial
// pivoting, blocked triangular solves with many right-hand sides, and the inverse built from them.
//
// Every batched kernel takes one descriptor per matrix (offset, size, leading dimension) and uses
// blockIdx.y as the batch index, so a launch covers matrices of different sizes; work past a
// matrix's own size returns early.  Matrices are column-major.  T is double or float; the float
// instantiations accumulate in float (the mixed-precision local factors).
#include <cfloat>

#include "internal.hpp"
#include "kernels.hpp"
#include "tile.hpp"
#include "wave.hpp"

namespace hkg {

constexpr int LU_NB = LU_BLOCK;    // LU / triangular-solve block size

// Copy `total` elements with `nt` threads, U loads in flight per thread: load(e) for e < total
// (called only with such e), store(e, value).  A plain loop whose iterations each load and then
// store would wait for every load in turn.
template <int U, typename F, typename G>
__device__ __forceinline__ void staged_copy(int total, int tid, int nt, F load, G store) {
    for (int e0 = tid; e0 < total; e0 += nt * U) {
        decltype(load(0)) v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = load(min(e0 + u * nt, total - 1));
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (e0 + u * nt < total) store(e0 + u * nt, v[u]);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_batched(const GemmJob *__restrict__ jobs, const T *__restrict__ Ab,
                                                      const T *__restrict__ Bb, T *__restrict__ Cb, T alpha, T beta,
                                                      int ta, int tb, int tiles_m_max) {
    const GemmJob J = jobs[blockIdx.y];
    const int tm = blockIdx.x % tiles_m_max, tn = blockIdx.x / tiles_m_max;
    if (tm * GT >= J.M || tn * GT >= J.N) return;
    gemm_tile<T>(J.M, J.N, J.K, Ab + J.offA, J.lda, ta, Bb + J.offB, J.ldb, tb, Cb + J.offC, J.ldc, alpha, beta, tm,
                 tn);
}

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_batched32(const GemmJob *__restrict__ jobs, const T *__restrict__ Ab,
                                                        const T *__restrict__ Bb, T *__restrict__ Cb, T alpha, T beta,
                                                        int ta, int tb, int tiles_m_max) {
    const GemmJob J = jobs[blockIdx.y];
    const int tm = blockIdx.x % tiles_m_max, tn = blockIdx.x / tiles_m_max;
    if (tm * GT2 >= J.M || tn * GT2 >= J.N || J.K <= 0) {
        if (J.K <= 0 && tm * GT2 < J.M && tn * GT2 < J.N) {
            // an empty sum: C = beta C
            const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
            for (int c = 0; c < 2; ++c)
                for (int r = 0; r < 2; ++r) {
                    const int gi = tm * GT2 + tx + 16 * r, gj = tn * GT2 + ty + 16 * c;
                    if (gi < J.M && gj < J.N) {
                        T *p = Cb + J.offC + gi + (int64_t)gj * J.ldc;
                        *p = beta == T(0) ? T(0) : beta * *p;
                    }
                }
        }
        return;
    }
    gemm_tile32<T>(J.M, J.N, J.K, Ab + J.offA, J.lda, ta, Bb + J.offB, J.ldb, tb, Cb + J.offC, J.ldc, alpha, beta, tm,
                   tn);
}

template <typename T>
int32_t gemm_batched(const GemmJob *d_jobs, int nbatch, int maxM, int maxN, const T *A, const T *B, T *C, T alpha,
                     T beta, bool ta, bool tb, hipStream_t s) {
    if (nbatch == 0 || maxM == 0 || maxN == 0) return HKG_OK;
    int tmm = (maxM + GT - 1) / GT, tnm = (maxN + GT - 1) / GT;
    if ((int64_t)tmm * tnm * nbatch < 256) {
        // too few 64 x 64 tiles to fill the CUs: 32 x 32 tiles (same sums, same bits)
        const int t2m = (maxM + GT2 - 1) / GT2, t2n = (maxN + GT2 - 1) / GT2;
        hipLaunchKernelGGL(k_gemm_batched32<T>, dim3(t2m * t2n, nbatch), dim3(256), 0, s, d_jobs, A, B, C, alpha, beta,
                           (int)ta, (int)tb, t2m);
    } else {
        dim3 grid(tmm * tnm, nbatch);
        hipLaunchKernelGGL(k_gemm_batched<T>, grid, dim3(256), 0, s, d_jobs, A, B, C, alpha, beta, (int)ta, (int)tb,
                           tmm);
    }
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}
template int32_t gemm_batched<double>(const GemmJob *, int, int, int, const double *, const double *, double *, double,
                                      double, bool, bool, hipStream_t);

// ------------------------------------------------------------------------------------------------
// LU with partial pivoting, right-looking blocked (panel, row swaps, U12 solve, trailing GEMM).
// Pivots are absolute row indices (0-based) stored at piv[m.off_piv + j]; info[b] = first zero
// pivot column + 1 (0 if none).  With pivot == false the factorisation is LU without row exchanges
// (used for symmetric positive definite matrices).
// ------------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_lu_panel(const DMat *__restrict__ mats, const int64_t *__restrict__ poff,
                                                  T *__restrict__ Ab, int32_t *__restrict__ piv, int32_t *__restrict__ info,
                                                  int j0, int pivot) {
    const DMat m = mats[blockIdx.x];
    const int n = m.n;
    if (j0 >= n) return;
    T *A = Ab + m.off;
    const int ld = m.ld;
    const int jend = min(j0 + LU_NB, n);
    __shared__ T sval[256];
    __shared__ int sidx[256];
    __shared__ int s_p;
    const int tid = threadIdx.x;
    int32_t *pv = piv + poff[blockIdx.x];
    for (int j = j0; j < jend; ++j) {
        int p = j;
        if (pivot) {
            // argmax |A[i, j]|, i >= j; ties resolved to the smallest row index
            T best = T(-1);
            int bi = n;
            for (int i = j + tid; i < n; i += 256) {
                T v = fabs(A[i + (int64_t)j * ld]);
                if (v > best) { best = v; bi = i; }
            }
            sval[tid] = best;
            sidx[tid] = bi;
            __syncthreads();
            for (int w = 128; w > 0; w >>= 1) {
                if (tid < w) {
                    T a = sval[tid], b = sval[tid + w];
                    int ia = sidx[tid], ib = sidx[tid + w];
                    if (b > a || (b == a && ib < ia)) { sval[tid] = b; sidx[tid] = ib; }
                }
                __syncthreads();
            }
            if (tid == 0) s_p = sidx[0] < n ? sidx[0] : j;
            __syncthreads();
            p = s_p;
        }
        if (tid == 0) pv[j] = p;
        // swap rows j and p inside the panel columns
        if (p != j) {
            for (int c = j0 + tid; c < jend; c += 256) {
                T t = A[j + (int64_t)c * ld];
                A[j + (int64_t)c * ld] = A[p + (int64_t)c * ld];
                A[p + (int64_t)c * ld] = t;
            }
        }
        __syncthreads();
        const T d = A[j + (int64_t)j * ld];
        if (d == T(0) || !isfinite(d)) {
            if (tid == 0 && info[blockIdx.x] == 0) info[blockIdx.x] = j + 1;
            __syncthreads();
            continue;
        }
        const T rd = T(1) / d;
        for (int i = j + 1 + tid; i < n; i += 256) A[i + (int64_t)j * ld] *= rd;
        __syncthreads();
        // rank-1 update of the rest of the panel
        const int w = jend - j - 1;
        if (w > 0) {
            const int rows = n - j - 1;
            for (int e = tid; e < rows * w; e += 256) {
                int i = j + 1 + e % rows, c = j + 1 + e / rows;
                A[i + (int64_t)c * ld] -= A[i + (int64_t)j * ld] * A[j + (int64_t)c * ld];
            }
        }
        __syncthreads();
    }
}

// Panel factorisation with the panel held in registers: thread t owns row j0 + t (the whole panel
// row, LU_NB entries), so a panel of up to 1024 rows needs no memory traffic between its columns.
// Two barriers per column.  The pivot candidates of column j + 1 are searched right after the
// rank-1 update of column j (wave arg-max by DPP lane moves, ties to the smallest row, as in the
// global-memory panel); after the barrier every wave reduces the 16 wave candidates within one DPP row, the
// owners of the pivot row and of row j publish them in LDS, and after the second barrier the rows
// are exchanged and the next update is applied.  NT threads (a multiple of 64, at most 1024) cover
// the panel rows j0 .. min(n, mlim) - 1; rows from mlim on are known to be zero in the panel columns
// (a banded matrix) and are left alone.
constexpr int PANEL_REG_ROWS = 1024;


// the panel factorisation of one matrix (A with n rows and leading dimension ld, pivots pv, info
// slot *info) by a workgroup of NT threads; load(r, c) gives the panel's entry (r, j0 + c) as the
// factorisation starts
template <typename T, int NT, typename LOAD>
__device__ __forceinline__ void lu_panel_reg_body(int n, T *__restrict__ A, int ld, int32_t *__restrict__ pv,
                                                  int32_t *__restrict__ info, int j0, int pivot, int mlim, LOAD load) {
    constexpr int NW = NT / 64;
    if (j0 >= n) return;
    const int nb = min(j0 + LU_NB, n) - j0;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int r = j0 + tid;
    const bool own = r < min(n, mlim);
    int bad = 0;                        // first zero (or non-finite) pivot column + 1
    int pmine = 0;                      // thread jj keeps the pivot of column jj: one store at the end
                                        // (a store per column would stall on its completion)
    __shared__ T prow[2][LU_NB];
    __shared__ T drow[2][LU_NB];
    __shared__ T wval[2][NW];
    __shared__ int widx[2][NW];
    T a[LU_NB];
#pragma unroll
    for (int c = 0; c < LU_NB; ++c) a[c] = (own && c < nb) ? load(r, c) : T(0);
    if (pivot) {
        T v = own ? fabs(a[0]) : T(-1);
        int idx = own ? r : 0x7fffffff;
        argmax_wave64(v, idx);
        if (lane == 0) {
            wval[0][wv] = v;
            widx[0][wv] = idx;
        }
    }
    __syncthreads();
#pragma clang loop unroll(full)
    for (int jj = 0; jj < LU_NB; ++jj) {
        if (jj < nb) {
            const int j = j0 + jj, buf = jj & 1;
            int p = j;
            if (pivot) {
                T v = lane < NW ? wval[buf][lane] : T(-1);
                int idx = lane < NW ? widx[buf][lane] : 0x7fffffff;
                static_assert(NW <= 16, "wave candidates must fit one DPP row");
                argmax_row16(v, idx);
                const int bi = __builtin_amdgcn_readlane(idx, 0);
                p = bi < n ? bi : j;
            }
            if (own && r == p) {
#pragma unroll
                for (int c = 0; c < LU_NB; ++c) prow[buf][c] = a[c];
            }
            if (own && r == j) {
#pragma unroll
                for (int c = 0; c < LU_NB; ++c) drow[buf][c] = a[c];
            }
            __syncthreads();
            if (own && r == j) {
#pragma unroll
                for (int c = 0; c < LU_NB; ++c) a[c] = prow[buf][c];
            } else if (own && r == p) {
#pragma unroll
                for (int c = 0; c < LU_NB; ++c) a[c] = drow[buf][c];
            }
            const T dpiv = prow[buf][jj];
            const bool ok = dpiv != T(0) && isfinite(dpiv);
            if (tid == jj) pmine = p;
            if (!ok && bad == 0) bad = j + 1;
            if (ok && own && r > j) {
                const T l = a[jj] * (T(1) / dpiv);
                a[jj] = l;
#pragma unroll
                for (int c = jj + 1; c < LU_NB; ++c) a[c] -= l * prow[buf][c];
            }
            if (pivot && jj + 1 < nb) {
                T v = (own && r > j) ? fabs(a[jj + 1 < LU_NB ? jj + 1 : jj]) : T(-1);
                int idx = (own && r > j) ? r : 0x7fffffff;
                argmax_wave64(v, idx);
                if (lane == 0) {
                    wval[buf ^ 1][wv] = v;
                    widx[buf ^ 1][wv] = idx;
                }
            }
            __syncthreads();
        }
    }
    if (own) {
#pragma unroll
        for (int c = 0; c < LU_NB; ++c)
            if (c < nb) A[r + (int64_t)(j0 + c) * ld] = a[c];
    }
    if (tid < nb) pv[j0 + tid] = pmine;
    if (tid == 0 && bad && *info == 0) *info = bad;
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_lu_panel_reg(const DMat *__restrict__ mats, const int64_t *__restrict__ poff,
                                                     T *__restrict__ Ab, int32_t *__restrict__ piv,
                                                     int32_t *__restrict__ info, int j0, int pivot, int mlim) {
    const DMat m = mats[blockIdx.x];
    T *A = Ab + m.off;
    const int ld = m.ld;
    lu_panel_reg_body<T, NT>(m.n, A, ld, piv + poff[blockIdx.x], info + blockIdx.x, j0, pivot, mlim,
                             [&](int r, int c) { return A[r + (int64_t)(j0 + c) * ld]; });
}

// Panel factorisation by one wave: lane l owns the physical rows j0 + l + 64 q (q < RPL), so panels
// of up to 64 RPL rows (banded matrices) need no barrier and no LDS.  Row exchanges are deferred:
// every physical row carries its logical row index, the pivot search runs over the rows whose
// logical index is still >= j (arg-max by DPP, ties to the smallest logical row, as in
// k_lu_panel_reg), an exchange swaps two logical indices, and the pivot row's entries reach the
// other lanes by v_readlane.  At the end each physical row is stored at its logical position, which
// gives the same factors as exchanging the rows as they are chosen.
template <typename T, int RPL>
__global__ __launch_bounds__(64) void k_lu_panel_wave(const DMat *__restrict__ mats, const int64_t *__restrict__ poff,
                                                      T *__restrict__ Ab, int32_t *__restrict__ piv,
                                                      int32_t *__restrict__ info, int j0, int pivot, int mlim) {
    const DMat m = mats[blockIdx.x];
    const int n = m.n;
    if (j0 >= n) return;
    T *A = Ab + m.off;
    const int ld = m.ld;
    const int nb = min(j0 + LU_NB, n) - j0;
    const int lane = threadIdx.x;
    const int rend = min(n, mlim);
    int32_t *pv = piv + poff[blockIdx.x];
    int bad = 0;
    int pmine = 0;                      // lane jj keeps the pivot of column jj (one store at the end)
    T a[RPL][LU_NB];
    int lrow[RPL];                      // logical row of each physical row (>= rend: absent)
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        const int r = j0 + lane + 64 * q;
        lrow[q] = r < rend ? r : 0x3fffffff;
#pragma unroll
        for (int c = 0; c < LU_NB; ++c) a[q][c] = (r < rend && c < nb) ? A[r + (int64_t)(j0 + c) * ld] : T(0);
    }
#pragma clang loop unroll(full)
    for (int jj = 0; jj < LU_NB; ++jj) {
        if (jj < nb) {
            const int j = j0 + jj;
            // winner: key = logical row * 256 + physical slot (smallest logical row on ties); the row
            // holding logical row j is always a candidate, and a NaN entry wins (the LU then fails)
            int key;
            if (pivot) {
                T v = T(-1);
                int kk = 0x7fffffff;
#pragma unroll
                for (int q = 0; q < RPL; ++q) {
                    const T t = fabs(a[q][jj]);
                    const T x = (lrow[q] >= j && lrow[q] < rend) ? (t != t ? T(INFINITY) : t) : T(-1);
                    const int k2 = (lrow[q] << 8) | (lane + 64 * q);
                    if (x > v || (x == v && k2 < kk)) {
                        v = x;
                        kk = k2;
                    }
                }
                argmax_wave64(v, kk);
                key = kk;
            } else {
                key = (j << 8) | (j - j0);     // no exchanges: logical row j is physical row j
            }
            const int p = key >> 8, slot = key & 255;
            const int lp = slot & 63, qp = slot >> 6;
            // the pivot row's entries c >= jj, from lane lp
            T prow[LU_NB];
#pragma unroll
            for (int c = jj; c < LU_NB; ++c) {
                T src = a[0][c];
#pragma unroll
                for (int q = 1; q < RPL; ++q) src = qp == q ? a[q][c] : src;
                prow[c] = readlane_any(src, lp);
            }
            // logical exchange of rows j and p
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                const bool is_p = lane == lp && q == qp;
                if (is_p) lrow[q] = j;
                else if (lrow[q] == j) lrow[q] = p;
            }
            const T dpiv = prow[jj];
            const bool ok = dpiv != T(0) && isfinite(dpiv);
            if (lane == jj) pmine = p;
            if (!ok && bad == 0) bad = j + 1;
            if (ok) {
                const T rdp = T(1) / dpiv;
#pragma unroll
                for (int q = 0; q < RPL; ++q) {
                    if (lrow[q] > j && lrow[q] < rend) {
                        const T l = a[q][jj] * rdp;
                        a[q][jj] = l;
#pragma unroll
                        for (int c = jj + 1; c < LU_NB; ++c) a[q][c] -= l * prow[c];
                    }
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        const int lr = lrow[q];
        if (lr < rend) {
#pragma unroll
            for (int c = 0; c < LU_NB; ++c)
                if (c < nb) A[lr + (int64_t)(j0 + c) * ld] = a[q][c];
        }
    }
    if (lane < nb) pv[j0 + lane] = pmine;
    if (lane == 0 && bad && info[blockIdx.x] == 0) info[blockIdx.x] = bad;
}

// apply the row exchanges of panel [j0, j0+NB) to the columns outside the panel
template <typename T>
__global__ __launch_bounds__(256) void k_lu_laswp(const DMat *__restrict__ mats, const int64_t *__restrict__ poff,
                                                  T *__restrict__ Ab, const int32_t *__restrict__ piv, int j0,
                                                  int tmax) {
    const DMat m = mats[blockIdx.y];
    const int n = m.n;
    if (j0 >= n) return;
    const int jend = min(j0 + LU_NB, n);
    const int outside = n - (jend - j0);
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= outside || t >= tmax) return;     // tmax = j0: the columns left of the panel only
    const int c = t < j0 ? t : t + (jend - j0);
    T *A = Ab + m.off + (int64_t)c * m.ld;
    const int32_t *pv = piv + poff[blockIdx.y];
    for (int j = j0; j < jend; ++j) {
        int p = pv[j];
        if (p != j) {
            T x = A[j];
            A[j] = A[p];
            A[p] = x;
        }
    }
}

// Triangular solve of one LU_NB block against a tile of TRI_COLS columns held in LDS: each thread
// solves its own column (x[r] in xs[r][tid]); T is the padded LU_NB x LU_NB triangle in LDS.
constexpr int TRI_COLS = 128;

template <typename T, int MODE>
__device__ __forceinline__ void solve_block_lds(T (*Ls)[LU_NB + 1], T (*xs)[TRI_COLS + 1], int tid) {
    if (MODE == TRI_LOWER_UNIT) {
        for (int r = 1; r < LU_NB; ++r) {
            T v = xs[r][tid];
            for (int k = 0; k < r; ++k) v -= Ls[r][k] * xs[k][tid];
            xs[r][tid] = v;
        }
    } else {
        for (int r = LU_NB - 1; r >= 0; --r) {
            T v = xs[r][tid];
            for (int k = r + 1; k < LU_NB; ++k) v -= Ls[r][k] * xs[k][tid];
            xs[r][tid] = (MODE == TRI_UPPER) ? v / Ls[r][r] : v;
        }
    }
}

// U12 = L11^{-1} A12 for the panel rows (the block is padded to LU_NB with the identity)
template <typename T>
__global__ __launch_bounds__(TRI_COLS) void k_lu_trsm_row(const DMat *__restrict__ mats, T *__restrict__ Ab, int j0,
                                                          int clim) {
    const DMat m = mats[blockIdx.y];
    const int n = min(m.n, clim);          // columns from clim on are zero in the panel rows
    const int jend = min(j0 + LU_NB, n);
    if (jend >= n) return;
    __shared__ T L[LU_NB][LU_NB + 1];
    __shared__ T xs[LU_NB][TRI_COLS + 1];
    T *A = Ab + m.off;
    const int ld = m.ld, nb = jend - j0;
    for (int e = threadIdx.x; e < LU_NB * LU_NB; e += TRI_COLS) {
        int r = e % LU_NB, c = e / LU_NB;
        L[r][c] = (r < nb && c < nb) ? A[j0 + r + (int64_t)(j0 + c) * ld] : T(r == c ? 1 : 0);
    }
    const int c = jend + blockIdx.x * TRI_COLS + threadIdx.x;
    const bool valid = c < n;
    {
        T v[LU_NB];
#pragma unroll
        for (int r = 0; r < LU_NB; ++r) v[r] = valid ? A[j0 + min(r, nb - 1) + (int64_t)c * ld] : T(0);
#pragma unroll
        for (int r = 0; r < LU_NB; ++r) xs[r][threadIdx.x] = r < nb ? v[r] : T(0);
    }
    __syncthreads();
    solve_block_lds<T, TRI_LOWER_UNIT>(L, xs, threadIdx.x);
    if (valid)
        for (int r = 0; r < nb; ++r) A[j0 + r + (int64_t)c * ld] = xs[r][threadIdx.x];
}

// A22 -= L21 U12 on rows [jend, rlim) and columns [jend, clim) (both limits capped at n)
template <typename T>
__global__ __launch_bounds__(256) void k_lu_update(const DMat *__restrict__ mats, T *__restrict__ Ab, int j0,
                                                   int tiles_m_max, int rlim, int clim) {
    const DMat m = mats[blockIdx.y];
    const int n = m.n;
    const int jend = min(j0 + LU_NB, n);
    const int rows = min(n, rlim) - jend, cols = min(n, clim) - jend;
    if (rows <= 0 || cols <= 0) return;
    const int tm = blockIdx.x % tiles_m_max, tn = blockIdx.x / tiles_m_max;
    if (tm * GT >= rows || tn * GT >= cols) return;
    T *A = Ab + m.off;
    const int ld = m.ld;
    gemm_tile<T>(rows, cols, jend - j0, A + jend + (int64_t)j0 * ld, ld, false, A + j0 + (int64_t)jend * ld, ld, false,
                 A + jend + (int64_t)jend * ld, ld, T(-1), T(1), tm, tn);
}

// x <- L^{-1} x for a unit lower LU_NB x LU_NB block (entry (r, k) at L[r * ldl + k]),
// right-looking in registers: once x[k] is final every
// later row subtracts its term, so the dependent chain is LU_NB steps long (each row still
// subtracts its terms in increasing k, as a left-looking substitution does)
template <typename T>
__device__ __forceinline__ void unit_lower_solve_regs(T (&x)[LU_NB], const T *__restrict__ L, int ldl) {
#pragma unroll
    for (int k = 0; k < LU_NB - 1; ++k) {
        const T xk = x[k];
#pragma unroll
        for (int r = k + 1; r < LU_NB; ++r) x[r] = fma(-L[r * ldl + k], xk, x[r]);
        // keep the loads of later steps from being hoisted (register pressure)
        __builtin_amdgcn_sched_barrier(0);
    }
}

// op(T) x = x for one full LU_NB block held in registers, right-looking (the same operation order as
// a wave-synchronous sweep): TRI_LOWER_UNIT forward; TRI_UPPER and TRI_LOWER_UNIT_TRANS backward
// (the latter unit diagonal).  Entry (r, k) of op(T) at Lb[r * ldl + k].
template <typename T, int MODE>
__device__ __forceinline__ void block_solve_regs(T (&x)[LU_NB], const T *__restrict__ Lb, int ldl) {
    if (MODE == TRI_LOWER_UNIT) {
        unit_lower_solve_regs(x, Lb, ldl);
    } else {
#pragma unroll
        for (int k = LU_NB - 1; k >= 0; --k) {
            if (MODE == TRI_UPPER) x[k] = x[k] / Lb[k * ldl + k];
            const T xk = x[k];
#pragma unroll
            for (int r = 0; r < k; ++r) x[r] = fma(-Lb[r * ldl + k], xk, x[r]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Everything after a panel in one launch, for panels of at most LP_MAXROWS rows (rows [j0, mlim)):
// each block takes LP_COLS columns right of the panel (up to clim) with the panel staged in LDS,
// exchanges their rows, solves U12 = L11^{-1} A12 and updates rows [jend, mlim) with L21 U12, all
// in LDS.  The exchanges of the columns left of the panel (the L factor) are deferred to
// k_lu_swap_left: nothing reads those columns before the factorisation ends, so applying a
// column's later exchanges at the end gives the same result.
constexpr int LP_COLS = 32;
constexpr int LP_MAXROWS = 256;

// fuse: block 0 (whose strip is the next panel's columns) goes on to factor the next panel (rows
// [jend, mlim_next)), taking the rows it has just updated from its LDS copy and those below from
// global memory, while the other blocks update their strips.
template <typename T>
__global__ __launch_bounds__(256) void k_lu_post(const DMat *__restrict__ mats, const int64_t *__restrict__ poff,
                                                 T *__restrict__ Ab, int32_t *__restrict__ piv, int j0, int mlim,
                                                 int clim, int pivot, int fuse, int mlim_next,
                                                 int32_t *__restrict__ info) {
    const DMat m = mats[blockIdx.y];
    const int n = m.n;
    if (j0 >= n) return;
    T *A = Ab + m.off;
    const int ld = m.ld;
    const int jend = min(j0 + LU_NB, n), nb = jend - j0;
    const int rend = min(n, mlim), cend = min(n, clim);
    const int32_t *pv = piv + poff[blockIdx.y];
    const int tid = threadIdx.x;
    const int cs = jend + blockIdx.x * LP_COLS;               // first column of this strip
    if (cs >= cend) return;
    const int ncs = min(LP_COLS, cend - cs);
    const int rw = rend - j0;                                   // rows [j0, rend)
    extern __shared__ double shp[];
    T *Ps = reinterpret_cast<T *>(shp);                         // rw x (LU_NB + 1): the panel
    T *Xs = Ps + (int64_t)rw * (LU_NB + 1);                     // rw x (LP_COLS + 1): the strip
    __shared__ int lp[LU_NB];
    staged_copy<16>(
        rw * LU_NB, tid, 256, [&](int e) { return A[(j0 + e % rw) + (int64_t)(j0 + min(e / rw, nb - 1)) * ld]; },
        [&](int e, T v) { Ps[(e % rw) * (LU_NB + 1) + e / rw] = e / rw < nb ? v : T(0); });
    staged_copy<16>(
        rw * LP_COLS, tid, 256, [&](int e) { return A[(j0 + e % rw) + (int64_t)(cs + min(e / rw, ncs - 1)) * ld]; },
        [&](int e, T v) { Xs[(e % rw) * (LP_COLS + 1) + e / rw] = e / rw < ncs ? v : T(0); });
    if (tid < LU_NB) lp[tid] = (pivot && tid < nb) ? pv[j0 + tid] - j0 : tid;
    __syncthreads();
    if (pivot && tid < LP_COLS) {
        for (int jj = 0; jj < nb; ++jj) {
            const int p = lp[jj];
            if (p != jj) {
                const T x = Xs[jj * (LP_COLS + 1) + tid];
                Xs[jj * (LP_COLS + 1) + tid] = Xs[p * (LP_COLS + 1) + tid];
                Xs[p * (LP_COLS + 1) + tid] = x;
            }
        }
    }
    __syncthreads();
    // U12 = L11^{-1} A12: one thread per column (a full panel: the column in registers)
    if (tid < LP_COLS) {
        if (nb == LU_NB) {
            T x[LU_NB];
#pragma unroll
            for (int r = 0; r < LU_NB; ++r) x[r] = Xs[r * (LP_COLS + 1) + tid];
            unit_lower_solve_regs(x, Ps, LU_NB + 1);
#pragma unroll
            for (int r = 0; r < LU_NB; ++r) Xs[r * (LP_COLS + 1) + tid] = x[r];
        } else {
            for (int r = 1; r < nb; ++r) {
                T v = Xs[r * (LP_COLS + 1) + tid];
                for (int k = 0; k < r; ++k) v -= Ps[r * (LU_NB + 1) + k] * Xs[k * (LP_COLS + 1) + tid];
                Xs[r * (LP_COLS + 1) + tid] = v;
            }
        }
    }
    __syncthreads();
    // rows [jend, rend): X -= L21 U12, each thread a block of rows (stride 32) x 4 columns
    {
        constexpr int RB = LP_MAXROWS / 32;
        const int cg = tid & 7, rg = tid >> 3;
        const int nr = rw - nb;
        T acc[RB][4];
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[i][u] = T(0);
        for (int k = 0; k < nb; ++k) {
            T x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) x[u] = Xs[k * (LP_COLS + 1) + 4 * cg + u];
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                const int r = nb + rg + 32 * i;
                const T l = r < rw ? Ps[r * (LU_NB + 1) + k] : T(0);
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[i][u] = fma(l, x[u], acc[i][u]);
            }
        }
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const int r = nb + rg + 32 * i;
            if (rg + 32 * i < nr) {
#pragma unroll
                for (int u = 0; u < 4; ++u) Xs[r * (LP_COLS + 1) + 4 * cg + u] -= acc[i][u];
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < rw * LP_COLS; e += 256) {
        const int r = e % rw, c = e / rw;
        if (c < ncs) A[(j0 + r) + (int64_t)(cs + c) * ld] = Xs[r * (LP_COLS + 1) + c];
    }
    if (fuse && blockIdx.x == 0 && jend < n) {
        __syncthreads();
        lu_panel_reg_body<T, 256>(n, A, ld, piv + poff[blockIdx.y], info + blockIdx.y, jend, pivot, mlim_next,
                                  [&](int r, int c) {
                                      return r < rend ? Xs[(r - j0) * (LP_COLS + 1) + c] : A[r + (int64_t)(jend + c) * ld];
                                  });
    }
}

// The deferred row exchanges of the L columns: column c (in the panel ending at e_c) receives the
// exchanges j = max(e_c, jf) .. n-1 in order (jf: first panel whose exchanges were deferred).  Each
// block holds LS_COLS columns' rows [jf, n) in LDS; one thread per column walks the exchanges.
constexpr int LS_COLS = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_lu_swap_left(const DMat *__restrict__ mats, const int64_t *__restrict__ poff,
                                                      T *__restrict__ Ab, const int32_t *__restrict__ piv, int jf) {
    const DMat m = mats[blockIdx.y];
    const int n = m.n;
    const int c0 = blockIdx.x * LS_COLS;
    if (c0 >= n || jf >= n) return;
    T *A = Ab + m.off;
    const int ld = m.ld;
    const int32_t *pv = piv + poff[blockIdx.y];
    const int rows = n - jf;
    extern __shared__ double shs[];
    T *Xs = reinterpret_cast<T *>(shs);                   // rows x LS_COLS, (i, c) at i * LS_COLS + c
    const int tid = threadIdx.x;
    staged_copy<8>(
        rows * LS_COLS, tid, 256, [&](int e) { return A[(jf + e % rows) + (int64_t)min(c0 + e / rows, n - 1) * ld]; },
        [&](int e, T v) { Xs[(e % rows) * LS_COLS + e / rows] = c0 + e / rows < n ? v : T(0); });
    __syncthreads();
    if (tid < LS_COLS && c0 + tid < n) {
        const int c = c0 + tid;
        const int ec = min(n, (c / LU_NB + 1) * LU_NB);
        for (int j = max(ec, jf); j < n; ++j) {
            const int p = pv[j];
            if (p != j) {
                const T x = Xs[(j - jf) * LS_COLS + tid];
                Xs[(j - jf) * LS_COLS + tid] = Xs[(p - jf) * LS_COLS + tid];
                Xs[(p - jf) * LS_COLS + tid] = x;
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < rows * LS_COLS; e += 256) {
        const int i = e % rows, c = e / rows;
        if (c0 + c < n) A[(jf + i) + (int64_t)(c0 + c) * ld] = Xs[i * LS_COLS + c];
    }
}

// Numerically singular factors: after the LU with partial pivoting, a pivot whose magnitude is at
// most 32 n eps times the largest pivot magnitude counts as a zero pivot (the backward error of the
// factorisation is of that order, so the matrix cannot be told from a singular one).  The first such
// column goes to info, as an exact zero pivot does; NaN pivots are caught the same way.  One block
// per matrix.
template <typename T>
__global__ __launch_bounds__(256) void k_lu_tiny_pivot(const DMat *__restrict__ mats, const T *__restrict__ Ab,
                                                       int32_t *__restrict__ info) {
    __shared__ double redm[4];
    __shared__ int redi[4];
    const DMat m = mats[blockIdx.x];
    const T *A = Ab + m.off;
    const int n = m.n, ld = m.ld;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double mx = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) mx = fmax(mx, fabs((double)A[j + (int64_t)j * ld]));
    mx = wave_max64(mx);
    if (lane == 0) redm[w] = mx;
    __syncthreads();
    mx = fmax(fmax(redm[0], redm[1]), fmax(redm[2], redm[3]));
    const double eps = sizeof(T) == 8 ? 2.220446049250313e-16 : 1.1920928955078125e-07;
    const double tiny = 32.0 * (double)n * eps * mx;
    int first = n;
    for (int j = threadIdx.x; j < n; j += 256)
        if (!(fabs((double)A[j + (int64_t)j * ld]) > tiny)) first = min(first, j);
    first = (int)wave_min64((double)first);
    if (lane == 0) redi[w] = first;
    __syncthreads();
    if (threadIdx.x == 0) {
        first = min(min(redi[0], redi[1]), min(redi[2], redi[3]));
        if (first < n && info[blockIdx.x] == 0) info[blockIdx.x] = first + 1;
    }
}

template <typename T>
int32_t lu_batched(const DMat *d_mats, const int64_t *d_poff, int nbatch, int maxn, T *A, int32_t *piv,
                   int32_t *info, bool pivot, hipStream_t s, int band) {
    if (nbatch == 0) return HKG_OK;
    HKG_HIP(hipMemsetAsync(info, 0, sizeof(int32_t) * nbatch, s));
    if (maxn == 0) return HKG_OK;
    // a band of half-width `band` (band < 0: dense): column j has no entry below row j + band, and
    // with row exchanges the rows of a panel reach at most 2 band columns past their diagonal
    const bool banded = band >= 0;
    // the left exchanges of fused panels are deferred when the deferred pass fits in LDS
    const bool defer = pivot && (size_t)maxn * LS_COLS * sizeof(T) <= (size_t)150 * 1024;
    int jf = -1;                        // first panel whose left exchanges are deferred
    bool factored = false;              // the panel at j0 was factored by the previous k_lu_post
    // one wave for narrow panels (float: up to 64 rows, where its registers suffice)
    const bool wide_wave = sizeof(T) == 8;
    auto panel_rows = [&](int j) {
        const int je = std::min(j + LU_NB, maxn);
        return (banded ? std::min(maxn, je + band) : maxn) - j;
    };
    auto uses_reg256 = [&](int rows) { return rows > (wide_wave ? 192 : 64) && rows <= 256; };
    for (int j0 = 0; j0 < maxn; j0 += LU_NB) {
        const int jend = std::min(j0 + LU_NB, maxn);
        const int mlim = banded ? std::min(maxn, jend + band) : maxn;           // panel rows end
        const int clim = banded ? std::min(maxn, jend + 2 * band) : maxn;       // columns reached
        const int rows = mlim - j0;
        const bool was_factored = factored;
        factored = false;
        if (was_factored)
            ;
        else if (rows <= 64)
            hipLaunchKernelGGL((k_lu_panel_wave<T, 1>), dim3(nbatch), dim3(64), 0, s, d_mats, d_poff, A, piv, info, j0,
                               (int)pivot, mlim);
        else if (wide_wave && rows <= 128)
            hipLaunchKernelGGL((k_lu_panel_wave<T, 2>), dim3(nbatch), dim3(64), 0, s, d_mats, d_poff, A, piv, info, j0,
                               (int)pivot, mlim);
        else if (wide_wave && rows <= 192)
            hipLaunchKernelGGL((k_lu_panel_wave<T, 3>), dim3(nbatch), dim3(64), 0, s, d_mats, d_poff, A, piv, info, j0,
                               (int)pivot, mlim);
        else if (rows <= 256)
            hipLaunchKernelGGL((k_lu_panel_reg<T, 256>), dim3(nbatch), dim3(256), 0, s, d_mats, d_poff, A, piv, info, j0,
                               (int)pivot, mlim);
        else if (rows <= 512)
            hipLaunchKernelGGL((k_lu_panel_reg<T, 512>), dim3(nbatch), dim3(512), 0, s, d_mats, d_poff, A, piv, info, j0,
                               (int)pivot, mlim);
        else if (rows <= PANEL_REG_ROWS)
            hipLaunchKernelGGL((k_lu_panel_reg<T, PANEL_REG_ROWS>), dim3(nbatch), dim3(PANEL_REG_ROWS), 0, s, d_mats,
                               d_poff, A, piv, info, j0, (int)pivot, mlim);
        else
            hipLaunchKernelGGL(k_lu_panel<T>, dim3(nbatch), dim3(256), 0, s, d_mats, d_poff, A, piv, info, j0,
                               (int)pivot);
        const int ccols = clim - jend, crows = mlim - jend;
        if (rows <= LP_MAXROWS) {
            // exchanges (right of the panel), U12 and the trailing update in one launch; the
            // exchanges of the columns on the left wait for k_lu_swap_left
            if (defer && jf < 0) jf = j0;
            if (pivot && !defer && j0 > 0)
                hipLaunchKernelGGL(k_lu_laswp<T>, dim3((j0 + 255) / 256, nbatch), dim3(256), 0, s, d_mats, d_poff, A,
                                   piv, j0, j0);     // the columns left of the panel only
            const int nright = ccols > 0 ? (ccols + LP_COLS - 1) / LP_COLS : 0;
            if (nright > 0) {
                // block 0 factors the next panel when that panel takes the 256-thread kernel
                const int jn = j0 + LU_NB;
                const bool fuse = jn < maxn && uses_reg256(panel_rows(jn));
                const int mlim_next = fuse ? jn + panel_rows(jn) : 0;
                const size_t shm = (size_t)rows * (LU_NB + 1 + LP_COLS + 1) * sizeof(T);
                hipLaunchKernelGGL(k_lu_post<T>, dim3(nright, nbatch), dim3(256), shm, s, d_mats, d_poff, A, piv, j0,
                                   mlim, clim, (int)pivot, (int)fuse, mlim_next, info);
                factored = fuse;
            }
            continue;
        }
        if (pivot) {
            int outside = maxn;
            hipLaunchKernelGGL(k_lu_laswp<T>, dim3((outside + 255) / 256, nbatch), dim3(256), 0, s, d_mats, d_poff, A,
                               piv, j0, 0x7fffffff);
        }
        if (ccols > 0) {
            hipLaunchKernelGGL(k_lu_trsm_row<T>, dim3((ccols + TRI_COLS - 1) / TRI_COLS, nbatch), dim3(TRI_COLS), 0, s,
                               d_mats, A, j0, clim);
            if (crows > 0) {
                const int tm = (crows + GT - 1) / GT, tn = (ccols + GT - 1) / GT;
                hipLaunchKernelGGL(k_lu_update<T>, dim3(tm * tn, nbatch), dim3(256), 0, s, d_mats, A, j0, tm, mlim,
                                   clim);
            }
        }
    }
    if (defer && jf >= 0 && jf + LU_NB < maxn) {
        const size_t shm = (size_t)(maxn - jf) * LS_COLS * sizeof(T);
        hipLaunchKernelGGL(k_lu_swap_left<T>, dim3((maxn - LU_NB + LS_COLS - 1) / LS_COLS, nbatch), dim3(256), shm, s,
                           d_mats, d_poff, A, piv, jf);
    }
    if (pivot && sizeof(T) == 8) hipLaunchKernelGGL(k_lu_tiny_pivot<T>, dim3(nbatch), dim3(256), 0, s, d_mats, (const T *)A, info);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}
template int32_t lu_batched<double>(const DMat *, const int64_t *, int, int, double *, int32_t *, int32_t *, bool,
                                    hipStream_t, int);

// ------------------------------------------------------------------------------------------------
// Blocked triangular solves op(T) X = X with many right-hand sides (T n x n, X n x ncol):
//   TRI_LOWER_UNIT        T unit lower (the L of an LU)
//   TRI_UPPER             T upper, non-unit (the U of an LU)
//   TRI_LOWER_UNIT_TRANS  T^T with T unit lower (i.e. unit upper read from the lower triangle)
// Diagonal blocks are solved one thread per column; off-diagonal blocks are GEMM updates.
// ------------------------------------------------------------------------------------------------
template <typename T, int MODE>
__global__ __launch_bounds__(TRI_COLS) void k_tri_diag(const TriJob *__restrict__ jobs, const T *__restrict__ Tb,
                                                       T *__restrict__ Xb, int k0) {
    const TriJob J = jobs[blockIdx.y];
    if (k0 >= J.n || (int)blockIdx.x * TRI_COLS >= J.ncol) return;
    const int nb = min(LU_NB, J.n - k0);
    __shared__ T Ls[LU_NB][LU_NB + 1];
    __shared__ T xs[LU_NB][TRI_COLS + 1];
    const T *Tm = Tb + J.offT;
    // Ls = op(T)[k0:k0+nb, k0:k0+nb] padded with the identity to LU_NB x LU_NB
    for (int e = threadIdx.x; e < LU_NB * LU_NB; e += TRI_COLS) {
        int r = e % LU_NB, c = e / LU_NB;
        T v = T(r == c ? 1 : 0);
        if (r < nb && c < nb)
            v = (MODE == TRI_LOWER_UNIT_TRANS) ? Tm[k0 + c + (int64_t)(k0 + r) * J.ldT]
                                               : Tm[k0 + r + (int64_t)(k0 + c) * J.ldT];
        Ls[r][c] = v;
    }
    const int col = blockIdx.x * TRI_COLS + threadIdx.x;
    const bool valid = col < J.ncol;
    T *X = Xb + J.offX + (int64_t)col * J.ldX + k0;
    {
        T v[LU_NB];
#pragma unroll
        for (int r = 0; r < LU_NB; ++r) v[r] = valid ? X[min(r, nb - 1)] : T(0);
#pragma unroll
        for (int r = 0; r < LU_NB; ++r) xs[r][threadIdx.x] = r < nb ? v[r] : T(0);
    }
    __syncthreads();
    solve_block_lds<T, MODE>(Ls, xs, threadIdx.x);
    if (valid)
        for (int r = 0; r < nb; ++r) X[r] = xs[r][threadIdx.x];
}

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_tri_update(const TriJob *__restrict__ jobs, const T *__restrict__ Tb,
                                                    T *__restrict__ Xb, int k0, int tiles_m_max, int band) {
    const TriJob J = jobs[blockIdx.y];
    if (k0 >= J.n) return;
    const int k1 = min(k0 + LU_NB, J.n);
    const T *Tm = Tb + J.offT;
    T *X = Xb + J.offX;
    const int tm = blockIdx.x % tiles_m_max, tn = blockIdx.x / tiles_m_max;
    // band >= 0: op(T) has no entry farther than `band` from the diagonal, so only that many rows
    // next to the block are updated
    if (MODE == TRI_LOWER_UNIT) {
        // rows below: X[k1:, :] -= T[k1:, k0:k1] X[k0:k1, :]
        const int r1 = band >= 0 ? min(J.n, k1 + band) : J.n;
        int M = r1 - k1;
        if (M <= 0 || tm * GT >= M || tn * GT >= J.ncol) return;
        gemm_tile<T>(M, J.ncol, k1 - k0, Tm + k1 + (int64_t)k0 * J.ldT, J.ldT, false, X + k0, J.ldX, false, X + k1,
                     J.ldX, T(-1), T(1), tm, tn);
    } else {
        // rows above: X[r0:k0, :] -= op(T)[r0:k0, k0:k1] X[k0:k1, :]
        const int r0 = band >= 0 ? max(0, k0 - band) : 0;
        int M = k0 - r0;
        if (M <= 0 || tm * GT >= M || tn * GT >= J.ncol) return;
        if (MODE == TRI_UPPER)
            gemm_tile<T>(M, J.ncol, k1 - k0, Tm + r0 + (int64_t)k0 * J.ldT, J.ldT, false, X + k0, J.ldX, false, X + r0,
                         J.ldX, T(-1), T(1), tm, tn);
        else
            gemm_tile<T>(M, J.ncol, k1 - k0, Tm + k0 + (int64_t)r0 * J.ldT, J.ldT, true, X + k0, J.ldX, false, X + r0,
                         J.ldX, T(-1), T(1), tm, tn);
    }
}

// Banded triangular solve in one launch: op(T) has no entry farther than `band` from the diagonal.
// Each block takes TB_COLS right-hand sides of one matrix and sweeps all its row blocks itself,
// the vectors in LDS: per row block, the band rows of op(T) next to it (and its diagonal block)
// are staged in LDS, every (row, column) subtracts its band product, and the diagonal block is
// solved wave-synchronously (lanes 0-31 and 32-63 of a wave hold one column each; a wave's LDS
// operations complete in order).  TIN: the right-hand sides are the rows of Xin (a square matrix
// with the layout of X), read as the transpose on the fly.
constexpr int TB_COLS = 8;

template <typename T, int MODE, bool TIN>
__global__ __launch_bounds__(256) void k_tri_band(const TriJob *__restrict__ jobs, const T *__restrict__ Tb,
                                                  const T *__restrict__ Xin, T *__restrict__ Xb, int band) {
    const TriJob J = jobs[blockIdx.y];
    const int c0 = blockIdx.x * TB_COLS;
    const int n = J.n;
    if (c0 >= J.ncol || n == 0) return;
    extern __shared__ double shb[];
    T *ys = reinterpret_cast<T *>(shb);                    // n x TB_COLS, (i, c) at i * TB_COLS + c
    T *Ls = ys + (int64_t)n * TB_COLS;                     // LU_NB rows x (band + LU_NB) of op(T)
    const int W = band + LU_NB;
    const T *Tm = Tb + J.offT;
    T *X = Xb + J.offX;
    const int tid = threadIdx.x, r = tid & 31, c = tid >> 5;
    if (TIN) {
        // right-hand side c0 + cc is row c0 + cc of Xin: eight consecutive entries per column of Xin
        const T *Xi = Xin + J.offX;
        staged_copy<8>(
            n * TB_COLS, tid, 256,
            [&](int q) { return Xi[min(c0 + q % TB_COLS, J.ncol - 1) + (int64_t)(q / TB_COLS) * J.ldX]; },
            [&](int q, T v) { ys[q] = c0 + q % TB_COLS < J.ncol ? v : T(0); });
    } else {
        staged_copy<8>(
            n * TB_COLS, tid, 256, [&](int q) { return X[q % n + (int64_t)min(c0 + q / n, J.ncol - 1) * J.ldX]; },
            [&](int q, T v) { ys[(q % n) * TB_COLS + q / n] = c0 + q / n < J.ncol ? v : T(0); });
    }
    const bool fwd = MODE == TRI_LOWER_UNIT;
    const int nblk = (n + LU_NB - 1) / LU_NB;
    for (int bb = 0; bb < nblk; ++bb) {
        const int b = fwd ? bb : nblk - 1 - bb;
        const int i0 = b * LU_NB, nb = min(LU_NB, n - i0);
        // columns k of op(T) staged: forward [ka, i0 + nb), backward [i0, kb)
        const int ka = fwd ? max(0, i0 - band) : i0;
        const int kb = fwd ? i0 + nb : min(n, i0 + nb + band);
        const int w = kb - ka;
        sync_lds();           // previous block done with Ls and with its rows of ys
        if (MODE == TRI_LOWER_UNIT_TRANS) {
            // op(T)[i][k] = T[k][i]: consecutive k are contiguous
            staged_copy<8>(
                LU_NB * w, tid, 256, [&](int e) { return Tm[(ka + e % w) + (int64_t)(i0 + min(e / w, nb - 1)) * J.ldT]; },
                [&](int e, T v) { Ls[(e / w) * W + e % w] = e / w < nb ? v : T(0); });
        } else {
            staged_copy<8>(
                LU_NB * w, tid, 256,
                [&](int e) { return Tm[(i0 + min(e % LU_NB, nb - 1)) + (int64_t)(ka + e / LU_NB) * J.ldT]; },
                [&](int e, T v) { Ls[(e % LU_NB) * W + e / LU_NB] = e % LU_NB < nb ? v : T(0); });
        }
        __syncthreads();
        // band product with the rows already solved
        if (r < nb) {
            T acc = T(0);
            if (fwd) {
                for (int k = ka; k < i0; ++k) acc = fma(Ls[r * W + (k - ka)], ys[k * TB_COLS + c], acc);
            } else {
                for (int k = i0 + nb; k < kb; ++k) acc = fma(Ls[r * W + (k - ka)], ys[k * TB_COLS + c], acc);
            }
            ys[(i0 + r) * TB_COLS + c] -= acc;
        }
        // the diagonal block: a full block by one thread per column in registers, the last
        // (partial) block wave-synchronously within each column
        const int dofs = fwd ? i0 - ka : 0;     // column offset of the block in Ls
        if (nb == LU_NB) {
            __syncthreads();
            if (tid < TB_COLS) {
                T x[LU_NB];
#pragma unroll
                for (int rr = 0; rr < LU_NB; ++rr) x[rr] = ys[(i0 + rr) * TB_COLS + tid];
                block_solve_regs<T, MODE>(x, Ls + dofs, W);
#pragma unroll
                for (int rr = 0; rr < LU_NB; ++rr) ys[(i0 + rr) * TB_COLS + tid] = x[rr];
            }
        } else if (fwd) {
            for (int k = 0; k < nb - 1; ++k) {
                const T yk = ys[(i0 + k) * TB_COLS + c];
                if (r > k && r < nb) ys[(i0 + r) * TB_COLS + c] -= Ls[r * W + dofs + k] * yk;
            }
        } else {
            for (int k = nb - 1; k >= 0; --k) {
                if (MODE == TRI_UPPER && r == k) ys[(i0 + k) * TB_COLS + c] /= Ls[k * W + dofs + k];
                const T yk = ys[(i0 + k) * TB_COLS + c];
                if (r < k) ys[(i0 + r) * TB_COLS + c] -= Ls[r * W + dofs + k] * yk;
            }
        }
    }
    sync_lds();
    // (TIN: scaled by D^{-1/2} on both sides, D the diagonal of T, into (offO, ldO))
    T *Xo = TIN ? Xb + J.offO : X;
    const int ldo = TIN ? J.ldO : J.ldX;
    for (int q = tid; q < n * TB_COLS; q += 256) {
        const int cc = q / n, i = q % n;
        if (c0 + cc < J.ncol) {
            T v = ys[i * TB_COLS + cc];
            if (TIN) {
                const int c = c0 + cc;
                v = v / (sqrt(Tm[i + (int64_t)i * J.ldT]) * sqrt(Tm[c + (int64_t)c * J.ldT]));
            }
            Xo[i + (int64_t)(c0 + cc) * ldo] = v;
        }
    }
}

// Wide banded triangular solve: TW_COLS right-hand sides per block and only a window of the solution
// in LDS (the band rows behind the current row block and the block itself, a ring of band + LU_NB
// rows), so the blocks are few and wide and all resident at once.  Per row block: the band of op(T)
// and the block's right-hand-side rows are staged; every thread takes a 4-row x 2-column tile of the
// band product (op(T) entries broadcast from LDS, two columns per 16-byte window read); threads
// 0..TW_COLS-1 solve the diagonal block for one column each in registers; the solved rows are
// written out by all threads, 32 consecutive rows of a column at a time.
constexpr int TW_COLS = 64;

template <typename T>
struct vec2_of;
template <>
struct vec2_of<double> {
    using type = double2;
};
template <>
struct vec2_of<float> {
    using type = float2;
};

size_t tri_bandw_lds(int band, size_t elem) {
    return ((size_t)(band + 2 * LU_NB) * TW_COLS + (size_t)LU_NB * (band + LU_NB)) * elem;
}

template <typename T, int MODE, bool TIN>
__global__ __launch_bounds__(256) void k_tri_bandw(const TriJob *__restrict__ jobs, const T *__restrict__ Tb,
                                                   const T *__restrict__ Xin, T *__restrict__ Xb, int band) {
    using T2 = typename vec2_of<T>::type;
    const TriJob J = jobs[blockIdx.y];
    const int c0 = blockIdx.x * TW_COLS;
    const int n = J.n;
    if (c0 >= J.ncol || n == 0) return;
    const int ncb = min(TW_COLS, J.ncol - c0);
    extern __shared__ double shw[];
    const int WIN = band + 2 * LU_NB;              // window rows; row r sits in slot r mod WIN
    const int W = band + LU_NB;                    // row stride of the staged band
    T *win = reinterpret_cast<T *>(shw);           // WIN x TW_COLS, row-major
    T *Ls = win + (int64_t)WIN * TW_COLS;          // LU_NB x W: Ls[r W + k - ka] = op(T)[i0 + r][k]
    const T *Tm = Tb + J.offT;
    T *X = Xb + J.offX;
    const T *Xi = TIN ? Xin + J.offX : X;
    const int tid = threadIdx.x;
    const bool fwd = MODE == TRI_LOWER_UNIT;
    const int nblk = (n + LU_NB - 1) / LU_NB;
    const int cp = tid & 31, rg = tid >> 5;        // band-product tile: rows 4 rg.., columns 2 cp..
    // the solved rows of a block out, 32 consecutive rows of a column at a time (the window keeps
    // them until the next block's rows are staged: its slots are band + 2 LU_NB, so the rows staged
    // next never land on the rows being written out)
    // (TIN: scaled by D^{-1/2} on both sides, D the diagonal of T, into (offO, ldO))
    T *Xo = TIN ? Xb + J.offO : X;
    const int ldo = TIN ? J.ldO : J.ldX;
    auto write_out = [&](int r0, int nr) {
        const int t0 = r0 % WIN;
        for (int q = tid; q < LU_NB * TW_COLS; q += 256) {
            const int rr = q % LU_NB, cc = q / LU_NB;
            if (rr < nr && cc < ncb) {
                int sl = t0 + rr;
                if (sl >= WIN) sl -= WIN;
                T v = win[sl * TW_COLS + cc];
                if (TIN) {
                    const int i = r0 + rr, c = c0 + cc;
                    v = v / (sqrt(Tm[i + (int64_t)i * J.ldT]) * sqrt(Tm[c + (int64_t)c * J.ldT]));
                }
                Xo[(r0 + rr) + (int64_t)(c0 + cc) * ldo] = v;
            }
        }
    };
    int pi0 = 0, pnb = 0;                          // the block solved last (pnb = 0: none)
    for (int bb = 0; bb < nblk; ++bb) {
        const int b = fwd ? bb : nblk - 1 - bb;
        const int i0 = b * LU_NB, nb = min(LU_NB, n - i0);
        const int ka = fwd ? max(0, i0 - band) : i0;
        const int kb = fwd ? i0 + nb : min(n, i0 + nb + band);
        const int w = kb - ka;
        const int s0 = i0 % WIN;                   // slot of row i0 (the block's rows are s0, s0+1, .. mod WIN)
        sync_lds();           // the previous block is solved; Ls is free
        if (pnb > 0) write_out(pi0, pnb);
        if (MODE == TRI_LOWER_UNIT_TRANS) {
            staged_copy<8>(
                LU_NB * w, tid, 256, [&](int e) { return Tm[(ka + e % w) + (int64_t)(i0 + min(e / w, nb - 1)) * J.ldT]; },
                [&](int e, T v) { Ls[(e / w) * W + e % w] = e / w < nb ? v : T(0); });
        } else {
            staged_copy<8>(
                LU_NB * w, tid, 256,
                [&](int e) { return Tm[(i0 + min(e % LU_NB, nb - 1)) + (int64_t)(ka + e / LU_NB) * J.ldT]; },
                [&](int e, T v) { Ls[(e % LU_NB) * W + e / LU_NB] = e % LU_NB < nb ? v : T(0); });
        }
        if (TIN) {            // right-hand side c is row c of Xin: consecutive columns contiguous
            staged_copy<8>(
                LU_NB * TW_COLS, tid, 256,
                [&](int q) {
                    return Xi[(c0 + min(q % TW_COLS, ncb - 1)) + (int64_t)(i0 + min(q / TW_COLS, nb - 1)) * J.ldX];
                },
                [&](int q, T v) {
                    const int rr = q / TW_COLS, cc = q % TW_COLS;
                    int sl = s0 + rr;
                    if (sl >= WIN) sl -= WIN;
                    if (rr < nb) win[sl * TW_COLS + cc] = cc < ncb ? v : T(0);
                });
        } else {              // 32 consecutive rows of a column at a time
            staged_copy<8>(
                LU_NB * TW_COLS, tid, 256,
                [&](int q) {
                    return Xi[(i0 + min(q % LU_NB, nb - 1)) + (int64_t)(c0 + min(q / LU_NB, ncb - 1)) * J.ldX];
                },
                [&](int q, T v) {
                    const int rr = q % LU_NB, cc = q / LU_NB;
                    int sl = s0 + rr;
                    if (sl >= WIN) sl -= WIN;
                    if (rr < nb) win[sl * TW_COLS + cc] = cc < ncb ? v : T(0);
                });
        }
        __syncthreads();
        // band product with the rows already solved (forward: [ka, i0); backward: [i0 + nb, kb))
        {
            const int kbeg = fwd ? ka : i0 + nb, kend = fwd ? i0 : kb;
            T acc[4][2];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u][0] = acc[u][1] = T(0);
            int sl = kbeg % WIN;
            for (int k = kbeg; k < kend; ++k) {
                const T2 yv = *reinterpret_cast<const T2 *>(win + sl * TW_COLS + 2 * cp);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const T l = Ls[(4 * rg + u) * W + (k - ka)];
                    acc[u][0] = fma(l, yv.x, acc[u][0]);
                    acc[u][1] = fma(l, yv.y, acc[u][1]);
                }
                if (++sl == WIN) sl = 0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int r = 4 * rg + u;
                if (r < nb) {
                    int slr = s0 + r;
                    if (slr >= WIN) slr -= WIN;
                    T2 *p = reinterpret_cast<T2 *>(win + slr * TW_COLS + 2 * cp);
                    T2 y = *p;
                    y.x -= acc[u][0];
                    y.y -= acc[u][1];
                    *p = y;
                }
            }
        }
        __syncthreads();
        // the diagonal block, one column per thread
        const int dofs = fwd ? i0 - ka : 0;        // column offset of the block in Ls
        if (tid < TW_COLS) {
            if (nb == LU_NB) {
                T x[LU_NB];
#pragma unroll
                for (int rr = 0; rr < LU_NB; ++rr) {
                    int sl = s0 + rr;
                    if (sl >= WIN) sl -= WIN;
                    x[rr] = win[sl * TW_COLS + tid];
                }
                block_solve_regs<T, MODE>(x, Ls + dofs, W);
#pragma unroll
                for (int rr = 0; rr < LU_NB; ++rr) {
                    int sl = s0 + rr;
                    if (sl >= WIN) sl -= WIN;
                    win[sl * TW_COLS + tid] = x[rr];
                }
            } else {
                auto at = [&](int r) -> T & {
                    int sl = s0 + r;
                    if (sl >= WIN) sl -= WIN;
                    return win[sl * TW_COLS + tid];
                };
                if (fwd) {
                    for (int k = 0; k < nb - 1; ++k) {
                        const T yk = at(k);
                        for (int r = k + 1; r < nb; ++r) at(r) -= Ls[r * W + dofs + k] * yk;
                    }
                } else {
                    for (int k = nb - 1; k >= 0; --k) {
                        if (MODE == TRI_UPPER) at(k) /= Ls[k * W + dofs + k];
                        const T yk = at(k);
                        for (int r = 0; r < k; ++r) at(r) -= Ls[r * W + dofs + k] * yk;
                    }
                }
            }
        }
        pi0 = i0;
        pnb = nb;
    }
    sync_lds();
    write_out(pi0, pnb);
}

static bool tri_band_fits_narrow(int maxn, int band, size_t elem) {
    return band >= 0 && ((size_t)maxn * TB_COLS + (size_t)LU_NB * (band + LU_NB)) * elem <= (size_t)144 * 1024;
}

bool tri_band_fits(int maxn, int band, size_t elem) {
    if (band >= 0 && tri_bandw_lds(band, elem) <= (size_t)80 * 1024) return true;
    return band >= 0 && ((size_t)maxn * TB_COLS + (size_t)LU_NB * (band + LU_NB)) * elem <= (size_t)144 * 1024;
}

template <typename T>
int32_t tri_solve_batched(const TriJob *d_jobs, int nbatch, int maxn, int maxcol, const T *Tm, T *X, int mode,
                          hipStream_t s, int band, const T *Xin) {
    if (nbatch == 0 || maxn == 0 || maxcol == 0) return HKG_OK;
    // wide blocks for many right-hand sides; a few (the coarse basis) keep the narrow blocks, which
    // give more blocks per matrix
    const bool narrow_ok = band >= 0 && !Xin && tri_band_fits_narrow(maxn, band, sizeof(T));
    if (band >= 0 && tri_bandw_lds(band, sizeof(T)) <= (size_t)80 * 1024 && !(maxcol <= TW_COLS / 2 && narrow_ok)) {
        const size_t shm = tri_bandw_lds(band, sizeof(T));
        const dim3 g((maxcol + TW_COLS - 1) / TW_COLS, nbatch);
        if (Xin) {
            if (mode != TRI_LOWER_UNIT) return HKG_EINVAL;
            hipLaunchKernelGGL((k_tri_bandw<T, TRI_LOWER_UNIT, true>), g, dim3(256), shm, s, d_jobs, Tm, Xin, X, band);
        } else if (mode == TRI_LOWER_UNIT) {
            hipLaunchKernelGGL((k_tri_bandw<T, TRI_LOWER_UNIT, false>), g, dim3(256), shm, s, d_jobs, Tm, X, X, band);
        } else if (mode == TRI_UPPER) {
            hipLaunchKernelGGL((k_tri_bandw<T, TRI_UPPER, false>), g, dim3(256), shm, s, d_jobs, Tm, X, X, band);
        } else {
            hipLaunchKernelGGL((k_tri_bandw<T, TRI_LOWER_UNIT_TRANS, false>), g, dim3(256), shm, s, d_jobs, Tm, X, X,
                               band);
        }
        HKG_HIP(hipGetLastError());
        return HKG_OK;
    }
    if (band >= 0 && tri_band_fits(maxn, band, sizeof(T))) {
        const size_t shm = ((size_t)maxn * TB_COLS + (size_t)LU_NB * (band + LU_NB)) * sizeof(T);
        const dim3 g((maxcol + TB_COLS - 1) / TB_COLS, nbatch);
        if (Xin) {
            if (mode != TRI_LOWER_UNIT) return HKG_EINVAL;
            hipLaunchKernelGGL((k_tri_band<T, TRI_LOWER_UNIT, true>), g, dim3(256), shm, s, d_jobs, Tm, Xin, X, band);
        } else if (mode == TRI_LOWER_UNIT) {
            hipLaunchKernelGGL((k_tri_band<T, TRI_LOWER_UNIT, false>), g, dim3(256), shm, s, d_jobs, Tm, X, X, band);
        } else if (mode == TRI_UPPER) {
            hipLaunchKernelGGL((k_tri_band<T, TRI_UPPER, false>), g, dim3(256), shm, s, d_jobs, Tm, X, X, band);
        } else {
            hipLaunchKernelGGL((k_tri_band<T, TRI_LOWER_UNIT_TRANS, false>), g, dim3(256), shm, s, d_jobs, Tm, X, X,
                               band);
        }
        HKG_HIP(hipGetLastError());
        return HKG_OK;
    }
    if (Xin) return HKG_EINVAL;
    const int nblk = (maxn + LU_NB - 1) / LU_NB;
    const int urows = band >= 0 ? std::min(maxn, band) : maxn;      // rows of one update at most
    const int tiles_m = (urows + GT - 1) / GT, tiles_n = (maxcol + GT - 1) / GT;
    const dim3 gd((maxcol + TRI_COLS - 1) / TRI_COLS, nbatch), gu(tiles_m * tiles_n, nbatch);
    for (int b = 0; b < nblk; ++b) {
        // block boundaries sit at multiples of LU_NB in every matrix, so one k0 serves the whole
        // batch: ascending for the lower solve, descending for the upper ones (blocks past a
        // matrix's own size return at once).
        if (mode == TRI_LOWER_UNIT) {
            int k0 = b * LU_NB;
            hipLaunchKernelGGL((k_tri_diag<T, TRI_LOWER_UNIT>), gd, dim3(TRI_COLS), 0, s, d_jobs, Tm, X, k0);
            hipLaunchKernelGGL((k_tri_update<T, TRI_LOWER_UNIT>), gu, dim3(256), 0, s, d_jobs, Tm, X, k0, tiles_m, band);
        } else {
            int k0 = (nblk - 1 - b) * LU_NB;
            if (mode == TRI_UPPER) {
                hipLaunchKernelGGL((k_tri_diag<T, TRI_UPPER>), gd, dim3(TRI_COLS), 0, s, d_jobs, Tm, X, k0);
                hipLaunchKernelGGL((k_tri_update<T, TRI_UPPER>), gu, dim3(256), 0, s, d_jobs, Tm, X, k0, tiles_m, band);
            } else {
                hipLaunchKernelGGL((k_tri_diag<T, TRI_LOWER_UNIT_TRANS>), gd, dim3(TRI_COLS), 0, s, d_jobs, Tm, X, k0);
                hipLaunchKernelGGL((k_tri_update<T, TRI_LOWER_UNIT_TRANS>), gu, dim3(256), 0, s, d_jobs, Tm, X, k0,
                                   tiles_m, band);
            }
        }
    }
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}
template int32_t tri_solve_batched<double>(const TriJob *, int, int, int, const double *, double *, int, hipStream_t,
                                           int, const double *);

// ------------------------------------------------------------------------------------------------
// L^{-1} applied to many right-hand sides, L the unit lower factor of a packed L D L^T with
// half-bandwidth band <= BW: one thread per right-hand side and no barrier after the staging.  Thread
// c keeps the last BW entries of its solution in registers (entry k in slot k mod BW, a compile-time
// index in the loop unrolled BW times), reads its right-hand side one block of BW entries ahead and
// writes its solution a block at a time.  Right-hand side c is row c of the input at the jobs'
// (offX, ldX) (consecutive threads read consecutive entries) or, with IN_COLS, its column c (a
// thread reads consecutive entries, two at a time); solution c is written as row c of the output at
// (offO, ldO) (consecutive threads write consecutive entries), with SCALE as D^{-1/2} Y D^{-1/2}.
// Row k of the band of L (L[k][k-1-i], i < BW, zero outside the band) and D^{-1/2} are staged in LDS.
// ------------------------------------------------------------------------------------------------
constexpr int TLW_THREADS = 256;

template <int BW, bool SCALE, bool IN_COLS>
__global__ __launch_bounds__(TLW_THREADS) void k_tri_lower_window(const TriJob *__restrict__ jobs,
                                                                  const double *__restrict__ Tb,
                                                                  const double *__restrict__ Xin,
                                                                  double *__restrict__ Xout, int band) {
    extern __shared__ double shl[];
    const TriJob J = jobs[blockIdx.y];
    const int n = J.n;
    if ((int)blockIdx.x * TLW_THREADS >= J.ncol || n == 0) return;
    const int tid = threadIdx.x, c = blockIdx.x * TLW_THREADS + tid;
    double *Lb = shl;                            // n x BW
    double *dsc = Lb + (int64_t)n * BW;          // n
    const double *Tm = Tb + J.offT;
    staged_copy<8>(
        n * BW, tid, TLW_THREADS,
        [&](int e) {
            const int k = e / BW, i = e % BW, col = max(k - 1 - i, 0);
            return Tm[k + (int64_t)col * J.ldT];
        },
        [&](int e, double v) {
            const int k = e / BW, i = e % BW;
            Lb[e] = (i < band && k - 1 - i >= 0) ? v : 0.0;
        });
    if (SCALE)
        for (int k = tid; k < n; k += TLW_THREADS) dsc[k] = 1.0 / sqrt(Tm[k + (int64_t)k * J.ldT]);
    __syncthreads();
    if (c >= J.ncol) return;
    const int64_t ldx = J.ldX, ldo = J.ldO;
    const double *xin = IN_COLS ? Xin + J.offX + (int64_t)c * ldx : Xin + J.offX + c;
    double *out = Xout + J.offO + c;             // entry k at out[k ldO]
    const double sc = SCALE ? dsc[min(c, n - 1)] : 1.0;
    const int klast = IN_COLS ? (n - 1) & ~1 : n - 1;   // pairs (k, k + 1) stay inside the padded column
    auto load_block = [&](int k0, double *b) {
        if (IN_COLS) {
#pragma unroll
            for (int u = 0; u < BW; u += 2) {
                const double2 v = *reinterpret_cast<const double2 *>(xin + min(k0 + u, klast));
                b[u] = v.x;
                b[u + 1] = v.y;
            }
        } else {
#pragma unroll
            for (int u = 0; u < BW; ++u) b[u] = xin[(int64_t)min(k0 + u, klast) * ldx];
        }
    };
    double win[BW], Lc[BW], b[BW];
#pragma unroll
    for (int u = 0; u < BW; ++u) {
        win[u] = 0.0;
        Lc[u] = Lb[u];
    }
    load_block(0, b);
    for (int k0 = 0; k0 < n; k0 += BW) {
#pragma unroll
        for (int u = 0; u < BW; ++u) {
            // the next row of the band is read while this one is used
            const double *Ln = Lb + (int64_t)min(k0 + u + 1, n - 1) * BW;
            double Lx[BW];
#pragma unroll
            for (int i = 0; i < BW; ++i) Lx[i] = Ln[i];
            // four partial sums: a chain of dependent double FMAs is long-latency
            double acc[4] = {b[u], 0.0, 0.0, 0.0};
#pragma unroll
            for (int i = BW - 1; i >= 1; --i) acc[i & 3] = fma(-Lc[i], win[(u - 1 - i + 2 * BW) % BW], acc[i & 3]);
            double x = fma(-Lc[0], win[(u - 1 + BW) % BW], (acc[0] + acc[1]) + (acc[2] + acc[3]));
            asm volatile("" : "+v"(x) : : "memory");    // no band row read before the step ends
            win[u] = x;
#pragma unroll
            for (int i = 0; i < BW; ++i) Lc[i] = Lx[i];
        }
        // the next block's right-hand side is read before this block's solution is written, so that
        // waiting for the reads does not wait for the writes
        load_block(k0 + BW, b);
#pragma unroll
        for (int u = 0; u < BW; ++u) {
            const int k = k0 + u;
            if (k < n) out[k * ldo] = SCALE ? win[u] * dsc[k] * sc : win[u];
        }
    }
}

static int tlw_width(int band) {
    if (band < 0) return 0;
    for (int bw : {16, 24, 32})
        if (band <= bw) return bw;
    return 0;
}

static size_t tlw_lds(int maxn, int bw) { return (size_t)maxn * (bw + 1) * sizeof(double); }

bool tri_lower_window_fits(int maxn, int band) {
    const int bw = tlw_width(band);
    return bw > 0 && tlw_lds(maxn, bw) <= (size_t)156 * 1024;
}

int32_t tri_lower_window_batched(const TriJob *d_jobs, int nbatch, int maxn, int maxcol, const double *Tm,
                                 const double *Xin, bool in_cols, double *Xout, bool scale, int band,
                                 hipStream_t s) {
    if (nbatch == 0 || maxn == 0 || maxcol == 0) return HKG_OK;
    if (!tri_lower_window_fits(maxn, band)) return HKG_EINVAL;
    const int bw = tlw_width(band);
    const size_t shm = tlw_lds(maxn, bw);
    const dim3 g((maxcol + TLW_THREADS - 1) / TLW_THREADS, nbatch);
#define HKG_TLW(BW)                                                                                                    \
    if (bw == BW) {                                                                                                    \
        if (scale && in_cols) hipLaunchKernelGGL((k_tri_lower_window<BW, true, true>), g, dim3(TLW_THREADS), shm, s,  \
                                                 d_jobs, Tm, Xin, Xout, band);                                         \
        else if (!scale && !in_cols) hipLaunchKernelGGL((k_tri_lower_window<BW, false, false>), g, dim3(TLW_THREADS),  \
                                                        shm, s, d_jobs, Tm, Xin, Xout, band);                          \
        else return HKG_EINVAL;                                                                                        \
    }
    HKG_TLW(16)
    HKG_TLW(24)
    HKG_TLW(32)
#undef HKG_TLW
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// L^{-T} applied to a few right-hand sides in place (the coarse basis: L^T X = X with L the unit
// lower factor of a packed L D L^T, half-bandwidth band <= BW), backward, one thread per right-hand
// side: x[k] = x[k] - sum_i L[k + 1 + i][k] x[k + 1 + i].  Column k of L below the diagonal is row k
// of the staged band; thread c keeps the last BW entries solved in registers as above and reads and
// writes its own column of X a block at a time.
template <int BW>
__global__ __launch_bounds__(64) void k_tri_ltrans_window(const TriJob *__restrict__ jobs, const double *__restrict__ Tb,
                                                          double *__restrict__ Xb, int band) {
    extern __shared__ double shl[];
    const TriJob J = jobs[blockIdx.y];
    const int n = J.n;
    if ((int)blockIdx.x * 64 >= J.ncol || n == 0) return;
    const int tid = threadIdx.x, c = blockIdx.x * 64 + tid;
    double *Lt = shl;                            // n x BW: Lt[k][i] = L[k + 1 + i][k]
    const double *Tm = Tb + J.offT;
    staged_copy<8>(
        n * BW, tid, 64, [&](int e) { const int k = e / BW, i = e % BW; return Tm[min(k + 1 + i, n - 1) + (int64_t)k * J.ldT]; },
        [&](int e, double v) {
            const int k = e / BW, i = e % BW;
            Lt[e] = (i < band && k + 1 + i < n) ? v : 0.0;
        });
    __syncthreads();
    if (c >= J.ncol) return;
    double *x = Xb + J.offX + (int64_t)c * J.ldX;
    double win[BW], Lc[BW], b[BW];
#pragma unroll
    for (int u = 0; u < BW; ++u) {
        win[u] = 0.0;
        Lc[u] = Lt[(int64_t)(n - 1) * BW + u];
    }
    for (int k0 = n - 1; k0 >= 0; k0 -= BW) {
        // step u of the block solves row k0 - u
#pragma unroll
        for (int u = 0; u < BW; ++u) b[u] = x[max(k0 - u, 0)];
#pragma unroll
        for (int u = 0; u < BW; ++u) {
            const double *Ln = Lt + (int64_t)max(k0 - u - 1, 0) * BW;
            double Lx[BW];
#pragma unroll
            for (int i = 0; i < BW; ++i) Lx[i] = Ln[i];
            double acc[4] = {b[u], 0.0, 0.0, 0.0};
#pragma unroll
            for (int i = BW - 1; i >= 1; --i) acc[i & 3] = fma(-Lc[i], win[(u - 1 - i + 2 * BW) % BW], acc[i & 3]);
            double xk = fma(-Lc[0], win[(u - 1 + BW) % BW], (acc[0] + acc[1]) + (acc[2] + acc[3]));
            asm volatile("" : "+v"(xk) : : "memory");   // no band row read before the step ends
            win[u] = xk;
#pragma unroll
            for (int i = 0; i < BW; ++i) Lc[i] = Lx[i];
        }
#pragma unroll
        for (int u = 0; u < BW; ++u)
            if (k0 - u >= 0) x[k0 - u] = win[u];
    }
}

int32_t tri_ltrans_window_batched(const TriJob *d_jobs, int nbatch, int maxn, int maxcol, const double *Tm, double *X,
                                  int band, hipStream_t s) {
    if (nbatch == 0 || maxn == 0 || maxcol == 0) return HKG_OK;
    if (!tri_lower_window_fits(maxn, band)) return HKG_EINVAL;
    const int bw = tlw_width(band);
    const size_t shm = (size_t)maxn * bw * sizeof(double);
    const dim3 g((maxcol + 63) / 64, nbatch);
    if (bw == 16) hipLaunchKernelGGL(k_tri_ltrans_window<16>, g, dim3(64), shm, s, d_jobs, Tm, X, band);
    else if (bw == 24) hipLaunchKernelGGL(k_tri_ltrans_window<24>, g, dim3(64), shm, s, d_jobs, Tm, X, band);
    else hipLaunchKernelGGL(k_tri_ltrans_window<32>, g, dim3(64), shm, s, d_jobs, Tm, X, band);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}


// ------------------------------------------------------------------------------------------------
// Inverse of one packed LU (P A = L U) by recursive block triangular inversion: the LU_NB diagonal
// blocks of L (unit lower) and U are inverted here; the driver then joins neighbouring blocks level
// by level with GEMMs ([[A, 0], [C, D]]^{-1} has off-diagonal block -D^{-1} C A^{-1}), forms
// U^{-1} (L^{-1} P) and A^{-1} = U^{-1} L^{-1} P.
// ------------------------------------------------------------------------------------------------
// grid (diagonal blocks, 2): y = 0 inverts the L block, y = 1 the U block; thread t computes column
// t of the block inverse from the block staged in LDS
__global__ __launch_bounds__(LU_NB) void k_tri_diag_inv(const double *__restrict__ LU, int n, int ld,
                                                        double *__restrict__ Linv, double *__restrict__ Uinv,
                                                        int ldo) {
    __shared__ double Ts[LU_NB][LU_NB + 1];
    __shared__ double Xs[LU_NB][LU_NB + 1];
    const int r0 = blockIdx.x * LU_NB, nb = min(LU_NB, n - r0), t = threadIdx.x;
    const bool upper = blockIdx.y == 1;
    for (int e = t; e < LU_NB * LU_NB; e += LU_NB) {
        const int i = e % LU_NB, j = e / LU_NB;
        Ts[i][j] = (i < nb && j < nb) ? LU[(r0 + i) + (int64_t)(r0 + j) * ld] : 0.0;
    }
    __syncthreads();
    if (t < nb) {
        if (!upper) {
            for (int i = 0; i < nb; ++i) {
                double s = (i == t) ? 1.0 : 0.0;
                for (int k = t; k < i; ++k) s -= Ts[i][k] * Xs[k][t];
                Xs[i][t] = (i < t) ? 0.0 : s;
            }
        } else {
            for (int i = nb - 1; i >= 0; --i) {
                double s = (i == t) ? 1.0 : 0.0;
                for (int k = i + 1; k <= t; ++k) s -= Ts[i][k] * Xs[k][t];
                Xs[i][t] = (i > t) ? 0.0 : s / Ts[i][i];
            }
        }
    }
    __syncthreads();
    double *out = upper ? Uinv : Linv;
    for (int e = t; e < nb * nb; e += LU_NB) {
        const int i = e % nb, j = e / nb;
        out[(r0 + i) + (int64_t)(r0 + j) * ldo] = Xs[i][j];
    }
}

int32_t tri_diag_inverse(const double *LU, int n, int ld, double *Linv, double *Uinv, int ldo, hipStream_t s) {
    const int nblk = (n + LU_NB - 1) / LU_NB;
    hipLaunchKernelGGL(k_tri_diag_inv, dim3(nblk, 2), dim3(LU_NB), 0, s, LU, n, ld, Linv, Uinv, ldo);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// out[:, c] = X[:, sigma(c)] with P e_c = e_{sigma(c)} for the row exchanges piv applied in order
__global__ __launch_bounds__(256) void k_gather_pivot_columns(int n, const double *__restrict__ X, int ldx,
                                                              const int32_t *__restrict__ piv,
                                                              double *__restrict__ out, int ldo) {
    __shared__ int sig;
    const int c = blockIdx.x;
    if (threadIdx.x == 0) {
        int r = c;
        for (int j = 0; j < n; ++j) {
            const int p = piv[j];
            if (r == j) r = p;
            else if (r == p) r = j;
        }
        sig = r;
    }
    __syncthreads();
    const double *src = X + (int64_t)sig * ldx;
    double *dst = out + (int64_t)c * ldo;
    for (int i = threadIdx.x; i < n; i += 256) dst[i] = src[i];
}

int32_t gather_pivot_columns(int n, const double *X, int ldx, const int32_t *piv, double *out, int ldo, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_pivot_columns, dim3(n), dim3(256), 0, s, n, X, ldx, piv, out, ldo);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// ------------------------------------------------------------------------------------------------
// A^{-1} from one packed LU (P A = L U, leading dimension ld), column by column: column j of A^{-1}
// solves L U x = P e_j.  The columns are independent, so each block takes INV_CB of them and runs
// both triangular sweeps itself with its vectors in LDS; the whole inverse is one launch (no
// sequence of block steps across the grid).  A sweep goes by blocks of LU_NB rows: the block's rows
// subtract the product with the part already solved (one thread per row and column, reading the
// factor from L2), then are multiplied by the inverse of the diagonal block (from tri_diag_inverse,
// at (i0, i0) of Dinv with leading dimension ldd).
// ------------------------------------------------------------------------------------------------
constexpr int INV_CB = 8;         // right-hand sides per block
constexpr int INV_NT = 1024;      // threads: LU_NB rows x INV_KQ groups of the summation index
constexpr int INV_KQ = INV_NT / LU_NB;

// acc(r, c) over k in [ka, kb) for every column c: thread (r, q) sums k = ka + q, ka + q + INV_KQ, ...
// (eight loads in flight), then the INV_KQ partial sums of each (r, c) are added in q order
__device__ __forceinline__ void inv_partial(const double *__restrict__ LU, int ld, int i0, int nb, int ka, int kb,
                                            const double *ys, double *part, int tid) {
    const int r = tid % LU_NB, q = tid / LU_NB;

    double acc[INV_CB];
#pragma unroll
    for (int c = 0; c < INV_CB; ++c) acc[c] = 0.0;
    const double *rp = LU + i0 + min(r, nb - 1);     // rows past the block's end repeat its last
    for (int k0 = ka + q; k0 < kb; k0 += 8 * INV_KQ) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = rp[(int64_t)min(k0 + u * INV_KQ, kb - 1) * ld];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + u * INV_KQ;
            if (k < kb) {
#pragma unroll
                for (int c = 0; c < INV_CB; ++c) acc[c] = fma(a[u], ys[k * INV_CB + c], acc[c]);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < INV_CB; ++c) part[(q * LU_NB + r) * INV_CB + c] = acc[c];
}

// y_B = Dinv_BB (y_B - acc): the partial sums are added, then the block is multiplied by the
// inverted diagonal block
__device__ __forceinline__ void inv_block_step(const double *__restrict__ Dinv, int ldd, int i0, int nb, double *ys,
                                               const double *part, double (*Ts)[LU_NB + 1], double (*tb)[INV_CB],
                                               int tid) {
    for (int e = tid; e < LU_NB * LU_NB; e += INV_NT) {
        const int rr = e % LU_NB, cc = e / LU_NB;
        Ts[rr][cc] = (rr < nb && cc < nb) ? Dinv[i0 + rr + (int64_t)(i0 + cc) * ldd] : 0.0;
    }
    __syncthreads();
    if (tid < LU_NB * INV_CB) {
        const int r = tid / INV_CB, c = tid % INV_CB;
        double acc = 0.0;
        for (int q = 0; q < INV_KQ; ++q) acc += part[(q * LU_NB + r) * INV_CB + c];
        tb[r][c] = r < nb ? ys[(i0 + r) * INV_CB + c] - acc : 0.0;
    }
    __syncthreads();
    if (tid < LU_NB * INV_CB) {
        const int r = tid / INV_CB, c = tid % INV_CB;
        if (r < nb) {
            double v = 0.0;
#pragma unroll 8
            for (int kk = 0; kk < LU_NB; ++kk) v = fma(Ts[r][kk], tb[kk][c], v);
            ys[(i0 + r) * INV_CB + c] = v;
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(INV_NT) void k_lu_inverse_cols(const double *__restrict__ LU, int n, int ld,
                                                            const int32_t *__restrict__ piv,
                                                            const double *__restrict__ Linv,
                                                            const double *__restrict__ Uinv, int ldd,
                                                            double *__restrict__ X, int ldx, int uband) {
    extern __shared__ double sh[];
    double *ys = sh;                               // n x INV_CB, entry (i, c) at i * INV_CB + c
    double *part = sh + (int64_t)n * INV_CB;       // INV_KQ x LU_NB x INV_CB partial sums
    __shared__ double Ts[LU_NB][LU_NB + 1];        // inverse of the current diagonal block
    __shared__ double tb[LU_NB][INV_CB];
    __shared__ int tstart[INV_CB];
    __shared__ int tmin;
    const int tid = threadIdx.x;
    const int c0 = blockIdx.x * INV_CB;
    // P e_j = e_t: follow index j through the exchanges in order
    if (tid < INV_CB) {
        int t = c0 + tid;
        if (t < n) {
            for (int k = 0; k < n; ++k) {
                const int p = piv[k];
                if (t == k) t = p;
                else if (t == p) t = k;
            }
        }
        tstart[tid] = t;
    }
    for (int q = tid; q < n * INV_CB; q += INV_NT) ys[q] = 0.0;
    __syncthreads();
    if (tid < INV_CB && c0 + tid < n) ys[tstart[tid] * INV_CB + tid] = 1.0;
    if (tid == 0) {
        int t = n;
        for (int c = 0; c < INV_CB; ++c)
            if (c0 + c < n) t = min(t, tstart[c]);
        tmin = t;
    }
    __syncthreads();
    const int nblk = (n + LU_NB - 1) / LU_NB;
    // forward sweep, L unit lower: y_B = L_BB^{-1} (y_B - L[B, :i0] y[:i0]); the blocks above the
    // first nonzero start entry stay zero
    const int bfirst = tmin / LU_NB;
    for (int b = bfirst; b < nblk; ++b) {
        const int i0 = b * LU_NB, nb = min(LU_NB, n - i0);
        inv_partial(LU, ld, i0, nb, bfirst * LU_NB, i0, ys, part, tid);
        inv_block_step(Linv, ldd, i0, nb, ys, part, Ts, tb, tid);
    }
    // backward sweep, U upper: x_B = U_BB^{-1} (y_B - U[B, i1:] x[i1:]); U has no entry farther
    // than uband from the diagonal when uband >= 0
    for (int b = nblk - 1; b >= 0; --b) {
        const int i0 = b * LU_NB, nb = min(LU_NB, n - i0), i1 = i0 + nb;
        inv_partial(LU, ld, i0, nb, i1, uband >= 0 ? min(n, i1 + uband) : n, ys, part, tid);
        inv_block_step(Uinv, ldd, i0, nb, ys, part, Ts, tb, tid);
    }
    for (int q = tid; q < n * INV_CB; q += INV_NT) {
        const int cc = q / n, ii = q % n;
        if (c0 + cc < n) X[ii + (int64_t)(c0 + cc) * ldx] = ys[ii * INV_CB + cc];
    }
}

int64_t lu_inverse_cols_lds(int n) {
    return ((int64_t)n * INV_CB + (int64_t)INV_KQ * LU_NB * INV_CB) * (int64_t)sizeof(double);
}

int32_t lu_inverse_cols(const double *LU, int n, int ld, const int32_t *piv, const double *Linv, const double *Uinv,
                        int ldd, double *X, int ldx, int uband, hipStream_t s) {
    const size_t shm = (size_t)lu_inverse_cols_lds(n);
    hipLaunchKernelGGL(k_lu_inverse_cols, dim3((n + INV_CB - 1) / INV_CB), dim3(INV_NT), shm, s, LU, n, ld, piv, Linv,
                       Uinv, ldd, X, ldx, uband);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// ------------------------------------------------------------------------------------------------
// helpers: X = P * I (row exchanges of an LU applied to the identity), transposes, copies
// ------------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_perm_identity(const DMat *__restrict__ mats, const int64_t *__restrict__ poff,
                                                       const int32_t *__restrict__ piv, T *__restrict__ Xb) {
    const DMat m = mats[blockIdx.y];
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= m.n) return;
    T *X = Xb + m.off + (int64_t)c * m.ld;
    for (int i = 0; i < m.n; ++i) X[i] = T(0);
    // column c of P: follow the exchanges applied in order to row c's unit entry
    int r = c;
    const int32_t *pv = piv + poff[blockIdx.y];
    for (int j = 0; j < m.n; ++j) {
        int p = pv[j];
        if (r == j) r = p;
        else if (r == p) r = j;
    }
    X[r] = T(1);
}

template <typename T>
int32_t perm_identity_batched(const DMat *d_mats, const int64_t *d_poff, int nbatch, int maxn, const int32_t *piv,
                              T *X, hipStream_t s) {
    if (nbatch == 0 || maxn == 0) return HKG_OK;
    hipLaunchKernelGGL(k_perm_identity<T>, dim3((maxn + 255) / 256, nbatch), dim3(256), 0, s, d_mats, d_poff, piv, X);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}
template int32_t perm_identity_batched<double>(const DMat *, const int64_t *, int, int, const int32_t *, double *,
                                               hipStream_t);

// X = I for every matrix of the list (grid-stride over the n x n entries of the block's matrix)
__global__ __launch_bounds__(256) void k_identity(const DMat *__restrict__ mats, double *__restrict__ Xb) {
    const DMat m = mats[blockIdx.y];
    const int64_t total = (int64_t)m.n * m.n;
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int r = (int)(e % m.n), c = (int)(e / m.n);
        Xb[m.off + r + (int64_t)c * m.ld] = r == c ? 1.0 : 0.0;
    }
}

int32_t identity_batched(const DMat *d_mats, int nbatch, int maxn, double *X, hipStream_t s) {
    if (nbatch == 0 || maxn == 0) return HKG_OK;
    const int64_t total = (int64_t)maxn * maxn;
    const int blocks = (int)std::min<int64_t>(256, (total + 255) / 256);
    hipLaunchKernelGGL(k_identity, dim3(blocks, nbatch), dim3(256), 0, s, d_mats, X);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

__global__ __launch_bounds__(256) void k_copy_blocks(const CopyJob *__restrict__ jobs, const double *__restrict__ src,
                                                     double *__restrict__ dst) {
    const CopyJob J = jobs[blockIdx.y];
    const int64_t total = (int64_t)J.rows * J.cols;
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int r = (int)(e % J.rows), c = (int)(e / J.rows);
        dst[J.offD + r + (int64_t)c * J.ldD] = src[J.offS + r + (int64_t)c * J.ldS];
    }
}

int32_t copy_blocks_batched(const CopyJob *d_jobs, int nbatch, int64_t max_elems, const double *src, double *dst,
                            hipStream_t s) {
    if (nbatch == 0 || max_elems == 0) return HKG_OK;
    const int blocks = (int)std::min<int64_t>(512, (max_elems + 255) / 256);
    hipLaunchKernelGGL(k_copy_blocks, dim3(blocks, nbatch), dim3(256), 0, s, d_jobs, src, dst);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// out = in^T for square matrices with the same descriptors (separate buffers)
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const DMat *__restrict__ mats, const T *__restrict__ in,
                                                   T *__restrict__ out, int tiles_max) {
    const DMat m = mats[blockIdx.y];
    __shared__ T tile[32][33];
    const int ti = blockIdx.x % tiles_max, tj = blockIdx.x / tiles_max;
    if (ti * 32 >= m.n || tj * 32 >= m.n) return;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        int i = ti * 32 + tx, j = tj * 32 + r;
        if (i < m.n && j < m.n) tile[r][tx] = in[m.off + i + (int64_t)j * m.ld];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        int i = tj * 32 + tx, j = ti * 32 + r;   // out[i, j] = in[j, i]
        if (i < m.n && j < m.n) out[m.off + i + (int64_t)j * m.ld] = tile[tx][r];
    }
}

template <typename T>
int32_t transpose_batched(const DMat *d_mats, int nbatch, int maxn, const T *in, T *out, hipStream_t s) {
    if (nbatch == 0 || maxn == 0) return HKG_OK;
    int tiles = (maxn + 31) / 32;
    hipLaunchKernelGGL(k_transpose<T>, dim3(tiles * tiles, nbatch), dim3(256), 0, s, d_mats, in, out, tiles);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}
template int32_t transpose_batched<double>(const DMat *, int, int, const double *, double *, hipStream_t);

// FP64 -> FP32 copy of a flat buffer
__global__ void k_cast_f64_f32(const double *__restrict__ in, float *__restrict__ out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

int32_t cast_f64_f32(const double *in, float *out, int64_t n, hipStream_t s) {
    if (n == 0) return HKG_OK;
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_cast_f64_f32, dim3(blocks), dim3(256), 0, s, in, out, n);
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

// ------------------------------------------------------------------------------------------------
// Batched inverse of small dense matrices by Gauss-Jordan elimination with partial pivoting, one
// workgroup per matrix and the whole matrix in registers: thread (r, g) holds row r, columns
// g, g + 4, g + 8, ... (CPT <= 64 of them; R a multiple of 64, so g is the same across a wave), and
// the 4 x R threads cover n <= min(R, 4 CPT).
// Step k picks the pivot row p among the rows not yet pivoted (largest |a_ik|, found by every wave
// from the column staged in LDS, DPP arg-max, lowest index on ties), stages row p divided by the
// pivot (with 1/pivot in column k), and updates every other row i: a_i -= a_ik * row_p after
// a_ik := 0.  Rows are never exchanged: physical row p_k holds logical row k, and the final store
// unscrambles (A^{-1})[k, p_j] = a[p_k, j].  The pivots are those of an LU with partial pivoting;
// info = 1 when one of them is at most 32 n eps times the largest (or any is not finite).
// Column slots rotate: the four columns of slot s sit in a[0] while their four steps run, then
// the slots move down by one, so the pivot column is a fixed register (no run-time indexing of the
// register array, one copy of the step code).  Two barriers per step, the column and pivot-row
// buffers double-buffered.  A step is a latency chain (barrier, LDS round trips, arg-max, staging,
// FMAs): about 3 us at n = 200, against the dozens of launches of a blocked LU and its inverse.
// Job: CopyJob {offS in, offD out, rows = cols = n, ldS, ldD}.
// ------------------------------------------------------------------------------------------------
template <int CPT, int R>
__global__ __launch_bounds__(4 * R) void k_inv_gj(const CopyJob *__restrict__ jobs, const double *__restrict__ in,
                                                  double *__restrict__ out, int32_t *__restrict__ info) {
    static_assert(R % 64 == 0, "a wave holds one column group");
    constexpr int G = 4;
    __shared__ double colv[2][R];
    __shared__ double cola[2][R];
    __shared__ double prow[2][G * CPT];
    __shared__ int32_t pk[R], kof[R];
    const CopyJob J = jobs[blockIdx.x];
    const int n = J.rows;
    const int t = threadIdx.x, r = t % R, g = t / R, lane = t & 63;
    if (n <= 0) {
        if (t == 0) info[blockIdx.x] = 0;
        return;
    }
    for (int i = t; i < R; i += G * R) {
        pk[i] = 0;
        kof[i] = 0;
    }
    const bool live = r < n;
    const int rc = min(r, n - 1);
    double a[CPT];
    const double *src = in + J.offS + rc;
#pragma unroll
    for (int q0 = 0; q0 < CPT; q0 += 4) {
#pragma unroll
        for (int u = 0; u < 4 && q0 + u < CPT; ++u) {
            const int j = G * (q0 + u) + g;
            double v = src[(int64_t)min(j, n - 1) * J.ldS];
            asm volatile("" : "+v"(v));     // keep the (in-range) load unconditional: no branch per load
            a[q0 + u] = (live && j < n) ? v : 0.0;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    bool used = false, finite = true;
    double pmax = 0.0, pmin = INFINITY;
    const int nslot = (n + G - 1) / G;
#pragma unroll 1
    for (int sl = 0; sl < nslot; ++sl) {
        const int gend = min(G, n - G * sl);
#pragma unroll 1
        for (int gk = 0; gk < gend; ++gk) {
            const int k = G * sl + gk;
            const int b = k & 1;
            if (g == gk) {
                colv[b][r] = a[0];
                cola[b][r] = (live && !used) ? fabs(a[0]) : -1.0;
            }
            __syncthreads();
            double best = -2.0;
            int bi = 0;
#pragma unroll
            for (int i0 = 0; i0 < R; i0 += 64) {
                const double x = cola[b][i0 + lane];
                if (x > best) {
                    best = x;
                    bi = i0 + lane;
                }
            }
            argmax_wave64(best, bi);
            // no admissible row (a column of NaNs): flagged; p is then some row < R, and the final
            // store clamps every index into the matrix
            const int p = __builtin_amdgcn_readfirstlane(bi);
            const double piv = colv[b][p];
            const double apiv = fabs(piv);
            finite = finite && best >= 0.0 && (apiv <= DBL_MAX);
            pmax = fmax(pmax, apiv);
            pmin = fmin(pmin, apiv);
            const bool isp = (r == p);
            if (isp) {
                used = true;
                const double inv = 1.0 / piv;
#pragma unroll
                for (int q0 = 0; q0 < CPT; q0 += 4) {
#pragma unroll
                    for (int u = 0; u < 4 && q0 + u < CPT; ++u) prow[b][g * CPT + q0 + u] = a[q0 + u] * inv;
                    __builtin_amdgcn_sched_barrier(0);
                }
                if (g == gk) prow[b][g * CPT] = inv;
                if (g == 0) {
                    pk[k] = p;
                    kof[p] = k;
                }
            }
            __syncthreads();
            // every row: a_ik := 0, then a_i -= a_ik * row_p; the pivot row then takes row_p.
            // Staged entries are read 4 at a time: a fence per chunk keeps the scheduler from
            // hoisting every LDS read, each of which costs a register pair.
            const double f = colv[b][r];
            if (g == gk) a[0] = 0.0;
#pragma unroll
            for (int q0 = 0; q0 < CPT; q0 += 4) {
                double pv[4];
#pragma unroll
                for (int u = 0; u < 4 && q0 + u < CPT; ++u) pv[u] = prow[b][g * CPT + q0 + u];
#pragma unroll
                for (int u = 0; u < 4 && q0 + u < CPT; ++u) a[q0 + u] = fma(-f, pv[u], a[q0 + u]);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (isp) {
#pragma unroll
                for (int q = 0; q < CPT; ++q) a[q] = prow[b][g * CPT + q];
            }
        }
        const double a0 = a[0];
#pragma unroll
        for (int q = 0; q + 1 < CPT; ++q) a[q] = a[q + 1];
        a[CPT - 1] = a0;
    }
    __syncthreads();
    // slot q now holds the columns of original slot (q + nslot) mod CPT
    if (live) {
        double *dst = out + J.offD + min(max(kof[r], 0), n - 1);
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int j = G * ((q + nslot) % CPT) + g;
            if (j < n) dst[(int64_t)min(max(pk[j], 0), n - 1) * J.ldD] = a[q];
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if (t == 0) {
        const double tiny = 32.0 * (double)n * 2.220446049250313e-16 * pmax;
        info[blockIdx.x] = (finite && pmin > tiny) ? 0 : 1;
    }
}

int inv_gj_max_n() { return 208; }

int32_t inv_gj_batched(const CopyJob *d_jobs, int nbatch, int maxn, const double *in, double *out, int32_t *info,
                       hipStream_t s) {
    if (nbatch == 0 || maxn == 0) return HKG_OK;
    if (maxn <= 64)
        hipLaunchKernelGGL((k_inv_gj<16, 64>), dim3(nbatch), dim3(256), 0, s, d_jobs, in, out, info);
    else if (maxn <= 128)
        hipLaunchKernelGGL((k_inv_gj<32, 128>), dim3(nbatch), dim3(512), 0, s, d_jobs, in, out, info);
    else if (maxn <= 192)
        hipLaunchKernelGGL((k_inv_gj<48, 192>), dim3(nbatch), dim3(768), 0, s, d_jobs, in, out, info);
    else if (maxn <= 208)
        hipLaunchKernelGGL((k_inv_gj<52, 256>), dim3(nbatch), dim3(1024), 0, s, d_jobs, in, out, info);
    else
        return HKG_EINVAL;
    HKG_HIP(hipGetLastError());
    return HKG_OK;
}

}  // namespace hkg
