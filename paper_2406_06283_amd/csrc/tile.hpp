// GEMM tile shared by the batched dense kernels: C[tm*GT.., tn*GT..] = beta C + alpha op(A) op(B).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hkg {

constexpr int GT = 64;       // GEMM tile (GT x GT outputs per 256-thread block, 4 x 4 per thread)
constexpr int GK = 16;       // GEMM k-step staged through LDS

// ------------------------------------------------------------------------------------------------
// GEMM tile: C[tm*GT.., tn*GT..] = beta C + alpha op(A) op(B) with op(A) M x K, op(B) K x N.
// ------------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void gemm_tile(int M, int N, int K, const T *__restrict__ A, int lda, bool ta,
                                          const T *__restrict__ B, int ldb, bool tb, T *__restrict__ C,
                                          int ldc, T alpha, T beta, int tm, int tn) {
    __shared__ T sA[GK][GT + 1];
    __shared__ T sB[GK][GT + 1];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int i0 = tm * GT, j0 = tn * GT;
    T acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = T(0);

    // element e (< GK GT) of a k-step's A and B tiles: its LDS slot and its value; the next step's
    // values are loaded into registers while the current step is computed
    constexpr int PER = GK * GT / 256;
    auto a_slot = [&](int e, int &kk, int &ii) {
        if (!ta) {
            ii = e % GT;
            kk = e / GT;
        } else {
            kk = e % GK;
            ii = e / GK;
        }
    };
    auto b_slot = [&](int e, int &kk, int &jj) {
        if (!tb) {
            kk = e % GK;
            jj = e / GK;
        } else {
            jj = e % GT;
            kk = e / GT;
        }
    };
    auto a_val = [&](int k0, int e) -> T {
        int kk, ii;
        a_slot(e, kk, ii);
        const int gi = i0 + ii, gk = k0 + kk;
        return (gi < M && gk < K) ? (ta ? A[gk + (int64_t)gi * lda] : A[gi + (int64_t)gk * lda]) : T(0);
    };
    auto b_val = [&](int k0, int e) -> T {
        int kk, jj;
        b_slot(e, kk, jj);
        const int gj = j0 + jj, gk = k0 + kk;
        return (gj < N && gk < K) ? (tb ? B[gj + (int64_t)gk * ldb] : B[gk + (int64_t)gj * ldb]) : T(0);
    };
    T ra[PER], rb[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        ra[u] = a_val(0, tid + 256 * u);
        rb[u] = b_val(0, tid + 256 * u);
    }
#pragma clang loop unroll(disable)
    for (int k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            int kk, ii;
            a_slot(tid + 256 * u, kk, ii);
            sA[kk][ii] = ra[u];
            b_slot(tid + 256 * u, kk, ii);
            sB[kk][ii] = rb[u];
        }
        __syncthreads();
        if (k0 + GK < K) {
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                ra[u] = a_val(k0 + GK, tid + 256 * u);
                rb[u] = b_val(k0 + GK, tid + 256 * u);
            }
        }
#pragma unroll
        for (int kk = 0; kk < GK; ++kk) {
            T a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = sA[kk][tx + 16 * r];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = sB[kk][ty + 16 * c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = fma(a[r], b[c], acc[r][c]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        int gj = j0 + ty + 16 * c;
        if (gj >= N) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int gi = i0 + tx + 16 * r;
            if (gi >= M) continue;
            T *p = C + gi + (int64_t)gj * ldc;
            *p = (beta == T(0) ? T(0) : beta * *p) + alpha * acc[r][c];
        }
    }
}

// ------------------------------------------------------------------------------------------------
// The same product on 32 x 32 output tiles (2 x 2 per thread, k-steps of 32): four times the blocks
// of gemm_tile for batches of small matrices that would leave most CUs idle.  Every output is the
// same FMA chain over k in increasing order as in gemm_tile, so the two give identical bits.
// ------------------------------------------------------------------------------------------------
constexpr int GT2 = 32;
constexpr int GK2 = 32;

template <typename T>
__device__ __forceinline__ void gemm_tile32(int M, int N, int K, const T *__restrict__ A, int lda, bool ta,
                                            const T *__restrict__ B, int ldb, bool tb, T *__restrict__ C,
                                            int ldc, T alpha, T beta, int tm, int tn) {
    __shared__ T sA[GK2][GT2 + 1];
    __shared__ T sB[GK2][GT2 + 1];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int i0 = tm * GT2, j0 = tn * GT2;
    T acc[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[r][c] = T(0);
    constexpr int PER = GK2 * GT2 / 256;
    // element e of a k-step's tile: (kk, ii) with the contiguous direction of the source fastest
    auto a_slot = [&](int e, int &kk, int &ii) {
        if (!ta) {
            ii = e % GT2;
            kk = e / GT2;
        } else {
            kk = e % GK2;
            ii = e / GK2;
        }
    };
    auto b_slot = [&](int e, int &kk, int &jj) {
        if (!tb) {
            kk = e % GK2;
            jj = e / GK2;
        } else {
            jj = e % GT2;
            kk = e / GT2;
        }
    };
    // loads clamped into range and masked after, so none is guarded by a branch
    auto a_val = [&](int k0, int e) -> T {
        int kk, ii;
        a_slot(e, kk, ii);
        const int gi = i0 + ii, gk = k0 + kk;
        const int ci = min(gi, M - 1), ck = min(gk, K - 1);
        const T v = ta ? A[ck + (int64_t)ci * lda] : A[ci + (int64_t)ck * lda];
        return (gi < M && gk < K) ? v : T(0);
    };
    auto b_val = [&](int k0, int e) -> T {
        int kk, jj;
        b_slot(e, kk, jj);
        const int gj = j0 + jj, gk = k0 + kk;
        const int cj = min(gj, N - 1), ck = min(gk, K - 1);
        const T v = tb ? B[cj + (int64_t)ck * ldb] : B[ck + (int64_t)cj * ldb];
        return (gj < N && gk < K) ? v : T(0);
    };
    T ra[PER], rb[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        ra[u] = a_val(0, tid + 256 * u);
        rb[u] = b_val(0, tid + 256 * u);
    }
#pragma clang loop unroll(disable)
    for (int k0 = 0; k0 < K; k0 += GK2) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            int kk, ii;
            a_slot(tid + 256 * u, kk, ii);
            sA[kk][ii] = ra[u];
            b_slot(tid + 256 * u, kk, ii);
            sB[kk][ii] = rb[u];
        }
        __syncthreads();
        if (k0 + GK2 < K) {
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                ra[u] = a_val(k0 + GK2, tid + 256 * u);
                rb[u] = b_val(k0 + GK2, tid + 256 * u);
            }
        }
#pragma unroll
        for (int kk = 0; kk < GK2; ++kk) {
            const T a0 = sA[kk][tx], a1 = sA[kk][tx + 16];
            const T b0 = sB[kk][ty], b1 = sB[kk][ty + 16];
            acc[0][0] = fma(a0, b0, acc[0][0]);
            acc[1][0] = fma(a1, b0, acc[1][0]);
            acc[0][1] = fma(a0, b1, acc[0][1]);
            acc[1][1] = fma(a1, b1, acc[1][1]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int gj = j0 + ty + 16 * c;
        if (gj >= N) continue;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int gi = i0 + tx + 16 * r;
            if (gi >= M) continue;
            T *p = C + gi + (int64_t)gj * ldc;
            *p = (beta == T(0) ? T(0) : beta * *p) + alpha * acc[r][c];
        }
    }
}

}  // namespace hkg
