// Internal declarations shared by the host driver and the HIP kernels of libhkgeneo.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hkgeneo.h"

namespace hkg {

#define HKG_HIP(call)                                                             \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            hkg::set_last_error(std::string(#call) + ": " + hipGetErrorString(e_)); \
            return HKG_EHIP;                                                      \
        }                                                                         \
    } while (0)

#define HKG_TRY(call)                 \
    do {                                  \
        int32_t s_ = (call);              \
        if (s_ != HKG_OK) return s_;      \
    } while (0)

void set_last_error(const std::string &msg);
extern thread_local std::string g_last_error;

// FGMRES stopping rule, shared by the host loop and the device kernels of both solve paths: a
// right-hand side keeps iterating while its residual norm is finite and above rtol ||f||.  A NaN or
// infinite residual (or ||f||) stops it; the result then reports non-convergence.
__host__ __device__ inline bool gmres_keeps_going(double rn, double fn, double rtol) {
    return rn > rtol * fn && rn <= 1.7976931348623157e308;   // comparisons with NaN are false
}
// ||f - B x|| / ||f||: 0 for a zero right-hand side, NaN when ||f|| is not finite
__host__ __device__ inline double gmres_relres(double rn, double fn) {
    if (fn == 0.0) return 0.0;
    return (fn > 0.0 && fn <= 1.7976931348623157e308) ? rn / fn : __builtin_nan("");
}

// ------------------------------------------------------------------------------------------------
// Host partitioner output (Def. 2.8, Def. 2.12, Def. 2.13, Lambda of Sec. 2.4)
// ------------------------------------------------------------------------------------------------
struct Partition {
    int n_sub = 0, n_dof = 0, npe = 0, lambda_overlap = 0;
    std::vector<int32_t> nI, nG;           // per subdomain: |dof(D)|, |ovdof(D) \ dof(D)|
    std::vector<int64_t> offI, offG;       // prefix sums (n_sub + 1)
    std::vector<int32_t> I_idx, G_idx;     // concatenated ascending global dof ids
    std::vector<int32_t> mu;               // multiplicity per dof
    // transpose map: for dof l, the positions offI[s] + a of l in every subdomain s with l internal
    std::vector<int32_t> tp_ptr, tp_pos;
    // elements of D carrying at least one Gamma dof, with the Gamma-local index of each vertex
    std::vector<int32_t> band_ptr, band_elem, band_loc;   // band_loc: npe entries per band element
    std::vector<int32_t> el_ptr, el_list;  // the (overlapping) element set of each subdomain, ascending
};

// sets == nullptr: subdomains from p->elem_part expanded by p->overlap layers (Def. 2.8); otherwise
// the given element sets as they are
int32_t build_partition(const hkgeneo_problem *p, Partition *out, int *bad_sub,
                        const std::vector<std::vector<int32_t>> *sets = nullptr);
// element sets of the first-level subdomains of the nested decomposition (Sec. 2.3) inside the
// coarse subdomains of Pc, and the coarse subdomain owning each
int32_t build_nested_sets(const hkgeneo_problem *p, const Partition &Pc, int layers,
                          std::vector<std::vector<int32_t>> *sets, std::vector<int32_t> *owner);

// Pairs (i, j) with ovdof(D_i) and dof(D_j) intersecting: the nonzero blocks of B_0 = Z^T B Z.
struct CoarsePairs {
    std::vector<int32_t> pi, pj;            // pair list
    std::vector<int32_t> ptr;               // entries of pair t: [ptr[t], ptr[t+1])
    std::vector<int32_t> qi, qj;            // position in ovdof(D_i) = [dof | Gamma], position in dof(D_j)
};
void build_coarse_pairs(const Partition &P, CoarsePairs *out);

// ------------------------------------------------------------------------------------------------
// Device buffers
// ------------------------------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// batched dense matrix descriptor (column-major, square n x n, leading dimension ld)
struct DMat {
    int64_t off;
    int32_t n;
    int32_t ld;
};

// triangular-solve job: triangle T (n x n at offT, ldT) and right-hand sides X (n x ncol at offX, ldX);
// offO, ldO: where a solve that reads its right-hand sides transposed writes its result
struct TriJob {
    int64_t offT;
    int64_t offX;
    int32_t n;
    int32_t ldT;
    int32_t ncol;
    int32_t ldX;
    int64_t offO = 0;
    int32_t ldO = 0;
    int32_t pad_ = 0;
};

// rectangular block copy: dst (rows x cols at offD, ldD) = src (rows x cols at offS, ldS)
struct CopyJob {
    int64_t offS, offD;
    int32_t rows, cols, ldS, ldD;
};

// general GEMM job: C (M x N) = beta C + alpha op(A) op(B)
struct GemmJob {
    int64_t offA, offB, offC;
    int32_t M, N, K;
    int32_t lda, ldb, ldc;
};

}  // namespace hkg

// the opaque context
struct hkgeneo_ctx;
