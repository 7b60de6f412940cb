// The context behind the opaque hkgeneo_ctx handle, and device-buffer helpers of the host driver.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"

struct hkgeneo_ctx {
    hkgeneo_options opt{};
    int n_dof = 0, nnz = 0, n_sub = 0, m0 = 0, max_nI = 0, max_nG = 0, max_m = 0, npe = 0, dim = 2;
    int64_t sum_nI = 0, nBIO = 0, nSq = 0, nGG = 0, nGI = 0, nPiv = 0, nM = 0;
    double k = 0.0;
    hkg::Partition P;
    hkg::CoarsePairs CP;
    std::vector<hkg::SubDev> subs;        // host copy of the per-subdomain descriptors
    std::vector<int32_t> m_host;
    std::vector<double> lam_host;         // n_sub x (max_eig_per_sub + 2)
    int64_t device_bytes = 0;
    int64_t peak_device_bytes = 0;       // high-water mark of device_bytes (setup workspace included)

    // resident inputs and static descriptors (analysis phase)
    hkg::DevBuf rowptr, colidx, Aval, Sval, I_idx, G_idx, winv, wloc, tp_ptr, tp_pos, tp_sub, subs_d;
    hkg::DevBuf bandK, bandM, bandLoc, pairs;
    hkg::DevBuf matsGG, matsSq, poffSub, jobsGI, jobsSq, jobsSqM, gjobsSchur, matsLoc, poffLoc, jobsLoc, matsM, jobsM;
    // numeric results (factorisation phase)
    hkg::DevBuf Bval, Minv, Z, Zr, B0inv;
    hkg::DevBuf tpZ;                      // per transpose-map position: its row of Z_i and slice of y
    hkg::DevBuf B0copy;                   // B_0 kept on the device for queries when m0 <= 2048
    int b0_band = -1;                     // half-bandwidth of B_0 used by its LU (-1: dense)
    int band_I = -1;                      // half-bandwidth of B[I, I] and C_II (-1: treated as dense)
    // factorisation workspace (kept between calls when opt.keep_workspace, freed otherwise)
    hkg::DevBuf wGGi, wGI2, jobsGGinv, gjobsGX;   // Gamma block inverse, gathered rows, their job lists
    hkg::DevBuf wDk, wBIO, wCII, wGG, wGI, wS, wW, wPiv, wInfo, wFlag, wD, wE, wTau, wM, wLam, wY, wB0, wLU, wPivL,
        wJobsZ, wGjobsY, wMisc, wPiv0, wInv, wVWV, wInfoL, wSL, wIv, wLinv, wJobsInv, wT, wPivC, wInfoC, wFlagSpd,
        wDC, wDCjobs, wDCpiv, wDCinfo, wAIO;
    // the local-inverse pipeline of the factorisation runs on a second stream beside the coarse-space
    // pipeline; its pivot flags come back through pinned host memory
    hipStream_t s2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // a third stream factors C_II while the Gamma block and the Schur complement are formed
    hipStream_t s3 = nullptr;
    hipEvent_t ev_fork3 = nullptr, ev_join3 = nullptr;
    // the divide-and-conquer inverse of B_0 runs part of each merge level on s3
    hipEvent_t ev_dc[4] = {nullptr, nullptr, nullptr, nullptr};
    int32_t *h_infoL = nullptr;
    int h_infoL_n = 0;
    // pinned staging for the job lists uploaded during a factorisation (reset at its start, after
    // the previous factorisation's final wait), so that those uploads need no wait
    uint8_t *h_stage = nullptr;
    size_t h_stage_cap = 0, h_stage_used = 0;
    // pinned readback of the eigenvalue counts, eigenvalues and flags of the coarse space
    uint8_t *h_read = nullptr;
    size_t h_read_cap = 0;
    // apply workspace
    hkg::DevBuf u, c, y, ypart;
    int ws_nrhs = 0;
    // gmres workspace
    hkg::DevBuf V, Zk, H, cs, sn, g, part, hcol, scal, active, want, rnorm, npart, fnorm, itersd;
    hkg::DevBuf DV;                       // D_k V of the D_k-inner-product variant
    int gm_nrhs = 0;
    // measurement hook: events around the local-solve kernel
    bool prof = false;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    hkgeneo_stats stats{};
    // nested decomposition (Sec. 2.3): this context holds the coarse subdomains and the coarse space
    // only (coarse_only: no local inverses), `fine` the first-level subdomains and their local
    // inverses (a one-level context), fine_owner the coarse subdomain of each
    hkgeneo_ctx *fine = nullptr;
    bool coarse_only = false;
    std::vector<int32_t> fine_owner;
};

namespace hkg {

int32_t dalloc(hkgeneo_ctx *c, DevBuf *b, size_t bytes);           // fresh allocation
int32_t walloc(hkgeneo_ctx *c, DevBuf *b, size_t bytes);           // reuse if large enough
void drelease(hkgeneo_ctx *c, DevBuf *b);
int32_t upload_bytes(hkgeneo_ctx *c, DevBuf *b, const void *host, size_t bytes, hipStream_t s, bool reuse);
// the same through the pinned staging area of the context: returns without waiting for the copy
int32_t upload_staged(hkgeneo_ctx *c, DevBuf *b, const void *host, size_t bytes, hipStream_t s);

template <typename T>
int32_t upload(hkgeneo_ctx *c, DevBuf *b, const T *host, size_t count, hipStream_t s, bool reuse = false) {
    return upload_bytes(c, b, host, count * sizeof(T), s, reuse);
}

template <typename T>
T *dp(const DevBuf &b) {
    return reinterpret_cast<T *>(b.p);
}

int32_t analyze(hkgeneo_ctx *c, const hkgeneo_problem *p, hipStream_t s, int32_t *bad,
                const std::vector<std::vector<int32_t>> *sets = nullptr);
int32_t factor(hkgeneo_ctx *c, hipStream_t s);
// B_0^{-1} into c->B0inv from the assembled c->wB0 by divide and conquer over its level blocks;
// *done = false when the structure does not allow it or a block needs pivoting across blocks
int32_t coarse_inverse_dc(hkgeneo_ctx *c, hipStream_t s, bool *done);
void free_workspace(hkgeneo_ctx *c);

}  // namespace hkg
