// Host driver of the setup: analysis (host partition and resident inputs) and factorisation (every
// numeric step, on the device, from the resident inputs).
//
// Factorisation, per subdomain D_i (batched over subdomains with uneven sizes):
//   B = A - k^2 S, D_k = A + k^2 S on the CSR pattern                               (Sec. 2.1)
//   [B_II | B_IG] and C_II = X D_k[I,I] X from the CSR rows of dof(D_i)        (eq. 2.22, Def. 2.14)
//   B~_GG from the elements of D_i carrying Gamma dofs                               (eq. 2.18)
//   S = B_II - B_IG B~_GG^{-1} B_GI,  C_II = L U (no exchanges),  S^ = L^-1 S L^-T    (Lemma 2.6)
//   tridiagonalise S^, select m_i (Def. 2.15), eigenvectors, back-transform, Z_i = X_I P_i
//   B_0 = Z^T B Z over neighbouring pairs, B_0 = P L U, B_0^{-1}                     (eq. 2.23)
//   B_D = P L U and B_D^{-1} in float64 or float32                                     (eq. 2.22)
#include <algorithm>
#include <array>
#include <string>
#include <thread>
#include <cstring>
#include <functional>

#include "ctx.hpp"

namespace hkg {

int32_t dalloc(hkgeneo_ctx *c, DevBuf *b, size_t bytes) {
    drelease(c, b);
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(&b->p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b->p = nullptr;
        set_last_error("hipMalloc of " + std::to_string(bytes) + " bytes failed");
        return HKG_ENOMEM;
    }
    b->bytes = bytes;
    c->device_bytes += (int64_t)bytes;
    c->peak_device_bytes = std::max(c->peak_device_bytes, c->device_bytes);
    return HKG_OK;
}

int32_t walloc(hkgeneo_ctx *c, DevBuf *b, size_t bytes) {
    if (b->p && b->bytes >= bytes && bytes > 0) return HKG_OK;
    return dalloc(c, b, bytes);
}

void drelease(hkgeneo_ctx *c, DevBuf *b) {
    if (b->p) {
        (void)hipFree(b->p);
        c->device_bytes -= (int64_t)b->bytes;
    }
    b->p = nullptr;
    b->bytes = 0;
}

// host -> device copy that has completed when it returns (the host source may be a temporary)
int32_t upload_bytes(hkgeneo_ctx *c, DevBuf *b, const void *host, size_t bytes, hipStream_t s, bool reuse) {
    HKG_TRY(reuse ? walloc(c, b, bytes) : dalloc(c, b, bytes));
    if (bytes) {
        HKG_HIP(hipMemcpyAsync(b->p, host, bytes, hipMemcpyHostToDevice, s));
        HKG_HIP(hipStreamSynchronize(s));
    }
    return HKG_OK;
}

int32_t upload_staged(hkgeneo_ctx *c, DevBuf *b, const void *host, size_t bytes, hipStream_t s) {
    HKG_TRY(walloc(c, b, bytes));
    if (!bytes) return HKG_OK;
    const size_t at = (c->h_stage_used + 255) / 256 * 256;
    if (at + bytes > c->h_stage_cap) {
        // a larger area: the copies from the old one finish first
        HKG_HIP(hipStreamSynchronize(s));
        if (c->h_stage) HKG_HIP(hipHostFree(c->h_stage));
        c->h_stage = nullptr;
        c->h_stage_cap = 0;
        c->h_stage_used = 0;
        const size_t cap = std::max<size_t>((size_t)1 << 20, 2 * bytes);
        HKG_HIP(hipHostMalloc((void **)&c->h_stage, cap));
        c->h_stage_cap = cap;
        return upload_staged(c, b, host, bytes, s);
    }
    std::memcpy(c->h_stage + at, host, bytes);
    HKG_HIP(hipMemcpyAsync(b->p, c->h_stage + at, bytes, hipMemcpyHostToDevice, s));
    c->h_stage_used = at + bytes;
    return HKG_OK;
}

void free_workspace(hkgeneo_ctx *c) {
    DevBuf *w[] = {&c->wGGi, &c->wGI2, &c->wDk, &c->wBIO, &c->wCII, &c->wGG, &c->wGI, &c->wS, &c->wW, &c->wPiv, &c->wInfo,
                   &c->wFlag, &c->wD, &c->wE, &c->wTau, &c->wM, &c->wLam, &c->wY, &c->wB0, &c->wLU,
                   &c->wPivL, &c->wJobsZ, &c->wGjobsY, &c->wMisc, &c->wPiv0, &c->wInv, &c->wVWV, &c->wInfoL, &c->wSL, &c->wIv,
                   &c->wLinv, &c->wJobsInv, &c->wT, &c->wPivC, &c->wInfoC, &c->wFlagSpd, &c->wDC, &c->wDCjobs,
                   &c->wDCpiv, &c->wDCinfo, &c->wAIO};
    for (DevBuf *b : w) drelease(c, b);
}

// ------------------------------------------------------------------------------------------------
// analysis: partition, layout, resident inputs, descriptors that depend on the partition only
// ------------------------------------------------------------------------------------------------
int32_t analyze(hkgeneo_ctx *c, const hkgeneo_problem *p, hipStream_t s, int32_t *bad,
                const std::vector<std::vector<int32_t>> *sets) {
    HKG_TRY(build_partition(p, &c->P, bad, sets));
    c->n_sub = c->P.n_sub;
    c->npe = c->P.npe;
    const Partition &P = c->P;
    const int ns = c->n_sub;
    c->subs.resize(ns);
    int64_t oBIO = 0, oSq = 0, oGG = 0, oGI = 0, oPiv = 0, oM = 0;
    for (int i = 0; i < ns; ++i) {
        SubDev &sd = c->subs[i];
        sd = SubDev{};
        sd.nI = P.nI[i];
        sd.nG = P.nG[i];
        sd.offI = P.offI[i];
        sd.offG = P.offG[i];
        sd.offBIO = oBIO;
        sd.offSq = oSq;
        sd.offGG = oGG;
        sd.offGI = oGI;
        sd.offPiv = oPiv;
        sd.ldM = (sd.nI + 31) / 32 * 32;
        sd.offM = oM;
        sd.bandBeg = P.band_ptr[i];
        sd.bandEnd = P.band_ptr[i + 1];
        oBIO += (int64_t)sd.nI * (sd.nI + sd.nG);
        oSq += (int64_t)sd.nI * sd.nI;
        oM += (int64_t)sd.ldM * sd.nI;
        oGG += (int64_t)sd.nG * sd.nG;
        oGI += (int64_t)sd.nG * sd.nI;
        oPiv += std::max(sd.nI, sd.nG);
        c->max_nI = std::max(c->max_nI, sd.nI);
        c->max_nG = std::max(c->max_nG, sd.nG);
    }
    c->nBIO = oBIO;
    c->nSq = oSq;
    c->nM = oM;
    c->nGG = oGG;
    c->nGI = oGI;
    c->nPiv = oPiv;
    c->sum_nI = P.offI[ns];
    // 1/mu from the multiplicities; local prolongation weights (1, or 1/mu for the weighted variant)
    std::vector<double> winv(c->n_dof), wloc(c->sum_nI);
    for (int d = 0; d < c->n_dof; ++d) winv[d] = 1.0 / (double)P.mu[d];
    for (int64_t t = 0; t < c->sum_nI; ++t) wloc[t] = (c->opt.prolong == HKG_PROLONG_POU) ? winv[P.I_idx[t]] : 1.0;
    // half-bandwidth of the local matrices B[I, I] and C_II in the ascending dof order of each
    // subdomain (the same sparsity as the global operator): their LUs and triangular solves
    // touch only that band (and the fill of row exchanges)
    {
        std::vector<int32_t> loc(c->n_dof, -1);
        int band = 0;
        for (int i = 0; i < ns; ++i) {
            for (int64_t t = P.offI[i]; t < P.offI[i + 1]; ++t) loc[P.I_idx[t]] = (int32_t)(t - P.offI[i]);
            for (int64_t t = P.offI[i]; t < P.offI[i + 1]; ++t) {
                const int g = P.I_idx[t], lg = (int)(t - P.offI[i]);
                for (int32_t q = p->row_ptr[g]; q < p->row_ptr[g + 1]; ++q) {
                    const int h = loc[p->col_idx[q]];
                    if (h >= 0) band = std::max(band, std::abs(h - lg));
                }
            }
            for (int64_t t = P.offI[i]; t < P.offI[i + 1]; ++t) loc[P.I_idx[t]] = -1;
        }
        c->band_I = (3 * band + LU_BLOCK < c->max_nI) ? band : -1;
    }
    HKG_TRY(upload(c, &c->rowptr, p->row_ptr, c->n_dof + 1, s));
    HKG_TRY(upload(c, &c->colidx, p->col_idx, c->nnz, s));
    HKG_TRY(upload(c, &c->Aval, p->A_val, c->nnz, s));
    HKG_TRY(upload(c, &c->Sval, p->S_val, c->nnz, s));
    HKG_TRY(upload(c, &c->I_idx, P.I_idx.data(), P.I_idx.size(), s));
    if (P.G_idx.empty()) HKG_TRY(dalloc(c, &c->G_idx, sizeof(int32_t)));
    else HKG_TRY(upload(c, &c->G_idx, P.G_idx.data(), P.G_idx.size(), s));
    HKG_TRY(upload(c, &c->winv, winv.data(), winv.size(), s));
    HKG_TRY(upload(c, &c->wloc, wloc.data(), wloc.size(), s));
    HKG_TRY(upload(c, &c->tp_ptr, P.tp_ptr.data(), P.tp_ptr.size(), s));
    HKG_TRY(upload(c, &c->tp_pos, P.tp_pos.data(), P.tp_pos.size(), s));
    {
        std::vector<int32_t> owner(c->sum_nI), tsub(P.tp_pos.size());
        for (int i = 0; i < ns; ++i)
            for (int64_t t = P.offI[i]; t < P.offI[i + 1]; ++t) owner[t] = i;
        for (size_t t = 0; t < P.tp_pos.size(); ++t) tsub[t] = owner[P.tp_pos[t]];
        HKG_TRY(upload(c, &c->tp_sub, tsub.data(), tsub.size(), s));
    }
    HKG_TRY(upload(c, &c->subs_d, c->subs.data(), ns, s));

    // element matrices of the band elements (the elements of each D_i carrying Gamma dofs)
    const int npe2 = c->npe * c->npe;
    const size_t nb = P.band_elem.size();
    {
        std::vector<double> hk(std::max<size_t>(nb * npe2, 1)), hm(std::max<size_t>(nb * npe2, 1));
        for (size_t b = 0; b < nb; ++b) {
            std::memcpy(&hk[b * npe2], p->elem_K + (size_t)P.band_elem[b] * npe2, npe2 * sizeof(double));
            std::memcpy(&hm[b * npe2], p->elem_M + (size_t)P.band_elem[b] * npe2, npe2 * sizeof(double));
        }
        HKG_TRY(upload(c, &c->bandK, hk.data(), hk.size(), s));
        HKG_TRY(upload(c, &c->bandM, hm.data(), hm.size(), s));
        std::vector<int32_t> bl(P.band_loc);
        if (bl.empty()) bl.push_back(-1);
        HKG_TRY(upload(c, &c->bandLoc, bl.data(), bl.size(), s));
    }

    // descriptors for the batched dense kernels
    std::vector<DMat> hGG(ns), hSq(ns);
    std::vector<int64_t> hpo(ns), hpl(ns);
    std::vector<TriJob> jGI(ns), jSq(ns), jSqM(ns), jM(ns);
    std::vector<DMat> hM(ns);
    std::vector<GemmJob> gS(ns), gX(ns);
    std::vector<CopyJob> jGinv(ns);
    int64_t pl = 0;
    for (int i = 0; i < ns; ++i) {
        const SubDev &sd = c->subs[i];
        const int ldG = std::max(sd.nG, 1);
        hGG[i] = {sd.offGG, sd.nG, ldG};
        hSq[i] = {sd.offSq, sd.nI, sd.nI};
        hpo[i] = sd.offPiv;
        hpl[i] = pl;
        pl += sd.nI;
        jGI[i] = {sd.offGG, sd.offGI, sd.nG, ldG, sd.nI, ldG};
        jSq[i] = {sd.offSq, sd.offSq, sd.nI, sd.nI, sd.nI, sd.nI, sd.offM, sd.ldM};
        jSqM[i] = {sd.offSq, sd.offM, sd.nI, sd.nI, sd.nI, sd.ldM, sd.offM, sd.ldM};
        hM[i] = {sd.offM, sd.nI, sd.ldM};
        jM[i] = {sd.offSq, sd.offM, sd.nI, sd.nI, sd.nI, sd.ldM};
        gS[i] = {sd.offBIO + (int64_t)sd.nI * sd.nI, sd.offGI, sd.offSq, sd.nI, sd.nI, sd.nG, sd.nI, ldG, sd.nI};
        jGinv[i] = {sd.offGG, sd.offGG, sd.nG, sd.nG, ldG, ldG};
        gX[i] = {sd.offGG, sd.offGI, sd.offGI, sd.nG, sd.nI, sd.nG, ldG, ldG, ldG};
    }
    HKG_TRY(upload(c, &c->matsGG, hGG.data(), ns, s));
    HKG_TRY(upload(c, &c->matsSq, hSq.data(), ns, s));
    HKG_TRY(upload(c, &c->poffSub, hpo.data(), ns, s));
    HKG_TRY(upload(c, &c->poffLoc, hpl.data(), ns, s));
    HKG_TRY(upload(c, &c->jobsGI, jGI.data(), ns, s));
    HKG_TRY(upload(c, &c->jobsSq, jSq.data(), ns, s));
    HKG_TRY(upload(c, &c->jobsSqM, jSqM.data(), ns, s));
    HKG_TRY(upload(c, &c->matsM, hM.data(), ns, s));
    HKG_TRY(upload(c, &c->jobsM, jM.data(), ns, s));
    HKG_TRY(upload(c, &c->gjobsSchur, gS.data(), ns, s));
    HKG_TRY(upload(c, &c->jobsGGinv, jGinv.data(), ns, s));
    HKG_TRY(upload(c, &c->gjobsGX, gX.data(), ns, s));

    // neighbouring pairs of the coarse matrix
    build_coarse_pairs(P, &c->CP);
    {
        const CoarsePairs &CP = c->CP;
        std::vector<int32_t> packed;
        packed.insert(packed.end(), CP.pi.begin(), CP.pi.end());
        packed.insert(packed.end(), CP.pj.begin(), CP.pj.end());
        packed.insert(packed.end(), CP.ptr.begin(), CP.ptr.end());
        packed.insert(packed.end(), CP.qi.begin(), CP.qi.end());
        packed.insert(packed.end(), CP.qj.begin(), CP.qj.end());
        HKG_TRY(upload(c, &c->pairs, packed.data(), packed.size(), s));
    }
    return HKG_OK;
}

// ------------------------------------------------------------------------------------------------
// factorisation
// ------------------------------------------------------------------------------------------------
namespace {

int32_t read_flags(hkgeneo_ctx *c, const DevBuf &buf, int n, std::vector<int32_t> *out, hipStream_t s) {
    out->assign(n, 0);
    HKG_HIP(hipMemcpyAsync(out->data(), buf.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipStreamSynchronize(s));
    (void)c;
    return HKG_OK;
}

// B_D = P L U and B_D^{-1} = U^{-1} L^{-1} P in float64 into `out` (the padded layout offM / ldM, nM
// entries).  Launches only (buffers come from local_buffers): the pivot flags are copied to
// c->h_infoL and checked by the caller.
int32_t local_inverses(hkgeneo_ctx *c, double *out, hipStream_t s) {
    const int ns = c->n_sub;
    const SubDev *dsub = dp<SubDev>(c->subs_d);
    HKG_TRY(copy_bii(dsub, ns, c->max_nI, dp<double>(c->wBIO), dp<double>(c->wLU), s));
    HKG_TRY(lu_batched<double>(dp<DMat>(c->matsSq), dp<int64_t>(c->poffLoc), ns, c->max_nI, dp<double>(c->wLU),
                               dp<int32_t>(c->wPivL), dp<int32_t>(c->wInfoL), true, s, c->band_I));
    HKG_HIP(hipMemcpyAsync(c->h_infoL, c->wInfoL.p, ns * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HKG_TRY(perm_identity_batched<double>(dp<DMat>(c->matsM), dp<int64_t>(c->poffLoc), ns, c->max_nI,
                                          dp<int32_t>(c->wPivL), out, s));
    HKG_TRY(tri_solve_batched<double>(dp<TriJob>(c->jobsM), ns, c->max_nI, c->max_nI, dp<double>(c->wLU), out,
                                      TRI_LOWER_UNIT, s));
    // U of a banded LU with row exchanges has half-bandwidth 2 band (L, with the exchanges applied to
    // its earlier columns, is not banded)
    HKG_TRY(tri_solve_batched<double>(dp<TriJob>(c->jobsM), ns, c->max_nI, c->max_nI, dp<double>(c->wLU), out,
                                      TRI_UPPER, s, c->band_I >= 0 ? 2 * c->band_I : -1));
    return HKG_OK;
}

// every buffer of the local-inverse pipeline, allocated by the calling thread
int32_t local_buffers(hkgeneo_ctx *c) {
    const bool store32 = c->opt.local_prec == 32;
    const size_t bytes = (size_t)c->nM * (store32 ? sizeof(float) : sizeof(double));
    if (c->Minv.bytes != bytes) HKG_TRY(dalloc(c, &c->Minv, bytes));
    HKG_TRY(walloc(c, &c->wLU, c->nSq * sizeof(double)));
    HKG_TRY(walloc(c, &c->wPivL, c->sum_nI * sizeof(int32_t)));
    HKG_TRY(walloc(c, &c->wInfoL, c->n_sub * sizeof(int32_t)));
    if (store32) HKG_TRY(walloc(c, &c->wSL, c->nM * sizeof(double)));
    return HKG_OK;
}

// the resident local operators in the storage precision of opt.local_prec: B_D = P L U and
// B_D^{-1} in float64, rounded once to float32 storage for local_prec 32
int32_t local_operators(hkgeneo_ctx *c, hipStream_t s) {
    const bool store32 = c->opt.local_prec == 32;
    if (!store32) return local_inverses(c, dp<double>(c->Minv), s);
    HKG_TRY(local_inverses(c, dp<double>(c->wSL), s));
    return cast_f64_f32(dp<double>(c->wSL), dp<float>(c->Minv), c->nM, s);
}

// A^{-1} = U^{-1} L^{-1} P for one packed n x n LU (ld = n): the diagonal blocks of L^{-1} and
// U^{-1} first, then level by level the off-diagonal block of each pair of neighbouring blocks
// (L: X21 = -X22 L21 X11;  U: X12 = -X11 U12 X22) by batched GEMMs, then L^{-1} P by a column
// gather and the product with U^{-1}.  About 4 log2(n / 32) + 4 launches.
int32_t lu_inverse(hkgeneo_ctx *c, int n, const double *LU, const int32_t *piv, double *out, int uband, hipStream_t s) {
    const size_t nn = (size_t)n * n;
    HKG_TRY(walloc(c, &c->wLinv, 3 * nn * sizeof(double)));
    double *Linv = dp<double>(c->wLinv), *Uinv = Linv + nn, *tmp = Uinv + nn;
    if (lu_inverse_cols_lds(n) <= (int64_t)144 * 1024) {
        // independent column solves with the inverted diagonal blocks: one launch after the blocks
        HKG_TRY(tri_diag_inverse(LU, n, n, Linv, Uinv, n, s));
        return lu_inverse_cols(LU, n, n, piv, Linv, Uinv, n, out, n, uband, s);
    }
    HKG_HIP(hipMemsetAsync(Linv, 0, 2 * nn * sizeof(double), s));
    HKG_TRY(tri_diag_inverse(LU, n, n, Linv, Uinv, n, s));
    // jobs of every level: [L first product | L second | U first | U second] per level
    struct Level {
        int first, count, maxM, maxN;
    };
    std::vector<GemmJob> jobs;
    std::vector<std::array<Level, 4>> levels;
    const int nblk = (n + LU_BLOCK - 1) / LU_BLOCK;
    for (int half = LU_BLOCK; half < n && (nblk > 1); half *= 2) {
        std::array<Level, 4> lv{};
        std::array<std::vector<GemmJob>, 4> js;
        for (int r0 = 0; r0 + half < n; r0 += 2 * half) {
            const int r1 = r0 + half, r2 = std::min(r0 + 2 * half, n);
            const int a = r1 - r0, b = r2 - r1;
            // L: T = L21 X11 (b x a), X21 = -X22 T
            js[0].push_back({r1 + (int64_t)r0 * n, r0 + (int64_t)r0 * n, r1 + (int64_t)r0 * n, b, a, a, n, n, n});
            js[1].push_back({r1 + (int64_t)r1 * n, r1 + (int64_t)r0 * n, r1 + (int64_t)r0 * n, b, a, b, n, n, n});
            // U: T = U12 Y22 (a x b), Y12 = -Y11 T
            js[2].push_back({r0 + (int64_t)r1 * n, r1 + (int64_t)r1 * n, r0 + (int64_t)r1 * n, a, b, b, n, n, n});
            js[3].push_back({r0 + (int64_t)r0 * n, r0 + (int64_t)r1 * n, r0 + (int64_t)r1 * n, a, b, a, n, n, n});
        }
        for (int q = 0; q < 4; ++q) {
            lv[q].first = (int)jobs.size();
            lv[q].count = (int)js[q].size();
            lv[q].maxM = 0;
            lv[q].maxN = 0;
            for (auto &j : js[q]) {
                lv[q].maxM = std::max(lv[q].maxM, (int)j.M);
                lv[q].maxN = std::max(lv[q].maxN, (int)j.N);
            }
            jobs.insert(jobs.end(), js[q].begin(), js[q].end());
        }
        levels.push_back(lv);
    }
    jobs.push_back({0, 0, 0, n, n, n, n, n, n});      // out = Uinv (L^{-1} P)
    HKG_TRY(upload(c, &c->wJobsInv, jobs.data(), jobs.size(), s, true));
    const GemmJob *dj = dp<GemmJob>(c->wJobsInv);
    for (auto &lv : levels) {
        HKG_TRY(gemm_batched<double>(dj + lv[0].first, lv[0].count, lv[0].maxM, lv[0].maxN, LU, Linv, tmp, 1.0, 0.0,
                                     false, false, s));
        HKG_TRY(gemm_batched<double>(dj + lv[1].first, lv[1].count, lv[1].maxM, lv[1].maxN, Linv, tmp, Linv, -1.0,
                                     0.0, false, false, s));
        HKG_TRY(gemm_batched<double>(dj + lv[2].first, lv[2].count, lv[2].maxM, lv[2].maxN, LU, Uinv, tmp, 1.0, 0.0,
                                     false, false, s));
        HKG_TRY(gemm_batched<double>(dj + lv[3].first, lv[3].count, lv[3].maxM, lv[3].maxN, Uinv, tmp, Uinv, -1.0,
                                     0.0, false, false, s));
    }
    HKG_TRY(gather_pivot_columns(n, Linv, n, piv, tmp, n, s));
    return gemm_batched<double>(dj + (jobs.size() - 1), 1, n, n, Uinv, tmp, out, 1.0, 0.0, false, false, s);
}

// start_side: forks the local-inverse pipeline to the second stream; called once the coarse blocks
// are enqueued, so that it fills the CUs the factorisation of B_0 leaves idle
int32_t coarse_space(hkgeneo_ctx *c, hipStream_t s, const std::function<int32_t()> &start_side) {
    const int ns = c->n_sub;
    const hkgeneo_options &o = c->opt;
    const int mmax = o.max_eig_per_sub;
    const SubDev *dsub = dp<SubDev>(c->subs_d);
    const bool delta = o.coarse_op == HKG_COARSE_DELTA;
    const double k2 = delta ? 0.0 : c->k * c->k;          // wavenumber of the local eigenproblem
    double *eigIO = delta ? dp<double>(c->wAIO) : dp<double>(c->wBIO);   // its [.._II | .._IG] blocks
    HKG_TRY(walloc(c, &c->wGG, std::max<int64_t>(c->nGG, 1) * sizeof(double)));
    HKG_TRY(walloc(c, &c->wGI, std::max<int64_t>(c->nGI, 1) * sizeof(double)));
    HKG_TRY(walloc(c, &c->wS, c->nSq * sizeof(double)));
    HKG_TRY(walloc(c, &c->wW, (size_t)std::max(c->nSq, c->nM) * sizeof(double)));
    HKG_TRY(walloc(c, &c->wPiv, c->nPiv * sizeof(int32_t)));
    HKG_TRY(walloc(c, &c->wInfo, ns * sizeof(int32_t)));
    HKG_TRY(walloc(c, &c->wFlag, ns * sizeof(int32_t)));
    HKG_TRY(walloc(c, &c->wPivC, c->nPiv * sizeof(int32_t)));
    HKG_TRY(walloc(c, &c->wInfoC, ns * sizeof(int32_t)));
    HKG_TRY(walloc(c, &c->wFlagSpd, ns * sizeof(int32_t)));
    // C_II = L U without exchanges (= L D L^T; positive pivots <=> SPD) on the third stream, concurrently with
    // the Gamma block's LU and the Schur complement; the flags are read back after the selection
    HKG_HIP(hipEventRecord(c->ev_fork3, s));
    HKG_HIP(hipStreamWaitEvent(c->s3, c->ev_fork3, 0));
    int32_t st_cii = HKG_OK;
    std::string err_cii;
    auto enqueue_cii = [&]() {
        if (ldl_band_fits(c->max_nI, c->band_I))
            st_cii = ldl_band(dsub, ns, c->max_nI, dp<double>(c->wCII), c->band_I, c->s3);
        else
            st_cii = lu_batched<double>(dp<DMat>(c->matsSq), dp<int64_t>(c->poffSub), ns, c->max_nI,
                                        dp<double>(c->wCII), dp<int32_t>(c->wPivC), dp<int32_t>(c->wInfoC), false,
                                        c->s3, c->band_I);
        if (st_cii == HKG_OK) st_cii = check_spd_pivots(dsub, ns, dp<double>(c->wCII), dp<int32_t>(c->wFlagSpd), c->s3);
        if (st_cii == HKG_OK && hipEventRecord(c->ev_join3, c->s3) != hipSuccess) {
            set_last_error("recording the end of the C_II factorisation");
            st_cii = HKG_EHIP;
        }
        if (st_cii != HKG_OK) err_cii = g_last_error;
    };
    // the one-launch L D L^T is enqueued here; the panel-chain LU (a hundred launches) by a helper
    std::thread enq_cii;
    if (ldl_band_fits(c->max_nI, c->band_I))
        enqueue_cii();
    else
        enq_cii = std::thread(enqueue_cii);
    // joined (and its status checked) before anything waits on its event
    struct Joiner {
        std::thread &t;
        ~Joiner() {
            if (t.joinable()) t.join();
        }
    } join_cii{enq_cii};
    // B~_GG and its LU
    HKG_HIP(hipMemsetAsync(c->wGG.p, 0, c->wGG.bytes, s));
    HKG_TRY(assemble_gamma(dsub, ns, c->max_nG, c->npe, nullptr, dp<int32_t>(c->bandLoc), dp<double>(c->bandK),
                           dp<double>(c->bandM), k2, dp<double>(c->wGG), s));
    std::vector<int32_t> flags;
    // X = B~_GG^{-1} B_GI ; S = B_II - B_IG X
    if (c->max_nG <= inv_gj_max_n()) {
        // small Gamma blocks: their inverses in one Gauss-Jordan launch (partial pivoting; the flags
        // mean what the LU's do), then X by one batched GEMM with the gathered rows
        HKG_TRY(walloc(c, &c->wGGi, std::max<int64_t>(c->nGG, 1) * sizeof(double)));
        HKG_TRY(walloc(c, &c->wGI2, std::max<int64_t>(c->nGI, 1) * sizeof(double)));
        // (no launch when every Gamma block is empty: the flags start at zero)
        HKG_HIP(hipMemsetAsync(c->wInfo.p, 0, ns * sizeof(int32_t), s));
        HKG_TRY(inv_gj_batched(dp<CopyJob>(c->jobsGGinv), ns, c->max_nG, dp<double>(c->wGG), dp<double>(c->wGGi),
                               dp<int32_t>(c->wInfo), s));
        HKG_TRY(gather_gamma_rows(dsub, ns, c->max_nI, c->max_nG, eigIO, dp<double>(c->wGI2), s));
        HKG_TRY(gemm_batched<double>(dp<GemmJob>(c->gjobsGX), ns, c->max_nG, c->max_nI, dp<double>(c->wGGi),
                                     dp<double>(c->wGI2), dp<double>(c->wGI), 1.0, 0.0, false, false, s));
    } else {
        HKG_TRY(lu_batched<double>(dp<DMat>(c->matsGG), dp<int64_t>(c->poffSub), ns, c->max_nG, dp<double>(c->wGG),
                                   dp<int32_t>(c->wPiv), dp<int32_t>(c->wInfo), true, s));
        HKG_TRY(gather_gamma_rows(dsub, ns, c->max_nI, c->max_nG, eigIO, dp<double>(c->wGI), s));
        HKG_TRY(apply_pivots_rows<double>(dsub, ns, c->max_nI, dp<int32_t>(c->wPiv), dp<double>(c->wGI), 0, s));
        // the Gamma block is dense: as a band of half-width n_G - 1 the solves take one launch each
        const int bandG = tri_band_fits(c->max_nG, c->max_nG - 1, sizeof(double)) ? c->max_nG - 1 : -1;
        HKG_TRY(tri_solve_batched<double>(dp<TriJob>(c->jobsGI), ns, c->max_nG, c->max_nI, dp<double>(c->wGG),
                                          dp<double>(c->wGI), TRI_LOWER_UNIT, s, bandG));
        HKG_TRY(tri_solve_batched<double>(dp<TriJob>(c->jobsGI), ns, c->max_nG, c->max_nI, dp<double>(c->wGG),
                                          dp<double>(c->wGI), TRI_UPPER, s, bandG));
    }
    HKG_TRY(copy_bii(dsub, ns, c->max_nI, eigIO, dp<double>(c->wS), s));
    HKG_TRY(gemm_batched<double>(dp<GemmJob>(c->gjobsSchur), ns, c->max_nI, c->max_nI, eigIO,
                                 dp<double>(c->wGI), dp<double>(c->wS), -1.0, 1.0, false, false, s));
    // S^ = D^{-1/2} L^{-1} S L^{-T} D^{-1/2} once C_II = L U is done
    if (enq_cii.joinable()) enq_cii.join();
    if (st_cii != HKG_OK) {
        set_last_error(err_cii);
        return st_cii;
    }
    HKG_HIP(hipStreamWaitEvent(s, c->ev_join3, 0));
    if (tri_lower_window_fits(c->max_nI, c->band_I)) {
        // X = L^{-1} S, right-hand side j read as row j of S (S is symmetric), written as X^T into wW
        // in the padded layout; then D^{-1/2} L^{-1} X^T D^{-1/2} (right-hand side j: row j of X, the
        // column j of wW) into the padded layout of the tridiagonalisation.  One thread per
        // right-hand side, the band of L in LDS, every global access coalesced or a thread's own run.
        HKG_TRY(walloc(c, &c->wT, (size_t)c->nM * sizeof(double)));
        HKG_TRY(tri_lower_window_batched(dp<TriJob>(c->jobsSq), ns, c->max_nI, c->max_nI, dp<double>(c->wCII),
                                         dp<double>(c->wS), false, dp<double>(c->wW), false, c->band_I, s));
        HKG_TRY(tri_lower_window_batched(dp<TriJob>(c->jobsSqM), ns, c->max_nI, c->max_nI, dp<double>(c->wCII),
                                         dp<double>(c->wW), true, dp<double>(c->wT), true, c->band_I, s));
    } else {
        HKG_TRY(tri_solve_batched<double>(dp<TriJob>(c->jobsSq), ns, c->max_nI, c->max_nI, dp<double>(c->wCII),
                                          dp<double>(c->wS), TRI_LOWER_UNIT, s, c->band_I));
        HKG_TRY(walloc(c, &c->wT, (size_t)c->nM * sizeof(double)));
        if (tri_band_fits(c->max_nI, c->band_I, sizeof(double))) {
            // the transpose read on the fly, D^{-1/2} on both sides applied as the result is written
            // into the padded layout of the tridiagonalisation
            HKG_TRY(tri_solve_batched<double>(dp<TriJob>(c->jobsSq), ns, c->max_nI, c->max_nI, dp<double>(c->wCII),
                                              dp<double>(c->wT), TRI_LOWER_UNIT, s, c->band_I, dp<double>(c->wS)));
        } else {
            HKG_TRY(transpose_batched<double>(dp<DMat>(c->matsSq), ns, c->max_nI, dp<double>(c->wS), dp<double>(c->wW), s));
            HKG_TRY(tri_solve_batched<double>(dp<TriJob>(c->jobsSq), ns, c->max_nI, c->max_nI, dp<double>(c->wCII),
                                              dp<double>(c->wW), TRI_LOWER_UNIT, s, c->band_I));
            HKG_TRY(scale_sym(dsub, ns, c->max_nI, dp<double>(c->wCII), dp<double>(c->wW), dp<double>(c->wT), s));
        }
    }
    // tridiagonal form and selection
    HKG_TRY(walloc(c, &c->wD, c->sum_nI * sizeof(double)));
    HKG_TRY(walloc(c, &c->wE, c->sum_nI * sizeof(double)));
    HKG_TRY(walloc(c, &c->wTau, c->sum_nI * sizeof(double)));
    HKG_TRY(walloc(c, &c->wVWV, (size_t)3 * 32 * c->sum_nI * sizeof(double)));
    HKG_TRY(tridiagonalize_blocked(dsub, ns, c->max_nI, dp<double>(c->wT), dp<double>(c->wVWV), dp<double>(c->wD),
                                   dp<double>(c->wE), dp<double>(c->wTau), s));
    HKG_TRY(walloc(c, &c->wM, ns * sizeof(int32_t)));
    HKG_TRY(walloc(c, &c->wLam, (size_t)ns * (mmax + 2) * sizeof(double)));
    HKG_TRY(walloc(c, &c->wIv, (size_t)5 * ns * sizeof(double)));
    HKG_TRY(select_eigs(dsub, ns, c->max_nI, dp<double>(c->wD), dp<double>(c->wE), o.eig_mode, o.tau, o.nev,
                        o.cluster_rtol, mmax, dp<int32_t>(c->wM), dp<double>(c->wLam), dp<int32_t>(c->wFlag),
                        dp<double>(c->wIv), s));
    // the counts, the eigenvalues and the three flag arrays come back together through pinned memory
    // (one wait); the checks deferred to this point follow in the order the quantities were computed
    const size_t nlam = (size_t)ns * (mmax + 2), rb_ints = 4 * (size_t)ns, rb_at = (rb_ints * 4 + 255) / 256 * 256;
    const size_t rb_bytes = rb_at + nlam * sizeof(double);
    if (c->h_read_cap < rb_bytes) {
        if (c->h_read) HKG_HIP(hipHostFree(c->h_read));
        c->h_read = nullptr;
        c->h_read_cap = 0;
        HKG_HIP(hipHostMalloc((void **)&c->h_read, rb_bytes));
        c->h_read_cap = rb_bytes;
    }
    int32_t *rb = reinterpret_cast<int32_t *>(c->h_read);
    double *rb_lam = reinterpret_cast<double *>(c->h_read + rb_at);
    HKG_HIP(hipMemcpyAsync(rb, c->wM.p, ns * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipMemcpyAsync(rb + ns, c->wInfo.p, ns * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipMemcpyAsync(rb + 2 * ns, c->wFlagSpd.p, ns * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipMemcpyAsync(rb + 3 * ns, c->wFlag.p, ns * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipMemcpyAsync(rb_lam, c->wLam.p, nlam * sizeof(double), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipStreamSynchronize(s));
    c->m_host.assign(rb, rb + ns);
    c->lam_host.assign(rb_lam, rb_lam + nlam);
    const std::vector<int32_t> fGamma(rb + ns, rb + 2 * ns), fSpd(rb + 2 * ns, rb + 3 * ns);
    flags.assign(rb + 3 * ns, rb + 4 * ns);
    for (int i = 0; i < ns; ++i)
        if (fGamma[i]) {
            set_last_error("the Gamma block of the local Neumann matrix is singular in subdomain " + std::to_string(i));
            return HKG_EEIG;
        }
    for (int i = 0; i < ns; ++i)
        if (fSpd[i]) {
            set_last_error("C_II is not positive definite in subdomain " + std::to_string(i));
            return HKG_EEIG;
        }
    for (int i = 0; i < ns; ++i)
        if (flags[i]) {
            set_last_error("subdomain " + std::to_string(i) + " needs " + std::to_string(c->m_host[i]) +
                           " eigenvectors, more than max_eig_per_sub");
            return HKG_EEIG;
        }
    // coarse layout
    int64_t offZ = 0, offY = 0;
    int offm = 0;
    c->max_m = 0;
    for (int i = 0; i < ns; ++i) {
        SubDev &sd = c->subs[i];
        sd.m = c->m_host[i];
        sd.offm = offm;
        sd.offZ = offZ;
        sd.offY = offY;
        offm += sd.m;
        offZ += (int64_t)sd.nI * sd.m;
        offY += (int64_t)sd.m * (sd.nI + sd.nG);
        c->max_m = std::max(c->max_m, sd.m);
    }
    c->m0 = offm;
    if (c->m0 > 7000) {
        set_last_error("coarse dimension " + std::to_string(c->m0) + " exceeds the supported 7000");
        return HKG_EINVAL;
    }
    // (c->subs stays as it is until the next analysis: no wait for the copy)
    HKG_HIP(hipMemcpyAsync(c->subs_d.p, c->subs.data(), ns * sizeof(SubDev), hipMemcpyHostToDevice, s));
    if (c->m0 == 0) return HKG_OK;
    // eigenvectors -> coarse basis Z_i = X_I P_i
    if (c->Z.bytes != (size_t)offZ * sizeof(double)) HKG_TRY(dalloc(c, &c->Z, offZ * sizeof(double)));
    HKG_TRY(walloc(c, &c->wInv, (size_t)offZ * (5 * sizeof(double) + 1)));
    int64_t max_nm = 0;
    for (int i = 0; i < ns; ++i) max_nm = std::max(max_nm, (int64_t)c->subs[i].nI * c->subs[i].m);
    HKG_TRY(tridiag_vectors_n(dsub, ns, c->max_nI, max_nm, dp<double>(c->wD), dp<double>(c->wE), dp<double>(c->wLam), mmax,
                              dp<double>(c->Z), dp<double>(c->wInv),
                              reinterpret_cast<unsigned char *>(dp<double>(c->wInv) + 5 * offZ), s));
    HKG_TRY(back_transform_n(dsub, ns, c->max_nI, c->max_m, dp<double>(c->wT), dp<double>(c->wTau), dp<double>(c->Z),
                             s));
    HKG_TRY(scale_rows_invsqrt_diag(dsub, ns, dp<double>(c->wCII), dp<double>(c->Z), s));
    {
        std::vector<TriJob> hj(ns);
        std::vector<GemmJob> hg(ns);
        int maxN = 0;
        for (int i = 0; i < ns; ++i) {
            const SubDev &sd = c->subs[i];
            hj[i] = {sd.offSq, sd.offZ, sd.nI, sd.nI, sd.m, sd.nI};
            hg[i] = {sd.offZ, sd.offBIO, sd.offY, sd.m, sd.nI + sd.nG, sd.nI, sd.nI, sd.nI, std::max(sd.m, 1)};
            maxN = std::max(maxN, sd.nI + sd.nG);
        }
        HKG_TRY(upload_staged(c, &c->wJobsZ, hj.data(), ns * sizeof(TriJob), s));
        HKG_TRY(upload_staged(c, &c->wGjobsY, hg.data(), ns * sizeof(GemmJob), s));
        if (tri_lower_window_fits(c->max_nI, c->band_I))
            HKG_TRY(tri_ltrans_window_batched(dp<TriJob>(c->wJobsZ), ns, c->max_nI, c->max_m, dp<double>(c->wCII),
                                              dp<double>(c->Z), c->band_I, s));
        else
            HKG_TRY(tri_solve_batched<double>(dp<TriJob>(c->wJobsZ), ns, c->max_nI, c->max_m, dp<double>(c->wCII),
                                              dp<double>(c->Z), TRI_LOWER_UNIT_TRANS, s, c->band_I));
        HKG_TRY(finish_basis(dsub, ns, dp<int32_t>(c->I_idx), dp<double>(c->winv), dp<double>(c->Z), s));
        if (c->Zr.bytes != (size_t)offZ * sizeof(double)) HKG_TRY(dalloc(c, &c->Zr, offZ * sizeof(double)));
        HKG_TRY(transpose_basis(dsub, ns, dp<double>(c->Z), dp<double>(c->Zr), s));
        const int64_t ntp = (int64_t)c->P.tp_pos.size();
        if (c->tpZ.bytes != (size_t)ntp * sizeof(TpCoarse)) HKG_TRY(dalloc(c, &c->tpZ, ntp * sizeof(TpCoarse)));
        HKG_TRY(tp_coarse(dsub, dp<int32_t>(c->tp_pos), dp<int32_t>(c->tp_sub), ntp, dp<TpCoarse>(c->tpZ), s));
        // Y_i = Z_i^T [B_II | B_IG]
        HKG_TRY(walloc(c, &c->wY, std::max<int64_t>(offY, 1) * sizeof(double)));
        HKG_TRY(gemm_batched<double>(dp<GemmJob>(c->wGjobsY), ns, c->max_m, maxN, dp<double>(c->Z), dp<double>(c->wBIO),
                                     dp<double>(c->wY), 1.0, 0.0, true, false, s));
    }
    // B_0 blocks over neighbouring pairs
    const CoarsePairs &CP = c->CP;
    const int npairs = (int)CP.pi.size();
    const int32_t *pp = dp<int32_t>(c->pairs);
    const int m0 = c->m0;
    HKG_TRY(walloc(c, &c->wB0, (size_t)m0 * m0 * sizeof(double)));
    HKG_HIP(hipMemsetAsync(c->wB0.p, 0, (size_t)m0 * m0 * sizeof(double), s));
    HKG_TRY(coarse_pairs(npairs, pp, pp + npairs, pp + 2 * npairs, pp + 3 * npairs + 1,
                         pp + 3 * npairs + 1 + CP.qi.size(), dsub, c->max_m, dp<double>(c->wY), dp<double>(c->Zr),
                         dp<double>(c->wB0), m0, s));
    if ((int64_t)m0 * m0 <= (int64_t)2048 * 2048) {
        // a device copy for queries (the LU below overwrites B_0); read back only when asked
        HKG_TRY(walloc(c, &c->B0copy, (size_t)m0 * m0 * sizeof(double)));
        HKG_HIP(hipMemcpyAsync(c->B0copy.p, c->wB0.p, (size_t)m0 * m0 * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
        drelease(c, &c->B0copy);
    }
    // the local-inverse pipeline runs beside the factorisation of B_0, whose panel chain keeps only
    // a few CUs busy (started earlier, it would compete with the tridiagonalisation, which fills
    // every CU)
    HKG_TRY(start_side());
    // B_0^{-1} by divide and conquer over the level blocks of B_0; the LU with partial pivoting of
    // the whole matrix (below) when the structure does not allow it or a block pivot is too small
    bool dc = false;
    HKG_TRY(coarse_inverse_dc(c, s, &dc));
    if (dc) return HKG_OK;
    // B_0 = P L U and B_0^{-1}
    DMat hm{0, m0, m0};
    int64_t hp0 = 0;
    TriJob tj{0, 0, m0, m0, m0, m0};
    uint8_t blob[sizeof(DMat) + sizeof(int64_t) + sizeof(TriJob)];
    std::memcpy(blob, &hm, sizeof(DMat));
    std::memcpy(blob + sizeof(DMat), &hp0, sizeof(int64_t));
    std::memcpy(blob + sizeof(DMat) + sizeof(int64_t), &tj, sizeof(TriJob));
    HKG_TRY(upload_bytes(c, &c->wMisc, blob, sizeof(blob), s, true));
    const DMat *dm = reinterpret_cast<const DMat *>(c->wMisc.p);
    const int64_t *dpo = reinterpret_cast<const int64_t *>((uint8_t *)c->wMisc.p + sizeof(DMat));
    const TriJob *dj = reinterpret_cast<const TriJob *>((uint8_t *)c->wMisc.p + sizeof(DMat) + sizeof(int64_t));
    HKG_TRY(walloc(c, &c->wPiv0, m0 * sizeof(int32_t)));
    // B_0 couples only overlapping subdomains: its half-bandwidth in the subdomain ordering bounds
    // the rows and columns each panel of the LU touches (dense when the band is not narrow)
    int band = 0;
    for (size_t t = 0; t < CP.pi.size(); ++t) {
        const SubDev &a = c->subs[CP.pi[t]], &b = c->subs[CP.pj[t]];
        if (a.m == 0 || b.m == 0) continue;
        band = std::max(band, std::max(a.offm + a.m - 1 - b.offm, b.offm + b.m - 1 - a.offm));
    }
    if (3 * band + LU_BLOCK >= m0) band = -1;
    c->b0_band = band;
    HKG_TRY(lu_batched<double>(dm, dpo, 1, m0, dp<double>(c->wB0), dp<int32_t>(c->wPiv0), dp<int32_t>(c->wInfo), true,
                               s, band));
    HKG_TRY(read_flags(c, c->wInfo, 1, &flags, s));
    if (flags[0]) {
        set_last_error("zero pivot in the coarse matrix B_0");
        return HKG_ESINGULAR_COARSE;
    }
    if (c->B0inv.bytes != (size_t)m0 * m0 * sizeof(double)) HKG_TRY(dalloc(c, &c->B0inv, (size_t)m0 * m0 * sizeof(double)));
    (void)dj;
    // U of the banded LU (row exchanges included) has half-bandwidth 2 band
    return lu_inverse(c, m0, dp<double>(c->wB0), dp<int32_t>(c->wPiv0), dp<double>(c->B0inv),
                      c->b0_band >= 0 ? 2 * c->b0_band : -1, s);
}

}  // namespace

int32_t factor(hkgeneo_ctx *c, hipStream_t s) {
    const int ns = c->n_sub;
    const SubDev *dsub = dp<SubDev>(c->subs_d);
    c->h_stage_used = 0;             // the previous factorisation ended with a wait on its streams
    if (!c->s2) {
        HKG_HIP(hipStreamCreateWithFlags(&c->s2, hipStreamNonBlocking));
        HKG_HIP(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        HKG_HIP(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    }
    if (!c->s3) {
        HKG_HIP(hipStreamCreateWithFlags(&c->s3, hipStreamNonBlocking));
        HKG_HIP(hipEventCreateWithFlags(&c->ev_fork3, hipEventDisableTiming));
        HKG_HIP(hipEventCreateWithFlags(&c->ev_join3, hipEventDisableTiming));
    }
    if (c->h_infoL_n < ns) {
        if (c->h_infoL) (void)hipHostFree(c->h_infoL);
        c->h_infoL = nullptr;
        c->h_infoL_n = 0;
        HKG_HIP(hipHostMalloc((void **)&c->h_infoL, ns * sizeof(int32_t)));
        c->h_infoL_n = ns;
    }
    HKG_TRY(walloc(c, &c->wDk, c->nnz * sizeof(double)));
    if (c->Bval.bytes != (size_t)c->nnz * sizeof(double)) HKG_TRY(dalloc(c, &c->Bval, c->nnz * sizeof(double)));
    HKG_TRY(form_operator(dp<double>(c->Aval), dp<double>(c->Sval), c->k * c->k, dp<double>(c->Bval), dp<double>(c->wDk),
                          c->nnz, s));
    HKG_TRY(walloc(c, &c->wBIO, c->nBIO * sizeof(double)));
    HKG_TRY(walloc(c, &c->wCII, c->nSq * sizeof(double)));
    HKG_HIP(hipMemsetAsync(c->wBIO.p, 0, c->nBIO * sizeof(double), s));
    HKG_HIP(hipMemsetAsync(c->wCII.p, 0, c->nSq * sizeof(double), s));
    // [B_II | B_IG] and C_II = X D_k[I, I] X; for Delta-GenEO the eigenproblem is that of the nearby SPD
    // problem (k = 0): C_II = X A[I, I] X and [A_II | A_IG] beside [B_II | B_IG] (the local solves and
    // the coarse matrix keep B)
    const bool delta = c->opt.coarse_op == HKG_COARSE_DELTA;
    HKG_TRY(extract_blocks(dsub, ns, c->max_nI, dp<int32_t>(c->rowptr), dp<int32_t>(c->colidx), dp<double>(c->Bval),
                           delta ? dp<double>(c->Aval) : dp<double>(c->wDk), dp<int32_t>(c->I_idx), dp<int32_t>(c->G_idx),
                           dp<double>(c->winv), dp<double>(c->wBIO), dp<double>(c->wCII), s));
    if (delta) {
        HKG_TRY(walloc(c, &c->wAIO, c->nBIO * sizeof(double)));
        HKG_HIP(hipMemsetAsync(c->wAIO.p, 0, c->nBIO * sizeof(double), s));
        HKG_TRY(extract_blocks(dsub, ns, c->max_nI, dp<int32_t>(c->rowptr), dp<int32_t>(c->colidx), dp<double>(c->Aval),
                               dp<double>(c->Aval), dp<int32_t>(c->I_idx), dp<int32_t>(c->G_idx), dp<double>(c->winv),
                               dp<double>(c->wAIO), dp<double>(c->wCII), s));
    }
    // the local inverses (reading B_II) on the second stream, the coarse space on the caller's: the
    // two pipelines share no buffer written after this point.  The local pipeline is enqueued by a
    // helper thread (about a hundred launches) while this thread enqueues the coarse space, which
    // waits on the device several times; it is forked once coarse_space has its first launches in.
    // (a coarse-only context of a nested decomposition has no local inverses: its first-level
    // subdomains live in a context of their own)
    if (!c->coarse_only) HKG_TRY(local_buffers(c));
    int32_t st_local = HKG_OK;
    std::string err_local;
    std::thread enq;
    auto start_side = [&]() -> int32_t {
        if (enq.joinable() || c->coarse_only) return HKG_OK;
        HKG_HIP(hipEventRecord(c->ev_fork, s));
        HKG_HIP(hipStreamWaitEvent(c->s2, c->ev_fork, 0));
        enq = std::thread([&]() {
            st_local = local_operators(c, c->s2);
            if (st_local != HKG_OK) err_local = g_last_error;
        });
        return HKG_OK;
    };
    int32_t st = c->opt.two_level ? coarse_space(c, s, start_side) : HKG_OK;
    if (!enq.joinable()) {
        const int32_t st2 = start_side();
        if (st == HKG_OK) st = st2;
    }
    if (enq.joinable()) enq.join();
    if (st == HKG_OK && st_local != HKG_OK) {
        set_last_error(err_local);
        st = st_local;
    }
    // join before returning, whatever happened on either side
    const hipError_t e1 = hipEventRecord(c->ev_join, c->s2);
    const hipError_t e2 = hipStreamWaitEvent(s, c->ev_join, 0);
    const hipError_t e3 = hipStreamSynchronize(s);
    const hipError_t e4 = hipStreamSynchronize(c->s3);
    HKG_TRY(st);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) {
        set_last_error("joining the side streams of the factorisation");
        return HKG_EHIP;
    }
    for (int i = 0; i < ns && !c->coarse_only; ++i)
        if (c->h_infoL[i]) {
            set_last_error("zero pivot in the local Dirichlet matrix of subdomain " + std::to_string(i));
            return HKG_ESINGULAR_LOCAL;
        }
    return HKG_OK;
}

}  // namespace hkg
