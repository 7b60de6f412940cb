// C ABI of libhkgeneo: setup of the two-level Schwarz preconditioner with the H_k-GenEO coarse
// space, its application, and right-preconditioned flexible GMRES, all on one HIP device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"

namespace hkg {
thread_local std::string g_last_error;
void set_last_error(const std::string &msg) { g_last_error = msg; }

// declared in krylov.hip
int32_t gmres_arnoldi_step(const GmresDev &G, int j, double rtol, hipStream_t s);
int32_t gmres_cycle_start(const GmresDev &G, const double *rnorm, double rtol, const int32_t *want, hipStream_t s);
int32_t gmres_cycle_update(const GmresDev &G, double *x, int ldx, hipStream_t s);
int gmres_rows_per_block();
}  // namespace hkg

using namespace hkg;

struct hkgeneo_ctx {
    hkgeneo_options opt{};
    int n_dof = 0, nnz = 0, n_sub = 0, m0 = 0, max_nI = 0, max_nG = 0, max_m = 0, npe = 0;
    int64_t sum_nI = 0;
    double k = 0.0;
    Partition P;
    std::vector<SubDev> subs;
    std::vector<int32_t> m_host;
    std::vector<double> lam_host;     // n_sub x (mmax + 2)
    std::vector<double> B0_host;      // kept for queries when m0 is small
    std::vector<DevBuf *> owned;
    int64_t device_bytes = 0;
    // resident device data
    DevBuf rowptr, colidx, Bval, I_idx, G_idx, winv, wloc, tp_ptr, tp_pos, subs_d;
    DevBuf Minv, Z, B0inv;
    // apply workspace
    DevBuf u, c, y;
    int ws_nrhs = 0;
    // gmres workspace
    DevBuf V, Zk, H, cs, sn, g, part, hcol, scal, active, want, rnorm, npart, fnorm;
    int gm_nrhs = 0;
    hkgeneo_stats stats{};
};

static int32_t alloc(hkgeneo_ctx *c, DevBuf *b, size_t bytes) {
    if (b->p) {
        (void)hipFree(b->p);
        c->device_bytes -= (int64_t)b->bytes;
        b->p = nullptr;
        b->bytes = 0;
    }
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
    return HKG_OK;
}

static void release(hkgeneo_ctx *c, DevBuf *b) {
    if (b->p) {
        (void)hipFree(b->p);
        c->device_bytes -= (int64_t)b->bytes;
    }
    b->p = nullptr;
    b->bytes = 0;
}

// host -> device copy that has completed when it returns (the host source may be a temporary)
template <typename T>
static int32_t upload(hkgeneo_ctx *c, DevBuf *b, const T *host, size_t count, hipStream_t s) {
    HKG_TRY(alloc(c, b, count * sizeof(T)));
    if (count) {
        HKG_HIP(hipMemcpyAsync(b->p, host, count * sizeof(T), hipMemcpyHostToDevice, s));
        HKG_HIP(hipStreamSynchronize(s));
    }
    return HKG_OK;
}

template <typename T>
static T *dp(const DevBuf &b) {
    return reinterpret_cast<T *>(b.p);
}

extern "C" void hkgeneo_default_options(hkgeneo_options *o) {
    if (!o) return;
    o->eig_mode = HKG_EIG_FIXED;
    o->tau = 0.0;
    o->nev = 10;
    o->cluster_rtol = 1e-8;
    o->max_eig_per_sub = 64;
    o->local_prec = 64;
    o->prolong = HKG_PROLONG_AS;
    o->two_level = 1;
    o->restart = 50;
    o->max_iter = 1000;
    o->rtol = 1e-8;
}

extern "C" const char *hkgeneo_strerror(int32_t st) {
    switch (st) {
        case HKG_OK: return "ok";
        case HKG_EINVAL: return "invalid argument";
        case HKG_ENOMEM: return "out of device memory";
        case HKG_EHIP: return "HIP runtime error";
        case HKG_ESINGULAR_LOCAL: return "singular local Dirichlet matrix";
        case HKG_EEIG: return "local eigenproblem failed";
        case HKG_ESINGULAR_COARSE: return "singular coarse matrix";
        case HKG_ENOTCONV: return "not converged";
        default: return "unknown status";
    }
}

extern "C" const char *hkgeneo_last_error(void) { return hkg::g_last_error.c_str(); }

static void destroy_all(hkgeneo_ctx *c) {
    DevBuf *bufs[] = {&c->rowptr, &c->colidx, &c->Bval,   &c->I_idx, &c->G_idx, &c->winv,  &c->wloc,  &c->tp_ptr,
                      &c->tp_pos, &c->subs_d, &c->Minv,   &c->Z,     &c->B0inv, &c->u,     &c->c,     &c->y,
                      &c->V,      &c->Zk,     &c->H,      &c->cs,    &c->sn,    &c->g,     &c->part,  &c->hcol,
                      &c->scal,   &c->active, &c->want,   &c->rnorm, &c->npart, &c->fnorm};
    for (DevBuf *b : bufs) release(c, b);
}

extern "C" void hkgeneo_destroy(hkgeneo_ctx *c) {
    if (!c) return;
    destroy_all(c);
    delete c;
}

// ------------------------------------------------------------------------------------------------
// setup
// ------------------------------------------------------------------------------------------------
namespace {

struct Transient {
    hkgeneo_ctx *c;
    std::vector<DevBuf> bufs;
    explicit Transient(hkgeneo_ctx *cc, int n) : c(cc), bufs(n) {}
    ~Transient() {
        for (auto &b : bufs) release(c, &b);
    }
};

int32_t check_problem(const hkgeneo_problem *p, const hkgeneo_options *o) {
    if (!p || !o) return HKG_EINVAL;
    if (!(p->dim == 2 || p->dim == 3)) return HKG_EINVAL;
    if (!(p->elem_type == HKG_P1 || p->elem_type == HKG_Q1)) return HKG_EINVAL;
    if (p->n_vert <= 0 || p->n_elem <= 0 || p->n_dof <= 0 || p->nnz <= 0 || p->n_sub <= 0) return HKG_EINVAL;
    if (!p->elem_vert || !p->vert_dof || !p->elem_K || !p->elem_M || !p->row_ptr || !p->col_idx || !p->A_val ||
        !p->S_val || !p->elem_part || !p->overlap)
        return HKG_EINVAL;
    if (!(p->k >= 0.0) || !std::isfinite(p->k)) return HKG_EINVAL;
    if (p->row_ptr[0] != 0 || p->row_ptr[p->n_dof] != p->nnz) return HKG_EINVAL;
    for (int i = 0; i < p->n_dof; ++i) {
        if (p->row_ptr[i + 1] < p->row_ptr[i]) return HKG_EINVAL;
        for (int t = p->row_ptr[i]; t < p->row_ptr[i + 1]; ++t) {
            if (p->col_idx[t] < 0 || p->col_idx[t] >= p->n_dof) return HKG_EINVAL;
            if (t > p->row_ptr[i] && p->col_idx[t] <= p->col_idx[t - 1]) return HKG_EINVAL;
        }
    }
    for (int s = 0; s < p->n_sub; ++s)
        if (p->overlap[s] < 1) return HKG_EINVAL;
    if (!(o->eig_mode == HKG_EIG_FIXED || o->eig_mode == HKG_EIG_THRESHOLD)) return HKG_EINVAL;
    if (o->nev < 0 || o->max_eig_per_sub < 1 || !(o->cluster_rtol >= 0.0)) return HKG_EINVAL;
    if (!(o->local_prec == 64 || o->local_prec == 32)) return HKG_EINVAL;
    if (!(o->prolong == HKG_PROLONG_AS || o->prolong == HKG_PROLONG_POU)) return HKG_EINVAL;
    if (o->restart < 1 || o->max_iter < 1 || !(o->rtol > 0.0)) return HKG_EINVAL;
    return HKG_OK;
}

template <typename T>
int32_t local_inverses(hkgeneo_ctx *c, const DevBuf &BIO, hipStream_t s, const DevBuf &subs_d, int32_t *bad) {
    const int ns = c->n_sub;
    Transient tr(c, 6);
    DevBuf &LU = tr.bufs[0], &piv = tr.bufs[1], &info = tr.bufs[2], &mats = tr.bufs[3], &poff = tr.bufs[4],
           &jobs = tr.bufs[5];
    std::vector<DMat> hm(ns);
    std::vector<int64_t> hp(ns);
    int64_t sq = 0, pv = 0;
    for (int i = 0; i < ns; ++i) {
        hm[i] = {c->subs[i].offSq, c->subs[i].nI, c->subs[i].nI};
        hp[i] = pv;
        sq += (int64_t)c->subs[i].nI * c->subs[i].nI;
        pv += c->subs[i].nI;
    }
    HKG_TRY(alloc(c, &LU, sq * sizeof(T)));
    HKG_TRY(alloc(c, &c->Minv, sq * sizeof(T)));
    HKG_TRY(alloc(c, &piv, pv * sizeof(int32_t)));
    HKG_TRY(alloc(c, &info, ns * sizeof(int32_t)));
    HKG_TRY(upload(c, &mats, hm.data(), hm.size(), s));
    HKG_TRY(upload(c, &poff, hp.data(), hp.size(), s));
    if (sizeof(T) == 8) HKG_TRY(copy_bii(dp<SubDev>(subs_d), ns, c->max_nI, dp<double>(BIO), (double *)LU.p, s));
    else HKG_TRY(copy_bii_f32(dp<SubDev>(subs_d), ns, c->max_nI, dp<double>(BIO), (float *)LU.p, s));
    HKG_TRY(lu_batched<T>(dp<DMat>(mats), dp<int64_t>(poff), ns, c->max_nI, dp<T>(LU), dp<int32_t>(piv),
                          dp<int32_t>(info), true, s));
    std::vector<int32_t> hinfo(ns);
    HKG_HIP(hipMemcpyAsync(hinfo.data(), info.p, ns * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < ns; ++i)
        if (hinfo[i] != 0) {
            *bad = i;
            set_last_error("zero pivot in the local Dirichlet matrix of subdomain " + std::to_string(i));
            return HKG_ESINGULAR_LOCAL;
        }
    // inverse from the factors: B_D^{-1} = U^{-1} L^{-1} P
    std::vector<TriJob> hj(ns);
    for (int i = 0; i < ns; ++i) hj[i] = {c->subs[i].offSq, c->subs[i].offSq, c->subs[i].nI, c->subs[i].nI,
                                          c->subs[i].nI, c->subs[i].nI};
    HKG_TRY(upload(c, &jobs, hj.data(), hj.size(), s));
    HKG_TRY(perm_identity_batched<T>(dp<DMat>(mats), dp<int64_t>(poff), ns, c->max_nI, dp<int32_t>(piv),
                                     dp<T>(c->Minv), s));
    HKG_TRY(tri_solve_batched<T>(dp<TriJob>(jobs), ns, c->max_nI, c->max_nI, dp<T>(LU), dp<T>(c->Minv), TRI_LOWER_UNIT,
                                 s));
    HKG_TRY(tri_solve_batched<T>(dp<TriJob>(jobs), ns, c->max_nI, c->max_nI, dp<T>(LU), dp<T>(c->Minv), TRI_UPPER, s));
    HKG_HIP(hipStreamSynchronize(s));
    return HKG_OK;
}

int32_t coarse_setup(hkgeneo_ctx *c, const hkgeneo_problem *p, const DevBuf &BIO, const DevBuf &CII, hipStream_t s,
                     int32_t *bad) {
    const int ns = c->n_sub;
    const hkgeneo_options &o = c->opt;
    const int mmax = o.max_eig_per_sub;
    Transient tr(c, 24);
    DevBuf &GG = tr.bufs[0], &GI = tr.bufs[1], &Sb = tr.bufs[2], &Wb = tr.bufs[3], &piv = tr.bufs[4],
           &info = tr.bufs[5], &matsGG = tr.bufs[6], &poff = tr.bufs[7], &jobs = tr.bufs[8], &gjobs = tr.bufs[9],
           &matsSq = tr.bufs[10], &dd = tr.bufs[11], &ee = tr.bufs[12], &tt = tr.bufs[13], &mbuf = tr.bufs[14],
           &lam = tr.bufs[15], &flag = tr.bufs[16], &Yb = tr.bufs[17], &B0 = tr.bufs[18], &pairs = tr.bufs[19],
           &bandK = tr.bufs[20], &bandM = tr.bufs[21], &bandLoc = tr.bufs[22], &misc = tr.bufs[23];
    const Partition &P = c->P;
    int64_t nGG = 0, nGI = 0, nSq = 0, npv = 0;
    std::vector<DMat> hGG(ns), hSq(ns);
    std::vector<int64_t> hpo(ns);
    for (int i = 0; i < ns; ++i) {
        const SubDev &sd = c->subs[i];
        hGG[i] = {sd.offGG, sd.nG, std::max(sd.nG, 1)};
        hSq[i] = {sd.offSq, sd.nI, sd.nI};
        hpo[i] = sd.offPiv;
        nGG += (int64_t)sd.nG * sd.nG;
        nGI += (int64_t)sd.nG * sd.nI;
        nSq += (int64_t)sd.nI * sd.nI;
        npv = std::max<int64_t>(npv, sd.offPiv + std::max(sd.nI, sd.nG));
    }
    const int npe = c->npe, npe2 = npe * npe;
    // band element matrices (only the elements of each subdomain that carry Gamma dofs)
    {
        const size_t nb = P.band_elem.size();
        std::vector<double> hk(nb * npe2), hmm(nb * npe2);
        for (size_t b = 0; b < nb; ++b) {
            std::memcpy(&hk[b * npe2], p->elem_K + (size_t)P.band_elem[b] * npe2, npe2 * sizeof(double));
            std::memcpy(&hmm[b * npe2], p->elem_M + (size_t)P.band_elem[b] * npe2, npe2 * sizeof(double));
        }
        HKG_TRY(upload(c, &bandK, hk.data(), hk.size(), s));
        HKG_TRY(upload(c, &bandM, hmm.data(), hmm.size(), s));
        HKG_TRY(upload(c, &bandLoc, P.band_loc.data(), P.band_loc.size(), s));
    }
    HKG_TRY(alloc(c, &GG, nGG * sizeof(double)));
    HKG_TRY(alloc(c, &GI, nGI * sizeof(double)));
    HKG_TRY(alloc(c, &Sb, nSq * sizeof(double)));
    HKG_TRY(alloc(c, &Wb, nSq * sizeof(double)));
    HKG_TRY(alloc(c, &piv, npv * sizeof(int32_t)));
    HKG_TRY(alloc(c, &info, ns * sizeof(int32_t)));
    HKG_TRY(upload(c, &matsGG, hGG.data(), ns, s));
    HKG_TRY(upload(c, &matsSq, hSq.data(), ns, s));
    HKG_TRY(upload(c, &poff, hpo.data(), ns, s));
    HKG_HIP(hipMemsetAsync(GG.p, 0, GG.bytes, s));
    const SubDev *dsub = dp<SubDev>(c->subs_d);
    const double k2 = c->k * c->k;
    // B~_GG and its LU
    HKG_TRY(assemble_gamma(dsub, ns, npe, nullptr, dp<int32_t>(bandLoc), dp<double>(bandK), dp<double>(bandM), k2,
                           dp<double>(GG), s));
    HKG_TRY(lu_batched<double>(dp<DMat>(matsGG), dp<int64_t>(poff), ns, c->max_nG, dp<double>(GG), dp<int32_t>(piv),
                               dp<int32_t>(info), true, s));
    std::vector<int32_t> hinfo(ns);
    HKG_HIP(hipMemcpyAsync(hinfo.data(), info.p, ns * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < ns; ++i)
        if (hinfo[i]) {
            *bad = i;
            set_last_error("the Gamma block of the local Neumann matrix is singular in subdomain " + std::to_string(i));
            return HKG_EEIG;
        }
    // X = B~_GG^{-1} B_GI
    HKG_TRY(gather_gamma_rows(dsub, ns, c->max_nI, dp<double>(BIO), dp<double>(GI), s));
    HKG_TRY(apply_pivots_rows<double>(dsub, ns, c->max_nI, dp<int32_t>(piv), dp<double>(GI), 0, s));
    {
        std::vector<TriJob> hj(ns);
        for (int i = 0; i < ns; ++i) {
            const SubDev &sd = c->subs[i];
            hj[i] = {sd.offGG, sd.offGI, sd.nG, std::max(sd.nG, 1), sd.nI, std::max(sd.nG, 1)};
        }
        HKG_TRY(upload(c, &jobs, hj.data(), ns, s));
        HKG_TRY(tri_solve_batched<double>(dp<TriJob>(jobs), ns, c->max_nG, c->max_nI, dp<double>(GG), dp<double>(GI),
                                          TRI_LOWER_UNIT, s));
        HKG_TRY(tri_solve_batched<double>(dp<TriJob>(jobs), ns, c->max_nG, c->max_nI, dp<double>(GG), dp<double>(GI),
                                          TRI_UPPER, s));
    }
    // S = B_II - B_IG X
    HKG_TRY(copy_bii(dsub, ns, c->max_nI, dp<double>(BIO), dp<double>(Sb), s));
    {
        std::vector<GemmJob> hg(ns);
        for (int i = 0; i < ns; ++i) {
            const SubDev &sd = c->subs[i];
            hg[i] = {sd.offBIO + (int64_t)sd.nI * sd.nI, sd.offGI, sd.offSq, sd.nI, sd.nI, sd.nG, sd.nI,
                     std::max(sd.nG, 1), sd.nI};
        }
        HKG_TRY(upload(c, &gjobs, hg.data(), ns, s));
        HKG_TRY(gemm_batched<double>(dp<GemmJob>(gjobs), ns, c->max_nI, c->max_nI, dp<double>(BIO), dp<double>(GI),
                                     dp<double>(Sb), -1.0, 1.0, false, false, s));
    }
    // C_II = L U without row exchanges (SPD check), then S^ = D^{-1/2} L^{-1} S L^{-T} D^{-1/2}
    HKG_TRY(lu_batched<double>(dp<DMat>(matsSq), dp<int64_t>(poff), ns, c->max_nI, dp<double>(CII), dp<int32_t>(piv),
                               dp<int32_t>(info), false, s));
    HKG_TRY(alloc(c, &flag, ns * sizeof(int32_t)));
    HKG_TRY(check_spd_pivots(dsub, ns, dp<double>(CII), dp<int32_t>(flag), s));
    std::vector<int32_t> hflag(ns);
    HKG_HIP(hipMemcpyAsync(hflag.data(), flag.p, ns * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < ns; ++i)
        if (hflag[i]) {
            *bad = i;
            set_last_error("C_II is not positive definite in subdomain " + std::to_string(i));
            return HKG_EEIG;
        }
    {
        std::vector<TriJob> hj(ns);
        for (int i = 0; i < ns; ++i) {
            const SubDev &sd = c->subs[i];
            hj[i] = {sd.offSq, sd.offSq, sd.nI, sd.nI, sd.nI, sd.nI};
        }
        HKG_TRY(upload(c, &jobs, hj.data(), ns, s));
        HKG_TRY(tri_solve_batched<double>(dp<TriJob>(jobs), ns, c->max_nI, c->max_nI, dp<double>(CII), dp<double>(Sb),
                                          TRI_LOWER_UNIT, s));
        HKG_TRY(transpose_batched<double>(dp<DMat>(matsSq), ns, c->max_nI, dp<double>(Sb), dp<double>(Wb), s));
        HKG_TRY(tri_solve_batched<double>(dp<TriJob>(jobs), ns, c->max_nI, c->max_nI, dp<double>(CII), dp<double>(Wb),
                                          TRI_LOWER_UNIT, s));
        HKG_TRY(scale_sym(dsub, ns, c->max_nI, dp<double>(CII), dp<double>(Wb), s));
    }
    // tridiagonal form, selection
    HKG_TRY(alloc(c, &dd, c->sum_nI * sizeof(double)));
    HKG_TRY(alloc(c, &ee, c->sum_nI * sizeof(double)));
    HKG_TRY(alloc(c, &tt, c->sum_nI * sizeof(double)));
    HKG_TRY(tridiagonalize_n(dsub, ns, c->max_nI, dp<double>(Wb), dp<double>(dd), dp<double>(ee), dp<double>(tt), s));
    HKG_TRY(alloc(c, &mbuf, ns * sizeof(int32_t)));
    HKG_TRY(alloc(c, &lam, (size_t)ns * (mmax + 2) * sizeof(double)));
    HKG_TRY(select_eigs(dsub, ns, dp<double>(dd), dp<double>(ee), o.eig_mode, o.tau, o.nev, o.cluster_rtol, mmax,
                        dp<int32_t>(mbuf), dp<double>(lam), dp<int32_t>(flag), s));
    c->m_host.assign(ns, 0);
    c->lam_host.assign((size_t)ns * (mmax + 2), 0.0);
    HKG_HIP(hipMemcpyAsync(c->m_host.data(), mbuf.p, ns * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipMemcpyAsync(hflag.data(), flag.p, ns * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipMemcpyAsync(c->lam_host.data(), lam.p, c->lam_host.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < ns; ++i)
        if (hflag[i]) {
            *bad = i;
            set_last_error("subdomain " + std::to_string(i) + " needs " + std::to_string(c->m_host[i]) +
                           " eigenvectors, more than max_eig_per_sub");
            return HKG_EEIG;
        }
    // offsets of the coarse basis
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
    HKG_HIP(hipMemcpyAsync(c->subs_d.p, c->subs.data(), ns * sizeof(SubDev), hipMemcpyHostToDevice, s));
    HKG_HIP(hipStreamSynchronize(s));
    if (c->m0 == 0) return HKG_OK;
    HKG_TRY(alloc(c, &c->Z, offZ * sizeof(double)));
    HKG_TRY(tridiag_vectors_n(dsub, ns, c->max_nI, dp<double>(dd), dp<double>(ee), dp<double>(lam), mmax, dp<double>(c->Z),
                              s));
    HKG_TRY(back_transform_n(dsub, ns, mmax, dp<double>(Wb), dp<double>(tt), dp<double>(c->Z), s));
    HKG_TRY(scale_rows_invsqrt_diag(dsub, ns, dp<double>(CII), dp<double>(c->Z), s));
    {
        std::vector<TriJob> hj(ns);
        for (int i = 0; i < ns; ++i) {
            const SubDev &sd = c->subs[i];
            hj[i] = {sd.offSq, sd.offZ, sd.nI, sd.nI, sd.m, sd.nI};
        }
        HKG_TRY(upload(c, &jobs, hj.data(), ns, s));
        HKG_TRY(tri_solve_batched<double>(dp<TriJob>(jobs), ns, c->max_nI, c->max_m, dp<double>(CII), dp<double>(c->Z),
                                          TRI_LOWER_UNIT_TRANS, s));
    }
    HKG_TRY(finish_basis(dsub, ns, dp<int32_t>(c->I_idx), dp<double>(c->winv), dp<double>(c->Z), s));
    // Y_i = Z_i^T [B_II | B_IG]
    HKG_TRY(alloc(c, &Yb, std::max<int64_t>(offY, 1) * sizeof(double)));
    {
        std::vector<GemmJob> hg(ns);
        int maxN = 0;
        for (int i = 0; i < ns; ++i) {
            const SubDev &sd = c->subs[i];
            hg[i] = {sd.offZ, sd.offBIO, sd.offY, sd.m, sd.nI + sd.nG, sd.nI, sd.nI, sd.nI, std::max(sd.m, 1)};
            maxN = std::max(maxN, sd.nI + sd.nG);
        }
        HKG_TRY(upload(c, &gjobs, hg.data(), ns, s));
        HKG_TRY(gemm_batched<double>(dp<GemmJob>(gjobs), ns, c->max_m, maxN, dp<double>(c->Z), dp<double>(BIO),
                                     dp<double>(Yb), 1.0, 0.0, true, false, s));
    }
    // B_0 blocks
    CoarsePairs CP;
    build_coarse_pairs(P, &CP);
    const int npairs = (int)CP.pi.size();
    std::vector<int32_t> packed;
    packed.insert(packed.end(), CP.pi.begin(), CP.pi.end());
    packed.insert(packed.end(), CP.pj.begin(), CP.pj.end());
    packed.insert(packed.end(), CP.ptr.begin(), CP.ptr.end());
    packed.insert(packed.end(), CP.qi.begin(), CP.qi.end());
    packed.insert(packed.end(), CP.qj.begin(), CP.qj.end());
    HKG_TRY(upload(c, &pairs, packed.data(), packed.size(), s));
    const int32_t *pp = dp<int32_t>(pairs);
    const int m0 = c->m0;
    HKG_TRY(alloc(c, &B0, (size_t)m0 * m0 * sizeof(double)));
    HKG_HIP(hipMemsetAsync(B0.p, 0, B0.bytes, s));
    HKG_TRY(coarse_pairs(npairs, pp, pp + npairs, pp + 2 * npairs, pp + 3 * npairs + 1,
                         pp + 3 * npairs + 1 + CP.qi.size(), dsub, dp<double>(Yb), dp<double>(c->Z), dp<double>(B0), m0,
                         s));
    if ((int64_t)m0 * m0 <= (int64_t)2048 * 2048) {
        c->B0_host.resize((size_t)m0 * m0);
        HKG_HIP(hipMemcpyAsync(c->B0_host.data(), B0.p, B0.bytes, hipMemcpyDeviceToHost, s));
    }
    // B_0 = P L U and B_0^{-1}
    {
        DMat hm{0, m0, m0};
        int64_t hp0 = 0;
        DevBuf &m1 = misc;
        std::vector<uint8_t> blob(sizeof(DMat) + sizeof(int64_t) + sizeof(TriJob));
        TriJob tj{0, 0, m0, m0, m0, m0};
        std::memcpy(blob.data(), &hm, sizeof(DMat));
        std::memcpy(blob.data() + sizeof(DMat), &hp0, sizeof(int64_t));
        std::memcpy(blob.data() + sizeof(DMat) + sizeof(int64_t), &tj, sizeof(TriJob));
        HKG_TRY(upload(c, &m1, blob.data(), blob.size(), s));
        const DMat *dm = reinterpret_cast<const DMat *>(m1.p);
        const int64_t *dpo = reinterpret_cast<const int64_t *>((uint8_t *)m1.p + sizeof(DMat));
        const TriJob *dj = reinterpret_cast<const TriJob *>((uint8_t *)m1.p + sizeof(DMat) + sizeof(int64_t));
        DevBuf &pv0 = mbuf;
        HKG_TRY(alloc(c, &pv0, m0 * sizeof(int32_t)));
        HKG_TRY(lu_batched<double>(dm, dpo, 1, m0, dp<double>(B0), dp<int32_t>(pv0), dp<int32_t>(info), true, s));
        int32_t hi0 = 0;
        HKG_HIP(hipMemcpyAsync(&hi0, info.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HKG_HIP(hipStreamSynchronize(s));
        if (hi0) {
            set_last_error("zero pivot in the coarse matrix B_0");
            return HKG_ESINGULAR_COARSE;
        }
        HKG_TRY(alloc(c, &c->B0inv, (size_t)m0 * m0 * sizeof(double)));
        HKG_TRY(perm_identity_batched<double>(dm, dpo, 1, m0, dp<int32_t>(pv0), dp<double>(c->B0inv), s));
        HKG_TRY(tri_solve_batched<double>(dj, 1, m0, m0, dp<double>(B0), dp<double>(c->B0inv), TRI_LOWER_UNIT, s));
        HKG_TRY(tri_solve_batched<double>(dj, 1, m0, m0, dp<double>(B0), dp<double>(c->B0inv), TRI_UPPER, s));
    }
    HKG_HIP(hipStreamSynchronize(s));
    return HKG_OK;
}

}  // namespace

static int32_t setup_body(hkgeneo_ctx *c, const hkgeneo_problem *p, const hkgeneo_options *o, hipStream_t s,
                          int32_t *bad) {
    HKG_TRY(build_partition(p, &c->P, bad));
    c->npe = c->P.npe;
    const Partition &P = c->P;
    const int ns = c->n_sub;
    // per-subdomain layout
    c->subs.resize(ns);
    int64_t oBIO = 0, oSq = 0, oGG = 0, oGI = 0, oPiv = 0;
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
        sd.bandBeg = P.band_ptr[i];
        sd.bandEnd = P.band_ptr[i + 1];
        oBIO += (int64_t)sd.nI * (sd.nI + sd.nG);
        oSq += (int64_t)sd.nI * sd.nI;
        oGG += (int64_t)sd.nG * sd.nG;
        oGI += (int64_t)sd.nG * sd.nI;
        oPiv += std::max(sd.nI, sd.nG);
        c->max_nI = std::max(c->max_nI, sd.nI);
        c->max_nG = std::max(c->max_nG, sd.nG);
    }
    c->sum_nI = P.offI[ns];
    // resident inputs (1/mu from the multiplicities of the partitioner)
    std::vector<double> winv(c->n_dof), wloc(c->sum_nI);
    for (int d = 0; d < c->n_dof; ++d) winv[d] = 1.0 / (double)P.mu[d];
    for (int64_t t = 0; t < c->sum_nI; ++t) wloc[t] = (o->prolong == HKG_PROLONG_POU) ? winv[P.I_idx[t]] : 1.0;
    HKG_TRY(upload(c, &c->rowptr, p->row_ptr, c->n_dof + 1, s));
    HKG_TRY(upload(c, &c->colidx, p->col_idx, c->nnz, s));
    HKG_TRY(upload(c, &c->I_idx, P.I_idx.data(), P.I_idx.size(), s));
    if (P.G_idx.empty()) HKG_TRY(alloc(c, &c->G_idx, sizeof(int32_t)));
    else HKG_TRY(upload(c, &c->G_idx, P.G_idx.data(), P.G_idx.size(), s));
    HKG_TRY(upload(c, &c->winv, winv.data(), winv.size(), s));
    HKG_TRY(upload(c, &c->wloc, wloc.data(), wloc.size(), s));
    HKG_TRY(upload(c, &c->tp_ptr, P.tp_ptr.data(), P.tp_ptr.size(), s));
    HKG_TRY(upload(c, &c->tp_pos, P.tp_pos.data(), P.tp_pos.size(), s));
    HKG_TRY(upload(c, &c->subs_d, c->subs.data(), ns, s));
    Transient tr(c, 5);
    DevBuf &Av = tr.bufs[0], &Sv = tr.bufs[1], &Dk = tr.bufs[2], &BIO = tr.bufs[3], &CII = tr.bufs[4];
    HKG_TRY(upload(c, &Av, p->A_val, c->nnz, s));
    HKG_TRY(upload(c, &Sv, p->S_val, c->nnz, s));
    HKG_TRY(alloc(c, &c->Bval, c->nnz * sizeof(double)));
    HKG_TRY(alloc(c, &Dk, c->nnz * sizeof(double)));
    HKG_TRY(form_operator(dp<double>(Av), dp<double>(Sv), c->k * c->k, dp<double>(c->Bval), dp<double>(Dk), c->nnz, s));
    HKG_TRY(alloc(c, &BIO, oBIO * sizeof(double)));
    HKG_TRY(alloc(c, &CII, oSq * sizeof(double)));
    HKG_HIP(hipMemsetAsync(BIO.p, 0, BIO.bytes, s));
    HKG_HIP(hipMemsetAsync(CII.p, 0, CII.bytes, s));
    HKG_TRY(extract_blocks(dp<SubDev>(c->subs_d), ns, c->max_nI, dp<int32_t>(c->rowptr), dp<int32_t>(c->colidx),
                           dp<double>(c->Bval), dp<double>(Dk), dp<int32_t>(c->I_idx), dp<int32_t>(c->G_idx),
                           dp<double>(c->winv), dp<double>(BIO), dp<double>(CII), s));
    HKG_HIP(hipStreamSynchronize(s));
    release(c, &Av);
    release(c, &Sv);
    release(c, &Dk);
    if (o->two_level) HKG_TRY(coarse_setup(c, p, BIO, CII, s, bad));
    if (o->local_prec == 32) HKG_TRY(local_inverses<float>(c, BIO, s, c->subs_d, bad));
    else HKG_TRY(local_inverses<double>(c, BIO, s, c->subs_d, bad));
    HKG_HIP(hipStreamSynchronize(s));
    return HKG_OK;
}

extern "C" int32_t hkgeneo_setup(const hkgeneo_problem *p, const hkgeneo_options *o, void *stream,
                                 hkgeneo_ctx **out) {
    if (!out) return HKG_EINVAL;
    *out = nullptr;
    int32_t st = check_problem(p, o);
    if (st != HKG_OK) {
        set_last_error("invalid problem or options");
        return st;
    }
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    hkgeneo_ctx *c = new hkgeneo_ctx();
    c->opt = *o;
    c->n_dof = p->n_dof;
    c->nnz = p->nnz;
    c->n_sub = p->n_sub;
    c->k = p->k;
    int32_t bad = -1;
    st = setup_body(c, p, o, s, &bad);
    if (st != HKG_OK) {
        if (st == HKG_EINVAL && hkg::g_last_error.empty())
            set_last_error("partition: invalid element/vertex data or a dof internal to no subdomain");
        (void)hipStreamSynchronize(s);
        hkgeneo_destroy(c);
        return st;
    }
    const auto t1 = std::chrono::steady_clock::now();
    c->stats.n_dof = c->n_dof;
    c->stats.n_sub = c->n_sub;
    c->stats.lambda_overlap = c->P.lambda_overlap;
    c->stats.m0 = c->m0;
    c->stats.sum_nI = (int32_t)c->sum_nI;
    c->stats.max_nI = c->max_nI;
    c->stats.max_nG = c->max_nG;
    c->stats.bad_sub = -1;
    c->stats.setup_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    *out = c;
    return HKG_OK;
}

// ------------------------------------------------------------------------------------------------
// apply / matvec / solve
// ------------------------------------------------------------------------------------------------
static int32_t ensure_apply_ws(hkgeneo_ctx *c, int nrhs) {
    if (c->ws_nrhs >= nrhs) return HKG_OK;
    HKG_TRY(alloc(c, &c->u, (size_t)c->sum_nI * nrhs * sizeof(double)));
    HKG_TRY(alloc(c, &c->c, (size_t)std::max(c->m0, 1) * nrhs * sizeof(double)));
    HKG_TRY(alloc(c, &c->y, (size_t)std::max(c->m0, 1) * nrhs * sizeof(double)));
    c->ws_nrhs = nrhs;
    return HKG_OK;
}

static ApplyPlan make_plan(hkgeneo_ctx *c, int nrhs) {
    ApplyPlan p{};
    p.nsub = c->n_sub;
    p.maxnI = c->max_nI;
    p.nrhs = nrhs;
    p.m0 = c->m0;
    p.two_level = c->opt.two_level;
    p.local_f32 = c->opt.local_prec == 32;
    p.n_dof = c->n_dof;
    p.max_m = c->max_m;
    p.d_sub = dp<SubDev>(c->subs_d);
    p.I_idx = dp<int32_t>(c->I_idx);
    p.winv_loc = dp<double>(c->wloc);
    p.Minv = c->Minv.p;
    p.Z = dp<double>(c->Z);
    p.B0inv = dp<double>(c->B0inv);
    p.tp_ptr = dp<int32_t>(c->tp_ptr);
    p.tp_pos = dp<int32_t>(c->tp_pos);
    p.u = dp<double>(c->u);
    p.c = dp<double>(c->c);
    p.y = dp<double>(c->y);
    p.sum_nI = c->sum_nI;
    return p;
}

extern "C" int32_t hkgeneo_apply(hkgeneo_ctx *c, const double *r, double *z, int32_t nrhs, int32_t ld, void *stream) {
    if (!c || !r || !z || nrhs < 1 || ld < c->n_dof) return HKG_EINVAL;
    HKG_TRY(ensure_apply_ws(c, nrhs));
    return apply_two_level(make_plan(c, nrhs), r, ld, z, ld, (hipStream_t)stream);
}

extern "C" int32_t hkgeneo_matvec(hkgeneo_ctx *c, const double *x, double *w, int32_t nrhs, int32_t ld, void *stream) {
    if (!c || !x || !w || nrhs < 1 || ld < c->n_dof) return HKG_EINVAL;
    return spmv(c->n_dof, nrhs, dp<int32_t>(c->rowptr), dp<int32_t>(c->colidx), dp<double>(c->Bval), x, ld, w, ld,
                nullptr, 0, (hipStream_t)stream);
}

static int32_t ensure_gmres_ws(hkgeneo_ctx *c, int nrhs) {
    if (c->gm_nrhs >= nrhs) return HKG_OK;
    const size_t n = c->n_dof, m = c->opt.restart;
    const int nblk = (int)((n + gmres_rows_per_block() - 1) / gmres_rows_per_block());
    HKG_TRY(alloc(c, &c->V, n * (m + 1) * nrhs * sizeof(double)));
    HKG_TRY(alloc(c, &c->Zk, n * m * nrhs * sizeof(double)));
    HKG_TRY(alloc(c, &c->H, (m + 1) * m * nrhs * sizeof(double)));
    HKG_TRY(alloc(c, &c->cs, m * nrhs * sizeof(double)));
    HKG_TRY(alloc(c, &c->sn, m * nrhs * sizeof(double)));
    HKG_TRY(alloc(c, &c->g, (m + 1) * nrhs * sizeof(double)));
    HKG_TRY(alloc(c, &c->part, (size_t)2 * nblk * (m + 2) * nrhs * sizeof(double)));
    HKG_TRY(alloc(c, &c->hcol, (m + 2) * nrhs * sizeof(double)));
    HKG_TRY(alloc(c, &c->scal, 8 * nrhs * sizeof(double)));
    HKG_TRY(alloc(c, &c->active, nrhs * sizeof(int32_t)));
    HKG_TRY(alloc(c, &c->want, nrhs * sizeof(int32_t)));
    HKG_TRY(alloc(c, &c->rnorm, nrhs * sizeof(double)));
    HKG_TRY(alloc(c, &c->fnorm, nrhs * sizeof(double)));
    HKG_TRY(alloc(c, &c->npart, (size_t)nblk * nrhs * sizeof(double)));
    c->gm_nrhs = nrhs;
    return HKG_OK;
}

extern "C" int32_t hkgeneo_gmres_solve(hkgeneo_ctx *c, const double *f, double *u, int32_t nrhs, int32_t ld,
                                       hkgeneo_rhs_info *info, void *stream) {
    if (!c || !f || !u || nrhs < 1 || ld < c->n_dof) return HKG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    HKG_TRY(ensure_apply_ws(c, nrhs));
    HKG_TRY(ensure_gmres_ws(c, nrhs));
    const int n = c->n_dof, m = c->opt.restart;
    const int nblk = (n + gmres_rows_per_block() - 1) / gmres_rows_per_block();
    GmresDev G{};
    G.n = n;
    G.nrhs = nrhs;
    G.restart = m;
    G.nblk = nblk;
    G.V = dp<double>(c->V);
    G.Zk = dp<double>(c->Zk);
    G.H = dp<double>(c->H);
    G.cs = dp<double>(c->cs);
    G.sn = dp<double>(c->sn);
    G.g = dp<double>(c->g);
    G.part = dp<double>(c->part);
    G.hcol = dp<double>(c->hcol);
    G.scal = dp<double>(c->scal);
    G.active = dp<int32_t>(c->active);
    const ApplyPlan plan = make_plan(c, nrhs);
    const int ldV = n * (m + 1), ldZ = n * m;
    const double rtol = c->opt.rtol;
    // x = 0, ||f||
    for (int r = 0; r < nrhs; ++r) HKG_HIP(hipMemsetAsync(u + (size_t)r * ld, 0, n * sizeof(double), s));
    HKG_HIP(hipMemsetAsync(c->V.p, 0, c->V.bytes, s));
    HKG_HIP(hipMemsetAsync(c->Zk.p, 0, c->Zk.bytes, s));
    HKG_HIP(hipMemsetAsync(c->scal.p, 0, c->scal.bytes, s));
    HKG_TRY(vec_norms(n, nrhs, f, ld, dp<double>(c->fnorm), dp<double>(c->npart), nblk, s));
    std::vector<double> fn(nrhs), rn(nrhs), sc((size_t)8 * nrhs);
    HKG_HIP(hipMemcpyAsync(fn.data(), c->fnorm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipStreamSynchronize(s));
    for (int r = 0; r < nrhs; ++r)
        HKG_HIP(hipMemcpyAsync(dp<double>(c->scal) + 8 * r + 1, &fn[r], sizeof(double), hipMemcpyHostToDevice, s));
    HKG_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> want(nrhs, 1), act(nrhs, 0), iters(nrhs, 0), conv(nrhs, 0);
    std::vector<double> est(nrhs, 0.0);
    for (int r = 0; r < nrhs; ++r)
        if (fn[r] == 0.0) { want[r] = 0; conv[r] = 1; }
    int total = 0;
    while (true) {
        // residual of the current iterate into V[:, 0], and its norm
        HKG_TRY(spmv(n, nrhs, dp<int32_t>(c->rowptr), dp<int32_t>(c->colidx), dp<double>(c->Bval), u, ld, G.V, ldV, f, ld,
                     s));
        HKG_TRY(vec_norms(n, nrhs, G.V, ldV, dp<double>(c->rnorm), dp<double>(c->npart), nblk, s));
        HKG_HIP(hipMemcpyAsync(rn.data(), c->rnorm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
        HKG_HIP(hipStreamSynchronize(s));
        bool any = false;
        for (int r = 0; r < nrhs; ++r) {
            if (!want[r]) continue;
            if (rn[r] <= rtol * fn[r]) { want[r] = 0; conv[r] = 1; continue; }
            if (iters[r] >= c->opt.max_iter) { want[r] = 0; continue; }
            any = true;
        }
        if (!any) break;
        HKG_HIP(hipMemcpyAsync(c->want.p, want.data(), nrhs * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HKG_TRY(gmres_cycle_start(G, dp<double>(c->rnorm), rtol, dp<int32_t>(c->want), s));
        for (int r = 0; r < nrhs; ++r) act[r] = want[r];
        int jrun = 0;
        for (int j = 0; j < m; ++j) {
            HKG_TRY(apply_two_level(plan, G.V + (size_t)j * n, ldV, G.Zk + (size_t)j * n, ldZ, s));
            HKG_TRY(spmv(n, nrhs, dp<int32_t>(c->rowptr), dp<int32_t>(c->colidx), dp<double>(c->Bval),
                         G.Zk + (size_t)j * n, ldZ, G.V + (size_t)(j + 1) * n, ldV, nullptr, 0, s));
            HKG_TRY(gmres_arnoldi_step(G, j, rtol, s));
            for (int r = 0; r < nrhs; ++r) iters[r] += act[r];
            jrun = j + 1;
            HKG_HIP(hipMemcpyAsync(act.data(), c->active.p, nrhs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HKG_HIP(hipStreamSynchronize(s));
            bool still = false, capped = false;
            for (int r = 0; r < nrhs; ++r) {
                if (act[r] && iters[r] >= c->opt.max_iter) { act[r] = 0; capped = true; }
                still = still || act[r];
            }
            if (!still || capped) break;
        }
        // a right-hand side stopped by max_iter while still active keeps every column built so far
        HKG_HIP(hipMemcpyAsync(sc.data(), c->scal.p, sc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HKG_HIP(hipStreamSynchronize(s));
        bool patched = false;
        for (int r = 0; r < nrhs; ++r)
            if (want[r] && sc[8 * r + 3] == 0.0) {
                sc[8 * r + 3] = (double)jrun;
                patched = true;
            }
        if (patched)
            HKG_HIP(hipMemcpyAsync(c->scal.p, sc.data(), sc.size() * sizeof(double), hipMemcpyHostToDevice, s));
        for (int r = 0; r < nrhs; ++r)
            if (want[r]) est[r] = sc[8 * r + 2] / (fn[r] > 0 ? fn[r] : 1.0);
        HKG_TRY(gmres_cycle_update(G, u, ld, s));
    }
    // true residuals
    HKG_TRY(spmv(n, nrhs, dp<int32_t>(c->rowptr), dp<int32_t>(c->colidx), dp<double>(c->Bval), u, ld, G.V, ldV, f, ld, s));
    HKG_TRY(vec_norms(n, nrhs, G.V, ldV, dp<double>(c->rnorm), dp<double>(c->npart), nblk, s));
    HKG_HIP(hipMemcpyAsync(rn.data(), c->rnorm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipStreamSynchronize(s));
    int32_t status = HKG_OK;
    for (int r = 0; r < nrhs; ++r) {
        double rel = fn[r] > 0 ? rn[r] / fn[r] : 0.0;
        int ok = rel <= rtol;
        if (!ok) status = HKG_ENOTCONV;
        if (info) {
            info[r].iters = iters[r];
            info[r].converged = ok;
            info[r].relres_est = est[r];
            info[r].relres_true = rel;
        }
    }
    (void)total;
    return status;
}

// ------------------------------------------------------------------------------------------------
// queries
// ------------------------------------------------------------------------------------------------
extern "C" int32_t hkgeneo_query(const hkgeneo_ctx *c, hkgeneo_stats *out) {
    if (!c || !out) return HKG_EINVAL;
    *out = c->stats;
    out->device_bytes = c->device_bytes;
    return HKG_OK;
}

extern "C" int32_t hkgeneo_query_subdomains(const hkgeneo_ctx *c, int32_t *nI, int32_t *nG, int32_t *m) {
    if (!c) return HKG_EINVAL;
    for (int i = 0; i < c->n_sub; ++i) {
        if (nI) nI[i] = c->subs[i].nI;
        if (nG) nG[i] = c->subs[i].nG;
        if (m) m[i] = c->subs[i].m;
    }
    return HKG_OK;
}

extern "C" int32_t hkgeneo_query_index_sets(const hkgeneo_ctx *c, int32_t sub, int32_t *dof, int32_t *gamma,
                                            int32_t *mu) {
    if (!c || sub < 0 || sub >= c->n_sub) return HKG_EINVAL;
    const Partition &P = c->P;
    if (dof) std::memcpy(dof, &P.I_idx[P.offI[sub]], P.nI[sub] * sizeof(int32_t));
    if (gamma && P.nG[sub]) std::memcpy(gamma, &P.G_idx[P.offG[sub]], P.nG[sub] * sizeof(int32_t));
    if (mu && sub == 0) std::memcpy(mu, P.mu.data(), P.mu.size() * sizeof(int32_t));
    return HKG_OK;
}

extern "C" int32_t hkgeneo_query_eigen(const hkgeneo_ctx *c, int32_t sub, double *lambda, int32_t count, double *Z) {
    if (!c || sub < 0 || sub >= c->n_sub) return HKG_EINVAL;
    if (!c->opt.two_level) return HKG_EINVAL;
    const SubDev &sd = c->subs[sub];
    const int avail = std::min(sd.nI, sd.m + 1);
    if (lambda) {
        if (count < 0 || count > avail) return HKG_EINVAL;
        std::memcpy(lambda, &c->lam_host[(size_t)sub * (c->opt.max_eig_per_sub + 2)], count * sizeof(double));
    }
    if (Z && sd.m > 0) {
        HKG_HIP(hipMemcpy(Z, dp<double>(c->Z) + sd.offZ, (size_t)sd.nI * sd.m * sizeof(double), hipMemcpyDeviceToHost));
    }
    return HKG_OK;
}

extern "C" int32_t hkgeneo_query_coarse_matrix(const hkgeneo_ctx *c, double *B0) {
    if (!c || !B0) return HKG_EINVAL;
    if (c->B0_host.size() != (size_t)c->m0 * c->m0) return HKG_EINVAL;
    std::memcpy(B0, c->B0_host.data(), c->B0_host.size() * sizeof(double));
    return HKG_OK;
}

extern "C" int32_t hkgeneo_partition(const hkgeneo_problem *p, int32_t *nI, int32_t *nG, int32_t *dof, int32_t *gamma,
                                     int32_t *mu, int32_t *lambda_overlap) {
    if (!p || !p->elem_vert || !p->vert_dof || !p->elem_part || !p->overlap) return HKG_EINVAL;
    if (!(p->dim == 2 || p->dim == 3) || !(p->elem_type == HKG_P1 || p->elem_type == HKG_Q1)) return HKG_EINVAL;
    if (p->n_vert <= 0 || p->n_elem <= 0 || p->n_dof <= 0 || p->n_sub <= 0) return HKG_EINVAL;
    Partition P;
    int bad = -1;
    int32_t st = build_partition(p, &P, &bad);
    if (st != HKG_OK) return st;
    for (int i = 0; i < P.n_sub; ++i) {
        if (nI) nI[i] = P.nI[i];
        if (nG) nG[i] = P.nG[i];
    }
    if (dof) std::memcpy(dof, P.I_idx.data(), P.I_idx.size() * sizeof(int32_t));
    if (gamma && !P.G_idx.empty()) std::memcpy(gamma, P.G_idx.data(), P.G_idx.size() * sizeof(int32_t));
    if (mu) std::memcpy(mu, P.mu.data(), P.mu.size() * sizeof(int32_t));
    if (lambda_overlap) *lambda_overlap = P.lambda_overlap;
    return HKG_OK;
}
