// C ABI of libhkgeneo: the two-level Schwarz preconditioner with the H_k-GenEO coarse space, its
// application, and right-preconditioned flexible GMRES on one HIP device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ctx.hpp"

namespace hkg {
thread_local std::string g_last_error;
void set_last_error(const std::string &msg) { g_last_error = msg; }

// declared in krylov.hip
int32_t gmres_arnoldi_step(const GmresDev &G, int j, double rtol, hipStream_t s, const int32_t *rowptr = nullptr,
                           const int32_t *colidx = nullptr, const double *Aval = nullptr, const double *Sval = nullptr,
                           double k2 = 0.0);
int32_t gmres_cycle_start(const GmresDev &G, const double *rnorm, double rtol, const int32_t *want, hipStream_t s);
int32_t gmres_cycle_update(const GmresDev &G, double *x, int ldx, hipStream_t s);
int gmres_rows_per_block();
}  // namespace hkg

using namespace hkg;

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
    o->keep_workspace = 0;
    o->local_factor_prec = 64;
    o->krylov = HKG_KRYLOV_RIGHT;
    o->coarse_op = HKG_COARSE_HK;
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

extern "C" void hkgeneo_destroy(hkgeneo_ctx *c) {
    if (!c) return;
    if (c->fine) hkgeneo_destroy(c->fine);
    c->fine = nullptr;
    DevBuf *bufs[] = {&c->rowptr, &c->colidx, &c->Aval,    &c->Sval,   &c->I_idx,   &c->G_idx,      &c->winv,
                      &c->wloc,   &c->tp_ptr, &c->tp_pos,  &c->tp_sub, &c->subs_d, &c->bandK,   &c->bandM,      &c->bandLoc,
                      &c->pairs,  &c->matsGG, &c->matsSq,  &c->poffSub, &c->jobsGI, &c->jobsSq, &c->jobsSqM, &c->gjobsSchur,
                      &c->matsLoc, &c->poffLoc, &c->jobsLoc, &c->matsM, &c->jobsM, &c->jobsGGinv, &c->gjobsGX, &c->Bval, &c->Minv,    &c->Z, &c->Zr,  &c->tpZ, &c->B0inv, &c->B0copy,
                      &c->u,      &c->c,      &c->y,       &c->ypart, &c->itersd,       &c->V,      &c->Zk,      &c->H,          &c->cs,
                      &c->sn,     &c->g,      &c->part,    &c->hcol,   &c->scal,    &c->active,     &c->want,
                      &c->rnorm,  &c->npart,  &c->fnorm, &c->DV};
    if (c->s2) (void)hipStreamSynchronize(c->s2);
    if (c->s3) (void)hipStreamSynchronize(c->s3);
    for (DevBuf *b : bufs) drelease(c, b);
    free_workspace(c);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->h_infoL) (void)hipHostFree(c->h_infoL);
    if (c->h_stage) (void)hipHostFree(c->h_stage);
    if (c->h_read) (void)hipHostFree(c->h_read);
    if (c->ev_fork3) (void)hipEventDestroy(c->ev_fork3);
    if (c->ev_join3) (void)hipEventDestroy(c->ev_join3);
    for (hipEvent_t e : c->ev_dc)
        if (e) (void)hipEventDestroy(e);
    if (c->s2) (void)hipStreamDestroy(c->s2);
    if (c->s3) (void)hipStreamDestroy(c->s3);
    delete c;
}

namespace {

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
    if (p->fine_part) {
        if (p->fine_overlap < 0) return HKG_EINVAL;
        for (int e = 0; e < p->n_elem; ++e)
            if (p->fine_part[e] < 0) return HKG_EINVAL;
    }
    if (!(o->eig_mode == HKG_EIG_FIXED || o->eig_mode == HKG_EIG_THRESHOLD)) return HKG_EINVAL;
    if (o->nev < 0 || o->max_eig_per_sub < 1 || o->max_eig_per_sub > 64 || !(o->cluster_rtol >= 0.0))
        return HKG_EINVAL;
    if (!(o->local_prec == 64 || o->local_prec == 32)) return HKG_EINVAL;
    // float32 factorisation of B_D is not offered: near a local resonance its O(cond(B_D) eps_32)
    // error costs FGMRES iterations (36 against 28 at h = 1/32, k = 10), so the float32 local
    // operators are always formed in float64 and rounded once
    if (o->local_factor_prec != 64) return HKG_EINVAL;
    if (!(o->prolong == HKG_PROLONG_AS || o->prolong == HKG_PROLONG_POU)) return HKG_EINVAL;
    if (!(o->krylov == HKG_KRYLOV_RIGHT || o->krylov == HKG_KRYLOV_LEFT_DK)) return HKG_EINVAL;
    if (!(o->coarse_op == HKG_COARSE_HK || o->coarse_op == HKG_COARSE_DELTA)) return HKG_EINVAL;
    if (o->restart < 1 || o->max_iter < 1 || !(o->rtol > 0.0)) return HKG_EINVAL;
    return HKG_OK;
}

}  // namespace

extern "C" int32_t hkgeneo_setup(const hkgeneo_problem *p, const hkgeneo_options *o, void *stream,
                                 hkgeneo_ctx **out) {
    if (!out) return HKG_EINVAL;
    *out = nullptr;
    g_last_error.clear();
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
    c->dim = p->dim;
    int32_t bad = -1;
    c->coarse_only = p->fine_part != nullptr;
    st = analyze(c, p, s, &bad);
    if (st == HKG_EINVAL && g_last_error.empty())
        set_last_error("partition: invalid element/vertex data or a dof internal to no subdomain");
    if (st == HKG_OK && p->fine_part) {
        // nested decomposition (Sec. 2.3): the first-level subdomains inside the coarse ones, in a
        // one-level context of their own that holds the local inverses
        std::vector<std::vector<int32_t>> sets;
        st = build_nested_sets(p, c->P, p->fine_overlap, &sets, &c->fine_owner);
        if (st == HKG_OK) {
            hkgeneo_ctx *f = new hkgeneo_ctx();
            f->opt = *o;
            f->opt.two_level = 0;
            f->n_dof = p->n_dof;
            f->nnz = p->nnz;
            f->k = p->k;
            f->dim = p->dim;
            c->fine = f;
            st = analyze(f, p, s, &bad, &sets);
            if (st == HKG_EINVAL && g_last_error.empty())
                set_last_error("nested partition: a dof internal to no first-level subdomain");
            if (st == HKG_OK) st = factor(f, s);
            if (st == HKG_OK && !f->opt.keep_workspace) free_workspace(f);
        }
    }
    if (st == HKG_OK) st = factor(c, s);
    if (st != HKG_OK) {
        (void)hipStreamSynchronize(s);
        hkgeneo_destroy(c);
        return st;
    }
    if (!c->opt.keep_workspace) free_workspace(c);
    const auto t1 = std::chrono::steady_clock::now();
    c->stats.n_dof = c->n_dof;
    c->stats.n_sub = c->n_sub;
    c->stats.lambda_overlap = c->fine ? c->fine->P.lambda_overlap : c->P.lambda_overlap;
    c->stats.m0 = c->m0;
    c->stats.sum_nI = (int32_t)c->sum_nI;
    c->stats.max_nI = c->max_nI;
    c->stats.max_nG = c->max_nG;
    c->stats.bad_sub = -1;
    c->stats.setup_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    *out = c;
    return HKG_OK;
}

extern "C" int32_t hkgeneo_factor(hkgeneo_ctx *c, void *stream) {
    if (!c) return HKG_EINVAL;
    g_last_error.clear();
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    int32_t st = HKG_OK;
    if (c->fine) {
        st = factor(c->fine, s);
        if (!c->fine->opt.keep_workspace) free_workspace(c->fine);
        c->fine->ws_nrhs = 0;
    }
    if (st == HKG_OK) st = factor(c, s);
    if (!c->opt.keep_workspace) free_workspace(c);
    c->ws_nrhs = 0;                       // the coarse dimension may have changed
    if (st != HKG_OK) return st;
    c->stats.m0 = c->m0;
    c->stats.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return HKG_OK;
}

// ------------------------------------------------------------------------------------------------
// apply / matvec / solve
// ------------------------------------------------------------------------------------------------
static int32_t ensure_apply_ws(hkgeneo_ctx *c, int nrhs) {
    if (c->ws_nrhs >= nrhs) return HKG_OK;
    HKG_TRY(dalloc(c, &c->u, (size_t)c->sum_nI * nrhs * sizeof(double)));
    HKG_TRY(dalloc(c, &c->c, (size_t)std::max(c->m0, 1) * nrhs * sizeof(double)));
    HKG_TRY(dalloc(c, &c->y, (size_t)std::max(c->m0, 1) * nrhs * sizeof(double)));
    HKG_TRY(dalloc(c, &c->ypart, (size_t)std::max(c->m0, 1) * apply_ypart_chunks(std::max(c->m0, 1)) * nrhs *
                                     sizeof(double)));
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
    p.Zr = dp<double>(c->Zr);
    p.B0inv = dp<double>(c->B0inv);
    p.tp_ptr = dp<int32_t>(c->tp_ptr);
    p.tp_pos = dp<int32_t>(c->tp_pos);
    p.tp_sub = dp<int32_t>(c->tp_sub);
    p.ypart = dp<double>(c->ypart);
    p.u = dp<double>(c->u);
    p.c = dp<double>(c->c);
    p.y = dp<double>(c->y);
    p.sum_nI = c->sum_nI;
    return p;
}

// one application, with the local-solve kernel bracketed by events when the measurement hook is on
static int32_t apply_once(hkgeneo_ctx *c, const ApplyPlan &plan, const double *r, int ldr, double *z, int ldz,
                          hipStream_t s) {
    ApplyPlan p = plan;
    if (c->prof) {
        if (c->ev_used + 2 > c->ev.size()) {
            for (int k = 0; k < 256; ++k) {
                hipEvent_t e;
                HKG_HIP(hipEventCreate(&e));
                c->ev.push_back(e);
            }
        }
        p.ev0 = c->ev[c->ev_used];
        p.ev1 = c->ev[c->ev_used + 1];
        c->ev_used += 2;
    }
    return apply_two_level(p, r, ldr, z, ldz, s);
}

// z = M^{-1} r.  For a nested decomposition (Sec. 2.3) the first-level solves come from the fine
// context, then the coarse correction of this (coarse-only) context is added: the same sum
// sum_{i,j} E_{i,j}^f (B_{i,j}^f)^{-1} R_{i,j}^f r + E_0 B_0^{-1} R_0 r of eqs. (2.22), (2.23).
struct Precond {
    ApplyPlan plan, fine;
};

static int32_t precond_plan(hkgeneo_ctx *c, int nrhs, const int32_t *active, Precond *P) {
    HKG_TRY(ensure_apply_ws(c, nrhs));
    P->plan = make_plan(c, nrhs);
    P->plan.active = active;
    if (c->fine) {
        HKG_TRY(ensure_apply_ws(c->fine, nrhs));
        P->fine = make_plan(c->fine, nrhs);
        P->fine.active = active;
        P->plan.Minv = nullptr;          // the coarse correction alone ...
        P->plan.accumulate = 1;          // ... added to the first-level solves
    }
    return HKG_OK;
}

static int32_t precond_apply(hkgeneo_ctx *c, const Precond &P, const double *r, int ldr, double *z, int ldz,
                             hipStream_t s) {
    if (c->fine) {
        HKG_TRY(apply_two_level(P.fine, r, ldr, z, ldz, s));
        return apply_two_level(P.plan, r, ldr, z, ldz, s);
    }
    return apply_once(c, P.plan, r, ldr, z, ldz, s);
}

extern "C" int32_t hkgeneo_apply(hkgeneo_ctx *c, const double *r, double *z, int32_t nrhs, int32_t ld, void *stream) {
    if (!c || !r || !z || nrhs < 1 || ld < c->n_dof) return HKG_EINVAL;
    Precond P;
    HKG_TRY(precond_plan(c, nrhs, nullptr, &P));
    return precond_apply(c, P, r, ld, z, ld, (hipStream_t)stream);
}

// ------------------------------------------------------------------------------------------------
// allocation-free application: the temporaries of hkgeneo_apply (local vectors, coarse restriction,
// partial sums of the coarse product) live in one fixed device array per GPU instead of the
// context's lazily allocated workspace
// ------------------------------------------------------------------------------------------------
namespace {
constexpr size_t kScratchDoubles = HKG_APPLY_NOALLOC_MAX_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};    // device address of `scratch` on each GPU, once looked up

// the address of this GPU's copy of `scratch` (looked up once per device, with that device current;
// the array's name in host code is not a device address)
int32_t scratch_on_current_device(double **out) {
    int dev = -1;
    HKG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_last_error("device ordinal out of range for the allocation-free scratch table");
        return HKG_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HKG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return HKG_OK;
}
}  // namespace

extern "C" int32_t hkgeneo_apply_noalloc(hkgeneo_ctx *c, const double *r, double *z, int32_t nrhs, int32_t ld,
                                         void *stream) {
    if (!c || !r || !z || nrhs < 1 || ld < c->n_dof) return HKG_EINVAL;
    if (c->fine) {
        set_last_error("hkgeneo_apply_noalloc: nested contexts use hkgeneo_apply");
        return HKG_EINVAL;
    }
    const int64_t m0 = std::max(c->m0, 1);
    const int64_t chunks = apply_ypart_chunks((int)m0);
    // u (sum n_I x nrhs), c (m0 x nrhs), ypart (chunks x m0 x nrhs), each at a 256-byte boundary
    auto round = [](int64_t d) { return (d + 31) / 32 * 32; };
    const int64_t nu = round(c->sum_nI * nrhs), nc = round(m0 * nrhs), np = round(chunks * m0 * nrhs);
    if ((uint64_t)(nu + nc + np) > (uint64_t)kScratchDoubles) {
        set_last_error("hkgeneo_apply_noalloc: " + std::to_string(8 * (nu + nc + np)) +
                       " bytes of temporaries exceed HKG_APPLY_NOALLOC_MAX_BYTES");
        return HKG_EINVAL;
    }
    double *base = nullptr;
    HKG_TRY(scratch_on_current_device(&base));
    ApplyPlan p = make_plan(c, nrhs);
    p.u = base;
    p.c = base + nu;
    p.y = nullptr;
    p.ypart = base + nu + nc;
    return apply_two_level(p, r, ld, z, ld, (hipStream_t)stream);
}

extern "C" int32_t hkgeneo_matvec(hkgeneo_ctx *c, const double *x, double *w, int32_t nrhs, int32_t ld, void *stream) {
    if (!c || !x || !w || nrhs < 1 || ld < c->n_dof) return HKG_EINVAL;
    return spmv(c->n_dof, nrhs, dp<int32_t>(c->rowptr), dp<int32_t>(c->colidx), dp<double>(c->Bval), x, ld, w, ld,
                nullptr, 0, (hipStream_t)stream);
}

extern "C" int32_t hkgeneo_profile(hkgeneo_ctx *c, int32_t enable) {
    if (!c) return HKG_EINVAL;
    c->prof = enable != 0;
    c->ev_used = 0;
    return HKG_OK;
}

extern "C" int32_t hkgeneo_profile_read(hkgeneo_ctx *c, double *total_ms, int64_t *launches) {
    if (!c) return HKG_EINVAL;
    double t = 0.0;
    for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
        HKG_HIP(hipEventSynchronize(c->ev[k + 1]));
        float ms = 0.0f;
        HKG_HIP(hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]));
        t += ms;
    }
    if (total_ms) *total_ms = t;
    if (launches) *launches = (int64_t)(c->ev_used / 2);
    return HKG_OK;
}

static int32_t ensure_gmres_ws(hkgeneo_ctx *c, int nrhs) {
    if (c->gm_nrhs >= nrhs) return HKG_OK;
    const size_t n = c->n_dof, m = c->opt.restart;
    const int nblk = (int)((n + gmres_rows_per_block() - 1) / gmres_rows_per_block());
    HKG_TRY(dalloc(c, &c->V, n * (m + 1) * nrhs * sizeof(double)));
    HKG_TRY(dalloc(c, &c->Zk, n * m * nrhs * sizeof(double)));
    HKG_TRY(dalloc(c, &c->H, (m + 1) * m * nrhs * sizeof(double)));
    HKG_TRY(dalloc(c, &c->cs, m * nrhs * sizeof(double)));
    HKG_TRY(dalloc(c, &c->sn, m * nrhs * sizeof(double)));
    HKG_TRY(dalloc(c, &c->g, (m + 1) * nrhs * sizeof(double)));
    HKG_TRY(dalloc(c, &c->part, (size_t)2 * nblk * (m + 2) * nrhs * sizeof(double)));
    HKG_TRY(dalloc(c, &c->hcol, (m + 2) * nrhs * sizeof(double)));
    HKG_TRY(dalloc(c, &c->scal, 8 * nrhs * sizeof(double)));
    HKG_TRY(dalloc(c, &c->active, nrhs * sizeof(int32_t)));
    HKG_TRY(dalloc(c, &c->want, nrhs * sizeof(int32_t)));
    HKG_TRY(dalloc(c, &c->rnorm, nrhs * sizeof(double)));
    HKG_TRY(dalloc(c, &c->fnorm, nrhs * sizeof(double)));
    HKG_TRY(dalloc(c, &c->npart, (size_t)nblk * nrhs * sizeof(double)));
    HKG_TRY(dalloc(c, &c->itersd, nrhs * sizeof(int32_t)));
    c->gm_nrhs = nrhs;
    return HKG_OK;
}

// GMRES(restart) on the left-preconditioned system M^{-1} B u = M^{-1} f (eq. 2.24) in the D_k inner
// product (Theorem 3.1): r = M^{-1}(f - B x), beta = ||r||_{D_k}; Arnoldi vectors w = M^{-1} B v_j
// orthogonalised by CGS2 against D_k V (kept beside V); x += V y at the cycle end.  Stops when
// ||M^{-1}(f - B x)||_{D_k} <= rtol ||M^{-1} f||_{D_k}; info also carries the Euclidean true residual.
static int32_t gmres_solve_dk(hkgeneo_ctx *c, const double *f, double *u, int nrhs, int ld, hkgeneo_rhs_info *info,
                              hipStream_t s) {
    HKG_TRY(ensure_apply_ws(c, nrhs));
    HKG_TRY(ensure_gmres_ws(c, nrhs));
    const int n = c->n_dof, m = c->opt.restart;
    const int nblk = (n + gmres_rows_per_block() - 1) / gmres_rows_per_block();
    if (c->DV.bytes != c->V.bytes) HKG_TRY(dalloc(c, &c->DV, c->V.bytes));
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
    G.iters = dp<int32_t>(c->itersd);
    G.max_iter = c->opt.max_iter;
    G.DV = dp<double>(c->DV);
    G.VD = G.DV;
    G.dk = 1;
    const int32_t *rp = dp<int32_t>(c->rowptr), *ci = dp<int32_t>(c->colidx);
    const double *Av = dp<double>(c->Aval), *Sv = dp<double>(c->Sval), *Bv = dp<double>(c->Bval);
    const double k2 = c->k * c->k;
    Precond plan, plan0;
    HKG_TRY(precond_plan(c, nrhs, G.active, &plan));                   // the iteration: columns in their cycle
    HKG_TRY(precond_plan(c, nrhs, dp<int32_t>(c->want), &plan0));      // the cycle start: columns that iterate
    const int ldV = n * (m + 1), ldZ = n * m;
    const double rtol = c->opt.rtol;
    for (int r = 0; r < nrhs; ++r) HKG_HIP(hipMemsetAsync(u + (size_t)r * ld, 0, n * sizeof(double), s));
    HKG_HIP(hipMemsetAsync(c->V.p, 0, c->V.bytes, s));
    HKG_HIP(hipMemsetAsync(c->DV.p, 0, c->DV.bytes, s));
    HKG_HIP(hipMemsetAsync(c->Zk.p, 0, c->Zk.bytes, s));
    HKG_HIP(hipMemsetAsync(c->scal.p, 0, c->scal.bytes, s));
    HKG_HIP(hipMemsetAsync(c->itersd.p, 0, c->itersd.bytes, s));
    HKG_TRY(vec_norms(n, nrhs, f, ld, dp<double>(c->fnorm), dp<double>(c->npart), nblk, s));
    std::vector<double> fe(nrhs), rn(nrhs), ref(nrhs, 0.0), sc((size_t)8 * nrhs);
    HKG_HIP(hipMemcpyAsync(fe.data(), c->fnorm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> want(nrhs, 1), act(nrhs, 0), iters(nrhs, 0);
    std::vector<double> est(nrhs, 0.0);
    for (int r = 0; r < nrhs; ++r)
        if (!(fe[r] > 0.0)) want[r] = 0;         // zero (u = 0) or non-finite right-hand side
    bool first = true;
    const int check = c->prof ? 1 : 4;
    while (true) {
        HKG_HIP(hipMemcpyAsync(c->want.p, want.data(), nrhs * sizeof(int32_t), hipMemcpyHostToDevice, s));
        // r = M^{-1}(f - B x) into V[:, 0] (f - B x staged in Zk[:, 0]), beta = ||r||_{D_k}
        HKG_TRY(spmv(n, nrhs, rp, ci, Bv, u, ld, G.Zk, ldZ, f, ld, s));
        HKG_TRY(precond_apply(c, plan0, G.Zk, ldZ, G.V, ldV, s));
        HKG_TRY(gmres_dk_norm(G, -1, rp, ci, Av, Sv, k2, s));
        HKG_TRY(gmres_dk_reduce(G, dp<double>(c->rnorm), s));
        HKG_HIP(hipMemcpyAsync(rn.data(), c->rnorm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
        HKG_HIP(hipMemcpyAsync(iters.data(), c->itersd.p, nrhs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HKG_HIP(hipStreamSynchronize(s));
        if (first) {
            // the reference norm ||M^{-1} f||_{D_k} (x = 0 on the first pass)
            for (int r = 0; r < nrhs; ++r) {
                ref[r] = want[r] ? rn[r] : 0.0;
                sc[8 * r + 1] = ref[r];
                HKG_HIP(hipMemcpyAsync(dp<double>(c->scal) + 8 * r + 1, &ref[r], sizeof(double), hipMemcpyHostToDevice,
                                       s));
            }
            HKG_HIP(hipStreamSynchronize(s));
            first = false;
        }
        bool any = false;
        for (int r = 0; r < nrhs; ++r) {
            if (!want[r]) continue;
            est[r] = ref[r] > 0 ? rn[r] / ref[r] : 0.0;
            if (!gmres_keeps_going(rn[r], ref[r], rtol) || iters[r] >= c->opt.max_iter) {
                want[r] = 0;
                continue;
            }
            any = true;
        }
        if (!any) break;
        HKG_HIP(hipMemcpyAsync(c->want.p, want.data(), nrhs * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HKG_TRY(gmres_cycle_start(G, dp<double>(c->rnorm), rtol, dp<int32_t>(c->want), s));
        for (int j = 0; j < m; ++j) {
            // w = M^{-1} B v_j into V[:, j+1] (B v_j staged in Zk[:, j])
            HKG_TRY(spmv(n, nrhs, rp, ci, Bv, G.V + (size_t)j * n, ldV, G.Zk + (size_t)j * n, ldZ, nullptr, 0, s,
                         G.active));
            HKG_TRY(precond_apply(c, plan, G.Zk + (size_t)j * n, ldZ, G.V + (size_t)(j + 1) * n, ldV, s));
            HKG_TRY(gmres_arnoldi_step(G, j, rtol, s, rp, ci, Av, Sv, k2));
            if ((j + 1) % check == 0 || j + 1 == m) {
                HKG_HIP(hipMemcpyAsync(act.data(), c->active.p, nrhs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
                HKG_HIP(hipStreamSynchronize(s));
                bool still = false;
                for (int r = 0; r < nrhs; ++r) still = still || act[r];
                if (!still) break;
            }
        }
        HKG_HIP(hipMemcpyAsync(sc.data(), c->scal.p, sc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HKG_HIP(hipStreamSynchronize(s));
        for (int r = 0; r < nrhs; ++r)
            if (want[r] && sc[8 * r + 5] != 0.0) want[r] = 0;    // singular Hessenberg column
        HKG_TRY(gmres_cycle_update(G, u, ld, s));
    }
    // Euclidean true residuals
    HKG_TRY(spmv(n, nrhs, rp, ci, Bv, u, ld, G.V, ldV, f, ld, s));
    HKG_TRY(vec_norms(n, nrhs, G.V, ldV, dp<double>(c->rnorm), dp<double>(c->npart), nblk, s));
    std::vector<double> rt(nrhs);
    HKG_HIP(hipMemcpyAsync(rt.data(), c->rnorm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipMemcpyAsync(iters.data(), c->itersd.p, nrhs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipStreamSynchronize(s));
    int32_t status = HKG_OK;
    for (int r = 0; r < nrhs; ++r) {
        const bool zero = fe[r] == 0.0;
        const int ok = zero || (est[r] <= rtol && std::isfinite(rt[r]));      // false for NaN
        if (!ok) status = HKG_ENOTCONV;
        if (info) {
            info[r].iters = iters[r];
            info[r].converged = ok;
            info[r].relres_est = zero ? 0.0 : est[r];
            info[r].relres_true = gmres_relres(rt[r], fe[r]);
        }
    }
    return status;
}

extern "C" int32_t hkgeneo_gmres_solve(hkgeneo_ctx *c, const double *f, double *u, int32_t nrhs, int32_t ld,
                                       hkgeneo_rhs_info *info, void *stream) {
    if (!c || !f || !u || nrhs < 1 || ld < c->n_dof) return HKG_EINVAL;
    if (c->opt.krylov == HKG_KRYLOV_LEFT_DK) return gmres_solve_dk(c, f, u, nrhs, ld, info, (hipStream_t)stream);
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
    G.iters = dp<int32_t>(c->itersd);
    G.max_iter = c->opt.max_iter;
    G.VD = G.V;
    Precond plan;
    HKG_TRY(precond_plan(c, nrhs, G.active, &plan));
    const int ldV = n * (m + 1), ldZ = n * m;
    const double rtol = c->opt.rtol;
    // x = 0, ||f||
    for (int r = 0; r < nrhs; ++r) HKG_HIP(hipMemsetAsync(u + (size_t)r * ld, 0, n * sizeof(double), s));
    HKG_HIP(hipMemsetAsync(c->V.p, 0, c->V.bytes, s));
    HKG_HIP(hipMemsetAsync(c->Zk.p, 0, c->Zk.bytes, s));
    HKG_HIP(hipMemsetAsync(c->scal.p, 0, c->scal.bytes, s));
    HKG_HIP(hipMemsetAsync(c->itersd.p, 0, c->itersd.bytes, s));
    HKG_TRY(vec_norms(n, nrhs, f, ld, dp<double>(c->fnorm), dp<double>(c->npart), nblk, s));
    std::vector<double> fn(nrhs), rn(nrhs), sc((size_t)8 * nrhs);
    HKG_HIP(hipMemcpyAsync(fn.data(), c->fnorm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipStreamSynchronize(s));
    for (int r = 0; r < nrhs; ++r)
        HKG_HIP(hipMemcpyAsync(dp<double>(c->scal) + 8 * r + 1, &fn[r], sizeof(double), hipMemcpyHostToDevice, s));
    HKG_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> want(nrhs, 1), act(nrhs, 0), iters(nrhs, 0);
    std::vector<double> est(nrhs, 0.0);
    for (int r = 0; r < nrhs; ++r)
        if (fn[r] == 0.0) want[r] = 0;
    // the host looks at the active flags every `check` iterations; iterations issued after every
    // column has stopped return at once
    const int check = c->prof ? 1 : 4;   // timed runs never issue no-op launches
    while (true) {
        // residual of the current iterate into V[:, 0], and its norm
        HKG_TRY(spmv(n, nrhs, dp<int32_t>(c->rowptr), dp<int32_t>(c->colidx), dp<double>(c->Bval), u, ld, G.V, ldV, f, ld,
                     s));
        HKG_TRY(vec_norms(n, nrhs, G.V, ldV, dp<double>(c->rnorm), dp<double>(c->npart), nblk, s));
        HKG_HIP(hipMemcpyAsync(rn.data(), c->rnorm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
        HKG_HIP(hipMemcpyAsync(iters.data(), c->itersd.p, nrhs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HKG_HIP(hipStreamSynchronize(s));
        bool any = false;
        for (int r = 0; r < nrhs; ++r) {
            if (!want[r]) continue;
            // the same predicate as the device's cycle start (k_cycle_start): a NaN or infinite
            // residual stops the column, which then reports non-convergence
            if (!gmres_keeps_going(rn[r], fn[r], rtol) || iters[r] >= c->opt.max_iter) { want[r] = 0; continue; }
            any = true;
        }
        if (!any) break;
        HKG_HIP(hipMemcpyAsync(c->want.p, want.data(), nrhs * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HKG_TRY(gmres_cycle_start(G, dp<double>(c->rnorm), rtol, dp<int32_t>(c->want), s));
        for (int j = 0; j < m; ++j) {
            HKG_TRY(precond_apply(c, plan, G.V + (size_t)j * n, ldV, G.Zk + (size_t)j * n, ldZ, s));
            HKG_TRY(spmv(n, nrhs, dp<int32_t>(c->rowptr), dp<int32_t>(c->colidx), dp<double>(c->Bval),
                         G.Zk + (size_t)j * n, ldZ, G.V + (size_t)(j + 1) * n, ldV, nullptr, 0, s, G.active));
            HKG_TRY(gmres_arnoldi_step(G, j, rtol, s));
            if ((j + 1) % check == 0 || j + 1 == m) {
                HKG_HIP(hipMemcpyAsync(act.data(), c->active.p, nrhs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
                HKG_HIP(hipStreamSynchronize(s));
                bool still = false;
                for (int r = 0; r < nrhs; ++r) still = still || act[r];
                if (!still) break;
            }
        }
        HKG_HIP(hipMemcpyAsync(sc.data(), c->scal.p, sc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HKG_HIP(hipStreamSynchronize(s));
        for (int r = 0; r < nrhs; ++r) {
            if (!want[r]) continue;
            est[r] = sc[8 * r + 2] / (fn[r] > 0 ? fn[r] : 1.0);
            if (sc[8 * r + 5] != 0.0) want[r] = 0;   // singular Hessenberg column: no further progress
        }
        HKG_TRY(gmres_cycle_update(G, u, ld, s));
    }
    // true residuals
    HKG_TRY(spmv(n, nrhs, dp<int32_t>(c->rowptr), dp<int32_t>(c->colidx), dp<double>(c->Bval), u, ld, G.V, ldV, f, ld, s));
    HKG_TRY(vec_norms(n, nrhs, G.V, ldV, dp<double>(c->rnorm), dp<double>(c->npart), nblk, s));
    HKG_HIP(hipMemcpyAsync(rn.data(), c->rnorm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipStreamSynchronize(s));
    HKG_HIP(hipMemcpyAsync(iters.data(), c->itersd.p, nrhs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipStreamSynchronize(s));
    int32_t status = HKG_OK;
    for (int r = 0; r < nrhs; ++r) {
        const double rel = gmres_relres(rn[r], fn[r]);
        const int ok = rel <= rtol;     // false for NaN
        if (!ok) status = HKG_ENOTCONV;
        if (info) {
            info[r].iters = iters[r];
            info[r].converged = ok;
            info[r].relres_est = est[r];
            info[r].relres_true = rel;
        }
    }
    return status;
}

// ------------------------------------------------------------------------------------------------
// queries
// ------------------------------------------------------------------------------------------------
extern "C" int32_t hkgeneo_query(const hkgeneo_ctx *c, hkgeneo_stats *out) {
    if (!c || !out) return HKG_EINVAL;
    *out = c->stats;
    out->device_bytes = c->device_bytes + (c->fine ? c->fine->device_bytes : 0);
    out->peak_device_bytes = c->peak_device_bytes + (c->fine ? c->fine->peak_device_bytes : 0);
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

extern "C" int32_t hkgeneo_query_fine(const hkgeneo_ctx *c, int32_t *n_fine, int32_t *nI, int32_t *owner,
                                      int32_t *lambda_fine) {
    if (!c) return HKG_EINVAL;
    const hkgeneo_ctx *f = c->fine ? c->fine : c;
    if (n_fine) *n_fine = f->n_sub;
    if (lambda_fine) *lambda_fine = f->P.lambda_overlap;
    for (int i = 0; i < f->n_sub; ++i) {
        if (nI) nI[i] = f->subs[i].nI;
        if (owner) owner[i] = c->fine ? c->fine_owner[i] : i;
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
    const size_t bytes = (size_t)c->m0 * c->m0 * sizeof(double);
    if (c->m0 == 0 || !c->B0copy.p || c->B0copy.bytes < bytes) return HKG_EINVAL;
    HKG_HIP(hipMemcpy(B0, c->B0copy.p, bytes, hipMemcpyDeviceToHost));
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
