// Batched FGMRES over several set-up problems (one launch per phase for all of them), with the
// iteration captured as a HIP graph and an autotuned local-solve launch shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "batch.hpp"
#include "ctx.hpp"

using namespace hkg;

struct hkgeneo_batch {
    std::vector<hkgeneo_ctx *> ctx;
    std::vector<int> nrhs;
    BatchGeom geom;
    int restart = 50, check = 4;
    std::vector<ProbDev> hp;                    // host copy of the descriptor table
    DevBuf d_probs, d_items, d_rblk, d_cblk, d_ints, d_rn, d_want, d_scratch;
    std::vector<DevBuf> arena;                  // per-problem workspace
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hkgeneo_ctx acct;                           // carries the allocation counters of the batch's own buffers
    hkgeneo_ctx *owner = &acct;
    std::vector<int64_t> shape;                 // per problem: n, m0, sum_nI, max_nI, n_sub at creation
};

namespace {

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, int> g_tune;    // (max_nI, items, any f32, max_nrhs) -> waves

// pointers to the resident operators of a context (they move when the context is factored again)
void fill_resident(ProbDev &P, const hkgeneo_ctx *c) {
    P.rowptr = dp<int32_t>(c->rowptr);
    P.colidx = dp<int32_t>(c->colidx);
    P.Bval = dp<double>(c->Bval);
    P.subs = dp<SubDev>(c->subs_d);
    P.I_idx = dp<int32_t>(c->I_idx);
    P.wloc = dp<double>(c->wloc);
    P.Minv = c->Minv.p;
    P.Z = dp<double>(c->Z);
    P.Zr = dp<double>(c->Zr);
    P.B0inv = dp<double>(c->B0inv);
    P.tp_ptr = dp<int32_t>(c->tp_ptr);
    P.tp_pos = dp<int32_t>(c->tp_pos);
    P.local_f32 = c->opt.local_prec == 32;
}

std::vector<int64_t> shape_of(const hkgeneo_ctx *c) {
    return {c->n_dof, c->opt.two_level ? c->m0 : 0, c->sum_nI, c->max_nI, c->n_sub, c->opt.local_prec};
}

int32_t upload_table(hkgeneo_batch *b, hipStream_t s) {
    return upload_bytes(b->owner, &b->d_probs, b->hp.data(), b->hp.size() * sizeof(ProbDev), s, true);
}

int32_t autotune(hkgeneo_batch *b) {
    const BatchGeom &g = b->geom;
    int any32 = 0;
    for (auto &P : b->hp) any32 |= P.local_f32;
    const auto key = std::make_tuple(g.max_nI, g.nitems, any32, g.max_nrhs);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            b->geom.local_waves = it->second;
            return HKG_OK;
        }
    }
    // time the local-solve launch (standalone mode on a zero input) for each shape
    int maxn = 0;
    for (auto &P : b->hp) maxn = std::max(maxn, P.n);
    HKG_TRY(walloc(b->owner, &b->d_scratch, (size_t)2 * maxn * g.max_nrhs * sizeof(double)));
    HKG_HIP(hipMemsetAsync(b->d_scratch.p, 0, b->d_scratch.bytes, b->stream));
    std::vector<ProbDev> save = b->hp;
    for (auto &P : b->hp) {
        P.xin = dp<double>(b->d_scratch);
        P.ldin = maxn;
        P.xout = dp<double>(b->d_scratch) + (size_t)maxn * g.max_nrhs;
        P.ldout = maxn;
    }
    HKG_TRY(upload_table(b, b->stream));
    hipEvent_t e0, e1;
    HKG_HIP(hipEventCreate(&e0));
    HKG_HIP(hipEventCreate(&e1));
    int best = 8;
    float best_ms = 1e30f;
    for (int waves : {4, 8, 16}) {
        BatchGeom gg = g;
        gg.local_waves = waves;
        float tot = 0.0f;
        for (int rep = 0; rep < 6; ++rep) {
            float ms = 0.0f;
            HKG_TRY(batch_apply(gg, dp<ProbDev>(b->d_probs), dp<WorkItem>(b->d_items), dp<WorkItem>(b->d_rblk),
                                dp<WorkItem>(b->d_cblk), 0, b->stream, e0, e1));
            HKG_HIP(hipEventSynchronize(e1));
            HKG_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) tot += ms;
        }
        if (tot < best_ms) {
            best_ms = tot;
            best = waves;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HKG_HIP(hipStreamSynchronize(b->stream));
    b->hp = save;
    HKG_TRY(upload_table(b, b->stream));
    b->geom.local_waves = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
    return HKG_OK;
}

int32_t capture(hkgeneo_batch *b) {
    if (b->exec) return HKG_OK;
    HKG_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    int32_t st = batch_apply(b->geom, dp<ProbDev>(b->d_probs), dp<WorkItem>(b->d_items), dp<WorkItem>(b->d_rblk),
                             dp<WorkItem>(b->d_cblk), 1, b->stream);
    if (st == HKG_OK) st = batch_arnoldi(b->geom, dp<ProbDev>(b->d_probs), dp<WorkItem>(b->d_rblk), b->stream);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &graph);
    if (st != HKG_OK) return st;
    if (e != hipSuccess) {
        set_last_error(std::string("graph capture: ") + hipGetErrorString(e));
        return HKG_EHIP;
    }
    b->graph = graph;
    HKG_HIP(hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0));
    return HKG_OK;
}

}  // namespace

namespace hkg {

void batch_free(hkgeneo_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (auto &a : b->arena) drelease(b->owner, &a);
    DevBuf *bufs[] = {&b->d_probs, &b->d_items, &b->d_rblk, &b->d_cblk, &b->d_ints, &b->d_rn, &b->d_want, &b->d_scratch};
    for (DevBuf *x : bufs) drelease(b->owner, x);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

int32_t batch_build(hkgeneo_ctx *const *ctxs, const int32_t *nrhs, int nprob, hkgeneo_batch **out) {
    *out = nullptr;
    if (nprob < 1) return HKG_EINVAL;
    hkgeneo_batch *b = new hkgeneo_batch();
    b->restart = ctxs[0]->opt.restart;
    int32_t st = HKG_OK;
    auto fail = [&](int32_t code) {
        batch_free(b);
        return code;
    };
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) return fail(HKG_EHIP);
    BatchGeom &g = b->geom;
    g.nprob = nprob;
    for (int p = 0; p < nprob; ++p) {
        hkgeneo_ctx *c = ctxs[p];
        if (!c || nrhs[p] < 1 || nrhs[p] > 65535 || c->opt.restart != b->restart) {
            set_last_error("batch: every problem needs a context, 1..65535 right-hand sides and the same restart");
            return fail(HKG_EINVAL);
        }
        b->ctx.push_back(c);
        const std::vector<int64_t> sh = shape_of(c);
        b->shape.insert(b->shape.end(), sh.begin(), sh.end());
        b->nrhs.push_back(nrhs[p]);
        g.max_nrhs = std::max(g.max_nrhs, (int)nrhs[p]);
        g.max_nI = std::max(g.max_nI, c->max_nI);
        g.max_tiles = std::max(g.max_tiles, (c->max_nI + 63) / 64);
        g.any_coarse = g.any_coarse || (c->opt.two_level && c->m0 > 0);
    }
    g.restart = b->restart;
    const int maxR = g.max_nrhs, m = b->restart;
    // the local-solve launch keeps two copies of the largest dof(D) vector and 16 x 64 partials in LDS
    if ((size_t)2 * g.max_nI * sizeof(double) + 16 * 64 * sizeof(double) > 160 * 1024 ||
        (size_t)5 * (m + 2) * sizeof(double) > 64 * 1024) {
        set_last_error("batch: subdomain or restart too large for the batched kernels");
        return fail(HKG_EINVAL);
    }
    std::vector<WorkItem> items, rblk, cblk;
    b->hp.resize(nprob);
    b->arena.resize(nprob);
    // pair arrays: active | iters | jcur (ints), rnorm (doubles), want (ints)
    if ((st = dalloc(b->owner, &b->d_ints, (size_t)3 * nprob * maxR * sizeof(int32_t))) != HKG_OK) return fail(st);
    if ((st = dalloc(b->owner, &b->d_rn, (size_t)nprob * maxR * sizeof(double))) != HKG_OK) return fail(st);
    if ((st = dalloc(b->owner, &b->d_want, (size_t)nprob * maxR * sizeof(int32_t))) != HKG_OK) return fail(st);
    int32_t *ints = dp<int32_t>(b->d_ints);
    for (int p = 0; p < nprob; ++p) {
        hkgeneo_ctx *c = ctxs[p];
        const int R = nrhs[p];
        ProbDev &P = b->hp[p];
        std::memset(&P, 0, sizeof(P));
        P.n = c->n_dof;
        P.nsub = c->n_sub;
        P.m0 = c->opt.two_level ? c->m0 : 0;
        P.maxnI = c->max_nI;
        P.nchunk = std::max(1, (P.m0 + 63) / 64);
        P.nblk = (P.n + BROWS - 1) / BROWS;
        P.nrhs = R;
        P.restart = m;
        P.local_f32 = c->opt.local_prec == 32;
        P.two_level = c->opt.two_level && c->m0 > 0;
        P.max_iter = c->opt.max_iter;
        P.sum_nI = c->sum_nI;
        P.rtol = c->opt.rtol;
        fill_resident(P, c);
        const size_t n = P.n, m0 = std::max(P.m0, 1);
        const size_t sizes[] = {(size_t)c->sum_nI * R,
                                m0 * R,
                                m0 * P.nchunk * R,
                                n * (m + 1) * R,
                                n * m * R,
                                (size_t)(m + 1) * m * R,
                                (size_t)m * R,
                                (size_t)m * R,
                                (size_t)(m + 1) * R,
                                (size_t)2 * P.nblk * (m + 2) * R,
                                (size_t)(m + 2) * R,
                                (size_t)8 * R};
        size_t total = 0;
        for (size_t z : sizes) total += z;
        if ((st = dalloc(b->owner, &b->arena[p], total * sizeof(double))) != HKG_OK) return fail(st);
        double *q = dp<double>(b->arena[p]);
        double **dst[] = {&P.u, &P.c, &P.ypart, &P.V, &P.Zk, &P.H, &P.cs, &P.sn, &P.g, &P.part, &P.hcol, &P.scal};
        for (int k = 0; k < 12; ++k) {
            *dst[k] = q;
            q += sizes[k];
        }
        P.active = ints + (size_t)p * maxR;
        P.iters = ints + (size_t)nprob * maxR + (size_t)p * maxR;
        P.jcur = ints + (size_t)2 * nprob * maxR + (size_t)p * maxR;
        P.rnorm = dp<double>(b->d_rn) + (size_t)p * maxR;
        for (int s = 0; s < c->n_sub; ++s) items.push_back({p, s});
        for (int k = 0; k < P.nblk; ++k) rblk.push_back({p, k});
        if (P.two_level)
            for (int k = 0; k < ((P.m0 + 63) / 64) * P.nchunk; ++k) cblk.push_back({p, k});
    }
    if (items.size() > 65535) {
        set_last_error("batch: more than 65535 subdomains in one batch");
        return fail(HKG_EINVAL);
    }
    g.nitems = (int)items.size();
    g.nrblk = (int)rblk.size();
    g.ncblk = (int)cblk.size();
    if (cblk.empty()) cblk.push_back({0, 0});
    if ((st = upload(b->owner, &b->d_items, items.data(), items.size(), b->stream)) != HKG_OK) return fail(st);
    if ((st = upload(b->owner, &b->d_rblk, rblk.data(), rblk.size(), b->stream)) != HKG_OK) return fail(st);
    if ((st = upload(b->owner, &b->d_cblk, cblk.data(), cblk.size(), b->stream)) != HKG_OK) return fail(st);
    if (hipMemsetAsync(b->d_ints.p, 0, b->d_ints.bytes, b->stream) != hipSuccess) return fail(HKG_EHIP);
    if ((st = upload_table(b, b->stream)) != HKG_OK) return fail(st);
    if ((st = autotune(b)) != HKG_OK) return fail(st);
    *out = b;
    return HKG_OK;
}

// FGMRES(restart) on every (problem, rhs) pair of the batch from x = 0.
int32_t batch_solve(hkgeneo_batch *b, const double *const *f, double *const *u, const int32_t *ld,
                    hkgeneo_rhs_info *info, hipStream_t user, bool prof, std::vector<hipEvent_t> *ev, size_t *ev_used) {
    BatchGeom &g = b->geom;
    const int np = g.nprob, maxR = g.max_nrhs, m = b->restart;
    for (int p = 0; p < np; ++p) {
        ProbDev &P = b->hp[p];
        if (!f[p] || !u[p] || ld[p] < P.n) return HKG_EINVAL;
        const std::vector<int64_t> sh = shape_of(b->ctx[p]);
        if (!std::equal(sh.begin(), sh.end(), b->shape.begin() + (size_t)p * sh.size())) {
            set_last_error("batch: a context changed shape since the batch was created");
            return HKG_EINVAL;
        }
        fill_resident(P, b->ctx[p]);
        P.f = f[p];
        P.x = u[p];
        P.ldf = ld[p];
        P.ldx = ld[p];
    }
    HKG_HIP(hipStreamSynchronize(user));       // the caller's inputs are ready
    hipStream_t s = b->stream;
    HKG_TRY(upload_table(b, s));
    const ProbDev *dprob = dp<ProbDev>(b->d_probs);
    const WorkItem *items = dp<WorkItem>(b->d_items), *rblk = dp<WorkItem>(b->d_rblk), *cblk = dp<WorkItem>(b->d_cblk);
    const int pairs = np * maxR;
    std::vector<double> rn(pairs), fn(pairs);
    std::vector<int32_t> want(pairs), act(pairs), iters(pairs);
    HKG_TRY(batch_residual(g, dprob, rblk, 1, s));
    HKG_HIP(hipMemcpyAsync(fn.data(), b->d_rn.p, pairs * sizeof(double), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipStreamSynchronize(s));
    rn = fn;
    if (!prof) HKG_TRY(capture(b));
    const int check = prof ? 1 : b->check;
    bool first = true;
    while (true) {
        if (!first) {
            HKG_TRY(batch_residual(g, dprob, rblk, 0, s));
            HKG_HIP(hipMemcpyAsync(rn.data(), b->d_rn.p, pairs * sizeof(double), hipMemcpyDeviceToHost, s));
        }
        HKG_HIP(hipMemcpyAsync(iters.data(), dp<int32_t>(b->d_ints) + pairs, pairs * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
        HKG_HIP(hipStreamSynchronize(s));
        first = false;
        bool any = false;
        for (int p = 0; p < np; ++p)
            for (int r = 0; r < maxR; ++r) {
                const int k = p * maxR + r;
                want[k] = r < b->nrhs[p] && fn[k] > 0.0 && rn[k] > b->hp[p].rtol * fn[k] && iters[k] < b->hp[p].max_iter;
                any = any || want[k];
            }
        if (!any) break;
        HKG_HIP(hipMemcpyAsync(b->d_want.p, want.data(), pairs * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HKG_TRY(batch_cycle_start(g, dprob, rblk, dp<int32_t>(b->d_want), s));
        for (int j = 0; j < m; ++j) {
            if (prof) {
                if (*ev_used + 2 > ev->size())
                    for (int k = 0; k < 256; ++k) {
                        hipEvent_t e;
                        HKG_HIP(hipEventCreate(&e));
                        ev->push_back(e);
                    }
                HKG_TRY(batch_apply(g, dprob, items, rblk, cblk, 1, s, (*ev)[*ev_used], (*ev)[*ev_used + 1]));
                *ev_used += 2;
                HKG_TRY(batch_arnoldi(g, dprob, rblk, s));
            } else {
                HKG_HIP(hipGraphLaunch(b->exec, s));
            }
            if ((j + 1) % check == 0 || j + 1 == m) {
                HKG_HIP(hipMemcpyAsync(act.data(), b->d_ints.p, pairs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
                HKG_HIP(hipStreamSynchronize(s));
                bool still = false;
                for (int k = 0; k < pairs; ++k) still = still || act[k];
                if (!still) break;
            }
        }
        HKG_TRY(batch_cycle_update(g, dprob, rblk, s));
    }
    HKG_TRY(batch_residual(g, dprob, rblk, 0, s));
    HKG_HIP(hipMemcpyAsync(rn.data(), b->d_rn.p, pairs * sizeof(double), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipMemcpyAsync(iters.data(), dp<int32_t>(b->d_ints) + pairs, pairs * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s));
    std::vector<std::vector<double>> sc(np);
    for (int p = 0; p < np; ++p) {
        sc[p].resize((size_t)8 * b->nrhs[p]);
        HKG_HIP(hipMemcpyAsync(sc[p].data(), b->hp[p].scal, sc[p].size() * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HKG_HIP(hipStreamSynchronize(s));
    int32_t status = HKG_OK;
    int q = 0;
    for (int p = 0; p < np; ++p)
        for (int r = 0; r < b->nrhs[p]; ++r, ++q) {
            const int k = p * maxR + r;
            const double rel = fn[k] > 0 ? rn[k] / fn[k] : 0.0;
            const int ok = rel <= b->hp[p].rtol;
            if (!ok) status = HKG_ENOTCONV;
            if (info) {
                info[q].iters = iters[k];
                info[q].converged = ok;
                info[q].relres_est = fn[k] > 0 ? sc[p][8 * r + 2] / fn[k] : 0.0;
                info[q].relres_true = rel;
            }
        }
    return status;
}

}  // namespace hkg

extern "C" int32_t hkgeneo_batch_create(hkgeneo_ctx *const *ctxs, const int32_t *nrhs, int32_t nprob,
                                        hkgeneo_batch **out) {
    if (!ctxs || !nrhs || !out || nprob < 1) return HKG_EINVAL;
    return batch_build(ctxs, nrhs, nprob, out);
}

extern "C" int32_t hkgeneo_batch_solve(hkgeneo_batch *b, const double *const *f, double *const *u, const int32_t *ld,
                                       hkgeneo_rhs_info *info, void *stream) {
    if (!b || !f || !u || !ld) return HKG_EINVAL;
    return batch_solve(b, f, u, ld, info, (hipStream_t)stream, false, nullptr, nullptr);
}

extern "C" void hkgeneo_batch_destroy(hkgeneo_batch *b) { batch_free(b); }

extern "C" int64_t hkgeneo_batch_bytes(const hkgeneo_batch *b) { return b ? b->acct.device_bytes : 0; }

extern "C" int32_t hkgeneo_batch_local_waves(const hkgeneo_batch *b) { return b ? b->geom.local_waves : 0; }
