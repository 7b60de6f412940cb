// Continuous-batching FGMRES engine over set-up problems, and the two C-ABI front ends built on it:
// hkgeneo_batch_* (a fixed set of problems solved together) and hkgeneo_server_* (requests that
// join and leave the live set at iteration boundaries).
//
// A request is one problem (a set-up context) with nrhs right-hand sides.  Admitted requests occupy
// a slot of the descriptor table and carry their own Krylov workspace.  The live set is stepped by
// two captured HIP graphs: the iteration (preconditioner application and CGS2 Arnoldi step for every
// iterating pair) and the restart phase (x update, true residual, stop or new cycle for every pair
// at a cycle boundary).  The host reads the pair states every `check` iterations, launches the
// restart graph when some pair waits for it, retires finished requests and admits queued ones; a
// change of the live set rebuilds the work lists and re-captures the graphs (the iteration once per
// parity of the double-buffered Arnoldi index, replayed alternately).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "batch.hpp"
#include "ctx.hpp"

using namespace hkg;

namespace {

struct Request {
    hkgeneo_ctx *ctx = nullptr;
    int nrhs = 0, ld = 0;
    const double *f = nullptr;
    double *u = nullptr;
    int64_t tag = 0;
    hipEvent_t ready = nullptr;     // recorded on the caller's stream at submission
    int slot = -1;
    DevBuf ws;
};

struct Done {
    int64_t tag;
    int32_t status;
    std::vector<hkgeneo_rhs_info> info;
};

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, int> g_tune;    // (max_nI, items bucket, any f32, max_nrhs) -> waves

int pow2_bucket(int v) {
    int b = 1;
    while (b < v) b <<= 1;
    return b;
}

}  // namespace

struct hkgeneo_server {
    hkgeneo_ctx acct;                   // allocation counters of the engine's own buffers
    int cap = 0, maxR = 0, restart = 0, check = 4;
    int64_t budget = 0, ws_in_use = 0;  // Krylov workspace bytes (including the reuse pool)
    std::vector<ProbDev> table;
    std::vector<Request *> slot_req;
    std::deque<Request *> queue;
    std::deque<Done> done;
    std::vector<DevBuf> pool;           // workspace buffers of retired requests, for reuse
    DevBuf d_probs, d_items, d_rblk, d_cblk, d_live, d_state, d_scratch;
    int32_t *h_state = nullptr;         // pinned mirror of d_state
    std::vector<int32_t> live;
    std::vector<int64_t> built_sig;     // geometry of the live set the graphs were captured for
    BatchGeom geom;
    bool dirty = true, need_restart = false, any_iter = false;
    hipStream_t stream = nullptr;
    hipGraph_t it_graph[2] = {nullptr, nullptr}, rs_graph = nullptr;
    hipGraphExec_t it_exec[2] = {nullptr, nullptr}, rs_exec = nullptr;
    int parity = 0;
    int64_t n_iter_launch = 0, n_restart_launch = 0, n_capture = 0, n_admitted = 0, n_retired = 0;
    // measurement hook: with prof set, iterations are launched directly (same kernels, same shapes)
    // with HIP events around every local-solve launch
    bool prof = false;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
};

namespace {

using Engine = hkgeneo_server;

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
    P.tpc = dp<TpCoarse>(c->tpZ);
}

constexpr int NWS = 15;

// workspace layout of one request (in doubles), in the order of the ProbDev pointers
void ws_sizes(const hkgeneo_ctx *c, int R, int m, size_t out[NWS]) {
    const size_t n = c->n_dof;
    const int m0r = c->opt.two_level ? c->m0 : 0;
    const size_t m0 = std::max(m0r, 1);
    const size_t nchunk = std::max(1, (m0r + 63) / 64);
    const size_t nblk = (n + BROWS - 1) / BROWS;
    const size_t v[NWS] = {(size_t)c->sum_nI * R,          // u
                           m0 * R,                         // c
                           m0 * nchunk * R,                // ypart
                           n * (m + 1) * R,                // V
                           n * m * R,                      // Zk
                           (size_t)(m + 1) * m * R,        // H
                           (size_t)m * R,                  // cs
                           (size_t)m * R,                  // sn
                           (size_t)(m + 1) * R,            // g
                           2 * nblk * (m + 2) * R,         // part
                           (size_t)(m + 2) * R,            // hcol
                           (size_t)8 * R,                  // scal
                           (size_t)R,                      // rnorm
                           (size_t)(R + 1) / 2,            // iters (int32)
                           (size_t)R};                     // jcur (2 int32 per rhs)
    // each region a whole number of 16-byte units, so that every region (and the coarse vector c of
    // each right-hand side when m_0 is even) starts 16-byte aligned for the paired loads
    for (int k = 0; k < NWS; ++k) out[k] = (v[k] + 1) & ~(size_t)1;
}

int64_t ws_bytes(const hkgeneo_ctx *c, int R, int m) {
    size_t z[NWS];
    ws_sizes(c, R, m, z);
    size_t t = 0;
    for (size_t v : z) t += v;
    return (int64_t)(t * sizeof(double));
}

void release_ws(Engine *E, DevBuf *b) {
    E->ws_in_use -= (int64_t)b->bytes;
    drelease(&E->acct, b);
}

// a workspace of at least `bytes`: from the reuse pool, else fresh if the budget allows (freeing
// pooled buffers first); *ok = false if it does not fit now
int32_t take_ws(Engine *E, int64_t bytes, DevBuf *out, bool *ok) {
    *ok = false;
    int best = -1;
    for (int k = 0; k < (int)E->pool.size(); ++k)
        if ((int64_t)E->pool[k].bytes >= bytes && (int64_t)E->pool[k].bytes <= 2 * bytes + (1 << 20) &&
            (best < 0 || E->pool[k].bytes < E->pool[best].bytes))
            best = k;
    if (best >= 0) {
        *out = E->pool[best];
        E->pool.erase(E->pool.begin() + best);
        *ok = true;
        return HKG_OK;
    }
    while (E->ws_in_use + bytes > E->budget && !E->pool.empty()) {
        release_ws(E, &E->pool.back());
        E->pool.pop_back();
    }
    if (E->ws_in_use + bytes > E->budget) return HKG_OK;
    HKG_TRY(dalloc(&E->acct, out, (size_t)bytes));
    E->ws_in_use += bytes;
    *ok = true;
    return HKG_OK;
}

int32_t admit_one(Engine *E, Request *q, int slot) {
    hkgeneo_ctx *c = q->ctx;
    const int R = q->nrhs, m = E->restart;
    ProbDev &P = E->table[slot];
    std::memset(&P, 0, sizeof(P));
    P.n = c->n_dof;
    P.nsub = c->n_sub;
    P.m0 = c->opt.two_level ? c->m0 : 0;
    P.maxnI = c->max_nI;
    P.nblk = (P.n + BROWS - 1) / BROWS;
    P.nchunk = std::max(1, (P.m0 + 63) / 64);
    P.nrhs = R;
    P.restart = m;
    P.local_f32 = c->opt.local_prec == 32;
    P.two_level = c->opt.two_level && c->m0 > 0;
    P.max_iter = c->opt.max_iter;
    P.sum_nI = c->sum_nI;
    P.rtol = c->opt.rtol;
    fill_resident(P, c);
    size_t z[NWS];
    ws_sizes(c, R, m, z);
    double *w = dp<double>(q->ws);
    double **dst[13] = {&P.u, &P.c, &P.ypart, &P.V, &P.Zk, &P.H, &P.cs, &P.sn, &P.g, &P.part, &P.hcol, &P.scal, &P.rnorm};
    for (int k = 0; k < 13; ++k) {
        *dst[k] = w;
        w += z[k];
    }
    P.iters = reinterpret_cast<int32_t *>(w);
    w += z[13];
    P.jcur = reinterpret_cast<int32_t *>(w);
    P.active = dp<int32_t>(E->d_state) + (size_t)slot * E->maxR;
    P.f = q->f;
    P.x = q->u;
    P.ldf = q->ld;
    P.ldx = q->ld;
    for (int r = 0; r < E->maxR; ++r) E->h_state[(size_t)slot * E->maxR + r] = r < R ? PS_NEW : PS_DONE;
    HKG_HIP(hipMemcpyAsync(P.active, E->h_state + (size_t)slot * E->maxR, E->maxR * sizeof(int32_t),
                           hipMemcpyHostToDevice, E->stream));
    HKG_HIP(hipStreamWaitEvent(E->stream, q->ready, 0));
    HKG_HIP(hipStreamSynchronize(E->stream));    // the pinned staging row is overwritten by the next scan
    q->slot = slot;
    E->slot_req[slot] = q;
    E->need_restart = true;
    E->dirty = true;
    E->n_admitted++;
    return HKG_OK;
}

// FIFO admission while a slot and the workspace budget allow
int32_t admit(Engine *E) {
    while (!E->queue.empty()) {
        Request *q = E->queue.front();
        int slot = -1;
        for (int s = 0; s < E->cap; ++s)
            if (!E->slot_req[s]) {
                slot = s;
                break;
            }
        if (slot < 0) return HKG_OK;
        bool ok = false;
        HKG_TRY(take_ws(E, ws_bytes(q->ctx, q->nrhs, E->restart), &q->ws, &ok));
        if (!ok) return HKG_OK;
        E->queue.pop_front();
        const int32_t st = admit_one(E, q, slot);
        if (st != HKG_OK) {
            E->pool.push_back(q->ws);
            if (q->ready) (void)hipEventDestroy(q->ready);
            delete q;
            return st;
        }
    }
    return HKG_OK;
}

int32_t autotune(Engine *E) {
    BatchGeom &g = E->geom;
    int any32 = 0, maxn = 0;
    for (int s : E->live) {
        any32 |= E->table[s].local_f32;
        maxn = std::max(maxn, E->table[s].n);
    }
    const auto key = std::make_tuple(g.max_nI, pow2_bucket(g.nitems), any32, g.max_nrhs);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            g.local_waves = it->second;
            return HKG_OK;
        }
    }
    // time the local-solve launch for each shape in standalone mode (scratch input and output; the
    // live requests' preconditioner temporaries are overwritten, which is harmless at an iteration
    // boundary)
    HKG_TRY(walloc(&E->acct, &E->d_scratch, (size_t)2 * maxn * g.max_nrhs * sizeof(double)));
    HKG_HIP(hipMemsetAsync(E->d_scratch.p, 0, E->d_scratch.bytes, E->stream));
    std::vector<ProbDev> save = E->table;
    for (int s : E->live) {
        ProbDev &P = E->table[s];
        P.xin = dp<double>(E->d_scratch);
        P.ldin = maxn;
        P.xout = dp<double>(E->d_scratch) + (size_t)maxn * g.max_nrhs;
        P.ldout = maxn;
    }
    HKG_TRY(upload_bytes(&E->acct, &E->d_probs, E->table.data(), E->table.size() * sizeof(ProbDev), E->stream, true));
    E->table = save;
    hipEvent_t e0, e1;
    HKG_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return HKG_EHIP;
    }
    // two warm-up launches per shape, then the median of nine timed launches (shapes interleaved so
    // that clock and cache drift affect all alike)
    const int cand[3] = {4, 8, 16};
    std::vector<float> t[3];
    int32_t st = HKG_OK;
    for (int rep = 0; rep < 11 && st == HKG_OK; ++rep)
        for (int w = 0; w < 3 && st == HKG_OK; ++w) {
            BatchGeom gg = g;
            gg.local_waves = cand[w];
            float ms = 0.0f;
            st = batch_apply(gg, dp<ProbDev>(E->d_probs), dp<WorkItem>(E->d_items), dp<WorkItem>(E->d_rblk),
                             dp<WorkItem>(E->d_cblk), 0, 0, E->stream, e0, e1);
            if (st == HKG_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                st = HKG_EHIP;
            if (rep >= 2) t[w].push_back(ms);
        }
    int best = 8;
    float best_ms = 1e30f;
    for (int w = 0; w < 3 && st == HKG_OK; ++w) {
        std::sort(t[w].begin(), t[w].end());
        const float med = t[w][t[w].size() / 2];
        if (med < best_ms) {
            best_ms = med;
            best = cand[w];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HKG_TRY(st);
    HKG_HIP(hipStreamSynchronize(E->stream));
    g.local_waves = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
    return HKG_OK;
}

void drop_graphs(Engine *E) {
    for (int k = 0; k < 2; ++k) {
        if (E->it_exec[k]) (void)hipGraphExecDestroy(E->it_exec[k]);
        if (E->it_graph[k]) (void)hipGraphDestroy(E->it_graph[k]);
        E->it_exec[k] = nullptr;
        E->it_graph[k] = nullptr;
    }
    if (E->rs_exec) (void)hipGraphExecDestroy(E->rs_exec);
    if (E->rs_graph) (void)hipGraphDestroy(E->rs_graph);
    E->rs_exec = nullptr;
    E->rs_graph = nullptr;
}

template <typename F>
int32_t capture(Engine *E, F &&body, hipGraph_t *graph, hipGraphExec_t *exec) {
    HKG_HIP(hipStreamBeginCapture(E->stream, hipStreamCaptureModeThreadLocal));
    const int32_t st = body();
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(E->stream, &gr);
    if (st != HKG_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return st;
    }
    if (e != hipSuccess) {
        set_last_error(std::string("graph capture: ") + hipGetErrorString(e));
        return HKG_EHIP;
    }
    *graph = gr;
    HKG_HIP(hipGraphInstantiate(exec, gr, nullptr, nullptr, 0));
    E->n_capture++;
    return HKG_OK;
}

// geometry of the live set: everything the work lists, launch shapes and graphs depend on (the
// descriptor contents are read by the kernels at run time and may change freely)
std::vector<int64_t> live_signature(const Engine *E) {
    std::vector<int64_t> sig;
    for (int s = 0; s < E->cap; ++s)
        if (E->slot_req[s]) {
            const ProbDev &P = E->table[s];
            sig.insert(sig.end(), {s, P.n, P.nsub, P.maxnI, P.nblk, P.two_level, P.local_f32, P.m0});
        }
    return sig;
}

// work lists, descriptor table and graphs for the current live set
int32_t rebuild(Engine *E) {
    HKG_HIP(hipStreamSynchronize(E->stream));    // no launch of the old graphs is in flight
    E->dirty = false;
    std::vector<int64_t> sig = live_signature(E);
    if (!sig.empty() && sig == E->built_sig && E->it_exec[0]) {
        // same geometry: the lists and graphs stand, only the descriptors change
        return upload_bytes(&E->acct, &E->d_probs, E->table.data(), E->table.size() * sizeof(ProbDev), E->stream,
                            true);
    }
    drop_graphs(E);
    E->built_sig.clear();
    E->live.clear();
    for (int s = 0; s < E->cap; ++s)
        if (E->slot_req[s]) E->live.push_back(s);
    BatchGeom &g = E->geom;
    const int waves = g.local_waves;
    g = BatchGeom{};
    g.local_waves = waves;
    g.restart = E->restart;
    g.nprob = (int)E->live.size();
    g.max_nrhs = E->maxR;
    if (E->live.empty()) return HKG_OK;
    std::vector<WorkItem> items, rblk, cblk;
    for (int s : E->live) {
        const ProbDev &P = E->table[s];
        g.max_nI = std::max(g.max_nI, P.maxnI);
        g.max_tiles = std::max(g.max_tiles, (P.maxnI + LTILE - 1) / LTILE);
        g.any_coarse = g.any_coarse || P.two_level;
        for (int k = 0; k < P.nsub; ++k) items.push_back({s, k});
        for (int k = 0; k < P.nblk; ++k) rblk.push_back({s, k});
        if (P.two_level)
            for (int k = 0; k < (P.m0 + 3) / 4; ++k) cblk.push_back({s, k});
    }
    if (items.size() > 65535) {
        set_last_error("more than 65535 subdomains in the live set");
        E->dirty = true;
        return HKG_EINVAL;
    }
    g.nitems = (int)items.size();
    g.nrblk = (int)rblk.size();
    g.ncblk = (int)cblk.size();
    if (cblk.empty()) cblk.push_back({E->live[0], 0});
    HKG_TRY(upload(&E->acct, &E->d_items, items.data(), items.size(), E->stream, true));
    HKG_TRY(upload(&E->acct, &E->d_rblk, rblk.data(), rblk.size(), E->stream, true));
    HKG_TRY(upload(&E->acct, &E->d_cblk, cblk.data(), cblk.size(), E->stream, true));
    HKG_TRY(upload(&E->acct, &E->d_live, E->live.data(), E->live.size(), E->stream, true));
    HKG_TRY(autotune(E));
    HKG_TRY(upload_bytes(&E->acct, &E->d_probs, E->table.data(), E->table.size() * sizeof(ProbDev), E->stream, true));
    const ProbDev *probs = dp<ProbDev>(E->d_probs);
    const WorkItem *it = dp<WorkItem>(E->d_items), *rb = dp<WorkItem>(E->d_rblk), *cb = dp<WorkItem>(E->d_cblk);
    const int32_t *lv = dp<int32_t>(E->d_live);
    for (int par = 0; par < 2; ++par)
        HKG_TRY(capture(
            E,
            [&]() {
                HKG_TRY(batch_apply(g, probs, it, rb, cb, 1, par, E->stream));
                return batch_arnoldi(g, probs, rb, par, E->stream);
            },
            &E->it_graph[par], &E->it_exec[par]));
    HKG_TRY(capture(E, [&]() { return batch_restart(g, probs, rb, lv, E->stream); }, &E->rs_graph, &E->rs_exec));
    E->built_sig = std::move(sig);
    return HKG_OK;
}

int32_t retire(Engine *E, int slot) {
    Request *q = E->slot_req[slot];
    const ProbDev &P = E->table[slot];
    const int R = q->nrhs;
    std::vector<double> rn(R), sc((size_t)8 * R);
    std::vector<int32_t> it(R);
    HKG_HIP(hipMemcpyAsync(rn.data(), P.rnorm, R * sizeof(double), hipMemcpyDeviceToHost, E->stream));
    HKG_HIP(hipMemcpyAsync(sc.data(), P.scal, sc.size() * sizeof(double), hipMemcpyDeviceToHost, E->stream));
    HKG_HIP(hipMemcpyAsync(it.data(), P.iters, R * sizeof(int32_t), hipMemcpyDeviceToHost, E->stream));
    HKG_HIP(hipStreamSynchronize(E->stream));
    Done d;
    d.tag = q->tag;
    d.status = HKG_OK;
    d.info.resize(R);
    for (int r = 0; r < R; ++r) {
        const double fn = sc[8 * r + 1];
        const double rel = gmres_relres(rn[r], fn);
        d.info[r].iters = it[r];
        d.info[r].converged = rel <= P.rtol;     // false for NaN
        d.info[r].relres_est = fn > 0 ? sc[8 * r + 2] / fn : 0.0;
        d.info[r].relres_true = rel;
        if (!d.info[r].converged) d.status = HKG_ENOTCONV;
    }
    E->done.push_back(std::move(d));
    E->pool.push_back(q->ws);
    if (q->ready) (void)hipEventDestroy(q->ready);
    delete q;
    E->slot_req[slot] = nullptr;
    E->dirty = true;
    E->n_retired++;
    return HKG_OK;
}

// one check period: admission, rebuild, restart phase if needed, `check` iterations, state scan and
// retirement.  *pending: requests live or queued afterwards.
int32_t pump_once(Engine *E, int *pending) {
    HKG_TRY(admit(E));
    if (E->dirty) HKG_TRY(rebuild(E));
    if (!E->live.empty()) {
        bool ran = false;
        if (E->need_restart) {
            HKG_HIP(hipGraphLaunch(E->rs_exec, E->stream));
            E->n_restart_launch++;
            E->need_restart = false;
            ran = true;
        }
        if (ran || E->any_iter) {
            for (int k = 0; k < E->check; ++k) {
                if (E->prof) {
                    if (E->ev_used + 2 > E->ev.size())
                        for (int q = 0; q < 256; ++q) {
                            hipEvent_t e;
                            HKG_HIP(hipEventCreate(&e));
                            E->ev.push_back(e);
                        }
                    const ProbDev *probs = dp<ProbDev>(E->d_probs);
                    HKG_TRY(batch_apply(E->geom, probs, dp<WorkItem>(E->d_items), dp<WorkItem>(E->d_rblk),
                                        dp<WorkItem>(E->d_cblk), 1, E->parity, E->stream, E->ev[E->ev_used],
                                        E->ev[E->ev_used + 1]));
                    E->ev_used += 2;
                    HKG_TRY(batch_arnoldi(E->geom, probs, dp<WorkItem>(E->d_rblk), E->parity, E->stream));
                } else {
                    HKG_HIP(hipGraphLaunch(E->it_exec[E->parity], E->stream));
                }
                E->parity ^= 1;
            }
            E->n_iter_launch += E->check;
        }
        HKG_HIP(hipMemcpyAsync(E->h_state, E->d_state.p, (size_t)E->cap * E->maxR * sizeof(int32_t),
                               hipMemcpyDeviceToHost, E->stream));
        HKG_HIP(hipStreamSynchronize(E->stream));
        E->any_iter = false;
        const std::vector<int32_t> live = E->live;
        for (int s : live) {
            const int32_t *st = E->h_state + (size_t)s * E->maxR;
            bool all_done = true;
            for (int r = 0; r < E->slot_req[s]->nrhs; ++r) {
                if (st[r] != PS_DONE) all_done = false;
                if (st[r] == PS_ITER) E->any_iter = true;
                if (st[r] == PS_CYCLE_END || st[r] == PS_NEW) E->need_restart = true;
            }
            if (all_done) HKG_TRY(retire(E, s));
        }
    }
    int n = (int)E->queue.size();
    for (int s = 0; s < E->cap; ++s) n += E->slot_req[s] != nullptr;
    *pending = n;
    return HKG_OK;
}

void engine_free(Engine *E) {
    if (!E) return;
    if (E->stream) (void)hipStreamSynchronize(E->stream);
    drop_graphs(E);
    for (Request *q : E->queue) {
        if (q->ready) (void)hipEventDestroy(q->ready);
        delete q;
    }
    for (int s = 0; s < E->cap; ++s)
        if (E->slot_req[s]) {
            release_ws(E, &E->slot_req[s]->ws);
            if (E->slot_req[s]->ready) (void)hipEventDestroy(E->slot_req[s]->ready);
            delete E->slot_req[s];
        }
    for (auto &b : E->pool) release_ws(E, &b);
    DevBuf *bufs[] = {&E->d_probs, &E->d_items, &E->d_rblk, &E->d_cblk, &E->d_live, &E->d_state, &E->d_scratch};
    for (DevBuf *x : bufs) drelease(&E->acct, x);
    if (E->h_state) (void)hipHostFree(E->h_state);
    for (hipEvent_t e : E->ev) (void)hipEventDestroy(e);
    if (E->stream) (void)hipStreamDestroy(E->stream);
    delete E;
}

int32_t engine_create(int cap, int maxR, int restart, int64_t budget, Engine **out) {
    *out = nullptr;
    if (cap < 1 || cap > 65535 || maxR < 1 || maxR > 65535 || restart < 1 || budget <= 0) return HKG_EINVAL;
    if (restart > 4 * BROWS) {
        set_last_error("restart too large for the batched kernels");
        return HKG_EINVAL;
    }
    Engine *E = new Engine();
    E->cap = cap;
    E->maxR = maxR;
    E->restart = restart;
    E->budget = budget;
    E->table.assign(cap, ProbDev{});
    E->slot_req.assign(cap, nullptr);
    int32_t st = HKG_OK;
    if (hipStreamCreateWithFlags(&E->stream, hipStreamNonBlocking) != hipSuccess) {
        E->stream = nullptr;
        st = HKG_EHIP;
    }
    if (st == HKG_OK && hipHostMalloc((void **)&E->h_state, (size_t)cap * maxR * sizeof(int32_t)) != hipSuccess) {
        E->h_state = nullptr;
        st = HKG_ENOMEM;
    }
    if (st == HKG_OK) st = dalloc(&E->acct, &E->d_state, (size_t)cap * maxR * sizeof(int32_t));
    if (st == HKG_OK && hipMemsetAsync(E->d_state.p, 0, E->d_state.bytes, E->stream) != hipSuccess) st = HKG_EHIP;
    if (st == HKG_OK) st = upload_bytes(&E->acct, &E->d_probs, E->table.data(), cap * sizeof(ProbDev), E->stream, true);
    if (st != HKG_OK) {
        engine_free(E);
        return st;
    }
    *out = E;
    return HKG_OK;
}

int32_t check_request(const Engine *E, const hkgeneo_ctx *c, const double *f, const double *u, int nrhs, int ld) {
    if (!c || !f || !u || nrhs < 1 || nrhs > E->maxR || ld < c->n_dof) return HKG_EINVAL;
    if (c->opt.restart != E->restart) {
        set_last_error("the context's restart length differs from the engine's");
        return HKG_EINVAL;
    }
    if ((size_t)2 * c->max_nI * sizeof(double) + 16 * LTILE * sizeof(double) > 160 * 1024) {
        set_last_error("subdomain too large for the batched local solve");
        return HKG_EINVAL;
    }
    if (ws_bytes(c, nrhs, E->restart) > E->budget) {
        set_last_error("the request's workspace exceeds the engine's budget");
        return HKG_ENOMEM;
    }
    return HKG_OK;
}

int32_t submit(Engine *E, hkgeneo_ctx *c, const double *f, double *u, int nrhs, int ld, int64_t tag, hipStream_t s) {
    HKG_TRY(check_request(E, c, f, u, nrhs, ld));
    Request *q = new Request();
    q->ctx = c;
    q->nrhs = nrhs;
    q->ld = ld;
    q->f = f;
    q->u = u;
    q->tag = tag;
    if (hipEventCreateWithFlags(&q->ready, hipEventDisableTiming) != hipSuccess) {
        delete q;
        set_last_error("event for a submitted request");
        return HKG_EHIP;
    }
    if (hipEventRecord(q->ready, s) != hipSuccess) {
        (void)hipEventDestroy(q->ready);
        delete q;
        set_last_error("event for a submitted request");
        return HKG_EHIP;
    }
    E->queue.push_back(q);
    return HKG_OK;
}

}  // namespace

// ------------------------------------------------------------------------------------------------
// fixed batch
// ------------------------------------------------------------------------------------------------
struct hkgeneo_batch {
    Engine *E = nullptr;
    std::vector<hkgeneo_ctx *> ctx;
    std::vector<int> nrhs;
};

extern "C" int32_t hkgeneo_batch_create(hkgeneo_ctx *const *ctxs, const int32_t *nrhs, int32_t nprob,
                                        hkgeneo_batch **out) {
    if (!ctxs || !nrhs || !out || nprob < 1) return HKG_EINVAL;
    *out = nullptr;
    int maxR = 0;
    for (int p = 0; p < nprob; ++p) {
        if (!ctxs[p] || nrhs[p] < 1 || nrhs[p] > 65535 || ctxs[p]->opt.restart != ctxs[0]->opt.restart ||
            ctxs[p]->opt.krylov != HKG_KRYLOV_RIGHT || ctxs[p]->fine) {
            set_last_error("batch: every problem needs a context (flexible GMRES), 1..65535 right-hand sides and "
                           "the same restart");
            return HKG_EINVAL;
        }
        maxR = std::max(maxR, (int)nrhs[p]);
    }
    Engine *E = nullptr;
    HKG_TRY(engine_create(nprob, maxR, ctxs[0]->opt.restart, INT64_MAX / 4, &E));
    hkgeneo_batch *b = new hkgeneo_batch();
    b->E = E;
    b->ctx.assign(ctxs, ctxs + nprob);
    b->nrhs.assign(nrhs, nrhs + nprob);
    *out = b;
    return HKG_OK;
}

extern "C" int32_t hkgeneo_batch_solve(hkgeneo_batch *b, const double *const *f, double *const *u, const int32_t *ld,
                                       hkgeneo_rhs_info *info, void *stream) {
    if (!b || !f || !u || !ld) return HKG_EINVAL;
    Engine *E = b->E;
    const int np = (int)b->ctx.size();
    for (int p = 0; p < np; ++p) HKG_TRY(check_request(E, b->ctx[p], f[p], u[p], b->nrhs[p], ld[p]));
    for (int p = 0; p < np; ++p) HKG_TRY(submit(E, b->ctx[p], f[p], u[p], b->nrhs[p], ld[p], p, (hipStream_t)stream));
    int pending = 1;
    int32_t st = HKG_OK;
    while (pending > 0 && st == HKG_OK) st = pump_once(E, &pending);
    std::vector<int> off(np + 1, 0);
    for (int p = 0; p < np; ++p) off[p + 1] = off[p] + b->nrhs[p];
    int32_t status = HKG_OK;
    while (!E->done.empty()) {
        Done &d = E->done.front();
        if (d.status != HKG_OK) status = d.status;
        if (info) std::copy(d.info.begin(), d.info.end(), info + off[d.tag]);
        E->done.pop_front();
    }
    return st != HKG_OK ? st : status;
}

extern "C" int64_t hkgeneo_batch_bytes(const hkgeneo_batch *b) { return b ? b->E->acct.device_bytes : 0; }

extern "C" int32_t hkgeneo_batch_local_waves(const hkgeneo_batch *b) { return b ? b->E->geom.local_waves : 0; }

extern "C" int32_t hkgeneo_batch_profile(hkgeneo_batch *b, int32_t enable) {
    if (!b) return HKG_EINVAL;
    Engine *E = b->E;
    HKG_HIP(hipStreamSynchronize(E->stream));
    E->prof = enable != 0;
    if (E->prof) E->ev_used = 0;
    return HKG_OK;
}

extern "C" int32_t hkgeneo_batch_profile_read(hkgeneo_batch *b, double *total_ms, int64_t *launches) {
    if (!b || !total_ms || !launches) return HKG_EINVAL;
    Engine *E = b->E;
    HKG_HIP(hipStreamSynchronize(E->stream));
    double t = 0.0;
    for (size_t k = 0; k + 1 < E->ev_used; k += 2) {
        float ms = 0.0f;
        HKG_HIP(hipEventElapsedTime(&ms, E->ev[k], E->ev[k + 1]));
        t += ms;
    }
    *total_ms = t;
    *launches = (int64_t)(E->ev_used / 2);
    return HKG_OK;
}

extern "C" void hkgeneo_batch_destroy(hkgeneo_batch *b) {
    if (!b) return;
    engine_free(b->E);
    delete b;
}

// ------------------------------------------------------------------------------------------------
// server: requests join and leave at iteration boundaries
// ------------------------------------------------------------------------------------------------
extern "C" int32_t hkgeneo_server_create(int64_t workspace_budget, int32_t max_requests, int32_t max_nrhs,
                                         int32_t restart, hkgeneo_server **out) {
    if (!out) return HKG_EINVAL;
    *out = nullptr;
    return engine_create(max_requests, max_nrhs, restart, workspace_budget, out);
}

extern "C" int32_t hkgeneo_server_submit(hkgeneo_server *s, hkgeneo_ctx *ctx, const double *f, double *u,
                                         int32_t nrhs, int32_t ld, int64_t tag, void *stream) {
    if (!s || !ctx || ctx->opt.krylov != HKG_KRYLOV_RIGHT || ctx->fine) return HKG_EINVAL;
    return submit(s, ctx, f, u, nrhs, ld, tag, (hipStream_t)stream);
}

extern "C" int32_t hkgeneo_server_pump(hkgeneo_server *s, int32_t periods, int32_t *pending) {
    if (!s || periods < 1) return HKG_EINVAL;
    int n = 0;
    for (int k = 0; k < periods; ++k) {
        HKG_TRY(pump_once(s, &n));
        if (n == 0) break;
    }
    if (pending) *pending = n;
    return HKG_OK;
}

extern "C" int32_t hkgeneo_server_poll(hkgeneo_server *s, int64_t *tag, int32_t *status, hkgeneo_rhs_info *info,
                                       int32_t cap) {
    if (!s || !tag || !status) return HKG_EINVAL;
    if (s->done.empty()) return 0;
    Done &d = s->done.front();
    if (info && cap < (int)d.info.size()) return HKG_EINVAL;
    *tag = d.tag;
    *status = d.status;
    if (info) std::copy(d.info.begin(), d.info.end(), info);
    const int n = (int)d.info.size();
    s->done.pop_front();
    return n;
}

extern "C" int32_t hkgeneo_server_query(const hkgeneo_server *s, hkgeneo_server_stats *out) {
    if (!s || !out) return HKG_EINVAL;
    std::memset(out, 0, sizeof(*out));
    out->queued = (int32_t)s->queue.size();
    for (int k = 0; k < s->cap; ++k)
        if (s->slot_req[k]) {
            out->live++;
            out->live_rhs += s->slot_req[k]->nrhs;
        }
    out->completed_waiting = (int32_t)s->done.size();
    out->local_waves = s->geom.local_waves;
    out->workspace_bytes = s->ws_in_use;
    out->device_bytes = s->acct.device_bytes;
    out->iterations = s->n_iter_launch;
    out->restarts = s->n_restart_launch;
    out->captures = s->n_capture;
    out->admitted = s->n_admitted;
    out->retired = s->n_retired;
    return HKG_OK;
}

extern "C" void hkgeneo_server_destroy(hkgeneo_server *s) { engine_free(s); }
