"""GPU: the serving loop (paper_2406_06283_amd.serve) end to end on a short request stream.

Requests for a few problem keys arrive by a Poisson schedule; misses are set up on the side
thread while other requests iterate, hits reuse the resident contexts, and the server batches
everything that is live.  Each request's solution must be bitwise the one the same context gives
for the same right-hand sides alone, and every right-hand side must reach the 1e-8 residual.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2406_06283_amd import hkgeneo as H  # noqa: E402
from paper_2406_06283_amd import problems as pb  # noqa: E402
from paper_2406_06283_amd import serve  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

KEYS = {
    "a": dict(N=16, k=6.0, s=2, overlap=1, coef="cells", seed=3, n_cells=4),
    "b": dict(N=24, k=8.0, s=3, overlap=2, coef="lognormal", seed=2),
    "c": dict(N=8, dim=3, elem_type=pb.Q1, k=4.0, s=2, overlap=1, coef="cells", seed=1, n_cells=3),
}
OPTS = dict(eig_mode=H.HKG_EIG_FIXED, nev=4, local_prec=32)


def _problem(key):
    kw = dict(KEYS[key])
    N = kw.pop("N")
    return pb.make_problem(N, **kw)


def test_serve_loop_results_equal_alone():
    print("[serve] 14 requests over 3 keys, Poisson arrivals", flush=True)
    problems = {k: _problem(k) for k in KEYS}
    rng = np.random.default_rng(5)
    arrivals = np.cumsum(rng.exponential(0.004, size=14))
    arrivals[10:] += 1.0        # the last four arrive once every setup has ended: cache hits
    reqs = []
    for q, t in enumerate(arrivals):
        key = "abc"[q % 3] if q < 6 else "abc"[int(rng.integers(0, 3))]
        p = problems[key]
        nrhs = int(rng.integers(1, 4))
        f = torch.from_numpy(rng.standard_normal((nrhs, p.n_dof))).to(DEV)
        reqs.append(serve.Request(tag=q, arrival=float(t), key=key, f=f))

    def make_solver(key, stream):
        return H.Solver(problems[key], H.default_options(**OPTS), stream=stream)

    cap = H.default_options(**OPTS).max_eig_per_sub

    def estimate(key):
        return serve.footprint_estimate(problems[key], 32, cap)

    cache = serve.ContextCache(8 << 30)
    try:
        done, summ = serve.run_stream(reqs, make_solver, estimate, ctx_budget=8 << 30, workspace_budget=1 << 30,
                                      max_requests=4, max_nrhs=8, cache=cache)
        assert summ["converged"] and summ["setups"] == 3 and summ["misses"] >= 3 and summ["hits"] >= 1
        # the reservation made at dispatch bounds every context's peak device bytes
        assert summ["reservation_overshoots"] == 0 and summ["over_budget_inserts"] == 0
        for r in done:
            assert all(i["relres_true"] <= 1e-8 for i in r.info)
            S = cache.acquire(r.key)
            with H.Batch([S], [r.f.shape[0]]) as B:
                (ua,), (ia,), _ = B.solve([r.f])
                torch.cuda.synchronize()
            cache.release(r.key)
            assert torch.equal(r.u, ua), r.tag
            assert [i["iters"] for i in ia] == [i["iters"] for i in r.info]
    finally:
        cache.close()
