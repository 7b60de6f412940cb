"""GPU: continuous batching (hkgeneo_server_*).

Requests join the live set while others iterate, leave it when their right-hand sides stop, and
are admitted only while the workspace budget allows.  Each result must be bitwise the same as the
same request solved alone (the per-pair arithmetic does not depend on the rest of the live set or on
when the pair joined), and must meet the FP64 oracle's bar (true relative residual <= 1e-8,
solution within 1e-8 of the oracle's, iterations within 2).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2406_06283_amd import hkgeneo as H  # noqa: E402
from paper_2406_06283_amd import problems as pb  # noqa: E402
from oracle import fgmres, local, schwarz  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(msg):
    print(msg, flush=True)


REQS = [
    (dict(N=16, k=6.0, s=2, overlap=1, coef="cells", seed=3, n_cells=4, rhs="normal", nrhs=2), dict(nev=3)),
    (dict(N=28, k=10.0, s=4, overlap=2, coef="lognormal", seed=2, rhs="normal", nrhs=1), dict(nev=5)),
    (dict(N=20, k=7.0, s=3, overlap=[1, 2, 3, 1, 2, 3, 2, 1, 1], coef="cells", seed=5, n_cells=5, rhs="normal",
          nrhs=3), dict(nev=4)),
    (dict(N=24, k=8.0, s=4, overlap=2, coef="cells", seed=8, n_cells=4, rhs="normal", nrhs=2),
     dict(nev=4, local_prec=32)),
]


def _make(pkw):
    pkw = dict(pkw)
    N = pkw.pop("N")
    return pb.make_problem(N, **pkw)


def _alone(S, f, with_bytes=False):
    with H.Server(1 << 34, max_requests=1, max_nrhs=8) as srv:
        srv.submit(S, f, tag=0)
        while srv.pump(8):
            pass
        ((_, u, info, st),) = srv.poll()
        ws = srv.stats()["workspace_bytes"]      # the retired request's buffer, kept for reuse
        torch.cuda.synchronize()
        return (u.clone(), info, st, ws) if with_bytes else (u.clone(), info, st)


def test_server_join_mid_flight_equals_alone_and_oracle():
    probs = [_make(p) for p, _ in REQS]
    solvers = [H.Solver(p, H.default_options(eig_mode=H.HKG_EIG_FIXED, **o)) for p, (_, o) in zip(probs, REQS)]
    try:
        fs = [torch.from_numpy(np.ascontiguousarray(p.f)).to(DEV) for p in probs]
        res = {}
        with H.Server(1 << 34, max_requests=8, max_nrhs=8) as srv:
            _say("[server] two requests, then two more while they iterate")
            srv.submit(solvers[0], fs[0], tag=0)
            srv.submit(solvers[1], fs[1], tag=1)
            srv.pump(2)
            srv.submit(solvers[2], fs[2], tag=2)
            srv.pump(1)
            srv.submit(solvers[3], fs[3], tag=3)
            while srv.pump(4):
                for tag, u, info, st in srv.poll():
                    res[tag] = (u, info, st)
            for tag, u, info, st in srv.poll():
                res[tag] = (u, info, st)
            stats = srv.stats()
        torch.cuda.synchronize()
        assert sorted(res) == [0, 1, 2, 3]
        assert stats["admitted"] == 4 and stats["retired"] == 4 and stats["live"] == 0
        assert stats["captures"] >= 4
        for q, p in enumerate(probs):
            _say(f"[server] request {q}: alone vs mix, oracle")
            u, info, st = res[q]
            ua, ia, _ = _alone(solvers[q], fs[q])
            assert torch.equal(u, ua), q
            assert [i["iters"] for i in info] == [i["iters"] for i in ia]
            o = dict(REQS[q][1])
            o.pop("local_prec", None)
            M = schwarz.TwoLevelSchwarz(p, schwarz.Options(eig_mode=local.EIG_FIXED, **o))
            U = u.cpu().numpy()
            for r in range(p.f.shape[0]):
                x, oinfo = fgmres.solve(p, M, f=p.f[r])
                rel = np.linalg.norm(p.f[r] - M.B @ U[r]) / np.linalg.norm(p.f[r])
                assert info[r]["converged"] and rel <= 1e-8 and abs(info[r]["relres_true"] - rel) <= 1e-9
                assert abs(info[r]["iters"] - oinfo["iters"]) <= 2, (q, r, info[r]["iters"], oinfo["iters"])
                assert np.linalg.norm(U[r] - x) / np.linalg.norm(x) <= 1e-8
    finally:
        for S in solvers:
            S.close()


def test_server_budget_admits_one_at_a_time():
    _say("[server] workspace budget for one request at a time")
    probs = [_make(p) for p, _ in REQS[:3]]
    solvers = [H.Solver(p, H.default_options(eig_mode=H.HKG_EIG_FIXED, **o)) for p, (_, o) in zip(probs, REQS)]
    try:
        fs = [torch.from_numpy(np.ascontiguousarray(p.f)).to(DEV) for p in probs]
        alone = [_alone(solvers[q], fs[q], with_bytes=True) for q in range(3)]
        ws = [a[3] for a in alone]
        # the largest single workspace is below the sum of any two: one request live at a time
        budget = max(ws)
        assert budget < sorted(ws)[0] + sorted(ws)[1]
        live_max = 0
        res = {}
        with H.Server(budget, max_requests=8, max_nrhs=8) as srv:
            for q in range(3):
                srv.submit(solvers[q], fs[q], tag=q)
            while True:
                pending = srv.pump(1)
                live_max = max(live_max, srv.stats()["live"])
                for tag, u, info, st in srv.poll():
                    res[tag] = (u, info, st)
                if pending == 0:
                    break
            for tag, u, info, st in srv.poll():
                res[tag] = (u, info, st)
        torch.cuda.synchronize()
        assert sorted(res) == [0, 1, 2]
        for q in range(3):
            assert torch.equal(res[q][0], alone[q][0])
            assert all(i["converged"] for i in res[q][1])
        assert live_max == 1
    finally:
        for S in solvers:
            S.close()


def test_server_rejects_oversized_request():
    _say("[server] request larger than the budget")
    p = _make(REQS[0][0])
    with H.Solver(p, H.default_options(eig_mode=H.HKG_EIG_FIXED, nev=3)) as S, \
            H.Server(1024, max_requests=2, max_nrhs=8) as srv:
        f = torch.from_numpy(np.ascontiguousarray(p.f)).to(DEV)
        with pytest.raises(H.HkgError) as e:
            srv.submit(S, f, tag=0)
        assert e.value.status == H.HKG_ENOMEM
