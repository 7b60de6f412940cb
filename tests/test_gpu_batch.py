"""GPU: batched solves (several problems of different sizes in one launch sequence per phase).

Every problem of a batch must give bitwise the same iterates alone and in a mix (the batched
kernels add in an order fixed by the problem alone, whatever the batch composition and the local
solve launch shape), and each must match the FP64 CPU oracle to the same bar as the single-problem
path: true relative residual <= 1e-8, solution within 1e-8 of the oracle's, iterations within 2.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2406_06283_amd import hkgeneo as H  # noqa: E402
from paper_2406_06283_amd import problems as pb  # noqa: E402
from paper_2406_06283_amd.configs import H32_K10  # noqa: E402
from oracle import fgmres, local, schwarz  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(msg):
    print(msg, flush=True)


# uneven problems: sizes, subdomain grids, overlaps (one non-uniform), coefficients, one-level,
# float32 local inverses, a 3D Q1 mesh; 1-3 right-hand sides each
MIX = [
    ("p1_n16_s2_k6", dict(N=16, k=6.0, s=2, overlap=1, coef="cells", seed=3, n_cells=4, rhs="normal", nrhs=2),
     dict(nev=3)),
    ("p1_n28_s4_k10_lognormal", dict(N=28, k=10.0, s=4, overlap=2, coef="lognormal", seed=2, rhs="normal", nrhs=1),
     dict(nev=5)),
    ("p1_n20_s3_uneven", dict(N=20, k=7.0, s=3, overlap=[1, 2, 3, 1, 2, 3, 2, 1, 1], coef="cells", seed=5, n_cells=5,
                              rhs="normal", nrhs=3), dict(nev=4)),
    ("p1_n24_s3_onelevel", dict(N=24, k=5.0, s=3, overlap=2, coef="cells", seed=7, n_cells=4, rhs="normal", nrhs=1),
     dict(nev=4, two_level=0)),
    ("p1_n24_s4_fp32", dict(N=24, k=8.0, s=4, overlap=2, coef="cells", seed=8, n_cells=4, rhs="normal", nrhs=2),
     dict(nev=4, local_prec=32)),
    ("q1_3d_n8_s2", dict(N=8, dim=3, elem_type=pb.Q1, k=4.0, s=2, overlap=1, coef="cells", seed=1, n_cells=3,
                         rhs="normal", nrhs=1), dict(nev=3)),
]


def _make(pkw):
    pkw = dict(pkw)
    N = pkw.pop("N")
    return pb.make_problem(N, **pkw)


def _solvers(probs, okws):
    return [H.Solver(p, H.default_options(eig_mode=H.HKG_EIG_FIXED, **okw)) for p, okw in zip(probs, okws)]


def _rhs(p):
    return torch.from_numpy(np.ascontiguousarray(p.f)).to(DEV)


def test_batch_of_one_matches_oracle():
    _say("[batch] h=1/32 k=10 4x4 nev=10, batch of one")
    p = H32_K10.problem()
    M = schwarz.TwoLevelSchwarz(p, schwarz.Options(eig_mode=local.EIG_FIXED, nev=10))
    x, oinfo = fgmres.solve(p, M)
    with H.Solver(p, H.options_for(H32_K10)) as S, H.Batch([S], [1]) as B:
        (u,), (info,), st = B.solve([_rhs(p)])
        torch.cuda.synchronize()
        u = u.cpu().numpy()[0]
    assert st == H.HKG_OK and info[0]["converged"]
    assert abs(info[0]["iters"] - oinfo["iters"]) <= 2, (info[0]["iters"], oinfo["iters"])
    assert np.linalg.norm(p.f[0] - M.B @ u) / np.linalg.norm(p.f[0]) <= 1e-8
    assert np.linalg.norm(u - x) / np.linalg.norm(x) <= 1e-8


_INPUTS = ("elem_vert", "vert_dof", "elem_K", "elem_M", "row_ptr", "col_idx", "A_val", "S_val", "elem_part", "overlap",
           "f")


def _snapshot(p):
    return {k: np.array(getattr(p, k), copy=True) for k in _INPUTS}


def _assert_inputs_unchanged(p, snap, name):
    # the library reads its host inputs and never writes them
    for k, v in snap.items():
        now = np.asarray(getattr(p, k))
        if not np.array_equal(now, v):
            bad = np.flatnonzero(now.ravel() != v.ravel())
            raise AssertionError(f"{name}: host input {k} changed at {bad.size} entries, first {bad[:8].tolist()}: "
                                 f"{v.ravel()[bad[:4]].tolist()} -> {now.ravel()[bad[:4]].tolist()}")


def test_batch_mix_equals_alone_and_matches_oracle():
    probs = [_make(c[1]) for c in MIX]
    snaps = [_snapshot(p) for p in probs]
    okws = [c[2] for c in MIX]
    solvers = _solvers(probs, okws)
    try:
        fs = [_rhs(p) for p in probs]
        _say("[batch] mix of " + ", ".join(c[0] for c in MIX))
        with H.Batch(solvers, [p.f.shape[0] for p in probs]) as B:
            assert B.local_waves in (4, 8, 16)
            um, im, st = B.solve(fs)
            torch.cuda.synchronize()
            um = [u.clone() for u in um]
        for q, (name, _, okw) in enumerate(MIX):
            _say(f"[batch] alone: {name}")
            with H.Batch([solvers[q]], [probs[q].f.shape[0]]) as B1:
                (ua,), (ia,), _ = B1.solve([fs[q]])
                torch.cuda.synchronize()
            assert torch.equal(ua, um[q]), name
            assert [i["iters"] for i in ia] == [i["iters"] for i in im[q]], name
            # against the oracle, column by column
            p = probs[q]
            _assert_inputs_unchanged(p, snaps[q], name)
            o = dict(okw)
            two = bool(o.pop("two_level", 1))
            o.pop("local_prec", None)
            M = schwarz.TwoLevelSchwarz(p, schwarz.Options(eig_mode=local.EIG_FIXED, two_level=two, **o))
            U = um[q].cpu().numpy()
            for r in range(p.f.shape[0]):
                x, oinfo = fgmres.solve(p, M, f=p.f[r])
                rel = np.linalg.norm(p.f[r] - M.B @ U[r]) / np.linalg.norm(p.f[r])
                assert im[q][r]["converged"] and rel <= 1e-8, (name, r, rel)
                assert abs(im[q][r]["iters"] - oinfo["iters"]) <= 2, (name, r, im[q][r]["iters"], oinfo["iters"])
                assert np.linalg.norm(U[r] - x) / np.linalg.norm(x) <= 1e-8, (name, r)
        assert st == H.HKG_OK
    finally:
        for S in solvers:
            S.close()


def test_batch_refactor_and_zero_rhs():
    _say("[batch] refactor between solves; zero right-hand side in the mix")
    p1 = pb.make_problem(20, k=7.0, s=2, overlap=2, coef="lognormal", seed=4, rhs="normal", nrhs=2)
    p2 = pb.make_problem(16, k=5.0, s=2, overlap=1, coef="cells", seed=6, n_cells=4)
    S1 = H.Solver(p1, H.default_options(eig_mode=H.HKG_EIG_FIXED, nev=4, keep_workspace=1))
    S2 = H.Solver(p2, H.default_options(eig_mode=H.HKG_EIG_FIXED, nev=3))
    try:
        f1 = _rhs(p1)
        f1[1].zero_()
        f2 = _rhs(p2)
        with H.Batch([S1, S2], [2, 1]) as B:
            ua, ia, _ = B.solve([f1, f2])
            torch.cuda.synchronize()
            ua = [u.clone() for u in ua]
            S1.factor()
            ub, ib, _ = B.solve([f1, f2])
            torch.cuda.synchronize()
        assert torch.equal(ua[0], ub[0]) and torch.equal(ua[1], ub[1])
        assert ia[0][1]["iters"] == 0 and float(ua[0][1].abs().max()) == 0.0
        assert ia[0][0]["converged"] and ia[1][0]["converged"]
    finally:
        S1.close()
        S2.close()


def test_batch_rejects_different_restart():
    _say("[batch] invalid: different restart lengths")
    p = pb.make_problem(12, k=4.0, s=2, overlap=1)
    with H.Solver(p, H.default_options(eig_mode=H.HKG_EIG_FIXED, nev=2)) as S1, \
            H.Solver(p, H.default_options(eig_mode=H.HKG_EIG_FIXED, nev=2, restart=30)) as S2:
        with pytest.raises(H.HkgError) as e:
            H.Batch([S1, S2], [1, 1])
        assert e.value.status == H.HKG_EINVAL


@pytest.mark.parametrize("restart", [8, 150])
def test_batch_restarted_cycles_match_oracle(restart):
    # restart = 8: every right-hand side needs several cycles, so the device-side restart phase
    # (x update from the cycle's triangle, true residual, next cycle) runs repeatedly; 150: the
    # long-restart sizes of the restart kernels
    _say(f"[batch] FGMRES({restart}) cycles vs oracle")
    p = pb.make_problem(20, k=7.0, s=3, overlap=2, coef="cells", seed=9, n_cells=4, rhs="normal", nrhs=2)
    M = schwarz.TwoLevelSchwarz(p, schwarz.Options(eig_mode=local.EIG_FIXED, nev=4))
    with H.Solver(p, H.default_options(eig_mode=H.HKG_EIG_FIXED, nev=4, restart=restart)) as S, \
            H.Batch([S], [2]) as B:
        (u,), (info,), st = B.solve([_rhs(p)])
        us, infos, _ = S.solve(_rhs(p))
        torch.cuda.synchronize()
        U, Us = u.cpu().numpy(), us.cpu().numpy()
    assert st == H.HKG_OK
    for r in range(2):
        x, oinfo = fgmres.solve(p, M, f=p.f[r], restart=restart)
        assert info[r]["converged"] and abs(info[r]["iters"] - oinfo["iters"]) <= 2, (info[r]["iters"], oinfo["iters"])
        assert abs(info[r]["iters"] - infos[r]["iters"]) <= 1
        assert np.linalg.norm(p.f[r] - M.B @ U[r]) / np.linalg.norm(p.f[r]) <= 1e-8
        assert np.linalg.norm(U[r] - x) / np.linalg.norm(x) <= 1e-8
        assert np.linalg.norm(U[r] - Us[r]) / np.linalg.norm(Us[r]) <= 1e-8
    if restart == 8:
        assert min(i["iters"] for i in info) > 2 * restart


def test_batch_of_24_uneven_problems_matches_oracle():
    # the batched-mix generator at small sizes: h in {1/24, ..., 1/48}, k = 0.3/h, 2x2 to 6x6 blocks
    # with overlaps drawn per subdomain from {1, 2, 3}, both coefficient fields, 1-4 right-hand sides
    # (67 in all), threshold selection; float32 local inverses in every other problem
    from paper_2406_06283_amd.configs import batch_mix, mix_options
    mix = batch_mix(24, seed0=1000, n_choices=(24, 32, 40, 48), s_range=(2, 6), nrhs_range=(1, 4), max_block=None)
    probs = [m.problem() for m in mix]
    solvers = [H.Solver(p, H.default_options(**mix_options(m, local_prec=32 if q % 2 == 0 else 64)))
               for q, (m, p) in enumerate(zip(mix, probs))]
    try:
        fs = [_rhs(p) for p in probs]
        _say(f"[batch] 24 problems, {sum(p.f.shape[0] for p in probs)} right-hand sides")
        with H.Batch(solvers, [p.f.shape[0] for p in probs]) as B:
            um, im, st = B.solve(fs)
            torch.cuda.synchronize()
            um = [u.cpu().numpy() for u in um]
        assert st == H.HKG_OK
        for q in (0, 11, 23):
            with H.Batch([solvers[q]], [probs[q].f.shape[0]]) as B1:
                (ua,), (ia,), _ = B1.solve([fs[q]])
                torch.cuda.synchronize()
            assert np.array_equal(ua.cpu().numpy(), um[q]), mix[q].name
            assert [i["iters"] for i in ia] == [i["iters"] for i in im[q]], mix[q].name
        # the coarse product reads paired entries for even m_0 and single ones for odd m_0: both occur
        assert {S.stats()["m0"] % 2 for S in solvers} == {0, 1}
        worst = 0.0
        for q, (m, p, S) in enumerate(zip(mix, probs, solvers)):
            M = schwarz.TwoLevelSchwarz(p, schwarz.Options(eig_mode=local.EIG_THRESHOLD, tau=m.tau))
            assert S.stats()["m0"] == M.m0 and list(S.subdomains()[2]) == M.m, m.name
            for r in range(p.f.shape[0]):
                x, oinfo = fgmres.solve(p, M, f=p.f[r], restart=200)
                rel = np.linalg.norm(p.f[r] - M.B @ um[q][r]) / np.linalg.norm(p.f[r])
                assert im[q][r]["converged"] and rel <= 1e-8, (m.name, r, rel)
                assert abs(im[q][r]["iters"] - oinfo["iters"]) <= 2, (m.name, r, im[q][r]["iters"], oinfo["iters"])
                err = np.linalg.norm(um[q][r] - x) / np.linalg.norm(x)
                if q % 2 == 1:          # float64 local inverses: the same iterates up to rounding
                    assert err <= 1e-8, (m.name, r, err)
                worst = max(worst, err)
        _say(f"[batch] every right-hand side within the bars; largest solution difference {worst:.1e}")
    finally:
        for S in solvers:
            S.close()
