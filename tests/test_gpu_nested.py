"""GPU parity for the nested decomposition of Sec. 2.3 (first-level subdomains inside the coarse ones).

The library builds the first-level subdomains itself (host, from the fine element partition and the
fine overlap) and runs the local solves of eq. (2.22) on them and the H_k-GenEO coarse space on the
coarse subdomains; the oracle does the same construction independently.  Bars as in test_gpu_parity:
index sets exact, apply within 1e-10 of max|z|, FGMRES solution within 1e-8 and iterations within 2.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2406_06283_amd import hkgeneo as H  # noqa: E402
from paper_2406_06283_amd import problems as pb  # noqa: E402
from oracle import fgmres, local, schwarz  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

CASES = [
    ("p1_n24_c3_f6", dict(N=24, k=9.0, s=3, overlap=2, coef="lognormal", seed=3, fine=6, fine_overlap=1), dict(nev=6)),
    ("p1_n32_c2_f8_ov2", dict(N=32, k=10.0, s=2, overlap=2, coef="cells", seed=4, n_cells=4, fine=8, fine_overlap=2),
     dict(nev=8)),
    ("q1_3d_n8_c2_f4", dict(N=8, dim=3, elem_type=pb.Q1, k=4.0, s=2, overlap=1, coef="cells", seed=1, n_cells=3, fine=4,
                            fine_overlap=1), dict(nev=4)),
]


def _say(msg):
    print(msg, flush=True)


def _make(pkw):
    pkw = dict(pkw)
    N = pkw.pop("N")
    return pb.make_problem(N, **pkw)


@pytest.mark.parametrize("name,pkw,okw", CASES, ids=[c[0] for c in CASES])
def test_nested_sets_apply_and_solve_match_oracle(name, pkw, okw):
    _say(f"[nested] {name}")
    p = _make(pkw)
    M = schwarz.TwoLevelSchwarz(p, schwarz.Options(eig_mode=local.EIG_FIXED, **okw))
    R = np.random.default_rng(21).standard_normal((2, p.n_dof))
    with H.Solver(p, H.default_options(eig_mode=H.HKG_EIG_FIXED, **okw)) as S:
        own, nI, lam = S.fine()
        assert list(own) == M.fine_owner and list(nI) == [s.dof.size for s in M.fine]
        assert lam == M.Lambda and S.stats()["lambda_overlap"] == M.Lambda
        assert S.stats()["m0"] == M.m0 and list(S.subdomains()[2]) == M.m
        r = torch.from_numpy(R).to(DEV)
        Zg = S.apply(r).cpu().numpy()
        f = torch.from_numpy(p.f).to(DEV)
        u, info, st = S.solve(f)
        torch.cuda.synchronize()
        u = u.cpu().numpy()[0]
        with pytest.raises(H.HkgError):
            H.Batch([S], [1])
    Zo = np.stack([M.apply(v) for v in R])
    scale = np.abs(Zo).max()
    assert np.abs(Zg - Zo).max() <= 1e-10 * scale, np.abs(Zg - Zo).max() / scale
    x, oinfo = fgmres.solve(p, M)
    assert st == H.HKG_OK and info[0]["converged"]
    assert abs(info[0]["iters"] - oinfo["iters"]) <= 2, (info[0]["iters"], oinfo["iters"])
    err = np.linalg.norm(u - x) / np.linalg.norm(x)
    plain = schwarz.TwoLevelSchwarz(_make({k: v for k, v in pkw.items() if k not in ("fine", "fine_overlap")}),
                                    schwarz.Options(eig_mode=local.EIG_FIXED, **okw))
    _, pinfo = fgmres.solve(p, plain)
    _say(f"  fine subdomains {len(M.fine)} (coarse {p.n_sub}), Lambda {M.Lambda}; iterations oracle "
         f"{oinfo['iters']} gpu {info[0]['iters']} (plain two-level {pinfo['iters']}); solution vs oracle {err:.2e}")
    assert err <= 1e-8


def test_nested_one_level_and_mixed_precision():
    p = _make(CASES[0][1])
    M = schwarz.TwoLevelSchwarz(p, schwarz.Options(eig_mode=local.EIG_FIXED, two_level=False, nev=6))
    R = np.random.default_rng(22).standard_normal((1, p.n_dof))
    with H.Solver(p, H.default_options(eig_mode=H.HKG_EIG_FIXED, nev=6, two_level=0)) as S:
        Zg = S.apply(torch.from_numpy(R).to(DEV)).cpu().numpy()
    Zo = M.apply(R[0])[None]
    assert np.abs(Zg - Zo).max() <= 1e-10 * np.abs(Zo).max()
    M2 = schwarz.TwoLevelSchwarz(p, schwarz.Options(eig_mode=local.EIG_FIXED, nev=6))
    x, oinfo = fgmres.solve(p, M2)
    with H.Solver(p, H.default_options(eig_mode=H.HKG_EIG_FIXED, nev=6, local_prec=32)) as S:
        u, info, st = S.solve(torch.from_numpy(p.f).to(DEV))
        u = u.cpu().numpy()[0]
    assert st == H.HKG_OK and abs(info[0]["iters"] - oinfo["iters"]) <= 2
    assert np.linalg.norm(p.f[0] - M2.B @ u) / np.linalg.norm(p.f[0]) <= 1e-8


def test_single_fine_block_matches_plain_decomposition():
    # Q_i = 1: the first-level subdomains are the coarse ones; the nested path (separate contexts)
    # and the fused path give the same operator up to rounding
    kw = dict(k=7.0, s=3, overlap=2, coef="cells", seed=2, n_cells=4)
    pn = pb.make_problem(24, fine=1, fine_overlap=1, **kw)
    pp = pb.make_problem(24, **kw)
    R = torch.from_numpy(np.random.default_rng(23).standard_normal((2, pp.n_dof))).to(DEV)
    opts = H.default_options(eig_mode=H.HKG_EIG_FIXED, nev=4)
    with H.Solver(pn, opts) as Sn, H.Solver(pp, opts) as Sp:
        own, nI, lam = Sn.fine()
        assert list(own) == list(range(pp.n_sub)) and list(nI) == list(Sp.subdomains()[0])
        zn = Sn.apply(R).cpu().numpy()
        zp = Sp.apply(R).cpu().numpy()
    np.testing.assert_allclose(zn, zp, rtol=0, atol=1e-12 * np.abs(zp).max())


def test_nested_pou_weights_and_dk_gmres():
    # PoU prolongation: W_D = diag(1/mu) with mu counted over the fine subdomains (Def 2.13 applied to the
    # subdomains of the local solves), while the coarse basis keeps Xi of the coarse subdomains (Def 2.15)
    pkw = CASES[0][1]
    p = _make(pkw)
    M = schwarz.TwoLevelSchwarz(p, schwarz.Options(eig_mode=local.EIG_FIXED, nev=6, prolong=schwarz.PROLONG_POU))
    R = np.random.default_rng(24).standard_normal((2, p.n_dof))
    with H.Solver(p, H.default_options(eig_mode=H.HKG_EIG_FIXED, nev=6, prolong=H.HKG_PROLONG_POU)) as S:
        Zg = S.apply(torch.from_numpy(R).to(DEV)).cpu().numpy()
    Zo = np.stack([M.apply(v) for v in R])
    assert np.abs(Zg - Zo).max() <= 1e-10 * np.abs(Zo).max()
    # GMRES on eq. 2.24 in the D_k inner product over the nested preconditioner
    Ma = schwarz.TwoLevelSchwarz(p, schwarz.Options(eig_mode=local.EIG_FIXED, nev=6))
    x, oinfo = fgmres.solve_left_dk(p, Ma, f=p.f[0], restart=30)
    opts = H.default_options(eig_mode=H.HKG_EIG_FIXED, nev=6, restart=30, krylov=H.HKG_KRYLOV_LEFT_DK)
    with H.Solver(p, opts) as S:
        u, info, st = S.solve(torch.from_numpy(p.f).to(DEV))
        u = u.cpu().numpy()[0]
    assert st == H.HKG_OK and info[0]["converged"] and oinfo["converged"]
    assert abs(info[0]["iters"] - oinfo["iters"]) <= 2, (info[0]["iters"], oinfo["iters"])
    err = np.linalg.norm(u - x) / np.linalg.norm(x)
    _say(f"[nested dk] iterations oracle {oinfo['iters']} gpu {info[0]['iters']}; solution vs oracle {err:.2e}")
    assert err <= 1e-8
