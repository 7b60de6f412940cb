"""Pins for the oracle's one- and two-level preconditioner (eqs. 2.22, 2.23) and its FGMRES."""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_2406_06283_amd import problems as pb
from oracle import decomposition as dec
from oracle import fgmres, local, reference, schwarz


def _M(p, **kw):
    return schwarz.TwoLevelSchwarz(p, schwarz.Options(**kw))


def test_single_subdomain_coarse_matrix_is_diagonal_of_eigenvalues():
    # N = 1: Z = P[:, :m] with P^T D_k P = I and B P = D_k P diag(lambda), so B_0 = diag(lambda_1..m).
    p = pb.make_problem(10, k=12.0, s=1, overlap=1, coef="cells", seed=3, n_cells=5)
    M = _M(p, eig_mode=local.EIG_FIXED, nev=6)
    assert M.m == [M.m0] and M.m0 >= 6
    np.testing.assert_allclose(M.B0, np.diag(M.eigvals[0][:M.m0]), atol=1e-11)


def test_single_subdomain_one_level_is_exact_inverse():
    p = pb.make_problem(8, k=9.0, s=1, overlap=1)
    M = _M(p, two_level=False)
    np.testing.assert_allclose(M.dense() @ M.B.toarray(), np.eye(p.n_dof), atol=1e-10)


def test_additive_preconditioner_is_symmetric():
    p = pb.make_problem(8, k=11.0, s=2, overlap=1, coef="cells", seed=1, n_cells=4)
    Minv = _M(p, eig_mode=local.EIG_FIXED, nev=3).dense()
    np.testing.assert_allclose(Minv, Minv.T, atol=1e-10 * np.abs(Minv).max())
    Mpou = _M(p, eig_mode=local.EIG_FIXED, nev=3, prolong=schwarz.PROLONG_POU).dense()
    assert np.abs(Mpou - Mpou.T).max() > 1e-6 * np.abs(Mpou).max()     # the weighted one is not


def test_dense_operator_from_boolean_matrices():
    # M^{-1} = sum_D R_D^T (R_D B R_D^T)^{-1} R_D + Z (Z^T B Z)^{-1} Z^T with explicit Boolean R_D.
    p = pb.make_problem(8, k=7.0, s=2, overlap=2, coef="lognormal", seed=4)
    M = _M(p, eig_mode=local.EIG_FIXED, nev=2)
    B = M.B.toarray()
    ref = np.zeros_like(B)
    for s in M.subs:
        R = dec.restriction_matrix(s.dof, p.n_dof).toarray()
        ref += R.T @ np.linalg.inv(R @ B @ R.T) @ R
    Z = M.Z.toarray()
    ref += Z @ np.linalg.inv(Z.T @ B @ Z) @ Z.T
    np.testing.assert_allclose(M.dense(), ref, atol=1e-10 * np.abs(ref).max())


def test_coarse_correction_invariant_under_basis_change():
    # Z B_0^{-1} Z^T with B_0 = Z^T B Z depends on span(Z) only: replacing Z by Z G (G invertible)
    # leaves it unchanged.  A transposed or missing factor in B_0 would break this.
    p = pb.make_problem(12, k=8.0, s=2, overlap=1, coef="cells", seed=2, n_cells=4)
    M = _M(p, eig_mode=local.EIG_FIXED, nev=4)
    B = M.B.toarray()
    Z = M.Z.toarray()
    G = np.random.default_rng(0).standard_normal((M.m0, M.m0)) + 3 * np.eye(M.m0)
    ZG = Z @ G
    c1 = Z @ np.linalg.solve(M.B0, Z.T)
    c2 = ZG @ np.linalg.solve(ZG.T @ B @ ZG, ZG.T)
    np.testing.assert_allclose(c1, c2, atol=1e-9 * np.abs(c1).max())


def test_coarse_basis_is_pou_weighted_eigenvectors():
    # Def 2.15: the coarse vectors are E_i Xi_i p, i.e. p/mu on dof(D_i) and zero elsewhere.
    p = pb.make_problem(12, k=8.0, s=3, overlap=2)
    M = _M(p, eig_mode=local.EIG_FIXED, nev=3)
    off = 0
    for s, Zi, m in zip(M.subs, M.Z_local, M.m):
        Bt, C = local.geneo_pencil(p, s, M.mu)
        _, P = local.geneo_eigenpairs(Bt, C, s.dof.size)
        block = M.Z.toarray()[:, off:off + m]
        np.testing.assert_allclose(block[s.dof], P[:, :m] / M.mu[s.dof][:, None], atol=1e-14)
        mask = np.ones(p.n_dof, bool); mask[s.dof] = False
        assert np.all(block[mask] == 0)
        off += m


# ------------------------------------------------------------------------------------------------
# FGMRES
# ------------------------------------------------------------------------------------------------

def test_fgmres_dense_solve_unpreconditioned():
    rng = np.random.default_rng(3)
    n = 40
    A = rng.standard_normal((n, n)) + 8 * np.eye(n)
    b = rng.standard_normal(n)
    x, info = fgmres.fgmres(lambda v: A @ v, lambda v: v, b, restart=60, tol=1e-12)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9)
    assert info["iters"] <= n and info["converged"]


def test_fgmres_zero_rhs_and_exact_preconditioner():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((20, 20)) + 6 * np.eye(20)
    x, info = fgmres.fgmres(lambda v: A @ v, lambda v: v, np.zeros(20))
    assert info["iters"] == 0 and np.all(x == 0)
    Ainv = np.linalg.inv(A)
    b = rng.standard_normal(20)
    x, info = fgmres.fgmres(lambda v: A @ v, lambda v: Ainv @ v, b)
    assert info["iters"] == 1 and info["relres_true"] < 1e-12


def test_fgmres_restarts_and_monotone_history():
    rng = np.random.default_rng(5)
    n = 60
    A = np.diag(np.linspace(1, 10, n)) + 0.1 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    x, info = fgmres.fgmres(lambda v: A @ v, lambda v: v, b, restart=5, tol=1e-10, max_iter=2000)
    assert info["converged"] and info["cycles"] > 1
    h = np.array(info["history"])
    for c in range(0, len(h), 5):                    # the recurrence residual never grows in a cycle
        seg = h[c:c + 5]
        assert np.all(np.diff(seg) <= 1e-15)


def test_two_level_single_subdomain_converges_in_two_steps():
    # N = 1: M^{-1} B = I + Z B_0^{-1} Z^T B has eigenvalues {1, 2} only, so GMRES ends in 2 steps.
    p = pb.make_problem(10, k=10.0, s=1, overlap=1)
    M = _M(p, eig_mode=local.EIG_FIXED, nev=4)
    x, info = fgmres.solve(p, M, tol=1e-10)
    assert info["iters"] == 2
    np.testing.assert_allclose(x, reference.direct_solve(p)[0], rtol=1e-8)


def test_near_resonant_h32_configuration():
    # h = 1/32, A = I, k = 10, 4 x 4 blocks, 2 layers, 10 eigenvectors per subdomain.
    p = pb.make_problem(32, k=10.0, s=4, overlap=2)
    M = _M(p, eig_mode=local.EIG_FIXED, nev=10)
    assert M.m0 == 160 and M.Lambda == 4
    x, info = fgmres.solve(p, M)
    assert info["converged"] and info["relres_true"] <= 1e-8
    u = reference.direct_solve(p)[0]
    B = M.B.toarray()
    kappa = np.linalg.cond(B)
    assert np.linalg.norm(x - u) / np.linalg.norm(u) <= kappa * 1e-8
    # tight tolerance: the solution itself to 1e-8
    x2, info2 = fgmres.solve(p, M, tol=1e-13)
    assert np.linalg.norm(x2 - u) / np.linalg.norm(u) <= 1e-8


def test_one_level_zero_overlap_rejected():
    p = pb.make_problem(8, s=2, overlap=0)
    with pytest.raises(ValueError):
        _M(p)
