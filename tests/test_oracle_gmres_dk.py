"""Pins for the oracle's GMRES on the left-preconditioned system in the D_k inner product (eq. 2.24,
Prop 2.11, the setting of Theorem 3.1)."""
import numpy as np

from paper_2406_06283_amd import problems as pb
from oracle import fgmres, local, reference, schwarz


def _system(n=30, seed=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 4 * np.eye(n)
    P = np.linalg.inv(A + 0.8 * rng.standard_normal((n, n)))          # an inexact preconditioner
    G = rng.standard_normal((n, n))
    D = G @ G.T + n * np.eye(n)                                        # SPD inner-product matrix
    b = rng.standard_normal(n)
    return A, P, D, b


def test_residual_is_the_minimum_over_the_krylov_space_in_the_dk_norm():
    # GMRES in <.,.>_D minimises ||P (b - A x)||_D over x in K_m(PA, Pb): compare every step with
    # the minimum computed by brute force from an explicit Krylov basis and the Cholesky factor of D.
    A, P, D, b = _system()
    m = 12
    x, info = fgmres.gmres_left_dk(lambda v: A @ v, lambda v: P @ v, lambda v: D @ v, b, restart=40, tol=1e-30,
                                   max_iter=m)
    L = np.linalg.cholesky(D)
    r0 = P @ b
    ref = np.sqrt(r0 @ D @ r0)
    PA = P @ A
    K = np.zeros((b.size, m))
    v = r0.copy()
    for j in range(m):
        K[:, j] = v
        v = PA @ v
    Q, _ = np.linalg.qr(K)                      # the same space, well-conditioned columns
    for k in range(1, m + 1):
        Y = np.linalg.lstsq(L.T @ PA @ Q[:, :k], L.T @ r0, rcond=None)[0]
        best = np.linalg.norm(L.T @ (r0 - PA @ Q[:, :k] @ Y)) / ref
        assert abs(info["history"][k - 1] - best) <= 1e-9 * max(best, 1e-6), (k, info["history"][k - 1], best)
    # the recurrence estimate is the true preconditioned D-norm residual of the returned iterate
    rp = P @ (b - A @ x)
    assert abs(np.sqrt(rp @ D @ rp) / ref - info["history"][-1]) <= 1e-9


def test_exact_preconditioner_one_step_and_restarts_converge():
    A, P, D, b = _system(seed=1)
    Ainv = np.linalg.inv(A)
    x, info = fgmres.gmres_left_dk(lambda v: A @ v, lambda v: Ainv @ v, lambda v: D @ v, b)
    assert info["iters"] == 1 and info["relres_true"] < 1e-12
    x, info = fgmres.gmres_left_dk(lambda v: A @ v, lambda v: P @ v, lambda v: D @ v, b, restart=10, tol=1e-12)
    assert info["converged"] and info["cycles"] > 1
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9)
    h = np.array(info["history"])
    for c in range(0, len(h), 10):               # never grows inside a cycle
        assert np.all(np.diff(h[c:c + 10]) <= 1e-15)


def test_two_level_schwarz_in_the_dk_inner_product():
    # the two-level preconditioner of eq. 2.23 with the H_k-GenEO coarse space, D_k = A + k^2 S:
    # converges, and a tight tolerance reproduces the direct solution
    p = pb.make_problem(24, k=9.0, s=3, overlap=2, coef="cells", seed=4, n_cells=4)
    M = schwarz.TwoLevelSchwarz(p, schwarz.Options(eig_mode=local.EIG_FIXED, nev=5))
    x, info = fgmres.solve_left_dk(p, M, tol=1e-12)
    assert info["converged"] and info["relres_prec"] <= 1e-12
    u = reference.direct_solve(p)[0]
    assert np.linalg.norm(x - u) / np.linalg.norm(u) <= 1e-9
