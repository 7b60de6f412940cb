"""Pins for the oracle's local matrices and the H_k-GenEO eigenproblem (Def 2.14, Lemma 2.6)."""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_2406_06283_amd import problems as pb
from oracle import decomposition as dec
from oracle import local
from oracle.schwarz import system_matrix, energy_matrix


def _setup(N, **kw):
    p = pb.make_problem(N, **kw)
    subs = dec.decompose(p)
    mu = dec.multiplicity(subs, p.n_dof)
    return p, subs, mu


def test_neumann_blocks_equal_global_on_internal_rows():
    # Internal dofs have support inside closure(D), so integrating over D or over Omega agrees:
    # B~[I, I] = B[I, I] and B~[I, Gamma] = B[I, Gamma]; only B~[Gamma, Gamma] differs from B.
    p, subs, mu = _setup(16, k=6.0, s=4, overlap=2, coef="cells", seed=2, n_cells=4)
    B = system_matrix(p).toarray()
    for s in subs:
        Bt, _ = local.neumann_matrices(p, s)
        nI = s.dof.size
        np.testing.assert_allclose(Bt[:nI, :nI], B[np.ix_(s.dof, s.dof)], rtol=0, atol=1e-12)
        np.testing.assert_allclose(Bt[:nI, nI:], B[np.ix_(s.dof, s.gamma)], rtol=0, atol=1e-12)


@pytest.mark.parametrize("kw", [dict(k=5.0, s=2, overlap=1), dict(k=9.0, s=3, overlap=2, coef="cells", seed=4, n_cells=3)])
def test_schur_reduction_matches_qz_brute_force(kw):
    # QZ on the full ovdof pencil (B~, C): its finite eigenvalues are exactly those of the reduced
    # definite pencil, and the other |Gamma| are infinite (Lemma 2.6 setting: C >= 0).
    p, subs, mu = _setup(8, **kw)
    for s in subs:
        Bt, C = local.geneo_pencil(p, s, mu)
        lam, _ = local.geneo_eigenpairs(Bt, C, s.dof.size)
        qz, imag = local.brute_force_finite_eigs(Bt, C)
        assert qz.size == s.dof.size
        assert imag < 1e-8
        np.testing.assert_allclose(qz, lam, rtol=1e-8, atol=1e-8)


def test_eigenpair_residual_and_c_orthonormality():
    p, subs, mu = _setup(24, k=12.0, s=3, overlap=2, coef="lognormal", seed=1)
    for s in subs:
        nI = s.dof.size
        Bt, C = local.geneo_pencil(p, s, mu)
        lam, P = local.geneo_eigenpairs(Bt, C, nI)
        S = local.schur_reduce(Bt, nI)
        CII = C[:nI, :nI]
        res = S @ P - CII @ P * lam[None, :]
        assert np.abs(res).max() <= 1e-10 * np.abs(S).max()
        np.testing.assert_allclose(P.T @ CII @ P, np.eye(nI), atol=1e-10)
        # the full ovdof vector satisfies the unreduced pencil B~ p = lambda C p
        Pf = local.extend_to_ovdof(Bt, nI, P[:, :5])
        r = Bt @ Pf - (C @ Pf) * lam[None, :5]
        assert np.abs(r).max() <= 1e-10 * np.abs(Bt).max()
        assert np.all(np.diff(lam) >= 0)


def test_zero_wavenumber_floating_subdomain_has_constant_mode():
    # k = 0 and D away from the boundary: B~ is the Neumann stiffness of D, which kills constants,
    # so lambda_1 = 0 with p constant (the eigenproblem's kernel on a floating subdomain).
    p, subs, mu = _setup(16, k=0.0, s=4, overlap=1, coef="cells", seed=0, n_cells=4)
    s = subs[5]                                     # block (1,1): no Dirichlet vertex
    assert s.elems.sum() > 0
    Bt, C = local.geneo_pencil(p, s, mu)
    lam, P = local.geneo_eigenpairs(Bt, C, s.dof.size)
    assert abs(lam[0]) < 1e-12 and lam[1] > 1e-3
    v = P[:, 0] / P[0, 0]
    np.testing.assert_allclose(v, 1.0, atol=1e-10)


@pytest.mark.parametrize("dim,N,k", [(2, 8, 7.0), (3, 5, 4.0)])
def test_single_subdomain_q1_closed_form(dim, N, k):
    # One subdomain = Omega: dof = all, Gamma empty, mu = 1, so the pencil is (A - k^2 S, A + k^2 S)
    # and each separable mode with (A, S)-eigenvalue alpha gives lambda = (alpha - k^2)/(alpha + k^2).
    p, subs, mu = _setup(N, dim=dim, elem_type=pb.Q1, k=k, s=1, overlap=1)
    s = subs[0]
    assert s.gamma.size == 0 and np.all(mu == 1)
    Bt, C = local.geneo_pencil(p, s, mu)
    lam, _ = local.geneo_eigenpairs(Bt, C, s.dof.size)
    h = 1.0 / N
    t = np.arange(1, N) * np.pi * h
    a1 = 6 * (1 - np.cos(t)) / (h * h * (2 + np.cos(t)))
    alpha = sum(np.meshgrid(*([a1] * dim), indexing="ij")).ravel()
    exact = np.sort((alpha - k * k) / (alpha + k * k))
    np.testing.assert_allclose(lam, exact, rtol=1e-10, atol=1e-12)


def test_single_subdomain_spectrum_in_unit_interval():
    # Lemma 3.9 (|b(u,v)| <= ||u||_{1,k} ||v||_{1,k}) gives eig(B, D_k) in [-1, 1] for one subdomain.
    p, subs, mu = _setup(12, k=40.0, s=1, overlap=1, coef="cells", seed=7, n_cells=4)
    Bt, C = local.geneo_pencil(p, subs[0], mu)
    lam, _ = local.geneo_eigenpairs(Bt, C, subs[0].dof.size)
    assert lam.min() >= -1 - 1e-12 and lam.max() <= 1 + 1e-12
    assert lam.min() < 0                               # k^2 above the smallest Dirichlet eigenvalue
    ref = sla.eigh(system_matrix(p).toarray(), energy_matrix(p).toarray(), eigvals_only=True)
    np.testing.assert_allclose(lam, ref, rtol=1e-10, atol=1e-12)


def test_small_subdomains_are_definite():
    # Lemma 3.7: H k < sqrt(2) makes b_D positive definite, so B_D = B[I, I] is SPD.
    p, subs, mu = _setup(32, k=3.0, s=8, overlap=1)
    B = system_matrix(p).tocsc()
    H = (4 + 2) / 32.0 * np.sqrt(2)                      # block of 4 squares + 1 layer each side
    assert H * p.k < np.sqrt(2)
    for s in subs:
        sla.cholesky(B[s.dof][:, s.dof].toarray())       # raises if not SPD


def test_selection_rules():
    lam = np.array([-0.5, -0.1, 0.2, 0.2 + 1e-12, 0.7, 0.9, 1.3])
    assert local.select_count(lam, local.EIG_THRESHOLD, tau=0.5) == 4
    assert local.select_count(lam, local.EIG_THRESHOLD, tau=0.0) == 2        # every lambda <= 0
    assert local.select_count(lam, local.EIG_FIXED, nev=1) == 2              # raised to lambda <= 0
    assert local.select_count(lam, local.EIG_FIXED, nev=3) == 4              # cluster 0.2 kept whole
    assert local.select_count(lam, local.EIG_FIXED, nev=20) == 7
    assert local.select_count(np.array([0.1, 0.2]), local.EIG_FIXED, nev=0) == 0


@pytest.mark.parametrize("k", [0.0, 3.0, 5.0])
def test_pou_scaling_in_eigenproblem_hand_computed(k):
    # N = 2, four blocks, one layer: the single dof (centre) is internal to all four subdomains
    # (mu = 4) and every subdomain contains its whole 6-triangle patch, so each local pencil is 1x1:
    #   B~_00 = 4 - k^2 h^2/2,  D~_00 = 4 + k^2 h^2/2  (5-point stiffness; mass diagonal 6 * (h^2/2)/6)
    # and C_00 = D~_00 / mu^2, hence lambda = 16 (4 - k^2/8) / (4 + k^2/8) at h = 1/2.
    p, subs, mu = _setup(2, k=k, s=2, overlap=1)
    assert list(mu) == [4]
    for s in subs:
        Bt, C = local.geneo_pencil(p, s, mu)
        lam, P = local.geneo_eigenpairs(Bt, C, 1)
        exact = 16 * (4 - k * k / 8) / (4 + k * k / 8)
        assert abs(lam[0] - exact) <= 1e-13 * max(1, abs(exact))
