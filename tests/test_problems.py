"""Pins for the seeded problem generator (the discrete system of Sec. 2.1, eqs. 2.11-2.12).

Closed forms that a mistake in the element matrices, the assembly or the numbering would break.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from paper_2406_06283_amd import problems as pb


def test_p1_stiffness_spectrum_closed_form():
    # On the "/" right-triangle mesh the P1 Laplacian stiffness matrix is the 5-point stencil
    # (4, -1, -1, -1, -1); its eigenvalues are 4 sin^2(i pi h/2) + 4 sin^2(j pi h/2).
    N = 16
    p = pb.make_problem(N)
    lam = np.linalg.eigvalsh(p.A.toarray())
    i = np.arange(1, N)
    s = 4 * np.sin(i * np.pi / (2 * N)) ** 2
    exact = np.sort((s[:, None] + s[None, :]).ravel())
    np.testing.assert_allclose(lam, exact, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dim,N", [(2, 9), (3, 5)])
def test_q1_pencil_spectrum_closed_form(dim, N):
    # Q1 stiffness/mass are tensor products of 1D P1 K1 = tridiag(-1,2,-1)/h, M1 = h tridiag(1,4,1)/6;
    # the pencil (A, S) has eigenvalues sum_d 6 (1 - cos t_d) / (h^2 (2 + cos t_d)), t_d = i_d pi h.
    p = pb.make_problem(N, dim=dim, elem_type=pb.Q1)
    lam = sla.eigh(p.A.toarray(), p.S.toarray(), eigvals_only=True)
    h = 1.0 / N
    t = np.arange(1, N) * np.pi * h
    a1 = 6 * (1 - np.cos(t)) / (h * h * (2 + np.cos(t)))
    grids = np.meshgrid(*([a1] * dim), indexing="ij")
    exact = np.sort(sum(grids).ravel())
    np.testing.assert_allclose(lam, exact, rtol=1e-11)


@pytest.mark.parametrize("dim,et", [(2, pb.P1), (2, pb.Q1), (3, pb.Q1)])
def test_mass_and_unit_load(dim, et):
    N = 6
    p = pb.make_problem(N, dim=dim, elem_type=et, rhs="one")
    # sum of all mass entries = |Omega| = 1 (the basis, boundary included, sums to one)
    assert abs(p.elem_M.sum() - 1.0) < 1e-13
    # f = 1: (1, phi_l) = h^d for every interior vertex of a uniform grid
    np.testing.assert_allclose(p.f[0], (1.0 / N) ** dim, rtol=1e-12)


def test_csr_structure():
    p = pb.make_problem(12, k=3.0, coef="cells", seed=3, n_cells=4)
    A = p.A.toarray(); S = p.S.toarray()
    assert np.allclose(A, A.T, atol=1e-14) and np.allclose(S, S.T, atol=1e-14)
    assert np.linalg.eigvalsh(A).min() > 0 and np.linalg.eigvalsh(S).min() > 0
    counts = np.diff(p.row_ptr)
    assert counts.max() == 7                       # P1 "/" mesh: 6 neighbours + diagonal
    for r in range(p.n_dof):
        cols = p.col_idx[p.row_ptr[r]:p.row_ptr[r + 1]]
        assert np.all(np.diff(cols) > 0)           # sorted, unique


def test_manufactured_solution_second_order():
    # u = sin(pi x) sin(pi y) solves -lap u - k^2 u = (2 pi^2 - k^2) u; P1 nodal error is O(h^2).
    k = 5.0
    errs = []
    for N in (16, 32, 64):
        p = pb.make_problem(N, k=k)
        x, y = p.coords[:, 0], p.coords[:, 1]
        uex = np.sin(np.pi * x) * np.sin(np.pi * y)
        f = pb.load_vector(p.elem_vert, p.vert_dof, p.elem_M, (2 * np.pi ** 2 - k * k) * uex, p.n_dof)
        B = (p.A - k * k * p.S).tocsc()
        uh = spla.spsolve(B, f)
        errs.append(np.abs(uh - uex[p.vert_dof >= 0]).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5, errs


def test_floor_partition_uneven():
    p = pb.make_problem(10, s=3)
    counts = np.bincount(p.elem_part, minlength=p.n_sub)
    assert p.n_sub == 9 and counts.sum() == p.n_elem
    # floor(i*3/10) splits 10 columns as 4/3/3
    side = np.array([4, 3, 3])
    np.testing.assert_array_equal(counts.reshape(3, 3), 2 * side[:, None] * side[None, :])


def test_seeded_coefficients_reproducible():
    a = pb.make_problem(16, coef="lognormal", seed=5).coef
    b = pb.make_problem(16, coef="lognormal", seed=5).coef
    c = pb.make_problem(16, coef="lognormal", seed=6).coef
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    cells = pb.make_problem(16, coef="cells", seed=1, n_cells=4).coef
    assert cells.min() >= 1.0 and cells.max() <= 100.0
    assert np.unique(cells).size == 16
