"""Pins for the oracle's overlapping decomposition (Def 2.8, Def 2.12, Def 2.13, Lambda)."""
import numpy as np
import pytest

from paper_2406_06283_amd import problems as pb
from oracle import decomposition as dec


def test_hand_count_single_dof():
    # N = 2: one interior vertex (the centre), four 1x1 blocks.  On the "/" mesh the centre's patch
    # is 6 triangles: the lower triangle of square (1,0) (element 2) and the upper triangle of
    # square (0,1) (element 5) miss it.  One layer adds the patch to each block, so block (0,0) and
    # block (1,1) become the patch and the two others keep their own off-patch triangle as well.
    p = pb.make_problem(2, s=2, overlap=1)
    subs = dec.decompose(p)
    patch = np.array([1, 1, 0, 1, 1, 0, 1, 1], dtype=bool)
    expect = [patch, patch | (np.arange(8) == 2), patch | (np.arange(8) == 5), patch]
    for s, e in zip(subs, expect):
        np.testing.assert_array_equal(s.elems, e)
        assert list(s.dof) == [0] and s.gamma.size == 0
    assert list(dec.multiplicity(subs, p.n_dof)) == [4]
    assert dec.overlap_count(subs) == 4


def _expected_nd(p, ov, b):
    """Internal dofs of each block of b x b squares after ov (1 or 2) layers on a uniform block grid.

    Along each axis the subdomain spans b squares plus ov per neighbouring block; its internal
    vertices are the ones strictly inside that span.  On the "/" mesh the corners that point
    against the diagonal (south-east, needing an east and a south neighbour; north-west, needing
    a west and a north neighbour) are cut: the first layer misses the lower triangle of the
    south-east corner square, so the vertex at the far corner of that square is not a vertex of
    the layer-1 region, and the second layer then misses both triangles touching the vertex
    diagonally inside the new corner, which therefore stops being internal.  Hence one internal
    vertex fewer per cut corner at 2 layers and none at 1 layer.
    """
    s = p.sub_grid[0]
    out = []
    for by in range(s):
        for bx in range(s):
            w, e, so, no = bx > 0, bx < s - 1, by > 0, by < s - 1
            nx = b + ov * w + ov * e - 1
            ny = b + ov * so + ov * no - 1
            cut = (ov >= 2) * (int(e and so) + int(w and no))
            out.append(nx * ny - cut)
    return np.array(out)


@pytest.mark.parametrize("N,s,ov", [(24, 3, 1), (24, 3, 2), (32, 4, 2), (40, 5, 1)])
def test_internal_dof_counts_on_block_grid(N, s, ov):
    p = pb.make_problem(N, s=s, overlap=ov)
    subs = dec.decompose(p)
    nd = np.array([x.dof.size for x in subs])
    np.testing.assert_array_equal(nd, _expected_nd(p, ov, N // s))


def test_config_sizes_h128():
    # h = 1/128, 8 x 8 blocks of 16 x 16 squares, 2 layers: the block rectangles give 17^2 / 17*19 /
    # 19^2 = 289 / 323 / 361 internal dofs, less one per cut corner (see _expected_nd).
    p = pb.make_problem(128, s=8, overlap=2)
    nd = np.array([x.dof.size for x in dec.decompose(p)]).reshape(8, 8)
    assert nd[0, 0] == 289 and nd[7, 7] == 289 and nd[0, 7] == 288
    assert nd[0, 3] == 322 and nd[3, 3] == 359
    np.testing.assert_array_equal(nd.ravel(), _expected_nd(p, 2, 16))


@pytest.mark.parametrize("kw", [dict(N=16, s=4, overlap=1), dict(N=20, s=3, overlap=2),
                                dict(N=12, s=2, overlap=[1, 3, 2, 1]),
                                dict(N=6, s=2, overlap=1, dim=3, elem_type=pb.Q1)])
def test_partition_of_unity(kw):
    N = kw.pop("N")
    p = pb.make_problem(N, **kw)
    subs = dec.decompose(p)
    mu = dec.multiplicity(subs, p.n_dof)
    assert mu.min() >= 1
    total = np.zeros(p.n_dof)
    for s in subs:
        R = dec.restriction_matrix(s.dof, p.n_dof)
        total += R.T @ ((1.0 / mu[s.dof]) * (R @ np.ones(p.n_dof)))
    np.testing.assert_allclose(total, 1.0, rtol=0, atol=4e-16)


def test_extension_contains_block_and_grows():
    p = pb.make_problem(16, s=4, overlap=0)
    E = dec.incidence(p)
    interior = p.vert_dof >= 0
    D0 = p.elem_part == 5
    D1 = dec.extend_one_layer(D0, E, interior)
    D2 = dec.extend_one_layer(D1, E, interior)
    assert np.all(D1[D0]) and np.all(D2[D1]) and D2.sum() > D1.sum() > D0.sum()


def test_zero_overlap_leaves_uncovered_dofs():
    p = pb.make_problem(8, s=2, overlap=0)
    mu = dec.multiplicity(dec.decompose(p), p.n_dof)
    assert (mu == 0).any()


def test_lambda_block_grid():
    p = pb.make_problem(32, s=4, overlap=2)
    assert dec.overlap_count(dec.decompose(p)) == 4


def test_gamma_is_ovdof_minus_dof():
    p = pb.make_problem(16, s=4, overlap=2, k=3.0)
    for s in dec.decompose(p):
        assert np.intersect1d(s.dof, s.gamma).size == 0
        # every Gamma dof is adjacent (in B's pattern) to an internal dof and vice versa
        A = p.A.tocsr()
        for g in s.gamma:
            nb = A.indices[A.indptr[g]:A.indptr[g + 1]]
            assert np.intersect1d(nb, s.dof).size > 0


# ------------------------------------------------------------------------------------------------
# nested decomposition (Sec. 2.3): fine subdomains inside each overlapping coarse subdomain
# ------------------------------------------------------------------------------------------------

def test_nested_fine_subdomains_hand_counted_q1():
    # Q1 on the unit square, 4 x 4 cells, one coarse subdomain (the whole square), fine blocks of
    # 2 x 2 cells expanded by one layer: each piece grows to 3 x 3 cells, so cell (x, y) lies in
    # (2 if x in {1, 2} else 1) * (2 if y in {1, 2} else 1) fine subdomains and Lambda = 4.
    p = pb.make_problem(4, dim=2, elem_type=pb.Q1, s=1, overlap=1, fine=2, fine_overlap=1)
    coarse = dec.decompose(p)
    fine = dec.nested_fine(p, coarse)
    assert len(fine) == 4 and all(ci == 0 for ci, _ in fine)
    cnt = np.zeros(p.n_elem, dtype=int)
    for _, s in fine:
        assert s.elems.sum() == 9
        cnt += s.elems
    cells = np.rint(p.coords[p.elem_vert].mean(axis=1) * 4 - 0.5).astype(int)     # cell (x, y) of each element
    want = np.where(np.isin(cells[:, 0], [1, 2]), 2, 1) * np.where(np.isin(cells[:, 1], [1, 2]), 2, 1)
    np.testing.assert_array_equal(cnt, want)
    assert dec.overlap_count([s for _, s in fine]) == 4
    # each piece's dofs: the interior vertices of its 3 x 3 cells that no outside cell touches (2 x 2)
    assert all(s.dof.size == 4 for _, s in fine)


def test_nested_pieces_cover_each_coarse_subdomain():
    # with at least one layer of fine overlap inside Omega_i^c, every dof of Omega_i^c is internal to one
    # of its pieces, and no piece reaches outside Omega_i^c (the expansion is restricted to it)
    p = pb.make_problem(24, k=5.0, s=3, overlap=2, fine=6, fine_overlap=1)
    coarse = dec.decompose(p)
    fine = dec.nested_fine(p, coarse)
    for ci, cs in enumerate(coarse):
        mine = [s for c, s in fine if c == ci]
        assert len(mine) > 1
        assert all(not np.any(s.elems & ~cs.elems) for s in mine)
        np.testing.assert_array_equal(np.unique(np.concatenate([s.dof for s in mine])), cs.dof)


def test_single_fine_block_reproduces_the_coarse_decomposition():
    # Q_i = 1 (one fine block covering the domain): every Omega_i^f is Omega_i^c itself
    p = pb.make_problem(16, k=6.0, s=2, overlap=2, coef="cells", seed=1, n_cells=4, fine=1, fine_overlap=1)
    coarse = dec.decompose(p)
    fine = dec.nested_fine(p, coarse)
    assert [c for c, _ in fine] == list(range(p.n_sub))
    for (c, f), s in zip(fine, coarse):
        np.testing.assert_array_equal(f.elems, s.elems)
        np.testing.assert_array_equal(f.dof, s.dof)
