"""Seeded synthetic Helmholtz problems: meshes, coefficients, element matrices, CSR, loads.

This module defines the *input* of the method and nothing else.  It builds the
Galerkin system of the model problem  -div(A grad u) - k^2 u = f,  u = 0 on the
boundary (paper Sec. 1, eq. (1.1); Sec. 2.1, eqs. (2.11)-(2.12)): the stiffness
matrix A_ij = a(phi_j, phi_i), the consistent mass matrix S_ij = (phi_j, phi_i),
the load vector f_i = (f, phi_i), the per-element matrices from which they are
summed, and the non-overlapping element partition that the decomposition starts
from (Sec. 2.3).  It contains none of the preconditioner's arithmetic (no
overlap, no local solve, no eigenproblem, no Krylov method): both the oracle and
the GPU library consume what it produces.

Conventions (readings of a paper that fixes no mesh):
  * 2D P1: uniform N x N squares of side h = 1/N, each cut along the "/" diagonal
    from (x_i, y_j) to (x_{i+1}, y_{j+1}) into a lower and an upper triangle.
  * Q1: tensor-product bilinear (2D) / trilinear (3D) elements on the same grid.
  * Vertices are numbered lexicographically, x fastest; the degrees of freedom
    are the interior vertices in the same order (V^h is a subspace of H^1_0).
  * The coefficient A(x) = a(x) I is constant on each element (value at the
    element centroid) and folded into the element stiffness matrix.
  * The partition assigns grid cell (i, j[, l]) to block (floor(i s / N), ...);
    both triangles of a square go to the same block.
All random draws use numpy's PCG64 seeded explicitly.
"""
from __future__ import annotations

import dataclasses
import numpy as np
import scipy.sparse as sp

P1 = 1
Q1 = 2


@dataclasses.dataclass
class Problem:
    """A discrete Helmholtz problem plus its non-overlapping element partition.

    Arrays are C-contiguous with the dtypes the C-ABI expects (int32 / float64).
    ``f`` has shape (nrhs, n_dof): row r is right-hand side r, i.e. a column-major
    n_dof x nrhs block with leading dimension n_dof.
    """

    name: str
    dim: int
    elem_type: int
    n_side: int
    h: float
    coords: np.ndarray      # (n_vert, dim) float64
    elem_vert: np.ndarray   # (n_elem, npe) int32
    vert_dof: np.ndarray    # (n_vert,) int32, -1 on the Dirichlet boundary
    elem_K: np.ndarray      # (n_elem, npe, npe) float64, coefficient folded in
    elem_M: np.ndarray      # (n_elem, npe, npe) float64
    row_ptr: np.ndarray     # (n_dof+1,) int32
    col_idx: np.ndarray     # (nnz,) int32, sorted within each row
    A_val: np.ndarray       # (nnz,) float64 stiffness
    S_val: np.ndarray       # (nnz,) float64 consistent mass
    elem_part: np.ndarray   # (n_elem,) int32 in [0, n_sub)
    n_sub: int
    overlap: np.ndarray     # (n_sub,) int32 layers of elements added to each block
    k: float
    f: np.ndarray           # (nrhs, n_dof) float64
    coef: np.ndarray        # (n_elem,) float64 value of a(x) per element
    sub_grid: tuple = ()
    seed: int = 0
    # nested decomposition (optional): a finer non-overlapping element partition and the layers by
    # which each of its pieces inside an overlapping coarse subdomain is expanded again
    fine_part: np.ndarray | None = None     # (n_elem,) int32 fine block ids, or None
    fine_overlap: int = 0

    @property
    def n_vert(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_elem(self) -> int:
        return int(self.elem_vert.shape[0])

    @property
    def npe(self) -> int:
        return int(self.elem_vert.shape[1])

    @property
    def n_dof(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def nrhs(self) -> int:
        return int(self.f.shape[0])

    def csr(self, vals: np.ndarray) -> sp.csr_matrix:
        return sp.csr_matrix((vals, self.col_idx, self.row_ptr), shape=(self.n_dof, self.n_dof))

    @property
    def A(self) -> sp.csr_matrix:
        return self.csr(self.A_val)

    @property
    def S(self) -> sp.csr_matrix:
        return self.csr(self.S_val)


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------

def _grid_vertices(N: int, dim: int):
    t = np.linspace(0.0, 1.0, N + 1)
    if dim == 2:
        X, Y = np.meshgrid(t, t, indexing="xy")          # Y varies along axis 0
        coords = np.stack([X.ravel(), Y.ravel()], axis=1)
        ij = np.stack(np.meshgrid(np.arange(N + 1), np.arange(N + 1), indexing="xy"), -1).reshape(-1, 2)
    else:
        Z, Y, X = np.meshgrid(t, t, t, indexing="ij")      # x fastest
        coords = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        L, J, I = np.meshgrid(np.arange(N + 1), np.arange(N + 1), np.arange(N + 1), indexing="ij")
        ij = np.stack([I.ravel(), J.ravel(), L.ravel()], axis=1)
    interior = np.all((ij > 0) & (ij < N), axis=1)
    vert_dof = -np.ones(coords.shape[0], dtype=np.int32)
    vert_dof[interior] = np.arange(int(interior.sum()), dtype=np.int32)
    return coords, vert_dof


def mesh_p1_2d(N: int):
    """Right-triangle mesh with "/" diagonals. Returns coords, elem_vert, vert_dof, cell index per element."""
    coords, vert_dof = _grid_vertices(N, 2)
    j, i = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    i = i.ravel(); j = j.ravel()
    v = lambda a, b: (b * (N + 1) + a)
    lower = np.stack([v(i, j), v(i + 1, j), v(i + 1, j + 1)], axis=1)
    upper = np.stack([v(i, j), v(i + 1, j + 1), v(i, j + 1)], axis=1)
    elem_vert = np.empty((2 * N * N, 3), dtype=np.int32)
    elem_vert[0::2] = lower
    elem_vert[1::2] = upper
    cell = np.repeat(np.stack([i, j], axis=1), 2, axis=0)
    return coords, elem_vert, vert_dof, cell


def mesh_q1(N: int, dim: int):
    coords, vert_dof = _grid_vertices(N, dim)
    if dim == 2:
        j, i = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
        i = i.ravel(); j = j.ravel()
        base = j * (N + 1) + i
        offs = np.array([0, 1, N + 1, N + 2])
        cell = np.stack([i, j], axis=1)
    else:
        l, j, i = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
        i = i.ravel(); j = j.ravel(); l = l.ravel()
        P = N + 1
        base = (l * P + j) * P + i
        offs = np.array([0, 1, P, P + 1, P * P, P * P + 1, P * P + P, P * P + P + 1])
        cell = np.stack([i, j, l], axis=1)
    elem_vert = (base[:, None] + offs[None, :]).astype(np.int32)
    return coords, elem_vert, vert_dof, cell


# ----------------------------------------------------------------------------
# element matrices (FE definitions of a(.,.) and (.,.) on one element)
# ----------------------------------------------------------------------------

def p1_element_matrices(coords: np.ndarray, elem_vert: np.ndarray, coef: np.ndarray):
    x = coords[elem_vert]                       # (ne, 3, 2)
    J = np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0]], axis=2)   # columns are edge vectors
    det = J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0]
    area = 0.5 * np.abs(det)
    Jinv = np.linalg.inv(J)                     # rows: gradients of barycentric coords 1, 2
    g12 = Jinv                                   # (ne, 2, 2)
    g0 = -(g12[:, 0] + g12[:, 1])
    G = np.stack([g0, g12[:, 0], g12[:, 1]], axis=1)   # (ne, 3, 2)
    K = (coef * area)[:, None, None] * np.einsum("eik,ejk->eij", G, G)
    M = (area / 12.0)[:, None, None] * (np.ones((3, 3)) + np.eye(3))[None]
    return K, M


def _k1_m1(h: float):
    K1 = (1.0 / h) * np.array([[1.0, -1.0], [-1.0, 1.0]])
    M1 = (h / 6.0) * np.array([[2.0, 1.0], [1.0, 2.0]])
    return K1, M1


def q1_element_matrices(h: float, dim: int, coef: np.ndarray):
    K1, M1 = _k1_m1(h)
    if dim == 2:   # local node a = ax + 2 ay, so the y factor is the slow kron index
        Kref = np.kron(M1, K1) + np.kron(K1, M1)
        Mref = np.kron(M1, M1)
    else:
        Kref = (np.kron(M1, np.kron(M1, K1)) + np.kron(M1, np.kron(K1, M1))
                + np.kron(K1, np.kron(M1, M1)))
        Mref = np.kron(M1, np.kron(M1, M1))
    ne = coef.shape[0]
    K = coef[:, None, None] * Kref[None]
    M = np.broadcast_to(Mref, (ne,) + Mref.shape).copy()
    return K, M


# ----------------------------------------------------------------------------
# coefficients a(x)
# ----------------------------------------------------------------------------

def coef_constant(centroids: np.ndarray) -> np.ndarray:
    return np.ones(centroids.shape[0])


def coef_cells(centroids: np.ndarray, n_cells: int, seed: int, log10_range=(0.0, 2.0)) -> np.ndarray:
    """Piecewise constant on an n_cells^d grid, log10(a) ~ U[lo, hi] per cell."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = centroids.shape[1]
    vals = 10.0 ** rng.uniform(log10_range[0], log10_range[1], size=(n_cells,) * d)
    idx = np.minimum((centroids * n_cells).astype(np.int64), n_cells - 1)
    flat = np.ravel_multi_index(tuple(idx[:, a] for a in reversed(range(d))), (n_cells,) * d)
    return vals.reshape(-1)[flat]


def coef_lognormal(centroids: np.ndarray, seed: int, sigma: float = 1.0, corr_len: float = 0.1,
                   n_features: int = 1024) -> np.ndarray:
    """a = exp(sigma g) / min(exp(sigma g)), g a unit-variance Gaussian field with covariance
    exp(-|x-y|^2 / (2 l^2)) approximated by n_features random Fourier features (Rahimi-Recht) and
    evaluated at the element centroids.  Dividing by the minimum over the mesh gives a_min = 1, the
    normalisation of Assumption 2.1(ii), so that kh keeps its meaning where a is small."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = centroids.shape[1]
    omega = rng.standard_normal((n_features, d)) / corr_len
    phase = rng.uniform(0.0, 2.0 * np.pi, size=n_features)
    g = np.sqrt(2.0 / n_features) * np.cos(centroids @ omega.T + phase[None, :]).sum(axis=1)
    a = np.exp(sigma * g)
    return a / a.min()


# ----------------------------------------------------------------------------
# assembly of the global CSR pattern / values / loads (paper Sec. 2.1)
# ----------------------------------------------------------------------------

def assemble_csr(elem_vert, vert_dof, elem_K, elem_M, n_dof):
    ed = vert_dof[elem_vert]                      # (ne, npe) dof ids or -1
    npe = ed.shape[1]
    r = np.repeat(ed, npe, axis=1).ravel()
    c = np.tile(ed, (1, npe)).ravel()
    keep = (r >= 0) & (c >= 0)
    r = r[keep]; c = c[keep]
    Kv = elem_K.reshape(elem_K.shape[0], -1).ravel()[keep]
    Mv = elem_M.reshape(elem_M.shape[0], -1).ravel()[keep]
    # one pattern for both matrices: assemble indices once, then reuse the permutation
    order = np.lexsort((c, r))
    r = r[order]; c = c[order]; Kv = Kv[order]; Mv = Mv[order]
    key = r.astype(np.int64) * n_dof + c
    first = np.ones(key.shape[0], dtype=bool)
    first[1:] = key[1:] != key[:-1]
    grp = np.cumsum(first) - 1
    nnz = int(first.sum())
    A_val = np.zeros(nnz); S_val = np.zeros(nnz)
    np.add.at(A_val, grp, Kv)
    np.add.at(S_val, grp, Mv)
    rows = r[first]; cols = c[first]
    row_ptr = np.zeros(n_dof + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return row_ptr, cols.astype(np.int32), A_val, S_val


def load_vector(elem_vert, vert_dof, elem_M, g_nodal: np.ndarray, n_dof: int) -> np.ndarray:
    """f_l = (f, phi_l) for f the P1/Q1 interpolant of nodal values g (all vertices)."""
    fe = np.einsum("eij,ej->ei", elem_M, g_nodal[elem_vert])
    ed = vert_dof[elem_vert]
    keep = ed >= 0
    f = np.zeros(n_dof)
    np.add.at(f, ed[keep], fe[keep])
    return f


def block_partition(cell: np.ndarray, N: int, s) -> tuple[np.ndarray, int, tuple]:
    d = cell.shape[1]
    s = (s,) * d if np.isscalar(s) else tuple(s)
    b = [(cell[:, a] * s[a]) // N for a in range(d)]
    pid = np.zeros(cell.shape[0], dtype=np.int64)
    for a in reversed(range(d)):
        pid = pid * s[a] + b[a]
    return pid.astype(np.int32), int(np.prod(s)), s


# ----------------------------------------------------------------------------
# problem builder
# ----------------------------------------------------------------------------

def make_problem(N: int, *, dim: int = 2, elem_type: int = P1, k: float = 0.0, s=1, overlap=1,
                 coef: str = "const", seed: int = 0, rhs: str = "one", nrhs: int = 1,
                 n_cells: int = 16, name: str = "", fine=None, fine_overlap: int = 1) -> Problem:
    if elem_type == P1:
        assert dim == 2, "P1 is generated on 2D triangle meshes"
        coords, elem_vert, vert_dof, cell = mesh_p1_2d(N)
    else:
        coords, elem_vert, vert_dof, cell = mesh_q1(N, dim)
    centroids = coords[elem_vert].mean(axis=1)
    if coef == "const":
        a = coef_constant(centroids)
    elif coef == "cells":
        a = coef_cells(centroids, n_cells, seed)
    elif coef == "lognormal":
        a = coef_lognormal(centroids, seed)
    else:
        raise ValueError(coef)
    h = 1.0 / N
    if elem_type == P1:
        K, M = p1_element_matrices(coords, elem_vert, a)
    else:
        K, M = q1_element_matrices(h, dim, a)
    n_dof = int((vert_dof >= 0).sum())
    row_ptr, col_idx, A_val, S_val = assemble_csr(elem_vert, vert_dof, K, M, n_dof)
    elem_part, n_sub, sub_grid = block_partition(cell, N, s)
    fine_part = None if fine is None else block_partition(cell, N, fine)[0]
    if np.isscalar(overlap):
        ov = np.full(n_sub, int(overlap), dtype=np.int32)
    else:
        ov = np.asarray(overlap, dtype=np.int32)
        assert ov.shape == (n_sub,)
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    fs = []
    for r in range(nrhs):
        if rhs == "one":
            g = np.ones(coords.shape[0])
        elif rhs == "normal":
            g = rng.standard_normal(coords.shape[0])
        elif rhs == "zero":
            g = np.zeros(coords.shape[0])
        else:
            raise ValueError(rhs)
        fs.append(load_vector(elem_vert, vert_dof, M, g, n_dof))
    f = np.ascontiguousarray(np.stack(fs, axis=0))
    return Problem(name=name or f"{'P1' if elem_type == P1 else 'Q1'}-{dim}d-N{N}", dim=dim,
                   elem_type=elem_type, n_side=N, h=h, coords=coords,
                   elem_vert=np.ascontiguousarray(elem_vert, dtype=np.int32),
                   vert_dof=vert_dof, elem_K=np.ascontiguousarray(K), elem_M=np.ascontiguousarray(M),
                   row_ptr=row_ptr, col_idx=col_idx, A_val=A_val, S_val=S_val,
                   elem_part=elem_part, n_sub=n_sub, overlap=ov, k=float(k), f=f, coef=a,
                   sub_grid=sub_grid, seed=seed, fine_part=fine_part,
                   fine_overlap=int(fine_overlap) if fine is not None else 0)
