"""Overlapping decomposition: Def 2.8, Def 2.12, Def 2.13, Lambda (Sec. 2.3-2.4) and the nested
first-level subdomains of Sec. 2.3.

Test infrastructure only (see the package docstring).

Reading of Def 2.8 (extension of D' by one layer of elements): the basis
functions phi_l of V^h belong to interior vertices only (V^h is inside H^1_0).
supp(phi_l) meets the open set D' exactly when vertex l is a vertex of an
element of D'.  The extended subdomain is the union of the supports of those
phi_l, i.e. every element that shares an *interior* vertex with an element of
D'.  D' itself is kept (an element with only boundary vertices has no basis
function but still belongs to the subdomain it was given to); this changes no
matrix because such an element carries no degree of freedom.
"""
from __future__ import annotations

import dataclasses
import numpy as np
import scipy.sparse as sp


def incidence(problem) -> sp.csr_matrix:
    """Element-vertex incidence matrix E (n_elem x n_vert), E[e, v] = 1 if v is a vertex of e."""
    ne, npe = problem.elem_vert.shape
    rows = np.repeat(np.arange(ne), npe)
    cols = problem.elem_vert.ravel()
    return sp.csr_matrix((np.ones(rows.shape[0]), (rows, cols)), shape=(ne, problem.n_vert))


def extend_one_layer(in_D: np.ndarray, E: sp.csr_matrix, interior: np.ndarray) -> np.ndarray:
    """Def 2.8: add every element in supp(phi_l) for each interior vertex l touching D'."""
    touched = np.asarray(E[in_D].sum(axis=0)).ravel() > 0          # vertices of D' elements
    basis = touched & interior                                       # basis functions meeting D'
    added = np.asarray(E[:, basis].sum(axis=1)).ravel() > 0          # elements in their supports
    return in_D | added


@dataclasses.dataclass
class Subdomain:
    elems: np.ndarray   # bool mask over elements (the overlapping subdomain D_i)
    dof: np.ndarray     # sorted global dof ids with supp(phi) inside closure(D)  (Def 2.12)
    gamma: np.ndarray   # sorted ovdof(D) \ dof(D)
    ovdof: np.ndarray   # concatenation [dof, gamma] -- the local ordering used everywhere


def subdomain(problem, E: sp.csr_matrix, interior: np.ndarray, in_D: np.ndarray) -> Subdomain:
    """Index sets of the subdomain with element mask in_D (Def 2.12)."""
    # ovdof(D): supp(phi_l) meets D  <=>  l is a vertex of an element of D
    verts_in = np.asarray(E[in_D].sum(axis=0)).ravel() > 0
    # dof(D): supp(phi_l) inside closure(D)  <=>  every element around l is in D
    outside = np.asarray(E[~in_D].sum(axis=0)).ravel() > 0
    ov_v = np.nonzero(verts_in & interior)[0]
    in_v = np.nonzero(verts_in & interior & ~outside)[0]
    dof = np.sort(problem.vert_dof[in_v])
    ovd = np.sort(problem.vert_dof[ov_v])
    gamma = np.setdiff1d(ovd, dof)
    return Subdomain(elems=in_D, dof=dof, gamma=gamma, ovdof=np.concatenate([dof, gamma]))


def decompose(problem) -> list[Subdomain]:
    """Overlapping subdomains from the element partition, Def 2.8 applied `overlap[i]` times."""
    E = incidence(problem)
    interior = problem.vert_dof >= 0
    subs = []
    for i in range(problem.n_sub):
        in_D = problem.elem_part == i
        for _ in range(int(problem.overlap[i])):
            in_D = extend_one_layer(in_D, E, interior)
        subs.append(subdomain(problem, E, interior, in_D))
    return subs


def nested_fine(problem, coarse: list[Subdomain]) -> list[tuple[int, Subdomain]]:
    """The first-level (fine) subdomains of the nested decomposition (Sec. 2.3), as (coarse index, sub).

    Reading of the construction (the paper partitions the overlapping coarse subdomain and expands
    the pieces "again" while requiring their union to be the coarse subdomain): the elements of each
    overlapping coarse subdomain are split into Q_i pieces by the fine element partition
    (``problem.fine_part``); each piece is expanded by ``problem.fine_overlap`` layers of Def 2.8
    restricted to the coarse subdomain's elements, so the union of the pieces of Omega_i^c is
    Omega_i^c.  Pieces are ordered by coarse subdomain, then by fine block id.
    """
    E = incidence(problem)
    interior = problem.vert_dof >= 0
    out = []
    for ci, cs in enumerate(coarse):
        for fid in np.unique(problem.fine_part[cs.elems]):
            in_F = cs.elems & (problem.fine_part == fid)
            for _ in range(int(problem.fine_overlap)):
                in_F = extend_one_layer(in_F, E, interior) & cs.elems
            sub = subdomain(problem, E, interior, in_F)
            if sub.dof.size:            # a sliver without interior dofs has no local problem
                out.append((ci, sub))
    return out


def multiplicity(subs: list[Subdomain], n_dof: int) -> np.ndarray:
    """Def 2.13: mu_l = number of subdomains having l as an internal dof."""
    mu = np.zeros(n_dof, dtype=np.int64)
    for s in subs:
        mu[s.dof] += 1
    return mu


def overlap_count(subs: list[Subdomain]) -> int:
    """Lambda (Sec. 2.4): max over elements of the number of subdomains containing it."""
    cnt = np.zeros(subs[0].elems.shape[0], dtype=np.int64)
    for s in subs:
        cnt += s.elems
    return int(cnt.max())


def restriction_matrix(idx: np.ndarray, n: int) -> sp.csr_matrix:
    """Boolean R_D (|idx| x n) with R_D[a, idx[a]] = 1; E_D = R_D^T is the zero extension."""
    m = idx.shape[0]
    return sp.csr_matrix((np.ones(m), (np.arange(m), idx)), shape=(m, n))
