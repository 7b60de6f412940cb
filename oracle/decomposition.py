"""Overlapping decomposition: Def 2.8, Def 2.12, Def 2.13 and Lambda (Sec. 2.3-2.4).

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


def decompose(problem) -> list[Subdomain]:
    """Overlapping subdomains from the element partition, Def 2.8 applied `overlap[i]` times."""
    E = incidence(problem)
    interior = problem.vert_dof >= 0
    subs = []
    for i in range(problem.n_sub):
        in_D = problem.elem_part == i
        for _ in range(int(problem.overlap[i])):
            in_D = extend_one_layer(in_D, E, interior)
        # ovdof(D): supp(phi_l) meets D  <=>  l is a vertex of an element of D
        verts_in = np.asarray(E[in_D].sum(axis=0)).ravel() > 0
        # dof(D): supp(phi_l) inside closure(D)  <=>  every element around l is in D
        outside = np.asarray(E[~in_D].sum(axis=0)).ravel() > 0
        ov_v = np.nonzero(verts_in & interior)[0]
        in_v = np.nonzero(verts_in & interior & ~outside)[0]
        dof = np.sort(problem.vert_dof[in_v])
        ovd = np.sort(problem.vert_dof[ov_v])
        gamma = np.setdiff1d(ovd, dof)
        subs.append(Subdomain(elems=in_D, dof=dof, gamma=gamma, ovdof=np.concatenate([dof, gamma])))
    return subs


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
