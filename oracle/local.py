"""Local matrices and the H_k-GenEO local eigenproblem (Def 2.14, Def 2.15, Lemma 2.6).

Test infrastructure only (see the package docstring).

Per subdomain D with local ordering ovdof = [dof(D), Gamma] (Gamma = ovdof minus dof):

  * Dirichlet matrix (eq. 2.22):  B_D = R_D B E_D = B[dof, dof].
  * Neumann matrices (eq. 2.18): B~ = sum over elements e in D of (K_e - k^2 M_e) on ovdof, and
    D~ = sum over e in D of (K_e + k^2 M_e), the Gram matrix of (.,.)_{1,k,D}.
  * Partition-of-unity operator (Def 2.13): Xi_D acts on coefficient vectors as X = diag(x) with
    x_l = 1/mu_l on dof(D) and 0 on Gamma.
  * Eigenproblem (Def 2.14): B~ p = lambda C p with C = X D~ X, positive semi-definite with kernel
    spanned by the Gamma coordinates.  Its finite eigenpairs are those of the reduced definite pencil
        S p_I = lambda C_II p_I,   S = B~_II - B~_IG (B~_GG)^{-1} B~_GI,   p_G = -(B~_GG)^{-1} B~_GI p_I,
    which follows from the Gamma rows of the pencil (their right-hand side is zero).  C_II is SPD, so
    the reduced pencil is symmetric-definite: real eigenvalues, C-orthonormal eigenvectors, which is the
    normalisation c(p_i, p_j) = delta_ij of Lemma 2.6.  The |Gamma| remaining eigenvalues are infinite.
  * Selection (Def 2.15 and the text around tau): eigenvalues ascending; m_i chosen so that
    lambda_{m_i+1} > 0.  The coarse vectors are E_i Xi_i p_l, i.e. X_I p_{I,l} on dof(D) (Xi drops Gamma).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

EIG_THRESHOLD = 0
EIG_FIXED = 1


def neumann_matrices(problem, sub):
    """B~ and D~ on ovdof(D), summed over the elements of D only (eq. 2.18 restricted to D)."""
    nloc = sub.ovdof.shape[0]
    g2l = -np.ones(problem.n_dof, dtype=np.int64)
    g2l[sub.ovdof] = np.arange(nloc)
    Bt = np.zeros((nloc, nloc))
    Dt = np.zeros((nloc, nloc))
    k2 = problem.k ** 2
    for e in np.nonzero(sub.elems)[0]:
        dofs = problem.vert_dof[problem.elem_vert[e]]          # -1 on Dirichlet vertices
        loc = np.where(dofs >= 0, g2l[np.maximum(dofs, 0)], -1)  # every dof of e lies in ovdof(D)
        Ke = problem.elem_K[e]
        Me = problem.elem_M[e]
        for a in range(loc.shape[0]):
            if loc[a] < 0:
                continue
            for b in range(loc.shape[0]):
                if loc[b] < 0:
                    continue
                Bt[loc[a], loc[b]] += Ke[a, b] - k2 * Me[a, b]
                Dt[loc[a], loc[b]] += Ke[a, b] + k2 * Me[a, b]
    return Bt, Dt


def pou_weights(sub, mu):
    """Diagonal of X = matrix of Xi_D on ovdof: 1/mu_l on dof(D), 0 on Gamma (Def 2.13)."""
    x = np.zeros(sub.ovdof.shape[0])
    x[: sub.dof.shape[0]] = 1.0 / mu[sub.dof]
    return x


def geneo_pencil(problem, sub, mu):
    """(B~, C) of Def 2.14 on ovdof(D): C = X D~ X."""
    Bt, Dt = neumann_matrices(problem, sub)
    x = pou_weights(sub, mu)
    C = x[:, None] * Dt * x[None, :]
    return Bt, C


def schur_reduce(Bt, nI):
    """S = B~_II - B~_IG B~_GG^{-1} B~_GI; eliminates the |Gamma| infinite eigenvalues."""
    BII = Bt[:nI, :nI]
    if Bt.shape[0] == nI:
        return BII.copy()
    BIG = Bt[:nI, nI:]
    BGI = Bt[nI:, :nI]
    BGG = Bt[nI:, nI:]
    return BII - BIG @ sla.solve(BGG, BGI)


def normalise_signs(P):
    """Sign convention: the entry of largest magnitude (first on ties) of each column is positive."""
    P = P.copy()
    for j in range(P.shape[1]):
        i = int(np.argmax(np.abs(P[:, j])))
        if P[i, j] < 0:
            P[:, j] = -P[:, j]
    return P


def geneo_eigenpairs(Bt, C, nI):
    """All finite eigenpairs of B~ p = lambda C p, ascending, C-orthonormal, on dof(D).

    Uses the symmetric-definite solver on the reduced pencil (S, C_II); only the lower triangles
    of S and C_II are referenced.
    """
    S = schur_reduce(Bt, nI)
    lam, P = sla.eigh(S, C[:nI, :nI], lower=True)
    return lam, normalise_signs(P)


def extend_to_ovdof(Bt, nI, PI):
    """p_G = -(B~_GG)^{-1} B~_GI p_I: the Gamma part of an eigenvector (Gamma rows of the pencil)."""
    if Bt.shape[0] == nI:
        return PI.copy()
    PG = -sla.solve(Bt[nI:, nI:], Bt[nI:, :nI] @ PI)
    return np.vstack([PI, PG])


def select_count(lam, mode, tau=0.0, nev=0, cluster_rtol=1e-8):
    """Number m_i of eigenvectors kept (Def 2.15 requires lambda_{m_i+1} > 0).

    threshold mode: m = #{lambda < tau};  fixed mode: m = nev.  Then m is raised to include every
    lambda <= 0, and raised further while lambda_{m+1} - lambda_m <= cluster_rtol max(1, |lambda_m|)
    so that a cluster is never cut (this makes the coarse space, and its dimension, well defined).
    """
    n = lam.shape[0]
    m = int(np.count_nonzero(lam < tau)) if mode == EIG_THRESHOLD else int(nev)
    m = min(max(m, int(np.count_nonzero(lam <= 0.0))), n)
    while 0 < m < n and lam[m] - lam[m - 1] <= cluster_rtol * max(1.0, abs(lam[m - 1])):
        m += 1
    return m


def brute_force_finite_eigs(Bt, C):
    """QZ on the full ovdof pencil; returns the finite eigenvalues ascending (tiny cases only)."""
    w = sla.eig(Bt, C, right=False, homogeneous_eigvals=True)
    alpha, beta = w[0], w[1]
    finite = np.abs(beta) > 1e-10 * np.abs(alpha).max()
    lam = (alpha[finite] / beta[finite])
    return np.sort(lam.real), np.max(np.abs(lam.imag)) if lam.size else 0.0
