"""One- and two-level additive Schwarz with the H_k-GenEO coarse space (eqs. 2.22, 2.23; Def 2.15).

Test infrastructure only (see the package docstring).

  M^{-1}_{AS,1} = sum_D E_D W_D B_D^{-1} R_D,   B_D = R_D B E_D                    (eq. 2.22)
  M^{-1}_{AS,2} = E_0 B_0^{-1} R_0 + M^{-1}_{AS,1},   B_0 = R_0 B E_0              (eq. 2.23)

W_D = I is the paper's additive Schwarz; W_D = X_D (the 1/mu weights of Def 2.13) is the
partition-of-unity weighted variant, kept as an option.  The coarse space is H_k-GenEO (Def 2.14,
2.15) or, as an option, Delta-GenEO (the same construction on the nearby SPD problem, k = 0).  The coarse space V_0 is spanned by the
columns of Z = [E_i X_i P_i] (Def 2.15); reading R_0 as the transpose of Z on nodal residual
vectors (the l2 form of the L2 adjoint, as for R_D = E_D^T), B_0 = Z^T B Z.
"""
from __future__ import annotations

import dataclasses
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import decomposition as dec
from . import local

PROLONG_AS = 0
PROLONG_POU = 1

COARSE_HK = 0        # H_k-GenEO: the local eigenproblem of Def 2.14 (indefinite B~, D~ of (.,.)_{1,k})
COARSE_DELTA = 1     # Delta-GenEO: the same eigenproblem built from the nearby SPD problem (k = 0)


@dataclasses.dataclass
class Options:
    eig_mode: int = local.EIG_FIXED
    tau: float = 0.0
    nev: int = 10
    cluster_rtol: float = 1e-8
    prolong: int = PROLONG_AS
    two_level: bool = True
    coarse_op: int = COARSE_HK


def system_matrix(problem) -> sp.csr_matrix:
    """B = A - k^2 S (Sec. 2.1)."""
    return (problem.A - (problem.k ** 2) * problem.S).tocsr()


def energy_matrix(problem) -> sp.csr_matrix:
    """D_k = A + k^2 S (Prop 2.11)."""
    return (problem.A + (problem.k ** 2) * problem.S).tocsr()


class TwoLevelSchwarz:
    """Setup and application of M^{-1}_{AS,2} (or M^{-1}_{AS,1} when two_level is False)."""

    def __init__(self, problem, opts: Options | None = None):
        self.problem = problem
        self.opts = opts or Options()
        n = problem.n_dof
        self.n = n
        self.B = system_matrix(problem)
        self.subs = dec.decompose(problem)              # the coarse subdomains Omega_i^c
        self.mu = dec.multiplicity(self.subs, n)        # their multiplicities (Xi of Def 2.13, 2.15)
        if np.any(self.mu == 0):
            raise ValueError("a degree of freedom is internal to no subdomain (overlap too small)")
        # the subdomains of the local solves (eq. 2.22): Omega_{i,j}^f of the nested decomposition
        # (Sec. 2.3) when the problem carries a fine partition, else the coarse subdomains (Q_i = 1)
        if getattr(problem, "fine_part", None) is not None:
            nested = dec.nested_fine(problem, self.subs)
            self.fine_owner = [ci for ci, _ in nested]
            self.fine = [sub for _, sub in nested]
        else:
            self.fine_owner = list(range(len(self.subs)))
            self.fine = self.subs
        self.mu_fine = dec.multiplicity(self.fine, n)
        if np.any(self.mu_fine == 0):
            raise ValueError("a degree of freedom is internal to no fine subdomain")
        self.Lambda = dec.overlap_count(self.fine)       # Lambda counts the Omega_{i,j}^f (Sec. 2.4)
        Bd = self.B.tocsc()
        # local Dirichlet factors, eq. 2.22 (partial pivoting: B_D is indefinite in general)
        self.local_lu = []
        for s in self.fine:
            BD = Bd[s.dof][:, s.dof].toarray()
            self.local_lu.append(sla.lu_factor(BD, check_finite=True))
        self.weights = [np.ones(s.dof.shape[0]) if self.opts.prolong == PROLONG_AS
                        else 1.0 / self.mu_fine[s.dof] for s in self.fine]
        self.eigvals, self.m = [], []
        self.Z_local = []
        if self.opts.two_level:
            self._coarse_setup()

    # --- coarse space (Def 2.14, Def 2.15) and coarse matrix (eq. 2.23) -------------------------
    def _coarse_setup(self):
        o = self.opts
        cols_r, cols_c, cols_v = [], [], []
        off = 0
        # Delta-GenEO (Sec. 1, the comparison method): the paper does not write its eigenproblem;
        # reading: Def 2.14 for the nearby SPD problem, i.e. B~ and D~ both the Neumann matrix of
        # a(.,.) (k = 0).  The coarse matrix B_0 = Z^T B Z keeps the indefinite B.
        eig_problem = dataclasses.replace(self.problem, k=0.0) if o.coarse_op == COARSE_DELTA else self.problem
        for s in self.subs:
            nI = s.dof.shape[0]
            Bt, C = local.geneo_pencil(eig_problem, s, self.mu)
            lam, P = local.geneo_eigenpairs(Bt, C, nI)
            m = local.select_count(lam, o.eig_mode, o.tau, o.nev, o.cluster_rtol)
            Zi = (1.0 / self.mu[s.dof])[:, None] * P[:, :m]          # X_I p_l, Gamma dropped by Xi
            self.eigvals.append(lam)
            self.m.append(m)
            self.Z_local.append(Zi)
            r, c = np.meshgrid(s.dof, np.arange(off, off + m), indexing="ij")
            cols_r.append(r.ravel()); cols_c.append(c.ravel()); cols_v.append(Zi.ravel())
            off += m
        self.m0 = off
        self.Z = sp.csr_matrix((np.concatenate(cols_v), (np.concatenate(cols_r), np.concatenate(cols_c))),
                               shape=(self.n, self.m0))
        self.B0 = (self.Z.T @ (self.B @ self.Z)).toarray() if self.m0 else np.zeros((0, 0))
        self.B0_lu = sla.lu_factor(self.B0) if self.m0 else None

    # --- application -------------------------------------------------------------------------
    def apply_one_level(self, r):
        z = np.zeros_like(r)
        for s, lu, w in zip(self.fine, self.local_lu, self.weights):
            z[s.dof] += w * sla.lu_solve(lu, r[s.dof])
        return z

    def apply_coarse(self, r):
        if not self.opts.two_level or self.m0 == 0:
            return np.zeros_like(r)
        y = sla.lu_solve(self.B0_lu, self.Z.T @ r)
        return self.Z @ y

    def apply(self, r):
        return self.apply_coarse(r) + self.apply_one_level(r)

    def dense(self):
        """M^{-1} as a dense matrix (tiny problems only), one column per unit vector."""
        I = np.eye(self.n)
        return np.stack([self.apply(I[:, j]) for j in range(self.n)], axis=1)
