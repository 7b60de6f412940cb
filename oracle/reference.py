"""Direct sparse solve u* = B^{-1} f, used only to state solution errors.

Test infrastructure only (see the package docstring).  B = A - k^2 S (Sec. 2.1, eq. 2.12).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .schwarz import system_matrix


def direct_solve(problem, f=None):
    B = system_matrix(problem).tocsc()
    f = problem.f if f is None else f
    lu = spla.splu(B)
    if f.ndim == 1:
        return lu.solve(f)
    return np.stack([lu.solve(fr) for fr in f], axis=0)
