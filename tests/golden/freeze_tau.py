"""Freeze the eigenvalue threshold tau of a threshold-mode workload from the oracle's spectra.

Calls only the oracle (and the input generator).  For seed 0 it computes every subdomain's
H_k-GenEO eigenvalues (Def 2.14), then scans tau and prints, for each candidate, the smallest and
largest number of eigenvalues below it and the distance from tau to the nearest eigenvalue.  The
chosen value is the one recorded in ``paper_2406_06283_amd/configs.py``.

usage: python tests/golden/freeze_tau.py p1_h128_k40_8x8 0.85 0.95 0.0025
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from paper_2406_06283_amd.configs import WORKLOADS  # noqa: E402
from oracle import decomposition as dec, local  # noqa: E402


def main():
    w = WORKLOADS[sys.argv[1]]
    lo, hi, step = (float(a) for a in sys.argv[2:5])
    p = w.problem(seed=0)
    subs = dec.decompose(p)
    mu = dec.multiplicity(subs, p.n_dof)
    lams = []
    for s in subs:
        Bt, C = local.geneo_pencil(p, s, mu)
        lam, _ = local.geneo_eigenpairs(Bt, C, s.dof.size)
        lams.append(lam)
    for tau in np.arange(lo, hi + 1e-12, step):
        ms = [int(np.count_nonzero(l < tau)) for l in lams]
        gap = min(float(np.min(np.abs(l - tau))) for l in lams)
        print(f"tau={tau:.5f} m_min={min(ms)} m_max={max(ms)} m0={sum(ms)} nearest={gap:.3e}")


if __name__ == "__main__":
    main()
