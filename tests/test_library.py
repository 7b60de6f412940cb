"""CPU checks of the C-ABI library: it loads, exports every declared entry point, its host
partitioner (Def. 2.8, 2.12, 2.13) reproduces the oracle's index sets, and argument validation
rejects bad input before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2406_06283_amd import hkgeneo as H
from paper_2406_06283_amd import problems as pb
from oracle import decomposition as dec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hkgeneo.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hkgeneo_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = H.load()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(H.SIGNATURES), "binding signatures and header disagree"


def test_strerror_and_defaults():
    lib = H.load()
    assert lib.hkgeneo_strerror(H.HKG_EEIG).decode() == "local eigenproblem failed"
    o = H.default_options()
    assert (o.restart, o.max_iter, o.rtol, o.nev, o.local_prec, o.two_level) == (50, 1000, 1e-8, 10, 64, 1)


@pytest.mark.parametrize("kw", [dict(N=32, k=10.0, s=4, overlap=2), dict(N=20, s=3, overlap=[1, 2, 3, 1, 2, 3, 1, 2, 3]),
                                dict(N=17, s=3, overlap=2), dict(N=6, dim=3, elem_type=pb.Q1, s=2, overlap=1),
                                dict(N=8, dim=3, elem_type=pb.Q1, s=2, overlap=2)])
def test_host_partitioner_matches_oracle(kw):
    N = kw.pop("N")
    p = pb.make_problem(N, **kw)
    nI, nG, dofs, gams, mu, lam = H.partition(p)
    subs = dec.decompose(p)
    for a, g, s in zip(dofs, gams, subs):
        np.testing.assert_array_equal(a, s.dof)
        np.testing.assert_array_equal(g, s.gamma)
    np.testing.assert_array_equal(mu, dec.multiplicity(subs, p.n_dof))
    assert lam == dec.overlap_count(subs)


def test_partition_rejects_uncovered_dofs():
    p = pb.make_problem(8, s=2, overlap=0)
    with pytest.raises(H.HkgError) as e:
        H.partition(p)
    assert e.value.status == H.HKG_EINVAL


def _setup_status(p, **opt):
    lib = H.load()
    pv = H._ProblemView(p)
    o = H.default_options(**opt)
    h = ctypes.c_void_p()
    return lib.hkgeneo_setup(ctypes.byref(pv.c), ctypes.byref(o), None, ctypes.byref(h)), h


@pytest.mark.parametrize("bad", ["overlap0", "negative_k", "local_prec", "factor32", "krylov", "coarse_op", "restart", "bad_part",
                                 "unsorted_csr"])
def test_setup_validates_before_device_work(bad):
    p = pb.make_problem(8, k=3.0, s=2, overlap=1)
    opt = {}
    if bad == "overlap0":
        p.overlap[:] = 0
    elif bad == "negative_k":
        p.k = -1.0
    elif bad == "local_prec":
        opt["local_prec"] = 16
    elif bad == "factor32":          # the float32 LU is not offered
        opt["local_prec"] = 32
        opt["local_factor_prec"] = 32
    elif bad == "krylov":
        opt["krylov"] = 2
    elif bad == "coarse_op":
        opt["coarse_op"] = 7
    elif bad == "restart":
        opt["restart"] = 0
    elif bad == "bad_part":
        p.elem_part[0] = p.n_sub
    elif bad == "unsorted_csr":
        p.col_idx[[0, 1]] = p.col_idx[[1, 0]]
    st, h = _setup_status(p, **opt)
    assert st == H.HKG_EINVAL and not h.value
