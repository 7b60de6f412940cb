"""Python binding of libhkgeneo (the C ABI declared in include/hkgeneo.h).

Argument marshalling only: every numerical step runs in the HIP library.  The functions named like
the C entry points take raw pointers; the ``Solver`` class wraps them for problems built by
``paper_2406_06283_amd.problems`` and torch tensors on the GPU (torch provides device memory and the
stream, nothing else).  There is no CPU fallback: if the library is missing or no HIP device is
present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhkgeneo.so")

HKG_OK = 0
HKG_EINVAL = -1
HKG_ENOMEM = -2
HKG_EHIP = -3
HKG_ESINGULAR_LOCAL = -4
HKG_EEIG = -5
HKG_ESINGULAR_COARSE = -6
HKG_ENOTCONV = 1
HKG_P1 = 1
HKG_Q1 = 2
HKG_EIG_THRESHOLD = 0
HKG_EIG_FIXED = 1
HKG_PROLONG_AS = 0
HKG_PROLONG_POU = 1
HKG_COARSE_HK = 0
HKG_COARSE_DELTA = 1
HKG_KRYLOV_RIGHT = 0
HKG_KRYLOV_LEFT_DK = 1
HKG_APPLY_NOALLOC_MAX_BYTES = 64 << 20     # size of the allocation-free scratch array per GPU

_i32p = POINTER(c_int32)
_f64p = POINTER(c_double)


class hkgeneo_problem(ctypes.Structure):
    _fields_ = [("dim", c_int32), ("elem_type", c_int32), ("n_vert", c_int32), ("n_elem", c_int32),
                ("n_dof", c_int32), ("nnz", c_int32), ("elem_vert", _i32p), ("vert_dof", _i32p),
                ("elem_K", _f64p), ("elem_M", _f64p), ("row_ptr", _i32p), ("col_idx", _i32p),
                ("A_val", _f64p), ("S_val", _f64p), ("elem_part", _i32p), ("n_sub", c_int32),
                ("overlap", _i32p), ("k", c_double), ("fine_part", _i32p), ("fine_overlap", c_int32)]


class hkgeneo_options(ctypes.Structure):
    _fields_ = [("eig_mode", c_int32), ("tau", c_double), ("nev", c_int32), ("cluster_rtol", c_double),
                ("max_eig_per_sub", c_int32), ("local_prec", c_int32), ("prolong", c_int32),
                ("two_level", c_int32), ("restart", c_int32), ("max_iter", c_int32), ("rtol", c_double),
                ("keep_workspace", c_int32), ("local_factor_prec", c_int32), ("krylov", c_int32),
                ("coarse_op", c_int32)]


class hkgeneo_rhs_info(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("converged", c_int32), ("relres_est", c_double), ("relres_true", c_double)]


class hkgeneo_stats(ctypes.Structure):
    _fields_ = [("n_dof", c_int32), ("n_sub", c_int32), ("lambda_overlap", c_int32), ("m0", c_int32),
                ("sum_nI", c_int32), ("max_nI", c_int32), ("max_nG", c_int32), ("bad_sub", c_int32),
                ("device_bytes", c_int64), ("setup_ms", c_double), ("peak_device_bytes", c_int64)]


class hkgeneo_server_stats(ctypes.Structure):
    _fields_ = [("queued", c_int32), ("live", c_int32), ("live_rhs", c_int32), ("completed_waiting", c_int32),
                ("local_waves", c_int32), ("pad_", c_int32), ("workspace_bytes", c_int64), ("device_bytes", c_int64),
                ("iterations", c_int64), ("restarts", c_int64), ("captures", c_int64), ("admitted", c_int64),
                ("retired", c_int64)]


# name -> (restype, argtypes); mirrors include/hkgeneo.h
SIGNATURES = {
    "hkgeneo_default_options": (None, [POINTER(hkgeneo_options)]),
    "hkgeneo_setup": (c_int32, [POINTER(hkgeneo_problem), POINTER(hkgeneo_options), c_void_p, POINTER(c_void_p)]),
    "hkgeneo_factor": (c_int32, [c_void_p, c_void_p]),
    "hkgeneo_profile": (c_int32, [c_void_p, c_int32]),
    "hkgeneo_profile_read": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_int64)]),
    "hkgeneo_apply": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_void_p]),
    "hkgeneo_gmres_solve": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int32, POINTER(hkgeneo_rhs_info),
                                      c_void_p]),
    "hkgeneo_apply_noalloc": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_void_p]),
    "hkgeneo_matvec": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_void_p]),
    "hkgeneo_query": (c_int32, [c_void_p, POINTER(hkgeneo_stats)]),
    "hkgeneo_query_subdomains": (c_int32, [c_void_p, _i32p, _i32p, _i32p]),
    "hkgeneo_query_index_sets": (c_int32, [c_void_p, c_int32, _i32p, _i32p, _i32p]),
    "hkgeneo_query_fine": (c_int32, [c_void_p, _i32p, _i32p, _i32p, _i32p]),
    "hkgeneo_query_eigen": (c_int32, [c_void_p, c_int32, _f64p, c_int32, _f64p]),
    "hkgeneo_query_coarse_matrix": (c_int32, [c_void_p, _f64p]),
    "hkgeneo_partition": (c_int32, [POINTER(hkgeneo_problem), _i32p, _i32p, _i32p, _i32p, _i32p, _i32p]),
    "hkgeneo_batch_create": (c_int32, [POINTER(c_void_p), _i32p, c_int32, POINTER(c_void_p)]),
    "hkgeneo_batch_solve": (c_int32, [c_void_p, POINTER(c_void_p), POINTER(c_void_p), _i32p, POINTER(hkgeneo_rhs_info),
                                      c_void_p]),
    "hkgeneo_batch_bytes": (c_int64, [c_void_p]),
    "hkgeneo_batch_local_waves": (c_int32, [c_void_p]),
    "hkgeneo_batch_profile": (c_int32, [c_void_p, c_int32]),
    "hkgeneo_batch_profile_read": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_int64)]),
    "hkgeneo_batch_destroy": (None, [c_void_p]),
    "hkgeneo_server_create": (c_int32, [c_int64, c_int32, c_int32, c_int32, POINTER(c_void_p)]),
    "hkgeneo_server_submit": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int64, c_void_p]),
    "hkgeneo_server_pump": (c_int32, [c_void_p, c_int32, _i32p]),
    "hkgeneo_server_poll": (c_int32, [c_void_p, POINTER(c_int64), _i32p, POINTER(hkgeneo_rhs_info), c_int32]),
    "hkgeneo_server_query": (c_int32, [c_void_p, POINTER(hkgeneo_server_stats)]),
    "hkgeneo_server_destroy": (None, [c_void_p]),
    "hkgeneo_destroy": (None, [c_void_p]),
    "hkgeneo_strerror": (c_char_p, [c_int32]),
    "hkgeneo_last_error": (c_char_p, []),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load the in-tree library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    try:   # share torch's HIP runtime when torch is present (same SONAME, one runtime per process)
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class HkgError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        detail = lib.hkgeneo_last_error().decode()
        super().__init__(f"{where}: {lib.hkgeneo_strerror(status).decode()} ({status}) {detail}")
        self.status = status


def _check(status: int, where: str):
    if status < 0:
        raise HkgError(status, where)
    return status


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(POINTER(ctype))


def default_options(**kw) -> hkgeneo_options:
    o = hkgeneo_options()
    load().hkgeneo_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class _ProblemView:
    """A hkgeneo_problem pointing at the problem's numpy arrays (kept alive here)."""

    def __init__(self, p):
        self.keep = dict(
            elem_vert=np.ascontiguousarray(p.elem_vert, dtype=np.int32).ravel(),
            vert_dof=np.ascontiguousarray(p.vert_dof, dtype=np.int32),
            elem_K=np.ascontiguousarray(p.elem_K, dtype=np.float64).ravel(),
            elem_M=np.ascontiguousarray(p.elem_M, dtype=np.float64).ravel(),
            row_ptr=np.ascontiguousarray(p.row_ptr, dtype=np.int32),
            col_idx=np.ascontiguousarray(p.col_idx, dtype=np.int32),
            A_val=np.ascontiguousarray(p.A_val, dtype=np.float64),
            S_val=np.ascontiguousarray(p.S_val, dtype=np.float64),
            elem_part=np.ascontiguousarray(p.elem_part, dtype=np.int32),
            overlap=np.ascontiguousarray(p.overlap, dtype=np.int32),
        )
        fine = getattr(p, "fine_part", None)
        if fine is not None:
            self.keep["fine_part"] = np.ascontiguousarray(fine, dtype=np.int32)
        k = self.keep
        self.c = hkgeneo_problem(
            dim=p.dim, elem_type=p.elem_type, n_vert=p.n_vert, n_elem=p.n_elem, n_dof=p.n_dof, nnz=p.nnz,
            elem_vert=_ptr(k["elem_vert"], c_int32), vert_dof=_ptr(k["vert_dof"], c_int32),
            elem_K=_ptr(k["elem_K"], c_double), elem_M=_ptr(k["elem_M"], c_double),
            row_ptr=_ptr(k["row_ptr"], c_int32), col_idx=_ptr(k["col_idx"], c_int32),
            A_val=_ptr(k["A_val"], c_double), S_val=_ptr(k["S_val"], c_double),
            elem_part=_ptr(k["elem_part"], c_int32), n_sub=p.n_sub, overlap=_ptr(k["overlap"], c_int32),
            k=float(p.k),
            fine_part=_ptr(k["fine_part"], c_int32) if "fine_part" in k else None,
            fine_overlap=int(getattr(p, "fine_overlap", 0)))


def partition(problem):
    """Host-only decomposition through the library: (nI, nG, dof list per sub, gamma list per sub, mu, Lambda)."""
    lib = load()
    pv = _ProblemView(problem)
    ns = problem.n_sub
    nI = np.zeros(ns, np.int32)
    nG = np.zeros(ns, np.int32)
    _check(lib.hkgeneo_partition(ctypes.byref(pv.c), _ptr(nI, c_int32), _ptr(nG, c_int32), None, None, None, None),
           "hkgeneo_partition")
    dof = np.zeros(max(int(nI.sum()), 1), np.int32)
    gam = np.zeros(max(int(nG.sum()), 1), np.int32)
    mu = np.zeros(problem.n_dof, np.int32)
    lam = np.zeros(1, np.int32)
    _check(lib.hkgeneo_partition(ctypes.byref(pv.c), None, None, _ptr(dof, c_int32), _ptr(gam, c_int32),
                                 _ptr(mu, c_int32), _ptr(lam, c_int32)), "hkgeneo_partition")
    oI = np.concatenate([[0], np.cumsum(nI)])
    oG = np.concatenate([[0], np.cumsum(nG)])
    dofs = [dof[oI[i]:oI[i + 1]].copy() for i in range(ns)]
    gams = [gam[oG[i]:oG[i + 1]].copy() for i in range(ns)]
    return nI, nG, dofs, gams, mu, int(lam[0])


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


class Solver:
    """A set-up preconditioner / FGMRES solver on the current HIP device."""

    def __init__(self, problem, options: hkgeneo_options | None = None, stream=None, **kw):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the hkgeneo library runs on the GPU only")
        self.lib = load()
        self.options = options if options is not None else default_options(**kw)
        self.n = problem.n_dof
        self.n_sub = problem.n_sub
        self._pv = _ProblemView(problem)
        h = c_void_p()
        _check(self.lib.hkgeneo_setup(ctypes.byref(self._pv.c), ctypes.byref(self.options), _stream_handle(stream),
                                      ctypes.byref(h)), "hkgeneo_setup")
        self.handle = h

    def factor(self, stream=None):
        """Redo the numeric setup on the device from the resident inputs."""
        _check(self.lib.hkgeneo_factor(self.handle, _stream_handle(stream)), "hkgeneo_factor")

    def profile(self, enable: bool):
        _check(self.lib.hkgeneo_profile(self.handle, int(enable)), "hkgeneo_profile")

    def profile_read(self):
        t = c_double()
        n = c_int64()
        _check(self.lib.hkgeneo_profile_read(self.handle, ctypes.byref(t), ctypes.byref(n)), "hkgeneo_profile_read")
        return t.value, n.value

    # --- raw-pointer style (same names as the C ABI) ---
    def _as_block(self, t):
        import torch
        if t.dtype != torch.float64 or not t.is_cuda:
            raise TypeError("expected a float64 tensor on the GPU")
        if t.dim() == 1:
            t = t.view(1, -1)
        if t.shape[-1] != self.n or not t.is_contiguous():
            raise ValueError("expected a contiguous (nrhs, n_dof) tensor")
        return t

    def apply(self, r, z=None, stream=None):
        import torch
        r2 = self._as_block(r)
        z2 = torch.empty_like(r2) if z is None else self._as_block(z)
        _check(self.lib.hkgeneo_apply(self.handle, c_void_p(r2.data_ptr()), c_void_p(z2.data_ptr()), r2.shape[0],
                                      self.n, _stream_handle(stream)), "hkgeneo_apply")
        return z2.view_as(r) if z is None else z

    def apply_noalloc(self, r, z, stream=None):
        """hkgeneo_apply_noalloc: z = M^{-1} r with the library's fixed scratch array (z preallocated)."""
        r2 = self._as_block(r)
        z2 = self._as_block(z)
        _check(self.lib.hkgeneo_apply_noalloc(self.handle, c_void_p(r2.data_ptr()), c_void_p(z2.data_ptr()),
                                              r2.shape[0], self.n, _stream_handle(stream)), "hkgeneo_apply_noalloc")
        return z

    def matvec(self, x, w=None, stream=None):
        import torch
        x2 = self._as_block(x)
        w2 = torch.empty_like(x2) if w is None else self._as_block(w)
        _check(self.lib.hkgeneo_matvec(self.handle, c_void_p(x2.data_ptr()), c_void_p(w2.data_ptr()), x2.shape[0],
                                       self.n, _stream_handle(stream)), "hkgeneo_matvec")
        return w2.view_as(x) if w is None else w

    def solve(self, f, u=None, stream=None):
        """FGMRES(restart) from u = 0; returns (u, [info dict per rhs], status)."""
        import torch
        f2 = self._as_block(f)
        u2 = torch.empty_like(f2) if u is None else self._as_block(u)
        nr = f2.shape[0]
        infos = (hkgeneo_rhs_info * nr)()
        st = _check(self.lib.hkgeneo_gmres_solve(self.handle, c_void_p(f2.data_ptr()), c_void_p(u2.data_ptr()), nr,
                                                 self.n, infos, _stream_handle(stream)), "hkgeneo_gmres_solve")
        out = [dict(iters=i.iters, converged=bool(i.converged), relres_est=i.relres_est, relres_true=i.relres_true)
               for i in infos]
        return (u2.view_as(f) if u is None else u), out, st

    # --- queries ---
    def stats(self) -> dict:
        s = hkgeneo_stats()
        _check(self.lib.hkgeneo_query(self.handle, ctypes.byref(s)), "hkgeneo_query")
        return {name: getattr(s, name) for name, _ in s._fields_}

    def subdomains(self):
        nI = np.zeros(self.n_sub, np.int32)
        nG = np.zeros(self.n_sub, np.int32)
        m = np.zeros(self.n_sub, np.int32)
        _check(self.lib.hkgeneo_query_subdomains(self.handle, _ptr(nI, c_int32), _ptr(nG, c_int32), _ptr(m, c_int32)),
               "hkgeneo_query_subdomains")
        return nI, nG, m

    def fine(self):
        """(owner coarse subdomain per fine subdomain, |dof| per fine subdomain, Lambda over them)."""
        n = c_int32()
        lam = c_int32()
        _check(self.lib.hkgeneo_query_fine(self.handle, ctypes.byref(n), None, None, ctypes.byref(lam)),
               "hkgeneo_query_fine")
        nI = np.zeros(n.value, np.int32)
        own = np.zeros(n.value, np.int32)
        _check(self.lib.hkgeneo_query_fine(self.handle, ctypes.byref(n), _ptr(nI, c_int32), _ptr(own, c_int32),
                                           ctypes.byref(lam)), "hkgeneo_query_fine")
        return own, nI, lam.value

    def index_sets(self, sub):
        nI, nG, _ = self.subdomains()
        dof = np.zeros(nI[sub], np.int32)
        gam = np.zeros(max(nG[sub], 1), np.int32)
        mu = np.zeros(self.n, np.int32)
        _check(self.lib.hkgeneo_query_index_sets(self.handle, sub, _ptr(dof, c_int32), _ptr(gam, c_int32),
                                                 _ptr(mu, c_int32) if sub == 0 else None), "hkgeneo_query_index_sets")
        return dof, gam[:nG[sub]], (mu if sub == 0 else None)

    def eigen(self, sub, count=None):
        nI, _, m = self.subdomains()
        if count is None:
            count = min(int(nI[sub]), int(m[sub]) + 1)
        lam = np.zeros(max(count, 1))
        Z = np.zeros((int(m[sub]), int(nI[sub])))      # row b = column b of the column-major Z_i
        _check(self.lib.hkgeneo_query_eigen(self.handle, sub, _ptr(lam, c_double), count,
                                            _ptr(Z, c_double) if m[sub] > 0 else None), "hkgeneo_query_eigen")
        return lam[:count], Z.T.copy()

    def coarse_matrix(self):
        m0 = self.stats()["m0"]
        B0 = np.zeros((m0, m0))
        _check(self.lib.hkgeneo_query_coarse_matrix(self.handle, _ptr(B0, c_double)), "hkgeneo_query_coarse_matrix")
        return B0.T.copy()          # column-major on the C side

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.hkgeneo_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Several set-up problems solved together (hkgeneo_batch_* of the C ABI).

    `solvers` are Solver objects (kept alive by the batch), `nrhs` the number of right-hand sides
    per problem.  solve(fs) takes one (nrhs_p, n_p) float64 GPU tensor per problem.
    """

    def __init__(self, solvers, nrhs):
        self.lib = load()
        self.solvers = list(solvers)
        self.nrhs = [int(r) for r in nrhs]
        if len(self.nrhs) != len(self.solvers):
            raise ValueError("one nrhs per solver")
        np_ = len(self.solvers)
        hs = (c_void_p * np_)(*[s.handle.value for s in self.solvers])
        nr = np.asarray(self.nrhs, np.int32)
        self.handle = c_void_p()
        _check(self.lib.hkgeneo_batch_create(hs, _ptr(nr, c_int32), np_, ctypes.byref(self.handle)),
               "hkgeneo_batch_create")

    @property
    def device_bytes(self) -> int:
        return int(self.lib.hkgeneo_batch_bytes(self.handle))

    @property
    def local_waves(self) -> int:
        return int(self.lib.hkgeneo_batch_local_waves(self.handle))

    def profile(self, enable: bool):
        _check(self.lib.hkgeneo_batch_profile(self.handle, int(enable)), "hkgeneo_batch_profile")

    def profile_read(self):
        t = c_double()
        n = c_int64()
        _check(self.lib.hkgeneo_batch_profile_read(self.handle, ctypes.byref(t), ctypes.byref(n)),
               "hkgeneo_batch_profile_read")
        return t.value, n.value

    def solve(self, fs, us=None, stream=None):
        """Returns ([u_p], [[info dict per rhs] per problem], status)."""
        import torch
        if len(fs) != len(self.solvers):
            raise ValueError("one right-hand-side block per problem")
        f2, u2 = [], []
        for p, (S, f) in enumerate(zip(self.solvers, fs)):
            fb = S._as_block(f)
            if fb.shape[0] != self.nrhs[p]:
                raise ValueError(f"problem {p}: expected {self.nrhs[p]} right-hand sides")
            f2.append(fb)
            u2.append(torch.empty_like(fb) if us is None else S._as_block(us[p]))
        np_ = len(fs)
        fp = (c_void_p * np_)(*[t.data_ptr() for t in f2])
        up = (c_void_p * np_)(*[t.data_ptr() for t in u2])
        ld = np.asarray([S.n for S in self.solvers], np.int32)
        infos = (hkgeneo_rhs_info * sum(self.nrhs))()
        st = _check(self.lib.hkgeneo_batch_solve(self.handle, fp, up, _ptr(ld, c_int32), infos, _stream_handle(stream)),
                    "hkgeneo_batch_solve")
        out, q = [], 0
        for r in self.nrhs:
            out.append([dict(iters=i.iters, converged=bool(i.converged), relres_est=i.relres_est,
                             relres_true=i.relres_true) for i in infos[q:q + r]])
            q += r
        res = [u.view_as(f) for u, f in zip(u2, fs)] if us is None else list(us)
        return res, out, st

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.hkgeneo_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Server:
    """Continuous batching of solve requests (hkgeneo_server_* of the C ABI).

    submit(solver, f, tag) queues a request (f: (nrhs, n) float64 GPU tensor; the solution tensor is
    allocated here and kept with the request); pump(periods) advances the live set; poll() returns
    the finished requests as (tag, u, [info dict per rhs], status).
    """

    def __init__(self, workspace_budget: int, max_requests: int = 64, max_nrhs: int = 8, restart: int = 50):
        self.lib = load()
        self.handle = c_void_p()
        self.max_nrhs = int(max_nrhs)
        self._reqs = {}
        _check(self.lib.hkgeneo_server_create(int(workspace_budget), int(max_requests), self.max_nrhs, int(restart),
                                              ctypes.byref(self.handle)), "hkgeneo_server_create")

    def submit(self, solver, f, tag: int, stream=None):
        import torch
        fb = solver._as_block(f)
        u = torch.empty_like(fb)
        if tag in self._reqs:
            raise ValueError(f"tag {tag} is already pending")
        _check(self.lib.hkgeneo_server_submit(self.handle, solver.handle, c_void_p(fb.data_ptr()),
                                              c_void_p(u.data_ptr()), fb.shape[0], solver.n, int(tag),
                                              _stream_handle(stream)), "hkgeneo_server_submit")
        self._reqs[tag] = (solver, fb, u)      # keeps f, u and the context alive until polled
        return u

    def pump(self, periods: int = 1) -> int:
        pending = c_int32()
        _check(self.lib.hkgeneo_server_pump(self.handle, int(periods), ctypes.byref(pending)), "hkgeneo_server_pump")
        return pending.value

    def poll(self):
        out = []
        infos = (hkgeneo_rhs_info * self.max_nrhs)()
        tag, st = c_int64(), c_int32()
        while True:
            n = _check(self.lib.hkgeneo_server_poll(self.handle, ctypes.byref(tag), ctypes.byref(st), infos,
                                                    self.max_nrhs), "hkgeneo_server_poll")
            if n == 0:
                return out
            _, _, u = self._reqs.pop(tag.value)
            out.append((tag.value, u, [dict(iters=i.iters, converged=bool(i.converged), relres_est=i.relres_est,
                                            relres_true=i.relres_true) for i in infos[:n]], st.value))

    def stats(self) -> dict:
        s = hkgeneo_server_stats()
        _check(self.lib.hkgeneo_server_query(self.handle, ctypes.byref(s)), "hkgeneo_server_query")
        return {name: getattr(s, name) for name, _ in s._fields_ if name != "pad_"}

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.hkgeneo_server_destroy(self.handle)
            self.handle = None
            self._reqs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def options_for(workload, **overrides) -> hkgeneo_options:
    """Options of a named workload (configs.Workload) with keyword overrides."""
    kw = dict(eig_mode=workload.eig_mode, nev=workload.nev, tau=workload.tau, restart=workload.restart)
    kw.update(overrides)
    return default_options(**kw)
