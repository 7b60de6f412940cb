"""hkgeneo_apply_noalloc (the allocation-free variant of hkgeneo_apply) against hkgeneo_apply.

Both run the same kernels on the same inputs, so the results must be identical bit for bit.  Two
calls in a row on the same GPU (the second with a smaller problem and fewer right-hand sides) show
that the shared scratch array carries nothing from one call to the next; a request whose
temporaries exceed the array's size is refused before any launch.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2406_06283_amd import hkgeneo as H  # noqa: E402
from paper_2406_06283_amd import problems as pb  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _both(S, R):
    lib = H.load()
    r = torch.from_numpy(np.ascontiguousarray(R)).to(DEV)
    z_ref = torch.empty_like(r)
    z_na = torch.full_like(r, float("nan"))
    st = lib.hkgeneo_apply(S.handle, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(z_ref.data_ptr()), r.shape[0],
                           S.n, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == H.HKG_OK
    st = lib.hkgeneo_apply_noalloc(S.handle, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(z_na.data_ptr()),
                                   r.shape[0], S.n, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == H.HKG_OK, H.load().hkgeneo_last_error().decode()
    torch.cuda.synchronize()
    return z_ref.cpu().numpy(), z_na.cpu().numpy()


@pytest.mark.parametrize("prec", [64, 32])
def test_noalloc_apply_matches_apply(prec):
    print(f"[noalloc] local_prec {prec}: h=1/48 3x3 four rhs, then h=1/24 2x2 two rhs", flush=True)
    rng = np.random.default_rng(3)
    pa = pb.make_problem(48, k=12.0, s=3, overlap=2, coef="cells", seed=2, n_cells=6)
    pb_ = pb.make_problem(24, k=8.0, s=2, overlap=1, coef="lognormal", seed=5)
    with H.Solver(pa, H.default_options(eig_mode=H.HKG_EIG_FIXED, nev=6, local_prec=prec)) as Sa, \
            H.Solver(pb_, H.default_options(eig_mode=H.HKG_EIG_FIXED, nev=4, local_prec=prec,
                                            prolong=H.HKG_PROLONG_POU)) as Sb:
        za, za_na = _both(Sa, rng.standard_normal((4, pa.n_dof)))
        zb, zb_na = _both(Sb, rng.standard_normal((2, pb_.n_dof)))
    np.testing.assert_array_equal(za_na, za)
    np.testing.assert_array_equal(zb_na, zb)


def test_noalloc_rejects_oversized_request():
    p = pb.make_problem(16, k=6.0, s=2, overlap=2)
    with H.Solver(p, H.default_options(eig_mode=H.HKG_EIG_FIXED, nev=4)) as S:
        st = S.stats()
        per_rhs = 8 * (st["sum_nI"] + st["m0"] * (1 + (st["m0"] + 63) // 64))
        nrhs = H.HKG_APPLY_NOALLOC_MAX_BYTES // per_rhs + 1
        r = torch.zeros((nrhs, p.n_dof), dtype=torch.float64, device=DEV)
        with pytest.raises(H.HkgError) as e:
            S.apply_noalloc(r, torch.empty_like(r))
        assert e.value.status == H.HKG_EINVAL
        # the entry point still works afterwards
        R = torch.from_numpy(np.random.default_rng(1).standard_normal((1, p.n_dof))).to(DEV)
        z = S.apply_noalloc(R, torch.empty_like(R))
        np.testing.assert_array_equal(z.cpu().numpy(), S.apply(R).cpu().numpy())
