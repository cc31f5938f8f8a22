"""GPU: hh_covariance_noalloc (partials in the library's static device scratch)
against hh_covariance with a caller workspace, through the C ABI: two calls in a
row, the second on a smaller stack, each equal to the workspace form bit for
bit (same kernels, same launch) and to the oracle within the covariance bar; a
size whose partials exceed the scratch is refused on the host."""
import numpy as np
import pytest

import oracle
from gpu_util import rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2004_00923_amd.hh as hh_mod
    hh_mod.lib()
    return hh_mod


def _holo(seed, nt, ny, nx):
    rng = np.random.default_rng(seed)
    H = (rng.standard_normal((nt, ny, nx)) + 1j * rng.standard_normal((nt, ny, nx))).astype(np.complex64)
    H += (2.0 - 1.0j) * rng.standard_normal((nt, 1, 1)).astype(np.complex64)
    return H


def test_noalloc_equals_workspace_form_twice(hh):
    import torch
    for seed, (nt, ny, nx) in ((1, (32, 512, 1024)), (2, (20, 64, 128))):
        say(f"noalloc covariance {nt}x{ny}x{nx}")
        H = _holo(seed, nt, ny, nx)
        p = hh.Params(nx=nx, ny=ny, nt=nt, k_lo=0, k_hi=nt - 1)
        Hd = to_dev(H)
        ws = hh.alloc_workspace(hh.covariance_workspace_bytes(p))
        c_ws = torch.empty((nt, nt), dtype=torch.complex128, device="cuda")
        hh.hh_covariance(p, Hd, c_ws, ws)
        c_na = torch.full((nt, nt), float("nan"), dtype=torch.complex128, device="cuda")
        hh.hh_covariance_noalloc(p, Hd, c_na)
        a, b = to_np(c_na), to_np(c_ws)
        assert np.array_equal(a, b), "no-alloc covariance differs from the workspace form"
        assert rel(a, oracle.covariance_ref(H.astype(np.complex128))) <= 2e-6


def test_noalloc_rejects_oversize(hh):
    import torch
    p = hh.Params(nx=4096, ny=4096, nt=32, k_lo=0, k_hi=31)
    H = torch.empty((32, 8, 8), dtype=torch.complex64, device="cuda")   # never read: refused before launch
    C = torch.empty((32, 32), dtype=torch.complex128, device="cuda")
    import ctypes
    st = hh.lib().hh_covariance_noalloc(ctypes.byref(p.c()), ctypes.c_void_p(H.data_ptr()),
                                        ctypes.c_void_p(C.data_ptr()), None)
    assert st == hh.HH_E_UNSUPPORTED
    assert "scratch" in hh.lib().hh_last_error().decode()
    assert hh.covariance_noalloc_max_bytes() == 48 << 20
