"""GPU: the SVD-filtered stack of Eq. (3) (hh_svd_filter) against the oracle,
in both evaluation modes, and its power against the Eq. (7) image."""
import numpy as np
import pytest

import oracle
from gpu_util import LAM, PITCH, Z, rel, say, to_dev, to_np
from paper_2004_00923_amd.synth import gen_stack

pytestmark = pytest.mark.gpu

F_TOL = 1e-5   # FP32 stack, normwise


@pytest.fixture(scope="module")
def hh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2004_00923_amd.hh as hh_mod
    hh_mod.lib()
    return hh_mod


@pytest.mark.parametrize("mode", ["auto", "direct", "complement"])
@pytest.mark.parametrize("nt,ny,nx,k_lo,k_hi", [(32, 128, 128, 2, 31), (32, 64, 64, 12, 31), (16, 32, 64, 0, 15),
                                                (64, 32, 32, 3, 63), (8, 16, 16, 1, 5)])
def test_svd_filter_parity(hh, mode, nt, ny, nx, k_lo, k_hi):
    import torch
    f = gen_stack(300 + nt + ny, nt, ny, nx)
    H = oracle.fresnel_ref(f, LAM, Z, PITCH)
    lam, V = oracle.eigh_ref(oracle.covariance_ref(H))
    H32 = H.astype(np.complex64)
    ref = oracle.svd_filter_ref(H32.astype(np.complex128), V, k_lo, k_hi)
    mode_id = {"auto": hh.HH_PROJ_AUTO, "direct": hh.HH_PROJ_DIRECT, "complement": hh.HH_PROJ_COMPLEMENT}[mode]
    p = hh.Params(nx=nx, ny=ny, nt=nt, k_lo=k_lo, k_hi=k_hi, proj_mode=mode_id)
    out = torch.empty((nt, ny, nx), dtype=torch.complex64, device="cuda")
    hh.hh_svd_filter(p, to_dev(H32), to_dev(V), out)
    got = to_np(out)
    e = rel(got, ref)
    say(f"svd_filter {nt}x{ny}x{nx} PCs {k_lo}..{k_hi} {mode}: {e:.2e}")
    assert e <= F_TOL
    # its power is the image of Eq. (7)
    img = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    hh.hh_project_render(p, to_dev(H32), to_dev(V), img)
    assert rel(np.sum(np.abs(got.astype(np.complex128)) ** 2, axis=0), to_np(img)) <= 2 * F_TOL


def test_svd_filter_rejects_overlap(hh):
    import torch
    p = hh.Params(nx=16, ny=16, nt=4, k_lo=1, k_hi=3)
    H = torch.zeros((4, 16, 16), dtype=torch.complex64, device="cuda")
    V = torch.eye(4, dtype=torch.complex128, device="cuda")
    with pytest.raises(hh.HHError) as ei:
        hh.hh_svd_filter(p, H, V, H)
    assert ei.value.status == hh.HH_E_INVALID
