"""GPU: the exact covariance from the frames (hh_covariance_frames and the
HH_EXACT form of the pipeline).  C = nx ny I^T I holds exactly for the
discretised Eq. (1) (unit-modulus chirp, unnormalised DFT), so the GPU result
must equal the integer Gram bit for bit, and agree with the oracle's H^H H."""
import numpy as np
import pytest

import oracle
from gpu_util import LAM, PITCH, Z, rel, say, to_dev, to_np
from paper_2004_00923_amd.synth import gen_stack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2004_00923_amd.hh as hh_mod
    hh_mod.lib()
    return hh_mod


def _integer_gram(frames):
    I = frames.reshape(frames.shape[0], -1).astype(np.int64)
    return I @ I.T   # exact in int64


@pytest.mark.parametrize("nt,ny,nx", [(2, 8, 8), (16, 64, 32), (32, 128, 128), (33, 64, 64), (48, 256, 256),
                                      (64, 1024, 2048)])
def test_covariance_frames_bit_exact(hh, nt, ny, nx):
    import torch
    rng = np.random.default_rng(nt * 7 + ny)
    f = rng.integers(0, 65536, size=(nt, ny, nx), dtype=np.uint16)   # full 16-bit range
    p = hh.Params(nx=nx, ny=ny, nt=nt, k_lo=0, k_hi=nt - 1)
    ws = hh.alloc_workspace(hh.covariance_workspace_bytes(p))
    C = torch.empty((nt, nt), dtype=torch.complex128, device="cuda")
    hh.hh_covariance_frames(p, to_dev(f), C, ws)
    got = to_np(C)
    want = _integer_gram(f).astype(np.float64) * (nx * ny)   # exact: an integer < 2^53 times a power of two
    say(f"covariance_frames {nt}x{ny}x{nx}: max |diff| {np.abs(got.real - want).max():.1e}")
    assert np.array_equal(got.real, want)
    assert np.all(got.imag == 0.0)


def test_covariance_frames_equals_hologram_gram(hh):
    f = gen_stack(3, 32, 128, 128)
    import torch
    p = hh.Params(nx=128, ny=128, nt=32, k_lo=2, k_hi=31)
    ws = hh.alloc_workspace(hh.covariance_workspace_bytes(p))
    C = torch.empty((32, 32), dtype=torch.complex128, device="cuda")
    hh.hh_covariance_frames(p, to_dev(f), C, ws)
    ref = oracle.covariance_ref(oracle.fresnel_ref(f, LAM, Z, PITCH))
    assert rel(to_np(C), ref) <= 1e-13


@pytest.mark.parametrize("nt,ny,nx,k_lo", [(32, 128, 128, 2), (64, 64, 64, 3), (32, 1024, 1024, 2)])
def test_exact_form_pipeline(hh, nt, ny, nx, k_lo):
    import torch
    f = gen_stack(nt + ny + 11, nt, ny, nx)
    p = hh.Params(nx=nx, ny=ny, nt=nt, k_lo=k_lo, k_hi=nt - 1, precision=hh.HH_EXACT)
    ws = hh.alloc_workspace(hh.workspace_bytes(p))
    img = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    ev = torch.empty(nt, dtype=torch.float64, device="cuda")
    hh.hh_pipeline(p, to_dev(f), img, ws, ev)
    r = oracle.pipeline_ref(f, LAM, Z, PITCH, k_lo, nt - 1)
    e = rel(to_np(img), r["image"])
    e_lam = float(np.abs(to_np(ev) - r["evals"]).max() / r["evals"][0])
    say(f"exact form {nt}x{ny}x{nx}: image {e:.2e} lambda {e_lam:.2e}")
    assert e <= 1e-5
    assert e_lam <= 1e-12
