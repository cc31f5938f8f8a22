"""GPU: every launch choice the autotuner can pick gives a result within the FP32
bar of the oracle, and the autotuner itself runs, keeps a valid choice, and the
pipeline under it still matches the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import LAM, PITCH, Z, rel, say, to_dev, to_np
from paper_2004_00923_amd.synth import gen_stack

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-5


@pytest.fixture(scope="module")
def hh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2004_00923_amd.hh as hh_mod
    hh_mod.lib()
    hh_mod.tuning_reset()
    yield hh_mod
    hh_mod.tuning_reset()


def _run(hh, p, frames):
    import torch
    ws = hh.alloc_workspace(hh.workspace_bytes(p))
    img = torch.empty((p.ny, p.nx), dtype=torch.float32, device="cuda")
    hh.hh_pipeline(p, frames, img, ws)
    return to_np(img)


@pytest.fixture(scope="module")
def case(hh):
    # 512 x 1024 frames: both FFT lengths have every launch shape
    nt, ny, nx = 32, 512, 1024
    f = gen_stack(77, nt, ny, nx)
    r = oracle.pipeline_ref(f, LAM, Z, PITCH, 2, nt - 1)
    return f, to_dev(f), r["image"]


@pytest.mark.parametrize("rows,cols,pxw,group", [(0, 0, 256, 0), (1, 0, 256, 0), (2, 0, 256, 0), (3, 0, 256, 0),
                                                 (4, 0, 256, 0), (5, 0, 256, 0), (6, 0, 256, 0), (7, 0, 256, 0),
                                                 (8, 0, 256, 0), (9, 0, 256, 0),
                                                 (0, 1, 256, 0), (0, 2, 256, 0), (0, 3, 256, 0), (0, 4, 256, 0),
                                                 (0, 5, 256, 0), (0, 6, 256, 0), (0, 7, 256, 0), (0, 0, 512, 0), (0, 0, 1024, 0),
                                                 (0, 0, 256, 3), (2, 2, 1024, 1), (6, 5, 512, 32), (7, 6, 256, 5)])
@pytest.mark.parametrize("precision,gram_ref", [("fp32", 0), ("fp32", 1), ("fp16store", 0)])
def test_every_launch_choice_meets_the_bar(hh, case, rows, cols, pxw, group, precision, gram_ref):
    f, fd, ref = case
    p = hh.Params(nx=1024, ny=512, nt=32, k_lo=2, k_hi=31, precision=hh.PRECISIONS[precision])
    # the row/column/covariance kernels on stored holograms (fused=0)
    hh.tuning_set(p, fft_rows=rows, fft_cols=cols, gram_pxw=pxw, group=group, gram_ref=gram_ref, fused=0)
    try:
        e = rel(_run(hh, p, fd), ref)
    finally:
        hh.tuning_reset()
    say(f"tuning rows={rows} cols={cols} pxw={pxw} group={group} ref={gram_ref} {precision}: image {e:.2e}")
    assert e <= (IMG_TOL if precision == "fp32" else 1e-3)


def test_autotune_picks_a_valid_choice(hh, case):
    f, fd, ref = case
    p = hh.Params(nx=1024, ny=512, nt=32, k_lo=2, k_hi=31)
    ws = hh.alloc_workspace(hh.workspace_bytes(p))
    best = hh.autotune(p, fd, ws, reps=3)
    say(f"autotune 32x512x1024: {best}")
    assert hh.tuning_get(p) == best
    assert rel(_run(hh, p, fd), ref) <= IMG_TOL
    hh.tuning_reset()


@pytest.mark.parametrize("nt,ny,nx", [(32, 128, 128), (16, 64, 64), (31, 32, 64), (3, 8, 8), (32, 1024, 1024),
                                      (64, 128, 128), (33, 64, 64), (64, 1024, 2048)])
def test_frame0_reference_covariance(hh, nt, ny, nx):
    # the covariance with the frame-0 reference of the split meets the FP32 bar on C
    import torch
    f = gen_stack(nt * 3 + nx, nt, ny, nx)
    H32 = oracle.fresnel_ref(f, LAM, Z, PITCH).astype(np.complex64)
    C_ref = oracle.covariance_ref(H32.astype(np.complex128))
    p = hh.Params(nx=nx, ny=ny, nt=nt, k_lo=0, k_hi=nt - 1)
    hh.tuning_set(p, gram_ref=1)
    try:
        ws = hh.alloc_workspace(hh.covariance_workspace_bytes(p))
        C = torch.empty((nt, nt), dtype=torch.complex128, device="cuda")
        hh.hh_covariance(p, to_dev(H32), C, ws)
        e = rel(to_np(C), C_ref)
    finally:
        hh.tuning_reset()
    say(f"frame-0 reference covariance {nt}x{ny}x{nx}: {e:.2e}")
    assert e <= 2e-6


@pytest.mark.parametrize("ny,nx", [(2048, 512), (512, 2048), (4096, 512), (512, 4096)])
@pytest.mark.parametrize("rows,cols", [(8, 7), (9, 7), (6, 5)])
def test_persistent_and_capped_shapes_at_other_lengths(hh, ny, nx, rows, cols):
    # the four-row and two-row persistent row FFTs and the register-capped column FFT
    # (LDS twiddles up to 2048 points, global twiddles beyond) at 512-4096 points
    f = gen_stack(ny + nx + rows, 8, ny, nx)
    r = oracle.pipeline_ref(f, LAM, Z, PITCH, 1, 7)
    p = hh.Params(nx=nx, ny=ny, nt=8, k_lo=1, k_hi=7)
    hh.tuning_set(p, fft_rows=rows, fft_cols=cols, fused=0)
    try:
        e = rel(_run(hh, p, to_dev(f)), r["image"])
    finally:
        hh.tuning_reset()
    say(f"shapes rows={rows} cols={cols} 8x{ny}x{nx}: image {e:.2e}")
    assert e <= IMG_TOL
