"""GPU: parity at the benchmark's own configuration.

bench.py times 32 x 1024 x 1024 stacks under pinned launch choices, in batches of
16 stacks over several streams.  Here every form it can time runs at that size
with exactly those launch choices, against the FP64 oracle on the same seeded
stack, and a batch of stacks through hh_pipeline_batch on four streams equals the
single-stack calls bit for bit."""
import numpy as np
import pytest

import bench
import oracle
from gpu_util import LAM, PITCH, Z, eig_parity, fmt_eig, rel, say, to_dev, to_np
from paper_2004_00923_amd.synth import gen_stack

pytestmark = pytest.mark.gpu

NT, NY, NX, K_LO, K_HI = bench.NT, bench.NY, bench.NX, bench.K_LO, bench.K_HI


@pytest.fixture(scope="module")
def hh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2004_00923_amd.hh as hh_mod
    hh_mod.lib()
    hh_mod.tuning_reset()
    yield hh_mod
    hh_mod.tuning_reset()


@pytest.fixture(scope="module")
def stack():
    f = gen_stack(0, NT, NY, NX)
    return f, oracle.pipeline_ref(f, LAM, Z, PITCH, K_LO, K_HI)


def p_key(form):
    return {"first": "exact"}.get(form, form)


def _params(hh, form):
    precision, proj = {"first": ("exact", "first")}.get(form, (form, "auto"))
    p = hh.Params(nx=NX, ny=NY, nt=NT, k_lo=K_LO, k_hi=K_HI, precision=hh.PRECISIONS[precision],
                  proj_mode=hh.PROJ_MODES[proj])
    vals = [int(v) for v in bench.PINNED_TUNING[precision].split(",")]
    hh.tuning_set(p, *vals)
    return p


# form, image bound, eigenvalue bound (/ lambda_0), covariance bound (normwise)
@pytest.mark.parametrize("form,tol,lam_tol,c_tol", [("fp32", 1e-5, 1e-6, 2e-6), ("exact", 1e-5, 1e-6, 1e-12),
                                                    ("first", 1e-5, 1e-6, 1e-12), ("fp16store", 1e-3, 1e-6, 1e-5),
                                                    ("bf16x3", 1e-5, 1e-6, 2e-6), ("fp16x3", 1e-5, 1e-6, 2e-6),
                                                    ("bf16", 1e-3, 1e-6, 1e-5), ("fp16", 1e-3, 1e-6, 1e-5),
                                                    ("fp8e4m3", 3e-2, 1e-5, 1e-4)])
def test_bench_forms_at_full_size(hh, stack, form, tol, lam_tol, c_tol):
    import torch
    f, ref = stack
    p = _params(hh, form)
    try:
        ws = hh.alloc_workspace(hh.workspace_bytes(p))
        img = torch.empty((NY, NX), dtype=torch.float32, device="cuda")
        ev = torch.empty(NT, dtype=torch.float64, device="cuda")
        V = torch.empty((NT, NT), dtype=torch.complex128, device="cuda")
        hh.hh_pipeline(p, to_dev(f), img, ws, ev, V)
        e = rel(to_np(img), ref["image"])
        w = to_np(ev)
        e_lam = float(np.abs(w - ref["evals"]).max() / ref["evals"][0])
        d = eig_parity(w, to_np(V), ref, K_LO, K_HI, c_tol, f"bench form {form}")
    finally:
        hh.tuning_reset()
    say(f"bench configuration {form} ({bench.PINNED_TUNING[p_key(form)]}): image {e:.2e} lambda {e_lam:.2e} "
        f"{fmt_eig(d)}")
    assert e <= tol
    assert e_lam <= lam_tol


def test_bench_batches_on_streams_equal_single_stacks(hh):
    # the timed loop's shape: batches of 16 stacks alternating over four streams
    import torch
    p = _params(hh, "fp32")
    try:
        host = [gen_stack(s, NT, NY, NX) for s in range(4)]
        frames = [to_dev(h) for h in host]
        singles = []
        ws1 = hh.alloc_workspace(hh.workspace_bytes(p))
        for fr in frames:
            img = torch.empty((NY, NX), dtype=torch.float32, device="cuda")
            hh.hh_pipeline(p, fr, img, ws1)
            singles.append(to_np(img))
        B, S = 16, 4
        streams = [torch.cuda.Stream() for _ in range(S)]
        lanes = []
        for s in range(S):
            imgs = [torch.empty((NY, NX), dtype=torch.float32, device="cuda") for _ in range(B)]
            ws = hh.alloc_workspace(hh.batch_workspace_bytes([p] * B))
            lanes.append((imgs, ws))
        torch.cuda.synchronize()
        for s in range(S):
            imgs, ws = lanes[s]
            with torch.cuda.stream(streams[s]):
                hh.hh_pipeline_batch([p] * B, [frames[(s + j) % 4] for j in range(B)], imgs, ws,
                                     stream=streams[s])
        torch.cuda.synchronize()
        for s in range(S):
            for j in range(B):
                assert np.array_equal(to_np(lanes[s][0][j]), singles[(s + j) % 4]), (s, j)
        say(f"{S} streams x {B} stacks equal their single-stack images")
    finally:
        hh.tuning_reset()
