"""GPU: the batched form captured as a HIP graph (hh_graph_*), on the 8 uneven
stacks of the batched workload (512x512, 1024x1024, 2048x1024 frames; 16, 32, 64
frame stacks; seeds 0..7).  Every replay must equal the eager hh_pipeline_batch
result bit for bit, with eager work between replays, and the eager result must
match the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import LAM, PITCH, Z, eig_parity, fmt_eig, rel, say, to_dev, to_np
from paper_2004_00923_amd.synth import gen_stack

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-5
SHAPES = [(512, 512), (1024, 1024), (1024, 2048)]   # (ny, nx)
NTS = [16, 32, 64]


def batch_specs():
    """Stack i: frame shape (i mod 3), stack length ((i + i // 3) mod 3), PCs 2..nt-1."""
    return [(NTS[(i + i // 3) % 3],) + SHAPES[i % 3] for i in range(8)]


@pytest.fixture(scope="module")
def hh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2004_00923_amd.hh as hh_mod
    hh_mod.lib()
    return hh_mod


def _setup(hh, precision_lp=None):
    import torch
    specs = batch_specs()
    ps, frames, imgs, host = [], [], [], []
    for i, (nt, ny, nx) in enumerate(specs):
        prec = hh.HH_FP32
        if precision_lp is not None and nt <= 32:
            prec = precision_lp
        ps.append(hh.Params(nx=nx, ny=ny, nt=nt, k_lo=2, k_hi=nt - 1, precision=prec))
        f = gen_stack(i, nt, ny, nx)
        host.append(f)
        frames.append(to_dev(f))
        imgs.append(torch.empty((ny, nx), dtype=torch.float32, device="cuda"))
    ws = hh.alloc_workspace(hh.batch_workspace_bytes(ps))
    return ps, frames, imgs, host, ws


@pytest.mark.parametrize("form", ["fp32", "bf16x3"])
def test_graph_replays_equal_eager(hh, form):
    import torch
    ps, frames, imgs, host, ws = _setup(hh, None if form == "fp32" else hh.HH_BF16X3)
    say(f"graph {form}: {sum(p.nt * p.nx * p.ny for p in ps)} px-frames in 8 stacks")
    hh.hh_pipeline_batch(ps, frames, imgs, ws)
    eager = [to_np(m) for m in imgs]
    g = hh.Graph(ps, frames, imgs, ws)
    other = gen_stack(50, 16, 64, 64)
    po = hh.Params(nx=64, ny=64, nt=16, k_lo=2, k_hi=15)
    wso = hh.alloc_workspace(hh.workspace_bytes(po))
    imo = torch.empty((64, 64), dtype=torch.float32, device="cuda")
    for r in range(3):
        for m in imgs:
            m.fill_(-1.0)
        g.launch()
        torch.cuda.synchronize()
        for i, m in enumerate(imgs):
            assert np.array_equal(to_np(m), eager[i]), f"replay {r}: stack {i} differs from eager"
        # the program's own eager work between replays
        hh.hh_pipeline(po, to_dev(other), imo, wso)
        torch.cuda.synchronize()
    # refill one stack's frames in place: the replay reads the new contents
    f2 = gen_stack(99, ps[1].nt, ps[1].ny, ps[1].nx)
    frames[1].copy_(to_dev(f2))
    g.launch()
    torch.cuda.synchronize()
    got = to_np(imgs[1])
    g.close()
    hh.hh_pipeline_batch(ps, frames, imgs, ws)
    assert np.array_equal(got, to_np(imgs[1]))
    if form == "fp32":
        r = oracle.pipeline_ref(f2, LAM, Z, PITCH, 2, ps[1].nt - 1)
        assert rel(got, r["image"]) <= IMG_TOL


def test_graph_batch_matches_oracle(hh):
    # the first three stacks cover every frame shape and every stack length
    import torch
    ps, frames, imgs, host, ws = _setup(hh)
    evs = [torch.empty(p.nt, dtype=torch.float64, device="cuda") for p in ps]
    vecs = [torch.empty((p.nt, p.nt), dtype=torch.complex128, device="cuda") for p in ps]
    g = hh.Graph(ps, frames, imgs, ws, evals=evs, evecs=vecs)
    g.launch()
    out = [to_np(m) for m in imgs]
    g.close()
    for i in range(3):
        p = ps[i]
        say(f"oracle for stack {i}: {p.nt}x{p.ny}x{p.nx}")
        r = oracle.pipeline_ref(host[i], LAM, Z, PITCH, p.k_lo, p.k_hi)
        e = rel(out[i], r["image"])
        d = eig_parity(to_np(evs[i]), to_np(vecs[i]), r, p.k_lo, p.k_hi, 2e-6, f"graph stack {i}")
        say(f"stack {i}: image error {e:.2e} {fmt_eig(d)}")
        assert e <= IMG_TOL


def test_graph_create_validates(hh):
    import torch
    p = hh.Params(nx=100, ny=64, nt=8, k_lo=1, k_hi=7)   # nx not a power of two
    f = torch.zeros((8, 64, 100), dtype=torch.uint16, device="cuda")
    img = torch.empty((64, 100), dtype=torch.float32, device="cuda")
    with pytest.raises(hh.HHError) as ei:
        hh.Graph([p], [f], [img], hh.alloc_workspace(1 << 20))
    assert ei.value.status in (hh.HH_E_INVALID, hh.HH_E_UNSUPPORTED)
