"""GPU: the projection-first image (HH_PROJ_FIRST, hh_project_frames).

Eq. (1) is linear in the frame, so the image of Eqs. (6)-(7) equals
sum over kept k of |Fresnel(sum_t V[t, k] I_t)|^2; the GPU evaluates it from the
uint16 frames without forming the holograms.  Compared element by element with
the FP64 oracle at the FP32 bar (1e-5 normwise), for given V (real and complex)
and for the whole path (exact covariance from the frames, Eq. (5), image)."""
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
    return hh_mod


def _frames(seed, nt, ny, nx):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 4096, size=(nt, ny, nx)).astype(np.uint16)


def _project_frames(hh, f, V, k_lo, k_hi):
    import torch
    nt, ny, nx = f.shape
    p = hh.Params(nx=nx, ny=ny, nt=nt, k_lo=k_lo, k_hi=k_hi)
    ws = hh.alloc_workspace(hh.project_frames_workspace_bytes(p))
    img = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    hh.hh_project_frames(p, to_dev(f), to_dev(V), img, ws)
    return to_np(img)


# shapes span several row and column tiles, ragged component groups (K not a
# multiple of the group), single and full component ranges, the smallest and
# largest sides, and nt = 2 and 64
CASES = [(32, 128, 128, 2, 31), (16, 64, 64, 2, 15), (3, 8, 8, 1, 2), (2, 8, 16, 0, 1), (64, 32, 32, 2, 63),
         (8, 16, 32, 5, 5), (32, 64, 128, 0, 31), (17, 256, 64, 5, 11), (32, 512, 1024, 2, 31),
         (5, 8, 4096, 0, 4), (5, 4096, 8, 1, 4), (9, 2048, 256, 3, 8)]


@pytest.mark.parametrize("nt,ny,nx,k_lo,k_hi", CASES)
def test_project_frames_eigenvectors(hh, nt, ny, nx, k_lo, k_hi):
    # V of the frames' covariance (real), as the pipeline uses it
    f = gen_stack(nt * 5 + ny, nt, ny, nx) if min(ny, nx) >= 32 else _frames(nt + nx, nt, ny, nx)
    lam, V = oracle.eigh_ref(oracle.covariance_frames_ref(f))
    got = _project_frames(hh, f, V, k_lo, k_hi)
    ref = oracle.project_first_ref(f, V, LAM, Z, PITCH, k_lo, k_hi)
    e = rel(got, ref)
    say(f"project_frames {nt}x{ny}x{nx} PCs {k_lo}..{k_hi}: image {e:.2e}")
    assert e <= IMG_TOL


@pytest.mark.parametrize("nt,ny,nx,k_lo,k_hi", [(32, 128, 128, 2, 31), (7, 64, 32, 0, 6), (64, 64, 64, 10, 40),
                                                (16, 1024, 1024, 1, 14)])
def test_project_frames_complex_unitary(hh, nt, ny, nx, k_lo, k_hi):
    # any complex V (the entry point does not assume real eigenvectors)
    rng = np.random.default_rng(nt + ny)
    f = _frames(nt * 3 + nx, nt, ny, nx)
    V, _ = np.linalg.qr(rng.standard_normal((nt, nt)) + 1j * rng.standard_normal((nt, nt)))
    got = _project_frames(hh, f, V, k_lo, k_hi)
    ref = oracle.project_render_ref(oracle.fresnel_ref(f, LAM, Z, PITCH), V, k_lo, k_hi)
    e = rel(got, ref)
    say(f"project_frames complex V {nt}x{ny}x{nx} PCs {k_lo}..{k_hi}: image {e:.2e}")
    assert e <= IMG_TOL


def _pipeline_first(hh, f, k_lo, k_hi, solver=0):
    import torch
    nt, ny, nx = f.shape
    p = hh.Params(nx=nx, ny=ny, nt=nt, k_lo=k_lo, k_hi=k_hi, precision=hh.HH_EXACT,
                  proj_mode=hh.HH_PROJ_FIRST, eigh_solver=solver)
    ws = hh.alloc_workspace(hh.workspace_bytes(p))
    img = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    ev = torch.empty(nt, dtype=torch.float64, device="cuda")
    V = torch.empty((nt, nt), dtype=torch.complex128, device="cuda")
    info = torch.empty(1, dtype=torch.int32, device="cuda")
    hh.hh_pipeline(p, to_dev(f), img, ws, ev, V, info)
    return to_np(img), to_np(ev), to_np(V), int(to_np(info)[0])


@pytest.mark.parametrize("solver", ["jacobi", "tridiag"])
@pytest.mark.parametrize("nt,ny,nx,k_lo", [(32, 128, 128, 2), (16, 64, 64, 2), (64, 32, 32, 2), (3, 8, 8, 1),
                                           (32, 1024, 1024, 2)])
def test_pipeline_first_matches_oracle(hh, nt, ny, nx, k_lo, solver):
    f = gen_stack(nt + ny, nt, ny, nx)
    M, w, V, info = _pipeline_first(hh, f, k_lo, nt - 1, 0 if solver == "jacobi" else 1)
    r = oracle.pipeline_first_ref(f, LAM, Z, PITCH, k_lo, nt - 1)
    e_img = rel(M, r["image"])
    e_lam = float(np.abs(w - r["evals"]).max() / r["evals"][0])
    im_v = float(np.abs(V.imag).max())
    say(f"pipeline first ({solver}) {nt}x{ny}x{nx} PCs {k_lo}..{nt - 1}: image {e_img:.2e} "
        f"lambda {e_lam:.2e} max|Im V| {im_v:.1e} info {info}")
    assert info >= 0
    assert e_img <= IMG_TOL
    assert e_lam <= 1e-12
    # C = N_pix I^T I is real symmetric: the solvers return real eigenvectors (the
    # projection reads Re V only)
    assert im_v <= 1e-14


def test_pipeline_first_equals_paper_order(hh):
    # the 32 x 128 x 128 configuration: same image as the paper's order of steps
    import torch
    f = gen_stack(0, 32, 128, 128)
    M, _, _, _ = _pipeline_first(hh, f, 2, 31)
    p = hh.Params(nx=128, ny=128, nt=32, k_lo=2, k_hi=31)
    ws = hh.alloc_workspace(hh.workspace_bytes(p))
    img = torch.empty((128, 128), dtype=torch.float32, device="cuda")
    hh.hh_pipeline(p, to_dev(f), img, ws)
    r = oracle.pipeline_ref(f, LAM, Z, PITCH, 2, 31)
    e1, e0 = rel(M, r["image"]), rel(to_np(img), r["image"])
    say(f"32x128x128: projection first {e1:.2e}, paper order {e0:.2e}")
    assert e1 <= IMG_TOL and e0 <= IMG_TOL


def test_pipeline_first_batch_and_graph(hh):
    # uneven stacks through one batched call and one captured graph: every stack
    # equals its own single-stack call bit for bit; graph replays equal eager
    import torch
    specs = [(16, 256, 256), (32, 512, 512), (64, 256, 128), (2, 8, 8), (32, 128, 256)]
    ps, frames, host, imgs = [], [], [], []
    for i, (nt, ny, nx) in enumerate(specs):
        ps.append(hh.Params(nx=nx, ny=ny, nt=nt, k_lo=min(2, nt - 1), k_hi=nt - 1, precision=hh.HH_EXACT,
                            proj_mode=hh.HH_PROJ_FIRST))
        f = gen_stack(40 + i, nt, ny, nx) if ny >= 32 else _frames(40 + i, nt, ny, nx)
        host.append(f)
        frames.append(to_dev(f))
        imgs.append(torch.empty((ny, nx), dtype=torch.float32, device="cuda"))
    ws = hh.alloc_workspace(hh.batch_workspace_bytes(ps))
    hh.hh_pipeline_batch(ps, frames, imgs, ws)
    eager = [to_np(m) for m in imgs]
    for i, (p, f) in enumerate(zip(ps, host)):
        single, _, _, _ = _pipeline_first(hh, f, p.k_lo, p.k_hi)
        assert np.array_equal(single, eager[i]), f"stack {i}"
        r = oracle.pipeline_first_ref(f, LAM, Z, PITCH, p.k_lo, p.k_hi)
        e = rel(eager[i], r["image"])
        say(f"batch first stack {i} {f.shape}: image {e:.2e}")
        assert e <= IMG_TOL
    g = hh.Graph(ps, frames, imgs, ws)
    try:
        for rep in range(3):
            for m in imgs:
                m.fill_(-1.0)
            g.launch()
            torch.cuda.synchronize()
            for i, m in enumerate(imgs):
                assert np.array_equal(to_np(m), eager[i]), f"replay {rep} stack {i}"
            # eager work between replays
            hh.hh_pipeline_batch(ps[:1], frames[:1], imgs[:1], ws)
            torch.cuda.synchronize()
    finally:
        g.close()
