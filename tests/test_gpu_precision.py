"""GPU: the low-precision forms of the covariance contraction (step (b), Eq. (4))
against the FP64 oracle.  Each form must stay within its own error bound on the
image, the eigenvalues and C itself; the table printed here (run with -s) is the
error table of the precision forms."""
import numpy as np
import pytest

import oracle
from gpu_util import LAM, PITCH, Z, eig_parity, rel, say, to_dev, to_np
from paper_2004_00923_amd.synth import gen_stack

pytestmark = pytest.mark.gpu

# form name -> (enum attribute, bound on the normwise image error, bound on the
# normwise error of the covariance the eigensolver received)
FORMS = {
    "fp32": ("HH_FP32", 1e-5, 2e-6),
    "bf16x3": ("HH_BF16X3", 1e-5, 2e-6),
    "fp16x3": ("HH_FP16X3", 1e-5, 2e-6),
    "fp16": ("HH_FP16", 1e-3, 1e-5),
    "bf16": ("HH_BF16", 1e-3, 1e-5),
    # FP8 e4m3 (3 mantissa bits) in both contractions measures ~1.5e-2 on the image:
    # it does not meet the 1e-3 mixed-precision bar; the bound is twice what it reaches
    "fp8e4m3": ("HH_FP8E4M3", 3e-2, 1e-4),
    "fp16store": ("HH_FP16_STORE", 1e-3, 1e-5),
}


# FP8 e4m3 keeps 3 mantissa bits: the projection of the kept components (after the
# frame-0 split) measures ~1.5e-2; twice that
PROJ_FP8_BOUND = 3e-2


@pytest.fixture(scope="module")
def hh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2004_00923_amd.hh as hh_mod
    hh_mod.lib()
    return hh_mod


def _run(hh, frames, k_lo, k_hi, precision):
    import torch
    nt, ny, nx = frames.shape
    p = hh.Params(nx=nx, ny=ny, nt=nt, k_lo=k_lo, k_hi=k_hi, precision=precision)
    ws = hh.alloc_workspace(hh.workspace_bytes(p))
    img = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    ev = torch.empty(nt, dtype=torch.float64, device="cuda")
    V = torch.empty((nt, nt), dtype=torch.complex128, device="cuda")
    hh.hh_pipeline(p, to_dev(frames), img, ws, ev, V)
    return to_np(img), to_np(ev), to_np(V)


def _cov(hh, H32, precision):
    import torch
    nt, ny, nx = H32.shape
    p = hh.Params(nx=nx, ny=ny, nt=nt, k_lo=0, k_hi=nt - 1, precision=precision)
    ws = hh.alloc_workspace(hh.covariance_workspace_bytes(p))
    C = torch.empty((nt, nt), dtype=torch.complex128, device="cuda")
    hh.hh_covariance(p, to_dev(H32), C, ws)
    return to_np(C)


@pytest.mark.parametrize("ny,nx,seed", [(128, 128, 0), (1024, 1024, 0)])
def test_precision_table(hh, ny, nx, seed):
    f = gen_stack(seed, 32, ny, nx)
    r = oracle.pipeline_ref(f, LAM, Z, PITCH, 2, 31)
    H32 = oracle.fresnel_ref(f, LAM, Z, PITCH).astype(np.complex64)
    C_ref = oracle.covariance_ref(H32.astype(np.complex128))
    say(f"\nprecision forms, 32 x {ny} x {nx}, PCs 2..31 (normwise vs the FP64 oracle)")
    say(f"{'form':>9} {'image':>9} {'lambda':>9} {'C(H32)':>9} {'C(pipe)':>9} {'subspace':>9} {'vectors':>9}")
    bad = []
    for name, (attr, bound, c_tol) in FORMS.items():
        prec = getattr(hh, attr)
        M, w, V = _run(hh, f, 2, 31, prec)
        e_img = rel(M, r["image"])
        e_lam = float(np.abs(w - r["evals"]).max() / r["evals"][0])
        e_c = rel(_cov(hh, H32, prec), C_ref) if prec != hh.HH_FP16_STORE else float("nan")
        # subspace: distance of the kept projectors (Davis-Kahan bounded inside eig_parity);
        # vectors: largest sin(angle) of the well-separated modes
        d = eig_parity(w, V, r, 2, 31, c_tol, f"form {name}")
        say(f"{name:>9} {e_img:9.2e} {e_lam:9.2e} {e_c:9.2e} {d['cov']:9.2e} {d['proj']:9.2e} {d['sin']:9.2e}")
        if not (np.isfinite(M).all() and e_img <= bound):
            bad.append((name, e_img, bound))
    assert not bad, f"forms over their image bound: {bad}"


def test_precision_rejects_long_stacks(hh):
    import torch
    p = hh.Params(nx=16, ny=16, nt=33, k_lo=2, k_hi=32, precision=hh.HH_BF16)
    ws = hh.alloc_workspace(1 << 20)
    C = torch.empty((33, 33), dtype=torch.complex128, device="cuda")
    H = torch.zeros((33, 16, 16), dtype=torch.complex64, device="cuda")
    with pytest.raises(hh.HHError) as ei:
        hh.hh_covariance(p, H, C, ws)
    assert ei.value.status == hh.HH_E_UNSUPPORTED


@pytest.mark.parametrize("attr", ["HH_BF16", "HH_FP16X3", "HH_FP8E4M3"])
def test_precision_degenerate_inputs(hh, attr):
    # a constant stack (R = 0: the per-pixel scales fall back to 1) and a stack
    # with one bright frame (wide dynamic range) stay finite and close to the oracle
    prec = getattr(hh, attr)
    const = np.full((32, 64, 64), 1000, dtype=np.uint16)
    M, w, _ = _run(hh, const, 2, 31, prec)
    r = oracle.pipeline_ref(const, LAM, Z, PITCH, 2, 31)
    assert np.isfinite(M).all() and np.isfinite(w).all()
    assert np.abs(w - r["evals"]).max() <= 1e-6 * r["evals"][0]
    f = gen_stack(5, 32, 64, 64)
    f[7] = np.minimum(f[7].astype(np.int64) * 2, 4095).astype(np.uint16)
    M, w, _ = _run(hh, f, 2, 31, prec)
    r = oracle.pipeline_ref(f, LAM, Z, PITCH, 2, 31)
    assert np.isfinite(M).all()
    assert np.abs(w - r["evals"]).max() <= 5e-2 * r["evals"][0]


@pytest.mark.parametrize("nt,ny,nx,k_lo", [(32, 128, 128, 2), (16, 64, 64, 2), (3, 8, 8, 1), (32, 64, 128, 12),
                                          (31, 32, 32, 2), (32, 1024, 1024, 3)])
def test_fp16_store_pipeline(hh, nt, ny, nx, k_lo):
    # the FP16 storage form within the mixed-precision bar, on several shapes
    f = gen_stack(nt + ny + 7, nt, ny, nx)
    M, w, _ = _run(hh, f, k_lo, nt - 1, hh.HH_FP16_STORE)
    r = oracle.pipeline_ref(f, LAM, Z, PITCH, k_lo, nt - 1)
    e = rel(M, r["image"])
    e_lam = float(np.abs(w - r["evals"]).max() / r["evals"][0])
    say(f"fp16store {nt}x{ny}x{nx} PCs {k_lo}..{nt - 1}: image {e:.2e} lambda {e_lam:.2e}")
    assert e <= 1e-3
    assert e_lam <= 1e-5


def test_fp16_store_batch_mixed_forms_equal_alone(hh):
    import torch
    specs = [(32, 64, 64, hh.HH_FP16_STORE), (16, 32, 128, hh.HH_FP32), (32, 128, 128, hh.HH_FP16_STORE)]
    ps, frames, imgs, host = [], [], [], []
    for i, (nt, ny, nx, prec) in enumerate(specs):
        f = gen_stack(400 + i, nt, ny, nx)
        host.append(f)
        ps.append(hh.Params(nx=nx, ny=ny, nt=nt, k_lo=2, k_hi=nt - 1, precision=prec))
        frames.append(to_dev(f))
        imgs.append(torch.empty((ny, nx), dtype=torch.float32, device="cuda"))
    ws = hh.alloc_workspace(hh.batch_workspace_bytes(ps))
    hh.hh_pipeline_batch(ps, frames, imgs, ws)
    for i, (nt, ny, nx, prec) in enumerate(specs):
        alone = _run(hh, host[i], 2, nt - 1, prec)[0]
        assert np.array_equal(to_np(imgs[i]), alone), f"stack {i}"


@pytest.mark.parametrize("ny,nx,nt,k_lo,k_hi", [(1024, 1024, 32, 2, 31), (128, 128, 32, 2, 31), (64, 128, 16, 1, 15),
                                                (8, 8, 31, 3, 30), (16, 16, 2, 0, 1)])
def test_projection_forms_on_mfma(hh, ny, nx, nt, k_lo, k_hi):
    # step (d)+(e) alone in each operand format (hh_project_render), on the FP32
    # holograms, with the oracle's eigenvectors: the image against the oracle's image
    # for the same H and V, element by element (normwise); the smallest frames (64
    # pixels: four 16-pixel tiles) and short stacks included
    import torch
    f = gen_stack(nt * 5 + nx, nt, ny, nx)
    H = oracle.fresnel_ref(f, LAM, Z, PITCH)
    H32 = H.astype(np.complex64)
    lam, V = oracle.eigh_ref(oracle.covariance_ref(H32.astype(np.complex128)))
    ref = oracle.project_render_ref(H32.astype(np.complex128), V, k_lo, k_hi)
    bounds = {"HH_BF16X3": 2e-5, "HH_FP16X3": 2e-5, "HH_BF16": 1e-3, "HH_FP16": 1e-3, "HH_FP8E4M3": PROJ_FP8_BOUND}
    Hd, Vd = to_dev(H32), to_dev(V)
    out = []
    for attr, bound in bounds.items():
        p = hh.Params(nx=nx, ny=ny, nt=nt, k_lo=k_lo, k_hi=k_hi, precision=getattr(hh, attr))
        img = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
        hh.hh_project_render(p, Hd, Vd, img)
        M = to_np(img)
        e = rel(M, ref)
        out.append((attr, e))
        assert np.isfinite(M).all() and e <= bound, f"{attr} {nt}x{ny}x{nx} PCs {k_lo}..{k_hi}: {e:.2e} > {bound:.0e}"
    say(f"projection forms {nt}x{ny}x{nx} PCs {k_lo}..{k_hi}: " + ", ".join(f"{a[3:]} {e:.2e}" for a, e in out))
