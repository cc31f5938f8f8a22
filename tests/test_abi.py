"""The C-ABI library loads, exports every declared symbol, and validates on the
host (no device work is done by any call in this file)."""
import ctypes
import os
import re

import pytest

import paper_2004_00923_amd.hh as hh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hh.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hh_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = hh.lib()
    names = declared_symbols()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/hh.h but not exported"
    assert set(names) == set(hh.SIGNATURES), "binding signatures out of sync with include/hh.h"


def test_params_struct_layout():
    # 3 doubles + 8 int32, no padding: the C struct is 56 bytes
    assert ctypes.sizeof(hh.hh_params) == 56
    src = open(HEADER).read()
    for f, _ in hh.hh_params._fields_:
        assert re.search(rf"\b{f}\b", src), f


def _call_fresnel(p, nframes=1):
    return hh.lib().hh_fresnel(ctypes.byref(p), ctypes.c_void_p(16), nframes, ctypes.c_void_p(16), None)


def good():
    return hh.Params(nx=1024, ny=1024, nt=32, k_lo=2, k_hi=31).c()


@pytest.mark.parametrize("field,value,status", [
    ("nx", 1000, hh.HH_E_UNSUPPORTED), ("ny", 4, hh.HH_E_UNSUPPORTED), ("nx", 8192, hh.HH_E_UNSUPPORTED),
    ("nx", 0, hh.HH_E_INVALID), ("wavelength_m", 0.0, hh.HH_E_INVALID), ("wavelength_m", float("nan"), hh.HH_E_INVALID),
    ("distance_m", 0.0, hh.HH_E_INVALID), ("pitch_m", -1.0, hh.HH_E_INVALID), ("eigh_solver", 2, hh.HH_E_INVALID),
])
def test_fresnel_rejects_bad_params(field, value, status):
    p = good()
    setattr(p, field, value)
    assert _call_fresnel(p) == status
    assert hh.lib().hh_last_error().decode() != ""


def test_null_and_counts():
    L = hh.lib()
    p = good()
    assert L.hh_fresnel(ctypes.byref(p), None, 1, ctypes.c_void_p(16), None) == hh.HH_E_INVALID
    assert L.hh_fresnel(None, ctypes.c_void_p(16), 1, ctypes.c_void_p(16), None) == hh.HH_E_INVALID
    assert _call_fresnel(p, -1) == hh.HH_E_INVALID
    assert _call_fresnel(p, 0) == hh.HH_OK          # empty stack: nothing to do
    assert L.hh_fresnel(ctypes.byref(p), ctypes.c_void_p(16), 1, ctypes.c_void_p(12), None) == hh.HH_E_INVALID
    # frames are read with 16-byte loads
    assert L.hh_fresnel(ctypes.byref(p), ctypes.c_void_p(24), 1, ctypes.c_void_p(16), None) == hh.HH_E_INVALID


@pytest.mark.parametrize("k_lo,k_hi,nt,status", [
    (2, 31, 32, hh.HH_OK), (0, 0, 2, hh.HH_OK), (3, 2, 32, hh.HH_E_INVALID), (-1, 5, 32, hh.HH_E_INVALID),
    (0, 32, 32, hh.HH_E_INVALID), (0, 0, 1, hh.HH_E_UNSUPPORTED), (0, 64, 65, hh.HH_E_UNSUPPORTED),
])
def test_selection_validation(k_lo, k_hi, nt, status):
    p = hh.Params(nx=64, ny=64, nt=nt, k_lo=k_lo, k_hi=k_hi).c()
    L = hh.lib()
    # too-small workspace makes a valid call stop at the workspace check, before any device work
    st = L.hh_pipeline(ctypes.byref(p), ctypes.c_void_p(16), ctypes.c_void_p(16), None, None, None,
                       ctypes.c_void_p(256), 1, None)
    assert st == (hh.HH_E_WORKSPACE if status == hh.HH_OK else status)
    assert (L.hh_workspace_bytes(ctypes.byref(p)) > 0) == (status == hh.HH_OK)


def test_workspace_sizes():
    p = hh.Params(nx=1024, ny=1024, nt=32, k_lo=2, k_hi=31)
    ws = hh.workspace_bytes(p)
    # the hologram stack (complex64) dominates: 32 x 1024^2 x 8 bytes
    assert 32 * 1024 * 1024 * 8 <= ws < 32 * 1024 * 1024 * 8 * 1.1
    cw = hh.covariance_workspace_bytes(p)
    assert 0 < cw < 32 << 20
    p64 = hh.Params(nx=1024, ny=1024, nt=64, k_lo=2, k_hi=63)
    assert hh.workspace_bytes(p64) > ws
    L = hh.lib()
    c = p.c()
    st = L.hh_covariance(ctypes.byref(c), ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(256), cw - 1, None)
    assert st == hh.HH_E_WORKSPACE


def test_precision_form_validation():
    L = hh.lib()
    for prec in (hh.HH_BF16, hh.HH_FP16, hh.HH_BF16X3, hh.HH_FP16X3, hh.HH_FP8E4M3):
        p = hh.Params(nx=64, ny=64, nt=8, k_lo=1, k_hi=7, precision=prec).c()
        # a 1-byte workspace stops a call that passes the precision check before device work
        st = L.hh_covariance(ctypes.byref(p), ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(256),
                             1, None)
        assert st == hh.HH_E_WORKSPACE
        # low-precision forms are built for stacks of at most 32 frames
        p = hh.Params(nx=64, ny=64, nt=33, k_lo=1, k_hi=7, precision=prec).c()
        st = L.hh_covariance(ctypes.byref(p), ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(256),
                             1, None)
        assert st == hh.HH_E_UNSUPPORTED
    # the FP16 storage and exact forms start from frames: entry points taking FP32 holograms reject them
    for prec in (hh.HH_FP16_STORE, hh.HH_EXACT):
        p = hh.Params(nx=64, ny=64, nt=8, k_lo=1, k_hi=7, precision=prec).c()
        assert L.hh_covariance(ctypes.byref(p), ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(256),
                               1, None) == hh.HH_E_UNSUPPORTED
        assert L.hh_project_render(ctypes.byref(p), ctypes.c_void_p(16), ctypes.c_void_p(16),
                                   ctypes.c_void_p(16), None) == hh.HH_E_UNSUPPORTED
    # the exact form takes stacks up to 64 frames and needs 16-byte aligned frames
    p = hh.Params(nx=64, ny=64, nt=64, k_lo=1, k_hi=7, precision=hh.HH_EXACT).c()
    assert L.hh_pipeline(ctypes.byref(p), ctypes.c_void_p(256), ctypes.c_void_p(16), None, None, None,
                         ctypes.c_void_p(256), 1, None) == hh.HH_E_WORKSPACE
    assert L.hh_pipeline(ctypes.byref(p), ctypes.c_void_p(264), ctypes.c_void_p(16), None, None, None,
                         ctypes.c_void_p(256), 1, None) == hh.HH_E_INVALID
    assert L.hh_covariance_frames(ctypes.byref(p), ctypes.c_void_p(8), ctypes.c_void_p(16), ctypes.c_void_p(256),
                                  1 << 30, None) == hh.HH_E_INVALID
    assert L.hh_covariance_frames(ctypes.byref(p), ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(256),
                                  1, None) == hh.HH_E_WORKSPACE
    p = hh.Params(nx=64, ny=64, nt=8, k_lo=1, k_hi=7, precision=hh.HH_FP16_STORE).c()
    st = L.hh_pipeline(ctypes.byref(p), ctypes.c_void_p(16), ctypes.c_void_p(16), None, None, None,
                       ctypes.c_void_p(256), 1, None)
    assert st == hh.HH_E_WORKSPACE
    # and its frames must be 8-byte aligned
    st = L.hh_pipeline(ctypes.byref(p), ctypes.c_void_p(18), ctypes.c_void_p(16), None, None, None,
                       ctypes.c_void_p(256), 1, None)
    assert st == hh.HH_E_INVALID
    # the storage form needs less workspace than the FP32 hologram
    a = hh.workspace_bytes(hh.Params(nx=1024, ny=1024, nt=32, k_lo=2, k_hi=31))
    b = hh.workspace_bytes(hh.Params(nx=1024, ny=1024, nt=32, k_lo=2, k_hi=31, precision=hh.HH_FP16_STORE))
    assert b < a
    p = hh.Params(nx=64, ny=64, nt=8, k_lo=1, k_hi=7, precision=99).c()
    assert L.hh_covariance(ctypes.byref(p), ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(256),
                           1, None) == hh.HH_E_INVALID


def test_projection_first_validation():
    L = hh.lib()
    v16, v256 = ctypes.c_void_p(16), ctypes.c_void_p(256)
    # projection first needs the exact form (C from the frames) ...
    p = hh.Params(nx=64, ny=64, nt=8, k_lo=2, k_hi=7, proj_mode=hh.HH_PROJ_FIRST).c()
    assert L.hh_pipeline(ctypes.byref(p), v256, v16, None, None, None, v256, 1 << 30, None) == hh.HH_E_INVALID
    # ... and an entry point that starts from frames
    for prec in (hh.HH_FP32, hh.HH_EXACT):
        p = hh.Params(nx=64, ny=64, nt=8, k_lo=2, k_hi=7, precision=prec, proj_mode=hh.HH_PROJ_FIRST).c()
        assert L.hh_project_render(ctypes.byref(p), v16, v16, v16, None) == hh.HH_E_UNSUPPORTED
        assert L.hh_svd_filter(ctypes.byref(p), v16, v16, v16, None) == hh.HH_E_UNSUPPORTED
        assert L.hh_fourier_render(ctypes.byref(p), v16, v16, None) == hh.HH_E_UNSUPPORTED
    p = hh.Params(nx=64, ny=64, nt=8, k_lo=2, k_hi=7, precision=hh.HH_EXACT, proj_mode=hh.HH_PROJ_FIRST).c()
    assert L.hh_pipeline(ctypes.byref(p), v256, v16, None, None, None, v256, 1, None) == hh.HH_E_WORKSPACE
    p.proj_mode = 4
    assert L.hh_pipeline(ctypes.byref(p), v256, v16, None, None, None, v256, 1 << 30, None) == hh.HH_E_INVALID
    # the pipeline workspace adds the partial images to the exact form's
    a = hh.workspace_bytes(hh.Params(nx=1024, ny=1024, nt=32, k_lo=2, k_hi=31, precision=hh.HH_EXACT))
    b = hh.workspace_bytes(hh.Params(nx=1024, ny=1024, nt=32, k_lo=2, k_hi=31, precision=hh.HH_EXACT,
                                     proj_mode=hh.HH_PROJ_FIRST))
    assert b == a + 8 * 1024 * 1024 * 4
    # hh_project_frames: K components and the partial images; alignment and size checks before device work
    q = hh.Params(nx=128, ny=64, nt=16, k_lo=3, k_hi=12)
    assert hh.project_frames_workspace_bytes(q) == 10 * 128 * 64 * 8 + 8 * 128 * 64 * 4
    qc = q.c()
    need = hh.project_frames_workspace_bytes(q)
    assert L.hh_project_frames(ctypes.byref(qc), ctypes.c_void_p(8), v16, v16, v256, need, None) == hh.HH_E_INVALID
    assert L.hh_project_frames(ctypes.byref(qc), v16, v16, v16, v256, need - 1, None) == hh.HH_E_WORKSPACE
    assert L.hh_project_frames(ctypes.byref(qc), v16, v16, v16, ctypes.c_void_p(64), need, None) == \
        hh.HH_E_WORKSPACE
    assert L.hh_project_frames(ctypes.byref(qc), None, v16, v16, v256, need, None) == hh.HH_E_INVALID
    bad = hh.Params(nx=128, ny=64, nt=16, k_lo=13, k_hi=12).c()
    assert L.hh_project_frames_workspace_bytes(ctypes.byref(bad)) == 0


def test_eigh_validation():
    L = hh.lib()
    v = ctypes.c_void_p(256)
    assert L.hh_eigh(1, v, v, v, v, None) == hh.HH_E_UNSUPPORTED
    assert L.hh_eigh(65, v, v, v, v, None) == hh.HH_E_UNSUPPORTED
    assert L.hh_eigh(32, None, v, v, v, None) == hh.HH_E_INVALID
    assert L.hh_eigh_ex(32, v, v, v, v, -1, None) == hh.HH_E_INVALID


def test_status_strings():
    L = hh.lib()
    for s in range(6):
        assert L.hh_status_string(s).decode()
    assert L.hh_status_string(77).decode() == "unknown status"


def test_tuning_validation_and_roundtrip():
    hh.tuning_reset()
    p = hh.Params(nx=1024, ny=1024, nt=32, k_lo=2, k_hi=31)
    assert hh.tuning_get(p) == {"fft_rows": 0, "fft_cols": 0, "gram_pxw": 256, "group": 0, "gram_ref": 0,
                                "fused": 0}
    hh.tuning_set(p, fft_rows=1, fft_cols=2, gram_pxw=1024, group=4, gram_ref=1, fused=1)
    assert hh.tuning_get(p) == {"fft_rows": 1, "fft_cols": 2, "gram_pxw": 1024, "group": 4, "gram_ref": 1,
                                "fused": 1}
    # FFT choices follow (nx, ny); the split-K chunk follows (nx * ny, nt, precision)
    q = hh.Params(nx=1024, ny=1024, nt=16, k_lo=2, k_hi=15)
    assert hh.tuning_get(q)["fft_rows"] == 1 and hh.tuning_get(q)["gram_pxw"] == 256
    for bad in ({"fft_rows": 10}, {"fft_cols": 8}, {"gram_pxw": 300}, {"group": -1}, {"group": 33}, {"gram_ref": 2},
                {"fused": 2}, {"fused": -1}):
        with pytest.raises(hh.HHError) as ei:
            hh.tuning_set(p, **bad)
        assert ei.value.status == hh.HH_E_INVALID
    small = hh.Params(nx=128, ny=128, nt=32, k_lo=2, k_hi=31)
    with pytest.raises(hh.HHError):
        hh.tuning_set(small, fft_rows=1)        # one row shape below 512 points
    hh.tuning_reset()
    assert hh.tuning_get(p)["fft_rows"] == 0
    # the autotuner validates before any device work
    L = hh.lib()
    t = hh.hh_tuning()
    assert L.hh_autotune(ctypes.byref(p.c()), None, None, 0, 3, ctypes.byref(t), None) == hh.HH_E_INVALID
    assert L.hh_autotune(ctypes.byref(p.c()), ctypes.c_void_p(16), None, 0, 0, ctypes.byref(t), None) == \
        hh.HH_E_INVALID
