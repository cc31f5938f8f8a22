"""Thin Python binding of libhh (ctypes): argument marshalling only.

Every step of the hot path runs in the HIP kernels of libhh.so; this module
checks tensor shapes/dtypes/devices, passes raw device pointers and the current
torch stream, and turns status codes into exceptions.  PyTorch provides device
memory and streams, nothing else.  There is no CPU fallback: if the library is
missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhh.so")

HH_OK, HH_E_INVALID, HH_E_UNSUPPORTED, HH_E_WORKSPACE, HH_E_DEVICE, HH_E_NOT_CONVERGED = range(6)
HH_FP32, HH_BF16, HH_FP16, HH_BF16X3, HH_FP16X3, HH_FP8E4M3, HH_FP16_STORE, HH_EXACT = range(8)
HH_PROJ_AUTO, HH_PROJ_DIRECT, HH_PROJ_COMPLEMENT, HH_PROJ_FIRST = range(4)
PROJ_MODES = {"auto": HH_PROJ_AUTO, "direct": HH_PROJ_DIRECT, "complement": HH_PROJ_COMPLEMENT,
              "first": HH_PROJ_FIRST}

PRECISIONS = {"fp32": HH_FP32, "bf16": HH_BF16, "fp16": HH_FP16, "bf16x3": HH_BF16X3,
              "fp16x3": HH_FP16X3, "fp8e4m3": HH_FP8E4M3, "fp16store": HH_FP16_STORE, "exact": HH_EXACT}


class hh_params(ctypes.Structure):
    _fields_ = [
        ("wavelength_m", ctypes.c_double),
        ("distance_m", ctypes.c_double),
        ("pitch_m", ctypes.c_double),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("nt", ctypes.c_int32),
        ("k_lo", ctypes.c_int32),
        ("k_hi", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("proj_mode", ctypes.c_int32),
        ("eigh_solver", ctypes.c_int32),
    ]


@dataclass
class Params:
    """Problem statement of one stack: optics, shape, kept components, arithmetic."""
    nx: int
    ny: int
    nt: int
    k_lo: int
    k_hi: int
    wavelength_m: float = 785e-9
    distance_m: float = 0.3
    pitch_m: float = 20e-6
    precision: int = HH_FP32
    proj_mode: int = HH_PROJ_AUTO
    eigh_solver: int = 0          # HH_EIGH_JACOBI; 1 = HH_EIGH_TRIDIAG

    def c(self) -> hh_params:
        return hh_params(self.wavelength_m, self.distance_m, self.pitch_m, self.nx, self.ny, self.nt,
                         self.k_lo, self.k_hi, self.precision, self.proj_mode, self.eigh_solver)


class hh_stack(ctypes.Structure):
    _fields_ = [("frames", ctypes.c_void_p), ("image", ctypes.c_void_p), ("evals", ctypes.c_void_p),
                ("evecs", ctypes.c_void_p), ("info", ctypes.c_void_p)]


class hh_window(ctypes.Structure):
    _fields_ = [("holo", ctypes.c_void_p), ("image", ctypes.c_void_p), ("evals", ctypes.c_void_p),
                ("evecs", ctypes.c_void_p), ("info", ctypes.c_void_p)]


class hh_tuning(ctypes.Structure):
    _fields_ = [("fft_rows", ctypes.c_int32), ("fft_cols", ctypes.c_int32), ("gram_pxw", ctypes.c_int32),
                ("group", ctypes.c_int32), ("gram_ref", ctypes.c_int32), ("fused", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class HHError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"hh status {status}: {detail}")
        self.status = status


_lib = None
_P = ctypes.c_void_p

# name -> (restype, argtypes); mirrors include/hh.h
SIGNATURES = {
    "hh_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(hh_params)]),
    "hh_covariance_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(hh_params)]),
    "hh_fresnel": (ctypes.c_int32, [ctypes.POINTER(hh_params), _P, ctypes.c_int32, _P, _P]),
    "hh_covariance": (ctypes.c_int32, [ctypes.POINTER(hh_params), _P, _P, _P, ctypes.c_size_t, _P]),
    "hh_covariance_frames": (ctypes.c_int32, [ctypes.POINTER(hh_params), _P, _P, _P, ctypes.c_size_t, _P]),
    "hh_covariance_noalloc": (ctypes.c_int32, [ctypes.POINTER(hh_params), _P, _P, _P]),
    "hh_covariance_noalloc_max_bytes": (ctypes.c_size_t, []),
    "hh_eigh": (ctypes.c_int32, [ctypes.c_int32, _P, _P, _P, _P, _P]),
    "hh_eigh_ex": (ctypes.c_int32, [ctypes.c_int32, _P, _P, _P, _P, ctypes.c_int32, _P]),
    "hh_eigh_tridiag": (ctypes.c_int32, [ctypes.c_int32, _P, _P, _P, _P, ctypes.c_int32, _P]),
    "hh_project_render": (ctypes.c_int32, [ctypes.POINTER(hh_params), _P, _P, _P, _P]),
    "hh_project_frames_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(hh_params)]),
    "hh_project_frames": (ctypes.c_int32, [ctypes.POINTER(hh_params), _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "hh_pipeline": (ctypes.c_int32, [ctypes.POINTER(hh_params), _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "hh_fourier_render": (ctypes.c_int32, [ctypes.POINTER(hh_params), _P, _P, _P]),
    "hh_fourier_render_windows": (ctypes.c_int32, [ctypes.POINTER(hh_params), _P, ctypes.c_int32, ctypes.c_int32, _P,
                                                   _P]),
    "hh_svd_filter": (ctypes.c_int32, [ctypes.POINTER(hh_params), _P, _P, _P, _P]),
    "hh_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(hh_params), ctypes.c_int32]),
    "hh_pipeline_batch": (ctypes.c_int32, [ctypes.POINTER(hh_params), ctypes.c_int32, ctypes.POINTER(hh_stack), _P,
                                           ctypes.c_size_t, _P]),
    "hh_analyze_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(hh_params), ctypes.c_int32]),
    "hh_analyze_batch": (ctypes.c_int32, [ctypes.POINTER(hh_params), ctypes.c_int32, ctypes.POINTER(hh_window), _P,
                                          ctypes.c_size_t, _P]),
    "hh_graph_create": (ctypes.c_int32, [ctypes.POINTER(hh_params), ctypes.c_int32, ctypes.POINTER(hh_stack), _P,
                                         ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)]),
    "hh_graph_launch": (ctypes.c_int32, [_P, _P]),
    "hh_graph_destroy": (None, [_P]),
    "hh_tuning_get": (ctypes.c_int32, [ctypes.POINTER(hh_params), ctypes.POINTER(hh_tuning)]),
    "hh_tuning_set": (ctypes.c_int32, [ctypes.POINTER(hh_params), ctypes.POINTER(hh_tuning)]),
    "hh_tuning_reset": (None, []),
    "hh_autotune": (ctypes.c_int32, [ctypes.POINTER(hh_params), _P, _P, ctypes.c_size_t, ctypes.c_int32,
                                     ctypes.POINTER(hh_tuning), _P]),
    "hh_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "hh_last_error": (ctypes.c_char_p, []),
    "hh_plan_cache_clear": (None, []),
    "hh_profile_enable": (None, [ctypes.c_int32]),
    "hh_profile_read": (ctypes.c_int32, [ctypes.c_char_p, ctypes.c_int32]),
    "hh_profile_reset": (None, []),
}


def lib() -> ctypes.CDLL:
    """Load libhh.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != HH_OK:
        raise HHError(status, lib().hh_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_tensor(t, dtype, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def workspace_bytes(p: Params) -> int:
    return int(lib().hh_workspace_bytes(ctypes.byref(p.c())))


def covariance_workspace_bytes(p: Params) -> int:
    return int(lib().hh_covariance_workspace_bytes(ctypes.byref(p.c())))


def hh_fresnel(p: Params, frames, holo, stream=None):
    """Step (a): frames uint16 [n, ny, nx] -> holo complex64 [n, ny, nx]."""
    import torch
    n = frames.shape[0]
    _dev_tensor(frames, torch.uint16, (n, p.ny, p.nx), "frames")
    _dev_tensor(holo, torch.complex64, (n, p.ny, p.nx), "holo")
    _check(lib().hh_fresnel(ctypes.byref(p.c()), _ptr(frames), n, _ptr(holo), _stream(stream)))
    return holo


def hh_covariance(p: Params, holo, cov, workspace, stream=None):
    """Step (b): holo complex64 [nt, ny, nx] -> cov complex128 [nt, nt]."""
    import torch
    _dev_tensor(holo, torch.complex64, (p.nt, p.ny, p.nx), "holo")
    _dev_tensor(cov, torch.complex128, (p.nt, p.nt), "cov")
    _check(lib().hh_covariance(ctypes.byref(p.c()), _ptr(holo), _ptr(cov), _ptr(workspace),
                               workspace.numel() * workspace.element_size(), _stream(stream)))
    return cov


def hh_covariance_noalloc(p: Params, holo, cov, stream=None):
    """hh_covariance with its partials in the library's static device scratch (no
    workspace, no device allocation); calls on one GPU must not overlap."""
    import torch
    _dev_tensor(holo, torch.complex64, (p.nt, p.ny, p.nx), "holo")
    _dev_tensor(cov, torch.complex128, (p.nt, p.nt), "cov")
    _check(lib().hh_covariance_noalloc(ctypes.byref(p.c()), _ptr(holo), _ptr(cov), _stream(stream)))
    return cov


def covariance_noalloc_max_bytes() -> int:
    return int(lib().hh_covariance_noalloc_max_bytes())


def hh_covariance_frames(p: Params, frames, cov, workspace, stream=None):
    """C = nx ny I^T I exactly from the uint16 frames; see include/hh.h."""
    import torch
    _dev_tensor(frames, torch.uint16, (p.nt, p.ny, p.nx), "frames")
    _dev_tensor(cov, torch.complex128, (p.nt, p.nt), "cov")
    _check(lib().hh_covariance_frames(ctypes.byref(p.c()), _ptr(frames), _ptr(cov), _ptr(workspace),
                                      workspace.numel() * workspace.element_size(), _stream(stream)))
    return cov


def hh_eigh(nt: int, cov, evals, evecs, info, max_sweeps=None, stream=None):
    """Step (c): cov complex128 [nt, nt] -> evals float64 [nt] (descending),
    evecs complex128 [nt, nt] (column k = eigenvector k), info int32 [1]."""
    import torch
    _dev_tensor(cov, torch.complex128, (nt, nt), "cov")
    _dev_tensor(evals, torch.float64, (nt,), "evals")
    _dev_tensor(evecs, torch.complex128, (nt, nt), "evecs")
    _dev_tensor(info, torch.int32, (1,), "info")
    if max_sweeps is None:
        st = lib().hh_eigh(nt, _ptr(cov), _ptr(evals), _ptr(evecs), _ptr(info), _stream(stream))
    else:
        st = lib().hh_eigh_ex(nt, _ptr(cov), _ptr(evals), _ptr(evecs), _ptr(info), int(max_sweeps),
                              _stream(stream))
    _check(st)


def hh_eigh_tridiag(nt: int, cov, evals, evecs, info, max_iter=40, stream=None):
    """Step (c) by Householder tridiagonalisation and implicit QL; see include/hh.h."""
    import torch
    _dev_tensor(cov, torch.complex128, (nt, nt), "cov")
    _dev_tensor(evals, torch.float64, (nt,), "evals")
    _dev_tensor(evecs, torch.complex128, (nt, nt), "evecs")
    _dev_tensor(info, torch.int32, (1,), "info")
    _check(lib().hh_eigh_tridiag(nt, _ptr(cov), _ptr(evals), _ptr(evecs), _ptr(info), int(max_iter),
                                 _stream(stream)))


def hh_project_render(p: Params, holo, evecs, image, stream=None):
    """Steps (d)+(e): holo complex64 [nt, ny, nx], evecs complex128 [nt, nt] -> image float32 [ny, nx]."""
    import torch
    _dev_tensor(holo, torch.complex64, (p.nt, p.ny, p.nx), "holo")
    _dev_tensor(evecs, torch.complex128, (p.nt, p.nt), "evecs")
    _dev_tensor(image, torch.float32, (p.ny, p.nx), "image")
    _check(lib().hh_project_render(ctypes.byref(p.c()), _ptr(holo), _ptr(evecs), _ptr(image), _stream(stream)))
    return image


def project_frames_workspace_bytes(p: Params) -> int:
    return int(lib().hh_project_frames_workspace_bytes(ctypes.byref(p.c())))


def hh_project_frames(p: Params, frames, evecs, image, workspace, stream=None):
    """Steps (d)+(e) from the frames (projection first): frames uint16 [nt, ny, nx],
    evecs complex128 [nt, nt] -> image float32 [ny, nx]; see include/hh.h."""
    import torch
    _dev_tensor(frames, torch.uint16, (p.nt, p.ny, p.nx), "frames")
    _dev_tensor(evecs, torch.complex128, (p.nt, p.nt), "evecs")
    _dev_tensor(image, torch.float32, (p.ny, p.nx), "image")
    _check(lib().hh_project_frames(ctypes.byref(p.c()), _ptr(frames), _ptr(evecs), _ptr(image), _ptr(workspace),
                                   workspace.numel() * workspace.element_size(), _stream(stream)))
    return image


def hh_svd_filter(p: Params, holo, evecs, out, stream=None):
    """Eq. (3): the stack with the dropped components removed; see include/hh.h."""
    import torch
    _dev_tensor(holo, torch.complex64, (p.nt, p.ny, p.nx), "holo")
    _dev_tensor(evecs, torch.complex128, (p.nt, p.nt), "evecs")
    _dev_tensor(out, torch.complex64, (p.nt, p.ny, p.nx), "out")
    _check(lib().hh_svd_filter(ctypes.byref(p.c()), _ptr(holo), _ptr(evecs), _ptr(out), _stream(stream)))
    return out


def hh_fourier_render(p: Params, holo, image, stream=None):
    """Eqs. (8)-(9): temporal-DFT band k_lo..k_hi power image."""
    import torch
    _dev_tensor(holo, torch.complex64, (p.nt, p.ny, p.nx), "holo")
    _dev_tensor(image, torch.float32, (p.ny, p.nx), "image")
    _check(lib().hh_fourier_render(ctypes.byref(p.c()), _ptr(holo), _ptr(image), _stream(stream)))
    return image


def hh_fourier_render_windows(p: Params, holo, nwin: int, hop: int, images, stream=None):
    """Eqs. (8)-(9) for nwin windows of a stream: window w is holo[w*hop : w*hop + nt]."""
    import torch
    _dev_tensor(holo, torch.complex64, ((nwin - 1) * hop + p.nt, p.ny, p.nx), "holo")
    _dev_tensor(images, torch.float32, (nwin, p.ny, p.nx), "images")
    _check(lib().hh_fourier_render_windows(ctypes.byref(p.c()), _ptr(holo), nwin, hop, _ptr(images),
                                           _stream(stream)))
    return images


def hh_pipeline(p: Params, frames, image, workspace, evals=None, evecs=None, info=None, stream=None):
    """Steps (a)-(e): frames uint16 [nt, ny, nx] -> image float32 [ny, nx]."""
    import torch
    _dev_tensor(frames, torch.uint16, (p.nt, p.ny, p.nx), "frames")
    _dev_tensor(image, torch.float32, (p.ny, p.nx), "image")
    if evals is not None:
        _dev_tensor(evals, torch.float64, (p.nt,), "evals")
    if evecs is not None:
        _dev_tensor(evecs, torch.complex128, (p.nt, p.nt), "evecs")
    if info is not None:
        _dev_tensor(info, torch.int32, (1,), "info")
    _check(lib().hh_pipeline(ctypes.byref(p.c()), _ptr(frames), _ptr(image), _ptr(evals), _ptr(evecs),
                             _ptr(info), _ptr(workspace), workspace.numel() * workspace.element_size(),
                             _stream(stream)))
    return image


def _param_array(ps):
    arr = (hh_params * len(ps))()
    for i, p in enumerate(ps):
        arr[i] = p.c()
    return arr


def batch_workspace_bytes(ps) -> int:
    return int(lib().hh_batch_workspace_bytes(_param_array(ps), len(ps)))


class Batch:
    """Prepared arguments of hh_pipeline_batch (built once, launched many times)."""

    def __init__(self, ps, frames, images, workspace, evals=None, evecs=None, infos=None):
        import torch
        n = len(ps)
        if not (len(frames) == len(images) == n):
            raise ValueError("one frames and one image tensor per stack")
        for i, p in enumerate(ps):
            _dev_tensor(frames[i], torch.uint16, (p.nt, p.ny, p.nx), f"frames[{i}]")
            _dev_tensor(images[i], torch.float32, (p.ny, p.nx), f"images[{i}]")
        self.params = _param_array(ps)
        self.stacks = (hh_stack * n)()
        for i in range(n):
            self.stacks[i] = hh_stack(frames[i].data_ptr(), images[i].data_ptr(),
                                      evals[i].data_ptr() if evals else None,
                                      evecs[i].data_ptr() if evecs else None,
                                      infos[i].data_ptr() if infos else None)
        self.n = n
        self.keep = (frames, images, workspace, evals, evecs, infos)
        self.ws = workspace

    def run(self, stream=None):
        _check(lib().hh_pipeline_batch(self.params, self.n, self.stacks, _ptr(self.ws),
                                       self.ws.numel() * self.ws.element_size(), _stream(stream)))


class Graph:
    """hh_graph_create / hh_graph_launch / hh_graph_destroy: a batch captured once as
    a HIP graph and replayed with one launch.  The tensors are kept alive with it."""

    def __init__(self, ps, frames, images, workspace, evals=None, evecs=None, infos=None):
        b = Batch(ps, frames, images, workspace, evals, evecs, infos)
        self.keep = b
        h = ctypes.c_void_p()
        _check(lib().hh_graph_create(b.params, b.n, b.stacks, _ptr(workspace),
                                     workspace.numel() * workspace.element_size(), ctypes.byref(h)))
        self.h = h

    def launch(self, stream=None):
        _check(lib().hh_graph_launch(self.h, _stream(stream)))

    def close(self):
        if self.h:
            import torch
            torch.cuda.synchronize()
            lib().hh_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hh_pipeline_batch(ps, frames, images, workspace, evals=None, evecs=None, infos=None, stream=None):
    """Steps (a)-(e) on a batch of (possibly uneven) stacks; see include/hh.h."""
    Batch(ps, frames, images, workspace, evals, evecs, infos).run(stream)
    return images


def analyze_batch_workspace_bytes(ps) -> int:
    return int(lib().hh_analyze_batch_workspace_bytes(_param_array(ps), len(ps)))


def hh_analyze_batch(ps, holos, images, workspace, evals=None, evecs=None, infos=None, stream=None):
    """Steps (b)-(e) on a batch of hologram stacks the caller holds (e.g. views of a
    ring of holograms); see include/hh.h."""
    import torch
    n = len(ps)
    if not (len(holos) == len(images) == n):
        raise ValueError("one hologram stack and one image tensor per stack")
    wins = (hh_window * n)()
    for i, p in enumerate(ps):
        _dev_tensor(holos[i], torch.complex64, (p.nt, p.ny, p.nx), f"holos[{i}]")
        _dev_tensor(images[i], torch.float32, (p.ny, p.nx), f"images[{i}]")
        if evals:
            _dev_tensor(evals[i], torch.float64, (p.nt,), f"evals[{i}]")
        if evecs:
            _dev_tensor(evecs[i], torch.complex128, (p.nt, p.nt), f"evecs[{i}]")
        if infos:
            _dev_tensor(infos[i], torch.int32, (1,), f"infos[{i}]")
        wins[i] = hh_window(holos[i].data_ptr(), images[i].data_ptr(),
                            evals[i].data_ptr() if evals else None,
                            evecs[i].data_ptr() if evecs else None,
                            infos[i].data_ptr() if infos else None)
    _check(lib().hh_analyze_batch(_param_array(ps), n, wins, _ptr(workspace),
                                  workspace.numel() * workspace.element_size(), _stream(stream)))
    return images


def tuning_get(p: Params) -> dict:
    t = hh_tuning()
    _check(lib().hh_tuning_get(ctypes.byref(p.c()), ctypes.byref(t)))
    return t.as_dict()


def tuning_set(p: Params, fft_rows=0, fft_cols=0, gram_pxw=256, group=0, gram_ref=0, fused=0):
    t = hh_tuning(fft_rows, fft_cols, gram_pxw, group, gram_ref, fused)
    _check(lib().hh_tuning_set(ctypes.byref(p.c()), ctypes.byref(t)))


def tuning_reset():
    lib().hh_tuning_reset()


def autotune(p: Params, frames, workspace, reps: int = 5, stream=None) -> dict:
    """Times the launch choices on `frames` and keeps the fastest for this shape; see include/hh.h."""
    import torch
    _dev_tensor(frames, torch.uint16, (p.nt, p.ny, p.nx), "frames")
    t = hh_tuning()
    _check(lib().hh_autotune(ctypes.byref(p.c()), _ptr(frames), _ptr(workspace),
                             workspace.numel() * workspace.element_size(), reps, ctypes.byref(t), _stream(stream)))
    return t.as_dict()


def alloc_workspace(nbytes: int, device="cuda"):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def profile_enable(on: bool = True):
    lib().hh_profile_enable(1 if on else 0)


def profile_reset():
    lib().hh_profile_reset()


def profile_read() -> dict:
    import json
    size = 1 << 16
    while True:  # one formatting per read: the buffer is grown until the text fits whole
        buf = ctypes.create_string_buffer(size)
        n = lib().hh_profile_read(buf, size)
        if n <= size:
            break
        size = n + 4096
    return {k: (int(v[0]), float(v[1])) for k, v in json.loads(buf.value.decode()).items()}
