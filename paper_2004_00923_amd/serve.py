"""Streaming PCA holography: sliding windows over camera streams on one GPU.

Each camera delivers uint16 frames at its frame rate.  An image is produced for
every window of `window` consecutive frames, one window every `hop` frames (the
paper's 32-frame stacks computed while the frames stream in, Sec. 2 and
Table 1).  Frames are copied to the device as they arrive, transformed once
(step (a), hh_fresnel) into a ring of holograms, and every window whose frames
have all been transformed is analysed (steps (b)-(e)).  Windows of all cameras
that are ready together go through one hh_analyze_batch call, which solves all
their eigenproblems in one launch (continuous batching across cameras).

Ring layout (per camera).  The hologram ring has R + M slots, R a multiple of
`hop` and M = max(window - hop, 0).  Frame k lands in slot k mod R, and again in
slot R + (k mod R) when k mod R < M.  Window c (frames c*hop .. c*hop+window-1)
starts at slot (c*hop) mod R <= R - hop, so it always occupies `window`
contiguous slots and is handed to the library as a plain [window][ny][nx]
stack.  Frame k + R reuses frame k's slots, so frames are only admitted below
next*hop + R, `next` being the oldest window not yet analysed.

The scheduling decisions are made by `Scheduler` (host arithmetic only, no
device); `Server` carries them out with HIP copies and the library calls.
Admission: a camera is admitted only if its rings, image buffers and analysis
workspace fit in the HBM budget still free; otherwise AdmissionError.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Dict, List, Optional, Tuple

from . import hh


class AdmissionError(RuntimeError):
    pass


@dataclasses.dataclass
class CameraSpec:
    name: str
    ny: int
    nx: int
    fps: float
    seed: int
    window: int = 32
    hop: int = 25
    k_lo: int = 2
    k_hi: Optional[int] = None       # default window - 1
    precision: str = "fp32"
    wavelength_m: float = 785e-9
    distance_m: float = 0.3
    pitch_m: float = 20e-6

    def params(self) -> hh.Params:
        return hh.Params(nx=self.nx, ny=self.ny, nt=self.window, k_lo=self.k_lo,
                         k_hi=self.window - 1 if self.k_hi is None else self.k_hi,
                         wavelength_m=self.wavelength_m, distance_m=self.distance_m, pitch_m=self.pitch_m,
                         precision=hh.PRECISIONS[self.precision])


class RingPlan:
    """Slot arithmetic of one camera's frame and hologram rings."""

    def __init__(self, window: int, hop: int, ring_hops: int = 2):
        if window < 2 or hop < 1:
            raise ValueError("window >= 2 and hop >= 1 required")
        self.window, self.hop = window, hop
        self.R = hop * max(ring_hops, -(-window // hop))   # >= window: one window always fits
        self.M = max(window - hop, 0)
        self.slots = self.R + self.M

    def slot(self, k: int) -> int:
        return k % self.R

    def window_frames(self, c: int) -> Tuple[int, int]:
        """Frame range [first, last + 1) of window c."""
        return c * self.hop, c * self.hop + self.window

    def window_slot(self, c: int) -> int:
        s = (c * self.hop) % self.R
        assert s + self.window <= self.slots
        return s

    def admit_limit(self, next_c: int) -> int:
        """Frames below this index may be written while window next_c is pending."""
        return next_c * self.hop + self.R

    def fresnel_runs(self, a: int, b: int) -> List[Tuple[int, int, int]]:
        """Transforms for frames [a, b): (source slot, destination slot, count) runs,
        contiguous in both rings, including the mirror copies."""
        runs = []
        k = a
        while k < b:
            s = self.slot(k)
            n = min(b - k, self.R - s)
            runs.append((s, s, n))
            if s < self.M:
                runs.append((s, self.R + s, min(n, self.M - s)))
            k += n
        return runs


@dataclasses.dataclass
class CamState:
    ring: RingPlan
    target: int                 # windows to produce
    delivered: int = 0          # frames copied to the device
    transformed: int = 0        # frames transformed into the hologram ring
    next_c: int = 0             # oldest window not yet analysed

    def done(self) -> bool:
        return self.next_c >= self.target


class Scheduler:
    """Plans one pass of the serving loop from the frames each camera has made
    available.  Returns actions in the order they are to be enqueued:
      ("copy", cam, a, b)       frames [a, b) into frame-ring slots (never wrapping past
                                 a window that is still pending)
      ("fresnel", cam, runs)    transforms (src slot, dst slot, n) of the copied frames
      ("analyse", [(cam, c)])   one batched analysis of the ready windows, oldest first,
                                 at most max_batch in all and per_camera per camera
    """

    def __init__(self, states: List[CamState], max_batch: int = 16, per_camera: int = 2):
        self.st = states
        self.max_batch = max_batch
        self.per_camera = per_camera

    def step(self, available: List[int]):
        acts, ready = [], []
        for i, s in enumerate(self.st):
            if s.done():
                continue
            need = s.ring.window_frames(s.target - 1)[1]
            upto = min(available[i], need, s.ring.admit_limit(s.next_c))
            if upto > s.delivered:
                acts.append(("copy", i, s.delivered, upto))
                s.delivered = upto
            if s.delivered > s.transformed:
                acts.append(("fresnel", i, s.ring.fresnel_runs(s.transformed, s.delivered)))
                s.transformed = s.delivered
        # continuous batching: ready windows of every camera, oldest window first
        cand = []
        for i, s in enumerate(self.st):
            c = s.next_c
            while c < s.target and s.ring.window_frames(c)[1] <= s.transformed:
                cand.append((s.ring.window_frames(c)[1], i, c))
                c += 1
        cand.sort()
        taken = {}
        for _, i, c in cand:
            if len(ready) >= self.max_batch:
                break
            if c != taken.get(i, self.st[i].next_c):   # keep each camera's windows in order
                continue
            if c - self.st[i].next_c >= self.per_camera:
                continue
            ready.append((i, c))
            taken[i] = c + 1
        for i, nxt in taken.items():
            self.st[i].next_c = nxt
        if ready:
            acts.append(("analyse", ready))
        return acts


PER_CAMERA = 2   # windows of one camera per analysis batch (sizes its workspace share)


def camera_bytes(spec: CameraSpec, ring: RingPlan, image_buffers: int,
                 batch_per_camera: int = PER_CAMERA) -> Dict[str, int]:
    """Device bytes one camera needs: frame ring, hologram ring, image buffers and
    its share of the analysis workspace (batch_per_camera windows)."""
    npix = spec.ny * spec.nx
    ws = hh.analyze_batch_workspace_bytes([spec.params()] * batch_per_camera)
    if ws == 0:
        raise ValueError(f"camera {spec.name}: parameters rejected by the library")
    return {"frames": ring.R * npix * 2, "holo": ring.slots * npix * 8, "images": image_buffers * npix * 4,
            "workspace": ws}


class Admission:
    """HBM budget bookkeeping (host only)."""

    def __init__(self, budget_bytes: int, image_buffers: int = 4):
        self.budget = int(budget_bytes)
        self.used = 0
        self.image_buffers = image_buffers

    def request(self, spec: CameraSpec, ring: RingPlan) -> Dict[str, int]:
        need = camera_bytes(spec, ring, self.image_buffers)
        total = sum(need.values())
        if self.used + total > self.budget:
            raise AdmissionError(f"camera {spec.name}: needs {total} bytes, {self.budget - self.used} of the "
                                 f"{self.budget}-byte HBM budget free")
        self.used += total
        return need


class _Camera:
    def __init__(self, spec: CameraSpec, ring: RingPlan, source, image_buffers: int, device):
        import torch
        self.spec, self.ring, self.src = spec, ring, source
        self.p = spec.params()
        self.n_src = source.shape[0]
        self.u16 = torch.empty((ring.R, spec.ny, spec.nx), dtype=torch.uint16, device=device)
        self.holo = torch.empty((ring.slots, spec.ny, spec.nx), dtype=torch.complex64, device=device)
        self.images = [torch.empty((spec.ny, spec.nx), dtype=torch.float32, device=device)
                       for _ in range(image_buffers)]
        self.slot_free = [None] * ring.R   # compute-stream event after the transform that read the slot
        self.last_copy = None              # copy-stream event after the latest copy
        self.copy_start = {}               # frame -> event recorded before its copy (latency start)


class Server:
    """Continuous-batching server over several cameras on one GPU."""

    def __init__(self, hbm_budget_bytes: int, device="cuda:0", image_buffers: int = 4, max_batch: int = 16):
        import torch
        self.device = torch.device(device)
        self.adm = Admission(hbm_budget_bytes, image_buffers)
        self.max_batch = max_batch
        self.cams: List[_Camera] = []
        self.copy_stream = torch.cuda.Stream(device=self.device)
        self.compute_stream = torch.cuda.Stream(device=self.device)
        self.ws = None
        self.kept: Dict[Tuple[str, int], object] = {}
        self.keep_windows = set()

    def admit(self, spec: CameraSpec, source) -> Dict[str, int]:
        """Admit a camera if its memory fits the budget still free (raises AdmissionError).
        `source`: pinned host uint16 tensor [n_src][ny][nx] of frames replayed cyclically."""
        if tuple(source.shape[1:]) != (spec.ny, spec.nx):
            raise ValueError(f"camera {spec.name}: source frames must be [n][{spec.ny}][{spec.nx}]")
        if spec.precision in ("fp16store", "exact"):
            raise ValueError(f"camera {spec.name}: the rings hold FP32 holograms; form {spec.precision} "
                             "starts from frames and does not apply")
        ring = RingPlan(spec.window, spec.hop)
        need = self.adm.request(spec, ring)
        self.cams.append(_Camera(spec, ring, source, self.adm.image_buffers, self.device))
        ws_bytes = sum(camera_bytes(c.spec, c.ring, self.adm.image_buffers)["workspace"] for c in self.cams)
        self.ws = hh.alloc_workspace(ws_bytes, self.device)
        return need

    def _copy(self, cam: _Camera, a: int, b: int):
        import torch
        with torch.cuda.stream(self.copy_stream):
            for k in range(a, b):
                s = cam.ring.slot(k)
                if cam.slot_free[s] is not None:
                    self.copy_stream.wait_event(cam.slot_free[s])
                e = torch.cuda.Event(enable_timing=True)
                e.record(self.copy_stream)
                cam.copy_start[k] = e
                cam.u16[s].copy_(cam.src[k % cam.n_src], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.copy_stream)
        cam.last_copy = ev

    def _fresnel(self, cam: _Camera, runs):
        import torch
        self.compute_stream.wait_event(cam.last_copy)
        for src, dst, n in runs:
            hh.hh_fresnel(cam.p, cam.u16[src:src + n], cam.holo[dst:dst + n], stream=self.compute_stream)
        ev = torch.cuda.Event()
        ev.record(self.compute_stream)
        for src, dst, n in runs:
            for s in range(src, src + n):
                cam.slot_free[s] = ev

    def _analyse(self, ready, records):
        import torch
        ps, holos, imgs = [], [], []
        for i, c in ready:
            cam = self.cams[i]
            s = cam.ring.window_slot(c)
            ps.append(cam.p)
            holos.append(cam.holo[s:s + cam.spec.window])
            imgs.append(cam.images[c % len(cam.images)])
        hh.hh_analyze_batch(ps, holos, imgs, self.ws, stream=self.compute_stream)
        done = torch.cuda.Event(enable_timing=True)
        done.record(self.compute_stream)
        with torch.cuda.stream(self.compute_stream):
            for (i, c), img in zip(ready, imgs):
                if (self.cams[i].spec.name, c) in self.keep_windows:
                    self.kept[(self.cams[i].spec.name, c)] = img.clone()
        for i, c in ready:
            cam = self.cams[i]
            last = cam.ring.window_frames(c)[1] - 1
            records.append((cam.spec.name, c, len(ready), cam.copy_start[last], done))
            for k in [k for k in cam.copy_start if k <= last]:
                del cam.copy_start[k]
        return done

    def run(self, windows: Dict[str, int], paced: bool = True, max_inflight: int = 2, poll_s: float = 2e-4):
        """Serve until each camera has produced windows[name] windows.  paced: frames
        arrive at each camera's rate (wall clock); else as fast as the GPU takes them,
        with at most `max_inflight` analysis batches queued.  Per-window latency is
        measured with GPU events from just before the copy of the window's last frame
        to the end of its analysis."""
        import torch
        states = [CamState(c.ring, windows.get(c.spec.name, 0)) for c in self.cams]
        sched = Scheduler(states, self.max_batch, PER_CAMERA)
        records, inflight, host_lag = [], [], []
        t0 = time.perf_counter()
        while not all(s.done() for s in states):
            now = time.perf_counter()
            if paced:
                avail = [int((now - t0) * c.spec.fps) + 1 for c in self.cams]
            else:
                avail = [s.ring.window_frames(s.next_c)[1] for s in states]
            acts = sched.step(avail)
            for a in acts:
                if a[0] == "copy":
                    cam = self.cams[a[1]]
                    if paced:
                        host_lag.append(now - (t0 + (a[3] - 1) / cam.spec.fps))
                    self._copy(cam, a[2], a[3])
                elif a[0] == "fresnel":
                    self._fresnel(self.cams[a[1]], a[2])
                else:
                    inflight.append(self._analyse(a[1], records))
                    while len(inflight) > max_inflight:
                        inflight.pop(0).synchronize()
            if paced and not acts:
                time.sleep(poll_s)
        torch.cuda.synchronize(self.device)
        wall = time.perf_counter() - t0
        out = [{"camera": n, "window": c, "batch": b, "latency_ms": s.elapsed_time(d)}
               for n, c, b, s, d in records]
        return {"windows": out, "wall_s": wall, "host_lag_ms_max": 1e3 * max(host_lag) if host_lag else 0.0}


def summarize(result: dict, cams: List[CameraSpec]) -> dict:
    import numpy as np
    out = {"wall_s": result["wall_s"], "host_lag_ms_max": result["host_lag_ms_max"]}
    for spec in cams:
        lat = np.array([w["latency_ms"] for w in result["windows"] if w["camera"] == spec.name])
        if lat.size == 0:
            continue
        out[spec.name] = {"windows": int(lat.size), "p50_ms": float(np.percentile(lat, 50)),
                          "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max()),
                          "windows_per_s": lat.size / result["wall_s"],
                          "interferograms_per_s": lat.size * spec.hop / result["wall_s"]}
    return out
