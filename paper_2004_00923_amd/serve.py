"""Streaming PCA holography: sliding windows over camera streams on one GPU.

Each camera delivers uint16 frames at its frame rate, numbered by a sequence
counter.  An image is produced for every window of `window` consecutive frames,
one window every `hop` frames (the paper's 32-frame stacks computed while the
frames stream in, Sec. 2 and Table 1).  Frames are copied to the device as they
arrive, transformed once (step (a), hh_fresnel) into a ring of holograms, and
every window whose frames have all been transformed is analysed (steps
(b)-(e)).  Windows of all cameras that are ready together go through one
hh_analyze_batch call, which solves all their eigenproblems in one launch
(continuous batching across cameras).

A camera may instead demodulate by the temporal Fourier transform (Eqs. (8)-(9),
the paper's comparison method, `demod="fourier"`): each window's image is the
power in a band of temporal frequencies (hh_fourier_render, no covariance or
eigenproblem), typically at hop 1, one image per frame (the FFT row of Table 1).

Ring layout (per camera).  The hologram ring has R + M slots, R a multiple of
`hop` and M = max(window - hop, 0).  Frame k lands in slot k mod R, and again in
slot R + (k mod R) when k mod R < M.  Window c (frames c*hop .. c*hop+window-1)
starts at slot (c*hop) mod R <= R - hop, so it always occupies `window`
contiguous slots and is handed to the library as a plain [window][ny][nx]
stack.  Frame k + R reuses frame k's slots, so frames are only copied below
next*hop + R, `next` being the oldest window not yet analysed.

Frames that never reach the device are "lost": a sequence number the camera
skipped (a gap), or a frame dropped because the bounded host ingest queue
(frames arrived but not yet copied) was full when it arrived.  A window that
contains a lost frame is skipped and counted; the paper's requirement is that
none are ("no frame drop", Table 1), which the counts make checkable.

The scheduling decisions are made by `Scheduler` (host arithmetic only, no
device); `Server` carries them out with HIP copies and the library calls.
Admission: a camera is admitted when its rings, image buffers and analysis
workspace fit in the HBM budget still free.  `Server.admit` admits at once or
raises AdmissionError; `Server.submit` queues a request that `Server.run`
admits, in arrival order, as soon as earlier cameras finish or disconnect and
release their memory, and that camera then joins the batches already running.
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
    ring_hops: int = 6               # frame ring of ring_hops * hop frames (>= one window): how
                                     # far frames may run ahead of the oldest pending window
    demod: str = "pca"               # "pca": Eqs. (4)-(7), components k_lo..k_hi; "fourier": Eqs. (8)-(9),
                                     # temporal frequencies k_lo..k_hi (0-based)

    def ring(self) -> "RingPlan":
        return RingPlan(self.window, self.hop, self.ring_hops)

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

    def window_runs(self, cs: List[int], n_images: int) -> List[Tuple[int, int]]:
        """Runs (first window, count) of the increasing window indices cs that one launch
        can take: consecutive windows whose frames lie in one contiguous stretch of the
        hologram ring (mirror copies included) and whose images are contiguous among the
        n_images buffers."""
        runs: List[Tuple[int, int]] = []
        for c in cs:
            if runs:
                c0, k = runs[-1]
                s0 = self.window_slot(c0)
                if c == c0 + k and s0 + k * self.hop + self.window <= self.slots and c0 % n_images + k < n_images:
                    runs[-1] = (c0, k + 1)
                    continue
            runs.append((c, 1))
        return runs

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
    target: int                 # windows to produce (or skip)
    queue_cap: int = 1 << 30    # frames the host ingest queue holds (arrived, not yet copied)
    missing: frozenset = frozenset()  # sequence numbers the camera never delivers (gaps)
    arrived: int = 0            # frames that have arrived (sequence numbers below this)
    delivered: int = 0          # frames below this are copied to the device or lost
    transformed: int = 0        # frames below this are transformed into the hologram ring
    next_c: int = 0             # oldest window not yet analysed or skipped
    lost: set = dataclasses.field(default_factory=set)   # gaps and ingest drops, not yet consumed
    dropped: int = 0            # frames dropped at ingest (queue full)
    gaps: int = 0               # frames missing from the camera's sequence
    skipped: int = 0            # windows skipped because they contain a lost frame
    analysed: int = 0           # windows sent to analysis
    stopped: bool = False       # disconnected: no more frames, pending windows abandoned

    def done(self) -> bool:
        return self.stopped or self.next_c >= self.target

    def queued(self) -> int:
        """Frames waiting in the ingest queue (arrived, neither copied nor lost)."""
        return self.arrived - self.delivered - sum(1 for k in self.lost if k >= self.delivered)

    def window_lost(self, c: int) -> bool:
        a, b = self.ring.window_frames(c)
        return any(a <= k < b for k in self.lost)


class Scheduler:
    """Plans one pass of the serving loop from the frames each camera has made
    available (a count of sequence numbers per camera name).  Returns actions in
    the order they are to be enqueued:
      ("copy", cam, a, b, lost) frames [a, b) into frame-ring slots (never wrapping past
                                 a window that is still pending), except the lost ones
                                 (the caller splits the copy around them)
      ("fresnel", cam, runs)    transforms (src slot, dst slot, n) of the copied frames
      ("analyse", [(cam, c)])   one batched analysis of the ready windows, oldest first,
                                 at most max_batch in all and per_camera per camera
    `cam` is the camera's name.  Cameras are added and removed while it runs."""

    def __init__(self, states=None, max_batch: int = 16, per_camera: int = 2):
        if isinstance(states, list):   # positional cameras, named 0..n-1
            states = {i: s for i, s in enumerate(states)}
        self.st: Dict = dict(states or {})
        self.max_batch = max_batch
        self.per_camera = per_camera

    def add(self, name, state: CamState):
        self.st[name] = state

    def remove(self, name) -> CamState:
        return self.st.pop(name)

    def _arrive(self, s: CamState, avail: int):
        # frames arriving since the last pass, in sequence order: a gap is lost; a
        # frame that finds the ingest queue full is dropped (tail drop)
        q = s.queued()
        for k in range(s.arrived, avail):
            if k in s.missing:
                s.lost.add(k)
                s.gaps += 1
            elif q >= s.queue_cap:
                s.lost.add(k)
                s.dropped += 1
            else:
                q += 1
        s.arrived = max(s.arrived, avail)

    def step(self, available):
        if isinstance(available, list):
            available = {i: a for i, a in enumerate(available)}
        acts, ready = [], []
        for i, s in self.st.items():
            if s.done():
                continue
            need = s.ring.window_frames(s.target - 1)[1]
            self._arrive(s, min(available.get(i, 0), need))
            upto = min(s.arrived, need, s.ring.admit_limit(s.next_c))
            if upto > s.delivered:
                acts.append(("copy", i, s.delivered, upto,
                             frozenset(k for k in s.lost if s.delivered <= k < upto)))
                s.delivered = upto
            if s.delivered > s.transformed:
                acts.append(("fresnel", i, s.ring.fresnel_runs(s.transformed, s.delivered)))
                s.transformed = s.delivered
        # windows holding a lost frame are skipped (in order, so the ring advances);
        # then continuous batching: ready windows of every camera, oldest first
        cand = []
        for i, s in self.st.items():
            if s.done():
                continue
            c = s.next_c
            while c < s.target and s.ring.window_frames(c)[1] <= s.transformed:
                cand.append((s.ring.window_frames(c)[1], i, c))
                c += 1
        cand.sort(key=lambda x: (x[0], str(x[1]), x[2]))
        taken = {}
        for _, i, c in cand:
            s = self.st[i]
            if c != taken.get(i, s.next_c):   # keep each camera's windows in order
                continue
            if s.window_lost(c):
                s.skipped += 1
                taken[i] = c + 1
                continue
            if len(ready) >= self.max_batch or sum(1 for j, _ in ready if j == i) >= self.per_camera:
                continue
            ready.append((i, c))
            taken[i] = c + 1
        for i, nxt in taken.items():
            s = self.st[i]
            s.next_c = nxt
            s.lost = {k for k in s.lost if k >= s.next_c * s.ring.hop}   # no later window holds them
        for i, _ in ready:
            self.st[i].analysed += 1
        if ready:
            acts.append(("analyse", ready))
        return acts


PER_CAMERA = 4   # windows of one camera per analysis batch (sizes its workspace share)


def camera_bytes(spec: CameraSpec, ring: RingPlan, image_buffers: int,
                 batch_per_camera: int = PER_CAMERA) -> Dict[str, int]:
    """Device bytes one camera needs: frame ring, hologram ring, image buffers and
    its share of the analysis workspace (batch_per_camera windows)."""
    npix = spec.ny * spec.nx
    ws = hh.analyze_batch_workspace_bytes([spec.params()] * batch_per_camera)
    if ws == 0:
        raise ValueError(f"camera {spec.name}: parameters rejected by the library")
    if spec.demod == "fourier":
        ws = 0   # the Fourier image needs no workspace
    return {"frames": ring.R * npix * 2, "holo": ring.slots * npix * 8, "images": image_buffers * npix * 4,
            "workspace": ws}


class Admission:
    """HBM budget bookkeeping (host only): what each admitted camera holds."""

    def __init__(self, budget_bytes: int, image_buffers: int = 4):
        self.budget = int(budget_bytes)
        self.used = 0
        self.image_buffers = image_buffers
        self.held: Dict[str, int] = {}

    def fits(self, spec: CameraSpec, ring: RingPlan) -> bool:
        return self.used + sum(camera_bytes(spec, ring, self.image_buffers).values()) <= self.budget

    def request(self, spec: CameraSpec, ring: RingPlan) -> Dict[str, int]:
        need = camera_bytes(spec, ring, self.image_buffers)
        total = sum(need.values())
        if spec.name in self.held:
            raise AdmissionError(f"camera {spec.name}: already admitted")
        if self.used + total > self.budget:
            raise AdmissionError(f"camera {spec.name}: needs {total} bytes, {self.budget - self.used} of the "
                                 f"{self.budget}-byte HBM budget free")
        self.used += total
        self.held[spec.name] = total
        return need

    def release(self, name: str) -> int:
        """Returns the camera's bytes to the budget (0 if it held none)."""
        total = self.held.pop(name, 0)
        self.used -= total
        return total


@dataclasses.dataclass
class CameraRequest:
    """A camera asking to be served (Server.submit).  It is admitted, in request
    order, once its memory fits the HBM budget; it streams from its admission on."""
    spec: CameraSpec
    source: object                       # pinned host uint16 tensor [n_src][ny][nx], replayed cyclically
    windows: int                         # windows to produce (analysed or skipped)
    at_s: float = 0.0                    # request time, seconds after Server.run starts
    disconnect_s: Optional[float] = None  # the camera stops streaming this long after its admission
    missing: frozenset = frozenset()     # sequence numbers the camera skips (gaps)
    queue_cap: int = 1 << 30             # frames the host ingest queue holds


class _Camera:
    def __init__(self, spec: CameraSpec, ring: RingPlan, source, image_buffers: int, device):
        import torch
        self.spec, self.ring, self.src = spec, ring, source
        self.p = spec.params()
        self.n_src = source.shape[0]
        self.u16 = torch.empty((ring.R, spec.ny, spec.nx), dtype=torch.uint16, device=device)
        self.holo = torch.empty((ring.slots, spec.ny, spec.nx), dtype=torch.complex64, device=device)
        # one buffer, so that the images of consecutive windows are contiguous
        self.image_buf = torch.empty((image_buffers, spec.ny, spec.nx), dtype=torch.float32, device=device)
        self.images = [self.image_buf[i] for i in range(image_buffers)]
        self.slot_free = [(-1, None)] * ring.R  # (order, compute-stream event after the transform that read it)
        self.last_copy = None                   # copy-stream event after the latest copy
        self.copy_start = {}                    # frame -> event recorded before its copy (latency start)
        self.req: Optional[CameraRequest] = None
        self.state: Optional[CamState] = None
        self.start = 0.0                        # wall time its stream starts
        self.admitted_s = 0.0


class Server:
    """Continuous-batching server over several cameras on one GPU."""

    def __init__(self, hbm_budget_bytes: int, device="cuda:0", image_buffers: int = 4, max_batch: int = 16):
        import torch
        self.device = torch.device(device)
        self.adm = Admission(hbm_budget_bytes, image_buffers)
        self.max_batch = max_batch
        self.cams: List[_Camera] = []
        self.pending: List[CameraRequest] = []
        self.copy_stream = torch.cuda.Stream(device=self.device)
        self.compute_stream = torch.cuda.Stream(device=self.device)
        self.ws = None
        self.kept: Dict[Tuple[str, int], object] = {}
        self.keep_windows = set()
        self.released: Dict[str, dict] = {}
        self._order = 0

    # -------------------------------------------------------------- admission ----
    def _check(self, spec: CameraSpec, source):
        if tuple(source.shape[1:]) != (spec.ny, spec.nx):
            raise ValueError(f"camera {spec.name}: source frames must be [n][{spec.ny}][{spec.nx}]")
        if spec.precision in ("fp16store", "exact"):
            raise ValueError(f"camera {spec.name}: the rings hold FP32 holograms; form {spec.precision} "
                             "starts from frames and does not apply")
        if spec.demod not in ("pca", "fourier"):
            raise ValueError(f"camera {spec.name}: demod must be 'pca' or 'fourier', not {spec.demod!r}")
        if any(c.spec.name == spec.name for c in self.cams) or any(r.spec.name == spec.name for r in self.pending):
            raise ValueError(f"camera {spec.name}: name already in use")

    def _resize_workspace(self):
        # no analysis may be in flight on the old workspace
        self.compute_stream.synchronize()
        ws_bytes = sum(camera_bytes(c.spec, c.ring, self.adm.image_buffers)["workspace"] for c in self.cams)
        self.ws = hh.alloc_workspace(ws_bytes, self.device) if ws_bytes else None

    def _add(self, spec: CameraSpec, source) -> Tuple[_Camera, Dict[str, int]]:
        ring = spec.ring()
        need = self.adm.request(spec, ring)
        cam = _Camera(spec, ring, source, self.adm.image_buffers, self.device)
        self.cams.append(cam)
        self._resize_workspace()
        return cam, need

    def admit(self, spec: CameraSpec, source) -> Dict[str, int]:
        """Admit a camera now if its memory fits the budget still free (raises
        AdmissionError).  `source`: pinned host uint16 tensor [n_src][ny][nx] of
        frames replayed cyclically.  Its windows are given to run()."""
        self._check(spec, source)
        return self._add(spec, source)[1]

    def submit(self, req: CameraRequest):
        """Queue a camera; run() admits it once it has been requested and fits."""
        self._check(req.spec, req.source)
        if sum(camera_bytes(req.spec, req.spec.ring(), self.adm.image_buffers).values()) > self.adm.budget:
            raise AdmissionError(f"camera {req.spec.name}: larger than the whole HBM budget")
        self.pending.append(req)

    @staticmethod
    def _stats(cam: _Camera) -> dict:
        st = cam.state
        return {"analysed": st.analysed, "skipped": st.skipped, "dropped_frames": st.dropped, "gap_frames": st.gaps,
                "abandoned": max(0, st.target - st.next_c) if st.stopped else 0, "admitted_s": cam.admitted_s}

    def _release(self, cam: _Camera, sched: Scheduler, now: float):
        # its last copies and analyses must be complete before its memory is reused
        self.copy_stream.synchronize()
        self.compute_stream.synchronize()
        self.released[cam.spec.name] = dict(self._stats(cam), released_s=now)
        sched.remove(cam.spec.name)
        self.adm.release(cam.spec.name)
        self.cams.remove(cam)
        self._resize_workspace()

    # ------------------------------------------------------------- execution ----
    def _copy(self, cam: _Camera, a: int, b: int, lost):
        """Frames [a, b) except the lost ones: one copy per run of frames that are
        contiguous in the ring and in the source."""
        import torch
        with torch.cuda.stream(self.copy_stream):
            k = a
            while k < b:
                if k in lost:
                    k += 1
                    continue
                s0, j0 = cam.ring.slot(k), k % cam.n_src
                n = 1
                while (k + n < b and k + n not in lost and s0 + n < cam.ring.R and j0 + n < cam.n_src):
                    n += 1
                # the slots' last reader: the transforms are ordered on the compute stream
                order, ev = max(cam.slot_free[s0:s0 + n], key=lambda x: x[0])
                if ev is not None:
                    self.copy_stream.wait_event(ev)
                e = torch.cuda.Event(enable_timing=True)
                e.record(self.copy_stream)
                for kk in range(k, k + n):
                    cam.copy_start[kk] = e
                cam.u16[s0:s0 + n].copy_(cam.src[j0:j0 + n], non_blocking=True)
                k += n
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
        self._order += 1
        for src, dst, n in runs:
            for s in range(src, src + n):
                cam.slot_free[s] = (self._order, ev)

    def _analyse(self, ready, records):
        import torch
        by_name = {c.spec.name: c for c in self.cams}
        ps, holos, pimgs, imgs = [], [], [], []
        fourier = {}   # camera -> its ready windows (Eqs. (8)-(9): no covariance, no eigenproblem)
        for name, c in ready:
            cam = by_name[name]
            s = cam.ring.window_slot(c)
            img = cam.images[c % len(cam.images)]
            imgs.append(img)
            if cam.spec.demod == "fourier":
                fourier.setdefault(name, []).append(c)
            else:
                ps.append(cam.p)
                holos.append(cam.holo[s:s + cam.spec.window])
                pimgs.append(img)
        for name, cs in fourier.items():
            # one launch per run of consecutive windows (the frames they share are read once from HBM)
            cam = by_name[name]
            n_img = len(cam.images)
            for c0, k in cam.ring.window_runs(sorted(cs), n_img):
                s, i0 = cam.ring.window_slot(c0), c0 % n_img
                frames = (k - 1) * cam.spec.hop + cam.spec.window
                hh.hh_fourier_render_windows(cam.p, cam.holo[s:s + frames], k, cam.spec.hop,
                                             cam.image_buf[i0:i0 + k], stream=self.compute_stream)
        if ps:
            hh.hh_analyze_batch(ps, holos, pimgs, self.ws, stream=self.compute_stream)
        done = torch.cuda.Event(enable_timing=True)
        done.record(self.compute_stream)
        with torch.cuda.stream(self.compute_stream):
            for (name, c), img in zip(ready, imgs):
                if (name, c) in self.keep_windows:
                    self.kept[(name, c)] = img.clone()
        for name, c in ready:
            cam = by_name[name]
            last = cam.ring.window_frames(c)[1] - 1
            records.append((name, c, len(ready), cam.copy_start[last], done))
            for k in [k for k in cam.copy_start if k <= last]:
                del cam.copy_start[k]
        return done

    def run(self, windows: Optional[Dict[str, int]] = None, paced: bool = True, max_inflight: int = 3,
            poll_s: float = 2e-4):
        """Serve until every camera has produced its windows (windows[name] for
        cameras admitted with admit(), which stay admitted for later runs; the
        request's count for submitted ones, which leave when served) or disconnected,
        and every submitted camera has been served.  paced: frames
        arrive at each camera's rate (wall clock); else as fast as the GPU takes them,
        with at most `max_inflight` analysis batches queued.  Per-window latency is
        measured with GPU events from just before the copy of the window's last frame
        to the end of its analysis.  A camera that is done releases its memory, and
        waiting requests are admitted in order as it frees up."""
        import torch
        windows = dict(windows or {})
        sched = Scheduler({}, self.max_batch, PER_CAMERA)
        t0 = time.perf_counter()
        for cam in self.cams:   # cameras admitted with admit() stay admitted across runs
            cam.state = CamState(cam.ring, windows.get(cam.spec.name, 0))
            cam.start, cam.admitted_s = t0, 0.0
            cam.slot_free = [(-1, None)] * cam.ring.R
            cam.copy_start = {}
            sched.add(cam.spec.name, cam.state)
        records, inflight, host_lag, waits = [], [], [], {}
        while True:
            now = time.perf_counter()
            for cam in list(self.cams):
                st = cam.state
                if (cam.req and cam.req.disconnect_s is not None and not st.stopped
                        and now - cam.start >= cam.req.disconnect_s):
                    st.stopped = True
                if st.done() and cam.req is not None:   # a served request leaves and frees its memory
                    self._release(cam, sched, now - t0)
            # admit waiting requests in order while they fit
            while self.pending and now - t0 >= self.pending[0].at_s:
                req = self.pending[0]
                if not self.adm.fits(req.spec, req.spec.ring()):
                    if all(c.req is None for c in self.cams):
                        # only cameras admitted with admit() hold memory, and they keep it
                        raise AdmissionError(f"camera {req.spec.name}: can never fit next to the cameras "
                                             f"admitted with admit() ({self.adm.used} of {self.adm.budget} bytes)")
                    break
                self.pending.pop(0)
                cam, _ = self._add(req.spec, req.source)
                now = time.perf_counter()
                cam.req, cam.start, cam.admitted_s = req, now, now - t0
                cam.state = CamState(cam.ring, req.windows, queue_cap=req.queue_cap, missing=req.missing)
                waits[req.spec.name] = now - t0 - req.at_s
                sched.add(req.spec.name, cam.state)
            if not self.pending and all(c.state.done() for c in self.cams):
                break
            avail = {}
            for cam in self.cams:
                st = cam.state
                if paced:
                    avail[cam.spec.name] = int((now - cam.start) * cam.spec.fps) + 1
                else:   # as many frames as the next batch of this camera's windows needs
                    avail[cam.spec.name] = st.ring.window_frames(st.next_c + PER_CAMERA - 1)[1]
            acts = sched.step(avail)
            by_name = {c.spec.name: c for c in self.cams}
            for a in acts:
                if a[0] == "copy":
                    cam = by_name[a[1]]
                    if paced:
                        host_lag.append(now - (cam.start + (a[3] - 1) / cam.spec.fps))
                    self._copy(cam, a[2], a[3], a[4])
                elif a[0] == "fresnel":
                    self._fresnel(by_name[a[1]], a[2])
                else:
                    inflight.append(self._analyse(a[1], records))
                    while len(inflight) > max_inflight:
                        inflight.pop(0).synchronize()
            if not acts:
                if paced or self.pending:
                    time.sleep(poll_s)
        torch.cuda.synchronize(self.device)
        wall = time.perf_counter() - t0
        out = [{"camera": n, "window": c, "batch": b, "latency_ms": s.elapsed_time(d)}
               for n, c, b, s, d in records]
        cams = dict(self.released)
        cams.update({c.spec.name: self._stats(c) for c in self.cams})
        return {"windows": out, "wall_s": wall, "host_lag_ms_max": 1e3 * max(host_lag) if host_lag else 0.0,
                "cameras": cams, "admission_wait_s": waits}


def summarize(result: dict, cams: List[CameraSpec]) -> dict:
    import numpy as np
    out = {"wall_s": result["wall_s"], "host_lag_ms_max": result["host_lag_ms_max"],
           "cameras": result.get("cameras", {})}
    for spec in cams:
        lat = np.array([w["latency_ms"] for w in result["windows"] if w["camera"] == spec.name])
        if lat.size == 0:
            continue
        out[spec.name] = {"windows": int(lat.size), "p50_ms": float(np.percentile(lat, 50)),
                          "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max()),
                          "windows_per_s": lat.size / result["wall_s"],
                          "interferograms_per_s": lat.size * spec.hop / result["wall_s"]}
    return out
