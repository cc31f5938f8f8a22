"""Seeded synthetic interferogram stacks (input synthesis only).

The paper's recordings of a volunteer's retina are not available, so every
input here is synthetic, with the shapes of the paper's workload: 16-bit
1024x1024 inline interferograms, stacks of 32 consecutive frames, 500 frames/s
(abstract; experimental set-up; Table 1).

Physical model (interferogram formation, the I = |E|^2 + |E_LO|^2 + H + H*
decomposition of the set-up section):

* the object field O_0 is circular-Gaussian speckle inside a disk of radius R;
* the left half of that disk is "static tissue" that carries one random global
  phase per frame (uniform in [0, 2 pi));
* a smaller "flow" disk of radius R_f carries a per-pixel phase random walk
  with N(0, 0.8 rad) increments per frame;
* the sensor field S_t is the object field back-propagated to the sensor
  plane, normalised to unit mean power, and mixed inline with a unit plane
  reference: I_t = |1 + 0.05 S_t|^2 + read noise (sigma 0.002);
* I_t is scaled to the 12-bit range (x 2048), rounded and clipped to
  [0, 4095], and stored as uint16.

This module only *makes inputs*.  It is shared by the tests, the benchmark
and the camera simulators; it holds none of the arithmetic of the
hologram-rendering method itself.  The back-propagation it needs is written
here, on its own, as the exact inverse of a chirp-times-FFT operator.

Random draw order (numpy.random.default_rng(seed), PCG64) is fixed:
two standard-normal planes for O_0; then per frame one uniform for the global
phase, one normal plane for the phase increments and one standard-normal
plane for the read noise.
"""
from __future__ import annotations

import hashlib
import os
from dataclasses import dataclass

import numpy as np

try:  # multi-threaded pocketfft; the transform is computed identically per line
    import scipy.fft as _fft

    _WORKERS = max(1, min(16, os.cpu_count() or 1))

    def _ifft2(x):
        return _fft.ifft2(x, workers=_WORKERS)
except Exception:  # pragma: no cover - scipy is part of the image
    def _ifft2(x):
        return np.fft.ifft2(x)


@dataclass(frozen=True)
class Physics:
    """Optical parameters (metres).  Defaults: 785 nm laser, 20 um pitch, 0.3 m."""

    wavelength: float = 785e-9
    pitch: float = 20e-6
    distance: float = 0.3


def radii(ny: int, nx: int) -> tuple[float, float]:
    """Speckle-disk and flow-disk radii (pixels) for a frame size."""
    if (ny, nx) == (128, 128):
        return 40.0, 12.0
    if (ny, nx) == (1024, 1024):
        return 400.0, 80.0
    m = float(min(ny, nx))
    return 0.39 * m, 0.078 * m


def _back_propagator(ny: int, nx: int, phys: Physics) -> np.ndarray:
    """Unit-modulus factor that undoes the sensor-plane quadratic phase.

    Sensor coordinates are taken about the sensor centre; the integer squared
    offsets are formed exactly before scaling by pi d^2 / (lambda z).
    """
    a = np.pi * phys.pitch ** 2 / (phys.wavelength * phys.distance)
    my = (np.arange(ny, dtype=np.int64) - ny // 2) ** 2
    mx = (np.arange(nx, dtype=np.int64) - nx // 2) ** 2
    q = my[:, None] + mx[None, :]
    return np.exp(1j * a * q.astype(np.float64))


class StackSource:
    """Stateful generator of consecutive frames for one simulated camera."""

    def __init__(self, seed: int, ny: int, nx: int, phys: Physics = Physics()):
        self.ny, self.nx, self.phys = int(ny), int(nx), phys
        self.rng = np.random.default_rng(seed)
        R, Rf = radii(ny, nx)
        yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
        cy, cx = ny / 2.0, nx / 2.0
        disk = (yy - cy) ** 2 + (xx - cx) ** 2 <= R * R
        self.static_half = disk & (xx < cx)
        self.flow = disk & ((yy - cy) ** 2 + (xx - (cx + R / 2.0)) ** 2 <= Rf * Rf)
        g1 = self.rng.standard_normal((ny, nx))
        g2 = self.rng.standard_normal((ny, nx))
        self.obj0 = np.where(disk, (g1 + 1j * g2) / np.sqrt(2.0), 0.0)
        self.flow_phase = np.zeros((ny, nx))
        self.bp = _back_propagator(ny, nx, phys)
        self.frames_made = 0

    def next_frame(self) -> np.ndarray:
        theta = self.rng.uniform(0.0, 2.0 * np.pi)
        self.flow_phase = self.flow_phase + self.rng.normal(0.0, 0.8, (self.ny, self.nx))
        obj = self.obj0.copy()
        obj[self.static_half] *= np.exp(1j * theta)
        obj[self.flow] *= np.exp(1j * self.flow_phase[self.flow])
        field = self.bp * _ifft2(obj)
        field /= np.sqrt(np.mean(np.abs(field) ** 2))
        inten = np.abs(1.0 + 0.05 * field) ** 2
        inten += 0.002 * self.rng.standard_normal((self.ny, self.nx))
        self.frames_made += 1
        return np.clip(np.rint(2048.0 * inten), 0, 4095).astype(np.uint16)

    def frames(self, n: int) -> np.ndarray:
        out = np.empty((n, self.ny, self.nx), dtype=np.uint16)
        for t in range(n):
            out[t] = self.next_frame()
        return out


def gen_stack(seed: int, nt: int, ny: int, nx: int, phys: Physics = Physics()) -> np.ndarray:
    """One stack of ``nt`` consecutive uint16 frames, shape (nt, ny, nx)."""
    return StackSource(seed, ny, nx, phys).frames(nt)


def sha256(a: np.ndarray) -> str:
    """Digest of an array's bytes (C order), with its shape and dtype."""
    h = hashlib.sha256()
    h.update(f"{a.dtype.str}{a.shape}".encode())
    h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


# Workload catalogue: the stack shapes of the benchmark configurations.
SMALL = dict(nt=32, ny=128, nx=128)          # one 32 x 128 x 128 stack
PAPER = dict(nt=32, ny=1024, nx=1024)        # one 32 x 1024 x 1024 stack
BATCH_SHAPES = [(512, 512), (1024, 1024), (1024, 2048)]   # (ny, nx)
BATCH_NTS = [16, 32, 64]


def batch_spec(i: int) -> tuple[int, int, int]:
    """(nt, ny, nx) of stack i of the uneven 8-stack batch."""
    ny, nx = BATCH_SHAPES[i % 3]
    nt = BATCH_NTS[(i + i // 3) % 3]
    return nt, ny, nx
