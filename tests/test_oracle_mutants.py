"""Planted mistakes in the oracle (on the CPU) must each fail some pin.

This checks that the pins are strong enough: a dropped term, a wrong sign
or index, or a transposed operand anywhere in the oracle is caught.
"""
import types

import numpy as np
import pytest

import oracle
from oracle_pins import ALL_PINS


def _mutant(**over):
    ns = types.SimpleNamespace(**{k: getattr(oracle, k) for k in dir(oracle) if not k.startswith("_")})
    for k, v in over.items():
        setattr(ns, k, v)
    return ns


def _fres(transform):
    def f(frames, lam, z, d):
        x = np.asarray(frames)
        nt, ny, nx = x.shape
        return transform(x.astype(np.complex128), ny, nx, lam, z, d)
    return f


def m_conj_chirp(x, ny, nx, lam, z, d):
    return np.fft.fft2(x * np.conj(oracle.chirp(nx, ny, lam, z, d)), axes=(-2, -1))


def m_inverse_dft(x, ny, nx, lam, z, d):
    return np.fft.ifft2(x * oracle.chirp(nx, ny, lam, z, d), axes=(-2, -1)) * (nx * ny)


def m_corner_origin(x, ny, nx, lam, z, d):
    a = np.pi * d * d / (lam * z)
    q = np.arange(ny)[:, None] ** 2 + np.arange(nx)[None, :] ** 2
    return np.fft.fft2(x * np.exp(-1j * a * q), axes=(-2, -1))


def m_no_chirp(x, ny, nx, lam, z, d):
    return np.fft.fft2(x, axes=(-2, -1))


def m_half_alpha(x, ny, nx, lam, z, d):
    return np.fft.fft2(x * oracle.chirp(nx, ny, lam, 2 * z, d), axes=(-2, -1))


def m_fftshift(x, ny, nx, lam, z, d):
    return np.fft.fftshift(np.fft.fft2(x * oracle.chirp(nx, ny, lam, z, d), axes=(-2, -1)), axes=(-2, -1))


def cov_conj(h):
    return np.conj(oracle.covariance_ref(h))


def cov_centered(h):
    Hm = oracle.space_time_matrix(np.asarray(h, dtype=np.complex128))
    Hm = Hm - Hm.mean(axis=0, keepdims=True)
    return Hm.conj().T @ Hm


def cov_normalised(h):
    return oracle.covariance_ref(h) / (h.shape[1] * h.shape[2])


def cov_transposed(h):
    Hm = oracle.space_time_matrix(np.asarray(h, dtype=np.complex128))
    return Hm.T @ Hm.conj()


def eigh_ascending(C):
    w, V = np.linalg.eigh(C)
    return w, oracle.phase_fix(V)


def eigh_vec_not_reversed(C):
    w, V = np.linalg.eigh(C)
    return w[::-1].copy(), oracle.phase_fix(V)


def phase_last_tie(V):
    V = np.array(V, dtype=np.complex128, copy=True)
    for k in range(V.shape[1]):
        mag = np.abs(V[:, k])
        j = int(np.nonzero(mag >= mag.max() * (1 - 1e-12))[0][-1])
        V[:, k] *= np.conj(V[j, k] / mag[j])
        V[j, k] = abs(V[j, k])
    return V


def eigh_lastie(C):
    w, V = np.linalg.eigh(C)
    return w[::-1].copy(), phase_last_tie(V[:, ::-1])


def proj_conjV(h, V, a, b):
    return oracle.project_render_ref(h, np.conj(V), a, b)


def proj_VT(h, V, a, b):
    return oracle.project_render_ref(h, np.asarray(V).T, a, b)


def proj_abs(h, V, a, b):
    Hm = oracle.space_time_matrix(np.asarray(h, dtype=np.complex128))
    return np.sum(np.abs(Hm @ V[:, a:b + 1]), axis=1).reshape(h.shape[1:])


def proj_exclusive(h, V, a, b):
    return oracle.project_render_ref(h, V, a, b - 1)


def w_plus(nt):
    m = np.arange(nt)
    return np.exp(2j * np.pi * np.outer(m, m) / nt) / np.sqrt(nt)


def w_nonorm(nt):
    m = np.arange(nt)
    return np.exp(-2j * np.pi * np.outer(m, m) / nt)


def fourier_with(W):
    def f(h, lo, hi):
        Hm = oracle.space_time_matrix(np.asarray(h, dtype=np.complex128))
        Ht = Hm @ W(h.shape[0])[:, lo:hi + 1]
        return np.sum(np.abs(Ht) ** 2, axis=1).reshape(h.shape[1:])
    return f


def first_conjV(f, V, lam, z, d, a, b):
    return _first_ok(f, np.conj(V), lam, z, d, a, b)


def first_VT(f, V, lam, z, d, a, b):
    return _first_ok(f, np.asarray(V).T, lam, z, d, a, b)


def first_no_chirp(f, V, lam, z, d, a, b):
    x = np.asarray(f)
    nt, ny, nx = x.shape
    J = (np.asarray(V)[:, a:b + 1].T @ x.reshape(nt, -1).astype(np.complex128)).reshape(-1, ny, nx)
    return np.sum(np.abs(np.fft.fft2(J, axes=(-2, -1))) ** 2, axis=0)


def first_exclusive(f, V, lam, z, d, a, b):
    return _first_ok(f, V, lam, z, d, a, b - 1) if b > a else np.zeros(np.asarray(f).shape[1:])


def _first_ok(*args):
    return oracle.project_first_ref(*args)


def covf_no_scale(f):
    return oracle.covariance_frames_ref(f) / (f.shape[1] * f.shape[2])


def covf_centred(f):
    x = np.asarray(f).reshape(f.shape[0], -1).astype(np.float64)
    x = x - x.mean(axis=0, keepdims=True)
    return ((x @ x.T) * (f.shape[1] * f.shape[2])).astype(np.complex128)


MUTANTS = {
    "projection first on conj(V)": dict(project_first_ref=first_conjV),
    "projection first on V^T": dict(project_first_ref=first_VT),
    "projection first without chirp": dict(project_first_ref=first_no_chirp),
    "projection first exclusive upper index": dict(project_first_ref=first_exclusive),
    "frame covariance without N_pix": dict(covariance_frames_ref=covf_no_scale),
    "centred frame covariance": dict(covariance_frames_ref=covf_centred),
    "conjugate chirp": dict(fresnel_ref=_fres(m_conj_chirp)),
    "inverse DFT": dict(fresnel_ref=_fres(m_inverse_dft)),
    "chirp origin at corner": dict(fresnel_ref=_fres(m_corner_origin)),
    "no chirp": dict(fresnel_ref=_fres(m_no_chirp)),
    "half chirp rate": dict(fresnel_ref=_fres(m_half_alpha)),
    "fftshift": dict(fresnel_ref=_fres(m_fftshift)),
    "conjugated covariance": dict(covariance_ref=cov_conj),
    "centred covariance": dict(covariance_ref=cov_centered),
    "normalised covariance": dict(covariance_ref=cov_normalised),
    "transposed covariance": dict(covariance_ref=cov_transposed),
    "ascending eigenvalues": dict(eigh_ref=eigh_ascending),
    "eigenvectors not reordered": dict(eigh_ref=eigh_vec_not_reversed),
    "phase tie takes last row": dict(eigh_ref=eigh_lastie, phase_fix=phase_last_tie),
    "projection on conj(V)": dict(project_render_ref=proj_conjV),
    "projection on V^T": dict(project_render_ref=proj_VT),
    "envelope |.| not |.|^2": dict(project_render_ref=proj_abs),
    "exclusive upper index": dict(project_render_ref=proj_exclusive),
    "DFT basis with + sign": dict(fourier_render_ref=fourier_with(w_plus), dft_basis=w_plus),
    "DFT basis without 1/sqrt(nt)": dict(fourier_render_ref=fourier_with(w_nonorm), dft_basis=w_nonorm),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    o = _mutant(**MUTANTS[name])
    fails = []
    for pin in ALL_PINS:
        try:
            fails += pin(o)
        except Exception as exc:          # a crash also counts as caught
            fails.append(f"{pin.__name__} raised {exc!r}")
        if fails:
            break
    assert fails, f"mutant '{name}' passed every pin"
