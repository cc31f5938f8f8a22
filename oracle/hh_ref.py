"""FP64 CPU oracle for the PCA holography hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product imports this module: only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark call
it.  It shares no code with the GPU path (no kernels, tables, constants or
helpers); the two meet only on the seeded uint16 inputs.

Plain, slow and obviously correct: numpy in float64 / complex128, with a
library FFT, matrix product and LAPACK Hermitian eigensolver as the only
primitives.  Every function follows one equation of Puyo et al., "Real-time
digital holography of the retina by principal component analysis"
(arXiv:2004.00923); the readings taken where the paper is silent or loose are
listed with each function.

Notation: a stack has n_t frames of n_y x n_x pixels, frame-major
(n_t, n_y, n_x).  The space-time matrix H of the paper is its
(n_x n_y, n_t) reshape: column t is frame t flattened row-major
(pixel p = y * n_x + x).
"""
from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------------------
# Step (a): Fresnel propagation, Eq. (1)
# ----------------------------------------------------------------------------

def chirp(nx: int, ny: int, wavelength: float, distance: float, pitch: float) -> np.ndarray:
    """Sensor-plane quadratic phase of the Fresnel kernel, Eq. (1).

    Expanding (x - x')^2 in Eq. (1) splits the kernel into an input-plane
    chirp exp(-i pi (x'^2 + y'^2) / (lambda z)), a Fourier kernel, and an
    output-plane chirp.  The input chirp is sampled at
    x' = (m - n_x/2) d, y' = (n - n_y/2) d (origin at the sensor centre):

        c[n, m] = exp(-i alpha ((m - n_x/2)^2 + (n - n_y/2)^2)),
        alpha   = pi d^2 / (lambda z).

    The squared offsets are exact integers; only the product with alpha is
    rounded (float64).
    """
    alpha = np.pi * pitch * pitch / (wavelength * distance)
    m2 = (np.arange(nx, dtype=np.int64) - nx // 2) ** 2
    n2 = (np.arange(ny, dtype=np.int64) - ny // 2) ** 2
    q = n2[:, None] + m2[None, :]
    return np.exp(-1j * (alpha * q.astype(np.float64)))


def fresnel_ref(frames: np.ndarray, wavelength: float, distance: float, pitch: float) -> np.ndarray:
    """Fresnel holograms of a frame stack, Eq. (1): chirp multiply then 2D FFT.

    ``frames``: (n, n_y, n_x), any real or complex dtype (uint16 in the hot
    path).  Returns complex128 (n, n_y, n_x):

        H_t[v, u] = sum_{n, m} I_t[n, m] c[n, m] exp(-2 pi i (u m / n_x + v n / n_y)).

    Readings of Eq. (1): the constant prefactor (i / lambda z) exp(-ikz) d^2 and
    the output-plane chirp are dropped (unit-modulus per-pixel factors and a
    global scale: they change neither the covariance eigenvectors nor the
    image beyond a global factor); the forward (negative-exponent) DFT is used,
    which mirrors Eq. (1)'s image through the origin; no fftshift, no padding.
    """
    x = np.asarray(frames)
    nt, ny, nx = x.shape
    c = chirp(nx, ny, wavelength, distance, pitch)
    return np.fft.fft2(x.astype(np.complex128) * c[None, :, :], axes=(-2, -1))


# ----------------------------------------------------------------------------
# Step (b): time-lagged covariance, Eq. (4)
# ----------------------------------------------------------------------------

def space_time_matrix(holo: np.ndarray) -> np.ndarray:
    """The (n_x n_y, n_t) matrix H whose column t is hologram t (reshape step
    before Eq. (2))."""
    nt = holo.shape[0]
    return holo.reshape(nt, -1).T


def covariance_ref(holo: np.ndarray) -> np.ndarray:
    """C = H^{t*} H, Eq. (4): (n_t, n_t) complex128, C[s, t] = sum_p conj(H[p, s]) H[p, t].

    Exactly the conjugate-transpose product: no mean removal, no 1/N.
    The paper calls C "complex-valued and symmetric"; as a product H^{t*} H it
    is Hermitian positive semi-definite, which is how it is treated here.
    """
    Hm = space_time_matrix(np.asarray(holo, dtype=np.complex128))
    return Hm.conj().T @ Hm


# ----------------------------------------------------------------------------
# Step (c): eigendecomposition, Eq. (5)
# ----------------------------------------------------------------------------

PHASE_TIE_REL = 1e-12


def phase_fix(V: np.ndarray) -> np.ndarray:
    """Fix the free unit phase of each eigenvector (Eq. (5) leaves it open).

    Column k is multiplied by exp(-i arg v_k[j*]), j* the row of largest
    modulus; rows whose modulus is within a relative 1e-12 of the largest
    count as tied and the lowest such row is taken.  The entry at j* is then
    real and positive.
    """
    V = np.array(V, dtype=np.complex128, copy=True)
    for k in range(V.shape[1]):
        mag = np.abs(V[:, k])
        jstar = int(np.nonzero(mag >= mag.max() * (1.0 - PHASE_TIE_REL))[0][0])
        ph = V[jstar, k] / mag[jstar]
        V[:, k] = V[:, k] * np.conj(ph)
        V[jstar, k] = complex(abs(V[jstar, k]), 0.0)
    return V


def eigh_ref(C: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """C = V Lambda V^{t*}, Eq. (5), with a LAPACK Hermitian solver (zheevd).

    Returns (lam, V): lam float64 (n_t,) in DESCENDING order, V complex128
    (n_t, n_t) unitary with column k the eigenvector of lam[k], phase-fixed.
    (The paper sorts ascending and counts its selector 1-based; the kept range
    of the projection is expressed 0-based on this descending order.)
    """
    w, V = np.linalg.eigh(np.asarray(C, dtype=np.complex128))
    return w[::-1].copy(), phase_fix(V[:, ::-1])


# ----------------------------------------------------------------------------
# Steps (d)+(e): projection and power image, Eqs. (6)-(7)
# ----------------------------------------------------------------------------

def project_render_ref(holo: np.ndarray, V: np.ndarray, k_lo: int, k_hi: int) -> np.ndarray:
    """Power-Doppler image of Eq. (7) from the principal components of Eq. (6).

    H_breve = H V I_f with I_f keeping columns k_lo..k_hi (0-based, inclusive,
    in descending-eigenvalue order); M[y, x] = sum_k |H_breve[p, k]|^2.
    Literal H V (not H conj(V)).  Returns float64 (n_y, n_x).
    """
    nt, ny, nx = holo.shape
    Hm = space_time_matrix(np.asarray(holo, dtype=np.complex128))
    Hb = Hm @ np.asarray(V, dtype=np.complex128)[:, k_lo:k_hi + 1]
    return np.sum(Hb.real ** 2 + Hb.imag ** 2, axis=1).reshape(ny, nx)


def pipeline_ref(frames: np.ndarray, wavelength: float, distance: float, pitch: float,
                 k_lo: int, k_hi: int) -> dict:
    """Steps (a)-(e) in the paper's order; returns every intermediate."""
    H = fresnel_ref(frames, wavelength, distance, pitch)
    C = covariance_ref(H)
    lam, V = eigh_ref(C)
    M = project_render_ref(H, V, k_lo, k_hi)
    return dict(holo=H, cov=C, evals=lam, evecs=V, image=M)


# ----------------------------------------------------------------------------
# Fourier demodulation, Eqs. (8)-(9) (the paper's comparison method)
# ----------------------------------------------------------------------------

def dft_basis(nt: int) -> np.ndarray:
    """W of Eq. (8): w_mn = exp(-2 i pi (m-1)(n-1) / n_t) / sqrt(n_t), written 0-based."""
    m = np.arange(nt)
    return np.exp(-2j * np.pi * np.outer(m, m) / nt) / np.sqrt(nt)


def fourier_render_ref(holo: np.ndarray, f_lo: int, f_hi: int) -> np.ndarray:
    """M_0 of Eq. (9): sum over kept temporal frequencies f_lo..f_hi (0-based,
    inclusive) of |H W|^2.  The paper's 1-based n_1..n_2 maps to n_1-1..n_2-1."""
    nt, ny, nx = holo.shape
    Hm = space_time_matrix(np.asarray(holo, dtype=np.complex128))
    Ht = Hm @ dft_basis(nt)[:, f_lo:f_hi + 1]
    return np.sum(Ht.real ** 2 + Ht.imag ** 2, axis=1).reshape(ny, nx)


# ----------------------------------------------------------------------------
# SVD filtering, Eq. (3), through the covariance eigenbasis
# ----------------------------------------------------------------------------

def svd_filter_ref(holo: np.ndarray, V: np.ndarray, k_lo: int, k_hi: int) -> np.ndarray:
    """H_f = U Delta I_f V^{t*} of Eq. (3).

    With H = U Delta V^{t*} (Eq. (2)) and the same V as Eq. (5),
    U Delta I_f V^{t*} = H V I_f V^{t*}.  Returns the filtered stack
    (n_t, n_y, n_x) complex128.
    """
    nt, ny, nx = holo.shape
    Hm = space_time_matrix(np.asarray(holo, dtype=np.complex128))
    Vk = np.asarray(V, dtype=np.complex128)[:, k_lo:k_hi + 1]
    Hf = (Hm @ Vk) @ Vk.conj().T
    return Hf.T.reshape(nt, ny, nx)


# ----------------------------------------------------------------------------
# Projection first: the covariance from the frames and the image from combined
# frames (a reformulation of steps (b), (d) and (e) that never forms H)
# ----------------------------------------------------------------------------

def covariance_frames_ref(frames: np.ndarray) -> np.ndarray:
    """C of Eq. (4) evaluated from the interferograms: C = N_pix I^T I.

    With the unit-modulus input chirp c and the unnormalised DFT F (F^H F =
    N_pix Id), H_t = F(c I_t) gives conj(H_s)^T H_t = N_pix sum_p I_s[p] I_t[p].
    The integer Gram is formed exactly in int64 (products below 2^32, sums below
    2^63 for the supported sizes), then scaled; returns complex128 (n_t, n_t)
    with zero imaginary part.
    """
    x = np.asarray(frames)
    nt, ny, nx = x.shape
    Im = x.reshape(nt, ny * nx).astype(np.int64)
    G = Im @ Im.T
    return (G.astype(np.float64) * float(ny * nx)).astype(np.complex128)


def project_first_ref(frames: np.ndarray, V: np.ndarray, wavelength: float, distance: float, pitch: float,
                      k_lo: int, k_hi: int) -> np.ndarray:
    """Image of Eq. (7) with the projection taken before the propagation.

    Eq. (1) is linear in the frame, so column k of H V (Eq. (6)) is the Fresnel
    hologram of the combined frame J_k = sum_t V[t, k] I_t:
        M[y, x] = sum_{k = k_lo..k_hi} |Fresnel(J_k)[y, x]|^2.
    Returns float64 (n_y, n_x).
    """
    x = np.asarray(frames)
    nt, ny, nx = x.shape
    Vk = np.asarray(V, dtype=np.complex128)[:, k_lo:k_hi + 1]
    J = (Vk.T @ x.reshape(nt, ny * nx).astype(np.complex128)).reshape(-1, ny, nx)
    Y = fresnel_ref(J, wavelength, distance, pitch)
    return np.sum(Y.real ** 2 + Y.imag ** 2, axis=0)


def pipeline_first_ref(frames: np.ndarray, wavelength: float, distance: float, pitch: float,
                       k_lo: int, k_hi: int) -> dict:
    """The projection-first path: C from the frames, Eq. (5), image from combined frames."""
    C = covariance_frames_ref(frames)
    lam, V = eigh_ref(C)
    M = project_first_ref(frames, V, wavelength, distance, pitch, k_lo, k_hi)
    return dict(cov=C, evals=lam, evecs=V, image=M)
