"""Pins that tie the FP64 oracle to facts fixed by the paper and by mathematics.

Each ``pin_*`` function takes an oracle-like namespace ``o`` (the real
``oracle`` package, or a planted mutant of it) and returns the list of
failed checks (empty = pinned).  None of them re-types the oracle's formula:
they use brute force on tiny inputs, closed forms, exact integer identities,
a different LAPACK routine, and invariances.
"""
from __future__ import annotations

import cmath
import math

import numpy as np

LAM = 785e-9
PITCH = 20e-6
Z = 0.3


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))


def _check(fails, name, ok, detail=""):
    if not ok:
        fails.append(f"{name}: {detail}")


def _rand_frames(rng, nt, ny, nx):
    return rng.integers(0, 4096, size=(nt, ny, nx)).astype(np.uint16)


# ---------------------------------------------------------------------------
# Fresnel, Eq. (1)
# ---------------------------------------------------------------------------

def _brute_fresnel(frame, lam, z, d):
    """Direct double sum of the discretised Eq. (1) kernel (input chirp times
    negative-exponent Fourier kernel), pure Python, O(N^4)."""
    ny, nx = frame.shape
    a = math.pi * d * d / (lam * z)
    out = np.zeros((ny, nx), dtype=np.complex128)
    for v in range(ny):
        for u in range(nx):
            acc = 0j
            for n in range(ny):
                for m in range(nx):
                    ph = -a * ((m - nx // 2) ** 2 + (n - ny // 2) ** 2) \
                         - 2.0 * math.pi * (u * m / nx + v * n / ny)
                    acc += float(frame[n, m]) * cmath.exp(1j * ph)
            out[v, u] = acc
    return out


def _literal_eq1_mag(frame, lam, z, d):
    """|Riemann sum of Eq. (1)| on the output grid x_u = u lambda z / (n_x d),
    with the full (x - x')^2 kernel and the (i / lambda z) exp(-ikz) d^2
    prefactor.  Pure Python."""
    ny, nx = frame.shape
    out = np.zeros((ny, nx))
    for v in range(ny):
        for u in range(nx):
            xu = u * lam * z / (nx * d)
            yv = v * lam * z / (ny * d)
            acc = 0j
            for n in range(ny):
                for m in range(nx):
                    xp = (m - nx // 2) * d
                    yp = (n - ny // 2) * d
                    acc += float(frame[n, m]) * cmath.exp(
                        -1j * math.pi / (lam * z) * ((xu - xp) ** 2 + (yv - yp) ** 2)) * d * d
            k = 2 * math.pi / lam
            out[v, u] = abs(1j / (lam * z) * cmath.exp(-1j * k * z) * acc)
    return out


def pin_fresnel(o):
    fails = []
    rng = np.random.default_rng(11)
    # 1. brute-force DFT of the discretised Eq. (1), square and rectangular
    for ny, nx in [(8, 8), (8, 16), (16, 8)]:
        f = _rand_frames(rng, 1, ny, nx)
        H = o.fresnel_ref(f, LAM, Z, PITCH)[0]
        B = _brute_fresnel(f[0], LAM, Z, PITCH)
        e = _rel(H, B)
        _check(fails, f"brute-force DFT {ny}x{nx}", e <= 1e-12, f"rel err {e:.2e}")
    # 2. literal Eq. (1) magnitude equals the oracle mirrored through the origin
    for ny, nx in [(8, 8), (8, 16)]:
        f = _rand_frames(rng, 1, ny, nx)
        H = o.fresnel_ref(f, LAM, Z, PITCH)[0]
        L = _literal_eq1_mag(f[0], LAM, Z, PITCH) * (LAM * Z) / (PITCH * PITCH)
        mir = np.abs(H)[(-np.arange(ny)) % ny][:, (-np.arange(nx)) % nx]
        e = _rel(mir, L)
        _check(fails, f"literal Eq.1 magnitude {ny}x{nx}", e <= 1e-10, f"rel err {e:.2e}")
    # 3. point source at the matched distance lambda z = n d^2 -> Kronecker delta
    for n, (m0, n0) in [(16, (3, -5)), (8, (0, 2)), (32, (7, 7))]:
        zm = n * PITCH * PITCH / LAM
        mm = np.arange(n)[None, :]
        nn = np.arange(n)[:, None]
        src = np.exp(1j * np.pi * ((mm - n // 2 - m0) ** 2 + (nn - n // 2 - n0) ** 2) / n)
        H = o.fresnel_ref(src[None], LAM, zm, PITCH)[0]
        E = np.zeros((n, n), dtype=np.complex128)
        E[(-n0) % n, (-m0) % n] = n * n * np.exp(1j * np.pi * (m0 * m0 + n0 * n0) / n) * (-1) ** (m0 + n0)
        err = np.abs(H - E).max() / (n * n)
        _check(fails, f"point source n={n}", err <= 1e-12, f"max err {err:.2e}")
    # 4. constant frame at the matched distance: |Fresnel(1)| = n everywhere
    for n in (8, 16, 32):
        zm = n * PITCH * PITCH / LAM
        H = o.fresnel_ref(np.ones((1, n, n)), LAM, zm, PITCH)[0]
        err = np.abs(np.abs(H) - n).max() / n
        _check(fails, f"constant n={n}", err <= 1e-12, f"max err {err:.2e}")
    # 5. Parseval per frame: ||H_t||^2 = N_pix ||I_t||^2 (integer right side)
    f = _rand_frames(rng, 3, 16, 32)
    H = o.fresnel_ref(f, LAM, Z, PITCH)
    lhs = np.sum(np.abs(H) ** 2, axis=(1, 2))
    rhs = np.array([16 * 32 * int(np.sum(f[t].astype(np.int64) ** 2)) for t in range(3)], dtype=np.float64)
    e = _rel(lhs, rhs)
    _check(fails, "Parseval", e <= 1e-13, f"rel err {e:.2e}")
    return fails


# ---------------------------------------------------------------------------
# Covariance, Eq. (4)
# ---------------------------------------------------------------------------

def pin_covariance(o, frames=None):
    fails = []
    rng = np.random.default_rng(12)
    if frames is None:
        frames = _rand_frames(rng, 6, 32, 32)
    nt, ny, nx = frames.shape
    H = o.fresnel_ref(frames, LAM, Z, PITCH)
    C = o.covariance_ref(H)
    # 1. Gram identity C = N_pix I^T I, exact in int64
    I = frames.reshape(nt, -1).astype(np.int64)
    G = (I @ I.T) * (nx * ny)
    e = _rel(C, G.astype(np.float64))
    _check(fails, "Gram identity C = N I^T I", e <= 1e-13, f"rel err {e:.2e}")
    # 2. Hermitian, PSD, trace = total stack energy (integer)
    _check(fails, "Hermitian", np.abs(C - C.conj().T).max() <= 1e-14 * np.abs(C).max(), "")
    w = np.linalg.eigvalsh(C)
    _check(fails, "PSD", w.min() >= -1e-12 * w.max(), f"min eig {w.min():.3e}")
    tr = float(np.trace(C).real)
    energy = float(nx * ny * int(np.sum(I * I)))
    _check(fails, "trace = stack energy", abs(tr - energy) <= 1e-13 * energy, f"{tr} vs {energy}")
    # 3. conjugation convention on a constructed complex stack: H = Q S W^H  =>  C = W S^2 W^H
    npix, k = 64, 5
    Q, _ = np.linalg.qr(rng.standard_normal((npix, k)) + 1j * rng.standard_normal((npix, k)))
    W, _ = np.linalg.qr(rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k)))
    s = np.array([5.0, 3.0, 2.0, 1.0, 0.5])
    Hm = (Q * s) @ W.conj().T                     # (npix, k): column t = hologram t
    stack = Hm.T.reshape(k, 8, 8)
    Cc = o.covariance_ref(stack)
    Ec = (W * s ** 2) @ W.conj().T
    e = _rel(Cc, Ec)
    _check(fails, "C = H^{t*} H on a constructed complex stack", e <= 1e-13, f"rel err {e:.2e}")
    return fails


# ---------------------------------------------------------------------------
# Eigendecomposition, Eq. (5)
# ---------------------------------------------------------------------------

def pin_eigh(o, frames=None):
    fails = []
    rng = np.random.default_rng(13)
    # 1. 2x2 Hermitian closed form
    a, b, beta = 3.0, 1.0, 0.5 - 0.75j
    lam, V = o.eigh_ref(np.array([[a, beta], [np.conj(beta), b]]))
    r = math.sqrt(((a - b) / 2) ** 2 + abs(beta) ** 2)
    _check(fails, "2x2 eigenvalues", np.allclose(lam, [(a + b) / 2 + r, (a + b) / 2 - r], rtol=0, atol=1e-14), str(lam))
    v = np.array([beta, (a + b) / 2 + r - a])
    v = v / np.linalg.norm(v)
    ov = abs(np.vdot(v, V[:, 0]))
    _check(fails, "2x2 leading eigenvector", abs(ov - 1) <= 1e-14, f"overlap {ov}")
    # 2. diagonal input: descending eigenvalues, permutation eigenvectors with +1 entries
    d = np.array([2.0, 7.0, -1.0, 4.0])
    lam, V = o.eigh_ref(np.diag(d).astype(np.complex128))
    _check(fails, "diagonal: descending", np.array_equal(lam, np.sort(d)[::-1]), str(lam))
    P = np.zeros((4, 4))
    for k, i in enumerate(np.argsort(-d)):
        P[i, k] = 1.0
    _check(fails, "diagonal: phase-fixed permutation", np.abs(V - P).max() <= 1e-15, "")
    # 3. residual / orthonormality / trace on a hologram covariance
    if frames is None:
        frames = _rand_frames(rng, 8, 16, 16)
    nt, ny, nx = frames.shape
    H = o.fresnel_ref(frames, LAM, Z, PITCH)
    C = o.covariance_ref(H)
    lam, V = o.eigh_ref(C)
    nC = np.linalg.norm(C)
    _check(fails, "residual", np.linalg.norm(C @ V - V * lam) <= 1e-12 * nC, "")
    _check(fails, "orthonormal", np.abs(V.conj().T @ V - np.eye(nt)).max() <= 1e-13, "")
    _check(fails, "descending", bool(np.all(np.diff(lam) <= 0)), "")
    _check(fails, "sum lambda = trace", abs(lam.sum() - np.trace(C).real) <= 1e-13 * abs(lam.sum()), "")
    # 4. Lambda = Delta^2 with a different LAPACK routine (SVD of H)
    sv = np.linalg.svd(o.space_time_matrix(H), compute_uv=False)
    e = np.abs(np.sort(sv ** 2)[::-1] - lam).max() / lam[0]
    _check(fails, "Lambda = Delta^2", e <= 1e-12, f"{e:.2e}")
    # 5. eigenvalues of the exact integer Gram N I^T I (real symmetric solver)
    I = frames.reshape(nt, -1).astype(np.int64)
    wg = np.linalg.eigvalsh((I @ I.T).astype(np.float64))[::-1] * (nx * ny)
    e = np.abs(wg - lam).max() / lam[0]
    _check(fails, "eigenvalues of N I^T I", e <= 1e-13, f"{e:.2e}")
    # 6. phase fix: the lowest row of largest modulus is real positive
    for k in range(nt):
        mag = np.abs(V[:, k])
        j = int(np.nonzero(mag >= mag.max() * (1 - 1e-12))[0][0])
        _check(fails, f"phase fix col {k}", V[j, k].imag == 0.0 and V[j, k].real > 0, str(V[j, k]))
    # 7. tie rule: equal moduli -> the lowest row is the real one
    U = np.array([[1j, 1.0], [-1.0, 1j]]) / math.sqrt(2)
    Vt = o.phase_fix(U)
    _check(fails, "tie rule", Vt[0, 0].imag == 0 and Vt[0, 0].real > 0 and Vt[0, 1].imag == 0, str(Vt))
    return fails


# ---------------------------------------------------------------------------
# Projection + render, Eqs. (6)-(7); Fourier, Eqs. (8)-(9); filter, Eq. (3)
# ---------------------------------------------------------------------------

def pin_project(o, frames=None, k_lo=2, k_hi=None):
    fails = []
    rng = np.random.default_rng(14)
    if frames is None:
        frames = _rand_frames(rng, 8, 16, 16)
    nt, ny, nx = frames.shape
    k_hi = nt - 1 if k_hi is None else k_hi
    H = o.fresnel_ref(frames, LAM, Z, PITCH)
    C = o.covariance_ref(H)
    lam, V = o.eigh_ref(C)
    M = o.project_render_ref(H, V, k_lo, k_hi)
    # 1. all components: Parseval with V unitary
    Mall = o.project_render_ref(H, V, 0, nt - 1)
    e = _rel(Mall, np.sum(np.abs(H) ** 2, axis=0))
    _check(fails, "all components = sum_t |H_t|^2", e <= 1e-12, f"{e:.2e}")
    # 2. image total = kept eigenvalue sum
    e = abs(M.sum() - lam[k_lo:k_hi + 1].sum()) / lam[k_lo:k_hi + 1].sum()
    _check(fails, "sum M = sum kept lambda", e <= 1e-9, f"{e:.2e}")
    # 3. additivity over a split of the kept range
    c = (k_lo + k_hi) // 2
    e = _rel(o.project_render_ref(H, V, k_lo, c) + o.project_render_ref(H, V, c + 1, k_hi), M)
    _check(fails, "additivity", e <= 1e-12, f"{e:.2e}")
    # 4. invariance to the free phases of the eigenvectors
    ph = np.exp(2j * np.pi * rng.random(nt))
    e = _rel(o.project_render_ref(H, V * ph[None, :], k_lo, k_hi), M)
    _check(fails, "eigenvector phase invariance", e <= 1e-12, f"{e:.2e}")
    # 5. cross-route by linearity: M = sum_k |Fresnel(sum_t I_t V[t,k])|^2
    comb = np.tensordot(V[:, k_lo:k_hi + 1].T, frames.astype(np.complex128), axes=(1, 0))
    Mx = np.sum(np.abs(o.fresnel_ref(comb, LAM, Z, PITCH)) ** 2, axis=0)
    e = _rel(Mx, M)
    _check(fails, "projection-first cross-route", e <= 1e-9, f"{e:.2e}")
    # 6. permuting frames in time leaves the image unchanged
    perm = rng.permutation(nt)
    Hp = o.fresnel_ref(frames[perm], LAM, Z, PITCH)
    lp, Vp = o.eigh_ref(o.covariance_ref(Hp))
    e = _rel(o.project_render_ref(Hp, Vp, k_lo, k_hi), M)
    _check(fails, "time-permutation invariance", e <= 1e-8, f"{e:.2e}")
    # 7. reconstruction from all components and filtered-stack power
    Hf = o.svd_filter_ref(H, V, 0, nt - 1)
    e = _rel(Hf, H)
    _check(fails, "reconstruction (H V) V^H = H", e <= 1e-12, f"{e:.2e}")
    Hf = o.svd_filter_ref(H, V, k_lo, k_hi)
    e = _rel(np.sum(np.abs(Hf) ** 2, axis=0), M)
    _check(fails, "filtered-stack power = image", e <= 1e-10, f"{e:.2e}")
    # Eq. (3) literally: U Delta I_f W^H from the library SVD of the space-time matrix
    # (Eq. (2)); singular values come in descending order, as the kept range counts
    Uh, dh, Whh = np.linalg.svd(o.space_time_matrix(H), full_matrices=False)
    Hs = ((Uh[:, k_lo:k_hi + 1] * dh[k_lo:k_hi + 1]) @ Whh[k_lo:k_hi + 1, :]).T.reshape(H.shape)
    e = _rel(Hf, Hs)
    _check(fails, "filtered stack = U Delta I_f V^H (SVD route)", e <= 1e-9, f"{e:.2e}")
    # 8. pure-Python brute force of Eqs. (6)-(7) on a tiny stack
    Ht = H[:3, :2, :2]
    Vt = V[:3, :3]
    Vt, _ = np.linalg.qr(Vt)
    Mb = np.zeros((2, 2))
    for y in range(2):
        for x in range(2):
            for k in range(1, 3):
                s = 0j
                for t in range(3):
                    s += complex(Ht[t, y, x]) * complex(Vt[t, k])
                Mb[y, x] += abs(s) ** 2
    e = _rel(o.project_render_ref(Ht, Vt, 1, 2), Mb)
    _check(fails, "brute-force Eqs. 6-7", e <= 1e-13, f"{e:.2e}")
    # 9. constructed complex stack H = Q S W^H (W complex unitary, S descending):
    #    the principal components are H W = Q S, so M[p] = sum_kept s_k^2 |Q[p, k]|^2
    npix, k = 64, 6
    Q, _ = np.linalg.qr(rng.standard_normal((npix, k)) + 1j * rng.standard_normal((npix, k)))
    W, _ = np.linalg.qr(rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k)))
    s = np.array([6.0, 4.0, 3.0, 2.0, 1.5, 1.0])
    stack = ((Q * s) @ W.conj().T).T.reshape(k, 8, 8)
    lam_c, V_c = o.eigh_ref(o.covariance_ref(stack))
    Mc = o.project_render_ref(stack, V_c, 1, 4)
    Ec = np.sum((s[1:5] ** 2)[None, :] * np.abs(Q[:, 1:5]) ** 2, axis=1).reshape(8, 8)
    e = _rel(Mc, Ec)
    _check(fails, "closed-form components of a complex stack", e <= 1e-12, f"{e:.2e}")
    return fails


def pin_fourier(o):
    fails = []
    rng = np.random.default_rng(15)
    frames = _rand_frames(rng, 8, 8, 16)
    H = o.fresnel_ref(frames, LAM, Z, PITCH)
    W = o.dft_basis(8)
    _check(fails, "W unitary", np.abs(W @ W.conj().T - np.eye(8)).max() <= 1e-14, "")
    e = _rel(o.fourier_render_ref(H, 0, 7), np.sum(np.abs(H) ** 2, axis=0))
    _check(fails, "Fourier all bands = sum |H|^2", e <= 1e-13, f"{e:.2e}")
    F = np.fft.fft(H, axis=0) / math.sqrt(8)
    e = _rel(o.fourier_render_ref(H, 2, 5), np.sum(np.abs(F[2:6]) ** 2, axis=0))
    _check(fails, "Fourier band = temporal FFT band", e <= 1e-13, f"{e:.2e}")
    return fails


def pin_first(o):
    """The projection-first reformulation against the paper's order of steps."""
    fails = []
    rng = np.random.default_rng(16)
    frames = _rand_frames(rng, 6, 8, 16)
    nt, ny, nx = frames.shape
    H = o.fresnel_ref(frames, LAM, Z, PITCH)
    # 1. covariance from the frames = Eq. (4) on the holograms (Parseval, unit chirp)
    Cf = o.covariance_frames_ref(frames)
    e = _rel(Cf, o.covariance_ref(H))
    _check(fails, "frame covariance = H^H H", e <= 1e-12, f"{e:.2e}")
    # 2. integer brute force of one entry
    s = sum(int(a) * int(b) for a, b in zip(frames[1].ravel(), frames[4].ravel())) * ny * nx
    _check(fails, "frame covariance entry (1, 4) exact", Cf[1, 4] == s and Cf[4, 1] == s, f"{Cf[1, 4]} vs {s}")
    # 3. image from combined frames = Eq. (6)-(7) on the holograms, for the
    #    covariance's eigenvectors and for a random complex unitary V
    lam, V = o.eigh_ref(Cf)
    for name, W in (("eigenvectors", V),
                    ("random unitary", np.linalg.qr(rng.standard_normal((nt, nt))
                                                    + 1j * rng.standard_normal((nt, nt)))[0])):
        for a, b in ((2, nt - 1), (0, 0), (1, 3)):
            e = _rel(o.project_first_ref(frames, W, LAM, Z, PITCH, a, b), o.project_render_ref(H, W, a, b))
            _check(fails, f"projection first = Eq. (6)-(7) ({name}, {a}..{b})", e <= 1e-10, f"{e:.2e}")
    # 4. Parseval on the combined frames: sum_p M = N_pix sum_k ||J_k||^2
    Vk = V[:, 2:nt]
    J = Vk.T @ frames.reshape(nt, -1).astype(np.float64)
    M = o.project_first_ref(frames, V, LAM, Z, PITCH, 2, nt - 1)
    e = abs(M.sum() - ny * nx * np.sum(np.abs(J) ** 2)) / M.sum()
    _check(fails, "sum M = N_pix sum ||J_k||^2", e <= 1e-10, f"{e:.2e}")
    # 5. a real symmetric C has real phase-fixed eigenvectors (used by the GPU path)
    _check(fails, "real eigenvectors", np.abs(V.imag).max() <= 1e-12, f"{np.abs(V.imag).max():.2e}")
    # 6. the path end to end equals the paper's order of steps
    r1 = o.pipeline_first_ref(frames, LAM, Z, PITCH, 2, nt - 1)
    r0 = o.pipeline_ref(frames, LAM, Z, PITCH, 2, nt - 1)
    e = _rel(r1["image"], r0["image"])
    _check(fails, "projection-first pipeline = pipeline", e <= 1e-9, f"{e:.2e}")
    return fails


ALL_PINS = (pin_fresnel, pin_covariance, pin_eigh, pin_project, pin_fourier, pin_first)
