"""Helpers shared by the GPU parity tests (device transfer and error metrics)."""
import numpy as np

LAM, PITCH, Z = 785e-9, 20e-6, 0.3


def torch_dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch_dev())


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) or np.iscomplexobj(b) else np.float64)
    b = np.asarray(b, dtype=a.dtype)
    d = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (d if d > 0 else 1.0))


def say(msg):
    print(msg, flush=True)


def eig_parity(w, V, ref, k_lo, k_hi, c_tol, label=""):
    """Eigen-outputs of a pipeline (Eq. 5) against the oracle, with bounds from
    perturbation theory rather than fixed numbers.

    The GPU's eigenpairs reconstruct the covariance it actually solved,
    C_g = V diag(w) V^H (to the solver's ~1e-13 residual).  With E = C_g - C_ref:
      * C itself: ||E||_F / ||C_ref||_F <= c_tol (the covariance bar);
      (below, ||E||_2 includes n 1e-15 lam_0 for the backward error of the
      two FP64 eigensolvers);
      * every eigenvalue, by Weyl: |w_k - lam_k| <= ||E||_2;
      * the kept projector P = V_kept V_kept^H, by Davis-Kahan:
        ||P - P_ref||_2 <= ||E||_2 / (delta - ||E||_2), delta the gap between the
        kept eigenvalues and the rest (when the gap exceeds 2 ||E||_2);
      * each mode k whose gap to its neighbours exceeds 10 ||E||_2 and 1e-6 lam_0:
        sin(angle) <= ||E||_2 / (gap_k - ||E||_2), and the phase-fixed vectors
        (largest-modulus entry real and positive, taken at the same row when that
        row is unambiguous) differ by at most sin(angle) (1 + 2 / rho), rho the
        modulus of that entry.
    Returns the measured errors (printed by the caller)."""
    lam, Vr, Cr = ref["evals"], ref["evecs"], ref["cov"]
    n = len(lam)
    Cg = (V * w) @ V.conj().T
    # plus the backward error of the two FP64 solvers (LAPACK's and the GPU's)
    E2 = float(np.linalg.norm(Cg - Cr, 2)) + n * 1e-15 * lam[0]
    e_c = float(np.linalg.norm(Cg - Cr) / np.linalg.norm(Cr))
    assert e_c <= c_tol, f"{label} covariance {e_c:.2e} > {c_tol:.0e}"
    assert np.all(np.diff(w) <= 0), f"{label} eigenvalues not descending"
    slack = 1e-12 * lam[0]
    assert np.abs(w - lam).max() <= E2 + slack, f"{label} eigenvalues outside the Weyl bound"
    # kept projector
    gaps = []
    if k_lo > 0:
        gaps.append(lam[k_lo - 1] - lam[k_lo])
    if k_hi < n - 1:
        gaps.append(lam[k_hi] - lam[k_hi + 1])
    delta = min(gaps) if gaps else np.inf
    Pk = V[:, k_lo:k_hi + 1] @ V[:, k_lo:k_hi + 1].conj().T
    Pr = Vr[:, k_lo:k_hi + 1] @ Vr[:, k_lo:k_hi + 1].conj().T
    e_proj = float(np.linalg.norm(Pk - Pr, 2))
    if delta > 2 * E2 + slack:
        b_proj = E2 / (delta - E2) + 1e-11 if np.isfinite(delta) else 1e-11
        assert e_proj <= b_proj, f"{label} projector {e_proj:.2e} > Davis-Kahan bound {b_proj:.2e}"
    # per-mode vectors
    checked, worst_sin, worst_vec = 0, 0.0, 0.0
    for k in range(n):
        gap = min([abs(lam[k] - lam[j]) for j in range(n) if j != k] + [np.inf])
        if not (gap > 10 * E2 + slack and gap > 1e-6 * lam[0]):
            continue
        b_sin = E2 / (gap - E2) + 1e-12
        # sin(angle) as the norm of the part of v_k orthogonal to the oracle's
        # (1 - |<.,.>|^2 would lose everything below 1e-8 to cancellation)
        s = float(np.linalg.norm(V[:, k] - Vr[:, k] * np.vdot(Vr[:, k], V[:, k])))
        assert s <= b_sin, f"{label} mode {k}: sin angle {s:.2e} > {b_sin:.2e}"
        worst_sin = max(worst_sin, s)
        mags = np.sort(np.abs(Vr[:, k]))[::-1]
        rho = mags[0]
        if n == 1 or mags[0] - mags[1] > 4 * b_sin:
            dv = float(np.linalg.norm(V[:, k] - Vr[:, k]))
            b_vec = b_sin * (1 + 2 / rho) + 1e-12
            assert dv <= b_vec, f"{label} phase-fixed mode {k}: {dv:.2e} > {b_vec:.2e}"
            worst_vec = max(worst_vec, dv)
        checked += 1
    return {"cov": e_c, "lam_rel_each": float(np.max(np.abs(w - lam) / np.maximum(np.abs(lam), 1e-300))),
            "proj": e_proj, "gap_b": float(delta / lam[0]) if np.isfinite(delta) else float("inf"),
            "modes": checked, "sin": worst_sin, "vec": worst_vec}


def fmt_eig(d):
    return (f"C {d['cov']:.2e} projector {d['proj']:.2e} (gap {d['gap_b']:.1e}) "
            f"modes {d['modes']} sin {d['sin']:.1e} vec {d['vec']:.1e}")
