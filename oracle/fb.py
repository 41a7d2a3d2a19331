"""FP64 oracle of the forward-backward loop around the data-fidelity gradient
(test infrastructure only).

Paper passages followed:
  * appendix A, eq. (A2): x^{k+1} = prox_{gamma lambda r}(x^k - gamma grad f(x^k)),
    gamma < 2/L, L = ||Re{Phi^dagger Phi}||_S; the l1 prox is soft-thresholding;
  * appendix B, eq. (B2): gamma lambda = tau / sqrt(2L), gamma = 1.98 / L;
  * appendix C, eqs. (C2)-(C3): rescaling by alpha, sigma = tau / (alpha sqrt(2L));
  * appendix F (footnote): dirty-beam normalisation beta = max(Re{Phi^dagger Phi} delta).

Readings where the paper is silent: the Haar-l1 + positivity prox is the
composition max(0, Psi soft_t(Psi^dagger z)) with Psi the orthonormal 2D Haar
basis, four levels, every coefficient thresholded; the power method starts
from a seeded Gaussian image and stops when the relative change of the
estimate drops below rtol; SNR = 20 log10(||x_true|| / ||x_true - x||).

Parity: Haar orthonormality, the identity-basis special case, the soft
threshold's optimality conditions and homogeneity pin the prox; a dense
eigensolver pins the power method; scale equivariance and a monotone objective
pin the iteration (tests/test_oracle_fb.py).
"""
from __future__ import annotations

import math

import numpy as np


# ----------------------------------------------------------------------------
# Orthonormal 2D Haar transform (Psi^dagger analysis, Psi synthesis)
# ----------------------------------------------------------------------------
def haar_analysis(x: np.ndarray, levels: int = 4):
    """Psi^dagger x: list of (LH, HL, HH) detail triples, finest first, then LL."""
    a = np.asarray(x, dtype=np.float64)
    out = []
    for _ in range(levels):
        x00, x01 = a[0::2, 0::2], a[0::2, 1::2]
        x10, x11 = a[1::2, 0::2], a[1::2, 1::2]
        ll = (x00 + x01 + x10 + x11) * 0.5
        lh = (x00 - x01 + x10 - x11) * 0.5
        hl = (x00 + x01 - x10 - x11) * 0.5
        hh = (x00 - x01 - x10 + x11) * 0.5
        out.append((lh, hl, hh))
        a = ll
    out.append(a)
    return out


def haar_synthesis(c) -> np.ndarray:
    """Psi c, the inverse (= transpose) of haar_analysis."""
    a = c[-1]
    for lh, hl, hh in reversed(c[:-1]):
        H, W = a.shape
        x = np.empty((2 * H, 2 * W))
        x[0::2, 0::2] = (a + lh + hl + hh) * 0.5
        x[0::2, 1::2] = (a - lh + hl - hh) * 0.5
        x[1::2, 0::2] = (a + lh - hl - hh) * 0.5
        x[1::2, 1::2] = (a - lh - hl + hh) * 0.5
        a = x
    return a


def haar_flat(c) -> np.ndarray:
    parts = [np.ravel(t) for trip in c[:-1] for t in trip] + [np.ravel(c[-1])]
    return np.concatenate(parts)


def soft(c: np.ndarray, t: float) -> np.ndarray:
    """Closed-form prox of t||.||_1 (appendix A): sign(c) max(|c| - t, 0)."""
    return np.sign(c) * np.maximum(np.abs(c) - t, 0.0)


def prox_haar_pos(z: np.ndarray, t: float, levels: int = 4) -> np.ndarray:
    """max(0, Psi soft_t(Psi^dagger z))."""
    c = haar_analysis(z, levels)
    c = [tuple(soft(u, t) for u in trip) for trip in c[:-1]] + [soft(c[-1], t)]
    return np.maximum(haar_synthesis(c), 0.0)


# ----------------------------------------------------------------------------
# Power method for L = ||Re{Phi^dagger Phi}||_S (appendix A)
# ----------------------------------------------------------------------------
def power_norm(apply_A, x0: np.ndarray, max_it: int = 500, rtol: float = 1e-8):
    """Returns (L, iterations). x <- A x / ||A x||, L = ||A x|| for unit x."""
    x = x0 / np.linalg.norm(x0)
    L = 0.0
    for it in range(1, max_it + 1):
        v = apply_A(x)
        Ln = float(np.linalg.norm(v))
        x = v / Ln
        if it > 1 and abs(Ln - L) <= rtol * Ln:
            return Ln, it
        L = Ln
    return L, max_it


# ----------------------------------------------------------------------------
# Parameter rules
# ----------------------------------------------------------------------------
def tau_from_isnr(phi_x: np.ndarray, isnr_db: float) -> float:
    """Noise std such that ||Phi x|| / (sqrt(M) tau) = 10^{iSNR/20}."""
    return float(np.linalg.norm(phi_x) * 10.0 ** (-isnr_db / 20.0) / math.sqrt(phi_x.size))


def complex_noise(tau: float, normals: np.ndarray) -> np.ndarray:
    """n = (tau / sqrt 2)(a + i b), so that E|n_m|^2 = tau^2 (eq. 1)."""
    return (tau / math.sqrt(2.0)) * normals


def threshold(tau: float, L: float) -> float:
    """gamma lambda = tau / sqrt(2L) (eq. B2)."""
    return tau / math.sqrt(2.0 * L)


def step_size(L: float) -> float:
    return 1.98 / L


def dirty_beam_peak(op) -> float:
    """beta = max_i (Re{Phi^dagger Phi} delta)_i, delta at the phase centre."""
    d = np.zeros((op.N, op.N))
    d[op.N // 2, op.N // 2] = 1.0
    return float(op.phi_adj_phi(d).max())


def alpha_rescale(dirty_peak: float, beta: float, tau: float, L: float, sigma_train: float) -> float:
    """alpha >= peak estimate; also large enough that tau/(alpha sqrt(2L)) <= sigma_train
    (eqs. C2-C3: data are matched to the denoiser)."""
    return max(dirty_peak / beta, tau / (sigma_train * math.sqrt(2.0 * L)))


def sigma_from(tau: float, alpha: float, L: float) -> float:
    """sigma = tau / (alpha sqrt(2L)) (eq. C3)."""
    return tau / (alpha * math.sqrt(2.0 * L))


def snr_db(x_true: np.ndarray, x: np.ndarray) -> float:
    return float(20.0 * math.log10(np.linalg.norm(x_true) / np.linalg.norm(x_true - x)))


# ----------------------------------------------------------------------------
# Forward-backward
# ----------------------------------------------------------------------------
def fb_step(op, x: np.ndarray, y: np.ndarray, gamma: float, denoise):
    """One iteration of eq. (A2). Returns (x_new, ||x_new - x||^2, ||x_new||^2, ||Phi x - y||^2)."""
    g, rr = op.grad(x, y)
    z = x - gamma * g
    xn = denoise(z)
    return xn, float(np.sum((xn - x) ** 2)), float(np.sum(xn ** 2)), rr


def fb(op, y: np.ndarray, L: float, t: float, n_iter: int, x0: np.ndarray | None = None,
       x_true: np.ndarray | None = None, denoise=None):
    """Plain FB with the Haar-l1 + positivity prox (or ``denoise``) from x0 (default 0)."""
    gamma = step_size(L)
    x = np.zeros((op.N, op.N)) if x0 is None else np.array(x0, dtype=np.float64)
    den = denoise if denoise is not None else (lambda z: prox_haar_pos(z, t))
    hist = []
    for _ in range(n_iter):
        x, dx2, x2, rr = fb_step(op, x, y, gamma, den)
        rec = {"rel_change": math.sqrt(dx2 / x2) if x2 > 0 else 0.0, "residual2": rr}
        if x_true is not None:
            rec["snr_db"] = snr_db(x_true, x)
        hist.append(rec)
    return x, hist


def objective(op, x: np.ndarray, y: np.ndarray, t_over_gamma: float, levels: int = 4) -> float:
    """f(x) + lambda r(x) with r = ||Psi^dagger x||_1 + indicator of x >= 0."""
    if (x < 0).any():
        return math.inf
    r = op.phi(x) - y
    return 0.5 * float(np.vdot(r, r).real) + t_over_gamma * float(np.abs(haar_flat(haar_analysis(x, levels))).sum())
