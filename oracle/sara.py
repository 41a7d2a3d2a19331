"""FP64 oracle of uSARA's denoiser and reweighting (test infrastructure only;
nothing in the product imports it).

Paper passages followed (section "uSARA's handcrafted denoiser"): the prior
is non-negativity plus sparsity in an overcomplete dictionary Psi that stacks
several orthogonal wavelet bases under one normalisation, with the log-sum
penalty lambda sum_n rho log(1 + |(Psi^dagger x)_n| / rho); the non-convex
problem is solved by reweighting: a series of weighted-l1 + non-negativity
problems, each by FB, whose prox has no closed form and is computed by
sub-iterations; gamma lambda = tau / sqrt(2L) (eq. lambda), gamma = 1.98 / L,
rho = gamma lambda.

Readings where the paper is silent (the dictionary is that of the SARA prior
it cites):
  * bases: Dirac and the Daubechies wavelets with 1..8 vanishing moments,
    each an orthonormal 2D separable transform with 4 levels and periodic
    boundaries; Psi = [Psi_1 ... Psi_9] / 3, so Psi Psi^dagger = I;
  * Daubechies filter with p vanishing moments: the minimum-phase spectral
    factor, h(z) = sqrt(2) ((1 + z) / 2)^p Q(z) / Q(1) with Q the monic
    polynomial whose roots are those of z^{p-1} P_p((2 - z - 1/z) / 4),
    P_p(y) = sum_{k<p} C(p-1+k, k) y^k, lying outside the unit circle
    (|Q(e^{i omega})|^2 is then proportional to P_p(sin^2(omega/2)));
    high-pass g[t] = (-1)^t h[L-1-t];
  * one analysis level on length n: a[k] = sum_t h[t] x[(2k + t) mod n],
    d[k] = sum_t g[t] x[(2k + t) mod n]; rows then columns; the low-pass
    block (top-left) is transformed again;
  * prox of t ||w . Psi^dagger x||_1 + iota_+(x) at z by dual
    forward-backward with unit step (valid since ||Psi^dagger|| = 1):
        x_k = max(0, z - Psi v_k),  v_{k+1} = clip(v_k + Psi^dagger x_k, -t w, t w),
    a fixed number of sub-iterations, warm-started from the previous dual
    variable; the output is the last x_k;
  * reweighting: w_n = rho / (rho + |(Psi^dagger x)_n|) (the weights of the
    log-sum's linear majorant at x), starting from w = 1.

Parity: pinned in tests/test_oracle_sara.py (closed forms of the first two
filters, orthonormality and vanishing moments of all eight, perfect
reconstruction and energy preservation of the transforms, the Haar level
against its closed form, Psi Psi^dagger = I, the prox against its closed form
for the Dirac basis alone and against an independent primal-dual solver for the
whole dictionary).
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import polynomial as PP

LEVELS = 4
N_DB = 8
N_BASES = 1 + N_DB


def daubechies(p: int) -> np.ndarray:
    """Low-pass filter (2p taps) of the minimum-phase Daubechies wavelet with p vanishing moments.

    The roots are taken in y = sin^2(omega/2) first (P_p has degree p - 1 there and is far better
    conditioned than its degree-2p-2 image in z), each polished by Newton steps, then mapped to
    the z-plane root of z^2 - 2(1 - 2y) z + 1 = 0 outside the unit circle."""
    coef = np.array([math.comb(p - 1 + k, k) for k in range(p)], dtype=np.float64)
    zs = []
    if p > 1:
        for y in PP.polyroots(coef):
            for _ in range(3):
                y = y - PP.polyval(y, coef) / PP.polyval(y, PP.polyder(coef))
            b = 1.0 - 2.0 * y
            disc = np.sqrt(complex(b * b - 1.0))
            z = b + disc if abs(b + disc) > 1.0 else b - disc
            zs.append(z)
    q = np.real(PP.polyfromroots(zs)) if zs else np.ones(1)
    h = PP.polymul(PP.polypow([0.5, 0.5], p), q)
    return h * (math.sqrt(2.0) / h.sum())


def highpass(h: np.ndarray) -> np.ndarray:
    L = h.size
    return np.array([(-1) ** t * h[L - 1 - t] for t in range(L)])


FILTERS = [daubechies(p) for p in range(1, N_DB + 1)]


def analysis(x: np.ndarray, h: np.ndarray, axis: int) -> np.ndarray:
    """One periodic analysis level along an axis: [low half, high half]."""
    n = x.shape[axis]
    g = highpass(h)
    k2 = 2 * np.arange(n // 2)
    a = sum(h[t] * np.take(x, (k2 + t) % n, axis=axis) for t in range(h.size))
    d = sum(g[t] * np.take(x, (k2 + t) % n, axis=axis) for t in range(h.size))
    return np.concatenate([a, d], axis=axis)


def synthesis(c: np.ndarray, h: np.ndarray, axis: int) -> np.ndarray:
    """Adjoint (and inverse) of ``analysis``."""
    n = c.shape[axis]
    g = highpass(h)
    a = np.take(c, np.arange(n // 2), axis=axis)
    d = np.take(c, np.arange(n // 2, n), axis=axis)
    x = np.zeros_like(c)
    k2 = 2 * np.arange(n // 2)
    xs = np.moveaxis(x, axis, 0)
    am, dm = np.moveaxis(a, axis, 0), np.moveaxis(d, axis, 0)
    for t in range(h.size):
        xs[(k2 + t) % n] += h[t] * am + g[t] * dm
    return x


def dwt2(x: np.ndarray, h: np.ndarray, levels: int = LEVELS) -> np.ndarray:
    c = np.array(x, dtype=np.float64, copy=True)
    n = c.shape[0]
    for _ in range(levels):
        c[:n, :n] = analysis(analysis(c[:n, :n], h, 1), h, 0)
        n //= 2
    return c


def idwt2(c: np.ndarray, h: np.ndarray, levels: int = LEVELS) -> np.ndarray:
    x = np.array(c, dtype=np.float64, copy=True)
    n = x.shape[0] >> (levels - 1)
    for _ in range(levels):
        x[:n, :n] = synthesis(synthesis(x[:n, :n], h, 0), h, 1)
        n *= 2
    return x


class Sara:
    """Psi = [Dirac, db1 .. db8] / 3 (or a subset of the bases), 4 levels."""

    def __init__(self, bases=("dirac",) + tuple(f"db{p}" for p in range(1, N_DB + 1)), levels: int = LEVELS):
        self.bases, self.levels = tuple(bases), levels
        self.scale = 1.0 / math.sqrt(len(self.bases))

    def _h(self, b):
        return FILTERS[int(b[2:]) - 1]

    def adj(self, x: np.ndarray) -> np.ndarray:
        """Psi^dagger x: [n_bases][N][N]."""
        out = []
        for b in self.bases:
            out.append(np.array(x, dtype=np.float64) if b == "dirac" else dwt2(x, self._h(b), self.levels))
        return np.stack(out) * self.scale

    def syn(self, c: np.ndarray) -> np.ndarray:
        """Psi c."""
        x = np.zeros(c.shape[1:])
        for i, b in enumerate(self.bases):
            x += c[i] if b == "dirac" else idwt2(c[i], self._h(b), self.levels)
        return x * self.scale

    def prox(self, z: np.ndarray, t: float, w: np.ndarray, n_sub: int, v0: np.ndarray | None = None):
        """Dual forward-backward for argmin_x ||x - z||^2/2 + t ||w . Psi^dagger x||_1 + iota_+(x).
        Returns (x, v) after n_sub sub-iterations."""
        v = np.zeros((len(self.bases),) + z.shape) if v0 is None else np.array(v0, dtype=np.float64)
        x = np.maximum(0.0, z - self.syn(v))
        for _ in range(n_sub):
            x = np.maximum(0.0, z - self.syn(v))
            v = np.clip(v + self.adj(x), -t * w, t * w)
        return x, v

    def reweight(self, x: np.ndarray, rho: float) -> np.ndarray:
        return rho / (rho + np.abs(self.adj(x)))

    def logsum(self, x: np.ndarray, rho: float) -> float:
        return float(np.sum(rho * np.log1p(np.abs(self.adj(x)) / rho)))


def usara(grad, x0: np.ndarray, gamma: float, t: float, iters: int, n_sub: int, reweight_every: int,
          sara: Sara | None = None):
    """Reweighted FB: x <- prox_{t, w}(x - gamma grad(x)) with the dual variable warm-started
    across iterations; every ``reweight_every`` iterations w <- rho / (rho + |Psi^dagger x|)
    with rho = t. ``grad(x)`` returns Re{Phi^dagger (Phi x - y)}. Returns (x, w)."""
    s = sara or Sara()
    x = np.array(x0, dtype=np.float64)
    w = np.ones((len(s.bases),) + x.shape)
    v = None
    for k in range(iters):
        x, v = s.prox(x - gamma * grad(x), t, w, n_sub, v)
        if reweight_every and (k + 1) % reweight_every == 0:
            w = s.reweight(x, t)
    return x, w
