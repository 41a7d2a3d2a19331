"""FP64 oracle of the wide-field measurement operator (test infrastructure only).

Paper passages followed:
  * eq. (1): y = Phi x + n with Phi = G F Z; Z zero-pads and corrects for the
    interpolation kernel, F is the DFT on the fine N' grid, G holds one sparse
    interpolation row per visibility;
  * appendix E: the w-term is a closed-form chirp; its offset part is applied
    as a small w-kernel convolved row-wise with the interpolation kernel in G;
    Phi^dagger Phi is a sum of per-block terms (eq. E2);
  * appendix A: the data-fidelity gradient Re{Phi^dagger Phi} x - Re{Phi^dagger y}.

Discrete operator (the readings where the paper is silent):
  * p = omega N'/(2 pi) per axis (FP64), window centre c = floor(p + 1/2),
    fraction f = p - c;
  * Kaiser-Bessel width J = 7, beta from Beatty et al. (2005) at sigma = 2;
    the correction in Z is the closed-form transform of the kernel;
  * w-planes: n_wplanes (odd) values w_j = (j - P_half) dw, dw = W / P_half;
    each visibility uses the nearest plane;
  * per-plane half support h_j = 0 for w_j = 0, else
    min(hmax, ceil(hex_j) + 1) with hex_j = |w_j| sigma N^2 delta^2 / 2 the
    per-axis half-bandwidth (in grid cells) of the paraxial chirp
    exp(i pi w (n delta)^2) at the image edge;
  * per-plane taps k_j[q], |q| <= h_j: least-squares fit of that chirp over the
    image support n in [-N/2, N/2) by the Fourier modes exp(2 pi i q n / N').

Parity: pinned by the brute-force direct model (tests/test_oracle_operator.py),
the adjoint identity, the closed forms for kappa_hat and the FFT.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import build as _build

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        d, i, i64, p = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
        op = [i, i, i, d, i, i64, p, p, p, p, p]
        L.or_i0.restype = d; L.or_i0.argtypes = [d]
        L.or_kb_beta.restype = d; L.or_kb_beta.argtypes = [i, d]
        L.or_kb.restype = d; L.or_kb.argtypes = [d, i, d]
        L.or_kb_hat.restype = d; L.or_kb_hat.argtypes = [d, i, d]
        L.or_phi_c.argtypes = op + [p, p]
        L.or_phi_adj_c.argtypes = op + [p, p]
        L.or_degrid_c.argtypes = op + [p, p]
        L.or_grid_c.argtypes = op + [p, p]
        L.or_g_row_c.argtypes = op + [i64, p, p]; L.or_g_row_c.restype = i
        L.or_grad_c.argtypes = op + [p, p, p]; L.or_grad_c.restype = d
        L.or_fft2d_c.argtypes = [p, i, i]
        L.or_fft1d_c.argtypes = [p, i, i]
        L.or_zpad_c.argtypes = [i, i, i, d, p, p]
        L.or_zpad_adj_c.argtypes = [i, i, i, d, p, p]
        L.or_dft_c.argtypes = [i, i64, p, d, i, p, p]
        L.or_dft_adj_c.argtypes = [i, i64, p, d, i, p, p]
        L.or_num_threads.restype = i
        L.or_set_num_threads.argtypes = [i]
        L.or_set_num_threads.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return lib().or_num_threads()


def set_num_threads(n: int) -> None:
    lib().or_set_num_threads(int(n))


# ----------------------------------------------------------------------------
# Kernel functions (exposed for the pins)
# ----------------------------------------------------------------------------
def i0(x: float) -> float:
    return lib().or_i0(x)


def kb_beta(J: int = 7, sigma: float = 2.0) -> float:
    return lib().or_kb_beta(J, sigma)


def kb(t: float, J: int = 7, beta: float | None = None) -> float:
    return lib().or_kb(t, J, kb_beta(J) if beta is None else beta)


def kb_hat(nu: float, J: int = 7, beta: float | None = None) -> float:
    return lib().or_kb_hat(nu, J, kb_beta(J) if beta is None else beta)


def fft2(a: np.ndarray, sign: int = -1) -> np.ndarray:
    """Unnormalised 2D DFT with the oracle's own radix-2 FFT (sign -1 forward)."""
    out = np.ascontiguousarray(a, dtype=np.complex128).copy()
    lib().or_fft2d_c(_ptr(out), out.shape[0], sign)
    return out


def fft1(a: np.ndarray, sign: int = -1) -> np.ndarray:
    out = np.ascontiguousarray(a, dtype=np.complex128).copy()
    lib().or_fft1d_c(_ptr(out), out.shape[0], sign)
    return out


# ----------------------------------------------------------------------------
# w-planes and w-kernels
# ----------------------------------------------------------------------------
def wplane_index(w: np.ndarray, W: float, n_wplanes: int) -> np.ndarray:
    """Nearest plane of each w: clip(floor(w/dw + 1/2), -P_half, P_half) + P_half."""
    P_half = (n_wplanes - 1) // 2
    if P_half == 0 or W == 0.0:
        return np.zeros(w.shape, dtype=np.int32)
    dw = W / P_half
    j = np.floor(w / dw + 0.5)
    return (np.clip(j, -P_half, P_half) + P_half).astype(np.int32)


def wplane_values(W: float, n_wplanes: int) -> np.ndarray:
    P_half = (n_wplanes - 1) // 2
    if P_half == 0 or W == 0.0:
        return np.zeros(n_wplanes)
    dw = W / P_half
    return (np.arange(n_wplanes) - P_half) * dw


def wplane_h(wj: np.ndarray, N: int, sigma: float, cell: float, hmax: int) -> np.ndarray:
    """Half support per plane: 0 at w = 0, else min(hmax, ceil(hex) + 1)."""
    h = np.zeros(wj.shape, dtype=np.int32)
    for idx, w in enumerate(wj):
        if w == 0.0:
            continue
        hex_ = abs(w) * sigma * N * N * cell * cell * 0.5
        h[idx] = min(hmax, int(math.ceil(hex_)) + 1)
    return h


def wkernel_taps(w: float, h: int, N: int, Np: int, cell: float) -> np.ndarray:
    """Least-squares taps k[q], |q| <= h, with sum_q k[q] exp(2 pi i q n/N')
    ~ exp(i pi w (n cell)^2) over n in [-N/2, N/2) (paraxial chirp, appendix E)."""
    n = np.arange(-N // 2, N // 2, dtype=np.float64)
    q = np.arange(-h, h + 1, dtype=np.float64)
    A = np.exp(2j * np.pi * np.outer(n, q) / Np)
    c = np.exp(1j * np.pi * w * (n * cell) ** 2)
    k, *_ = np.linalg.lstsq(A, c, rcond=None)
    return k


class Operator:
    """Phi = G F Z for fixed visibility coordinates, FP64 throughout.

    Parameters follow the C interface: ``uvw`` float64 [M, 3] = (omega_u,
    omega_v rad/pixel, w wavelengths), ``cell`` the pixel size (rad) used by
    the w-term, ``W`` the w bound of the plane table, ``n_wplanes`` odd.
    """

    def __init__(self, N: int, uvw: np.ndarray, cell: float = 0.0, W: float = 0.0,
                 n_wplanes: int = 1, J: int = 7, sigma: float = 2.0, hmax: int = 5):
        self.N, self.J, self.sigma, self.hmax = N, J, sigma, hmax
        self.Np = int(round(sigma * N))
        if N < 2 or N % 2 or self.Np & (self.Np - 1) or n_wplanes % 2 == 0 or J % 2 == 0:
            raise ValueError("oracle needs even N with a power-of-two grid N', odd J and n_wplanes")
        self.beta = kb_beta(J, sigma)
        self.cell, self.W, self.n_wplanes = cell, W, n_wplanes
        self.uvw = np.ascontiguousarray(uvw, dtype=np.float64)
        self.M = self.uvw.shape[0]
        scale = self.Np / (2.0 * np.pi)
        self.pu = np.ascontiguousarray(self.uvw[:, 0] * scale)
        self.pv = np.ascontiguousarray(self.uvw[:, 1] * scale)
        self.plane = np.ascontiguousarray(wplane_index(self.uvw[:, 2], W, n_wplanes))
        self.wj = wplane_values(W, n_wplanes)
        self.plane_h = np.ascontiguousarray(wplane_h(self.wj, N, sigma, cell, hmax))
        K = 2 * hmax + 1
        taps = np.zeros((n_wplanes, K), dtype=np.complex128)
        used = np.unique(self.plane) if self.M else np.zeros(0, np.int32)
        for j in used:
            h = int(self.plane_h[j])
            taps[j, hmax - h: hmax + h + 1] = wkernel_taps(self.wj[j], h, N, self.Np, cell)
        self.plane_k = np.ascontiguousarray(taps)

    # -- plumbing -------------------------------------------------------------
    def _args(self):
        return (self.N, self.Np, self.J, self.beta, self.hmax, self.M, _ptr(self.pu),
                _ptr(self.pv), _ptr(self.plane), _ptr(self.plane_h), _ptr(self.plane_k))

    def subset(self, idx: np.ndarray) -> "Operator":
        """The operator restricted to the visibilities ``idx`` (a data block)."""
        o = object.__new__(Operator)
        o.__dict__.update(self.__dict__)
        o.uvw = np.ascontiguousarray(self.uvw[idx])
        o.M = o.uvw.shape[0]
        o.pu = np.ascontiguousarray(self.pu[idx])
        o.pv = np.ascontiguousarray(self.pv[idx])
        o.plane = np.ascontiguousarray(self.plane[idx])
        return o

    # -- the operator ---------------------------------------------------------
    def phi(self, x: np.ndarray) -> np.ndarray:
        """y = G F Z x (complex128 [M])."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.shape == (self.N, self.N)
        y = np.empty(self.M, dtype=np.complex128)
        lib().or_phi_c(*self._args(), _ptr(x), _ptr(y))
        return y

    def phi_adj(self, y: np.ndarray) -> np.ndarray:
        """Re{Phi^dagger y} = Re{Z^dagger F^dagger G^H y} (float64 [N, N])."""
        y = np.ascontiguousarray(y, dtype=np.complex128)
        assert y.shape == (self.M,)
        x = np.empty((self.N, self.N), dtype=np.float64)
        lib().or_phi_adj_c(*self._args(), _ptr(y), _ptr(x))
        return x

    def phi_adj_phi(self, x: np.ndarray) -> np.ndarray:
        return self.phi_adj(self.phi(x))

    def grad(self, x: np.ndarray, y: np.ndarray | None = None):
        """(Re{Phi^dagger (Phi x - y)}, ||Phi x - y||^2) (appendix A)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        g = np.empty((self.N, self.N), dtype=np.float64)
        yp = None
        if y is not None:
            y = np.ascontiguousarray(y, dtype=np.complex128)
            yp = _ptr(y)
        rr = lib().or_grad_c(*self._args(), _ptr(x), yp, _ptr(g))
        return g, rr

    def degrid(self, X: np.ndarray) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.complex128)
        y = np.empty(self.M, dtype=np.complex128)
        lib().or_degrid_c(*self._args(), _ptr(X), _ptr(y))
        return y

    def grid(self, r: np.ndarray) -> np.ndarray:
        r = np.ascontiguousarray(r, dtype=np.complex128)
        Y = np.empty((self.Np, self.Np), dtype=np.complex128)
        lib().or_grid_c(*self._args(), _ptr(r), _ptr(Y))
        return Y

    def zpad(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        X0 = np.empty((self.Np, self.Np), dtype=np.complex128)
        lib().or_zpad_c(self.N, self.Np, self.J, self.beta, _ptr(x), _ptr(X0))
        return X0

    def zpad_adj(self, Y: np.ndarray) -> np.ndarray:
        Y = np.ascontiguousarray(Y, dtype=np.complex128)
        x = np.empty((self.N, self.N), dtype=np.float64)
        lib().or_zpad_adj_c(self.N, self.Np, self.J, self.beta, _ptr(Y), _ptr(x))
        return x

    def g_row(self, m: int):
        """Dense values and flat grid indices of row m of G (window order)."""
        S = 2 * self.hmax + self.J
        vals = np.empty(S * S, dtype=np.complex128)
        cols = np.empty(S * S, dtype=np.int64)
        s = lib().or_g_row_c(*self._args(), int(m), _ptr(vals), _ptr(cols))
        return vals[: s * s].copy(), cols[: s * s].copy(), s

    def nnz(self) -> int:
        s = 2 * self.plane_h[self.plane].astype(np.int64) + self.J
        return int((s * s).sum())

    # -- the direct model -----------------------------------------------------
    def dft(self, x: np.ndarray, paraxial: bool = False) -> np.ndarray:
        """Brute-force exact model, O(M N^2): tiny inputs only."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(self.M, dtype=np.complex128)
        lib().or_dft_c(self.N, self.M, _ptr(self.uvw), self.cell, int(paraxial), _ptr(x), _ptr(y))
        return y

    def dft_adj(self, y: np.ndarray, paraxial: bool = False) -> np.ndarray:
        y = np.ascontiguousarray(y, dtype=np.complex128)
        x = np.empty((self.N, self.N), dtype=np.float64)
        lib().or_dft_adj_c(self.N, self.M, _ptr(self.uvw), self.cell, int(paraxial), _ptr(y), _ptr(x))
        return x


def block_sum_phi_adj_phi(op: Operator, offsets: np.ndarray, x: np.ndarray) -> np.ndarray:
    """sum_p Re{Phi_p^dagger Phi_p} x over contiguous visibility blocks (eq. E2)."""
    out = np.zeros((op.N, op.N))
    for b in range(len(offsets) - 1):
        sub = op.subset(np.arange(offsets[b], offsets[b + 1]))
        out += sub.phi_adj_phi(x)
    return out
