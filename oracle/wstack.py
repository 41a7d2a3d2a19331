"""FP64 oracle of the w-stacking hybrid (test infrastructure only; nothing in
the product imports it).

Paper passages followed: appendix E. The w-term is split in two: the
visibilities are binned into P stacks by w; the image of stack p is multiplied
by the exact phase screen of the stack's central w_p before zero padding and
the DFT (each stack has its own Z_p and FFT), and the residual w - w_p is
carried, as in the unstacked operator, by the small w-kernel convolved
row-wise with the interpolation kernel in G_p:

    Phi x = sum_p G_p F Z_p x,      Re{Phi^dagger y} = Re sum_p Z_p^dagger F^dagger G_p^H y_p,
    Z_p x = Z (c_p x),              c_p(n) = exp(-2 pi i w_p (sqrt(1 - l^2 - m^2) - 1)),

with l = n_x delta, m = n_y delta for the centred pixel n (the direct model's
w-phase, eq. 1 with the closed-form w-term of appendix E).

Readings where the paper is silent: P stacks of equal width over [-W, W],
centres w_p = -W + (2p + 1) W / P; each visibility joins the stack whose
interval holds its w (|w| = W clipped into the end stacks); the residual's
w-plane table spans [-W/P, W/P] with the same number of planes, and its
supports follow the unstacked rule. With P = 1 the operator is the unstacked
one (w_0 = 0, c_0 = 1).

Parity: pinned in tests/test_oracle_wstack.py (P = 1 against the unstacked
oracle, the adjoint identity, visibilities at stack centres against the
brute-force direct model to the interpolation accuracy, and the gain over
w-projection alone when W outgrows the largest w-kernel).
"""
from __future__ import annotations

import numpy as np

from . import phi as OP


def stack_of(w: np.ndarray, W: float, P: int) -> np.ndarray:
    """Stack index of each w: floor((w + W) P / (2W)) clipped to [0, P)."""
    if P <= 1 or W == 0.0:
        return np.zeros(np.shape(w), dtype=np.int32)
    s = np.floor((np.asarray(w) + W) * P / (2.0 * W))
    return np.clip(s, 0, P - 1).astype(np.int32)


def stack_centres(W: float, P: int) -> np.ndarray:
    if P <= 1 or W == 0.0:
        return np.zeros(max(P, 1))
    return -W + (2.0 * np.arange(P) + 1.0) * W / P


def phase_screen(N: int, cell: float, w: float) -> np.ndarray:
    """c(n) = exp(-2 pi i w (sqrt(1 - l^2 - m^2) - 1)), [iy, ix], n = index - N/2."""
    n = (np.arange(N, dtype=np.float64) - N // 2) * cell
    s = n[:, None] ** 2 + n[None, :] ** 2
    return np.exp(-2j * np.pi * w * (np.sqrt(1.0 - s) - 1.0))


class StackedOperator:
    """Phi = sum_p G_p F Z_p over P w-stacks, FP64 throughout."""

    def __init__(self, N: int, uvw: np.ndarray, cell: float, W: float, n_wplanes: int, P: int,
                 J: int = 7, sigma: float = 2.0, hmax: int = 5):
        self.N, self.cell, self.W, self.P = N, cell, W, P
        self.uvw = np.ascontiguousarray(uvw, dtype=np.float64)
        self.M = self.uvw.shape[0]
        self.stack = stack_of(self.uvw[:, 2], W, P)
        self.centres = stack_centres(W, P)
        self.W_res = W / P if P > 1 else W
        self.idx, self.ops, self.screens = [], [], []
        for p in range(max(P, 1)):
            idx = np.nonzero(self.stack == p)[0]
            res = self.uvw[idx].copy()
            res[:, 2] -= self.centres[p]
            self.idx.append(idx)
            self.ops.append(OP.Operator(N, res, cell=cell, W=self.W_res, n_wplanes=n_wplanes, J=J, sigma=sigma,
                                        hmax=hmax))
            self.screens.append(phase_screen(N, cell, self.centres[p]))
        op0 = self.ops[0]
        self.Np, self.J, self.beta = op0.Np, J, op0.beta
        # Z's correction 1 / (kappa_hat(n_x / N') kappa_hat(n_y / N')) and the cell map n -> n mod N'
        k1 = np.array([1.0 / OP.kb_hat((i - N // 2) / self.Np, J, self.beta) for i in range(N)])
        self.icorr = np.outer(k1, k1)
        self.cells = (np.arange(N) - N // 2) % self.Np

    def zpad(self, xc: np.ndarray) -> np.ndarray:
        """Z of a complex image: X0[n mod N'] = x_n / (kappa_hat kappa_hat), zero elsewhere."""
        X0 = np.zeros((self.Np, self.Np), dtype=np.complex128)
        X0[np.ix_(self.cells, self.cells)] = xc * self.icorr
        return X0

    def zpad_adj(self, Y: np.ndarray) -> np.ndarray:
        """Z^dagger: crop the N centred cells and apply the correction (complex)."""
        return Y[np.ix_(self.cells, self.cells)] * self.icorr

    def phi(self, x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        y = np.zeros(self.M, dtype=np.complex128)
        for p, op in enumerate(self.ops):
            if self.idx[p].size == 0:
                continue
            X = OP.fft2(self.zpad(x * self.screens[p]), -1)
            y[self.idx[p]] = op.degrid(X)
        return y

    def phi_adj(self, y: np.ndarray) -> np.ndarray:
        y = np.asarray(y, dtype=np.complex128)
        x = np.zeros((self.N, self.N))
        for p, op in enumerate(self.ops):
            if self.idx[p].size == 0:
                continue
            Y = OP.fft2(op.grid(y[self.idx[p]]), +1)
            x += np.real(np.conj(self.screens[p]) * self.zpad_adj(Y))
        return x

    def phi_adj_phi(self, x: np.ndarray) -> np.ndarray:
        return self.phi_adj(self.phi(x))

    def nnz(self) -> int:
        return sum(op.nnz() for op in self.ops)
