"""FP64 oracle of the holographic form of Phi^dagger Phi (test infrastructure
only; nothing in the product imports it).

Paper passage followed: appendix E. With the data split into blocks p,
Phi^dagger Phi = sum_p Z^dagger F^dagger G_p^H G_p F Z = Z^dagger F^dagger H F Z with
H = sum_p H_p and H_p = G_p^H G_p (the holographic matrices): an N'^2 x N'^2
matrix on the fine grid whose size depends on the uv coverage and the
kernel supports, not on the number of visibilities. Entry
H[k, k'] = sum_m conj(G[m, k]) G[m, k'] is non-zero only when one window
holds both cells, so per axis |k - k'| <= S_max - 1 (S_max the largest
window side): H is a banded grid operator.

The oracle forms G from the operator oracle's rows (oracle/phi.py) as a sparse
matrix and H by a sparse product; the normal operator is then the composition
above, with the operator oracle's own Z, FFT and Z^dagger.

Parity: pinned in tests/test_oracle_holo.py against the operator oracle's
Re{Phi^dagger Phi} (pinned itself by the brute-force direct model), a closed
form for one visibility on a grid node, the per-block sum of eq. (E2), the
band, the Hermitian symmetry and positivity, and the blindness to M
(repeating every visibility doubles H).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import phi as OP


def g_matrix(op: OP.Operator) -> sp.csr_matrix:
    """G as an M x N'^2 sparse matrix (complex128), one window per row."""
    rows, cols, vals = [], [], []
    for m in range(op.M):
        v, c, _ = op.g_row(m)
        rows.append(np.full(v.size, m, dtype=np.int64))
        cols.append(c)
        vals.append(v)
    n = op.Np * op.Np
    if not rows:
        return sp.csr_matrix((op.M, n), dtype=np.complex128)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(op.M, n))


def holographic(op: OP.Operator) -> sp.csr_matrix:
    """H = G^H G (N'^2 x N'^2, complex128, sparse)."""
    G = g_matrix(op)
    return (G.conj().T @ G).tocsr()


def apply(H: sp.csr_matrix, X: np.ndarray) -> np.ndarray:
    """H X for a grid X [N'][N'] (row-major flat cell index gy N' + gx)."""
    return (H @ np.ascontiguousarray(X, dtype=np.complex128).ravel()).reshape(X.shape)


def normal(op: OP.Operator, H: sp.csr_matrix, x: np.ndarray) -> np.ndarray:
    """Re{Z^dagger F^dagger H F Z} x = Re{Phi^dagger Phi} x."""
    X = OP.fft2(op.zpad(x), -1)
    return op.zpad_adj(OP.fft2(apply(H, X), +1))


def band(H: sp.csr_matrix, Np: int) -> tuple[int, int]:
    """Largest per-axis cyclic distance |k - k'| over the stored entries (y, x)."""
    C = H.tocoo()
    ky, kx = C.row // Np, C.row % Np
    qy, qx = C.col // Np, C.col % Np
    dy = np.minimum((qy - ky) % Np, (ky - qy) % Np)
    dx = np.minimum((qx - kx) % Np, (kx - qx) % Np)
    return (int(dy.max()) if dy.size else 0, int(dx.max()) if dx.size else 0)
