"""Pins of the oracle's measurement operator (no GPU).

* GFZ against the brute-force direct model (paper eq. 1; appendix E w-term);
* the adjoint identity Re<Phi x, y> = <x, Re Phi^dagger y>;
* block additivity Phi^dagger Phi = sum_p Phi_p^dagger Phi_p (eq. E2);
* the least-squares w-kernel against the chirp it approximates.
"""
import math

import numpy as np
import pytest

import synth
from oracle import phi as O


def _tiny(N=32, M=500, W=0.0, n_wplanes=1, cell=20 * synth.ARCSEC, seed=11):
    uvw = synth.random_uvw(M, 2 * math.pi / 3, W, seed)
    return O.Operator(N, uvw, cell=cell, W=W, n_wplanes=n_wplanes)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_gfz_matches_direct_model_w0():
    op = _tiny()
    x = synth.random_image(op.N, 3)
    err = _rel(op.phi(x), op.dft(x))
    print(f"GFZ vs direct model (w=0): rel l2 {err:.3e}")
    assert err <= 1e-5


def test_adjoint_matches_direct_model_w0():
    op = _tiny()
    y = synth.noise_normals(op.M, 5)
    err = _rel(op.phi_adj(y), op.dft_adj(y))
    print(f"Re Phi^dagger vs direct adjoint (w=0): rel l2 {err:.3e}")
    assert err <= 1e-5


def test_gfz_matches_direct_model_wide_field():
    # Wide field: N = 64 at 60" cells (~1.07 deg), supports 7..17.
    N, cell = 64, 60 * synth.ARCSEC
    W = 2 * 4.0 / (2 * N * N * cell ** 2)          # hex(W) = 4 cells -> h = 5
    uvw = synth.random_uvw(400, 2 * math.pi / 3, W, 12)
    op = O.Operator(N, uvw, cell=cell, W=W, n_wplanes=2049)
    assert set(np.unique(op.plane_h[op.plane])) >= {2, 3, 4, 5}
    x = synth.random_image(N, 4)
    y = op.phi(x)
    err_par = _rel(y, op.dft(x, paraxial=True))
    err_exact = _rel(y, op.dft(x, paraxial=False))
    print(f"GFZ vs paraxial direct model: {err_par:.3e}; vs exact w-term: {err_exact:.3e}")
    # measured 1.3e-3 (paraxial) / 1.3e-3 (exact) -> gate at about twice that
    assert err_par <= 3e-3
    assert err_exact <= 3e-3
    # without the w-kernel (same data, w forced to 0) the error is two orders larger
    op0 = O.Operator(N, np.c_[uvw[:, :2], np.zeros(len(uvw))], cell=cell)
    assert _rel(op0.phi(x), op.dft(x, paraxial=True)) > 30 * err_par


@pytest.mark.parametrize("W,n_wplanes", [(0.0, 1), (30000.0, 257)])
def test_adjoint_identity(W, n_wplanes):
    op = _tiny(N=64, M=700, W=W, n_wplanes=n_wplanes, seed=21)
    x = synth.random_image(op.N, 6, positive=False)
    y = synth.noise_normals(op.M, 7)
    lhs = np.vdot(y, op.phi(x)).real          # Re <Phi x, y>
    rhs = float(np.sum(x * op.phi_adj(y)))    # <x, Re Phi^dagger y>
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_zpad_adjoint_and_grid_adjoint():
    op = _tiny(N=32, M=300, W=30000.0, n_wplanes=129, seed=5)
    rng = np.random.default_rng(0)
    x = rng.standard_normal((op.N, op.N))
    Y = rng.standard_normal((op.Np, op.Np)) + 1j * rng.standard_normal((op.Np, op.Np))
    assert np.vdot(Y, op.zpad(x)).real == pytest.approx(float(np.sum(x * op.zpad_adj(Y))), rel=1e-12)
    X = rng.standard_normal((op.Np, op.Np)) + 1j * rng.standard_normal((op.Np, op.Np))
    r = synth.noise_normals(op.M, 9)
    assert np.vdot(r, op.degrid(X)) == pytest.approx(np.vdot(op.grid(r), X), rel=1e-12)


def test_g_row_matches_degrid():
    op = _tiny(N=32, M=50, W=30000.0, n_wplanes=129, seed=8)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((op.Np, op.Np)) + 1j * rng.standard_normal((op.Np, op.Np))
    y = op.degrid(X)
    for m in range(op.M):
        vals, cols, s = op.g_row(m)
        assert s == 2 * op.plane_h[op.plane[m]] + 7
        assert y[m] == pytest.approx(np.sum(vals * X.ravel()[cols]), rel=1e-13)


def test_block_additivity():
    op = _tiny(N=32, M=600, W=30000.0, n_wplanes=129, seed=13)
    x = synth.random_image(op.N, 2)
    offsets = np.array([0, 17, 250, 251, 600])
    ref = op.phi_adj_phi(x)
    assert _rel(O.block_sum_phi_adj_phi(op, offsets, x), ref) <= 1e-13


def test_dirty_beam_peak_is_M_for_direct_model():
    # Phi delta at the phase centre is 1 for every visibility, so beta = M exactly
    op = _tiny(N=16, M=123)
    d = np.zeros((16, 16)); d[8, 8] = 1.0
    assert op.dft_adj(op.dft(d))[8, 8] == pytest.approx(op.M, rel=1e-14)
    assert op.phi_adj_phi(d)[8, 8] == pytest.approx(op.M, rel=1e-5)


@pytest.mark.parametrize("hex_,h,bound", [(0.5, 2, 3.0e-3), (1.0, 2, 1.0e-2), (2.0, 3, 7.5e-3),
                                         (3.0, 4, 4.5e-3), (4.0, 5, 2.6e-3)])
def test_wkernel_least_squares_fit(hex_, h, bound):
    N, cell = 2048, 1.68 * synth.ARCSEC
    Np = 2 * N
    w = 2 * hex_ / (2 * N * N * cell ** 2)
    assert O.wplane_h(np.array([w]), N, 2.0, cell, 5)[0] == h
    k = O.wkernel_taps(w, h, N, Np, cell)
    n = np.arange(-N // 2, N // 2)
    approx = (k[None, :] * np.exp(2j * np.pi * np.outer(n, np.arange(-h, h + 1)) / Np)).sum(1)
    err = np.abs(approx - np.exp(1j * np.pi * w * (n * cell) ** 2)).max()
    assert err <= bound
    # the fit is optimal: the residual is orthogonal to every Fourier mode used
    A = np.exp(2j * np.pi * np.outer(n, np.arange(-h, h + 1)) / Np)
    res = np.exp(1j * np.pi * w * (n * cell) ** 2) - approx
    assert np.abs(A.conj().T @ res).max() <= 1e-9 * N


def test_wplane_index_nearest():
    W, P = 1000.0, 11        # dw = 200
    w = np.array([-1000.0, -901.0, -899.0, -100.0, -99.9, 0.0, 99.9, 100.0, 1000.0, 1e9, -1e9])
    j = O.wplane_index(w, W, P)
    assert list(j) == [0, 0, 1, 5, 5, 5, 5, 6, 10, 10, 0]
