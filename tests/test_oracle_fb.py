"""Pins of the oracle's prox, power method and forward-backward loop (no GPU)."""
import math

import numpy as np
import pytest

import synth
from oracle import fb as F
from oracle import phi as O


def _op(N=16, M=300, seed=31):
    uvw = synth.random_uvw(M, 2 * math.pi / 3, 0.0, seed)
    return O.Operator(N, uvw)


def test_haar_one_level_closed_form():
    x = np.array([[1.0, 2.0], [3.0, 4.0]])
    c = F.haar_analysis(x, 1)
    lh, hl, hh = c[0]
    assert c[1][0, 0] == pytest.approx(5.0)          # (1+2+3+4)/2
    assert lh[0, 0] == pytest.approx(-1.0)           # (1-2+3-4)/2
    assert hl[0, 0] == pytest.approx(-2.0)           # (1+2-3-4)/2
    assert hh[0, 0] == pytest.approx(0.0)            # (1-2-3+4)/2


def test_haar_orthonormal():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((64, 64))
    c = F.haar_analysis(x, 4)
    flat = F.haar_flat(c)
    assert flat.size == x.size
    assert np.linalg.norm(flat) == pytest.approx(np.linalg.norm(x), rel=1e-14)
    assert np.abs(F.haar_synthesis(c) - x).max() <= 1e-13
    # Psi^dagger is linear and isometric -> inner products are kept
    y = rng.standard_normal((64, 64))
    assert float(np.dot(F.haar_flat(F.haar_analysis(y, 4)), flat)) == pytest.approx(float(np.sum(x * y)), rel=1e-12)


def test_haar_blockwise_on_16_aligned_blocks():
    # four levels act on each 16x16 aligned block independently (facet exactness)
    rng = np.random.default_rng(1)
    z = rng.standard_normal((64, 48))
    full = F.prox_haar_pos(z, 0.3)
    for by in range(0, 64, 16):
        for bx in range(0, 48, 16):
            blk = F.prox_haar_pos(z[by:by + 16, bx:bx + 16], 0.3)
            assert np.array_equal(blk, full[by:by + 16, bx:bx + 16])


def test_prox_identity_basis_is_shifted_positive_part():
    rng = np.random.default_rng(2)
    z = rng.standard_normal((32, 32))
    assert np.array_equal(F.prox_haar_pos(z, 0.25, levels=0), np.maximum(z - 0.25, 0.0))


def test_soft_threshold_optimality():
    # u = soft(c, t) minimises t|u| + (u - c)^2/2: c - u in t * subdifferential of |u|
    rng = np.random.default_rng(3)
    c = rng.standard_normal(10000) * 2
    t = 0.7
    u = F.soft(c, t)
    nz = u != 0
    assert np.allclose(c[nz] - u[nz], t * np.sign(u[nz]), rtol=0, atol=1e-15)
    assert (np.abs(c[~nz]) <= t).all()


def test_prox_homogeneity():
    rng = np.random.default_rng(4)
    z = rng.standard_normal((32, 32))
    for a in [0.01, 3.0, 1e4]:
        assert np.allclose(F.prox_haar_pos(a * z, a * 0.2), a * F.prox_haar_pos(z, 0.2), rtol=1e-14, atol=1e-14 * a)


def test_power_method_matches_dense_eigensolver():
    op = _op()
    N = op.N
    A = np.empty((N * N, N * N))
    for j in range(N * N):
        e = np.zeros(N * N); e[j] = 1.0
        A[:, j] = op.phi_adj_phi(e.reshape(N, N)).ravel()
    assert np.abs(A - A.T).max() <= 1e-9 * np.abs(A).max()
    lam = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert lam.min() >= -1e-9 * lam.max()                 # positive semi-definite
    L, it = F.power_norm(op.phi_adj_phi, synth.power_start(N), max_it=5000, rtol=1e-13)
    print(f"power method: L = {L:.12e} after {it} its; eigvalsh {lam.max():.12e}, "
          f"gap ratio {lam[-2] / lam[-1]:.5f}")
    # the estimate approaches lambda_max from below; its accuracy at a given stopping
    # tolerance depends on the gap lambda_2 / lambda_1 (measured 6e-9 here)
    assert L <= lam.max() * (1 + 1e-12)
    assert L == pytest.approx(lam.max(), rel=1e-7)
    beta = F.dirty_beam_peak(op)
    assert beta <= L * (1 + 1e-12)
    assert beta == pytest.approx(op.M, rel=1e-5)


def test_fb_scale_equivariance():
    op = _op(N=32, M=800, seed=32)
    xt = synth.sky(32, n_compact=5, n_ext=0) + 0.01
    y = op.phi(xt)
    L, _ = F.power_norm(op.phi_adj_phi, synth.power_start(32), rtol=1e-10)
    x1, _ = F.fb(op, y, L, 1e-3, 15)
    a = 37.5
    x2, _ = F.fb(op, a * y, L, a * 1e-3, 15)
    assert np.abs(x2 - a * x1).max() <= 1e-11 * a * np.abs(x1).max()


def test_fb_objective_monotone_with_exact_prox():
    # With Psi = I the composed prox is the exact prox of t||x||_1 + positivity, so
    # FB with gamma < 2/L decreases f + lambda r at every step.
    op = _op(N=32, M=800, seed=33)
    xt = synth.sky(32, n_compact=6, n_ext=0)
    y = op.phi(xt) + F.complex_noise(1e-3, synth.noise_normals(op.M, 2))
    L, _ = F.power_norm(op.phi_adj_phi, synth.power_start(32), rtol=1e-10)
    gamma = F.step_size(L)
    t = 0.05
    x = np.zeros((32, 32))
    prev = F.objective(op, x, y, t / gamma, levels=0)
    for _ in range(40):
        x, *_ = F.fb_step(op, x, y, gamma, lambda z: F.prox_haar_pos(z, t, levels=0))
        cur = F.objective(op, x, y, t / gamma, levels=0)
        assert cur <= prev * (1 + 1e-12)
        prev = cur


def test_noise_and_threshold_rules():
    phix = np.full(10000, 3.0 + 4.0j)               # ||Phi x|| / sqrt(M) = 5
    tau = F.tau_from_isnr(phix, 40.0)
    assert tau == pytest.approx(5.0 * 1e-2)
    n = F.complex_noise(tau, synth.noise_normals(200000, 2))
    assert np.mean(np.abs(n) ** 2) == pytest.approx(tau ** 2, rel=0.01)
    assert F.threshold(2.0, 8.0) == pytest.approx(0.5)
    assert F.sigma_from(2.0, 4.0, 8.0) == pytest.approx(0.125)
    assert F.alpha_rescale(10.0, 5.0, 2.0, 8.0, 1.0) == pytest.approx(2.0)
    assert F.alpha_rescale(10.0, 5.0, 2.0, 8.0, 0.01) == pytest.approx(50.0)
