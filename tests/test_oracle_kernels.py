"""Pins of the oracle's kernel functions and FFT against library routines and
closed forms (no GPU)."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import phi as O


def test_i0_matches_scipy():
    for x in [0.0, 1e-3, 0.5, 1.0, 3.75, 7.0, 12.0, 16.252239469813198, 30.0]:
        assert O.i0(x) == pytest.approx(float(special.i0(x)), rel=2e-15)


def test_kb_beta_beatty_closed_form():
    # Beatty et al. 2005 at J = 7, sigma = 2: pi sqrt((3.5 * 1.5)^2 - 0.8) = pi sqrt(26.7625)
    assert O.kb_beta(7, 2.0) == pytest.approx(math.pi * math.sqrt(26.7625), rel=1e-15)


def test_kb_values():
    beta = O.kb_beta()
    assert O.kb(0.0) == pytest.approx(1.0, rel=1e-15)
    assert O.kb(3.5) == pytest.approx(1.0 / float(special.i0(beta)), rel=1e-13)
    assert O.kb(-3.5) == O.kb(3.5)
    assert O.kb(3.5000001) == 0.0 and O.kb(-4.0) == 0.0
    for t in [0.3, 1.7, 2.9]:
        ref = float(special.i0(beta * math.sqrt(1 - (2 * t / 7) ** 2)) / special.i0(beta))
        assert O.kb(t) == pytest.approx(ref, rel=1e-13)
        assert O.kb(t) == O.kb(-t)


@pytest.mark.parametrize("nu", [0.0, 0.05, 0.125, 0.2, 0.25, 0.4, 0.9])
def test_kb_hat_matches_quadrature(nu):
    # kappa_hat(nu) = int kappa(t) exp(-2 pi i nu t) dt (kappa is even: cosine transform)
    val, err = integrate.quad(lambda t: O.kb(t) * math.cos(2 * math.pi * nu * t), -3.5, 3.5,
                              epsabs=1e-15, epsrel=1e-13, limit=200)
    assert O.kb_hat(nu) == pytest.approx(val, rel=1e-10, abs=1e-14)


@pytest.mark.parametrize("n", [8, 16, 64, 128, 512])
def test_fft1_matches_numpy(n):
    rng = np.random.default_rng(n)
    a = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = np.fft.fft(a)
    out = O.fft1(a, -1)
    assert np.linalg.norm(out - ref) <= 1e-13 * np.linalg.norm(ref)
    inv = O.fft1(a, +1)
    ref_inv = np.fft.ifft(a) * n
    assert np.linalg.norm(inv - ref_inv) <= 1e-13 * np.linalg.norm(ref_inv)


@pytest.mark.parametrize("n", [16, 64, 256])
def test_fft2_matches_numpy_and_parseval(n):
    rng = np.random.default_rng(100 + n)
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    out = O.fft2(a, -1)
    ref = np.fft.fft2(a)
    assert np.linalg.norm(out - ref) <= 1e-13 * np.linalg.norm(ref)
    assert np.linalg.norm(out) ** 2 == pytest.approx(n * n * np.linalg.norm(a) ** 2, rel=1e-13)
    back = O.fft2(out, +1) / (n * n)
    assert np.linalg.norm(back - a) <= 1e-13 * np.linalg.norm(a)
