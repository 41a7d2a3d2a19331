"""Pins of the uSARA oracle (section "uSARA's handcrafted denoiser") against
things other than itself: the closed forms of the first two Daubechies
filters, orthonormality and vanishing moments of all eight, the transforms'
perfect reconstruction, energy preservation and adjointness, one Haar level
against its closed form, Psi Psi^dagger = I, the prox against its closed form
for the Dirac basis alone and against an independent primal-dual solver for
the whole dictionary, and the reweighting rule."""
import math

import numpy as np
import pytest

import synth
from oracle import sara as S

R2 = math.sqrt(2.0)


def test_first_two_filters_closed_form():
    assert np.allclose(S.daubechies(1), [1 / R2, 1 / R2], atol=1e-15)
    r3 = math.sqrt(3.0)
    db2 = np.array([1 + r3, 3 + r3, 3 - r3, 1 - r3]) / (4 * R2)
    assert np.abs(S.daubechies(2) - db2).max() <= 1e-14


@pytest.mark.parametrize("p", range(1, 9))
def test_filter_orthonormality_and_vanishing_moments(p):
    h = S.daubechies(p)
    g = S.highpass(h)
    assert h.size == 2 * p
    assert abs(h.sum() - R2) <= 1e-13
    for m in range(p):
        dot = float(np.dot(h[2 * m:], h[: h.size - 2 * m]))
        assert abs(dot - (1.0 if m == 0 else 0.0)) <= 1e-12, (p, m, dot)
    t = np.arange(h.size, dtype=np.float64)
    for j in range(p):
        mom = float(np.dot(g, (t - t.mean()) ** j))
        assert abs(mom) <= 1e-10 * max(1.0, float(np.abs(t - t.mean()).max()) ** j), (p, j, mom)
    # minimum phase: the partial energy of the first taps is at least that of the reversed filter
    e = np.cumsum(h ** 2)
    er = np.cumsum(h[::-1] ** 2)
    assert np.all(e >= er - 1e-12)


@pytest.mark.parametrize("p", [1, 4, 8])
def test_transform_is_orthonormal(p):
    rng = np.random.default_rng(p)
    x = rng.standard_normal((64, 64))
    h = S.daubechies(p)
    c = S.dwt2(x, h)
    assert abs(np.linalg.norm(c) - np.linalg.norm(x)) <= 1e-12 * np.linalg.norm(x)
    assert np.abs(S.idwt2(c, h) - x).max() <= 1e-12
    d = rng.standard_normal((64, 64))
    assert abs(np.sum(c * d) - np.sum(x * S.idwt2(d, h))) <= 1e-11 * np.linalg.norm(x) * np.linalg.norm(d)


def test_haar_level_closed_form():
    """db1, one level: the 2x2 block averages and differences over sqrt(2)^2."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal((8, 8))
    c = S.dwt2(x, S.daubechies(1), levels=1)
    a, b, cc, d = x[0::2, 0::2], x[0::2, 1::2], x[1::2, 0::2], x[1::2, 1::2]
    assert np.allclose(c[:4, :4], (a + b + cc + d) / 2, atol=1e-15)       # low rows, low columns
    # high pass g = (h[1], -h[0]) = (1, -1)/sqrt2: differences even minus odd
    assert np.allclose(c[:4, 4:], (a - b + cc - d) / 2, atol=1e-15)
    assert np.allclose(c[4:, :4], (a + b - cc - d) / 2, atol=1e-15)
    assert np.allclose(c[4:, 4:], (a - b - cc + d) / 2, atol=1e-15)


@pytest.mark.parametrize("p", [2, 5, 8])
def test_details_vanish_on_polynomials(p):
    """One level along x of x^j (j < p): the detail coefficients away from the wrap are zero."""
    n = 128
    h = S.daubechies(p)
    for j in range(p):
        row = ((np.arange(n) - 40.0) / 40.0) ** j
        c = S.analysis(row[None, :], h, 1)[0]
        d = c[n // 2: n // 2 + (n - 2 * p) // 2]
        assert np.abs(d).max() <= 1e-9 * max(1.0, np.abs(row).max()), (p, j)


def test_dictionary_is_a_tight_frame():
    x = synth.sky(64, seed=2, n_compact=6, n_ext=1)
    s = S.Sara()
    c = s.adj(x)
    assert c.shape == (9, 64, 64)
    assert abs(np.linalg.norm(c) - np.linalg.norm(x)) <= 1e-12 * np.linalg.norm(x)
    assert np.abs(s.syn(c) - x).max() <= 1e-12 * np.abs(x).max()


def test_prox_dirac_closed_form():
    """Psi = I: the prox of t ||w x||_1 + iota_+ is max(0, z - t w)."""
    rng = np.random.default_rng(5)
    z = rng.standard_normal((32, 32))
    w = rng.uniform(0.2, 1.0, (1, 32, 32))
    s = S.Sara(bases=("dirac",))
    x, _ = s.prox(z, 0.3, w, n_sub=3)
    assert np.abs(x - np.maximum(0.0, z - 0.3 * w[0])).max() <= 1e-15


def _chambolle_pock(s, z, t, w, iters):
    """Independent solver of the same prox: primal-dual (Chambolle-Pock) on
    min ||x - z||^2/2 + iota_+(x) + t ||w . K x||_1 with K = Psi^dagger (||K|| = 1)."""
    tau = sig = 0.99
    x = np.maximum(z, 0.0)
    xb = x.copy()
    y = np.zeros((len(s.bases),) + z.shape)
    for _ in range(iters):
        y = np.clip(y + sig * s.adj(xb), -t * w, t * w)
        xn = np.maximum(0.0, (x - tau * s.syn(y) + tau * z) / (1.0 + tau))
        xb = 2 * xn - x
        x = xn
    return x


def test_prox_matches_primal_dual_solver():
    """A four-basis dictionary (Dirac, db1, db3, db8; normalised by 1/2) at two levels: the dual
    forward-backward prox and Chambolle-Pock reach the same minimiser."""
    rng = np.random.default_rng(7)
    s = S.Sara(bases=("dirac", "db1", "db3", "db8"), levels=2)
    z = np.where(rng.uniform(size=(16, 16)) < 0.1, 1.0, 0.0) + 0.05 * rng.standard_normal((16, 16))
    w = rng.uniform(0.3, 1.0, (4, 16, 16))
    t = 0.02
    x, _ = s.prox(z, t, w, n_sub=800)
    ref = _chambolle_pock(s, z, t, w, 1000)
    obj = lambda u: 0.5 * np.sum((u - z) ** 2) + t * np.sum(w * np.abs(s.adj(u)))  # noqa: E731
    assert np.abs(x - ref).max() <= 1e-8 * np.abs(z).max()
    assert abs(obj(x) - obj(ref)) <= 1e-10 * obj(ref)
    assert x.min() >= 0.0
    assert np.abs(x - np.maximum(z, 0.0)).max() > 1e-3     # the penalty is active


def test_reweighting_rule_and_logsum_majorant():
    """w = rho / (rho + |Psi^dagger x|) is the slope of rho log(1 + |c| / rho) at x: the weighted-l1
    majorant touches the log-sum at x and lies above it at another point."""
    s = S.Sara()
    x = synth.sky(32, seed=6, n_compact=4, n_ext=1)
    rho = 0.01
    w = s.reweight(x, rho)
    c = s.adj(x)
    assert np.all((w > 0) & (w <= 1))
    assert np.allclose(w, 1.0 / (1.0 + np.abs(c) / rho), rtol=1e-15)
    u = x + 0.05 * synth.random_image(32, 8)
    maj = s.logsum(x, rho) + np.sum(w * (np.abs(s.adj(u)) - np.abs(c)))
    assert s.logsum(u, rho) <= maj + 1e-12
