"""Pins of the w-stacking oracle (appendix E: per-stack phase screen in Z_p,
residual w carried by the w-kernel in G_p) against things other than itself:
the unstacked oracle (P = 1 must reduce to it), the brute-force direct model
(visibilities at stack centres leave only the interpolation error), the
adjoint identity, and the stack assignment rule."""
import math

import numpy as np
import pytest

import synth
from oracle import phi as OP
from oracle import wstack as WS

pytestmark = pytest.mark.filterwarnings("ignore")
N = 64
CELL = 60 * synth.ARCSEC


def _W(hex_cells):
    """w bound at which the paraxial chirp's half-bandwidth at the image edge is hex_cells grid cells."""
    return 2 * hex_cells / (2.0 * N * N * CELL ** 2)


def _sky():
    return synth.sky(N, seed=1, n_compact=8, n_ext=1) + 0.1 * synth.random_image(N, 3)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_one_stack_is_the_unstacked_operator():
    W = _W(4.0)
    uvw = synth.random_uvw(500, 2.0, W, seed=9)
    a = OP.Operator(N, uvw, cell=CELL, W=W, n_wplanes=129)
    b = WS.StackedOperator(N, uvw, CELL, W, 129, 1)
    x = _sky()
    r = np.random.default_rng(4).standard_normal(500) + 1j * np.random.default_rng(5).standard_normal(500)
    assert _rel(b.phi(x), a.phi(x)) <= 1e-14
    assert _rel(b.phi_adj(r), a.phi_adj(r)) <= 1e-14


def test_adjoint_identity():
    W = _W(8.0)
    uvw = synth.random_uvw(700, 2.0, W, seed=11)
    so = WS.StackedOperator(N, uvw, CELL, W, 129, 4)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((N, N))
    y = rng.standard_normal(700) + 1j * rng.standard_normal(700)
    lhs = np.vdot(so.phi(x), y).real
    rhs = float(np.sum(x * so.phi_adj(y)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_phase_screen_is_the_direct_models_w_phase():
    """A one-pixel image seen at omega = 0 by the direct model is the pixel's w-phase."""
    W = _W(8.0)
    w = 0.7 * W
    scr = WS.phase_screen(N, CELL, w)
    for (iy, ix) in [(N // 2, N // 2), (0, 0), (5, 50), (N - 1, 17)]:
        x = np.zeros((N, N))
        x[iy, ix] = 1.0
        y = OP.Operator(N, np.array([[0.0, 0.0, w]]), cell=CELL, W=W, n_wplanes=3).dft(x)
        assert abs(y[0] - scr[iy, ix]) <= 1e-13
    assert abs(scr[N // 2, N // 2] - 1.0) == 0.0
    assert np.allclose(np.abs(scr), 1.0, atol=1e-15)


def test_stack_assignment_and_residuals():
    W, P = 1000.0, 4
    w = np.linspace(-W, W, 10001)
    s = WS.stack_of(w, W, P)
    c = WS.stack_centres(W, P)
    assert np.array_equal(c, np.array([-750.0, -250.0, 250.0, 750.0]))
    assert s[0] == 0 and s[-1] == P - 1
    assert np.all(np.abs(w - c[s]) <= W / P + 1e-9)
    assert np.all(np.diff(s) >= 0)


@pytest.mark.parametrize("hex_cells", [4.0, 16.0])
def test_visibilities_at_stack_centres_match_the_direct_model(hex_cells):
    """With every w at a stack centre the residual w-kernel is the identity and
    the phase screen is exact (non-paraxial): only the Kaiser-Bessel
    interpolation error remains, while w-projection alone carries the whole
    w-term with its paraxial, truncated kernel."""
    W, P = _W(hex_cells), 4
    rng = np.random.default_rng(8)
    uvw = synth.random_uvw(600, 0.95 * 2 * math.pi / 3, W, seed=7)
    uvw[:, 2] = WS.stack_centres(W, P)[rng.integers(0, P, 600)]
    x = _sky()
    exact = OP.Operator(N, uvw, cell=CELL, W=W, n_wplanes=257)
    yt = exact.dft(x)
    e_stack = _rel(WS.StackedOperator(N, uvw, CELL, W, 257, P).phi(x), yt)
    e_proj = _rel(exact.phi(x), yt)
    assert e_stack <= 1e-5
    assert e_proj >= 100 * e_stack


def test_stacking_keeps_accuracy_beyond_the_largest_w_kernel():
    """At a w range whose chirp needs supports far beyond 17 x 17, w-projection
    alone fails (its kernel is capped) while four stacks keep the error at the
    level of the residual's paraxial w-kernel."""
    W = _W(16.0)
    uvw = synth.random_uvw(600, 0.95 * 2 * math.pi / 3, W, seed=7)
    x = _sky()
    exact = OP.Operator(N, uvw, cell=CELL, W=W, n_wplanes=257)
    yt = exact.dft(x)
    e_proj = _rel(exact.phi(x), yt)
    e_stack = _rel(WS.StackedOperator(N, uvw, CELL, W, 257, 4).phi(x), yt)
    assert e_proj > 0.1
    assert e_stack < 1e-2
    assert e_stack < e_proj / 20
