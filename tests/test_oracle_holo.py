"""Pins of the holographic-matrix oracle (appendix E: Phi^dagger Phi =
Z^dagger F^dagger (sum_p H_p) F Z with H_p = G_p^H G_p) against things other
than itself: the operator oracle's Re{Phi^dagger Phi} (pinned by the
brute-force direct model), a closed form for one visibility on a grid node,
the per-block sum, the band the GPU storage relies on, Hermitian symmetry and
positivity, and the blindness to M."""
import math

import numpy as np
import pytest

import synth
from oracle import holo as HO
from oracle import phi as OP

pytestmark = pytest.mark.filterwarnings("ignore")
N = 32
CELL = 60 * synth.ARCSEC


def _W(hex_cells, n=N):
    return 2 * hex_cells / (2.0 * n * n * CELL ** 2)


@pytest.fixture(scope="module")
def case():
    W = _W(4.0)
    uvw = synth.random_uvw(400, 0.9 * math.pi, W, seed=5)
    op = OP.Operator(N, uvw, cell=CELL, W=W, n_wplanes=65)
    return op, HO.holographic(op)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_normal_is_phi_adjoint_phi(case):
    op, H = case
    x = synth.sky(N, seed=3, n_compact=6, n_ext=1) + 0.1 * synth.random_image(N, 4)
    assert _rel(HO.normal(op, H, x), op.phi_adj_phi(x)) <= 1e-12


def test_band_symmetry_and_positivity(case):
    op, H = case
    hmax_used = int(op.plane_h[op.plane].max())
    assert hmax_used == 5
    by, bx = HO.band(H, op.Np)
    assert by == bx == 2 * hmax_used + 6
    assert abs(H - H.conj().T).max() == 0.0
    rng = np.random.default_rng(8)
    X = rng.standard_normal((op.Np, op.Np)) + 1j * rng.standard_normal((op.Np, op.Np))
    q = np.vdot(X.ravel(), HO.apply(H, X).ravel())
    gx = HO.g_matrix(op) @ X.ravel()
    assert abs(q.imag) <= 1e-12 * abs(q.real)
    assert q.real == pytest.approx(np.vdot(gx, gx).real, rel=1e-12)


def test_one_visibility_on_a_grid_node():
    """w = 0 and p on a grid node: G's row is the Kaiser-Bessel outer product
    kappa(3 - a_y) kappa(3 - a_x) on the 7 x 7 window around the node, so
    H = g g^T with those weights, zero elsewhere."""
    n = 16
    Np = 2 * n
    cu, cv = 5, 29
    uvw = np.array([[cu * 2 * math.pi / Np, (cv - Np) * 2 * math.pi / Np, 0.0]])
    op = OP.Operator(n, uvw)
    H = HO.holographic(op).toarray()
    k = np.array([OP.kb(3.0 - a) for a in range(7)])
    g = np.zeros((Np, Np))
    for ay in range(7):
        for ax in range(7):
            g[(cv + ay - 3) % Np, (cu + ax - 3) % Np] = k[ay] * k[ax]
    ref = np.outer(g.ravel(), g.ravel())
    assert np.abs(H - ref).max() <= 1e-14 * np.abs(ref).max()


def test_block_sum(case):
    """sum_p G_p^H G_p over contiguous blocks equals H of the whole data (eq. E2)."""
    op, H = case
    offs = [0, 90, 250, 400]
    Hs = sum(HO.holographic(op.subset(np.arange(offs[b], offs[b + 1]))) for b in range(3))
    assert abs(Hs - H).max() <= 1e-14 * abs(H).max()


def test_blind_to_the_number_of_visibilities(case):
    """Repeating every visibility doubles H and leaves its pattern: the
    matrix's size follows the coverage, not M."""
    op, H = case
    op2 = OP.Operator(N, np.concatenate([op.uvw, op.uvw]), cell=op.cell, W=op.W, n_wplanes=op.n_wplanes)
    H2 = HO.holographic(op2)
    assert H2.nnz == H.nnz
    assert abs(H2 - 2 * H).max() <= 1e-14 * abs(H).max()
