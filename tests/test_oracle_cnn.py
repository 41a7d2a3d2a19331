"""Pins of the CNN oracle (no GPU): convolution against scipy, bfloat16
rounding against torch's conversion, analytic gradients against central
finite differences, facet exactness for a halo covering the receptive field."""
import numpy as np
import pytest
from scipy import signal

from oracle import cnn as C


def test_conv3x3_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 9, 11))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = C.conv3x3(x, w, b)
    for bi in range(2):
        for o in range(4):
            ref = b[o] + sum(signal.correlate2d(x[bi, c], w[o, c], mode="same", boundary="fill")
                             for c in range(3))
            assert np.abs(out[bi, o] - ref).max() <= 1e-12


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    a = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.uniform(-6, 6, 5000),
                        [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 0.0, 3e-39]])
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(C.bf16_round(a), ref)
    assert C.bf16_round(np.array([1 + 2 ** -8]))[0] == 1.0              # tie to even
    assert C.bf16_round(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6   # tie to even (up)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    params = C.init_params(layers=3, channels=4, seed=3)
    params = [(w, rng.standard_normal(b.shape) * 0.1) for w, b in params]
    z = rng.standard_normal((2, 8, 8))
    g = rng.standard_normal((2, 8, 8))

    def objective(ps):
        D, _ = C.forward(ps, z)
        return float(np.sum(g * (z - D)))          # sum(g * net(z))

    _, acts = C.forward(params, z)
    grads = C.backward(params, acts, g)
    eps = 1e-6
    for l, (w, b) in enumerate(params):
        for idx in [(0, 0, 0, 0), (w.shape[0] - 1, w.shape[1] - 1, 2, 1), (0, w.shape[1] - 1, 1, 2)]:
            wp = w.copy(); wp[idx] += eps
            wm = w.copy(); wm[idx] -= eps
            pp = list(params); pp[l] = (wp, b)
            pm = list(params); pm[l] = (wm, b)
            fd = (objective(pp) - objective(pm)) / (2 * eps)
            assert grads[l][0][idx] == pytest.approx(fd, rel=1e-6, abs=1e-9), (l, idx)
        j = b.shape[0] - 1
        bp = b.copy(); bp[j] += eps
        bm = b.copy(); bm[j] -= eps
        pp = list(params); pp[l] = (w, bp)
        pm = list(params); pm[l] = (w, bm)
        fd = (objective(pp) - objective(pm)) / (2 * eps)
        assert grads[l][1][j] == pytest.approx(fd, rel=1e-6, abs=1e-9), (l, "bias")


def test_l1_gradient():
    rng = np.random.default_rng(4)
    D = rng.standard_normal((2, 5, 5))
    u = rng.standard_normal((2, 5, 5))
    g = C.l1_dnet(D, u)
    eps = 1e-7
    for idx in [(0, 0, 0), (1, 4, 2)]:
        Dp = D.copy(); Dp[idx] -= eps       # net up by eps -> D down by eps
        Dm = D.copy(); Dm[idx] += eps
        fd = (C.l1_loss(Dp, u) - C.l1_loss(Dm, u)) / (2 * eps)
        assert g[idx] == pytest.approx(fd, rel=1e-6)


@pytest.mark.parametrize("bf16", [False, True])
def test_facets_with_receptive_halo_are_exact(bf16):
    rng = np.random.default_rng(5)
    layers = 4                                   # receptive radius 4
    params = C.init_params(layers=layers, channels=6, seed=6)
    params = [(w, rng.standard_normal(b.shape) * 0.2) for w, b in params]
    z = rng.standard_normal((32, 32))
    whole, _ = C.forward(params, z[None], bf16=bf16)
    fac = C.denoise_facets(params, z, core=16, halo=layers, bf16=bf16)
    assert np.abs(fac - whole[0]).max() <= (1e-12 if not bf16 else 0.0) + 1e-12
    # a halo below the receptive radius is not exact
    short = C.denoise_facets(params, z, core=16, halo=layers - 2, bf16=bf16)
    assert np.abs(short - whole[0]).max() > 1e-6


# ---------------------------------------------------------------------------
# Jacobian-vector products and the firm-nonexpansiveness norm
# ---------------------------------------------------------------------------
def _small_net(seed=3, layers=4, ch=8):
    rng = np.random.default_rng(seed)
    ps = C.init_params(layers, ch, seed=seed)
    return [(w, rng.standard_normal(b.shape) * 0.1) for w, b in ps]


def test_jvp_and_vjp_are_adjoint():
    ps = _small_net()
    rng = np.random.default_rng(1)
    z = rng.standard_normal((2, 12, 12))
    _, acts = C.forward(ps, z)
    v, u = rng.standard_normal(z.shape), rng.standard_normal(z.shape)
    lhs = float(np.sum(C.jvp(ps, acts, v) * u))
    rhs = float(np.sum(v * C.vjp(ps, acts, u)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_jvp_matches_central_differences():
    ps = _small_net(seed=5)
    rng = np.random.default_rng(2)
    z = rng.standard_normal((1, 12, 12))
    v = rng.standard_normal(z.shape)
    eps = 1e-6

    def net(x):
        D, _ = C.forward(ps, x)
        return x - D

    fd = (net(z + eps * v) - net(z - eps * v)) / (2 * eps)
    _, acts = C.forward(ps, z)
    jv = C.jvp(ps, acts, v)
    assert np.linalg.norm(jv - fd) <= 1e-6 * np.linalg.norm(fd)


@pytest.mark.parametrize("a", [0.8, 0.25, 2.0])
def test_fne_norm_closed_form(a):
    """A two-layer, one-channel network that passes z through its centre taps
    with an always-active ReLU is net(z) = a (z + 5): J_net = a I and
    ||I - 2 J_net||_S = |1 - 2a|."""
    w0 = np.zeros((1, 1, 3, 3)); w0[0, 0, 1, 1] = 1.0
    w1 = np.zeros((1, 1, 3, 3)); w1[0, 0, 1, 1] = a
    ps = [(w0, np.array([5.0])), (w1, np.array([0.0]))]
    z = np.random.default_rng(4).uniform(-1, 1, (1, 8, 8))
    assert C.fne_norm(ps, z, iters=5) == pytest.approx(abs(1 - 2 * a), rel=1e-12)


def test_fne_norm_of_a_dead_network_is_one():
    """All hidden pre-activations negative: J_net = 0 and ||I||_S = 1."""
    ps = _small_net(seed=7)
    ps = [(w, np.full(b.shape, -100.0) if l < len(ps) - 1 else b) for l, (w, b) in enumerate(ps)]
    z = np.random.default_rng(5).standard_normal((1, 8, 8))
    assert C.fne_norm(ps, z, iters=3) == pytest.approx(1.0, rel=1e-12)


def test_jvp_param_grad_matches_central_differences():
    """d(u^T J_net(z) v)/dW by central differences of the weights (FP64, away
    from ReLU kinks), and zero for the biases."""
    ps = _small_net(seed=9, layers=3, ch=4)
    rng = np.random.default_rng(6)
    z = rng.standard_normal((1, 8, 8))
    v, u = rng.standard_normal(z.shape), rng.standard_normal(z.shape)

    def f(params):
        _, acts = C.forward(params, z)
        return float(np.sum(u * C.jvp(params, acts, v)))

    _, acts = C.forward(ps, z)
    gr = C.jvp_param_grad(ps, acts, v, u)
    eps = 1e-6
    for l in range(len(ps)):
        w, b = ps[l]
        idx = [tuple(rng.integers(0, n) for n in w.shape) for _ in range(4)]
        for ix in idx:
            wp, wm = w.copy(), w.copy()
            wp[ix] += eps
            wm[ix] -= eps
            psp = [p if k != l else (wp, b) for k, p in enumerate(ps)]
            psm = [p if k != l else (wm, b) for k, p in enumerate(ps)]
            fd = (f(psp) - f(psm)) / (2 * eps)
            assert gr[l][0][ix] == pytest.approx(fd, rel=1e-5, abs=1e-8)
        bp = b.copy()
        bp[0] += 1e-3
        assert f([p if k != l else (w, bp) for k, p in enumerate(ps)]) == pytest.approx(f(ps), rel=1e-12)
        assert np.all(gr[l][1] == 0)


def test_adam_three_steps_by_hand():
    """Adam (beta1 0.9, beta2 0.999, eps 1e-8, lr 0.1) on a scalar from p = 1
    with gradients 0.5, -1, 2, worked by hand:
      t=1: m = 0.05, v = 0.00025, m^ = 0.5, v^ = 0.25,
           p = 1 - 0.1 * 0.5 / (0.5 + 1e-8) = 0.900000002;
      t=2: m = 0.045 - 0.1 = -0.055, v = 0.00024975 + 0.001 = 0.00124975,
           m^ = -0.055 / 0.19 = -0.2894736842, v^ = 0.00124975 / 0.001999 = 0.6251875938,
           p = 0.900000002 + 0.1 * 0.2894736842 / (0.7906886516 + 1e-8) = 0.9366103542;
      t=3: m = -0.0495 + 0.2 = 0.1505, v = 0.00124850025 + 0.004 = 0.00524850025,
           m^ = 0.1505 / 0.271 = 0.5553505535, v^ = 0.00524850025 / 0.002997001 = 1.7512507503,
           p = 0.9366103542 - 0.1 * 0.5553505535 / (1.3233483027 + 1e-8) = 0.8946447927."""
    p, m, v = np.array([1.0]), np.zeros(1), np.zeros(1)
    want = [0.900000002, 0.93661035424056560, 0.89464479271810477]
    for t, (g, w) in enumerate(zip((0.5, -1.0, 2.0), want), 1):
        p, m, v = C.adam_step(p, np.array([g]), m, v, t, 0.1)
        assert p[0] == pytest.approx(w, rel=1e-15, abs=1e-15)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias corrections give m^ = g and
    v^ = g^2 at every step, so each step moves p by exactly lr g / (|g| + eps);
    a missing or wrong correction (or a beta slip) breaks this at t >= 2."""
    rng = np.random.default_rng(3)
    g = rng.standard_normal(50) * 10.0 ** rng.uniform(-6, 2, 50)
    p0 = rng.standard_normal(50)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        p, m, v = C.adam_step(p, g, m, v, t, 1e-3)
        np.testing.assert_allclose(p, p0 - t * 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-13, atol=1e-16)
