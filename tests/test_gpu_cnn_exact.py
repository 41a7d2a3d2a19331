"""The CNN kernels against the oracle where no rounding can differ: a network
whose arithmetic is exact in FP32 whatever the summation order (appendix C's
denoiser and its training maps; the precision points of the GPU are those the
oracle reproduces with bf16=True).

Construction. Inputs, tangents and cotangents are multiples of 2^-4 with small
magnitudes; every weight is 0 or +-1 (exact in bfloat16), each hidden channel has four
non-zero taps and the output channel sixteen, biases are multiples of 2^-4. Then
every product is a multiple of 2^-4 (activations, tangents, pre-activation
gradients) or of 2^-8 (parameter gradients: an activation times a gradient),
and as long as the sum of the magnitudes of a sum's terms stays below 2^20
(resp. 2^16) every partial sum is an exact FP32 number, so MFMA and the
oracle's FP64 sums agree exactly; a bfloat16 rounding of an exact value is
the same on both sides (round to nearest even). The test checks these bounds
on the CPU before it compares.

Gates: forward, parameter gradients (ri_cnn_grad), the input gradient J^T u
(ri_cnn_vjp), the tangent J v (ri_cnn_jvp) and the firm-nonexpansiveness
penalty's parameter gradient (ri_cnn_jvp_grad) within 1e-6 relative l2 of the
oracle (they come out equal). Then three consecutive training steps
(ri_cnn_train_step, sigma = 0 so the data term is mean|D(u) - u| exactly)
against the oracle's Adam fed the oracle's own gradients: the first step's
gradients are exact, so the first update agrees to FP32 rounding (1e-6, against
the oracle's parameters rounded to FP32, the library's parameter type); after
it the parameters leave the dyadic grid and FP32 sums round, so steps two and
three are held to 1e-4 relative l2 on the parameter change (and the loss), which still
catches a wrong beta, a missing bias correction or a wrong step count (each
changes the update by tens of percent)."""
import numpy as np
import pytest

from _cases import rel
from oracle import cnn as OC

torch = pytest.importorskip("torch")
import paper_2207_11336_amd.ri as R  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
L, CH, B, H, W = 5, 64, 2, 32, 32


def _exact_net(seed):
    rng = np.random.default_rng(seed)
    params = []
    for l in range(L):
        ci = 1 if l == 0 else CH
        co = 1 if l == L - 1 else CH
        w = np.zeros((co, ci, 3, 3))
        if l == 0:
            w[:] = rng.choice([-1.0, 0.0, 0.0, 1.0], size=w.shape)
        else:
            k = 16 if l == L - 1 else 4
            for o in range(co):
                flat = rng.choice(ci * 9, size=k, replace=False)
                w[o].reshape(-1)[flat] = rng.choice([-1.0, 1.0], size=k)
        b = rng.integers(-4, 5, size=co) / 16.0
        params.append((w, b))
    return params


def _dyadic(shape, seed, lo, hi):
    return np.random.default_rng(seed).integers(lo, hi, size=shape) / 16.0


def _on_grid(a, q):
    return bool(np.all(np.abs(a * q - np.round(a * q)) == 0.0))


def _check_exact_forward(params, acts):
    """Every layer: activations on the 2^-4 grid, sum of |terms| < 2^20."""
    for l, (w, b) in enumerate(params):
        a = acts[l]
        assert _on_grid(a, 16), l
        bound = OC.conv3x3(np.abs(a), np.abs(w), np.abs(b))
        assert float(bound.max()) < 2.0 ** 20, (l, float(bound.max()))
    assert _on_grid(acts[-1], 16)


def _check_exact_backward(params, acts, g):
    """Pre-activation gradients on the 2^-4 grid (cotangents of 2^-4, integer
    weights); parameter gradient sums of |a g| below 2^16 (grid 2^-8)."""
    gg = g[:, None]
    for l in range(L - 1, -1, -1):
        w, _ = params[l]
        _, dw_abs, db_abs = OC.conv3x3_backward(np.abs(acts[l]), np.abs(w), np.abs(gg), need_dx=False)
        assert float(dw_abs.max()) < 2.0 ** 16 and float(db_abs.max()) < 2.0 ** 16, l
        if l > 0:
            dx, _, _ = OC.conv3x3_backward(acts[l], w, gg, need_dx=True)
            gg = dx * (acts[l] > 0)
            assert _on_grid(gg, 16), l


@pytest.fixture(scope="module")
def case():
    params = _exact_net(5)
    z = _dyadic((B, H, W), 6, 0, 32)          # [0, 2) on the 2^-4 grid
    g = _dyadic((B, H, W), 7, -8, 9)          # cotangent of net(z)
    v = _dyadic((B, H, W), 8, -8, 9)          # tangent
    u = _dyadic((B, H, W), 9, -8, 9)          # cotangent of J v
    _, acts = OC.forward(params, z, bf16=True)
    _check_exact_forward(params, acts)
    _check_exact_backward(params, acts, g)
    _check_exact_backward(params, acts, u)
    # tangents: integer weights keep them on the 2^-4 grid; bound their sums
    t = v[:, None]
    for l, (w, b) in enumerate(params):
        assert float(OC.conv3x3(np.abs(t), np.abs(w), 0 * b).max()) < 2.0 ** 20
        if l < L - 1:
            t = OC.conv3x3(t, w, 0 * b) * (acts[l + 1] > 0)
            assert _on_grid(t, 16)
    net = R.ri_cnn_create(layers=L, max_batch=B, max_h=H, max_w=W, training=True)
    R.ri_cnn_set_params(net, torch.tensor(OC.flatten_params(params), dtype=torch.float32, device=DEV))
    yield net, params, acts, z, g, v, u
    net.close()


def _t(a):
    return torch.tensor(a, dtype=torch.float32, device=DEV)


def test_exact_forward_gradients_and_jacobian_products(case):
    net, params, acts, z, g, v, u = case
    zt, gt, vt, ut = _t(z), _t(g), _t(v), _t(u)
    out = torch.empty_like(zt)
    R.ri_cnn_forward(net, zt, out)
    D_ref, _ = OC.forward(params, z, bf16=True)
    grads = torch.empty(net.n_params, dtype=torch.float32, device=DEV)
    R.ri_cnn_grad(net, zt, gt, grads)
    g_ref = OC.flatten_params(OC.backward(params, acts, g, bf16=True))
    jv = torch.empty_like(zt)
    R.ri_cnn_jvp(net, zt, vt, jv)
    jv_ref = OC.jvp(params, acts, v, bf16=True)
    jtu = torch.empty_like(zt)
    R.ri_cnn_vjp(net, zt, ut, jtu)
    jtu_ref = OC.vjp(params, acts, u, bf16=True)
    pg = torch.empty_like(grads)
    R.ri_cnn_jvp_grad(net, zt, vt, ut, pg)
    pg_ref = OC.flatten_params(OC.jvp_param_grad(params, acts, v, u, bf16=True))
    torch.cuda.synchronize()
    errs = {"forward": rel(out.cpu().numpy(), D_ref), "dW": rel(grads.cpu().numpy(), g_ref),
            "jvp": rel(jv.cpu().numpy(), jv_ref), "vjp (dX)": rel(jtu.cpu().numpy(), jtu_ref),
            "penalty grad": rel(pg.cpu().numpy(), pg_ref)}
    print("exact network: " + ", ".join(f"{k} {e:.1e}" for k, e in errs.items()))
    for k, e in errs.items():
        assert e <= 1e-6, (k, e)
    # the cases are not degenerate: every map has a sizeable non-zero output
    for ref in (D_ref - z, g_ref, jv_ref, jtu_ref, pg_ref):
        assert np.count_nonzero(ref) > 0.2 * ref.size


def test_three_adam_steps_against_oracle(case):
    _, params, _, z, _, _, _ = case
    net = R.ri_cnn_create(layers=L, max_batch=B, max_h=H, max_w=W, training=True)
    p0 = OC.flatten_params(params)
    R.ri_cnn_set_params(net, _t(p0))
    zt = _t(z)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    pg = torch.empty(net.n_params, dtype=torch.float32, device=DEV)
    lr = 1e-3
    p, m, vv = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for t in (1, 2, 3):
        # oracle: gradient of mean|D(u) - u| at its own parameters (sigma = 0), then Adam
        ps = OC.unflatten_params(p, params)
        D, acts = OC.forward(ps, z, bf16=True)
        gr = OC.flatten_params(OC.backward(ps, acts, OC.l1_dnet(D, z), bf16=True))
        loss_ref = OC.l1_loss(D, z)
        p, m, vv = OC.adam_step(p, gr, m, vv, t, lr)
        R.ri_cnn_train_step(net, zt, 0.0, 100 + t, lr, loss)
        R.ri_cnn_get_params(net, pg)
        torch.cuda.synchronize()
        got = pg.cpu().numpy().astype(np.float64)
        # the library keeps FP32 parameters: compare with the oracle's rounded to FP32
        # (near |p| = 1 one FP32 spacing is 6e-5 of a 1e-3 update)
        e = rel(got - p0, p.astype(np.float32).astype(np.float64) - p0)
        el = abs(loss.item() - loss_ref) / loss_ref
        print(f"Adam step {t}: parameter change rel {e:.2e}, loss {loss.item():.6e} vs {loss_ref:.6e}")
        assert el <= (1e-6 if t == 1 else 1e-4)
        assert e <= (1e-6 if t == 1 else 1e-4)
    net.close()
