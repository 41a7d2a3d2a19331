"""The network's Jacobian on the GPU (appendix C: the firm-nonexpansiveness
condition ||J_{2D - I}||_S <= 1 of the training loss, measured here): the
Jacobian-vector products against the FP64 oracle emulating the GPU's
bfloat16 rounding, their adjoint identity, the power-iteration norm against
the oracle's and against a closed form."""
import numpy as np
import pytest

import synth
from _cases import rel
from oracle import cnn as OC

torch = pytest.importorskip("torch")
import paper_2207_11336_amd.ri as R  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
L = 10


def _net(seed=31):
    rng = np.random.default_rng(seed)
    ps = OC.init_params(L, 64, seed=seed)
    ps = [(w, rng.standard_normal(b.shape) * 0.05) for w, b in ps]
    vec = np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in ps]).astype(np.float32)
    ps32 = [(w.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for w, b in ps]
    net = R.ri_cnn_create(layers=L, max_batch=2, max_h=64, max_w=64, training=True)
    R.ri_cnn_set_params(net, torch.tensor(vec, device=DEV))
    return net, ps32


def _inputs(B=2, h=32, w=48, seed=4):
    rng = np.random.default_rng(seed)
    z = np.stack([synth.sky(64, seed=seed + i)[:h, :w] for i in range(B)])
    z = (z / z.max() + 0.05 * rng.standard_normal(z.shape)).astype(np.float32)
    v = rng.standard_normal(z.shape).astype(np.float32)
    u = rng.standard_normal(z.shape).astype(np.float32)
    return z, v, u


def test_jvp_vjp_match_oracle_and_are_adjoint():
    net, ps = _net()
    z, v, u = _inputs()
    zt, vt, ut = (torch.tensor(a, device=DEV) for a in (z, v, u))
    jv, ju = torch.empty_like(zt), torch.empty_like(zt)
    R.ri_cnn_jvp(net, zt, vt, jv)
    R.ri_cnn_vjp(net, zt, ut, ju)
    _, acts = OC.forward(ps, z.astype(np.float64), bf16=True)
    ref_jv = OC.jvp(ps, acts, v.astype(np.float64), bf16=True)
    ref_ju = OC.vjp(ps, acts, u.astype(np.float64), bf16=True)
    e_jv, e_ju = rel(jv.cpu().numpy(), ref_jv), rel(ju.cpu().numpy(), ref_ju)
    lhs = float(torch.sum(jv.double() * ut.double()))
    rhs = float(torch.sum(vt.double() * ju.double()))
    e_adj = abs(lhs - rhs) / abs(lhs)
    print(f"JVP rel {e_jv:.2e}, VJP rel {e_ju:.2e} against the bf16-emulating oracle; <Jv,u> vs <v,J^T u> {e_adj:.2e}")
    # signed tangents: ReLU masks that flip under rounding differences are
    # amplified by cancellation, as for the signed parameter gradients
    assert e_jv <= 8e-2 and e_ju <= 8e-2
    assert e_adj <= 2e-2


def test_fne_norm_matches_oracle():
    net, ps = _net(seed=32)
    z, _, _ = _inputs(B=1, h=32, w=32, seed=9)
    s_gpu = R.ri_cnn_fne_norm(net, torch.tensor(z, device=DEV), iters=40, seed=3)
    s_ref = OC.fne_norm(ps, z.astype(np.float64), iters=40, seed=3, bf16=True)
    print(f"||I - 2 J_net||_S: GPU {s_gpu:.5f}, oracle {s_ref:.5f}")
    assert s_gpu == pytest.approx(s_ref, rel=2e-2)


@pytest.mark.parametrize("a", [0.75, 2.0])
def test_fne_norm_closed_form(a):
    """Channel 0 carries z + 5 through centre taps with always-active ReLUs,
    the other 63 channels are dead (negative bias): net(z) = a (z + 5), so
    J_net = a I and ||I - 2 J_net||_S = |1 - 2a| (a exact in bfloat16)."""
    ps = []
    for l in range(L):
        ci = 1 if l == 0 else 64
        co = 1 if l == L - 1 else 64
        w = np.zeros((co, ci, 3, 3))
        b = np.zeros(co)
        if l == 0:
            w[0, 0, 1, 1] = 1.0
            b[:] = -1.0
            b[0] = 5.0
        elif l < L - 1:
            w[0, 0, 1, 1] = 1.0
            b[1:] = -1.0
        else:
            w[0, 0, 1, 1] = a
        ps.append((w, b))
    vec = np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in ps]).astype(np.float32)
    net = R.ri_cnn_create(layers=L, max_batch=1, max_h=32, max_w=32, training=True)
    R.ri_cnn_set_params(net, torch.tensor(vec, device=DEV))
    z = torch.tensor(np.random.default_rng(2).uniform(-1, 1, (1, 32, 32)).astype(np.float32), device=DEV)
    s = R.ri_cnn_fne_norm(net, z, iters=10, seed=5)
    print(f"a = {a}: ||I - 2 J_net||_S = {s:.5f} (closed form {abs(1 - 2 * a):.5f})")
    assert s == pytest.approx(abs(1 - 2 * a), rel=1e-2)


def test_jvp_param_grad_matches_oracle():
    """d(u^T J_net(z) v)/d params (the penalty's gradient pass: the parameter
    gradient pass fed with the tangents of v) against the oracle."""
    net, ps = _net(seed=33)
    z, _, _ = _inputs(B=2, h=32, w=32, seed=13)
    rng = np.random.default_rng(14)
    v = rng.uniform(0, 1, z.shape).astype(np.float32)
    u = rng.uniform(0, 1, z.shape).astype(np.float32)
    grads = torch.empty(net.n_params, dtype=torch.float32, device=DEV)
    R.ri_cnn_jvp_grad(net, torch.tensor(z, device=DEV), torch.tensor(v, device=DEV), torch.tensor(u, device=DEV),
                      grads)
    _, acts = OC.forward(ps, z.astype(np.float64), bf16=True)
    ref = OC.jvp_param_grad(ps, acts, v.astype(np.float64), u.astype(np.float64), bf16=True)
    g = grads.cpu().numpy().astype(np.float64)
    off = 0
    errs = []
    for l, (w, b) in enumerate(ref):
        gw = g[off:off + w.size].reshape(w.shape)
        off += w.size
        gb = g[off:off + b.size]
        off += b.size
        assert np.all(gb == 0.0)
        errs.append(rel(gw, w))
    print("d(u^T J v)/dW per layer, rel:", " ".join(f"{e:.1e}" for e in errs))
    assert max(errs) <= 3e-2


@pytest.mark.parametrize("point", [R.RI_FNE_AT_INPUT, R.RI_FNE_AT_MIX], ids=["at-input", "at-mix"])
def test_penalty_lowers_the_jacobian_norm(point):
    """The relaxed firm-nonexpansiveness penalty (lambda 1e-3, every fourth
    step, four warm-started power iterations), with the Jacobian taken at the
    noisy inputs or at random points between the clean and the denoised
    images, lowers ||J_{2D - I}||_S of the trained network on held-out noisy
    patches."""
    from paper_2207_11336_amd.train import train_denoiser
    sig = 1e-2
    patches = torch.tensor(synth.training_patches(512, 64, seed=synth.SEED_TRAIN), device=DEV)
    test = synth.training_patches(4, 64, seed=98)
    noisy = torch.tensor((test + sig * np.random.default_rng(6).standard_normal(test.shape)).astype(np.float32),
                         device=DEV)
    norms = {}
    for lam in (0.0, 1e-3):
        params, _ = train_denoiser(patches, sig, steps=1500, batch=16, lr=1e-3, lr_min=1e-5, fne_lambda=lam,
                                   fne_iters=4, fne_every=4, fne_point=point)
        net = R.ri_cnn_create(layers=L, max_batch=4, max_h=64, max_w=64, training=True)
        R.ri_cnn_set_params(net, params)
        norms[lam] = R.ri_cnn_fne_norm(net, noisy, iters=30, seed=3)
        net.close()
    print(f"||J_(2D-I)||_S on held-out noisy patches: plain l1 {norms[0.0]:.3f}, with the penalty {norms[1e-3]:.3f} "
          f"(point {point})")
    assert norms[1e-3] < 0.85 * norms[0.0]
