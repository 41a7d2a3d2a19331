"""GPU parity of the residual CNN denoiser (forward, parameter gradients,
training step, facet-wise application, PnP step and solve) against the FP64
oracle in oracle/cnn.py, through the C ABI (ri_cnn_* and the imaging
context's denoise / fb_step / pnp_solve with RI_PROX_CNN).

Tolerances. The oracle with bf16=True rounds to bfloat16 at the same points as
the GPU (hidden weights, hidden activations, hidden pre-activation gradients)
and accumulates exactly; the GPU accumulates in FP32 (MFMA). An FP32
accumulation error of ~1e-6 relative flips a bfloat16 rounding (spacing 2^-8)
with probability ~5e-4 per value, and a flip changes that value by 2^-8; so
the network output net(z) = z - D(z) agrees to 3e-4 .. 3e-3 in relative l2
(observed; the flips propagate through nine layers, more of them where many
activations sit near a ReLU kink), bounded at 5e-3. Gradient bounds are
derived in test_grad_matches_oracle."""
import math

import numpy as np
import pytest

import synth
from _cases import rel, wide
from oracle import cnn as OC
from oracle import fb as OF

torch = pytest.importorskip("torch")
import paper_2207_11336_amd.ri as R  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
LAYERS = 10


def _params_to_list(vec: np.ndarray, layers: int, ch: int = 64):
    """FP32 parameter vector (per layer W[co][ci][3][3] then b[co]) -> oracle list."""
    out, o = [], 0
    for l in range(layers):
        ci = 1 if l == 0 else ch
        co = 1 if l == layers - 1 else ch
        w = vec[o:o + co * ci * 9].reshape(co, ci, 3, 3).astype(np.float64)
        o += co * ci * 9
        b = vec[o:o + co].astype(np.float64)
        o += co
        out.append((w, b))
    assert o == vec.size
    return out


def _list_to_params(params) -> np.ndarray:
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params]).astype(np.float32)


def _trained_like_params(seed=11):
    """He-normal weights with small random biases (so that every bias path is exercised)."""
    rng = np.random.default_rng(seed)
    ps = OC.init_params(LAYERS, 64, seed=seed)
    return [(w, rng.standard_normal(b.shape) * 0.05) for w, b in ps]


def _images(B, h, w, seed):
    """Sky-like images: positive compact sources and smooth structure, peak 1."""
    out = np.empty((B, h, w))
    for b in range(B):
        n = max(h, w, 64)
        s = synth.sky(n, seed=seed + b, n_compact=8, n_ext=1)[:h, :w]
        out[b] = s / max(s.max(), 1e-12)
    return out


def _net_out(z, D):
    return z - D


def test_param_count_and_roundtrip():
    net = R.ri_cnn_create(layers=LAYERS, max_batch=1, max_h=32, max_w=32, seed=3)
    assert net.n_params == 576 + 64 + 8 * (36864 + 64) + 576 + 1
    p = torch.tensor(_list_to_params(_trained_like_params()), device=DEV)
    R.ri_cnn_set_params(net, p)
    q = torch.empty_like(p)
    R.ri_cnn_get_params(net, q)
    torch.cuda.synchronize()
    assert torch.equal(p, q)


def test_init_is_he_normal():
    net = R.ri_cnn_create(layers=LAYERS, max_batch=1, max_h=32, max_w=32, seed=5)
    q = torch.empty(net.n_params, dtype=torch.float32, device=DEV)
    R.ri_cnn_get_params(net, q)
    ps = _params_to_list(q.cpu().numpy(), LAYERS)
    for l, (w, b) in enumerate(ps):
        ci = 1 if l == 0 else 64
        assert np.all(b == 0)
        std = math.sqrt(2.0 / (9 * ci))
        assert abs(w.std() / std - 1) < (0.2 if w.size < 1000 else 0.03), l
        assert abs(w.mean()) < 4 * std / math.sqrt(w.size)


@pytest.mark.parametrize("B,h,w", [(1, 16, 16), (2, 48, 32), (3, 32, 80)])
def test_forward_matches_oracle(B, h, w):
    ps = _trained_like_params()
    net = R.ri_cnn_create(layers=LAYERS, max_batch=4, max_h=64, max_w=96, seed=0)
    R.ri_cnn_set_params(net, torch.tensor(_list_to_params(ps), device=DEV))
    z = _images(B, h, w, seed=20) + 0.01 * np.random.default_rng(1).standard_normal((B, h, w))
    zt = torch.tensor(z, dtype=torch.float32, device=DEV)
    out = torch.empty_like(zt)
    R.ri_cnn_forward(net, zt, out)
    D = out.cpu().numpy().astype(np.float64)
    z32 = zt.cpu().numpy().astype(np.float64)
    ps32 = [(w_.astype(np.float32).astype(np.float64), b_.astype(np.float32).astype(np.float64)) for w_, b_ in ps]
    Dref, _ = OC.forward(ps32, z32, bf16=True)
    e_bf = rel(_net_out(z32, D), _net_out(z32, Dref))
    Dfull, _ = OC.forward(ps32, z32, bf16=False)
    e_full = rel(_net_out(z32, D), _net_out(z32, Dfull))
    print(f"B{B} {h}x{w}: net rel err vs bf16 oracle {e_bf:.2e}, vs FP64 oracle {e_full:.2e}")
    assert e_bf <= 5e-3
    assert e_full <= 5e-2


@pytest.mark.parametrize("g_kind,tol", [("positive", 5e-3), ("signed", 8e-2)])
def test_grad_matches_oracle(g_kind, tol):
    """Parameter gradients against the oracle's backward on the oracle's own
    activations. With a positive g the per-channel sums over pixels hardly
    cancel and the bound is the rounding one. With a zero-mean g they cancel
    to ~sqrt(#pixels) of a term, and the few activations that sit within the
    forward pass's rounding difference of a ReLU kink (~1e-3 of them) switch
    a whole term on one side only: that sets a bound of a few 1e-2 on the
    relative error of the sums, independent of the kernels' arithmetic."""
    ps = _trained_like_params(seed=12)
    B, h, w = 2, 32, 48
    net = R.ri_cnn_create(layers=LAYERS, max_batch=B, max_h=h, max_w=w, training=True)
    R.ri_cnn_set_params(net, torch.tensor(_list_to_params(ps), device=DEV))
    rng = np.random.default_rng(7)
    z = _images(B, h, w, seed=30) + 0.02 * rng.standard_normal((B, h, w))
    g = 1.0 + rng.uniform(0.0, 0.5, (B, h, w)) if g_kind == "positive" else rng.standard_normal((B, h, w))
    zt = torch.tensor(z, dtype=torch.float32, device=DEV)
    gt = torch.tensor(g, dtype=torch.float32, device=DEV)
    grads = torch.empty(net.n_params, dtype=torch.float32, device=DEV)
    R.ri_cnn_grad(net, zt, gt, grads)
    got = _params_to_list(grads.cpu().numpy(), LAYERS)
    ps32 = [(w_.astype(np.float32).astype(np.float64), b_.astype(np.float32).astype(np.float64)) for w_, b_ in ps]
    _, acts = OC.forward(ps32, zt.cpu().numpy().astype(np.float64), bf16=True)
    ref = OC.backward(ps32, acts, gt.cpu().numpy().astype(np.float64), bf16=True)
    worst = 0.0
    for l in range(LAYERS):
        ew, eb = rel(got[l][0], ref[l][0]), rel(got[l][1], ref[l][1])
        print(f"{g_kind} g, layer {l}: dW rel {ew:.2e}  db rel {eb:.2e}")
        worst = max(worst, ew, eb)
    assert worst <= tol


def test_train_step_is_adam_on_the_l1_gradient():
    """sigma = 0: one step must equal p - lr * g / (|g| + eps) (first Adam step) with
    g the gradient of mean|D(u) - u|, and the reported loss that mean."""
    ps = _trained_like_params(seed=13)
    B, h, w = 2, 32, 32
    net = R.ri_cnn_create(layers=LAYERS, max_batch=B, max_h=h, max_w=w, training=True)
    p0 = torch.tensor(_list_to_params(ps), device=DEV)
    R.ri_cnn_set_params(net, p0)
    u = torch.tensor(_images(B, h, w, seed=40), dtype=torch.float32, device=DEV)
    D = torch.empty_like(u)
    R.ri_cnn_forward(net, u, D)
    Dn, un = D.cpu().numpy().astype(np.float64), u.cpu().numpy().astype(np.float64)
    gnet = torch.tensor(OC.l1_dnet(Dn, un), dtype=torch.float32, device=DEV)
    grads = torch.empty_like(p0)
    R.ri_cnn_grad(net, u, gnet, grads)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    lr = 1e-3
    R.ri_cnn_train_step(net, u, 0.0, 1, lr, loss)
    p1 = torch.empty_like(p0)
    R.ri_cnn_get_params(net, p1)
    torch.cuda.synchronize()
    gg = grads.cpu().numpy().astype(np.float64)
    want = p0.cpu().numpy().astype(np.float64) - lr * gg / (np.abs(gg) + 1e-8)
    assert np.abs(p1.cpu().numpy() - want).max() <= 1e-6
    assert loss.item() == pytest.approx(OC.l1_loss(Dn, un), rel=1e-9)


def test_training_reduces_the_loss():
    B, h, w = 8, 64, 64
    net = R.ri_cnn_create(layers=LAYERS, max_batch=B, max_h=h, max_w=w, training=True, seed=21)
    u = torch.tensor(_images(B, h, w, seed=50), dtype=torch.float32, device=DEV)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    hist = []
    for it in range(60):
        R.ri_cnn_train_step(net, u, 0.05, 1000 + it, 1e-3, loss)
        hist.append(loss.item())
    print("loss", hist[:3], hist[-3:])
    assert all(np.isfinite(hist))
    assert np.mean(hist[-10:]) < 0.8 * np.mean(hist[:5])


def _ctx(c, prec, core, halo, mode=R.RI_G_OTF):
    d = R.plan_desc(c.N, c.M, cell_rad=c.cell, w_max=c.W, n_wplanes=c.n_wplanes, precision=prec, g_mode=mode,
                    facet_core=core, facet_halo=halo)
    return R.ri_create(d, c.uvw)


@pytest.mark.parametrize("prec", [32, 64])
def test_facets_equal_whole_image_and_oracle(prec):
    c = wide()
    ps = _trained_like_params(seed=14)
    pv = torch.tensor(_list_to_params(ps), device=DEV)
    dt = torch.float32 if prec == 32 else torch.float64
    z = c.x / c.x.max() + 0.01 * np.random.default_rng(3).standard_normal((c.N, c.N))
    zt = torch.tensor(z, dtype=dt, device=DEV)
    outs = {}
    for core, halo in [(0, 0), (64, 10), (48, 16)]:
        ctx = _ctx(c, prec, core, halo)
        R.ri_load_denoiser(ctx, pv, LAYERS)
        o = torch.full_like(zt, float("nan"))
        R.denoise(ctx, zt, o, R.RI_PROX_CNN, 0.0)
        outs[(core, halo)] = o.cpu().numpy()
    whole = outs[(0, 0)]
    assert np.isfinite(whole).all()
    for k, v in outs.items():
        print(f"facets {k}: max |diff| vs whole image {np.abs(v - whole).max():.3e}")
        assert np.array_equal(v, whole), k       # halo >= receptive radius 10: exact
    z32 = zt.cpu().numpy().astype(np.float32).astype(np.float64)
    ps32 = [(w_.astype(np.float32).astype(np.float64), b_.astype(np.float32).astype(np.float64)) for w_, b_ in ps]
    ref = OC.denoise_facets(ps32, z32, core=64, halo=10, bf16=True)
    e = rel(z32 - whole, z32 - ref)
    print(f"prec {prec}: facet denoiser net rel err vs oracle {e:.2e}")
    assert e <= 5e-3


def test_short_halo_is_not_exact_but_close():
    c = wide()
    pv = torch.tensor(_list_to_params(_trained_like_params(seed=15)), device=DEV)
    z = torch.tensor(c.x / c.x.max(), dtype=torch.float32, device=DEV)
    res = {}
    for core, halo in [(0, 0), (64, 4)]:
        ctx = _ctx(c, 32, core, halo)
        R.ri_load_denoiser(ctx, pv, LAYERS)
        o = torch.empty_like(z)
        R.denoise(ctx, z, o, R.RI_PROX_CNN, 0.0)
        res[halo] = o.cpu().numpy()
    d = np.abs(res[4] - res[0])
    assert d.max() > 0
    # pixels farther than the receptive radius from every facet seam are unaffected
    assert np.all(d[16:48, 16:48] == 0)


@pytest.mark.parametrize("prec", [32, 64])
def test_pnp_fb_step_matches_oracle(prec):
    c = wide()
    ps = _trained_like_params(seed=16)
    ctx = _ctx(c, prec, 64, 16)
    R.ri_load_denoiser(ctx, torch.tensor(_list_to_params(ps), device=DEV), LAYERS)
    dt = torch.float32 if prec == 32 else torch.float64
    cdt = torch.complex64 if prec == 32 else torch.complex128
    L = float(c.M) * 1.5
    gamma = 1.98 / L
    alpha = c.x.max()
    x = np.clip(c.x / alpha + 0.01 * c.xr, 0, None)
    y = c.y / alpha
    xo = torch.empty((c.N, c.N), dtype=dt, device=DEV)
    norms = torch.zeros(3, dtype=torch.float64, device=DEV)
    R.fb_step(ctx, torch.tensor(x, dtype=dt, device=DEV), torch.tensor(y, dtype=cdt, device=DEV), gamma,
              R.RI_PROX_CNN, 0.0, xo, norms)
    ps32 = [(w_.astype(np.float32).astype(np.float64), b_.astype(np.float32).astype(np.float64)) for w_, b_ in ps]
    g, rr = c.op.grad(x, y)
    z = (x - gamma * g).astype(np.float32).astype(np.float64)
    ref = OC.denoise_facets(ps32, z, core=64, halo=16, bf16=True)
    got = xo.cpu().numpy()
    e = rel(z - got, z - ref)
    n = norms.cpu().numpy()
    print(f"prec {prec}: PnP step net rel err {e:.2e}; norms {n} vs "
          f"{(np.sum((ref - x) ** 2), np.sum(ref ** 2), rr)}")
    assert e <= 5e-3
    assert n[0] == pytest.approx(np.sum((got - x) ** 2), rel=1e-5)
    assert n[1] == pytest.approx(np.sum(got ** 2), rel=1e-5)
    assert n[2] == pytest.approx(rr, rel=5e-5 if prec == 32 else 1e-9)


def test_pnp_solve_alpha_and_first_iterations():
    """alpha and sigma follow eqs. (C2)-(C3) with the oracle's dirty image and
    dirty-beam peak; three graph-replayed PnP iterations from 0 track the
    oracle's iteration on the rescaled problem."""
    c = wide()
    ps = _trained_like_params(seed=17)
    ctx = _ctx(c, 64, 64, 16)
    R.ri_load_denoiser(ctx, torch.tensor(_list_to_params(ps), device=DEV), LAYERS)
    L, _ = R.ri_power_norm(ctx, 300, 1e-10)
    beta = OF.dirty_beam_peak(c.op)
    peak = float(c.op.phi_adj(c.y).max())
    sigma_train = 1e-3
    alpha = OF.alpha_rescale(peak, beta, c.tau, L, sigma_train)
    o = R.ri_solve_opts()
    o.max_iter, o.rel_tol, o.prox_kind, o.tau, o.sigma_train, o.L = 4, 0.0, R.RI_PROX_CNN, c.tau, sigma_train, L
    o.check_every, o.use_graph, o.diverge_checks = 4, 1, 100
    xo = torch.empty((c.N, c.N), dtype=torch.float64, device=DEV)
    rep = R.pnp_solve(ctx, torch.tensor(c.y, dtype=torch.complex128, device=DEV), o, xo)
    print(f"alpha {rep.alpha} vs {alpha}; sigma {rep.t_or_sigma}")
    assert rep.alpha == pytest.approx(alpha, rel=1e-9)
    assert rep.t_or_sigma == pytest.approx(OF.sigma_from(c.tau, alpha, L), rel=1e-9)
    assert rep.fell_back == 0 and rep.iters == 4
    ps32 = [(w_.astype(np.float32).astype(np.float64), b_.astype(np.float32).astype(np.float64)) for w_, b_ in ps]
    den = lambda z: OC.denoise_facets(ps32, z.astype(np.float32).astype(np.float64), core=64, halo=16, bf16=True)
    xr, _ = OF.fb(c.op, c.y / alpha, L, 0.0, 4, denoise=den)
    e = rel(xo.cpu().numpy(), alpha * xr)
    print(f"4 PnP iterations: rel err vs oracle {e:.2e}")
    assert e <= 1e-2


def test_expansive_denoiser_falls_back_to_haar():
    """A denoiser that adds a constant every step makes the residual grow: the
    solve must report RI_FELLBACK and finish with the Haar prox."""
    c = wide()
    ps = _trained_like_params(seed=18)
    w_last, b_last = ps[-1]
    ps[-1] = (w_last * 0.0, b_last * 0.0 - 5.0)      # net(z) = -5 -> D(z) = z + 5
    ctx = _ctx(c, 32, 0, 0)
    R.ri_load_denoiser(ctx, torch.tensor(_list_to_params(ps), device=DEV), LAYERS)
    L, _ = R.ri_power_norm(ctx, 300, 1e-10)
    o = R.ri_solve_opts()
    o.max_iter, o.rel_tol, o.prox_kind, o.tau, o.sigma_train, o.L = 30, 0.0, R.RI_PROX_CNN, c.tau, 1e-3, L
    o.check_every, o.use_graph, o.diverge_checks = 1, 1, 3
    xo = torch.empty((c.N, c.N), dtype=torch.float32, device=DEV)
    rep = R.ri_solve_report()
    import ctypes
    st = R.load().pnp_solve(ctx.handle, R._vis(ctx, torch.tensor(c.y, dtype=torch.complex64, device=DEV), "y"),
                            ctypes.byref(o), R._image(ctx, xo, "x"), ctypes.byref(rep))
    torch.cuda.synchronize()
    msg = R.load().ri_last_error(ctx.handle)
    print(f"status {st} ({msg}), fell_back {rep.fell_back}, iters {rep.iters}, snr {rep.snr_db}")
    assert st == R.RI_FELLBACK and rep.fell_back == 1
    assert np.isfinite(xo.cpu().numpy()).all()
    assert xo.cpu().numpy().min() >= 0.0      # finished with the positive Haar prox


def test_denoiser_argument_errors():
    c = wide()
    ctx = _ctx(c, 32, 64, 16)
    z = torch.zeros((c.N, c.N), dtype=torch.float32, device=DEV)
    o = torch.empty_like(z)
    with pytest.raises(R.RIError) as e:          # no network loaded yet
        R.denoise(ctx, z, o, R.RI_PROX_CNN, 0.0)
    assert e.value.status == R.RI_EINVAL and "ri_load_denoiser" in str(e.value)
    with pytest.raises(R.RIError) as e:          # parameter count of a 10-layer network, 8 layers claimed
        R.ri_load_denoiser(ctx, torch.tensor(_list_to_params(_trained_like_params()), device=DEV), 8)
    assert e.value.status == R.RI_EINVAL
    R.ri_load_denoiser(ctx, torch.tensor(_list_to_params(_trained_like_params()), device=DEV), LAYERS)
    with pytest.raises(R.RIError) as e:          # in place is not allowed for the CNN
        R.denoise(ctx, z, z, R.RI_PROX_CNN, 0.0)
    assert e.value.status == R.RI_EINVAL
    net = R.ri_cnn_create(layers=LAYERS, max_batch=1, max_h=32, max_w=32)
    with pytest.raises(ValueError):              # beyond the network's buffers (binding check)
        R.ri_cnn_forward(net, torch.zeros((1, 48, 32), device=DEV), torch.zeros((1, 48, 32), device=DEV))
    with pytest.raises(R.RIError) as e:          # gradients need training buffers
        R.ri_cnn_grad(net, torch.zeros((1, 32, 32), device=DEV), torch.zeros((1, 32, 32), device=DEV),
                      torch.zeros(net.n_params, device=DEV))
    assert e.value.status == R.RI_EINVAL


def test_training_is_deterministic():
    """The weight-gradient sums run in a fixed order: two networks trained on the same
    batches end with identical parameters."""
    u = torch.tensor(_images(4, 32, 32, seed=60), dtype=torch.float32, device=DEV)
    out = []
    for _ in range(2):
        net = R.ri_cnn_create(layers=LAYERS, max_batch=4, max_h=32, max_w=32, training=True, seed=9)
        for it in range(5):
            R.ri_cnn_train_step(net, u, 0.05, 100 + it, 1e-3)
        p = torch.empty(net.n_params, dtype=torch.float32, device=DEV)
        R.ri_cnn_get_params(net, p)
        torch.cuda.synchronize()
        out.append(p.cpu())
    assert torch.equal(out[0], out[1])


def test_sample_batch_draws_pool_patches_in_the_eight_orientations():
    """ri_cnn_sample_batch: every item is some pool patch in one of the eight
    symmetries of the square (exact copy), and over a batch the draws cover
    several patches and orientations."""
    rng = np.random.default_rng(4)
    n, side, B = 7, 32, 64
    pool = rng.standard_normal((n, side, side)).astype(np.float32)
    net = R.ri_cnn_create(layers=3, max_batch=1, max_h=16, max_w=16)
    pt = torch.tensor(pool, device=DEV)
    out = torch.full((B, side, side), float("nan"), device=DEV)
    R.ri_cnn_sample_batch(net, pt, 12345, out)
    got = out.cpu().numpy()
    net.close()
    seen = set()
    for b in range(B):
        match = None
        for p in range(n):
            for o in range(8):
                v = pool[p].T if o & 1 else pool[p]
                v = v[::-1, :] if o & 2 else v
                v = v[:, ::-1] if o & 4 else v
                if np.array_equal(got[b], v):
                    match = (p, o)
        assert match is not None, b
        seen.add(match)
    assert len({p for p, _ in seen}) >= 5 and len({o for _, o in seen}) >= 6
