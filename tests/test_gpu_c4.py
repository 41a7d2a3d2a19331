"""Parity at full scale (C4: 4096^2 image, 8192^2 grid, M = 49,996,800
visibilities as two channels of one 64-antenna track at 1053 and 1399 MHz,
128 uneven angular-sector blocks, 64 facets of 512^2 cores), in the launch
configuration of the full-scale bench run (FP32, on-the-fly G, autotuned
tile, all blocks in one persistent launch):

* Phi x on a seeded sample of visibilities (with the largest |omega| and the
  extreme w of both channels) against the FP64 oracle on that sample;
* Re{Phi^dagger y} for data living only on the sampled visibilities;
* the adjoint identity and the fused gradient against separate passes (any
  size);
* the FP64 operator on a sample, and the FP64 power iteration's L against
  lower bounds that hold for any operator (Rayleigh quotients);
* the CNN denoiser on 64 facets of 576^2 (32 px halo) against the whole
  4096^2 image bit for bit, and at sampled pixels against the oracle.
"""
import numpy as np
import pytest

import synth
from _cases import rel
from oracle import cnn as OC
from oracle import phi as OP

torch = pytest.importorskip("torch")
import paper_2207_11336_amd.ri as R  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
WL = synth.C4


@pytest.fixture(scope="module")
def c4():
    uvw = synth.uvw(WL)
    sizes = synth.block_sizes(WL.n_blocks, WL.M, WL.block_lo, WL.block_hi)
    perm, offs = synth.blocked(uvw, sizes)
    uvwp = uvw[perm]
    del uvw
    x = synth.sky(WL.N).astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(321)
    om = np.hypot(uvwp[:, 0], uvwp[:, 1])
    half = np.nonzero(perm < WL.M // 2)[0]            # the 1053 MHz channel, in block order
    extra = [int(np.argmax(om)), int(np.argmax(uvwp[:, 2])), int(np.argmin(uvwp[:, 2])),
             int(half[np.argmax(om[half])]), int(half[np.argmax(uvwp[half, 2])]), 0, WL.M - 1]
    extra += [int(o) for o in offs[1:-1:16]]             # first visibility of every 16th block
    idx = np.unique(np.concatenate([rng.choice(WL.M, 3000, replace=False), extra]))
    return uvwp, offs, x, idx


def _ctx(c4, prec=32):
    uvwp, offs, _, _ = c4
    d = R.plan_desc(WL.N, WL.M, cell_rad=WL.cell_rad, w_max=WL.W, n_wplanes=WL.n_wplanes, precision=prec,
                    g_mode=R.RI_G_OTF, n_blocks=WL.n_blocks)
    return R.ri_create(d, uvwp, block_offsets=offs)


@pytest.fixture(scope="module")
def ctx32(c4):
    ctx = _ctx(c4)
    yield ctx
    ctx.close()
    torch.cuda.empty_cache()


def _oracle_sub(c4):
    uvwp, _, _, idx = c4
    return OP.Operator(WL.N, uvwp[idx], cell=WL.cell_rad, W=WL.W, n_wplanes=WL.n_wplanes)


def test_c4_forward_and_adjoint_sampled(c4, ctx32):
    _, _, x, idx = c4
    st = R.ri_get_plan_stats(ctx32)
    print(f"C4 plan: {st.n_blocks} blocks, tile {st.tile}, items {st.n_items}, "
          f"device {st.device_bytes / 2**30:.2f} GiB")
    xt = torch.tensor(x, dtype=torch.float32, device=DEV)
    y = torch.empty(WL.M, dtype=torch.complex64, device=DEV)
    R.phi_forward(ctx32, xt, y)
    sub = _oracle_sub(c4)
    ti = torch.as_tensor(idx, device=DEV)
    e_fwd = rel(y[ti].cpu().numpy(), sub.phi(x))
    rng = np.random.default_rng(8)
    ys = (rng.standard_normal(idx.size) + 1j * rng.standard_normal(idx.size)) * 1e3
    yfull = torch.zeros(WL.M, dtype=torch.complex64, device=DEV)
    yfull[ti] = torch.tensor(ys, dtype=torch.complex64, device=DEV)
    g = torch.empty_like(xt)
    R.phi_adjoint(ctx32, yfull, g)
    e_adj = rel(g.cpu().numpy(), sub.phi_adj(ys.astype(np.complex64).astype(np.complex128)))
    print(f"C4: Phi x on {idx.size} sampled visibilities rel {e_fwd:.2e}; Phi^dagger of sampled data rel {e_adj:.2e}")
    assert e_fwd <= 1e-5
    assert e_adj <= 1e-5


def test_c4_adjoint_identity_and_fused_gradient(c4, ctx32):
    _, _, x, _ = c4
    xt = torch.tensor(x, dtype=torch.float32, device=DEV)
    gen = torch.Generator(device=DEV).manual_seed(4)
    y = torch.complex(torch.randn(WL.M, device=DEV, generator=gen), torch.randn(WL.M, device=DEV, generator=gen))
    phx = torch.empty_like(y)
    R.phi_forward(ctx32, xt, phx)
    ady = torch.empty_like(xt)
    R.phi_adjoint(ctx32, y, ady)
    lhs = torch.sum(phx.to(torch.complex128).conj() * y.to(torch.complex128)).real.item()
    rhs = torch.sum(xt.double() * ady.double()).item()
    e_id = abs(lhs - rhs) / abs(lhs)
    yd = (phx * 0.9 + y * 1e-3).contiguous()
    del y, ady
    g = torch.empty_like(xt)
    r2 = torch.zeros(1, dtype=torch.float64, device=DEV)
    R.ri_gradient(ctx32, xt, yd, g, r2)
    res = (phx - yd).contiguous()
    g2 = torch.empty_like(xt)
    R.phi_adjoint(ctx32, res, g2)
    e_g = rel(g.cpu().numpy(), g2.cpu().numpy())
    r2_ref = torch.sum(torch.abs(res.to(torch.complex128)) ** 2).item()
    print(f"C4: adjoint identity rel {e_id:.2e}; fused gradient vs separate passes rel {e_g:.2e}")
    assert e_id <= 1e-5
    assert e_g <= 1e-5
    assert r2.item() == pytest.approx(r2_ref, rel=1e-5)


def test_c4_power_norm_fp64(c4, ctx32):
    """L from the FP64 power iteration bounds every Rayleigh quotient from
    above: ||Phi v||^2 / ||v||^2 <= L for the sky and for the centre pixel's
    delta (whose quotient is beta = Re Phi^dagger Phi delta at the centre)."""
    _, _, x, _ = c4
    L, its = R.ri_power_norm(ctx32, 60, 1e-7)
    xt = torch.tensor(x, dtype=torch.float32, device=DEV)
    y = torch.empty(WL.M, dtype=torch.complex64, device=DEV)
    R.phi_forward(ctx32, xt, y)
    q_sky = float(torch.sum(torch.abs(y.to(torch.complex128)) ** 2)) / float(torch.sum(xt.double() ** 2))
    d = torch.zeros_like(xt)
    d[WL.N // 2, WL.N // 2] = 1.0
    R.phi_forward(ctx32, d, y)
    beam = torch.empty_like(xt)
    R.phi_adjoint(ctx32, y, beam)
    beta = float(beam[WL.N // 2, WL.N // 2])
    print(f"C4: L = {L:.6e} after {its} FP64 iterations; sky quotient {q_sky:.4e}, beta {beta:.6e}")
    assert np.isfinite(L) and L > 0
    assert q_sky <= L * (1 + 1e-6)
    assert beta <= L * (1 + 1e-6)


def test_c4_fp64_forward_sampled(c4):
    _, _, x, idx = c4
    ctx = _ctx(c4, prec=64)
    try:
        xt = torch.tensor(x, dtype=torch.float64, device=DEV)
        y = torch.empty(WL.M, dtype=torch.complex128, device=DEV)
        R.phi_forward(ctx, xt, y)
        e = rel(y[torch.as_tensor(idx, device=DEV)].cpu().numpy(), _oracle_sub(c4).phi(x))
        del y
    finally:
        ctx.close()
        torch.cuda.empty_cache()
    print(f"C4: FP64 Phi x on {idx.size} sampled visibilities rel {e:.2e}")
    assert e <= 1e-11


def test_c4_cnn_64_facets():
    """64 facets of 512^2 cores with 32 px halos (576^2 tiles) against the whole
    4096^2 image (bit for bit), and at sampled pixels against the oracle on
    each pixel's receptive field (facet borders and image corners included)."""
    N, L = WL.N, 10
    rng = np.random.default_rng(12)
    ps = OC.init_params(L, 64, seed=23)
    ps = [(w, rng.standard_normal(b.shape) * 0.05) for w, b in ps]
    vec = np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in ps]).astype(np.float32)
    ps32 = [(w.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for w, b in ps]
    sky = synth.sky(N)
    z = (sky / sky.max() + 0.01 * rng.standard_normal((N, N))).astype(np.float32)
    zt = torch.tensor(z, device=DEV)
    outs = []
    for core, halo in [(0, 0), (512, 32)]:
        uvw = synth.random_uvw(16, 1.0, 0.0, seed=5)
        ctx = R.ri_create(R.plan_desc(N, 16, precision=32, g_mode=R.RI_G_OTF, facet_core=core, facet_halo=halo),
                          uvw)
        R.ri_load_denoiser(ctx, torch.tensor(vec, device=DEV), L)
        o = torch.full_like(zt, float("nan"))
        R.denoise(ctx, zt, o, R.RI_PROX_CNN, 0.0)
        torch.cuda.synchronize()
        ctx.close()
        outs.append(o)
    torch.cuda.empty_cache()
    assert torch.isfinite(outs[0]).all()
    assert torch.equal(outs[0], outs[1])
    got_img = outs[1].cpu().numpy().astype(np.float64)
    rad = L
    pix = [(0, 0), (0, N - 1), (N - 1, 0), (N - 1, N - 1), (511, 512), (512, 511), (2047, 2048), (3584, 3583)]
    pix += [tuple(p) for p in rng.integers(0, N, size=(40, 2))]
    got, ref = [], []
    for (py, px) in pix:
        ys, xs = py - rad, px - rad
        win = np.zeros((2 * rad + 1, 2 * rad + 1))
        mask = np.zeros_like(win)
        y0, y1, x0, x1 = max(ys, 0), min(ys + 2 * rad + 1, N), max(xs, 0), min(xs + 2 * rad + 1, N)
        win[y0 - ys:y1 - ys, x0 - xs:x1 - xs] = z[y0:y1, x0:x1]
        mask[y0 - ys:y1 - ys, x0 - xs:x1 - xs] = 1.0
        D, _ = OC.forward(ps32, win[None], bf16=True, mask=mask[None])
        ref.append(z[py, px] - D[0, rad, rad])
        got.append(z[py, px] - got_img[py, px])
    e = rel(np.array(got), np.array(ref))
    print(f"C4 CNN on 64 facets: equal to the whole image; net(z) at {len(pix)} sampled pixels rel {e:.2e}")
    assert e <= 1e-2


def test_c4_normal_operator_equals_oracle_at_full_size(c4, ctx32):
    """Re{Phi^dagger Phi} x at the sky over all 49,996,800 visibilities of both
    channels (appendix A with y = 0; eq. E2's sum over the 128 blocks in one
    persistent launch), element by element on the whole 4096^2 image against
    the FP64 oracle (one full gradient, about a minute on 16 cores): relative
    l2 <= 1e-5, largest pixel error <= 1e-5 of max|g|, ||Phi x||^2 to 1e-5."""
    uvwp, _, x, _ = c4
    op = OP.Operator(WL.N, uvwp, cell=WL.cell_rad, W=WL.W, n_wplanes=WL.n_wplanes)
    ref, rr_ref = op.grad(x, None)
    del op
    xt = torch.tensor(x, dtype=torch.float32, device=DEV)
    g = torch.empty_like(xt)
    r2 = torch.zeros(1, dtype=torch.float64, device=DEV)
    R.ri_gradient(ctx32, xt, "none", g, r2)
    torch.cuda.synchronize()
    got = g.cpu().numpy().astype(np.float64)
    e2 = rel(got, ref)
    emax = float(np.abs(got - ref).max() / np.abs(ref).max())
    er = abs(r2.item() - rr_ref) / rr_ref
    print(f"C4 Re Phi^dagger Phi x over all {WL.M:,} visibilities: rel l2 {e2:.2e}, max {emax:.2e}, "
          f"||Phi x||^2 rel {er:.2e}")
    assert e2 <= 1e-5
    assert emax <= 1e-5
    assert er <= 1e-5
