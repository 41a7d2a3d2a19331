"""Parity at the benchmark's full size (C1: 2048^2 image, 4096^2 grid,
M = 16,777,152 visibilities, supports 11..17, 4,097 w-planes), in the launch
configuration bench.py times (FP32, autotuned tile, default work items):

* Phi x on a seeded sample of visibilities (including the largest |omega| and
  the extreme w) against the FP64 oracle restricted to those visibilities;
* Re{Phi^dagger y} for data that are non-zero only on a seeded sample of
  visibilities, against the oracle's adjoint over that sample (the whole
  launch still runs over all work items);
* properties that hold at any size: the adjoint identity, and the fused
  gradient against separate forward and adjoint passes;
* FP64 Phi (the operator of the power iteration) on a sample;
* the CNN denoiser on the whole 2048^2 image at sampled pixels, each against
  the oracle on the pixel's receptive field.
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
WL = synth.C1


@pytest.fixture(scope="module")
def full():
    uvw = synth.uvw(WL)
    x = synth.sky(WL.N).astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(123)
    om = np.hypot(uvw[:, 0], uvw[:, 1])
    extra = [int(np.argmax(om)), int(np.argmax(uvw[:, 2])), int(np.argmin(uvw[:, 2])), 0, WL.M - 1]
    idx = np.unique(np.concatenate([rng.choice(WL.M, 4000, replace=False), extra]))
    return uvw, x, idx


def _ctx(uvw, prec, mode):
    d = R.plan_desc(WL.N, WL.M, cell_rad=WL.cell_rad, w_max=WL.W, n_wplanes=WL.n_wplanes, precision=prec,
                    g_mode=mode)
    return R.ri_create(d, uvw)


def _oracle_sub(uvw, idx):
    return OP.Operator(WL.N, uvw[idx], cell=WL.cell_rad, W=WL.W, n_wplanes=WL.n_wplanes)


@pytest.mark.parametrize("mode", [R.RI_G_OTF, R.RI_G_CSR], ids=["otf", "csr"])
def test_forward_and_adjoint_sampled(full, mode):
    uvw, x, idx = full
    ctx = _ctx(uvw, 32, mode)
    st = R.ri_get_plan_stats(ctx)
    print(f"plan: tile {st.tile}, items {st.n_items}, nnz {st.nnz:,}")
    xt = torch.tensor(x, dtype=torch.float32, device=DEV)
    y = torch.empty(WL.M, dtype=torch.complex64, device=DEV)
    R.phi_forward(ctx, xt, y)
    sub = _oracle_sub(uvw, idx)
    ref = sub.phi(x)
    got = y[torch.as_tensor(idx, device=DEV)].cpu().numpy()
    e_fwd = rel(got, ref)
    # adjoint of data living on the sampled visibilities only
    rng = np.random.default_rng(7)
    ys = (rng.standard_normal(idx.size) + 1j * rng.standard_normal(idx.size)) * 1e3
    yfull = torch.zeros(WL.M, dtype=torch.complex64, device=DEV)
    yfull[torch.as_tensor(idx, device=DEV)] = torch.tensor(ys, dtype=torch.complex64, device=DEV)
    g = torch.empty_like(xt)
    R.phi_adjoint(ctx, yfull, g)
    ref_adj = sub.phi_adj(ys.astype(np.complex64).astype(np.complex128))
    e_adj = rel(g.cpu().numpy(), ref_adj)
    print(f"mode {mode}: Phi x on {idx.size} sampled visibilities rel {e_fwd:.2e}; "
          f"Phi^dagger of sampled data rel {e_adj:.2e}")
    assert e_fwd <= 1e-5
    assert e_adj <= 1e-5


def test_adjoint_identity_and_fused_gradient(full):
    uvw, x, _ = full
    ctx = _ctx(uvw, 32, R.RI_G_OTF)
    xt = torch.tensor(x, dtype=torch.float32, device=DEV)
    gen = torch.Generator(device=DEV).manual_seed(3)
    y = torch.complex(torch.randn(WL.M, device=DEV, generator=gen), torch.randn(WL.M, device=DEV, generator=gen))
    phx = torch.empty_like(y)
    R.phi_forward(ctx, xt, phx)
    ady = torch.empty_like(xt)
    R.phi_adjoint(ctx, y, ady)
    lhs = torch.sum(phx.to(torch.complex128).conj() * y.to(torch.complex128)).real.item()
    rhs = torch.sum(xt.double() * ady.double()).item()
    e_id = abs(lhs - rhs) / abs(lhs)
    # fused degrid -> residual -> grid against the separate passes
    yd = (phx * 0.9 + y * 1e-3).contiguous()
    g = torch.empty_like(xt)
    r2 = torch.zeros(1, dtype=torch.float64, device=DEV)
    R.ri_gradient(ctx, xt, yd, g, r2)
    res = (phx - yd).contiguous()
    g2 = torch.empty_like(xt)
    R.phi_adjoint(ctx, res, g2)
    e_g = rel(g.cpu().numpy(), g2.cpu().numpy())
    r2_ref = torch.sum(torch.abs(res.to(torch.complex128)) ** 2).item()
    print(f"adjoint identity rel {e_id:.2e}; fused gradient vs separate passes rel {e_g:.2e}; "
          f"r2 {r2.item():.6e} vs {r2_ref:.6e}")
    assert e_id <= 1e-5
    assert e_g <= 1e-5
    assert r2.item() == pytest.approx(r2_ref, rel=1e-5)


def test_fp64_forward_sampled(full):
    uvw, x, idx = full
    ctx = _ctx(uvw, 64, R.RI_G_OTF)
    xt = torch.tensor(x, dtype=torch.float64, device=DEV)
    y = torch.empty(WL.M, dtype=torch.complex128, device=DEV)
    R.phi_forward(ctx, xt, y)
    ref = _oracle_sub(uvw, idx).phi(x)
    e = rel(y[torch.as_tensor(idx, device=DEV)].cpu().numpy(), ref)
    print(f"FP64 Phi x on {idx.size} sampled visibilities rel {e:.2e}")
    assert e <= 1e-11
    # the adjoint of data on the sampled visibilities only (the inverse FFT path)
    rng = np.random.default_rng(77)
    ys = rng.standard_normal(idx.size) + 1j * rng.standard_normal(idx.size)
    yfull = torch.zeros(WL.M, dtype=torch.complex128, device=DEV)
    yfull[torch.as_tensor(idx, device=DEV)] = torch.tensor(ys, device=DEV)
    g = torch.empty_like(xt)
    R.phi_adjoint(ctx, yfull, g)
    e_a = rel(g.cpu().numpy(), _oracle_sub(uvw, idx).phi_adj(ys))
    print(f"FP64 Re Phi^dagger y for data on the sampled visibilities rel {e_a:.2e}")
    assert e_a <= 1e-11


def test_cnn_whole_image_sampled_pixels():
    N, L = WL.N, 10
    rng = np.random.default_rng(11)
    ps = OC.init_params(L, 64, seed=21)
    ps = [(w, rng.standard_normal(b.shape) * 0.05) for w, b in ps]
    vec = np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in ps]).astype(np.float32)
    ps32 = [(w.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for w, b in ps]
    z = synth.sky(N) / 1.0
    z = (z / z.max() + 0.01 * rng.standard_normal((N, N))).astype(np.float32)
    uvw = synth.random_uvw(16, 1.0, 0.0, seed=5)
    ctx = R.ri_create(R.plan_desc(N, 16, precision=32, g_mode=R.RI_G_OTF), uvw)
    R.ri_load_denoiser(ctx, torch.tensor(vec, device=DEV), L)
    zt = torch.tensor(z, device=DEV)
    out = torch.empty_like(zt)
    R.denoise(ctx, zt, out, R.RI_PROX_CNN, 0.0)
    got_img = out.cpu().numpy().astype(np.float64)
    rad = L                                        # receptive radius of L 3x3 layers
    pix = [(0, 0), (0, N - 1), (N - 1, 0), (N - 1, N - 1), (N // 2, N // 2), (5, N // 3), (N - 3, 700)]
    pix += [tuple(p) for p in rng.integers(0, N, size=(57, 2))]
    got, ref = [], []
    for (py, px) in pix:
        ys, xs = py - rad, px - rad
        win = np.zeros((2 * rad + 1, 2 * rad + 1))
        mask = np.zeros_like(win)
        y0, y1, x0, x1 = max(ys, 0), min(ys + 2 * rad + 1, N), max(xs, 0), min(xs + 2 * rad + 1, N)
        win[y0 - ys:y1 - ys, x0 - xs:x1 - xs] = z[y0:y1, x0:x1]
        mask[y0 - ys:y1 - ys, x0 - xs:x1 - xs] = 1.0
        D, _ = OC.forward(ps32, win[None], bf16=True, mask=mask[None])
        ref.append(z[py, px] - D[0, rad, rad])       # net(z) at the pixel
        got.append(z[py, px] - got_img[py, px])
    e = rel(np.array(got), np.array(ref))
    print(f"CNN on 2048^2: net(z) at {len(pix)} sampled pixels rel {e:.2e}")
    assert e <= 1e-2


def test_blocked_operator_equals_monolithic(full):
    """C2: the 64 uneven angular-sector blocks go through the same persistent
    launch; Phi x per visibility is the same sum (bit for bit), the adjoint the
    same sum in another order."""
    uvw, x, _ = full
    W2 = synth.C2
    sizes = synth.block_sizes(W2.n_blocks, WL.M, W2.block_lo, W2.block_hi)
    perm, offs = synth.blocked(uvw, sizes)
    d = R.plan_desc(WL.N, WL.M, cell_rad=WL.cell_rad, w_max=WL.W, n_wplanes=WL.n_wplanes, precision=32,
                    g_mode=R.RI_G_OTF, n_blocks=W2.n_blocks)
    ctxb = R.ri_create(d, uvw[perm], block_offsets=offs)
    ctx = _ctx(uvw, 32, R.RI_G_OTF)
    stb, st = R.ri_get_plan_stats(ctxb), R.ri_get_plan_stats(ctx)
    xt = torch.tensor(x, dtype=torch.float32, device=DEV)
    y, yb = (torch.empty(WL.M, dtype=torch.complex64, device=DEV) for _ in range(2))
    R.phi_forward(ctx, xt, y)
    R.phi_forward(ctxb, xt, yb)
    pt = torch.as_tensor(perm, device=DEV)
    same_tile = stb.tile == st.tile
    e_f = rel(yb.cpu().numpy(), y[pt].cpu().numpy())
    g, gb = torch.empty_like(xt), torch.empty_like(xt)
    R.phi_adjoint(ctx, y, g)
    R.phi_adjoint(ctxb, yb, gb)
    e_a = rel(gb.cpu().numpy(), g.cpu().numpy())
    print(f"{stb.n_blocks} blocks, {stb.n_items} items (tile {stb.tile}) vs {st.n_items} items (tile {st.tile}): "
          f"forward rel {e_f:.2e}, adjoint rel {e_a:.2e}")
    if same_tile:
        assert torch.equal(yb, y[pt])
    assert e_f <= 1e-6
    assert e_a <= 1e-6


def test_cnn_facets_equal_whole_image_full_size():
    """16 facets of 512^2 cores with 32-pixel halos (576^2 tiles) in one launch per
    layer give the whole-image result bit for bit at 2048^2."""
    N, L = WL.N, 10
    ps = OC.init_params(L, 64, seed=22)
    vec = np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in ps]).astype(np.float32)
    z = torch.tensor(synth.sky(N) / synth.sky(N).max(), dtype=torch.float32, device=DEV)
    outs = []
    for core, halo in [(0, 0), (512, 32)]:
        uvw = synth.random_uvw(16, 1.0, 0.0, seed=5)
        ctx = R.ri_create(R.plan_desc(N, 16, precision=32, g_mode=R.RI_G_OTF, facet_core=core, facet_halo=halo),
                          uvw)
        R.ri_load_denoiser(ctx, torch.tensor(vec, device=DEV), L)
        o = torch.full_like(z, float("nan"))
        R.denoise(ctx, z, o, R.RI_PROX_CNN, 0.0)
        outs.append(o)
    assert torch.isfinite(outs[0]).all()
    assert torch.equal(outs[0], outs[1])
