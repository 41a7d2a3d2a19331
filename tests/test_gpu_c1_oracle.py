"""The timed gradient pass against the FP64 oracle over every visibility of the
benchmark's workload (C1: 2048^2 image, 4096^2 grid, M = 16,777,152,
supports 11..17, 4,097 w-planes), element by element on the whole image.

The operator is eq. (1), Phi = G F Z; the gradient is appendix A's
Re{Phi^dagger (Phi x - y)} = Re{Phi^dagger Phi} x - Re{Phi^dagger y}, one fused
degrid -> residual -> grid pass on the GPU in the launch configuration the
benchmark times (FP32, autotuned tile, default work items), for the stored,
the on-the-fly and the axis-factor G and for the 64 uneven angular-sector blocks of eq. (E2) in
one persistent launch; with the axis factors also at tiles 8 and 16 explicitly, so both gather
forms (the VALU one on a 24-cell subgrid side, the matrix-core one on 32) are compared whichever
tile the autotuner picks. The oracle computes all three cases once (about 12 s
per gradient on 16 cores), so the dense uv core, where the GPU accumulates
tens of visibilities per cell through FP64 LDS partial sums and FP32 global
atomics, is compared as a whole.

Gates (FP32 arithmetic against FP64):
  * Re{Phi^dagger Phi} x at the sky (y = 0): relative l2 <= 1e-5 and the
    largest pixel error <= 1e-5 max|g|; ||Phi x||^2 to 1e-5;
  * the gradient with the 40 dB data at a random positive image (a large
    residual): the same bounds, ||Phi x - y||^2 to 1e-5;
  * the gradient with the 40 dB data at the sky itself: there the residual is
    the noise, 1% of Phi x, so an FP32 Phi x resolves it only to about 1e-7 / 1e-2
    of its own size; the error is bounded by 1e-5 of ||Re{Phi^dagger Phi} x||
    (the operator's FP32 resolution) and reported relative to the gradient too;
    ||r||^2 to 1e-4.
"""
import numpy as np
import pytest

import synth
from _cases import rel
from oracle import fb as OF
from oracle import phi as OP

torch = pytest.importorskip("torch")
import paper_2207_11336_amd.ri as R  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
WL = synth.C1


@pytest.fixture(scope="module")
def c1():
    uvw = synth.uvw(WL)
    op = OP.Operator(WL.N, uvw, cell=WL.cell_rad, W=WL.W, n_wplanes=WL.n_wplanes)
    x = synth.sky(WL.N).astype(np.float32).astype(np.float64)
    xr = (synth.random_image(WL.N, 61) * x.max()).astype(np.float32).astype(np.float64)
    y0 = op.phi(x)
    tau = OF.tau_from_isnr(y0, 40.0)
    y = (y0 + OF.complex_noise(tau, synth.noise_normals(WL.M, synth.SEED_NOISE))).astype(np.complex64)
    y = y.astype(np.complex128)
    ref = {
        "gram": op.grad(x, None),       # (Re Phi^dagger Phi x, ||Phi x||^2)
        "rand": op.grad(xr, y),         # large residual
        "sky": op.grad(x, y),           # residual at the noise level
    }
    print(f"oracle: {OP.num_threads()} threads, ||Phi x||^2 {ref['gram'][1]:.6e}, tau {tau:.4e}")
    return uvw, x, xr, y, ref


@pytest.mark.parametrize("which", ["otf", "csr", "sep", "sep-tile8", "sep-tile16", "otf-64-blocks"])
def test_gradient_equals_oracle_at_full_size(c1, which):
    uvw, x, xr, y, ref = c1
    ctx, perm = _make_ctx(uvw, which)
    name = which
    st = R.ri_get_plan_stats(ctx)
    yd = y if perm is None else y[perm]
    xt = torch.tensor(x, dtype=torch.float32, device=DEV)
    xrt = torch.tensor(xr, dtype=torch.float32, device=DEV)
    yt = torch.tensor(yd, dtype=torch.complex64, device=DEV)
    g = torch.empty_like(xt)
    r2 = torch.zeros(1, dtype=torch.float64, device=DEV)
    out = {}
    for key, xin, data in (("gram", xt, "none"), ("rand", xrt, yt), ("sky", xt, yt)):
        R.ri_gradient(ctx, xin, data, g, r2)
        torch.cuda.synchronize()
        out[key] = (g.cpu().numpy().astype(np.float64), float(r2.item()))
    ctx.close()
    gram_ref, rr_gram = ref["gram"]
    line = [f"{name}: tile {st.tile}, {st.n_items} items, {st.n_blocks} blocks"]
    for key in ("gram", "rand"):
        got, rr = out[key]
        gr, rr_ref = ref[key]
        e2 = rel(got, gr)
        emax = float(np.abs(got - gr).max() / np.abs(gr).max())
        er = abs(rr - rr_ref) / rr_ref
        line.append(f"{key}: rel l2 {e2:.2e}, max {emax:.2e}, r2 rel {er:.2e}")
        assert e2 <= 1e-5, (key, e2)
        assert emax <= 1e-5, (key, emax)
        assert er <= 1e-5, (key, er)
    got, rr = out["sky"]
    gr, rr_ref = ref["sky"]
    e_op = float(np.linalg.norm(got - gr) / np.linalg.norm(gram_ref))
    e_g = rel(got, gr)
    er = abs(rr - rr_ref) / rr_ref
    line.append(f"sky+data: err/||Phi^dagger Phi x|| {e_op:.2e}, rel l2 {e_g:.2e}, r2 rel {er:.2e}")
    print("; ".join(line))
    assert e_op <= 1e-5
    assert er <= 1e-4


def _make_ctx(uvw, which):
    base = dict(cell_rad=WL.cell_rad, w_max=WL.W, n_wplanes=WL.n_wplanes, precision=32)
    if which == "otf":
        return R.ri_create(R.plan_desc(WL.N, WL.M, g_mode=R.RI_G_OTF, **base), uvw), None
    if which == "csr":
        return R.ri_create(R.plan_desc(WL.N, WL.M, g_mode=R.RI_G_CSR, **base), uvw), None
    if which.startswith("sep"):
        tile = int(which[len("sep-tile"):]) if which != "sep" else 0
        return R.ri_create(R.plan_desc(WL.N, WL.M, g_mode=R.RI_G_SEP, tile=tile, **base), uvw), None
    W2 = synth.C2
    sizes = synth.block_sizes(W2.n_blocks, WL.M, W2.block_lo, W2.block_hi)
    perm, offs = synth.blocked(uvw, sizes)
    d = R.plan_desc(WL.N, WL.M, g_mode=R.RI_G_OTF, n_blocks=W2.n_blocks, **base)
    return R.ri_create(d, uvw[perm], block_offsets=offs), perm
