"""ri_gradient_noalloc (the gradient with its work buffers in the library's
static device workspace) against ri_gradient through the C ABI: two calls in a
row, the second on a smaller problem (the workspace keeps the first call's
contents), with caller data, stored data and no data; the largest context the
workspace takes (FP32, N' = 2048) and one it refuses (FP64, N' = 2048).
The two entry points run the same kernels; gridding atomics make the sums
order-dependent at the rounding level, hence the 1e-6 (FP32) and 1e-13 (FP64)
relative bounds instead of bit equality."""
import math

import numpy as np
import pytest

import synth
from _cases import rel

torch = pytest.importorskip("torch")
import paper_2207_11336_amd.ri as R  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _case(N, M, prec, mode, seed):
    cell = 30 * synth.ARCSEC
    W = 2 * 4.0 / (2 * N * N * cell ** 2)
    uvw = synth.random_uvw(M, 2 * math.pi / 3, W, seed=seed)
    ctx = R.ri_create(R.plan_desc(N, M, cell_rad=cell, w_max=W, n_wplanes=129, precision=prec, g_mode=mode), uvw)
    rdt = torch.float32 if prec == 32 else torch.float64
    cdt = torch.complex64 if prec == 32 else torch.complex128
    rng = np.random.default_rng(seed)
    x = torch.tensor(synth.random_image(N, seed + 1), dtype=rdt, device=DEV)
    y = torch.tensor(rng.standard_normal(M) + 1j * rng.standard_normal(M), dtype=cdt, device=DEV) * 50.0
    return ctx, x, y


def _compare(ctx, x, y, tol):
    out = []
    for data in (y, "none"):
        g0, g1 = torch.empty_like(x), torch.full_like(x, float("nan"))
        r0 = torch.zeros(1, dtype=torch.float64, device=DEV)
        r1 = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
        R.ri_gradient(ctx, x, data, g0, r0)
        R.ri_gradient_noalloc(ctx, x, data, g1, r1)
        torch.cuda.synchronize()
        e = rel(g1.cpu().numpy(), g0.cpu().numpy())
        er = abs(r1.item() - r0.item()) / r0.item()
        out.append((e, er))
        assert e <= tol, e
        assert er <= tol, er
    return out


@pytest.mark.parametrize("prec,tol", [(32, 1e-6), (64, 1e-13)])
def test_noalloc_matches_gradient_twice_second_smaller(prec, tol):
    big, xb, yb = _case(128, 20000, prec, R.RI_G_OTF, 5)
    small, xs, ys = _case(64, 3001, prec, R.RI_G_CSR, 9)
    e_big = _compare(big, xb, yb, tol)
    e_small = _compare(small, xs, ys, tol)
    # the stored data (y = NULL) of the smaller context
    R.ri_set_data(small, ys)
    g0, g1 = torch.empty_like(xs), torch.empty_like(xs)
    R.ri_gradient(small, xs, None, g0)
    R.ri_gradient_noalloc(small, xs, None, g1)
    torch.cuda.synchronize()
    e_st = rel(g1.cpu().numpy(), g0.cpu().numpy())
    print(f"FP{prec}: 128^2 {e_big}, then 64^2 {e_small}, stored data {e_st:.2e}")
    assert e_st <= tol
    big.close()
    small.close()


@pytest.mark.parametrize("prec,tol", [(32, 1e-6), (64, 1e-13)])
def test_noalloc_axis_factors_twice_second_smaller(prec, tol):
    # G as stored axis factors (FP32: the gather-form tile kernel)
    big, xb, yb = _case(128, 20000, prec, R.RI_G_SEP, 7)
    small, xs, ys = _case(64, 3001, prec, R.RI_G_SEP, 11)
    e_big = _compare(big, xb, yb, tol)
    e_small = _compare(small, xs, ys, tol)
    print(f"FP{prec} axis factors: 128^2 {e_big}, then 64^2 {e_small}")
    big.close()
    small.close()


def test_noalloc_workspace_limits():
    # FP32 at N' = 2048 fills 64 MiB of the 72 MiB workspace: accepted
    ctx, x, y = _case(1024, 4000, 32, R.RI_G_OTF, 21)
    _compare(ctx, x, y, 1e-6)
    ctx.close()
    # FP64 at N' = 2048 needs 128 MiB: refused with RI_EINVAL before any launch
    ctx, x, y = _case(1024, 500, 64, R.RI_G_OTF, 22)
    g = torch.full_like(x, 7.0)
    with pytest.raises(R.RIError) as ei:
        R.ri_gradient_noalloc(ctx, x, y, g)
    assert ei.value.status == R.RI_EINVAL
    assert "workspace" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((g == 7.0).all())
    ctx.close()
