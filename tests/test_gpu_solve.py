"""GPU tests of the data-block decomposition (eq. E2) and of the solver loop:
uneven angular-sector blocks in one persistent launch against the single-block
operator and the oracle's per-block sum; hipGraph replay of the FB iteration
against eager steps, replay by replay."""
import math

import numpy as np
import pytest

import synth
from _cases import rel, wide
from oracle import fb as OF
from oracle import phi as OP

torch = pytest.importorskip("torch")
import paper_2207_11336_amd.ri as R  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _img(a, prec):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32 if prec == 32 else torch.float64, device=DEV)


def _vis(a, prec):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.complex64 if prec == 32 else torch.complex128,
                        device=DEV)


def _blocked_case():
    c = wide()
    sizes = synth.block_sizes(7, c.M, 200, 4000, seed=synth.SEED_BLOCKS)
    perm, offs = synth.blocked(c.uvw, sizes)
    return c, c.uvw[perm], offs


@pytest.mark.parametrize("prec,mode", [(32, R.RI_G_CSR), (32, R.RI_G_OTF), (32, R.RI_G_SEP), (64, R.RI_G_OTF)])
def test_blocks_sum_to_monolithic_operator(prec, mode):
    c, uvw_b, offs = _blocked_case()
    mk = lambda uvw, nb, bo: R.ri_create(R.plan_desc(c.N, c.M, cell_rad=c.cell, w_max=c.W, n_wplanes=c.n_wplanes,
                                                     precision=prec, g_mode=mode, n_blocks=nb), uvw,
                                         block_offsets=bo)
    ctx_b = mk(uvw_b, len(offs) - 1, offs)
    ctx_1 = mk(uvw_b, 1, None)
    assert R.ri_get_plan_stats(ctx_b).n_blocks == len(offs) - 1
    x = _img(c.xr, prec)
    gb = torch.zeros_like(x)
    g1 = torch.zeros_like(x)
    R.ri_gradient(ctx_b, x, "none", gb)
    R.ri_gradient(ctx_1, x, "none", g1)
    op_b = OP.Operator(c.N, uvw_b, cell=c.cell, W=c.W, n_wplanes=c.n_wplanes)
    ref = OP.block_sum_phi_adj_phi(op_b, offs, c.xr)
    e_blocks = rel(gb.cpu().numpy(), g1.cpu().numpy())
    e_ref = rel(gb.cpu().numpy(), ref)
    print(f"prec {prec} mode {mode}: blocks vs single {e_blocks:.3e}, vs oracle block sum {e_ref:.3e}")
    assert e_blocks <= (1e-6 if prec == 32 else 1e-13)
    assert e_ref <= (1e-5 if prec == 32 else 1e-11)


@pytest.mark.parametrize("prec", [32, 64])
def test_graph_replay_matches_eager_iterations(prec):
    c = wide()
    d = R.plan_desc(c.N, c.M, cell_rad=c.cell, w_max=c.W, n_wplanes=c.n_wplanes, precision=prec,
                    g_mode=R.RI_G_OTF)
    ctx = R.ri_create(d, c.uvw)
    R.ri_set_data(ctx, _vis(c.y, prec))
    L, _ = R.ri_power_norm(ctx, max_it=200, rtol=1e-9)
    K = 12
    xt = _img(c.x, prec)
    runs = {}
    for g in (0, 1):
        trace = np.zeros((K, 4))
        opts = R.ri_solve_opts(max_iter=K, rel_tol=0.0, prox_kind=R.RI_PROX_HAAR, tau=c.tau, sigma_train=0.0,
                               L=L, check_every=1, x_true=xt.data_ptr(),
                               trace=trace.ctypes.data, use_graph=g, diverge_checks=0)
        x = torch.empty((c.N, c.N), dtype=xt.dtype, device=DEV)
        rep = R.pnp_solve(ctx, None, opts, x)
        runs[g] = (x.cpu().numpy(), trace.copy(), rep)
    (xe, te, re_), (xg, tg, rg) = runs[0], runs[1]
    assert re_.iters == rg.iters == K
    tol = 1e-5 if prec == 32 else 1e-12
    for k in range(K):   # every replay against the eager step
        assert tg[k, 1] == pytest.approx(te[k, 1], rel=tol), k
        assert tg[k, 2] == pytest.approx(te[k, 2], abs=1e-3 if prec == 32 else 1e-9), k
    assert rel(xg, xe) <= tol
    assert rg.snr_db == pytest.approx(OF.snr_db(c.x, xg), abs=1e-3)
    print(f"prec {prec}: graph {rg.ms:.2f} ms vs eager {re_.ms:.2f} ms for {K} its; SNR {rg.snr_db:.3f} dB")


def test_solve_waits_for_data_still_in_flight():
    """pnp_solve takes no stream: data written by work still queued on the caller's
    stream when it is called (here behind a spin kernel of fixed length) must be
    the data it solves with. Reference: the same solve after a device sync."""
    c = wide()
    d = R.plan_desc(c.N, c.M, cell_rad=c.cell, w_max=c.W, n_wplanes=c.n_wplanes, precision=32,
                    g_mode=R.RI_G_OTF)
    ctx = R.ri_create(d, c.uvw)
    L, _ = R.ri_power_norm(ctx, max_it=200, rtol=1e-9)
    y = _vis(c.y, 32)
    opts = R.ri_solve_opts(max_iter=6, rel_tol=0.0, prox_kind=R.RI_PROX_HAAR, tau=c.tau, sigma_train=0.0, L=L,
                           check_every=6, use_graph=1, diverge_checks=0)
    torch.cuda.synchronize()
    x_ref = torch.empty((c.N, c.N), dtype=torch.float32, device=DEV)
    R.pnp_solve(ctx, y, opts, x_ref)
    y_late = torch.zeros_like(y)
    torch.cuda.synchronize()
    torch.cuda._sleep(20_000_000)          # a bounded spin on the current stream
    y_late.copy_(y)                        # queued behind it
    x = torch.empty_like(x_ref)
    R.pnp_solve(ctx, y_late, opts, x)
    e = rel(x.cpu().numpy(), x_ref.cpu().numpy())
    print(f"solve on data still in flight vs after a sync: {e:.2e}; |x| {float(torch.linalg.vector_norm(x)):.3e}")
    assert float(torch.linalg.vector_norm(x_ref)) > 0.0
    assert e <= 1e-5
