"""GPU parity of the prox and the forward-backward iteration against the FP64
CPU oracle, through the C ABI (denoise, fb_step, pnp_solve)."""
import math

import numpy as np
import pytest

import synth
from _cases import narrow, rel, wide
from oracle import fb as OF

torch = pytest.importorskip("torch")
import paper_2207_11336_amd.ri as R  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _img(a, prec):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32 if prec == 32 else torch.float64, device=DEV)


def _vis(a, prec):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.complex64 if prec == 32 else torch.complex128,
                        device=DEV)


def _ctx(c, prec, mode=R.RI_G_CSR):
    d = R.plan_desc(c.N, c.M, cell_rad=c.cell, w_max=c.W, n_wplanes=c.n_wplanes, precision=prec, g_mode=mode)
    return R.ri_create(d, c.uvw)


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("t", [0.0, 0.05, 0.3])
def test_haar_denoise_matches_oracle(prec, t):
    c = wide()
    ctx = _ctx(c, prec, R.RI_G_OTF)
    z = synth.random_image(c.N, 4, positive=False)
    out = torch.empty((c.N, c.N), dtype=torch.float32 if prec == 32 else torch.float64, device=DEV)
    R.denoise(ctx, _img(z, prec), out, R.RI_PROX_HAAR, t)
    ref = OF.prox_haar_pos(z, t)
    err = float(np.abs(out.cpu().numpy() - ref).max())
    print(f"prec {prec} t {t}: max abs err {err:.3e}")
    assert err <= (2e-6 if prec == 32 else 1e-14)


@pytest.mark.parametrize("prec,mode", [(32, R.RI_G_CSR), (32, R.RI_G_OTF), (32, R.RI_G_SEP), (64, R.RI_G_OTF)])
def test_fb_step_matches_oracle(prec, mode):
    c = wide()
    ctx = _ctx(c, prec, mode)
    L = float(c.M) * 1.5
    gamma, t = 1.98 / L, OF.threshold(c.tau, L)
    x = OF.prox_haar_pos(c.xr * 0.01, 0.0)
    xo = torch.empty((c.N, c.N), dtype=torch.float32 if prec == 32 else torch.float64, device=DEV)
    norms = torch.zeros(3, dtype=torch.float64, device=DEV)
    R.fb_step(ctx, _img(x, prec), _vis(c.y, prec), gamma, R.RI_PROX_HAAR, t, xo, norms)
    ref, dx2, x2, rr = OF.fb_step(c.op, x, c.y, gamma, lambda z: OF.prox_haar_pos(z, t))
    err = rel(xo.cpu().numpy(), ref)
    n = norms.cpu().numpy()
    print(f"prec {prec} mode {mode}: fb_step rel err {err:.3e}; norms {n} vs {(dx2, x2, rr)}")
    assert err <= (1e-5 if prec == 32 else 1e-11)
    tol = 1e-5 if prec == 32 else 1e-11
    assert n[0] == pytest.approx(dx2, rel=10 * tol) and n[1] == pytest.approx(x2, rel=tol)
    assert n[2] == pytest.approx(rr, rel=tol)


def test_fb_200_iterations_fp64_narrow_field():
    """The narrow-field workload: 200 FP64 FB iterations on the GPU against the oracle."""
    c = narrow()
    ctx = _ctx(c, 64, R.RI_G_OTF)
    L, _ = R.ri_power_norm(ctx, max_it=500, rtol=1e-9, x0=torch.tensor(synth.power_start(c.N), device=DEV))
    Lref, _ = OF.power_norm(c.op.phi_adj_phi, synth.power_start(c.N), max_it=500, rtol=1e-9)
    assert L == pytest.approx(Lref, rel=1e-7)
    t = OF.threshold(c.tau, Lref)
    n_iter = 200
    trace = np.zeros((n_iter, 4))
    xt = torch.tensor(c.x, device=DEV)
    opts = R.ri_solve_opts(max_iter=n_iter, rel_tol=0.0, prox_kind=R.RI_PROX_HAAR, tau=c.tau, sigma_train=0.0,
                           L=Lref, check_every=50, x_true=xt.data_ptr(), trace=trace.ctypes.data, use_graph=1)
    x = torch.empty((c.N, c.N), dtype=torch.float64, device=DEV)
    rep = R.pnp_solve(ctx, _vis(c.y, 64), opts, x)
    xr, hist = OF.fb(c.op, c.y, Lref, t, n_iter, x_true=c.x)
    xg = x.cpu().numpy()
    snr_g, snr_o = OF.snr_db(c.x, xg), OF.snr_db(c.x, xr)
    print(f"C0 FB x200: SNR gpu {snr_g:.4f} dB oracle {snr_o:.4f} dB; rel diff {rel(xg, xr):.3e}; {rep.ms:.1f} ms")
    assert rep.iters == n_iter
    assert abs(snr_g - snr_o) <= 0.01
    assert rel(xg, xr) <= 1e-8
    # the per-iteration SNR trace follows the oracle's history
    snr_hist = np.array([h["snr_db"] for h in hist])
    assert np.abs(trace[:, 2] - snr_hist).max() <= 0.01
    assert rep.snr_db == pytest.approx(snr_o, abs=0.01)
