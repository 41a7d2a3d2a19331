"""GPU parity of uSARA's denoiser (section "uSARA's handcrafted denoiser")
against the FP64 oracle (oracle/sara.py): the dictionary's analysis and
synthesis, the sub-iterative dual forward-backward prox with its warm start,
the log-sum reweighting, the FB step with that prox, and a reweighted uSARA
solve; at the full C1 size the frame properties and two whole bases."""
import math

import numpy as np
import pytest

import synth
from _cases import rel
from oracle import fb as OF
from oracle import phi as OP
from oracle import sara as S

torch = pytest.importorskip("torch")
import paper_2207_11336_amd.ri as R  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _ctx(n, prec, uvw=None):
    if uvw is None:
        uvw = synth.random_uvw(200, 0.9 * math.pi, 0.0, seed=1)
    return R.ri_create(R.plan_desc(n, uvw.shape[0], precision=prec, g_mode=R.RI_G_OTF), uvw)


def _ft(prec):
    return torch.float64 if prec == 64 else torch.float32


def _img(n, seed):
    if n < 32:
        return np.abs(synth.random_image(n, seed))
    return synth.sky(n, seed=seed, n_compact=max(4, n // 8), n_ext=1) + 0.02 * synth.random_image(n, seed + 1)


@pytest.mark.parametrize("n", [16, 64])
@pytest.mark.parametrize("prec", [64, 32])
def test_analysis_and_synthesis_match_oracle(n, prec):
    ctx = _ctx(n, prec)
    x = _img(n, 3)
    if prec == 32:
        x = x.astype(np.float32).astype(np.float64)
    xt = torch.tensor(x, dtype=_ft(prec), device=DEV)
    c = torch.empty(9, n, n, dtype=_ft(prec), device=DEV)
    R.ri_sara_analysis(ctx, xt, c)
    ref = S.Sara().adj(x)
    e_a = rel(c.cpu().numpy(), ref)
    per_basis = [rel(c[b].cpu().numpy(), ref[b]) for b in range(9)]
    rng = np.random.default_rng(4)
    cr = rng.standard_normal((9, n, n))
    if prec == 32:
        cr = cr.astype(np.float32).astype(np.float64)
    xs = torch.empty_like(xt)
    R.ri_sara_synthesis(ctx, torch.tensor(cr, dtype=_ft(prec), device=DEV), xs)
    e_s = rel(xs.cpu().numpy(), S.Sara().syn(cr))
    xr = torch.empty_like(xt)
    R.ri_sara_synthesis(ctx, c, xr)
    e_pr = rel(xr.cpu().numpy(), x)
    print(f"N {n} FP{prec}: Psi^dagger x {e_a:.2e} (worst basis {max(per_basis):.2e}), Psi c {e_s:.2e}, "
          f"Psi Psi^dagger x - x {e_pr:.2e}")
    tol = 1e-13 if prec == 64 else 2e-6
    assert e_a <= tol and max(per_basis) <= tol and e_s <= tol and e_pr <= tol


@pytest.mark.parametrize("prec", [64, 32])
def test_prox_warm_start_and_state_match_oracle(prec):
    n, t, nsub = 64, 0.02, 7
    ctx = _ctx(n, prec)
    R.ri_sara_setup(ctx, nsub)
    s = S.Sara()
    rng = np.random.default_rng(9)
    w = rng.uniform(0.2, 1.0, (9, n, n))
    x_for_w = _img(n, 21)
    rho = 0.05
    R.ri_sara_reweight(ctx, torch.tensor(x_for_w, dtype=_ft(prec), device=DEV), rho)
    w = s.reweight(x_for_w.astype(np.float32).astype(np.float64) if prec == 32 else x_for_w, rho)
    v = None
    for call, seed in enumerate((5, 6)):
        z = _img(n, seed) + 0.05 * rng.standard_normal((n, n))
        if prec == 32:
            z = z.astype(np.float32).astype(np.float64)
        out = torch.empty(n, n, dtype=_ft(prec), device=DEV)
        R.denoise(ctx, torch.tensor(z, dtype=_ft(prec), device=DEV), out, R.RI_PROX_SARA, t)
        xr, v = s.prox(z, t, w, nsub, v)
        vg = torch.empty(9, n, n, dtype=_ft(prec), device=DEV)
        wg = torch.empty_like(vg)
        R.ri_sara_get_state(ctx, vg, wg)
        e_x, e_v, e_w = rel(out.cpu().numpy(), xr), rel(vg.cpu().numpy(), v), rel(wg.cpu().numpy(), w)
        print(f"FP{prec} call {call}: x {e_x:.2e}, dual {e_v:.2e}, weights {e_w:.2e}")
        tol = 1e-12 if prec == 64 else 2e-5
        assert e_x <= tol and e_v <= tol and e_w <= (1e-14 if prec == 64 else 1e-6)
        assert float(out.min()) >= 0.0
        assert np.all(np.abs(vg.cpu().numpy()) <= t * wg.cpu().numpy() * (1 + 1e-6))


def test_fb_step_with_sara_matches_oracle():
    """x_out = prox(x - gamma Re{Phi^dagger (Phi x - y)}) on C0's geometry at N = 64."""
    n = 64
    uvw = synth.random_uvw(4000, 2 * math.pi / 3, 0.0, seed=7)
    op = OP.Operator(n, uvw)
    xt_ = _img(n, 2)
    y = op.phi(xt_) + 0.01 * (np.random.default_rng(3).standard_normal(4000) + 1j)
    ctx = _ctx(n, 64, uvw)
    R.ri_sara_setup(ctx, 5)
    gamma, t = 1.0 / 4000.0, 1e-3
    x0 = 0.5 * xt_
    xin = torch.tensor(x0, device=DEV)
    xo = torch.empty_like(xin)
    norms = torch.zeros(3, dtype=torch.float64, device=DEV)
    R.fb_step(ctx, xin, torch.tensor(y, device=DEV), gamma, R.RI_PROX_SARA, t, xo, norms)
    g, r2 = op.grad(x0, y)
    ref, _ = S.Sara().prox(x0 - gamma * g, t, np.ones((9, n, n)), 5)
    e = rel(xo.cpu().numpy(), ref)
    print(f"FB step with the SARA prox: {e:.2e}; ||r||^2 {norms[2].item():.6e} vs {r2:.6e}")
    assert e <= 1e-12
    assert norms[2].item() == pytest.approx(r2, rel=1e-12)
    assert norms[0].item() == pytest.approx(float(np.sum((ref - x0) ** 2)), rel=1e-10)


@pytest.mark.parametrize("graph", [0, 1])
def test_usara_solve_matches_oracle(graph):
    """Reweighted uSARA (FP64): 24 FB iterations, 4 sub-iterations each,
    reweighting every 8, t = tau / sqrt(2L); against the oracle's loop."""
    n = 64
    uvw = synth.random_uvw(6000, 2 * math.pi / 3, 0.0, seed=8)
    op = OP.Operator(n, uvw)
    x_true = _img(n, 12)
    y0 = op.phi(x_true)
    tau = OF.tau_from_isnr(y0, 30.0)
    y = y0 + OF.complex_noise(tau, synth.noise_normals(6000, synth.SEED_NOISE))
    L, _ = OF.power_norm(op.phi_adj_phi, synth.random_image(n, 30), max_it=300, rtol=1e-10)
    ctx = _ctx(n, 64, uvw)
    R.ri_sara_setup(ctx, 4)
    opts = R.ri_solve_opts(max_iter=24, rel_tol=0.0, prox_kind=R.RI_PROX_SARA, tau=tau, sigma_train=0.0, L=L,
                           check_every=4, use_graph=graph, reweight_every=8)
    xs = torch.empty(n, n, dtype=torch.float64, device=DEV)
    rep = R.pnp_solve(ctx, torch.tensor(y, device=DEV), opts, xs)
    gamma, t = 1.98 / L, tau / math.sqrt(2 * L)
    ref, w = S.usara(lambda u: op.grad(u, y)[0], np.zeros((n, n)), gamma, t, 24, 4, 8)
    e = rel(xs.cpu().numpy(), ref)
    snr = lambda u: 20 * np.log10(np.linalg.norm(x_true) / np.linalg.norm(u - x_true))  # noqa: E731
    print(f"uSARA x24 (graph {graph}): rel to oracle {e:.2e}; SNR GPU {snr(xs.cpu().numpy()):.3f} dB, "
          f"oracle {snr(ref):.3f} dB; t {rep.t_or_sigma:.3e}")
    assert rep.iters == 24 and rep.fell_back == 0
    assert rep.t_or_sigma == pytest.approx(t, rel=1e-12)
    assert e <= 1e-10


def test_errors():
    ctx = _ctx(64, 32)
    with pytest.raises(R.RIError):
        R.ri_sara_setup(ctx, 0)
    with pytest.raises(R.RIError):
        R.ri_sara_reweight(ctx, torch.zeros(64, 64, device=DEV), 0.0)
    z = torch.zeros(64, 64, device=DEV)
    with pytest.raises(R.RIError):
        R.denoise(ctx, z, z, R.RI_PROX_SARA, 0.1)
    with pytest.raises(R.RIError):
        R.denoise(ctx, z, torch.empty_like(z), R.RI_PROX_SARA, -1.0)
    with pytest.raises(R.RIError):
        R.ri_sara_get_state(_ctx(64, 32), torch.empty(9, 64, 64, device=DEV))   # no state yet
    opts = R.ri_solve_opts(max_iter=2, prox_kind=R.RI_PROX_SARA, tau=1.0, L=1.0, check_every=1, reweight_every=-1)
    with pytest.raises(R.RIError):
        R.pnp_solve(ctx, torch.zeros(200, dtype=torch.complex64, device=DEV), opts, z)


def test_full_size_dictionary_c1():
    """2048^2, FP32 as the bench runs it: Psi Psi^dagger x = x, ||Psi^dagger x|| = ||x||, the
    adjoint identity, and the db1 and db8 slots against the oracle over the whole image."""
    n = 2048
    wl = synth.C1
    ctx = _ctx(n, 32)
    x = synth.sky(wl.N).astype(np.float32).astype(np.float64)
    xt = torch.tensor(x, dtype=torch.float32, device=DEV)
    c = torch.empty(9, n, n, dtype=torch.float32, device=DEV)
    R.ri_sara_analysis(ctx, xt, c)
    xr = torch.empty_like(xt)
    R.ri_sara_synthesis(ctx, c, xr)
    e_pr = rel(xr.cpu().numpy(), x)
    e_en = abs(float(torch.linalg.vector_norm(c.double())) / np.linalg.norm(x) - 1)
    d = torch.randn(9, n, n, device=DEV)
    xd = torch.empty_like(xt)
    R.ri_sara_synthesis(ctx, d, xd)
    lhs, rhs = float(torch.sum(c.double() * d.double())), float(torch.sum(xt.double() * xd.double()))
    e_adj = abs(lhs - rhs) / (float(torch.linalg.vector_norm(c.double())) * float(torch.linalg.vector_norm(d.double())))
    e1 = rel(c[1].cpu().numpy(), S.dwt2(x, S.daubechies(1)) / 3)
    e8 = rel(c[8].cpu().numpy(), S.dwt2(x, S.daubechies(8)) / 3)
    print(f"C1 dictionary: reconstruction {e_pr:.2e}, energy {e_en:.2e}, adjoint {e_adj:.2e}, "
          f"db1 {e1:.2e}, db8 {e8:.2e}")
    assert e_pr <= 2e-6 and e_en <= 2e-6 and e_adj <= 1e-6 and e1 <= 2e-6 and e8 <= 2e-6


@pytest.mark.parametrize("prec", [32, 64])
def test_full_size_dictionary_c4(prec):
    """4096^2 in both precisions (the last row synthesis takes two 8-output blocks
    per lane at this size): Psi Psi^dagger x = x, ||Psi^dagger x|| = ||x||, the adjoint identity,
    the db1 slot against the oracle over the whole image, and two prox
    sub-iterations from v = 0 against the same step composed from the checked
    analysis and synthesis: x1 = max(0, z - Psi clip(Psi^dagger max(0, z), +-t))."""
    n = 4096
    ctx = _ctx(n, prec)
    x = synth.sky(n, seed=3, n_compact=64, n_ext=4)
    if prec == 32:
        x = x.astype(np.float32).astype(np.float64)
    xt = torch.tensor(x, dtype=_ft(prec), device=DEV)
    c = torch.empty(9, n, n, dtype=_ft(prec), device=DEV)
    R.ri_sara_analysis(ctx, xt, c)
    xr = torch.empty_like(xt)
    R.ri_sara_synthesis(ctx, c, xr)
    e_pr = rel(xr.cpu().numpy(), x)
    e_en = abs(float(torch.linalg.vector_norm(c.double())) / np.linalg.norm(x) - 1)
    d = torch.randn(9, n, n, dtype=_ft(prec), device=DEV)
    xd = torch.empty_like(xt)
    R.ri_sara_synthesis(ctx, d, xd)
    lhs, rhs = float(torch.sum(c.double() * d.double())), float(torch.sum(xt.double() * xd.double()))
    e_adj = abs(lhs - rhs) / (float(torch.linalg.vector_norm(c.double())) * float(torch.linalg.vector_norm(d.double())))
    e1 = rel(c[1].cpu().numpy(), S.dwt2(x, S.daubechies(1)) / 3)
    del d, xd
    # prox: two sub-iterations from the fresh state (v = 0, w = 1)
    t = 0.3 * float(x.max()) / 3
    R.ri_sara_setup(ctx, 2)
    z = xt - 0.05 * float(x.max())
    out = torch.empty_like(xt)
    R.denoise(ctx, z, out, R.RI_PROX_SARA, t)
    x0 = torch.clamp(z, min=0.0)
    v1 = torch.empty_like(c)
    R.ri_sara_analysis(ctx, x0, v1)
    v1.clamp_(-t, t)
    sv = torch.empty_like(xt)
    R.ri_sara_synthesis(ctx, v1, sv)
    ref = torch.clamp(z - sv, min=0.0)
    e_px = float(torch.linalg.vector_norm((out - ref).double()) / torch.linalg.vector_norm(ref.double()))
    print(f"C4 dictionary FP{prec}: reconstruction {e_pr:.2e}, energy {e_en:.2e}, adjoint {e_adj:.2e}, db1 {e1:.2e}, "
          f"prox step vs composed {e_px:.2e}")
    tol = 2e-6 if prec == 32 else 1e-13
    assert e_pr <= tol and e_en <= tol and e_adj <= (1e-6 if prec == 32 else 1e-13) and e1 <= tol
    assert e_px <= (1e-5 if prec == 32 else 1e-12)
