"""GPU parity of the holographic matrices (appendix E: Phi^dagger Phi =
Z^dagger F^dagger H F Z with H = sum_p G_p^H G_p): the stored H applied to
random grids against the FP64 oracle's sparse G^H G, the normal operator
through H against the oracle and against the GPU's own pass over the
visibilities, the storage figures against a host recount of the plan, and the
edge cases (no visibilities, no w-term, blocks, w-stacking refused)."""
import math

import numpy as np
import pytest

import synth
from _cases import rel
from oracle import holo as HO
from oracle import phi as OP

torch = pytest.importorskip("torch")
import paper_2207_11336_amd.ri as R  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
N = 64
CELL = 60 * synth.ARCSEC
NPL = 129


def _W(hex_cells, n=N):
    return 2 * hex_cells / (2.0 * n * n * CELL ** 2)


@pytest.fixture(scope="module")
def case():
    W = _W(4.0)
    M = 3001
    uvw = synth.random_uvw(M, 0.97 * math.pi, W, seed=41)
    op = OP.Operator(N, uvw, cell=CELL, W=W, n_wplanes=NPL)
    return W, uvw, op, HO.holographic(op)


def _ctx(uvw, W, prec, n_blocks=1, offs=None, wstacks=0, n=N):
    d = R.plan_desc(n, uvw.shape[0], cell_rad=CELL, w_max=W, n_wplanes=NPL, precision=prec, g_mode=R.RI_G_OTF,
                    n_blocks=n_blocks, n_wstacks=wstacks)
    return R.ri_create(d, uvw, block_offsets=offs)


def _types(prec):
    return (torch.float64, torch.complex128) if prec == 64 else (torch.float32, torch.complex64)


def _reach_recount(ctx, n):
    """Tiles, stored entries and build pairs recomputed on the host from the plan arrays."""
    cu, cv, pl, ph = R.ri_get_plan_arrays(ctx)
    Np = 2 * n
    h = ph[pl].astype(np.int64)
    S = 2 * h + 7
    ntx = Np // 32
    reach = np.full(ntx * ntx, -1, dtype=np.int64)
    for a in (-1, 1):
        for b in (-1, 1):
            t = (((cv + a * (h + 3)) % Np) // 32) * ntx + ((cu + b * (h + 3)) % Np) // 32
            np.maximum.at(reach, t, S - 1)
    r = reach[reach >= 0]
    return r.size, int(((r + 1) * (2 * r + 1) * 1024).sum()), int((S * S * (S * S + 1) // 2).sum()), int(r.max())


@pytest.mark.parametrize("prec", [64, 32])
def test_apply_matches_oracle(case, prec):
    W, uvw, op, H = case
    ctx = _ctx(uvw, W, prec)
    R.ri_holo_build(ctx)
    _, ct = _types(prec)
    rng = np.random.default_rng(7)
    Np = 2 * N
    for trial in range(2):
        X = rng.standard_normal((Np, Np)) + 1j * rng.standard_normal((Np, Np))
        if prec == 32:
            X = X.astype(np.complex64).astype(np.complex128)
        Xt = torch.tensor(X, dtype=ct, device=DEV)
        Yt = torch.full_like(Xt, 3.0)          # overwritten, not accumulated
        R.ri_holo_apply(ctx, Xt, Yt)
        ref = HO.apply(H, X)
        e = rel(Yt.cpu().numpy(), ref)
        print(f"FP{prec} trial {trial}: H X against the oracle's G^H G: {e:.2e}")
        # H's entries sum w-kernel products that cancel, accumulated in another
        # order than the oracle's sparse product: FP64 agrees to about 1e-13
        assert e <= (1e-12 if prec == 64 else 2e-6)


@pytest.mark.parametrize("prec", [64, 32])
def test_normal_matches_oracle_and_the_visibility_pass(case, prec):
    W, uvw, op, H = case
    ctx = _ctx(uvw, W, prec)
    R.ri_holo_build(ctx)
    ft, ct = _types(prec)
    x = synth.sky(N, seed=6, n_compact=8, n_ext=1) + 0.1 * synth.random_image(N, 7)
    if prec == 32:
        x = x.astype(np.float32).astype(np.float64)
    xt = torch.tensor(x, dtype=ft, device=DEV)
    out = torch.empty_like(xt)
    R.ri_holo_normal(ctx, xt, out)
    y = torch.empty(uvw.shape[0], dtype=ct, device=DEV)
    R.phi_forward(ctx, xt, y)
    ref_gpu = torch.empty_like(xt)
    R.phi_adjoint(ctx, y, ref_gpu)
    g = torch.empty_like(xt)
    R.ri_gradient(ctx, xt, "none", g)
    ref = op.phi_adj_phi(x)
    e_o, e_g, e_f = rel(out.cpu().numpy(), ref), rel(out.cpu().numpy(), ref_gpu.cpu().numpy()), \
        rel(out.cpu().numpy(), g.cpu().numpy())
    print(f"FP{prec}: Re Z^H F^H H F Z x against the oracle {e_o:.2e}, against G^H (G x) on the GPU {e_g:.2e}, "
          f"against the fused pass {e_f:.2e}")
    tol = 1e-12 if prec == 64 else 1e-5
    assert e_o <= tol and e_g <= tol and e_f <= tol


def test_storage_matches_the_plan(case):
    W, uvw, _, _ = case
    ctx = _ctx(uvw, W, 32)
    R.ri_holo_build(ctx)
    s = R.ri_holo_get_stats(ctx)
    tiles, entries, pairs, rmax = _reach_recount(ctx, N)
    print(f"tiles {s.tiles}, entries {s.entries}, bytes {s.bytes}, pairs {s.pairs}, reach {s.max_reach}, "
          f"build {s.build_ms:.1f} ms")
    assert (s.tiles, s.entries, s.pairs, s.max_reach) == (tiles, entries, pairs, rmax)
    assert s.bytes == 8 * entries
    R.ri_holo_release(ctx)
    assert R.ri_holo_get_stats(ctx).entries == 0
    with pytest.raises(R.RIError):
        R.ri_holo_normal(ctx, torch.zeros(N, N, device=DEV), torch.empty(N, N, device=DEV))


def test_blocks_give_the_same_matrix(case):
    """sum_p H_p over uneven blocks (eq. E2) is the same H."""
    W, uvw, _, _ = case
    offs = np.array([0, 500, 2200, 3001], dtype=np.int64)
    c1, c3 = _ctx(uvw, W, 64), _ctx(uvw, W, 64, n_blocks=3, offs=offs)
    R.ri_holo_build(c1)
    R.ri_holo_build(c3)
    X = torch.randn(2 * N, 2 * N, dtype=torch.complex128, device=DEV)
    Y1, Y3 = torch.empty_like(X), torch.empty_like(X)
    R.ri_holo_apply(c1, X, Y1)
    R.ri_holo_apply(c3, X, Y3)
    assert rel(Y3.cpu().numpy(), Y1.cpu().numpy()) <= 1e-14


def test_no_w_term_and_no_visibilities():
    """w = 0 everywhere (7 x 7 windows, band reach 6) against the oracle; and an
    empty data set: H = 0, normal = 0."""
    n = 32
    uvw = synth.random_uvw(700, 0.9 * math.pi, 0.0, seed=3)
    op = OP.Operator(n, uvw)
    H = HO.holographic(op)
    d = R.plan_desc(n, 700, precision=64, g_mode=R.RI_G_OTF)
    ctx = R.ri_create(d, uvw)
    R.ri_holo_build(ctx)
    assert R.ri_holo_get_stats(ctx).max_reach == 6
    X = np.random.default_rng(2).standard_normal((2 * n, 2 * n)) + 0j
    Y = torch.empty(2 * n, 2 * n, dtype=torch.complex128, device=DEV)
    R.ri_holo_apply(ctx, torch.tensor(X, device=DEV), Y)
    assert rel(Y.cpu().numpy(), HO.apply(H, X)) <= 1e-12
    e = R.ri_create(R.plan_desc(n, 0, precision=64, g_mode=R.RI_G_OTF), np.zeros((0, 3)))
    R.ri_holo_build(e)
    assert R.ri_holo_get_stats(e).tiles == 0
    x = torch.ones(n, n, dtype=torch.float64, device=DEV)
    out = torch.full_like(x, 5.0)
    R.ri_holo_normal(e, x, out)
    assert float(out.abs().max()) == 0.0


def test_wstacking_is_refused(case):
    W, uvw, _, _ = case
    ctx = _ctx(uvw, W, 32, wstacks=2)
    with pytest.raises(R.RIError) as ei:
        R.ri_holo_build(ctx)
    assert ei.value.status == -4


def test_full_size_normal_through_h():
    """C1 (2048^2 image, 16.8 M visibilities, FP32): Re{Phi^dagger Phi} x through
    the stored H against the pass over the visibilities (the fused gradient
    with y = 0), over the whole image, and H's storage against the host
    recount of the plan."""
    wl = synth.C1
    uvw = synth.uvw(wl)
    ctx = R.ri_create(R.plan_desc(wl.N, wl.M, cell_rad=wl.cell_rad, w_max=wl.W, n_wplanes=wl.n_wplanes,
                                  precision=32, g_mode=R.RI_G_OTF), uvw)
    R.ri_holo_build(ctx)
    s = R.ri_holo_get_stats(ctx)
    tiles, entries, pairs, rmax = _reach_recount(ctx, wl.N)
    print(f"C1 H: {s.tiles} tiles, {s.bytes / 1e9:.2f} GB, reach {s.max_reach}, {s.pairs:.3g} pairs, "
          f"build {s.build_ms:.0f} ms")
    assert (s.tiles, s.entries, s.pairs) == (tiles, entries, pairs)
    x = torch.tensor(synth.sky(wl.N).astype(np.float32), device=DEV)
    out = torch.empty_like(x)
    R.ri_holo_normal(ctx, x, out)
    g = torch.empty_like(x)
    R.ri_gradient(ctx, x, "none", g)
    e = rel(out.cpu().numpy(), g.cpu().numpy())
    print(f"C1: normal through H against the visibility pass {e:.2e}")
    assert e <= 1e-5
    R.ri_holo_release(ctx)


@pytest.mark.parametrize("prec,graph", [(64, 1), (64, 0), (32, 1)])
def test_solve_through_h_matches_the_visibility_solve(case, prec, graph):
    """pnp_solve with use_holo: FB (Haar) iterations whose gradients come from the
    stored H reach the same iterates, residuals and SNR trace as the solve over the
    visibilities."""
    from oracle import fb as OF
    W, uvw, op, _ = case
    x_true = synth.sky(N, seed=7, n_compact=8, n_ext=1)
    y0 = op.phi(x_true)
    tau = OF.tau_from_isnr(y0, 30.0)
    y = y0 + OF.complex_noise(tau, synth.noise_normals(uvw.shape[0], synth.SEED_NOISE))
    ft, ct = _types(prec)
    ctx = _ctx(uvw, W, prec)
    R.ri_holo_build(ctx)
    yt = torch.tensor(y, dtype=ct, device=DEV)
    xt = torch.tensor(x_true, dtype=ft, device=DEV)
    L, _ = R.ri_power_norm(ctx, max_it=300, rtol=1e-10)
    out, tr = {}, {}
    for use_holo in (0, 1):
        trace = np.zeros((40, 4))
        opts = R.ri_solve_opts(max_iter=40, rel_tol=0.0, prox_kind=R.RI_PROX_HAAR, tau=tau, L=L, check_every=10,
                               x_true=xt.data_ptr(), trace=trace.ctypes.data, use_graph=graph, use_holo=use_holo)
        xs = torch.empty(N, N, dtype=ft, device=DEV)
        rep = R.pnp_solve(ctx, yt, opts, xs)
        assert rep.iters == 40
        out[use_holo], tr[use_holo] = xs.cpu().numpy(), trace
    e_x = rel(out[1], out[0])
    e_r = np.abs(tr[1][:, 1] - tr[0][:, 1]).max() / tr[0][:, 1].max()
    e_snr = np.abs(tr[1][:, 2] - tr[0][:, 2]).max()
    print(f"FP{prec} graph {graph}: x through H vs over the visibilities {e_x:.2e}; residual trace {e_r:.2e}; "
          f"SNR trace {e_snr:.2e} dB (final {tr[1][-1, 2]:.3f} dB)")
    tol_x, tol_r = (1e-11, 1e-9) if prec == 64 else (1e-4, 1e-3)
    assert e_x <= tol_x and e_r <= tol_r and e_snr <= (1e-9 if prec == 64 else 1e-3)


def test_solve_through_h_needs_h(case):
    W, uvw, _, _ = case
    ctx = _ctx(uvw, W, 32)
    opts = R.ri_solve_opts(max_iter=2, prox_kind=R.RI_PROX_HAAR, tau=1.0, L=1.0, check_every=1, use_holo=1)
    with pytest.raises(R.RIError):
        R.pnp_solve(ctx, torch.zeros(uvw.shape[0], dtype=torch.complex64, device=DEV), opts,
                    torch.empty(N, N, device=DEV))


def test_pnp_solve_through_h_with_the_cnn(case):
    """PnP-FB (random He-normal CNN, facets; FP64 context) through H and over the
    visibilities: the same rescaling alpha and, over four graph-replayed
    iterations, the same iterates. FP64 keeps the two paths' differences far below
    the BF16 rounding steps inside the network, so the iterates agree closely."""
    from oracle import cnn as OC
    from oracle import fb as OF
    W, uvw, op, _ = case
    x_true = synth.sky(N, seed=8, n_compact=8, n_ext=1)
    y0 = op.phi(x_true)
    tau = OF.tau_from_isnr(y0, 30.0)
    y = y0 + OF.complex_noise(tau, synth.noise_normals(uvw.shape[0], synth.SEED_NOISE))
    d = R.plan_desc(N, uvw.shape[0], cell_rad=CELL, w_max=W, n_wplanes=NPL, precision=64, g_mode=R.RI_G_OTF,
                    facet_core=32, facet_halo=10)
    ctx = R.ri_create(d, uvw)
    params = OC.init_params(10, 64, seed=5)
    vec = np.concatenate([np.concatenate([w_.ravel(), b_.ravel()]) for w_, b_ in params]).astype(np.float32)
    R.ri_load_denoiser(ctx, torch.tensor(vec, device=DEV), 10)
    R.ri_holo_build(ctx)
    L, _ = R.ri_power_norm(ctx, max_it=300, rtol=1e-10)
    yt = torch.tensor(y, dtype=torch.complex128, device=DEV)
    out, reps = {}, {}
    for use_holo in (0, 1):
        opts = R.ri_solve_opts(max_iter=4, rel_tol=0.0, prox_kind=R.RI_PROX_CNN, tau=tau, sigma_train=1e-2, L=L,
                               check_every=4, use_graph=1, use_holo=use_holo)
        xs = torch.empty(N, N, dtype=torch.float64, device=DEV)
        reps[use_holo] = R.pnp_solve(ctx, yt, opts, xs)
        out[use_holo] = xs.cpu().numpy()
    e = rel(out[1], out[0])
    print(f"PnP x4 through H vs over the visibilities: {e:.2e}; alpha {reps[1].alpha:.6e} vs {reps[0].alpha:.6e}")
    assert reps[0].fell_back == 0 and reps[1].fell_back == 0
    assert reps[0].iters == 4 and reps[1].iters == 4
    assert reps[1].alpha == pytest.approx(reps[0].alpha, rel=1e-12)
    assert e <= 1e-6
