"""What the learned denoiser gains over the method without it (plain FB with
the Haar-l1 + positivity prox), on the GPU path end to end: the network is
trained by the library's own kernels on synthetic patches, then

* as a denoiser on held-out patches at its training noise level it must beat
  the Haar soft-threshold prox at the same level (eq. B2's threshold);
* inside the forward-backward loop (PnP-FB, eq. A2 with D the network) on a
  small wide-field problem whose rescaled image-domain noise equals the
  training level (eqs. C2-C3) it must reach a higher reconstruction SNR than
  plain FB in the same number of iterations.

The Haar prox is the fallback and the judge: both runs use the same data,
step size and iteration count."""
import math

import numpy as np
import pytest

import synth
from _cases import wide

torch = pytest.importorskip("torch")
import paper_2207_11336_amd.ri as R  # noqa: E402
from paper_2207_11336_amd.train import train_denoiser  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SIGMA = 1e-2


@pytest.fixture(scope="module")
def trained():
    patches = torch.tensor(synth.training_patches(1024, 64, seed=synth.SEED_TRAIN), device=DEV)
    params, hist = train_denoiser(patches, SIGMA, steps=2000, batch=16, lr=1e-3, lr_min=1e-5, log_every=500)
    print("training loss", [(h[0], round(h[1], 6)) for h in hist])
    return params


def _snr(ref, x):
    return 20 * math.log10(np.linalg.norm(ref) / np.linalg.norm(ref - x))


def test_denoiser_beats_haar_on_held_out_patches(trained):
    test = synth.training_patches(16, 64, seed=99)
    noisy = test + SIGMA * np.random.default_rng(5).standard_normal(test.shape)
    net = R.ri_cnn_create(layers=10, max_batch=16, max_h=64, max_w=64)
    R.ri_cnn_set_params(net, trained)
    zt = torch.tensor(noisy, dtype=torch.float32, device=DEV)
    out = torch.empty_like(zt)
    R.ri_cnn_forward(net, zt, out)
    cnn = out.cpu().numpy().astype(np.float64)
    # Haar-l1 + positivity prox at the noise level, through an imaging context of the patch size
    uvw = synth.random_uvw(64, 2.0, 0.0, seed=1)
    ctx = R.ri_create(R.plan_desc(64, 64, precision=32, g_mode=R.RI_G_OTF), uvw)
    haar = np.empty_like(cnn)
    for i in range(test.shape[0]):
        o = torch.empty((64, 64), dtype=torch.float32, device=DEV)
        R.denoise(ctx, zt[i].contiguous(), o, R.RI_PROX_HAAR, SIGMA)
        haar[i] = o.cpu().numpy()
    s_in, s_cnn, s_haar = _snr(test, noisy), _snr(test, cnn), _snr(test, haar)
    print(f"held-out patches at sigma {SIGMA}: input {s_in:.2f} dB, Haar prox {s_haar:.2f} dB, CNN {s_cnn:.2f} dB")
    assert s_cnn > s_in + 6.0
    assert s_cnn > s_haar + 2.0


def test_pnp_reaches_higher_snr_than_fb(trained):
    c = wide()
    x_true = c.x / c.x.max()
    ctx = R.ri_create(R.plan_desc(c.N, c.M, cell_rad=c.cell, w_max=c.W, n_wplanes=c.n_wplanes, precision=32,
                                  g_mode=R.RI_G_OTF), c.uvw)
    xt = torch.tensor(x_true, dtype=torch.float32, device=DEV)
    L, _ = R.ri_power_norm(ctx, 300, 1e-10)
    y0 = torch.empty(c.M, dtype=torch.complex64, device=DEV)
    R.phi_forward(ctx, xt, y0)
    dirty = torch.empty_like(xt)
    R.phi_adjoint(ctx, y0, dirty)
    delta = torch.zeros_like(xt)
    delta[c.N // 2, c.N // 2] = 1.0
    yd = torch.empty_like(y0)
    R.phi_forward(ctx, delta, yd)
    beam = torch.empty_like(xt)
    R.phi_adjoint(ctx, yd, beam)
    alpha0 = float(dirty.max()) / float(beam.max())
    tau = SIGMA * alpha0 * math.sqrt(2 * L)
    noise = torch.tensor(synth.noise_normals(c.M, synth.SEED_NOISE), dtype=torch.complex64, device=DEV)
    y = y0 + noise * (tau / math.sqrt(2))
    R.ri_load_denoiser(ctx, trained, 10)
    K = 300
    res = {}
    for kind in (R.RI_PROX_HAAR, R.RI_PROX_CNN):
        tr = np.zeros((K, 4))
        o = R.ri_solve_opts(max_iter=K, rel_tol=0.0, prox_kind=kind, tau=tau, sigma_train=SIGMA, L=L,
                            check_every=50, x_true=xt.data_ptr(), trace=tr.ctypes.data, use_graph=1)
        xo = torch.empty_like(xt)
        rep = R.pnp_solve(ctx, y, o, xo)
        res[kind] = (rep, tr)
        print(f"{'Haar FB' if kind == R.RI_PROX_HAAR else 'PnP-FB'}: SNR at 50/100/300 its "
              f"{tr[49, 2]:.2f} / {tr[99, 2]:.2f} / {tr[K - 1, 2]:.2f} dB, residual {rep.final_residual2:.4e}, "
              f"fell back {rep.fell_back}, {rep.ms:.1f} ms")
    fb, pnp = res[R.RI_PROX_HAAR][0], res[R.RI_PROX_CNN][0]
    assert pnp.fell_back == 0
    assert pnp.snr_db > fb.snr_db + 1.0
