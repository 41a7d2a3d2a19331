"""Training driver of the residual CNN denoiser (paper appendix C, eq. C1:
minimise E||D(u + sigma n) - u||_1 over clean images u and Gaussian noise n).

Every step runs in libri.so's kernels: ri_cnn_sample_batch draws the batch
from the clean patches resident on the GPU (random patches in random
orientations: the training images have no preferred orientation), then
ri_cnn_train_step (noise draw, forward, l1 loss gradient, backward, Adam
update). This module only sets the seeds and the learning rate (cosine
decay).
"""
from __future__ import annotations

import math
import time

from . import ri as R


def train_denoiser(patches, sigma: float, steps: int = 2000, batch: int = 16, lr: float = 1e-3,
                   lr_min: float = 1e-5, layers: int = 10, seed: int = 5, log_every: int = 0, log=None,
                   fne_lambda: float = 0.0, fne_eps: float = 0.05, fne_iters: int = 2, fne_every: int = 1,
                   fne_point: int = 0):
    """Train a fresh network on ``patches`` (float32 GPU tensor [n, s, s], s a
    multiple of 16) at noise level ``sigma``. Returns (params, history) with
    params the FP32 GPU parameter vector (ri_cnn layout) and history a list of
    (step, loss, seconds, squared Jacobian-norm estimate or None).

    fne_lambda > 0 adds the relaxed firm-nonexpansiveness penalty
    fne_lambda max(||J_{2D - I}||_S^2, 1 - fne_eps) every fne_every steps
    (fne_iters warm-started power iterations per penalised step), the Jacobian
    taken at the noisy inputs (fne_point 0) or at random points between the
    clean and the denoised images (fne_point 1)."""
    import torch
    n, s, s2 = patches.shape
    if s != s2 or s % 16:
        raise ValueError("patches must be square with a side multiple of 16")
    dev = patches.device
    net = R.ri_cnn_create(layers=layers, max_batch=batch, max_h=s, max_w=s, training=True, seed=seed)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    fsq = torch.zeros(1, dtype=torch.float64, device=dev)
    buf = torch.empty((batch, s, s), dtype=torch.float32, device=dev)
    hist = []
    t0 = time.perf_counter()
    for it in range(steps):
        R.ri_cnn_sample_batch(net, patches, int(seed) * 7_000_003 + it, buf)
        rate = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * it / max(1, steps)))
        fne_step = fne_lambda > 0 and it % fne_every == 0
        if fne_step:
            R.ri_cnn_train_step_fne(net, buf, sigma, int(seed) * 1_000_003 + it, rate, fne_lambda, fne_eps, fne_iters,
                                    loss, fsq, point=fne_point)
        else:
            R.ri_cnn_train_step(net, buf, sigma, int(seed) * 1_000_003 + it, rate, loss)
        if log_every and (it % log_every == 0 or it == steps - 1):
            hist.append((it, float(loss.item()), time.perf_counter() - t0,
                         float(fsq.item()) if fne_lambda > 0 else None))
            if log:
                extra = f", ||J||^2 {hist[-1][3]:.3f}" if fne_lambda > 0 else ""
                log(f"train step {it}: loss {hist[-1][1]:.4e}{extra} ({hist[-1][2]:.1f} s)")
    params = torch.empty(net.n_params, dtype=torch.float32, device=dev)
    R.ri_cnn_get_params(net, params)
    torch.cuda.synchronize()
    net.close()
    return params, hist
