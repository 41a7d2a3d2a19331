"""Seeded test cases shared by the GPU parity tests: synthetic inputs from
``synth`` plus the FP64 oracle's results on them (never anything from the GPU)."""
from __future__ import annotations

import functools
import math

import numpy as np

import synth
from oracle import fb as OF
from oracle import phi as OP


class Case:
    def __init__(self, name, N, uvw, cell, W, n_wplanes, seed=0, blocks=None):
        self.name, self.N, self.uvw, self.cell, self.W, self.n_wplanes = name, N, uvw, cell, W, n_wplanes
        self.M = uvw.shape[0]
        self.blocks = blocks
        self.op = OP.Operator(N, uvw, cell=cell, W=W, n_wplanes=n_wplanes)
        self.x = synth.sky(N, seed=seed, n_compact=max(4, N // 8), n_ext=2)
        self.xr = synth.random_image(N, seed + 50)
        y0 = self.op.phi(self.x)
        self.tau = OF.tau_from_isnr(y0, 40.0)
        self.y = y0 + OF.complex_noise(self.tau, synth.noise_normals(self.M, synth.SEED_NOISE))

    @functools.cached_property
    def phi_xr(self):
        return self.op.phi(self.xr)

    @functools.cached_property
    def adj_y(self):
        return self.op.phi_adj(self.y)

    @functools.cached_property
    def gram_xr(self):
        return self.op.phi_adj_phi(self.xr)

    @functools.cached_property
    def grad_x(self):
        return self.op.grad(self.xr, self.y)


@functools.lru_cache(maxsize=None)
def wide(N=128):
    """Wide-field case: 16-antenna tracks (M = 11,640), supports 7..17, 257 planes."""
    wl = synth.scaled(synth.T_SMALL_W, N=N)
    uvw = synth.uvw(wl)
    return Case(f"wide{N}", N, uvw, wl.cell_rad, wl.W, wl.n_wplanes)


@functools.lru_cache(maxsize=None)
def edge():
    """Scattered coordinates up to |omega| = 0.999 pi: windows wrap round the grid edge."""
    N, cell = 64, 40 * synth.ARCSEC
    W = 2 * 4.0 / (2 * N * N * cell ** 2)
    uvw = synth.random_uvw(3001, 0.999 * math.pi, W, seed=77)
    return Case("edge64", N, uvw, cell, W, 129, seed=3)


@functools.lru_cache(maxsize=None)
def narrow():
    """The narrow-field FP64 workload: 256^2 sky, 32 antennas, M = 65,472, w = 0."""
    wl = synth.C0
    uvw = synth.uvw(wl)
    return Case("C0", wl.N, uvw, wl.cell_rad, 0.0, 1)


def rel(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
