"""Seeded synthetic inputs for the imaging workloads.

This module is shared by the FP64 CPU oracle and the GPU path. It only draws
random numbers and lays out test geometry (sky models, antenna layouts, the
earth-rotation uvw tracks, noise draws, block sizes, training patches); it holds
none of the imaging method's arithmetic (no gridding, no interpolation kernel,
no Fourier transform of the measurement operator, no prox).

Units: the visibility coordinates are returned as ``uvw[:, 0:2] = omega`` in
radians per pixel (so that the exact model reads
``y_m = sum_n x_n exp(-i omega_m . n)`` for centred pixel indices n) and
``uvw[:, 2] = w`` in wavelengths.

Seeds (numpy PCG64): sky 0, array 1, noise 2, w 3, blocks 4, training 5,
power-method start 7.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_SKY = 0
SEED_ARRAY = 1
SEED_NOISE = 2
SEED_W = 3
SEED_BLOCKS = 4
SEED_TRAIN = 5
SEED_POWER = 7

ARCSEC = math.pi / (180.0 * 3600.0)


# ----------------------------------------------------------------------------
# Workload descriptions (numbers only)
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    N: int                      # image side
    n_ant: int                  # antennas
    n_times: int                # time steps of the track
    omega_max: float            # max |omega| (rad/pixel) after scaling
    cell_rad: float             # pixel size delta (rad), used by the w-term
    w_mode: str                 # "zero" | "uniform"
    w_hex_max: float = 0.0      # per-axis chirp half-bandwidth (cells) at |w| = W
    n_wplanes: int = 1          # odd; w = 0 is the centre plane
    dec_deg: float = -60.0
    lat_deg: float = -30.7
    hours: float = 8.0
    isnr_db: float = 40.0
    n_blocks: int = 1
    block_lo: int = 0
    block_hi: int = 0
    # frequency of each channel over the reference frequency at which omega_max
    # and W are quoted; one channel is the uv track scaled by its ratio
    # (omega and w in wavelengths both scale with frequency)
    channels: tuple = (1.0,)
    extra: dict = field(default_factory=dict)

    @property
    def Np(self) -> int:
        return 2 * self.N

    @property
    def M(self) -> int:
        return self.n_ant * (self.n_ant - 1) // 2 * self.n_times * len(self.channels)

    @property
    def W(self) -> float:
        """|w| bound (wavelengths) at which the per-axis chirp half-bandwidth at
        the image edge equals ``w_hex_max`` grid cells (hex = w sigma N^2 delta^2 / 2)."""
        if self.w_mode == "zero":
            return 0.0
        return 2.0 * self.w_hex_max / (2.0 * self.N * self.N * self.cell_rad ** 2)


# Plain FB, narrow field, FP64 (w = 0).
C0 = Workload("C0-narrow-256", N=256, n_ant=32, n_times=132,
              omega_max=2 * math.pi / 3, cell_rad=1.68 * ARCSEC, w_mode="zero")
# Wide-field operator bench: 2048^2 image, 4096^2 grid, M = 16,777,152,
# w uniform in [-W, W] with supports 11..17 (7 at w = 0).
C1 = Workload("C1-wide-2048", N=2048, n_ant=64, n_times=8322,
              omega_max=2 * math.pi / 3, cell_rad=1.68 * ARCSEC, w_mode="uniform",
              w_hex_max=4.0, n_wplanes=4097)
# C1 data cut into 64 uneven angular-sector blocks.
C2 = Workload("C2-blocks-2048", N=2048, n_ant=64, n_times=8322,
              omega_max=2 * math.pi / 3, cell_rad=1.68 * ARCSEC, w_mode="uniform",
              w_hex_max=4.0, n_wplanes=4097, n_blocks=64,
              block_lo=50_000, block_hi=2_000_000)

# Small wide-field cases for parity tests (several tiles plus a ragged tail).
T_SMALL_W = Workload("T-wide-128", N=128, n_ant=16, n_times=97,
                     omega_max=2 * math.pi / 3, cell_rad=20 * ARCSEC, w_mode="uniform",
                     w_hex_max=4.0, n_wplanes=257)

# Full scale: 4096^2 image, 8192^2 grid, one 64-antenna track of 12,400 steps
# as two channels at 1053 and 1399 MHz (max |omega| = pi/1.6 and W quoted at
# 1399 MHz), M = 49,996,800, 128 uneven angular-sector blocks, 64 facets of
# 512^2 cores (32 px CNN halo, 16 px Haar halo).
C4 = Workload("C4-full-4096", N=4096, n_ant=64, n_times=12400,
              omega_max=math.pi / 1.6, cell_rad=1.68 * ARCSEC, w_mode="uniform",
              w_hex_max=4.0, n_wplanes=4097, n_blocks=128,
              block_lo=50_000, block_hi=2_000_000, channels=(1053.0 / 1399.0, 1.0),
              extra={"freqs_mhz": (1053.0, 1399.0), "facet_core": 512, "facet_halo": 32})

WORKLOADS = {w.name: w for w in (C0, C1, C2, C4, T_SMALL_W)}


def scaled(base: Workload, **kw) -> Workload:
    """A copy of ``base`` with some fields replaced (used for small test cases)."""
    d = dict(base.__dict__)
    d.update(kw)
    return Workload(**d)


# C1's geometry with a four times larger w range: the per-axis chirp at the
# image edge spans 16 grid cells at |w| = W (57,503 wavelengths), beyond any
# 17 x 17 w-kernel; the w-stacking hybrid's workload.
C1W = scaled(C1, name="C1W-wide-2048-w16", w_hex_max=16.0)
WORKLOADS[C1W.name] = C1W


# ----------------------------------------------------------------------------
# Sky
# ----------------------------------------------------------------------------
def sky(N: int, seed: int = SEED_SKY, n_compact: int = 30, n_ext: int = 2) -> np.ndarray:
    """Positive test sky, float64 [N, N] indexed [iy, ix].

    ``n_compact`` round Gaussians (FWHM ~ U[1,3] px, peak 10^U[-4,0], centres
    U[16, N-16)^2) plus ``n_ext`` elliptical Gaussians (FWHM_a, FWHM_b ~
    U[20,40] px, angle U[0,pi), peak 10^U[-3,-2], centres U[N/4, 3N/4)^2).
    """
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:N, 0:N].astype(np.float64)
    img = np.zeros((N, N))
    k = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))   # FWHM -> sigma
    for _ in range(n_compact):
        fwhm = rng.uniform(1.0, 3.0)
        peak = 10.0 ** rng.uniform(-4.0, 0.0)
        cy, cx = rng.uniform(16, N - 16, size=2)
        s = fwhm * k
        r = 4.0 * s + 2.0
        y0, y1 = int(max(0, cy - r)), int(min(N, cy + r + 1))
        x0, x1 = int(max(0, cx - r)), int(min(N, cx + r + 1))
        sub = (yy[y0:y1, x0:x1] - cy) ** 2 + (xx[y0:y1, x0:x1] - cx) ** 2
        img[y0:y1, x0:x1] += peak * np.exp(-sub / (2 * s * s))
    for _ in range(n_ext):
        fa, fb = rng.uniform(20.0, 40.0, size=2)
        ang = rng.uniform(0.0, math.pi)
        peak = 10.0 ** rng.uniform(-3.0, -2.0)
        cy, cx = rng.uniform(N / 4, 3 * N / 4, size=2)
        sa, sb = fa * k, fb * k
        c, s_ = math.cos(ang), math.sin(ang)
        dx, dy = xx - cx, yy - cy
        a = c * dx + s_ * dy
        b = -s_ * dx + c * dy
        img += peak * np.exp(-(a * a) / (2 * sa * sa) - (b * b) / (2 * sb * sb))
    return img


def random_image(N: int, seed: int, positive: bool = True) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x = rng.random((N, N)) if positive else rng.standard_normal((N, N))
    return x


def training_patches(n: int, size: int, seed: int = SEED_TRAIN) -> np.ndarray:
    """Denoiser training images, float32 [n, size, size], positive, with the
    statistics of ``sky`` at patch scale and an adaptive peak.

    Per patch: Poisson(8) + 1 round compact sources (FWHM ~ U[1,3] px, peak
    10^U[-4,0], centres U[0, size)^2), Poisson(1.5) elliptical Gaussians
    (FWHM ~ U[4,40] px per axis, angle U[0,pi), peak 10^U[-3.5,-1.5], centres
    U[0, size)^2); the patch is then scaled so that its peak is 10^U[-1,0]
    (peak values upper-bounded by 1, dynamic range varying from patch to patch).
    """
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:size, 0:size].astype(np.float64)
    k = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    out = np.zeros((n, size, size), dtype=np.float32)
    for i in range(n):
        img = np.zeros((size, size))
        for _ in range(rng.poisson(8.0) + 1):
            s = rng.uniform(1.0, 3.0) * k
            peak = 10.0 ** rng.uniform(-4.0, 0.0)
            cy, cx = rng.uniform(0, size, size=2)
            img += peak * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * s * s))
        for _ in range(rng.poisson(1.5)):
            sa, sb = rng.uniform(4.0, 40.0, size=2) * k
            ang = rng.uniform(0.0, math.pi)
            peak = 10.0 ** rng.uniform(-3.5, -1.5)
            cy, cx = rng.uniform(0, size, size=2)
            c, s_ = math.cos(ang), math.sin(ang)
            a = c * (xx - cx) + s_ * (yy - cy)
            b = -s_ * (xx - cx) + c * (yy - cy)
            img += peak * np.exp(-(a * a) / (2 * sa * sa) - (b * b) / (2 * sb * sb))
        out[i] = img * (10.0 ** rng.uniform(-1.0, 0.0) / img.max())
    return out


def _grf_chunk(seed_seq, count: int, size: int, log_k: np.ndarray, dynamic_range: float) -> np.ndarray:
    rng = np.random.default_rng(seed_seq)
    beta = rng.uniform(2.0, 4.0, size=(count, 1, 1)).astype(np.float32)
    amp = np.exp(-0.5 * beta * log_k)              # |spectrum| = k^(-beta/2): power ~ k^-beta
    amp[:, 0, 0] = 0.0
    shape = (count, size, size // 2 + 1)
    spec = rng.standard_normal(shape, dtype=np.float32) * amp \
        + 1j * (rng.standard_normal(shape, dtype=np.float32) * amp)
    g = np.fft.irfft2(spec, s=(size, size), axes=(1, 2))
    lo = g.min(axis=(1, 2), keepdims=True)
    hi = g.max(axis=(1, 2), keepdims=True)
    g = (g - lo) / (hi - lo)                       # rescaled to [0, 1]
    u = np.expm1(g * np.float32(math.log(dynamic_range))) / np.float32(dynamic_range - 1.0)
    for i in range(count):
        npt = int(rng.integers(0, 21))
        ys, xs = rng.integers(0, size, npt), rng.integers(0, size, npt)
        np.add.at(u[i], (ys, xs), (10.0 ** rng.uniform(-4.0, 0.0, npt)).astype(np.float32))
    u /= u.max(axis=(1, 2), keepdims=True)
    return u.astype(np.float32)


def grf_patches(n: int, size: int, seed: int = SEED_TRAIN, dynamic_range: float = 1e4,
                workers: int | None = None) -> np.ndarray:
    """High-dynamic-range training images, float32 [n, size, size], positive,
    peak 1 (the normalised database of the learned denoiser's training).

    Per patch: a Gaussian random field g with power spectrum ~ k^-beta,
    beta ~ U[2, 4], rescaled to [0, 1], exponentiated as
    u = (D^g - 1) / (D - 1) with D the dynamic range (1e4), plus 0..20 point
    sources (uniform integer positions, peaks 10^U[-4, 0]); the patch is then
    divided by its peak. Chunks of 250 patches draw from independent child
    seeds of ``seed`` (numpy SeedSequence.spawn), so the result does not
    depend on ``workers`` (threads; default min(16, cpu count))."""
    from concurrent.futures import ThreadPoolExecutor
    import os
    ky = np.fft.fftfreq(size)[:, None]
    kx = np.fft.rfftfreq(size)[None, :]
    k = np.hypot(ky, kx)
    k[0, 0] = 1.0
    log_k = np.log(k).astype(np.float32)
    chunk = 250
    starts = list(range(0, n, chunk))
    seqs = np.random.SeedSequence(seed).spawn(len(starts))
    out = np.empty((n, size, size), dtype=np.float32)
    nw = workers or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max(1, nw)) as ex:
        jobs = ex.map(lambda a: _grf_chunk(a[1], min(chunk, n - a[0]), size, log_k, dynamic_range),
                      zip(starts, seqs))
        for s0, u in zip(starts, jobs):
            out[s0:s0 + u.shape[0]] = u
    return out


# ----------------------------------------------------------------------------
# Array geometry and earth-rotation synthesis (Thompson-Moran-Swenson)
# ----------------------------------------------------------------------------
def antenna_enu(n_ant: int, radius: float = 1.0, seed: int = SEED_ARRAY) -> np.ndarray:
    """Antennas uniform in a disk on the ground: r = R sqrt(U), theta = 2 pi U."""
    rng = np.random.default_rng(seed)
    r = radius * np.sqrt(rng.random(n_ant))
    th = 2 * math.pi * rng.random(n_ant)
    enu = np.zeros((n_ant, 3))
    enu[:, 0] = r * np.cos(th)
    enu[:, 1] = r * np.sin(th)
    return enu


def baseline_uvw(enu: np.ndarray, n_times: int, dec_deg: float, lat_deg: float,
                 hours: float) -> np.ndarray:
    """uvw (same length unit as ``enu``) for all baselines i<j over hour angles
    H in [-hours/2, +hours/2] (n_times steps). Order: time-major within each
    baseline, baselines in (i, j) lexicographic order."""
    i, j = np.triu_indices(enu.shape[0], k=1)
    b = enu[j] - enu[i]                                      # E, N, U
    lat = math.radians(lat_deg)
    X = -math.sin(lat) * b[:, 1] + math.cos(lat) * b[:, 2]
    Y = b[:, 0]
    Z = math.cos(lat) * b[:, 1] + math.sin(lat) * b[:, 2]
    H = np.linspace(-hours / 2, hours / 2, n_times) * (2 * math.pi / 24.0)
    d = math.radians(dec_deg)
    sH, cH = np.sin(H)[None, :], np.cos(H)[None, :]
    u = sH * X[:, None] + cH * Y[:, None]
    v = -math.sin(d) * cH * X[:, None] + math.sin(d) * sH * Y[:, None] + math.cos(d) * Z[:, None]
    w = math.cos(d) * cH * X[:, None] - math.cos(d) * sH * Y[:, None] + math.sin(d) * Z[:, None]
    return np.stack([u.ravel(), v.ravel(), w.ravel()], axis=1)


def uvw(wl: Workload) -> np.ndarray:
    """Visibility coordinates for a workload: float64 [M, 3] = (omega_u, omega_v
    in rad/pixel, w in wavelengths). Several channels are stacked channel by
    channel, each the reference track scaled by its frequency ratio."""
    enu = antenna_enu(wl.n_ant)
    b = baseline_uvw(enu, wl.n_times, wl.dec_deg, wl.lat_deg, wl.hours)
    rad = np.sqrt(b[:, 0] ** 2 + b[:, 1] ** 2).max()
    ref = np.empty_like(b)
    ref[:, 0:2] = b[:, 0:2] * (wl.omega_max / rad)
    del b
    if wl.w_mode == "zero":
        ref[:, 2] = 0.0
    elif wl.w_mode == "uniform":
        rng = np.random.default_rng(SEED_W)
        ref[:, 2] = rng.uniform(-wl.W, wl.W, size=ref.shape[0])
    else:
        raise ValueError(wl.w_mode)
    if tuple(wl.channels) == (1.0,):
        return ref
    n = ref.shape[0]
    out = np.empty((n * len(wl.channels), 3))
    for k, f in enumerate(wl.channels):
        np.multiply(ref, f, out=out[k * n:(k + 1) * n])
    return out


def random_uvw(M: int, omega_max: float, W: float, seed: int) -> np.ndarray:
    """Uniformly scattered test coordinates (|omega| < omega_max per axis)."""
    rng = np.random.default_rng(seed)
    out = np.empty((M, 3))
    out[:, 0:2] = rng.uniform(-omega_max, omega_max, size=(M, 2))
    out[:, 2] = rng.uniform(-W, W, size=M) if W > 0 else 0.0
    return out


# ----------------------------------------------------------------------------
# Noise and other random draws
# ----------------------------------------------------------------------------
def noise_normals(M: int, seed: int = SEED_NOISE) -> np.ndarray:
    """Complex draws a + i b with a, b ~ N(0, 1) independent (complex128 [M])."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(M)
    b = rng.standard_normal(M)
    return a + 1j * b


def power_start(N: int, seed: int = SEED_POWER) -> np.ndarray:
    """Start vector of the power iteration: float64 [N, N] standard normal."""
    return np.random.default_rng(seed).standard_normal((N, N))


# ----------------------------------------------------------------------------
# Data blocks: angular sectors of the uv plane with uneven sizes
# ----------------------------------------------------------------------------
def block_sizes(n_blocks: int, M: int, lo: float, hi: float, seed: int = SEED_BLOCKS) -> np.ndarray:
    """Log-uniform sizes in [lo, hi], rescaled to sum exactly to M (int64)."""
    rng = np.random.default_rng(seed)
    s = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_blocks))
    s = s * (M / s.sum())
    out = np.floor(s).astype(np.int64)
    out[np.argsort(-(s - out))[: M - out.sum()]] += 1
    assert out.sum() == M and (out > 0).all()
    return out


def sector_order(uvw_: np.ndarray) -> np.ndarray:
    """Permutation that orders visibilities by polar angle atan2(v, u) (stable)."""
    ang = np.arctan2(uvw_[:, 1], uvw_[:, 0])
    return np.argsort(ang, kind="stable")


def blocked(uvw_: np.ndarray, sizes: np.ndarray):
    """Reorder visibilities into contiguous angular-sector blocks of the given
    sizes. Returns (perm, offsets[n_blocks+1]); uvw_[perm] is in block order."""
    perm = sector_order(uvw_)
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    return perm, offsets
