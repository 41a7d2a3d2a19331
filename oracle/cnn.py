"""FP64 oracle of the residual CNN denoiser and its training gradients
(test infrastructure only).

Paper passages followed: appendix C (a DnCNN-type denoiser D trained with the
l1 loss E||D(u + sigma n) - u||_1 of eq. C1; the relaxed firm-nonexpansiveness
penalty through the Jacobian products below; the optimiser, which the paper
does not name, is Adam), appendix D (the denoiser is applied to
image facets independently thanks to its compact receptive field).

Readings (the paper gives only "a simple DnCNN"): L layers of 3x3
convolutions with zero "same" padding and biases, no batch normalisation,
ReLU after every layer but the last, one input and one output channel,
C hidden channels; D(z) = z - net(z).

Precision points of the GPU path, reproduced when ``bf16=True``: the first
layer computes in full precision from the input, its output (after ReLU) is
rounded to bfloat16; layers 2..L use bfloat16 weights and bfloat16 inputs with
exact accumulation (FP32 on the GPU, FP64 here); hidden activations are
rounded to bfloat16 after each ReLU; the last layer's output and the residual
subtraction stay in full precision. In the backward pass the pre-activation
gradients of layers L-1..1 are rounded to bfloat16 where the GPU stores them.

Parity: the forward convolution is pinned against scipy.signal.correlate2d,
the analytic gradients against central finite differences in FP64, Adam
against a hand-computed three-step example and the constant-gradient closed
form (tests/test_oracle_cnn.py).
"""
from __future__ import annotations

import numpy as np


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """out[b,o,i,j] = bias[o] + sum_{c,dy,dx} w[o,c,dy,dx] x[b,c,i+dy-1,j+dx-1] (zero outside)."""
    B, C, H, W = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    out = np.empty((B, w.shape[0], H, W))
    out[:] = b[None, :, None, None]
    for dy in range(3):
        for dx in range(3):
            out += np.einsum("oc,bchw->bohw", w[:, :, dy, dx], xp[:, :, dy:dy + H, dx:dx + W], optimize=True)
    return out


def conv3x3_backward(x: np.ndarray, w: np.ndarray, dout: np.ndarray, need_dx: bool = True):
    """Gradients of sum(dout * conv3x3(x, w, b)): (dx, dw, db).
    dw[o,c,dy,dx] = sum dout[b,o,i,j] x[b,c,i+dy-1,j+dx-1];
    dx[b,c,i,j] = sum_{o,dy,dx} w[o,c,dy,dx] dout[b,o,i-dy+1,j-dx+1]."""
    B, C, H, W = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    dw = np.empty_like(w, dtype=np.float64)
    for dy in range(3):
        for dx in range(3):
            dw[:, :, dy, dx] = np.einsum("bohw,bchw->oc", dout, xp[:, :, dy:dy + H, dx:dx + W], optimize=True)
    db = dout.sum(axis=(0, 2, 3))
    dxv = None
    if need_dx:
        dp = np.pad(dout, ((0, 0), (0, 0), (1, 1), (1, 1)))
        dxv = np.zeros_like(x, dtype=np.float64)
        for dy in range(3):
            for dx in range(3):
                # dout at (i - dy + 1, j - dx + 1) sits at padded index (i - dy + 2, j - dx + 2)
                dxv += np.einsum("oc,bohw->bchw", w[:, :, dy, dx],
                                 dp[:, :, 2 - dy:2 - dy + H, 2 - dx:2 - dx + W], optimize=True)
    return dxv, dw, db


def init_params(layers: int = 10, channels: int = 64, seed: int = 0):
    """He-normal weights, zero biases (same recipe as the GPU trainer)."""
    rng = np.random.default_rng(seed)
    params = []
    for l in range(layers):
        ci = 1 if l == 0 else channels
        co = 1 if l == layers - 1 else channels
        std = np.sqrt(2.0 / (9 * ci))
        params.append((rng.standard_normal((co, ci, 3, 3)) * std, np.zeros(co)))
    return params


def forward(params, z: np.ndarray, bf16: bool = False, mask: np.ndarray | None = None):
    """D(z) = z - net(z) for z [B, H, W]. Returns (D, cache).
    mask [B, H, W] (optional): positions outside it are zero after every hidden
    layer, as zero "same" padding at the image edge requires when a facet's
    halo extends beyond the image."""
    x = z[:, None].astype(np.float64)
    m = None if mask is None else mask[:, None].astype(np.float64)
    acts = [x if m is None else x * m]
    L = len(params)
    h = acts[0]
    for l, (w, b) in enumerate(params):
        wl = bf16_round(w) if (bf16 and l > 0) else w
        pre = conv3x3(h, wl, b)
        if l < L - 1:
            h = np.maximum(pre, 0.0)
            if m is not None:
                h = h * m
            if bf16:
                h = bf16_round(h)
        else:
            h = pre
        acts.append(h)
    out = acts[-1][:, 0]
    return z - out, acts


def backward(params, acts, d_out: np.ndarray, bf16: bool = False):
    """Gradients of sum(g * net(z)) for g = d_out [B, H, W] (so for D = z - net,
    pass d_out = -dL/dD). Returns [(dw, db)] per layer."""
    L = len(params)
    grads = [None] * L
    g = d_out[:, None].astype(np.float64)
    for l in range(L - 1, -1, -1):
        w, _ = params[l]
        wl = bf16_round(w) if (bf16 and l > 0) else w
        dxv, dw, db = conv3x3_backward(acts[l], wl, g, need_dx=l > 0)
        grads[l] = (dw, db)
        if l > 0:
            g = dxv * (acts[l] > 0)          # ReLU of layer l (acts[l] is post-ReLU)
            if bf16:
                g = bf16_round(g)
    return grads


def l1_loss(D: np.ndarray, u: np.ndarray) -> float:
    """mean |D - u| (eq. C1 without the firm-nonexpansiveness term)."""
    return float(np.mean(np.abs(D - u)))


def l1_dnet(D: np.ndarray, u: np.ndarray) -> np.ndarray:
    """d loss / d net(z) for D = z - net(z): -sign(D - u) / numel."""
    return -np.sign(D - u) / D.size


def adam_step(p: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, t: int, lr: float,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma and Ba 2015), the optimiser of the training
    (the paper names none; this reading is the build's). With the moment
    estimates m, v (zero before the first step) and the step count t >= 1:
      m <- beta1 m + (1 - beta1) g,  v <- beta2 v + (1 - beta2) g^2,
      p <- p - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps).
    Returns (p, m, v) as new arrays."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def flatten_params(params) -> np.ndarray:
    """The parameter vector in the library's layout: per layer W[c_out][c_in][3][3], then b[c_out]."""
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def unflatten_params(vec: np.ndarray, like) -> list:
    out, o = [], 0
    for w, b in like:
        nw, nb = w.size, b.size
        out.append((vec[o:o + nw].reshape(w.shape).copy(), vec[o + nw:o + nw + nb].copy()))
        o += nw + nb
    return out


def denoise_facets(params, z: np.ndarray, core: int, halo: int, bf16: bool = False) -> np.ndarray:
    """Apply D facet by facet (appendix D): each core x core facet is processed
    with a zero-padded halo and only its core is kept."""
    N = z.shape[0]
    out = np.empty_like(z, dtype=np.float64)
    zp = np.pad(z, halo)
    inside = np.pad(np.ones_like(z, dtype=bool), halo)
    for y0 in range(0, N, core):
        for x0 in range(0, N, core):
            sl = (slice(y0, y0 + core + 2 * halo), slice(x0, x0 + core + 2 * halo))
            d, _ = forward(params, zp[sl][None], bf16=bf16, mask=inside[sl][None])
            out[y0:y0 + core, x0:x0 + core] = d[0, halo:halo + core, halo:halo + core]
    return out


# ----------------------------------------------------------------------------
# Jacobian of the network at z (the firm-nonexpansiveness check, appendix C:
# the training penalty asks ||J_{2D - I}||_S <= 1; here it is measured, not
# imposed). ReLU networks are piecewise linear: at z, layer l's Jacobian is
# the convolution without bias followed by the mask [pre-activation > 0].
# ----------------------------------------------------------------------------
def jvp(params, acts, v: np.ndarray, bf16: bool = False) -> np.ndarray:
    """J_net(z) v for v [B, H, W], with acts = forward(params, z, bf16)[1].
    bf16: tangent activations rounded to bfloat16 where the forward pass
    rounds its activations (weights of layers 2..L in bfloat16)."""
    t = v[:, None].astype(np.float64)
    L = len(params)
    for l, (w, b) in enumerate(params):
        wl = bf16_round(w) if (bf16 and l > 0) else w
        pre = conv3x3(t, wl, np.zeros_like(b))
        if l == L - 1:
            return pre[:, 0]
        t = pre * (acts[l + 1] > 0)
        if bf16:
            t = bf16_round(t)
    return t[:, 0]


def vjp(params, acts, u: np.ndarray, bf16: bool = False) -> np.ndarray:
    """J_net(z)^T u for u [B, H, W] (the gradient of sum(u * net) with respect
    to z); bf16 rounds the pre-activation gradients as backward() does."""
    g = u[:, None].astype(np.float64)
    L = len(params)
    for l in range(L - 1, -1, -1):
        w, _ = params[l]
        wl = bf16_round(w) if (bf16 and l > 0) else w
        dxv, _, _ = conv3x3_backward(acts[l], wl, g, need_dx=True)
        if l == 0:
            return dxv[:, 0]
        g = dxv * (acts[l] > 0)
        if bf16:
            g = bf16_round(g)
    return g[:, 0]


def fne_norm(params, z: np.ndarray, iters: int = 50, seed: int = 0, bf16: bool = False) -> float:
    """||I - 2 J_net(z)||_S = ||J_{2D - I}(z)||_S (D = I - net) by the power
    method on J^T J from a seeded normal start."""
    _, acts = forward(params, z, bf16)
    v = np.random.default_rng(seed).standard_normal(z.shape)
    v /= np.linalg.norm(v)
    s = 0.0
    for _ in range(iters):
        a = v - 2.0 * jvp(params, acts, v, bf16)
        s = float(np.linalg.norm(a))
        b = a - 2.0 * vjp(params, acts, a, bf16)
        v = b / np.linalg.norm(b)
    return s


def jvp_param_grad(params, acts, v: np.ndarray, u: np.ndarray, bf16: bool = False):
    """Gradient of u^T J_net(z) v with respect to the parameters, [(dw, db)]
    per layer (db = 0: the Jacobian does not depend on the biases). With the
    ReLU masks fixed (piecewise linearity), J_net(z) v is linear in each
    layer's weights: the gradient of layer l is the correlation of the
    pre-activation adjoint of u at layer l with the tangent of v at layer l's
    input, i.e. backward() run with the tangents as layer inputs while the
    masks stay those of the activations at z."""
    L = len(params)
    t = v[:, None].astype(np.float64)
    tin = []
    for l, (w, b) in enumerate(params):
        tin.append(t)
        wl = bf16_round(w) if (bf16 and l > 0) else w
        if l == L - 1:
            break
        t = conv3x3(t, wl, np.zeros_like(b)) * (acts[l + 1] > 0)
        if bf16:
            t = bf16_round(t)
    grads = [None] * L
    g = u[:, None].astype(np.float64)
    for l in range(L - 1, -1, -1):
        w, b = params[l]
        wl = bf16_round(w) if (bf16 and l > 0) else w
        dxv, dw, _ = conv3x3_backward(tin[l], wl, g, need_dx=l > 0)
        grads[l] = (dw, np.zeros_like(b))
        if l > 0:
            g = dxv * (acts[l] > 0)
            if bf16:
                g = bf16_round(g)
    return grads
