"""Thin ctypes binding of libri.so (the C ABI declared in include/ri.h).

Argument marshalling only: every entry point takes torch tensors that live on
the GPU, checks their dtype, shape and contiguity against the context (the C
side cannot see sizes), and passes raw device pointers plus the current HIP
stream. All arithmetic runs in the library's HIP kernels. Nothing here falls
back to a CPU path: if libri.so is missing the import of any entry point fails.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libri.so")

RI_OK, RI_EINVAL, RI_ENOMEM, RI_EDEVICE, RI_EUNSUPPORTED, RI_ENOTCONV, RI_FELLBACK = 0, -1, -2, -3, -4, -5, 1
RI_G_CSR, RI_G_OTF, RI_G_SEP = 0, 1, 2
RI_GRID_GATHER, RI_GRID_SCATTER = 0, 1
RI_PROX_HAAR, RI_PROX_CNN, RI_PROX_SARA = 0, 1, 2
RI_NO_DATA = c_void_p(-1 & 0xFFFFFFFFFFFFFFFF)

EXPORTS = ("ri_create", "ri_destroy", "ri_last_error", "phi_forward", "phi_adjoint", "ri_set_data",
           "ri_gradient", "ri_power_norm", "denoise", "fb_step", "ri_load_denoiser", "pnp_solve",
           "ri_get_plan_stats", "ri_get_plan_arrays", "ri_profile", "ri_profile_read",
           "ri_cnn_create", "ri_cnn_destroy", "ri_cnn_last_error", "ri_cnn_param_count", "ri_cnn_set_params",
           "ri_cnn_get_params", "ri_cnn_forward", "ri_cnn_grad", "ri_cnn_train_step", "ri_cnn_jvp", "ri_cnn_vjp",
           "ri_cnn_fne_norm", "ri_cnn_jvp_grad", "ri_cnn_train_step_fne", "ri_holo_build", "ri_holo_release",
           "ri_holo_apply", "ri_holo_normal", "ri_holo_get_stats", "ri_sara_setup", "ri_sara_reweight",
           "ri_sara_analysis", "ri_sara_synthesis", "ri_sara_get_state", "ri_gradient_noalloc",
           "ri_cnn_sample_batch")
RI_NOALLOC_SCRATCH_BYTES = 72 << 20


class RIError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libri status {status}: {msg}")
        self.status = status


class ri_plan_desc(ctypes.Structure):
    _fields_ = [("N", c_int32), ("oversample", c_int32), ("kb_support", c_int32), ("hmax", c_int32),
                ("cell_rad", c_double), ("w_max", c_double), ("n_wplanes", c_int32), ("g_mode", c_int32),
                ("precision", c_int32), ("tile", c_int32), ("M", c_int64), ("n_blocks", c_int32),
                ("block_offsets", c_void_p), ("facet_core", c_int32), ("facet_halo", c_int32),
                ("item_vis", c_int32), ("n_wstacks", c_int32), ("grid_form", c_int32)]


class ri_solve_opts(ctypes.Structure):
    _fields_ = [("max_iter", c_int32), ("rel_tol", c_double), ("prox_kind", c_int32), ("tau", c_double),
                ("sigma_train", c_double), ("L", c_double), ("check_every", c_int32), ("x_true", c_void_p),
                ("trace", c_void_p), ("use_graph", c_int32), ("diverge_checks", c_int32),
                ("reweight_every", c_int32), ("use_holo", c_int32)]


class ri_solve_report(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("L", c_double), ("gamma", c_double), ("alpha", c_double),
                ("t_or_sigma", c_double), ("final_rel_change", c_double), ("final_residual2", c_double),
                ("snr_db", c_double), ("fell_back", c_int32), ("ms", c_double)]


class ri_cnn_desc(ctypes.Structure):
    _fields_ = [("layers", c_int32), ("channels", c_int32), ("max_batch", c_int32), ("max_h", c_int32),
                ("max_w", c_int32), ("training", c_int32)]


class ri_plan_stats(ctypes.Structure):
    _fields_ = [("M", c_int64), ("nnz", c_int64), ("N", c_int32), ("Np", c_int32), ("tile", c_int32),
                ("n_tiles", c_int32), ("n_items", c_int32), ("n_blocks", c_int32), ("max_item_vis", c_int64),
                ("device_bytes", c_int64), ("plan_ms", c_double), ("n_tuned", c_int32),
                ("tuned_tile", c_int32 * 4), ("tuned_ms", c_double * 4)]


class ri_holo_stats(ctypes.Structure):
    _fields_ = [("tiles", c_int64), ("entries", c_int64), ("bytes", c_int64), ("pairs", c_int64),
                ("max_reach", c_int32), ("build_ms", c_double)]


class ri_kernel_times(ctypes.Structure):
    _fields_ = [("n_tiles", c_int32), ("n_fft", c_int32), ("n_prox", c_int32), ("n_other", c_int32),
                ("tiles_ms", c_double), ("fft_ms", c_double), ("prox_ms", c_double), ("other_ms", c_double)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libri.so (built in-tree by ``__graft_entry__.build()``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    L = ctypes.CDLL(LIB_PATH)
    st = c_int32
    L.ri_create.argtypes = [POINTER(ri_plan_desc), c_void_p, POINTER(c_void_p)]; L.ri_create.restype = st
    L.ri_destroy.argtypes = [c_void_p]; L.ri_destroy.restype = None
    L.ri_last_error.argtypes = [c_void_p]; L.ri_last_error.restype = ctypes.c_char_p
    L.phi_forward.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]; L.phi_forward.restype = st
    L.phi_adjoint.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]; L.phi_adjoint.restype = st
    L.ri_set_data.argtypes = [c_void_p, c_void_p, c_void_p]; L.ri_set_data.restype = st
    L.ri_gradient.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]; L.ri_gradient.restype = st
    L.ri_gradient_noalloc.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.ri_gradient_noalloc.restype = st
    L.ri_power_norm.argtypes = [c_void_p, c_int32, c_double, c_void_p, POINTER(c_double), POINTER(c_int32), c_void_p]
    L.ri_power_norm.restype = st
    L.denoise.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_double, c_void_p]; L.denoise.restype = st
    L.fb_step.argtypes = [c_void_p, c_void_p, c_void_p, c_double, c_int32, c_double, c_void_p, c_void_p, c_void_p]
    L.fb_step.restype = st
    L.ri_load_denoiser.argtypes = [c_void_p, c_void_p, c_int64, c_int32, c_void_p]
    L.ri_load_denoiser.restype = st
    L.pnp_solve.argtypes = [c_void_p, c_void_p, POINTER(ri_solve_opts), c_void_p, POINTER(ri_solve_report)]
    L.pnp_solve.restype = st
    L.ri_get_plan_stats.argtypes = [c_void_p, POINTER(ri_plan_stats)]; L.ri_get_plan_stats.restype = st
    L.ri_get_plan_arrays.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.ri_get_plan_arrays.restype = st
    L.ri_profile.argtypes = [c_void_p, c_int32]; L.ri_profile.restype = st
    L.ri_sara_setup.argtypes = [c_void_p, c_int32, c_void_p]; L.ri_sara_setup.restype = st
    L.ri_sara_reweight.argtypes = [c_void_p, c_void_p, c_double, c_void_p]; L.ri_sara_reweight.restype = st
    L.ri_sara_analysis.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]; L.ri_sara_analysis.restype = st
    L.ri_sara_synthesis.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]; L.ri_sara_synthesis.restype = st
    L.ri_sara_get_state.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]; L.ri_sara_get_state.restype = st
    L.ri_holo_build.argtypes = [c_void_p, c_void_p]; L.ri_holo_build.restype = st
    L.ri_holo_release.argtypes = [c_void_p]; L.ri_holo_release.restype = st
    L.ri_holo_apply.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]; L.ri_holo_apply.restype = st
    L.ri_holo_normal.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]; L.ri_holo_normal.restype = st
    L.ri_holo_get_stats.argtypes = [c_void_p, POINTER(ri_holo_stats)]; L.ri_holo_get_stats.restype = st
    L.ri_profile_read.argtypes = [c_void_p, POINTER(ri_kernel_times)]; L.ri_profile_read.restype = st
    L.ri_cnn_create.argtypes = [POINTER(ri_cnn_desc), ctypes.c_uint64, POINTER(c_void_p)]
    L.ri_cnn_create.restype = st
    L.ri_cnn_destroy.argtypes = [c_void_p]; L.ri_cnn_destroy.restype = None
    L.ri_cnn_last_error.argtypes = [c_void_p]; L.ri_cnn_last_error.restype = ctypes.c_char_p
    L.ri_cnn_param_count.argtypes = [c_void_p]; L.ri_cnn_param_count.restype = c_int64
    L.ri_cnn_set_params.argtypes = [c_void_p, c_void_p, c_void_p]; L.ri_cnn_set_params.restype = st
    L.ri_cnn_get_params.argtypes = [c_void_p, c_void_p, c_void_p]; L.ri_cnn_get_params.restype = st
    L.ri_cnn_forward.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p]
    L.ri_cnn_forward.restype = st
    L.ri_cnn_grad.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p]
    L.ri_cnn_grad.restype = st
    L.ri_cnn_train_step.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_int32, ctypes.c_float,
                                    ctypes.c_uint64, ctypes.c_float, c_void_p, c_void_p]
    L.ri_cnn_train_step.restype = st
    L.ri_cnn_sample_batch.argtypes = [c_void_p, c_void_p, c_int64, c_int32, c_int32, ctypes.c_uint64, c_void_p,
                                      c_void_p]
    L.ri_cnn_sample_batch.restype = st
    for f in (L.ri_cnn_jvp, L.ri_cnn_vjp):
        f.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p]
        f.restype = st
    L.ri_cnn_fne_norm.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_int32, ctypes.c_uint64, c_void_p,
                                  c_void_p]
    L.ri_cnn_fne_norm.restype = st
    L.ri_cnn_jvp_grad.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p,
                                  c_void_p]
    L.ri_cnn_jvp_grad.restype = st
    L.ri_cnn_train_step_fne.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_int32, ctypes.c_float,
                                        ctypes.c_uint64, ctypes.c_float, ctypes.c_float, ctypes.c_float, c_int32,
                                        c_int32, c_void_p, c_void_p, c_void_p]
    L.ri_cnn_train_step_fne.restype = st
    _lib = L
    return L


# ----------------------------------------------------------------------------
# Context
# ----------------------------------------------------------------------------
class Context:
    """Owns one ``ri_ctx``. Keeps the plan description for size checks."""

    def __init__(self, handle: int, desc: ri_plan_desc, n_wplanes: int):
        self.handle = c_void_p(handle)
        self.N = desc.N
        self.M = desc.M
        self.precision = desc.precision
        self.g_mode = desc.g_mode
        self.n_wplanes = n_wplanes

    @property
    def real_dtype(self):
        import torch
        return torch.float32 if self.precision == 32 else torch.float64

    def close(self):
        if self.handle is not None and self.handle.value:
            load().ri_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check(ctx: Context | None, status: int):
    if status not in (RI_OK, RI_FELLBACK):
        L = load()
        msg = L.ri_last_error(ctx.handle if ctx is not None else None)
        raise RIError(status, msg.decode() if msg else "")
    return status


def _stream(stream):
    import torch
    if stream is None:
        return c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return c_void_p(stream)
    return c_void_p(stream.cuda_stream)


def _dev(t, dtype, numel: int, name: str):
    import torch
    if t is None:
        raise ValueError(f"{name} is None")
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return c_void_p(t.data_ptr())


def _image(ctx, t, name):
    return _dev(t, ctx.real_dtype, ctx.N * ctx.N, name)


def _vis(ctx, t, name):
    import torch
    cd = torch.complex64 if ctx.precision == 32 else torch.complex128
    return _dev(t, cd, ctx.M, name)


def plan_desc(N: int, M: int, *, cell_rad: float = 0.0, w_max: float = 0.0, n_wplanes: int = 1,
              hmax: int = 5, g_mode: int = RI_G_CSR, precision: int = 32, tile: int = 0, n_blocks: int = 1,
              facet_core: int = 0, facet_halo: int = 0, item_vis: int = 0, n_wstacks: int = 0,
              grid_form: int = RI_GRID_GATHER) -> ri_plan_desc:
    d = ri_plan_desc()
    d.N, d.oversample, d.kb_support, d.hmax = N, 2, 7, hmax
    d.cell_rad, d.w_max, d.n_wplanes = cell_rad, w_max, n_wplanes
    d.g_mode, d.precision, d.tile = g_mode, precision, tile
    d.M, d.n_blocks = M, n_blocks
    d.block_offsets = None
    d.facet_core, d.facet_halo = facet_core, facet_halo
    d.item_vis = item_vis
    d.n_wstacks = n_wstacks
    d.grid_form = grid_form
    return d


# ----------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ----------------------------------------------------------------------------
def ri_create(desc: ri_plan_desc, uvw: np.ndarray, block_offsets: np.ndarray | None = None) -> Context:
    L = load()
    uvw = np.ascontiguousarray(uvw, dtype=np.float64)
    if uvw.ndim != 2 or uvw.shape[1] != 3 or uvw.shape[0] != desc.M:
        raise ValueError(f"uvw must be float64 [M={desc.M}, 3], got {uvw.shape}")
    offs = None
    if block_offsets is not None:
        offs = np.ascontiguousarray(block_offsets, dtype=np.int64)
        if offs.shape != (desc.n_blocks + 1,):
            raise ValueError("block_offsets must have n_blocks + 1 entries")
        desc.block_offsets = offs.ctypes.data_as(c_void_p)
    out = c_void_p()
    _check(None, L.ri_create(ctypes.byref(desc), uvw.ctypes.data_as(c_void_p), ctypes.byref(out)))
    return Context(out.value, desc, desc.n_wplanes)


def ri_destroy(ctx: Context):
    ctx.close()


def phi_forward(ctx: Context, x, y, stream=None):
    _check(ctx, load().phi_forward(ctx.handle, _image(ctx, x, "x"), _vis(ctx, y, "y"), _stream(stream)))


def phi_adjoint(ctx: Context, y, x, stream=None):
    _check(ctx, load().phi_adjoint(ctx.handle, _vis(ctx, y, "y"), _image(ctx, x, "x"), _stream(stream)))


def ri_set_data(ctx: Context, y, stream=None):
    _check(ctx, load().ri_set_data(ctx.handle, _vis(ctx, y, "y"), _stream(stream)))


def _data_arg(ctx, y):
    if y is None:
        return None
    if isinstance(y, str) and y == "none":
        return RI_NO_DATA
    return _vis(ctx, y, "y")


def ri_gradient(ctx: Context, x, y, g, r2=None, stream=None):
    """g = Re{Phi^dagger (Phi x - y)}; y: tensor, None (stored data) or "none" (y = 0)."""
    import torch
    r2p = _dev(r2, torch.float64, 1, "r2") if r2 is not None else None
    _check(ctx, load().ri_gradient(ctx.handle, _image(ctx, x, "x"), _data_arg(ctx, y), _image(ctx, g, "g"),
                                   r2p, _stream(stream)))


def ri_gradient_noalloc(ctx: Context, x, y, g, r2=None, stream=None):
    """ri_gradient with every work buffer in the library's static device workspace (no allocation)."""
    import torch
    r2p = _dev(r2, torch.float64, 1, "r2") if r2 is not None else None
    _check(ctx, load().ri_gradient_noalloc(ctx.handle, _image(ctx, x, "x"), _data_arg(ctx, y),
                                           _image(ctx, g, "g"), r2p, _stream(stream)))


def ri_power_norm(ctx: Context, max_it: int = 500, rtol: float = 1e-8, x0=None, stream=None, allow_notconv=True):
    import torch
    x0p = _dev(x0, torch.float64, ctx.N * ctx.N, "x0") if x0 is not None else None
    Lv, it = c_double(0.0), c_int32(0)
    st = load().ri_power_norm(ctx.handle, max_it, rtol, x0p, ctypes.byref(Lv), ctypes.byref(it), _stream(stream))
    if not (allow_notconv and st == RI_ENOTCONV):
        _check(ctx, st)
    return Lv.value, it.value


def denoise(ctx: Context, z, out, kind: int = RI_PROX_HAAR, param: float = 0.0, stream=None):
    _check(ctx, load().denoise(ctx.handle, _image(ctx, z, "z"), _image(ctx, out, "out"), kind, param,
                               _stream(stream)))


def fb_step(ctx: Context, x_in, y, gamma: float, kind: int, param: float, x_out, norms=None, stream=None):
    import torch
    np_ = _dev(norms, torch.float64, 3, "norms") if norms is not None else None
    if x_in is not None and x_out is not None and x_in.data_ptr() == x_out.data_ptr():
        raise ValueError("x_in and x_out must not alias")
    _check(ctx, load().fb_step(ctx.handle, _image(ctx, x_in, "x_in"), _data_arg(ctx, y), gamma, kind, param,
                               _image(ctx, x_out, "x_out"), np_, _stream(stream)))


def ri_load_denoiser(ctx: Context, params, layers: int = 10, stream=None):
    """Load the CNN of RI_PROX_CNN from its FP32 parameter vector (ri_cnn.h layout)."""
    import torch
    if not (isinstance(params, torch.Tensor) and params.is_cuda):
        raise TypeError("params must be a GPU tensor")
    p = _dev(params, torch.float32, params.numel(), "params")
    _check(ctx, load().ri_load_denoiser(ctx.handle, p, params.numel(), layers, _stream(stream)))


def pnp_solve(ctx: Context, y, opts: ri_solve_opts, x_out) -> ri_solve_report:
    rep = ri_solve_report()
    yp = _vis(ctx, y, "y") if y is not None else None
    _check(ctx, load().pnp_solve(ctx.handle, yp, ctypes.byref(opts), _image(ctx, x_out, "x_out"),
                                 ctypes.byref(rep)))
    return rep


def ri_get_plan_stats(ctx: Context) -> ri_plan_stats:
    s = ri_plan_stats()
    _check(ctx, load().ri_get_plan_stats(ctx.handle, ctypes.byref(s)))
    return s


def ri_get_plan_arrays(ctx: Context):
    M = ctx.M
    cu = np.empty(M, np.int32); cv = np.empty(M, np.int32); pl = np.empty(M, np.int32)
    ph = np.empty(ctx.n_wplanes, np.int32)
    _check(ctx, load().ri_get_plan_arrays(ctx.handle, cu.ctypes.data_as(c_void_p), cv.ctypes.data_as(c_void_p),
                                          pl.ctypes.data_as(c_void_p), ph.ctypes.data_as(c_void_p)))
    return cu, cv, pl, ph


def ri_profile(ctx: Context, enable: bool):
    _check(ctx, load().ri_profile(ctx.handle, 1 if enable else 0))


def ri_profile_read(ctx: Context) -> ri_kernel_times:
    t = ri_kernel_times()
    _check(ctx, load().ri_profile_read(ctx.handle, ctypes.byref(t)))
    return t


def _grid(ctx, t, name):
    import torch
    cd = torch.complex64 if ctx.precision == 32 else torch.complex128
    return _dev(t, cd, 4 * ctx.N * ctx.N, name)


def _coef9(ctx, t, name):
    return _dev(t, ctx.real_dtype, 9 * ctx.N * ctx.N, name)


def ri_sara_setup(ctx: Context, sub_iters: int = 10, stream=None):
    _check(ctx, load().ri_sara_setup(ctx.handle, int(sub_iters), _stream(stream)))


def ri_sara_reweight(ctx: Context, x, rho: float, stream=None):
    _check(ctx, load().ri_sara_reweight(ctx.handle, _image(ctx, x, "x"), float(rho), _stream(stream)))


def ri_sara_analysis(ctx: Context, x, coef, stream=None):
    _check(ctx, load().ri_sara_analysis(ctx.handle, _image(ctx, x, "x"), _coef9(ctx, coef, "coef"), _stream(stream)))


def ri_sara_synthesis(ctx: Context, coef, x, stream=None):
    _check(ctx, load().ri_sara_synthesis(ctx.handle, _coef9(ctx, coef, "coef"), _image(ctx, x, "x"),
                                         _stream(stream)))


def ri_sara_get_state(ctx: Context, v=None, w=None, stream=None):
    _check(ctx, load().ri_sara_get_state(ctx.handle, _coef9(ctx, v, "v") if v is not None else None,
                                         _coef9(ctx, w, "w") if w is not None else None, _stream(stream)))


def ri_holo_build(ctx: Context, stream=None):
    _check(ctx, load().ri_holo_build(ctx.handle, _stream(stream)))


def ri_holo_release(ctx: Context):
    _check(ctx, load().ri_holo_release(ctx.handle))


def ri_holo_apply(ctx: Context, X, Y, stream=None):
    _check(ctx, load().ri_holo_apply(ctx.handle, _grid(ctx, X, "X"), _grid(ctx, Y, "Y"), _stream(stream)))


def ri_holo_normal(ctx: Context, x, out, stream=None):
    _check(ctx, load().ri_holo_normal(ctx.handle, _image(ctx, x, "x"), _image(ctx, out, "out"), _stream(stream)))


def ri_holo_get_stats(ctx: Context) -> ri_holo_stats:
    s = ri_holo_stats()
    _check(ctx, load().ri_holo_get_stats(ctx.handle, ctypes.byref(s)))
    return s


# ----------------------------------------------------------------------------
# CNN denoiser (include/ri_cnn.h)
# ----------------------------------------------------------------------------
class Cnn:
    """Owns one ``ri_cnn``; keeps its buffer limits for shape checks."""

    def __init__(self, handle: int, desc: ri_cnn_desc):
        self.handle = c_void_p(handle)
        self.layers, self.max_batch = desc.layers, desc.max_batch
        self.max_h, self.max_w, self.training = desc.max_h, desc.max_w, desc.training
        self.n_params = int(load().ri_cnn_param_count(self.handle))

    def close(self):
        if self.handle is not None and self.handle.value:
            load().ri_cnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_cnn(net: Cnn | None, status: int):
    if status != RI_OK:
        msg = load().ri_cnn_last_error(net.handle if net is not None else None)
        raise RIError(status, msg.decode() if msg else "")


def _batch(net: Cnn, t, name):
    import torch
    if t is None or t.dim() != 3:
        raise ValueError(f"{name} must be a [batch, h, w] tensor")
    B, h, w = t.shape
    if B > net.max_batch or h > net.max_h or w > net.max_w or h % 16 or w % 16:
        raise ValueError(f"{name} shape {tuple(t.shape)} exceeds the network's buffers or is not a multiple of 16")
    return _dev(t, torch.float32, t.numel(), name), B, h, w


def ri_cnn_create(layers: int = 10, max_batch: int = 1, max_h: int = 256, max_w: int = 256, training: bool = False,
                  seed: int = 0, channels: int = 64) -> Cnn:
    d = ri_cnn_desc()
    d.layers, d.channels, d.max_batch, d.max_h, d.max_w, d.training = layers, channels, max_batch, max_h, max_w, \
        1 if training else 0
    out = c_void_p()
    _check_cnn(None, load().ri_cnn_create(ctypes.byref(d), seed, ctypes.byref(out)))
    return Cnn(out.value, d)


def ri_cnn_destroy(net: Cnn):
    net.close()


def ri_cnn_param_count(net: Cnn) -> int:
    return int(load().ri_cnn_param_count(net.handle))


def ri_cnn_set_params(net: Cnn, params, stream=None):
    import torch
    _check_cnn(net, load().ri_cnn_set_params(net.handle, _dev(params, torch.float32, net.n_params, "params"),
                                             _stream(stream)))


def ri_cnn_get_params(net: Cnn, params, stream=None):
    import torch
    _check_cnn(net, load().ri_cnn_get_params(net.handle, _dev(params, torch.float32, net.n_params, "params"),
                                             _stream(stream)))


def ri_cnn_forward(net: Cnn, z, out, stream=None):
    """out = z - net(z) for z, out: float32 [batch, h, w] on the GPU."""
    zp, B, h, w = _batch(net, z, "z")
    if out.shape != z.shape:
        raise ValueError("out must have the shape of z")
    op, _, _, _ = _batch(net, out, "out")
    _check_cnn(net, load().ri_cnn_forward(net.handle, zp, op, B, h, w, _stream(stream)))


def ri_cnn_grad(net: Cnn, z, g, grads, stream=None):
    """grads = d sum(g * net(z)) / d params."""
    import torch
    zp, B, h, w = _batch(net, z, "z")
    if g.shape != z.shape:
        raise ValueError("g must have the shape of z")
    gp, _, _, _ = _batch(net, g, "g")
    _check_cnn(net, load().ri_cnn_grad(net.handle, zp, gp, B, h, w, _dev(grads, torch.float32, net.n_params, "grads"),
                                       _stream(stream)))


def ri_cnn_jvp(net: Cnn, z, v, out, stream=None):
    """out = J_net(z) v (training-mode network)."""
    zp, B, h, w = _batch(net, z, "z")
    if v.shape != z.shape or out.shape != z.shape:
        raise ValueError("v and out must have the shape of z")
    vp, _, _, _ = _batch(net, v, "v")
    op, _, _, _ = _batch(net, out, "out")
    _check_cnn(net, load().ri_cnn_jvp(net.handle, zp, vp, op, B, h, w, _stream(stream)))


def ri_cnn_vjp(net: Cnn, z, u, out, stream=None):
    """out = J_net(z)^T u (training-mode network)."""
    zp, B, h, w = _batch(net, z, "z")
    if u.shape != z.shape or out.shape != z.shape:
        raise ValueError("u and out must have the shape of z")
    up, _, _, _ = _batch(net, u, "u")
    op, _, _, _ = _batch(net, out, "out")
    _check_cnn(net, load().ri_cnn_vjp(net.handle, zp, up, op, B, h, w, _stream(stream)))


def ri_cnn_fne_norm(net: Cnn, z, iters: int = 30, seed: int = 1, stream=None) -> float:
    """||I - 2 J_net(z)||_S by the power method (the firm-nonexpansiveness check)."""
    zp, B, h, w = _batch(net, z, "z")
    out = ctypes.c_double(0.0)
    _check_cnn(net, load().ri_cnn_fne_norm(net.handle, zp, B, h, w, iters, seed, ctypes.byref(out),
                                           _stream(stream)))
    return out.value


def ri_cnn_jvp_grad(net: Cnn, z, v, u, grads, stream=None):
    """grads = d(u^T J_net(z) v) / d params (bias entries 0)."""
    import torch
    zp, B, h, w = _batch(net, z, "z")
    if v.shape != z.shape or u.shape != z.shape:
        raise ValueError("v and u must have the shape of z")
    vp, _, _, _ = _batch(net, v, "v")
    up, _, _, _ = _batch(net, u, "u")
    _check_cnn(net, load().ri_cnn_jvp_grad(net.handle, zp, vp, up, B, h, w,
                                           _dev(grads, torch.float32, net.n_params, "grads"), _stream(stream)))


RI_FNE_AT_INPUT, RI_FNE_AT_MIX = 0, 1


def ri_cnn_train_step_fne(net: Cnn, clean, sigma: float, seed: int, lr: float, lam: float, eps: float = 0.05,
                          power_iters: int = 2, loss=None, fne_sq=None, stream=None, point: int = RI_FNE_AT_INPUT):
    """Training step with the relaxed firm-nonexpansiveness penalty (Jacobian at the
    noisy input, or at random points between the clean and the denoised images)."""
    import torch
    cp, B, h, w = _batch(net, clean, "clean")
    lp = _dev(loss, torch.float64, 1, "loss") if loss is not None else None
    fp = _dev(fne_sq, torch.float64, 1, "fne_sq") if fne_sq is not None else None
    _check_cnn(net, load().ri_cnn_train_step_fne(net.handle, cp, B, h, w, sigma, seed, lr, lam, eps, power_iters,
                                                 point, lp, fp, _stream(stream)))


def ri_cnn_train_step(net: Cnn, clean, sigma: float, seed: int, lr: float, loss=None, stream=None):
    import torch
    cp, B, h, w = _batch(net, clean, "clean")
    lp = _dev(loss, torch.float64, 1, "loss") if loss is not None else None
    _check_cnn(net, load().ri_cnn_train_step(net.handle, cp, B, h, w, sigma, seed, lr, lp, _stream(stream)))


def ri_cnn_sample_batch(net: Cnn, pool, seed: int, out, stream=None):
    """out[b] = a pool patch in one of the square's eight orientations, both drawn from (seed, b)."""
    import torch
    if pool is None or pool.dim() != 3 or out is None or out.dim() != 3:
        raise ValueError("pool and out must be [n, side, side] tensors")
    n, side, side2 = pool.shape
    B, h, w = out.shape
    if side != side2 or (h, w) != (side, side):
        raise ValueError(f"pool {tuple(pool.shape)} and out {tuple(out.shape)} must hold square patches of one side")
    pp = _dev(pool, torch.float32, pool.numel(), "pool")
    op = _dev(out, torch.float32, out.numel(), "out")
    _check_cnn(net, load().ri_cnn_sample_batch(net.handle, pp, n, side, B, seed, op, _stream(stream)))
