/*
 * ri.h -- C ABI of the MI355X plug-and-play forward-backward imaging library
 * (libri.so, HIP kernels for gfx950).
 *
 * The library computes the hot path of radio-interferometric imaging by
 * forward-backward iterations (Dabbech et al., "First AI for deep
 * super-resolution wide-field imaging in radio astronomy"):
 *
 *   y = Phi x + n,  Phi = G F Z                                  (eq. 1)
 *   x^{k+1} = D(x^k - gamma Re{Phi^dagger (Phi x^k - y)})        (eq. A2)
 *
 * with Z the zero padding by two plus the kernel correction, F the
 * oversampled 2D FFT and G the sparse Kaiser-Bessel interpolation convolved
 * row-wise with small w-kernels (appendix E); Phi^dagger Phi is the sum of the
 * per-block terms (eq. E2); D is the Haar-l1 + positivity prox or a learned
 * residual CNN (appendices B and C).
 *
 * Conventions used throughout:
 *  - Images are real, row-major [N][N], index [iy][ix] for the centred pixel
 *    (ix - N/2, iy - N/2); element type float (precision 32) or double (64).
 *  - Visibilities are complex, interleaved (re, im) float or double pairs, in
 *    the caller's order (the library's internal tile order never leaks out).
 *  - uvw rows are (omega_u, omega_v) in radians per pixel (|omega| < pi) and w
 *    in wavelengths; the Fourier kernel is exp(-i omega . n) forward.
 *  - Every buffer argument marked "dev" is device memory owned by the caller;
 *    the library never frees it and keeps no pointer to it after the call
 *    returns. "host" buffers are read during the call only.
 *  - Calls taking a stream only enqueue work on it (no host synchronisation)
 *    unless stated otherwise; a NULL stream is the default stream.
 *  - Every call returns a status; on failure ri_last_error() describes it and
 *    no output buffer has been partially written by a kernel of that call
 *    (argument checks run before any launch).
 *  - A context is used by one host thread at a time.
 */
#ifndef RI_H
#define RI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ri_ctx ri_ctx;
typedef void *ri_stream; /* hipStream_t */

typedef enum {
    RI_OK = 0,
    RI_EINVAL = -1,       /* bad argument: sizes, NULL pointers, non-finite or |omega| >= pi */
    RI_ENOMEM = -2,       /* device or host allocation failed */
    RI_EDEVICE = -3,      /* a HIP call failed (message has the HIP error string) */
    RI_EUNSUPPORTED = -4, /* valid request this build does not implement */
    RI_ENOTCONV = -5,     /* an iteration hit its limit without meeting its tolerance */
    RI_FELLBACK = 1       /* pnp_solve detected divergence and finished with the Haar prox */
} ri_status;

enum { RI_G_CSR = 0, RI_G_OTF = 1, RI_G_SEP = 2 };
enum { RI_GRID_GATHER = 0, RI_GRID_SCATTER = 1 };
enum { RI_PROX_HAAR = 0, RI_PROX_CNN = 1, RI_PROX_SARA = 2 };

/* Plan description. All sizes explicit; nothing is read through globals. */
typedef struct {
    int32_t N;             /* image side; even, N' = 2N a power of two, 16 <= N <= 4096 */
    int32_t oversample;    /* grid oversampling sigma; must be 2 */
    int32_t kb_support;    /* Kaiser-Bessel width J; must be 7 */
    int32_t hmax;          /* largest w-kernel half support, 0..5 (windows up to 7+2*hmax) */
    double cell_rad;       /* pixel size delta [rad], enters the w-term */
    double w_max;          /* W [wavelengths]: the w-plane table spans [-W, W]; 0 => no w-term */
    int32_t n_wplanes;     /* odd number of w-planes (w = 0 is the centre plane) */
    int32_t g_mode;        /* RI_G_CSR: G stored row by row: the complex values of each row's
                              window in window order, int64 row pointers; the columns follow
                              from the window and are not stored;
                              RI_G_OTF: G rows computed on the fly from the KB and w-tables;
                              RI_G_SEP: each row stored as its two axis factors (a row is
                              g_v[ay] g_u[ax] on its window): 17 (g_u, g_v) pairs per
                              visibility, 34 complex values, computed once in FP64 */
    int32_t precision;     /* 32 or 64: element type of Phi, Phi^dagger and the FFT */
    int32_t tile;          /* uv tile side in grid cells (8..128, divides N'); 0 => autotuned at
                              ri_create among 8, 16, 32 by timing fused gradient passes (the
                              side also selects the gridding form, see grid_form). The choice
                              depends on the coverage; a caller creating several contexts on
                              one coverage passes the tile found once (ri_get_plan_stats) and
                              skips the timing. */
    int64_t M;             /* number of visibilities, >= 0 */
    int32_t n_blocks;      /* data blocks (eq. E1), >= 1 */
    const int64_t *block_offsets; /* host, n_blocks+1 ascending offsets into the caller's
                                     visibility order (0 ... M); NULL => one block */
    int32_t facet_core;    /* denoiser facet core side (multiple of 16); 0 => whole image */
    int32_t facet_halo;    /* facet halo in pixels (the CNN needs >= its receptive radius) */
    int32_t item_vis;      /* visibilities per work item of the tile launch (0 => 2048) */
    int32_t n_wstacks;     /* w-stacking hybrid (appendix E): 0 or 1 => the w-term rides on the
                              w-kernels alone; P in 2..64 => P stacks of equal width over [-W, W]
                              (centres w_p = -W + (2p+1) W/P, a visibility joins the stack whose
                              interval holds its w). Stack p's image is multiplied by the exact
                              phase screen exp(-2 pi i w_p (sqrt(1 - l^2 - m^2) - 1)) in Z and has
                              its own FFT pair; the w-plane table then spans the residual
                              [-W/P, W/P]. Costs P FFT pairs and 2P grids per pass. */
    int32_t grid_form;     /* how G^H accumulates a work item's subgrid. RI_GRID_GATHER (0, the
                              default): in FP32 with G on the fly or as stored axis factors and a
                              subgrid side tile + 2 (hmax + 3) <= 32, every wave keeps the whole
                              subgrid in FP32 registers and gathers its visibilities' separable
                              contributions (no LDS atomics): by VALU FMAs up to a side of 24, by
                              FP32 matrix-core products (K = a wave's four visibilities) up to
                              32; other cases fall back to the scatter form. RI_GRID_SCATTER (1): each visibility's window is added into
                              FP64 LDS planes by atomics. The two differ by FP32 rounding order. */
} ri_plan_desc;

/* Build a context: validates the description, computes every visibility's
 * grid cell and fraction in FP64 (p = omega N'/(2 pi), c = floor(p + 1/2)),
 * its w-plane, the least-squares w-kernel table, the kernel-correction and
 * twiddle tables, sorts the visibilities by (block, uv tile, support), forms
 * the work items of the persistent launches and, for RI_G_CSR (RI_G_SEP), fills
 * the stored G (its axis factors) on the device (appendix E: the sparse
 * matrices are computed once). uvw: host, M x 3 doubles.
 * Synchronous. On success *out owns all device memory it allocated. */
ri_status ri_create(const ri_plan_desc *desc, const double *uvw, ri_ctx **out);
void ri_destroy(ri_ctx *ctx);
/* Message for the last non-OK status of this context (or of the last failed
 * ri_create when ctx is NULL). Valid until the next call on the context. */
const char *ri_last_error(const ri_ctx *ctx);

/* y = Phi x = G F Z x (eq. 1). x: dev [N][N] real; y: dev [M] complex, caller's
 * order. Element types follow the context precision. */
ri_status phi_forward(ri_ctx *ctx, const void *x, void *y, ri_stream stream);

/* x = Re{Phi^dagger y} = Re{Z^dagger F^dagger G^H y} (the real-image adjoint).
 * y: dev [M] complex (caller's order); x: dev [N][N] real. */
ri_status phi_adjoint(ri_ctx *ctx, const void *y, void *x, ri_stream stream);

/* Store the data vector y (dev [M] complex, caller's order) inside the
 * context, permuted to the internal order; used by ri_gradient, fb_step and
 * pnp_solve when they are passed y = NULL. */
ri_status ri_set_data(ri_ctx *ctx, const void *y, ri_stream stream);

/* Gradient of f(x) = ||Phi x - y||^2 / 2 (appendix A):
 *   g = Re{Phi^dagger (Phi x - y)} = Re{Phi^dagger Phi} x - Re{Phi^dagger y},
 * computed in one fused degrid -> residual -> grid pass over the blocks.
 * y: dev [M] complex in the caller's order, or NULL for the stored data, or
 * RI_NO_DATA for y = 0 (then g = Re{Phi^dagger Phi} x).
 * r2: dev double[1] receiving ||Phi x - y||^2 in FP64, or NULL. */
#define RI_NO_DATA ((const void *)(intptr_t)-1)
ri_status ri_gradient(ri_ctx *ctx, const void *x, const void *y, void *g, double *r2,
                      ri_stream stream);

/* ri_gradient without any device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same gradient, ||Phi x - y||^2 and arguments as
 * ri_gradient, but every work buffer of its kernels (the two oversampled
 * grids per w-stack, the persistent launch's work counter, the FP64 partial
 * sums) lies in a workspace compiled into the library, RI_NOALLOC_SCRATCH_BYTES
 * per device, held by each GPU the library runs on until the process ends.
 * A y in the caller's order is read in place (no staging copy).
 * The call allocates nothing: no hipMalloc, hipFree or allocating library
 * routine. Limits and errors: RI_EINVAL when the context's buffers do not
 * fit the workspace (about 2 x w-stacks x N'^2 complex cells plus 20 KB:
 * FP32 up to N' = 2048, FP64 up to N' = 1024 without w-stacking), or while
 * kernel timing (ri_profile) is on. Every call on a GPU shares that GPU's one
 * workspace: calls that overlap in time on one GPU (other host threads, other
 * streams, other contexts) race and corrupt each other's results; serialise
 * them, e.g. on one stream. The workspace keeps the last call's contents;
 * each call clears what must start at zero itself. */
#define RI_NOALLOC_SCRATCH_BYTES ((int64_t)72 << 20)
ri_status ri_gradient_noalloc(ri_ctx *ctx, const void *x, const void *y, void *g, double *r2,
                              ri_stream stream);

/* L = ||Re{Phi^dagger Phi}||_S by the power method in FP64 on the device
 * (appendix A), whatever the context precision: x <- A x / ||A x||, stop when
 * the relative change of ||A x|| is <= rtol or after max_it applications.
 * x0: dev double [N][N] start vector, or NULL for a built-in deterministic one.
 * Synchronises the stream once per iteration. Returns RI_ENOTCONV (with *L
 * set to the last estimate) when max_it is reached first and rtol > 0. */
ri_status ri_power_norm(ri_ctx *ctx, int32_t max_it, double rtol, const double *x0,
                        double *L, int32_t *iters, ri_stream stream);

/* Denoiser D (the backward step of eq. A2):
 *   RI_PROX_HAAR: D(z) = max(0, Psi soft_t(Psi^dagger z)), Psi the orthonormal
 *                 2D Haar basis with four levels, every coefficient
 *                 thresholded at t = param (eq. B2: t = tau / sqrt(2L));
 *   RI_PROX_SARA: uSARA's denoiser (section "uSARA's handcrafted denoiser"):
 *                 D(z) = argmin_x ||x - z||^2 / 2 + t ||w . Psi^dagger x||_1 + iota_+(x),
 *                 t = param, Psi = [Dirac, db1, ..., db8] / 3 (orthonormal 2D
 *                 periodic Daubechies wavelets with 1..8 vanishing moments, 4
 *                 levels, minimum-phase filters), w the context's weights (1
 *                 until ri_sara_reweight). Computed by the context's number of
 *                 dual forward-backward sub-iterations (ri_sara_setup; 10 by
 *                 default), warm-started from the dual variable the previous
 *                 call left; z and out may not alias; needs N divisible by 16;
 *   RI_PROX_CNN:  D(z) = z - net(z), the residual CNN loaded by
 *                 ri_load_denoiser (appendix C), applied facet by facet
 *                 (appendix D): each facet's tile carries a halo, pixels
 *                 outside the image are zero, only the core is written; all
 *                 facets go through each layer in one launch. param is unused;
 *                 z and out may not alias.
 * z, out: dev [N][N] (context precision; the CNN computes in FP32/bfloat16). */
ri_status denoise(ri_ctx *ctx, const void *z, void *out, int32_t kind, double param,
                  ri_stream stream);

/* One forward-backward iteration (eq. A2):
 *   x_out = D(x_in - gamma Re{Phi^dagger (Phi x_in - y)}).
 * y as in ri_gradient. norms: dev double[3] receiving, in FP64,
 * ||x_out - x_in||^2, ||x_out||^2, ||Phi x_in - y||^2 (or NULL).
 * x_in and x_out may not alias. */
ri_status fb_step(ri_ctx *ctx, const void *x_in, const void *y, double gamma, int32_t kind,
                  double param, void *x_out, double *norms, ri_stream stream);

/* Load the CNN denoiser of RI_PROX_CNN (appendix C): a residual network of
 * `layers` 3x3 convolutions with 64 hidden channels, parameters in the FP32
 * layout of ri_cnn.h (n_params = ri_cnn_param_count of such a network; dev,
 * copied on `stream`, converted to the bfloat16 kernel layout). The context
 * sizes the network's buffers for all its facets: facet_core x facet_core
 * facets with facet_halo pixels of halo (tiles rounded up to multiples of
 * 16), or the whole image when facet_core is 0. Needs N divisible by 16.
 * RI_EINVAL when n_params does not match `layers`. */
ri_status ri_load_denoiser(ri_ctx *ctx, const float *params, int64_t n_params, int32_t layers,
                           ri_stream stream);

/* Whole solve: parameters from the paper's rules (appendices B, C, F), FB or
 * PnP-FB iterations from x = 0, divergence watch with Haar fallback (CNN).
 * Haar and SARA: t = tau / sqrt(2L) (eq. B2, eq. lambda); SARA starts from
 * w = 1 and a zero dual variable and reweights every reweight_every
 * iterations (uSARA). CNN: the problem is rescaled by
 * alpha = max(dirty peak / beta, tau / (sigma_train sqrt(2L))) with beta the
 * dirty-beam peak (appendix F), so that the rescaled noise level
 * tau / (alpha sqrt(2L)) does not exceed the training level (eqs. C2-C3); the
 * result is multiplied back by alpha. */
typedef struct {
    int32_t max_iter;      /* iterations */
    double rel_tol;        /* stop when ||x^{k+1}-x^k|| / ||x^{k+1}|| <= rel_tol (0: never) */
    int32_t prox_kind;     /* RI_PROX_HAAR or RI_PROX_CNN */
    double tau;            /* visibility noise std (eq. 1) */
    double sigma_train;    /* CNN training noise level (eq. C3); ignored for Haar */
    double L;              /* ||Phi||_S^2 if known (> 0), else computed by ri_power_norm */
    int32_t check_every;   /* host reads the FP64 norms every check_every iterations (>= 1) */
    const void *x_true;    /* optional dev [N][N] ground truth for the SNR trace, or NULL */
    double *trace;         /* optional host [max_iter][4]: rel change, ||r||^2, SNR dB, ms */
    int32_t use_graph;     /* 1: replay a hipGraph of two captured iterations */
    int32_t diverge_checks;/* CNN only: fall back to Haar after this many consecutive checks at
                              which the residual ||Phi x - y||^2 grew by more than 1% since the
                              previous check, or at once on a non-finite norm (0: 3) */
    int32_t reweight_every;/* SARA only: after every this many iterations the log-sum weights
                              are renewed, w = rho / (rho + |Psi^dagger x|) with rho = t
                              (0: plain weighted l1 with w = 1, no reweighting) */
    int32_t use_holo;      /* 1: every gradient through the holographic matrix built by
                              ri_holo_build, Re{Z^dagger F^dagger H F Z} x - Re{Phi^dagger y}, with
                              Re{Phi^dagger y} and ||y||^2 from one pass over the visibilities at the
                              start; the reported ||Phi x - y||^2 is then
                              <x, Re Phi^dagger Phi x> - 2 <x, Re Phi^dagger y> + ||y||^2 (FP64 sums of
                              context-precision terms, so it loses relative accuracy as the residual
                              approaches the noise level). 0: the pass over the visibilities. */
} ri_solve_opts;

typedef struct {
    int32_t iters;
    double L, gamma, alpha, t_or_sigma;
    double final_rel_change, final_residual2, snr_db;
    int32_t fell_back;
    double ms;             /* wall time of the iterations (setup excluded) */
} ri_solve_report;

/* y: dev [M] complex (caller's order) or NULL for the stored data.
 * x_out: dev [N][N] (context precision), the solution multiplied back by alpha.
 * Synchronous: waits for all work already issued on the device (y and x_true
 * may come from asynchronous calls on any stream), runs on a stream of its own
 * and returns when x_out is written. */
ri_status pnp_solve(ri_ctx *ctx, const void *y, const ri_solve_opts *opts, void *x_out,
                    ri_solve_report *report);

/* uSARA's denoiser state (RI_PROX_SARA). ri_sara_setup allocates it on first
 * use (dual variable and weights, [9][N][N] each, plus two [8][N][N] work
 * arrays, in the context precision), sets the number of dual forward-backward
 * sub-iterations per prox (>= 1), and resets the dual variable to 0 and the
 * weights to 1. Needs N divisible by 16. */
ri_status ri_sara_setup(ri_ctx *ctx, int32_t sub_iters, ri_stream stream);

/* Log-sum reweighting: w = rho / (rho + |Psi^dagger x|) (the weights of the
 * penalty's linear majorant at x), rho > 0. x: dev [N][N]. */
ri_status ri_sara_reweight(ri_ctx *ctx, const void *x, double rho, ri_stream stream);

/* The dictionary itself: coef = Psi^dagger x and x = Psi coef, coef dev
 * [9][N][N] (slot 0 the Dirac basis, slot p the Daubechies wavelet with p
 * vanishing moments in the usual pyramid layout: each level's low-low block in
 * the top-left corner, then its three detail blocks), both scaled by 1/3. */
ri_status ri_sara_analysis(ri_ctx *ctx, const void *x, void *coef, ri_stream stream);
ri_status ri_sara_synthesis(ri_ctx *ctx, const void *coef, void *x, ri_stream stream);

/* Copy the dual variable and/or the weights (dev [9][N][N] each, NULL to skip). */
ri_status ri_sara_get_state(ri_ctx *ctx, void *v, void *w, ri_stream stream);

/* Holographic form of the normal operator (appendix E): with the data in
 * blocks p, Phi^dagger Phi = Z^dagger F^dagger H F Z with H = sum_p G_p^H G_p
 * (eq. E2), an N'^2 x N'^2 grid operator whose size follows the uv coverage
 * and the window sides, not the number of visibilities. H is banded: entry
 * H[k][k'] vanishes unless one window holds both cells (per axis
 * |k - k'| <= largest window side - 1).
 *
 * ri_holo_build accumulates H on the device from the context's plan (FP64
 * window weights, stored in the context precision) and keeps it in the
 * context: the upper half of the band of every 32 x 32 grid tile that some
 * window touches, the lower half being its conjugate transpose. Replaces a
 * previous H. Synchronous. RI_EUNSUPPORTED with w-stacking (n_wstacks > 1) or
 * when a tile's band does not fit the workgroup LDS; RI_ENOMEM when H does
 * not fit the device. ri_holo_release frees it (also done by ri_destroy). */
ri_status ri_holo_build(ri_ctx *ctx, ri_stream stream);
ri_status ri_holo_release(ri_ctx *ctx);

/* Y = H X on the fine grid. X, Y: dev [N'][N'] complex (context precision),
 * row-major [ky][kx] with the image centre at cell 0 (frequency index k at
 * k mod N'); Y is overwritten; X and Y may not alias. RI_EINVAL before
 * ri_holo_build. */
ri_status ri_holo_apply(ri_ctx *ctx, const void *X, void *Y, ri_stream stream);

/* out = Re{Phi^dagger Phi} x = Re{Z^dagger F^dagger H F Z} x through H (no pass
 * over the visibilities). x, out: dev [N][N] real (context precision). */
ri_status ri_holo_normal(ri_ctx *ctx, const void *x, void *out, ri_stream stream);

typedef struct {
    int64_t tiles;         /* stored 32 x 32 grid tiles */
    int64_t entries;       /* stored complex entries (upper half of each tile's band) */
    int64_t bytes;         /* device bytes of those entries */
    int64_t pairs;         /* window-cell pairs accumulated by the build */
    int32_t max_reach;     /* largest band half-width R over the tiles */
    double build_ms;       /* wall time of the last ri_holo_build */
} ri_holo_stats;
ri_status ri_holo_get_stats(const ri_ctx *ctx, ri_holo_stats *out);

/* Plan statistics for tests and the benchmark. */
typedef struct {
    int64_t M, nnz;        /* visibilities, stored/implied G entries */
    int32_t N, Np, tile, n_tiles, n_items, n_blocks;
    int64_t max_item_vis;  /* largest work item */
    int64_t device_bytes;  /* device memory held by the context */
    double plan_ms;        /* host + device time of ri_create */
    int32_t n_tuned;       /* tile sides the autotuner timed (0 when the tile was given) */
    int32_t tuned_tile[4];
    double tuned_ms[4];    /* milliseconds per fused gradient pass at each timed tile */
} ri_plan_stats;
ri_status ri_get_plan_stats(const ri_ctx *ctx, ri_plan_stats *out);

/* Copy internal per-visibility plan data to host arrays for exact checks
 * (each may be NULL): cell_u, cell_v (int32, window centres mod N'), plane
 * (int32), in the caller's visibility order; plane_h (int32 [n_wplanes]). */
ri_status ri_get_plan_arrays(const ri_ctx *ctx, int32_t *cell_u, int32_t *cell_v,
                             int32_t *plane, int32_t *plane_h);

/* Kernel timing for benchmarks: while enabled, every launch group records a
 * pair of HIP events on the stream it is launched on; ri_profile_read
 * synchronises on the last event and sums the elapsed times per category.
 * ri_profile(ctx, 1) clears previous records. Adds two event records per
 * launch group; leave it off in production loops. */
typedef struct {
    int32_t n_tiles, n_fft, n_prox, n_other;     /* timed launch groups per category */
    double tiles_ms;   /* persistent uv-tile kernel (degrid / grid / fused gradient pass) */
    double fft_ms;     /* Z + row FFTs + column passes, and their inverses */
    double prox_ms;    /* denoiser kernels */
    double other_ms;
} ri_kernel_times;
ri_status ri_profile(ri_ctx *ctx, int32_t enable);
ri_status ri_profile_read(ri_ctx *ctx, ri_kernel_times *out);

#ifdef __cplusplus
}
#endif

#endif /* RI_H */
