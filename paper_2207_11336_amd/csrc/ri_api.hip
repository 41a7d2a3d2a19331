// C ABI of libri.so: argument checks, context lifetime, and the sequencing of
// the kernels for each entry point. Every numerical step runs in the HIP
// kernels of fft.hip, gridding.hip and image.hip.
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "ri_internal.h"

using namespace ri;

namespace {

thread_local std::string g_last_error;

template <typename F>
ri_status guard(const ri_ctx *c, F &&fn) {
    try {
        fn();
        return RI_OK;
    } catch (const Error &e) {
        if (c) const_cast<ri_ctx *>(c)->err = e.msg;
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        if (c) const_cast<ri_ctx *>(c)->err = "host allocation failed";
        g_last_error = "host allocation failed";
        return RI_ENOMEM;
    } catch (const std::exception &e) {
        if (c) const_cast<ri_ctx *>(c)->err = e.what();
        g_last_error = e.what();
        return RI_EDEVICE;
    }
}

void require(bool ok, const std::string &msg) {
    if (!ok) throw Error(RI_EINVAL, msg);
}

int pick_tile(ri_ctx *c, int requested, int elem_bytes) {
    int t = requested > 0 ? requested : 16;
    if (t > c->Np) t = c->Np;
    if (requested > 0) {
        require((t & (t - 1)) == 0 || c->Np % t == 0, "tile must divide N'");
        if (lds_for_tile(t, c->H, elem_bytes) > (size_t)c->dev.lds_per_block)
            throw Error(RI_EUNSUPPORTED, "tile " + std::to_string(t) + " does not fit the workgroup LDS");
        return t;
    }
    while (t > 8 && lds_for_tile(t, c->H, elem_bytes) > (size_t)c->dev.lds_per_block) t /= 2;
    return t;
}

hipStream_t st(ri_stream s) { return reinterpret_cast<hipStream_t>(s); }

double *tile_part(ri_ctx *c) { return c->d_partials; }
double *img_part(ri_ctx *c) { return c->d_partials + tiles_partials(c); }

// FP64 view for the power iteration: the main view when it already carries
// FP64 fractions at a tile that fits FP64 subgrids, else a dedicated one at
// the main view's (autotuned) tile, halved until its FP64 subgrids fit (at C1
// tile 8 runs the FP64 pass 8% faster than tile 16).
const View &view_fp64(ri_ctx *c) {
    if (c->view.frac_bytes == 8 && lds_for_tile(c->view.tile, c->H, 16) <= (size_t)c->dev.lds_per_block)
        return c->view;
    if (!c->view64.items) {
        int t = c->view.tile > 0 ? c->view.tile : 16;
        while (t > 8 && lds_for_tile(t, c->H, 16) > (size_t)c->dev.lds_per_block) t /= 2;
        build_view(c, c->view64, pick_tile(c, t, 16), 8);
    }
    return c->view64;
}

template <typename T>
Prec<T> &prec(ri_ctx *c);
template <>
Prec<float> &prec<float>(ri_ctx *c) { return c->p32; }
template <>
Prec<double> &prec<double>(ri_ctx *c) { return c->p64; }

template <typename T>
void do_forward(ri_ctx *c, const T *x, cx<T> *y, hipStream_t s) {
    Prec<T> &p = prec<T>(c);
    fwd_zpad_fft<T>(c, p, x, s);
    launch_tiles<T>(c, c->view, p, OP_DEGRID, c->d.g_mode, nullptr, nullptr, y, nullptr, s);
}

template <typename T>
void do_adjoint(ri_ctx *c, const cx<T> *y, T *x, hipStream_t s) {
    Prec<T> &p = prec<T>(c);
    fill_zero<T>(p.gridA, (int64_t)c->P * c->Np * c->Np, s);
    launch_tiles<T>(c, c->view, p, OP_GRID, c->d.g_mode, nullptr, y, nullptr, nullptr, s);
    adj_fft_crop<T>(c, p, x, s);
}

// g = Re{Phi^dagger (Phi x - y)} with y in internal order (or none); r2 partials in tile_part.
template <typename T>
void do_gradient(ri_ctx *c, const View &v, int gm, const T *x, const cx<T> *y_sorted, T *g, hipStream_t s) {
    Prec<T> &p = prec<T>(c);
    fwd_zpad_fft<T>(c, p, x, s);
    fill_zero<T>(p.gridA, (int64_t)c->P * c->Np * c->Np, s);
    launch_tiles<T>(c, v, p, OP_FUSED, gm, y_sorted, nullptr, nullptr, tile_part(c), s);
    adj_fft_crop<T>(c, p, g, s);
}

template <typename T>
const cx<T> *resolve_data(ri_ctx *c, const void *y, hipStream_t s) {
    if (y == RI_NO_DATA) return nullptr;
    Prec<T> &p = prec<T>(c);
    if (y != nullptr) {
        permute_to_internal<T>((const cx<T> *)y, p.ydata, c->view.perm, c->M, s);
        return p.ydata;
    }
    require(c->has_data, "y is NULL but no data was stored with ri_set_data");
    return p.ydata;
}

// One iteration of eq. (A2) with the data in internal order (or none). norms
// (dev double[3], or [4] with x_true): ||x_out - x_in||^2, ||x_out||^2,
// ||Phi x_in - y||^2 and ||alpha x_out - x_true||^2.
// With holo_dirty (and holo_yy), the gradient comes from the stored holographic
// matrix: g = Re{Z^dagger F^dagger H F Z} x - Re{Phi^dagger y}, and
// ||Phi x - y||^2 = <x, Re Phi^dagger Phi x> - 2 <x, Re Phi^dagger y> + ||y||^2.
template <typename T>
void fb_step_sorted(ri_ctx *c, const T *x_in, const cx<T> *ys, double gamma, int kind, double param, T *x_out,
                    double *norms, const T *x_true, double alpha, hipStream_t s, const T *holo_dirty = nullptr,
                    const double *holo_yy = nullptr) {
    Prec<T> &p = prec<T>(c);
    const bool holo = holo_dirty != nullptr;
    if (holo) {
        const int64_t nn = (int64_t)c->N * c->N;
        holo_normal<T>(c, p, x_in, p.img0, s);
        if (norms) {
            double *dots = c->d_scalars + 40;
            dot_partials<T>(x_in, p.img0, nn, img_part(c), s);
            reduce_partials(img_part(c), 1024, 1, 1, dots, s);
            dot_partials<T>(x_in, holo_dirty, nn, img_part(c), s);
            reduce_partials(img_part(c), 1024, 1, 1, dots + 1, s);
            holo_residual(norms + 2, dots, holo_yy, s);
        }
        axpby<T>(p.img0, p.img0, (T)1, holo_dirty, (T)(-1), nn, s);
    } else {
        do_gradient<T>(c, c->view, c->d.g_mode, x_in, ys, p.img0, s);
    }
    if (kind == RI_PROX_HAAR) {
        const int nwg = ((c->N / 16) * (c->N / 16) + 3) / 4;
        haar_prox<T>(c, x_in, p.img0, (T)gamma, nullptr, (T)param, x_out, img_part(c), s);
        if (norms) {
            reduce_partials(img_part(c), nwg, 2, 2, norms, s);
            if (!holo) reduce_partials(tile_part(c), tiles_partials(c), 1, 1, norms + 2, s);
        }
    } else {
        // z = x - gamma g, x_out = D(z): the CNN facet by facet (PnP step) or
        // uSARA's sub-iterative prox
        const int64_t n = (int64_t)c->N * c->N;
        axpby<T>(p.img1, x_in, (T)1, p.img0, (T)(-gamma), n, s);
        if (kind == RI_PROX_SARA) {
            if (!c->sara.ready) sara_setup(c, 0, s);
            sara_prox<T>(c, p.img1, (T)param, x_out, s);
        } else {
            require(c->cnn != nullptr, "no CNN denoiser loaded (ri_load_denoiser)");
            ProfScope ps(c, PROF_PROX, s);
            cnn_denoise<T>(c->cnn, p.img1, x_out, c->N, c->d.facet_core, c->d.facet_halo, s);
        }
        if (norms) {
            diff2_partials<T>(x_out, (T)1, x_in, n, img_part(c), s);
            reduce_partials(img_part(c), 1024, 1, 1, norms, s);
            dot_partials<T>(x_out, x_out, n, img_part(c), s);
            reduce_partials(img_part(c), 1024, 1, 1, norms + 1, s);
            if (!holo) reduce_partials(tile_part(c), tiles_partials(c), 1, 1, norms + 2, s);
        }
    }
    if (norms && x_true) {
        diff2_partials<T>(x_out, (T)alpha, x_true, (int64_t)c->N * c->N, img_part(c), s);
        reduce_partials(img_part(c), 1024, 1, 1, norms + 3, s);
    }
}

template <typename T>
void do_fb_step(ri_ctx *c, const T *x_in, const void *y, double gamma, int kind, double param, T *x_out,
                double *norms, hipStream_t s) {
    const cx<T> *ys = resolve_data<T>(c, y, s);
    fb_step_sorted<T>(c, x_in, ys, gamma, kind, param, x_out, norms, nullptr, 1.0, s);
}

// Main view at tile T (FP64 fractions when G is stored or the context is
// FP64), plus the CSR G in that view's order. The holographic matrix and the
// SARA state are grid- and image-level and do not depend on the view's
// visibility order, so they are kept.
void build_main_view(ri_ctx *c, int tile) {
    const bool f64frac = c->d.g_mode != RI_G_OTF || c->d.precision == 64;
    free_view(c, c->view);
    if (c->csr.val) {
        dev_free(c, c->csr.rowptr);
        dev_free(c, c->csr.val);
        c->csr = CSR();
    }
    if (c->sep.w) {
        dev_free(c, c->sep.w);
        c->sep = Sep();
    }
    build_view(c, c->view, tile, f64frac ? 8 : 4);
    if (c->d.g_mode == RI_G_CSR) {
        if (c->d.precision == 32) fill_csr<float>(c, nullptr);
        else fill_csr<double>(c, nullptr);
    } else if (c->d.g_mode == RI_G_SEP) {
        if (c->d.precision == 32) fill_sep<float>(c, nullptr);
        else fill_sep<double>(c, nullptr);
    }
}

// Tile autotuner: for each candidate tile side whose subgrids fit the
// workgroup LDS, build the view (and the CSR G in its order), time three fused
// gradient passes on a constant image after one warm-up, keep the fastest.
// The side also selects the gridding form of FP32 contexts with separable
// rows (VALU gather, matrix-core gather or scatter by the subgrid side), so
// the timing compares forms as well as item sizes.
template <typename T>
void autotune_tile(ri_ctx *c) {
    const int eb = sizeof(T) == 4 ? 8 : 16;
    Prec<T> &p = prec<T>(c);
    const int64_t n = (int64_t)c->N * c->N;
    fill_real<T>(p.img1, n, (T)1, nullptr);
    int best = 0;
    float best_ms = 1e30f;
    hipEvent_t e0, e1;
    RI_CHECK_HIP(hipEventCreate(&e0));
    RI_CHECK_HIP(hipEventCreate(&e1));
    for (int t : {8, 16, 32}) {
        if (t > c->Np || c->Np % t) continue;
        if (lds_for_tile(t, c->H, eb) > (size_t)c->dev.lds_per_block) continue;
        build_main_view(c, t);
        do_gradient<T>(c, c->view, c->d.g_mode, p.img1, nullptr, p.img0, nullptr);
        RI_CHECK_HIP(hipEventRecord(e0, nullptr));
        for (int r = 0; r < 3; ++r)
            do_gradient<T>(c, c->view, c->d.g_mode, p.img1, nullptr, p.img0, nullptr);
        RI_CHECK_HIP(hipEventRecord(e1, nullptr));
        RI_CHECK_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        RI_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
        c->tune_ms.push_back({t, ms / 3});
        if (ms < best_ms) { best_ms = ms; best = t; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best == 0) throw Error(RI_EUNSUPPORTED, "no tile size fits the workgroup LDS");
    if (c->view.tile != best) build_main_view(c, best);
}

template <typename T>
double power_iteration(ri_ctx *c, int max_it, double rtol, const double *x0, int *iters, bool *conv,
                       hipStream_t s) {
    ensure_prec<double>(c, c->p64);
    const View &v = view_fp64(c);
    Prec<double> &p = c->p64;
    const int64_t n = (int64_t)c->N * c->N;
    double *x = p.img0, *y = p.img1;
    if (x0) RI_CHECK_HIP(hipMemcpyAsync(x, x0, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    else {
        std::vector<double> h(n);
        uint64_t z = 0x9E3779B97F4A7C15ull;
        for (int64_t i = 0; i < n; ++i) {   // splitmix64 stream -> uniform [-1/2, 1/2)
            z += 0x9E3779B97F4A7C15ull;
            uint64_t r = z;
            r = (r ^ (r >> 30)) * 0xBF58476D1CE4E5B9ull;
            r = (r ^ (r >> 27)) * 0x94D049BB133111EBull;
            r ^= r >> 31;
            h[i] = (double)(r >> 11) * (1.0 / 9007199254740992.0) - 0.5;
        }
        RI_CHECK_HIP(hipMemcpyAsync(x, h.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
        RI_CHECK_HIP(hipStreamSynchronize(s));
    }
    double *ss = c->d_scalars;
    dot_partials<double>(x, x, n, img_part(c), s);
    reduce_partials(img_part(c), 1024, 1, 1, ss, s);
    scale_by_inv_sqrt(x, ss, n, s);
    double L = 0.0;
    *conv = false;
    int it = 0;
    for (it = 1; it <= max_it; ++it) {
        do_gradient<double>(c, v, RI_G_OTF, x, nullptr, y, s);
        dot_partials<double>(y, y, n, img_part(c), s);
        reduce_partials(img_part(c), 1024, 1, 1, ss, s);
        scale_by_inv_sqrt(y, ss, n, s);
        RI_CHECK_HIP(hipMemcpyAsync(c->h_pinned, ss, sizeof(double), hipMemcpyDeviceToHost, s));
        RI_CHECK_HIP(hipStreamSynchronize(s));
        const double Ln = std::sqrt(c->h_pinned[0]);
        std::swap(x, y);
        if (it > 1 && std::fabs(Ln - L) <= rtol * Ln) { L = Ln; *conv = true; break; }
        L = Ln;
    }
    if (it > max_it) it = max_it;
    *iters = it;
    // keep the latest unit vector in img0
    if (x != p.img0) RI_CHECK_HIP(hipMemcpyAsync(p.img0, x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    return L;
}

// Peak of the dirty image Re{Phi^dagger y} (y in internal order), via the
// fused gradient at x = 0, which returns -Re{Phi^dagger y}.
template <typename T>
double dirty_peak(ri_ctx *c, const cx<T> *ys, hipStream_t s) {
    Prec<T> &p = prec<T>(c);
    const int64_t n = (int64_t)c->N * c->N;
    fill_real<T>(p.img1, n, (T)0, s);
    do_gradient<T>(c, c->view, c->d.g_mode, p.img1, ys, p.img0, s);
    axpby<T>(p.img0, p.img0, (T)-1, nullptr, (T)0, n, s);
    max_value<T>(p.img0, n, img_part(c), c->d_scalars, s);
    RI_CHECK_HIP(hipMemcpyAsync(c->h_pinned, c->d_scalars, sizeof(double), hipMemcpyDeviceToHost, s));
    RI_CHECK_HIP(hipStreamSynchronize(s));
    return c->h_pinned[0];
}

// beta = max_i (Re{Phi^dagger Phi} delta)_i, delta = 1 at the phase centre
// (pixel (N/2, N/2) of the row-major image whose centre is index 0 of the grid).
template <typename T>
double dirty_beam_peak(ri_ctx *c, hipStream_t s) {
    Prec<T> &p = prec<T>(c);
    const int64_t n = (int64_t)c->N * c->N;
    fill_real<T>(p.img1, n, (T)0, s);
    fill_real<T>(p.img1 + (int64_t)(c->N / 2) * c->N + c->N / 2, 1, (T)1, s);
    do_gradient<T>(c, c->view, c->d.g_mode, p.img1, nullptr, p.img0, s);
    max_value<T>(p.img0, n, img_part(c), c->d_scalars, s);
    RI_CHECK_HIP(hipMemcpyAsync(c->h_pinned, c->d_scalars, sizeof(double), hipMemcpyDeviceToHost, s));
    RI_CHECK_HIP(hipStreamSynchronize(s));
    return c->h_pinned[0];
}

// Forward-backward solve on its own stream. The iteration is captured once
// as a graph of two steps (a -> b -> a) when requested and replayed; the FP64
// norms of every step are copied out of the graph's fixed slots after each
// replay, and read on the host every check_every iterations.
template <typename T>
bool solve(ri_ctx *c, const void *y, const ri_solve_opts &o, T *x_out, ri_solve_report *rep) {
    // The caller's y, x_true and denoiser may still be in flight on any
    // stream (the solve takes none): wait for all work issued so far, since
    // the solve's own stream does not order itself after the others.
    RI_CHECK_HIP(hipDeviceSynchronize());
    hipStream_t s = nullptr;
    RI_CHECK_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    const int64_t n = (int64_t)c->N * c->N;
    const int K = o.max_iter;
    std::vector<void *> owned;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<hipEvent_t> evs;
    auto cleanup = [&] {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        for (auto e : evs) (void)hipEventDestroy(e);
        for (void *q : owned) dev_free(c, q);
        (void)hipStreamDestroy(s);
    };
    bool fell = false;
    try {
        const cx<T> *ys = resolve_data<T>(c, y, s);
        if (y) c->has_data = true;
        require(c->has_data || c->M == 0, "no data: pass y or store it with ri_set_data");
        double L = o.L;
        if (!(L > 0.0)) {
            bool conv = false;
            int it = 0;
            L = power_iteration<double>(c, 500, 1e-8, nullptr, &it, &conv, s);
        }
        ri_solve_report rr{};
        rr.L = L;
        rr.gamma = 1.98 / L;
        rr.alpha = 1.0;
        int kind = o.prox_kind;
        double param = o.tau / std::sqrt(2.0 * L);
        if (kind == RI_PROX_CNN) {
            // Rescaled problem (eqs. C2-C3): alpha bounds the image peak (from
            // the dirty image normalised by the dirty-beam peak) and is raised
            // until the image-domain noise tau / (alpha sqrt(2L)) is at most
            // the training level; the data are divided by alpha.
            require(c->cnn != nullptr, "no CNN denoiser loaded (ri_load_denoiser)");
            require(o.sigma_train > 0.0, "sigma_train must be > 0 for the CNN denoiser");
            const double peak = dirty_peak<T>(c, ys, s);
            const double beta = dirty_beam_peak<T>(c, s);
            require(beta > 0.0, "dirty-beam peak is not positive");
            rr.alpha = std::max(peak / beta, o.tau / (o.sigma_train * std::sqrt(2.0 * L)));
            require(std::isfinite(rr.alpha) && rr.alpha > 0.0, "alpha is not positive (empty data?)");
            cx<T> *yscaled = (cx<T> *)dev_alloc(c, sizeof(cx<T>) * std::max<int64_t>(1, c->M));
            owned.push_back(yscaled);
            axpby<T>((T *)yscaled, (const T *)ys, (T)(1.0 / rr.alpha), nullptr, (T)0, 2 * c->M, s);
            ys = yscaled;
            param = o.tau / (rr.alpha * std::sqrt(2.0 * L));
        }
        rr.t_or_sigma = param;
        if (kind == RI_PROX_SARA) sara_setup(c, 0, s);   // v = 0, w = 1 (plain weighted l1 first)
        T *xa = (T *)dev_alloc(c, sizeof(T) * n); owned.push_back(xa);
        T *hdirty = nullptr;
        double *hyy = nullptr;
        if (o.use_holo) {
            // Re{Phi^dagger y} and ||y||^2 from one pass over the visibilities at x = 0
            require(c->holo.ready, "use_holo needs the holographic matrix (ri_holo_build)");
            hdirty = (T *)dev_alloc(c, sizeof(T) * n); owned.push_back(hdirty);
            hyy = (double *)dev_alloc(c, sizeof(double)); owned.push_back(hyy);
            fill_real<T>(xa, n, (T)0, s);
            do_gradient<T>(c, c->view, c->d.g_mode, xa, ys, hdirty, s);
            reduce_partials(tile_part(c), tiles_partials(c), 1, 1, hyy, s);
            axpby<T>(hdirty, hdirty, (T)(-1), nullptr, (T)0, n, s);
        }
        T *xb = (T *)dev_alloc(c, sizeof(T) * n); owned.push_back(xb);
        T *xsave = (T *)dev_alloc(c, sizeof(T) * n); owned.push_back(xsave);
        double *slots = (double *)dev_alloc(c, sizeof(double) * 8); owned.push_back(slots);
        double *nrm = (double *)dev_alloc(c, sizeof(double) * 4 * std::max(1, K)); owned.push_back(nrm);
        fill_real<T>(xa, n, (T)0, s);
        fill_real<T>(xsave, n, (T)0, s);
        fill_zero_f64(slots, 8, s);
        fill_zero_f64(nrm, 4 * (int64_t)std::max(1, K), s);
        const T *xt = (const T *)o.x_true;
        double xt2 = 0.0;
        if (xt) {
            dot_partials<T>(xt, xt, n, img_part(c), s);
            reduce_partials(img_part(c), 1024, 1, 1, c->d_scalars, s);
            RI_CHECK_HIP(hipMemcpyAsync(c->h_pinned, c->d_scalars, sizeof(double), hipMemcpyDeviceToHost, s));
        }
        RI_CHECK_HIP(hipStreamSynchronize(s));
        if (xt) xt2 = c->h_pinned[0];
        const bool prof_was = c->prof_on;
        c->prof_on = false;
        auto capture = [&](int kd, double prm) {
            if (gexec) { (void)hipGraphExecDestroy(gexec); gexec = nullptr; }
            if (graph) { (void)hipGraphDestroy(graph); graph = nullptr; }
            RI_CHECK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            try {
                fb_step_sorted<T>(c, xa, ys, rr.gamma, kd, prm, xb, slots, xt, rr.alpha, s, hdirty, hyy);
                fb_step_sorted<T>(c, xb, ys, rr.gamma, kd, prm, xa, slots + 4, xt, rr.alpha, s, hdirty, hyy);
            } catch (...) {
                hipGraph_t g2 = nullptr;
                (void)hipStreamEndCapture(s, &g2);
                if (g2) (void)hipGraphDestroy(g2);
                throw;
            }
            RI_CHECK_HIP(hipStreamEndCapture(s, &graph));
            RI_CHECK_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
        };
        if (o.use_graph && K >= 2) capture(kind, param);
        hipEvent_t e0;
        RI_CHECK_HIP(hipEventCreate(&e0)); evs.push_back(e0);
        std::vector<std::pair<int, hipEvent_t>> marks;   // (iterations done, event)
        RI_CHECK_HIP(hipEventRecord(e0, s));
        const int div_n = o.diverge_checks > 0 ? o.diverge_checks : 3;
        int rising = 0, k = 0, next_check = o.check_every, reweights = 0;
        double last_r2 = -1.0;
        std::vector<double> h(4 * std::max(1, K));
        while (k < K) {
            if (gexec && k + 2 <= K) {
                RI_CHECK_HIP(hipGraphLaunch(gexec, s));
                RI_CHECK_HIP(hipMemcpyAsync(nrm + 4 * k, slots, sizeof(double) * 8, hipMemcpyDeviceToDevice, s));
                k += 2;
            } else {
                fb_step_sorted<T>(c, xa, ys, rr.gamma, kind, param, xb, nrm + 4 * k, xt, rr.alpha, s, hdirty, hyy);
                RI_CHECK_HIP(hipMemcpyAsync(xa, xb, sizeof(T) * n, hipMemcpyDeviceToDevice, s));
                k += 1;
            }
            if (kind == RI_PROX_SARA && o.reweight_every > 0 && k / o.reweight_every > reweights && k < K) {
                // log-sum reweighting (rho = gamma lambda): w = rho / (rho + |Psi^dagger x|)
                reweights = k / o.reweight_every;
                sara_reweight<T>(c, xa, (T)param, s);
            }
            hipEvent_t ev;
            RI_CHECK_HIP(hipEventCreate(&ev)); evs.push_back(ev);
            RI_CHECK_HIP(hipEventRecord(ev, s));
            marks.push_back({k, ev});
            if (k >= next_check || k == K) {
                next_check = k + o.check_every;
                RI_CHECK_HIP(hipMemcpyAsync(h.data() + 4 * (k - 1), nrm + 4 * (k - 1), sizeof(double) * 4,
                                            hipMemcpyDeviceToHost, s));
                RI_CHECK_HIP(hipStreamSynchronize(s));
                const double *q = h.data() + 4 * (k - 1);
                const bool finite = std::isfinite(q[0]) && std::isfinite(q[1]) && std::isfinite(q[2]);
                // a check counts as rising when the residual grew by more than 1%:
                // a converging PnP iterate may drift up by less on its way to the
                // fixed point, a diverging one grows geometrically
                rising = (last_r2 >= 0.0 && q[2] > 1.01 * last_r2) ? rising + 1 : 0;
                last_r2 = q[2];
                if (!finite || (kind == RI_PROX_CNN && rising >= div_n)) {
                    if (kind != RI_PROX_CNN) throw Error(RI_EDEVICE, "non-finite iterate with a convex prox");
                    // restore the last healthy iterate and continue with the Haar prox
                    RI_CHECK_HIP(hipMemcpyAsync(xa, xsave, sizeof(T) * n, hipMemcpyDeviceToDevice, s));
                    kind = RI_PROX_HAAR;
                    param = o.tau / (rr.alpha * std::sqrt(2.0 * L));
                    fell = true;
                    rising = 0;
                    last_r2 = -1.0;
                    if (gexec) capture(kind, param);
                    continue;
                }
                RI_CHECK_HIP(hipMemcpyAsync(xsave, xa, sizeof(T) * n, hipMemcpyDeviceToDevice, s));
                rr.final_rel_change = q[1] > 0 ? std::sqrt(q[0] / q[1]) : 0.0;
                if (o.rel_tol > 0 && rr.final_rel_change <= o.rel_tol) break;
            }
        }
        RI_CHECK_HIP(hipStreamSynchronize(s));
        c->prof_on = prof_was;
        float ms_total = 0.f;
        if (!marks.empty()) RI_CHECK_HIP(hipEventElapsedTime(&ms_total, e0, marks.back().second));
        rr.iters = k;
        rr.ms = ms_total;
        rr.fell_back = fell ? 1 : 0;
        if (k > 0) {
            RI_CHECK_HIP(hipMemcpy(h.data(), nrm, sizeof(double) * 4 * k, hipMemcpyDeviceToHost));
            const double *q = h.data() + 4 * (k - 1);
            rr.final_rel_change = q[1] > 0 ? std::sqrt(q[0] / q[1]) : 0.0;
            rr.final_residual2 = q[2];
            rr.snr_db = xt && q[3] > 0 ? 10.0 * std::log10(xt2 / q[3]) : 0.0;
            if (o.trace) {
                float prev_ms = 0.f;
                int prev_k = 0;
                for (auto &mk_ : marks) {
                    float ms = 0.f;
                    RI_CHECK_HIP(hipEventElapsedTime(&ms, e0, mk_.second));
                    for (int j = prev_k; j < mk_.first; ++j) {
                        const double *qq = h.data() + 4 * j;
                        double *tr = o.trace + 4 * j;
                        tr[0] = qq[1] > 0 ? std::sqrt(qq[0] / qq[1]) : 0.0;
                        tr[1] = qq[2];
                        tr[2] = xt && qq[3] > 0 ? 10.0 * std::log10(xt2 / qq[3]) : 0.0;
                        tr[3] = prev_ms + (ms - prev_ms) * (double)(j + 1 - prev_k) / (double)(mk_.first - prev_k);
                    }
                    prev_ms = ms;
                    prev_k = mk_.first;
                }
            }
        }
        axpby<T>(x_out, xa, (T)rr.alpha, nullptr, (T)0, n, s);
        RI_CHECK_HIP(hipStreamSynchronize(s));
        if (rep) *rep = rr;
    } catch (...) {
        (void)hipStreamSynchronize(s);
        cleanup();
        throw;
    }
    cleanup();
    return fell;
}

}  // namespace

extern "C" {

ri_status ri_create(const ri_plan_desc *desc, const double *uvw, ri_ctx **out) {
    if (!out) { g_last_error = "out is NULL"; return RI_EINVAL; }
    *out = nullptr;
    ri_ctx *c = nullptr;
    ri_status st_ = guard(nullptr, [&] {
        require(desc != nullptr, "desc is NULL");
        const ri_plan_desc &d = *desc;
        require(d.N >= 16 && d.N <= 4096 && d.N % 2 == 0, "N must be even, 16..4096");
        const int Np = 2 * d.N;
        require((Np & (Np - 1)) == 0, "N' = 2N must be a power of two");
        require(d.oversample == 2, "oversample must be 2");
        require(d.kb_support == 7, "kb_support must be 7");
        require(d.hmax >= 0 && d.hmax <= 5, "hmax must be 0..5");
        require(d.n_wplanes >= 1 && d.n_wplanes % 2 == 1 && d.n_wplanes <= 65535, "n_wplanes must be odd, <= 65535");
        require(std::isfinite(d.w_max) && d.w_max >= 0.0, "w_max must be finite and >= 0");
        require(d.w_max == 0.0 || (std::isfinite(d.cell_rad) && d.cell_rad > 0.0), "cell_rad must be > 0");
        require(d.g_mode == RI_G_CSR || d.g_mode == RI_G_OTF || d.g_mode == RI_G_SEP,
                "g_mode must be RI_G_CSR, RI_G_OTF or RI_G_SEP");
        require(d.precision == 32 || d.precision == 64, "precision must be 32 or 64");
        require(d.tile == 0 || (d.tile >= 8 && d.tile <= 128 && Np % d.tile == 0), "tile must be 0 or divide N'");
        require(d.M >= 0 && d.M < (int64_t)1 << 31, "M must be in [0, 2^31)");
        require(d.M == 0 || uvw != nullptr, "uvw is NULL");
        require(d.n_blocks >= 1, "n_blocks must be >= 1");
        require(d.facet_core >= 0 && d.facet_core % 16 == 0 && d.facet_halo >= 0, "facet sizes");
        require(d.item_vis >= 0 && d.item_vis <= (1 << 20), "item_vis must be in [0, 2^20]");
        require(d.n_wstacks >= 0 && d.n_wstacks <= 64, "n_wstacks must be in [0, 64]");
        require(d.n_wstacks <= 1 || d.w_max > 0.0, "w-stacking needs w_max > 0");
        require(d.grid_form == RI_GRID_GATHER || d.grid_form == RI_GRID_SCATTER, "grid_form must be 0 or 1");
        c = new ri_ctx();
        c->d = d;
        c->d.block_offsets = nullptr;
        c->N = d.N;
        c->Np = Np;
        c->logNp = 0;
        while ((1 << c->logNp) < Np) ++c->logNp;
        c->J = 7;
        c->jh = 3;
        c->hmax = d.hmax;
        c->H = d.hmax + 3;
        c->M = d.M;
        c->P = d.n_wstacks > 1 ? d.n_wstacks : 1;
        {
            double a = 7.0 / 2.0 * (2.0 - 0.5);
            c->beta = M_PI * std::sqrt(a * a - 0.8);
        }
        if (d.block_offsets) {
            c->block_offsets.assign(d.block_offsets, d.block_offsets + d.n_blocks + 1);
            require(c->block_offsets.front() == 0 && c->block_offsets.back() == d.M, "block offsets must span 0..M");
            for (int b = 0; b < d.n_blocks; ++b)
                require(c->block_offsets[b] <= c->block_offsets[b + 1], "block offsets must be ascending");
        } else {
            require(d.n_blocks == 1, "n_blocks > 1 needs block_offsets");
            c->block_offsets = {0, d.M};
        }
        auto t0 = std::chrono::steady_clock::now();
        RI_CHECK_HIP(hipGetDevice(&c->device));
        noalloc_init_device(c->device);
        hipDeviceProp_t prop;
        RI_CHECK_HIP(hipGetDeviceProperties(&prop, c->device));
        c->dev.cu_count = prop.multiProcessorCount;
        c->dev.lds_per_block = (int)prop.sharedMemPerBlock;

        build_plan(c, uvw);
        const int eb = d.precision == 64 ? 16 : 8;
        if (d.precision == 32) ensure_prec<float>(c, c->p32);
        else ensure_prec<double>(c, c->p64);
        c->n_partials = tiles_partials(c);
        c->d_partials = (double *)dev_alloc(c, sizeof(double) * (size_t)(tiles_partials(c) + image_partials(c)));
        c->d_counter = (int32_t *)dev_alloc(c, 64 * sizeof(int32_t));
        c->d_scalars = (double *)dev_alloc(c, 64 * sizeof(double));
        RI_CHECK_HIP(hipHostMalloc((void **)&c->h_pinned, 64 * sizeof(double), hipHostMallocDefault));
        if (d.tile > 0 || c->M == 0) {
            build_main_view(c, pick_tile(c, d.tile, eb));
        } else {
            if (d.precision == 32) autotune_tile<float>(c);
            else autotune_tile<double>(c);
        }
        RI_CHECK_HIP(hipDeviceSynchronize());
        c->plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    });
    if (st_ != RI_OK) {
        if (c) ri_destroy(c);
        return st_;
    }
    *out = c;
    return RI_OK;
}

void ri_destroy(ri_ctx *c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    free_view(c, c->view);
    free_view(c, c->view64);
    dev_free(c, c->csr.rowptr); dev_free(c, c->csr.val);
    dev_free(c, c->sep.w);
    holo_free(c);
    auto freep = [c](auto &p) {
        dev_free(c, p.icorr); dev_free(c, p.tw); dev_free(c, p.wtaps); dev_free(c, p.gridA); dev_free(c, p.gridB);
        dev_free(c, p.chirp);
        dev_free(c, p.img0); dev_free(c, p.img1); dev_free(c, p.ydata);
    };
    freep(c->p32);
    freep(c->p64);
    dev_free(c, c->d_plane_h);
    dev_free(c, c->d_counter);
    dev_free(c, c->d_partials);
    dev_free(c, c->d_scalars);
    if (c->cnn) cnn_destroy(c->cnn);
    for (auto &a : c->allocs) (void)hipFree(a.first);
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    for (auto &e : c->prof_ev) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    for (auto &e : c->prof_pool) (void)hipEventDestroy(e);
    delete c;
}

const char *ri_last_error(const ri_ctx *c) { return c ? c->err.c_str() : g_last_error.c_str(); }

ri_status phi_forward(ri_ctx *c, const void *x, void *y, ri_stream s) {
    if (!c) return RI_EINVAL;
    return guard(c, [&] {
        require(x && (y || c->M == 0), "x or y is NULL");
        if (c->d.precision == 32) do_forward<float>(c, (const float *)x, (cx<float> *)y, st(s));
        else do_forward<double>(c, (const double *)x, (cx<double> *)y, st(s));
        RI_CHECK_HIP(hipGetLastError());
    });
}

ri_status phi_adjoint(ri_ctx *c, const void *y, void *x, ri_stream s) {
    if (!c) return RI_EINVAL;
    return guard(c, [&] {
        require(x && (y || c->M == 0), "x or y is NULL");
        if (c->d.precision == 32) do_adjoint<float>(c, (const cx<float> *)y, (float *)x, st(s));
        else do_adjoint<double>(c, (const cx<double> *)y, (double *)x, st(s));
        RI_CHECK_HIP(hipGetLastError());
    });
}

ri_status ri_set_data(ri_ctx *c, const void *y, ri_stream s) {
    if (!c) return RI_EINVAL;
    return guard(c, [&] {
        require(y || c->M == 0, "y is NULL");
        if (c->d.precision == 32) (void)resolve_data<float>(c, y, st(s));
        else (void)resolve_data<double>(c, y, st(s));
        c->has_data = true;
        RI_CHECK_HIP(hipGetLastError());
    });
}

ri_status ri_gradient(ri_ctx *c, const void *x, const void *y, void *g, double *r2, ri_stream s) {
    if (!c) return RI_EINVAL;
    return guard(c, [&] {
        require(x && g, "x or g is NULL");
        if (c->d.precision == 32) {
            const cx<float> *ys = resolve_data<float>(c, y, st(s));
            do_gradient<float>(c, c->view, c->d.g_mode, (const float *)x, ys, (float *)g, st(s));
        } else {
            const cx<double> *ys = resolve_data<double>(c, y, st(s));
            do_gradient<double>(c, c->view, c->d.g_mode, (const double *)x, ys, (double *)g, st(s));
        }
        if (r2) reduce_partials(tile_part(c), tiles_partials(c), 1, 1, r2, st(s));
        RI_CHECK_HIP(hipGetLastError());
    });
}

ri_status ri_power_norm(ri_ctx *c, int32_t max_it, double rtol, const double *x0, double *L, int32_t *iters,
                        ri_stream s) {
    if (!c) return RI_EINVAL;
    bool conv = false;
    ri_status r = guard(c, [&] {
        require(L != nullptr, "L is NULL");
        require(max_it >= 1 && rtol >= 0.0, "max_it >= 1 and rtol >= 0 required");
        int it = 0;
        *L = power_iteration<double>(c, max_it, rtol, x0, &it, &conv, st(s));
        if (iters) *iters = it;
        RI_CHECK_HIP(hipGetLastError());
    });
    if (r == RI_OK && rtol > 0.0 && !conv) {
        c->err = "power iteration reached max_it before rtol";
        return RI_ENOTCONV;
    }
    return r;
}

ri_status denoise(ri_ctx *c, const void *z, void *out, int32_t kind, double param, ri_stream s) {
    if (!c) return RI_EINVAL;
    return guard(c, [&] {
        require(z && out, "z or out is NULL");
        require(kind == RI_PROX_HAAR || kind == RI_PROX_CNN || kind == RI_PROX_SARA, "unknown denoiser kind");
        if (kind == RI_PROX_SARA) {
            require(c->N % 16 == 0, "the SARA dictionary needs N divisible by 16");
            require(std::isfinite(param) && param >= 0.0, "threshold must be finite and >= 0");
            require(z != out, "z and out may not alias for the SARA prox");
            if (!c->sara.ready) sara_setup(c, 0, st(s));
            if (c->d.precision == 32) sara_prox<float>(c, (const float *)z, (float)param, (float *)out, st(s));
            else sara_prox<double>(c, (const double *)z, param, (double *)out, st(s));
        } else if (kind == RI_PROX_HAAR) {
            require(c->N % 16 == 0, "the Haar prox needs N divisible by 16");
            require(std::isfinite(param) && param >= 0.0, "threshold must be finite and >= 0");
            if (c->d.precision == 32)
                haar_prox<float>(c, nullptr, nullptr, 0.f, (const float *)z, (float)param, (float *)out, nullptr, st(s));
            else
                haar_prox<double>(c, nullptr, nullptr, 0.0, (const double *)z, param, (double *)out, nullptr, st(s));
        } else {
            require(c->cnn != nullptr, "no CNN denoiser loaded (ri_load_denoiser)");
            require(z != out, "z and out may not alias for the CNN denoiser");
            if (c->d.precision == 32)
                cnn_denoise<float>(c->cnn, (const float *)z, (float *)out, c->N, c->d.facet_core, c->d.facet_halo, st(s));
            else
                cnn_denoise<double>(c->cnn, (const double *)z, (double *)out, c->N, c->d.facet_core, c->d.facet_halo,
                                    st(s));
        }
        RI_CHECK_HIP(hipGetLastError());
    });
}

ri_status fb_step(ri_ctx *c, const void *x_in, const void *y, double gamma, int32_t kind, double param, void *x_out,
                  double *norms, ri_stream s) {
    if (!c) return RI_EINVAL;
    return guard(c, [&] {
        require(x_in && x_out && x_in != x_out, "x_in, x_out must be distinct non-NULL buffers");
        require(std::isfinite(gamma) && gamma > 0.0, "gamma must be finite and > 0");
        require(kind == RI_PROX_HAAR || kind == RI_PROX_CNN || kind == RI_PROX_SARA, "unknown denoiser kind");
        require(c->N % 16 == 0, "the denoisers need N divisible by 16");
        if (c->d.precision == 32)
            do_fb_step<float>(c, (const float *)x_in, y, gamma, kind, param, (float *)x_out, norms, st(s));
        else
            do_fb_step<double>(c, (const double *)x_in, y, gamma, kind, param, (double *)x_out, norms, st(s));
        RI_CHECK_HIP(hipGetLastError());
    });
}

ri_status ri_load_denoiser(ri_ctx *c, const float *params, int64_t n_params, int32_t layers, ri_stream s) {
    if (!c) return RI_EINVAL;
    return guard(c, [&] {
        require(params != nullptr, "params is NULL");
        require(layers >= 3 && layers <= 64, "layers must be in 3..64");
        require(n_params == cnn_param_count_for(layers), "n_params does not match the 64-channel layout");
        require(c->N % 16 == 0, "the CNN denoiser needs N divisible by 16");
        const bool whole = c->d.facet_core <= 0 || c->d.facet_core >= c->N;
        const int core = whole ? c->N : c->d.facet_core;
        const int nfx = (c->N + core - 1) / core;
        const int side = cnn_tile_side(c->N, c->d.facet_core, c->d.facet_halo);
        if (c->cnn && cnn_layers(c->cnn) != layers) {
            cnn_destroy(c->cnn);
            c->cnn = nullptr;
        }
        if (!c->cnn) c->cnn = cnn_create_inference(layers, nfx * nfx, side);
        cnn_load_params(c->cnn, params, st(s));
    });
}

ri_status pnp_solve(ri_ctx *c, const void *y, const ri_solve_opts *o, void *x_out, ri_solve_report *rep) {
    if (!c) return RI_EINVAL;
    bool fell = false;
    ri_status r = guard(c, [&] {
        require(o && x_out, "opts or x_out is NULL");
        require(o->max_iter >= 0 && o->check_every >= 1 && o->tau >= 0.0, "bad solve options");
        require(o->prox_kind == RI_PROX_HAAR || o->prox_kind == RI_PROX_CNN || o->prox_kind == RI_PROX_SARA,
                "unknown denoiser kind");
        require(o->reweight_every >= 0, "reweight_every must be >= 0");
        require(c->N % 16 == 0, "the Haar prox needs N divisible by 16");
        if (c->d.precision == 32) fell = solve<float>(c, y, *o, (float *)x_out, rep);
        else fell = solve<double>(c, y, *o, (double *)x_out, rep);
    });
    if (r == RI_OK && fell) return RI_FELLBACK;
    return r;
}

ri_status ri_profile(ri_ctx *c, int32_t enable) {
    if (!c) return RI_EINVAL;
    return guard(c, [&] {
        if (enable) {
            for (auto &e : c->prof_ev) { c->prof_pool.push_back(e.a); c->prof_pool.push_back(e.b); }
            c->prof_ev.clear();
        }
        c->prof_on = enable != 0;
    });
}

ri_status ri_profile_read(ri_ctx *c, ri_kernel_times *o) {
    if (!c || !o) return RI_EINVAL;
    return guard(c, [&] {
        *o = ri_kernel_times{};
        if (!c->prof_ev.empty()) RI_CHECK_HIP(hipEventSynchronize(c->prof_ev.back().b));
        for (auto &e : c->prof_ev) {
            float ms = 0.f;
            RI_CHECK_HIP(hipEventElapsedTime(&ms, e.a, e.b));
            switch (e.cat) {
                case PROF_TILES: o->tiles_ms += ms; o->n_tiles++; break;
                case PROF_FFT: o->fft_ms += ms; o->n_fft++; break;
                case PROF_PROX: o->prox_ms += ms; o->n_prox++; break;
                default: o->other_ms += ms; o->n_other++; break;
            }
        }
    });
}

ri_status ri_get_plan_stats(const ri_ctx *c, ri_plan_stats *o) {
    if (!c || !o) return RI_EINVAL;
    o->M = c->M;
    int64_t nnz = 0;
    for (int64_t m = 0; m < c->M; ++m) {
        const int S = 2 * c->plane_h[c->plane[m]] + c->J;
        nnz += (int64_t)S * S;
    }
    o->nnz = nnz;
    o->N = c->N;
    o->Np = c->Np;
    o->tile = c->view.tile;
    o->n_tiles = (c->Np / c->view.tile) * (c->Np / c->view.tile);
    o->n_items = c->view.n_items;
    o->n_blocks = (int32_t)c->block_offsets.size() - 1;
    o->max_item_vis = c->view.max_item_vis;
    o->device_bytes = c->device_bytes;
    o->plan_ms = c->plan_ms;
    o->n_tuned = 0;
    for (auto &t : c->tune_ms) {
        if (o->n_tuned >= 4) break;
        o->tuned_tile[o->n_tuned] = t.first;
        o->tuned_ms[o->n_tuned] = t.second;
        o->n_tuned++;
    }
    return RI_OK;
}

ri_status ri_sara_setup(ri_ctx *c, int32_t sub_iters, ri_stream s) {
    if (!c) return RI_EINVAL;
    return guard(c, [&] {
        require(sub_iters >= 1 && sub_iters <= 100000, "sub_iters must be in 1..100000");
        sara_setup(c, sub_iters, st(s));
        RI_CHECK_HIP(hipGetLastError());
    });
}

ri_status ri_sara_reweight(ri_ctx *c, const void *x, double rho, ri_stream s) {
    if (!c) return RI_EINVAL;
    return guard(c, [&] {
        require(x != nullptr, "x is NULL");
        require(std::isfinite(rho) && rho > 0.0, "rho must be finite and > 0");
        if (!c->sara.ready) sara_setup(c, 0, st(s));
        if (c->d.precision == 32) sara_reweight<float>(c, (const float *)x, (float)rho, st(s));
        else sara_reweight<double>(c, (const double *)x, rho, st(s));
        RI_CHECK_HIP(hipGetLastError());
    });
}

ri_status ri_sara_analysis(ri_ctx *c, const void *x, void *coef, ri_stream s) {
    if (!c) return RI_EINVAL;
    return guard(c, [&] {
        require(x && coef, "x or coef is NULL");
        if (!c->sara.ready) sara_setup(c, 0, st(s));
        if (c->d.precision == 32) sara_analysis<float>(c, (const float *)x, (float *)coef, st(s));
        else sara_analysis<double>(c, (const double *)x, (double *)coef, st(s));
        RI_CHECK_HIP(hipGetLastError());
    });
}

ri_status ri_sara_synthesis(ri_ctx *c, const void *coef, void *x, ri_stream s) {
    if (!c) return RI_EINVAL;
    return guard(c, [&] {
        require(x && coef, "x or coef is NULL");
        if (!c->sara.ready) sara_setup(c, 0, st(s));
        if (c->d.precision == 32) sara_synthesis<float>(c, (const float *)coef, (float *)x, st(s));
        else sara_synthesis<double>(c, (const double *)coef, (double *)x, st(s));
        RI_CHECK_HIP(hipGetLastError());
    });
}

ri_status ri_sara_get_state(ri_ctx *c, void *v, void *w, ri_stream s) {
    if (!c) return RI_EINVAL;
    return guard(c, [&] {
        require(c->sara.ready, "no SARA state: call ri_sara_setup or use the SARA prox first");
        const size_t bytes = (c->d.precision == 64 ? 8 : 4) * 9 * (size_t)c->N * c->N;
        if (v) RI_CHECK_HIP(hipMemcpyAsync(v, c->sara.v, bytes, hipMemcpyDeviceToDevice, st(s)));
        if (w) RI_CHECK_HIP(hipMemcpyAsync(w, c->sara.w, bytes, hipMemcpyDeviceToDevice, st(s)));
    });
}

ri_status ri_holo_build(ri_ctx *c, ri_stream s) {
    if (!c) return RI_EINVAL;
    return guard(c, [&] {
        if (c->P > 1) throw Error(RI_EUNSUPPORTED, "holographic matrices with w-stacking are not implemented");
        holo_build(c, view_fp64(c), st(s));
    });
}

ri_status ri_holo_release(ri_ctx *c) {
    if (!c) return RI_EINVAL;
    return guard(c, [&] {
        RI_CHECK_HIP(hipDeviceSynchronize());
        holo_free(c);
    });
}

ri_status ri_holo_apply(ri_ctx *c, const void *X, void *Y, ri_stream s) {
    if (!c) return RI_EINVAL;
    return guard(c, [&] {
        require(X && Y, "X or Y is NULL");
        require(X != Y, "X and Y may not alias");
        require(c->holo.ready, "no holographic matrix: call ri_holo_build first");
        if (c->d.precision == 32) holo_apply<float>(c, (const cx<float> *)X, (cx<float> *)Y, st(s));
        else holo_apply<double>(c, (const cx<double> *)X, (cx<double> *)Y, st(s));
    });
}

ri_status ri_holo_normal(ri_ctx *c, const void *x, void *out, ri_stream s) {
    if (!c) return RI_EINVAL;
    return guard(c, [&] {
        require(x && out, "x or out is NULL");
        require(c->holo.ready, "no holographic matrix: call ri_holo_build first");
        if (c->d.precision == 32) holo_normal<float>(c, c->p32, (const float *)x, (float *)out, st(s));
        else holo_normal<double>(c, c->p64, (const double *)x, (double *)out, st(s));
    });
}

ri_status ri_holo_get_stats(const ri_ctx *c, ri_holo_stats *o) {
    if (!c || !o) return RI_EINVAL;
    const Holo &h = c->holo;
    o->tiles = h.n_slots;
    o->entries = h.entries;
    o->bytes = h.entries * (c->d.precision == 64 ? 16 : 8);
    o->pairs = h.pairs;
    o->max_reach = h.max_R;
    o->build_ms = h.build_ms;
    return RI_OK;
}

ri_status ri_get_plan_arrays(const ri_ctx *c, int32_t *cell_u, int32_t *cell_v, int32_t *plane, int32_t *plane_h) {
    if (!c) return RI_EINVAL;
    if (cell_u) std::memcpy(cell_u, c->cu.data(), sizeof(int32_t) * c->M);
    if (cell_v) std::memcpy(cell_v, c->cv.data(), sizeof(int32_t) * c->M);
    if (plane) std::memcpy(plane, c->plane.data(), sizeof(int32_t) * c->M);
    if (plane_h) std::memcpy(plane_h, c->plane_h.data(), sizeof(int32_t) * c->plane_h.size());
    return RI_OK;
}

}  // extern "C"
