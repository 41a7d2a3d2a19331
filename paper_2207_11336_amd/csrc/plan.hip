// Plan construction for one context: per-visibility grid cells, w-planes,
// w-kernel tables, the tile sort into work items, and the device tables.
//
// Everything here runs once per context (the paper builds its sparse
// operator blocks "only once" at initialisation, appendix E). The integer
// decisions (window centre, w-plane, support) are taken in FP64 with
// contraction disabled so that they are reproducible bit for bit.
#pragma clang fp contract(off)

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <numeric>
#include <thread>

#include "ri_internal.h"

namespace ri {

void *dev_alloc(ri_ctx *c, size_t bytes) {
    if (bytes == 0) bytes = 16;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(RI_ENOMEM, "hipMalloc(" + std::to_string(bytes) + " B) failed: " + hipGetErrorString(e));
    }
    c->device_bytes += (int64_t)bytes;
    c->allocs.emplace_back(p, bytes);
    return p;
}

void dev_free(ri_ctx *c, void *p) {
    if (!p) return;
    for (size_t i = 0; i < c->allocs.size(); ++i)
        if (c->allocs[i].first == p) {
            c->device_bytes -= (int64_t)c->allocs[i].second;
            c->allocs[i] = c->allocs.back();
            c->allocs.pop_back();
            break;
        }
    (void)hipFree(p);
}

static hipEvent_t take_event(ri_ctx *c) {
    if (!c->prof_pool.empty()) {
        hipEvent_t e = c->prof_pool.back();
        c->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    RI_CHECK_HIP(hipEventCreate(&e));
    return e;
}

ProfScope::ProfScope(ri_ctx *c_, int cat_, hipStream_t s_) : c(c_), cat(cat_), s(s_) {
    if (!c->prof_on) return;
    a = take_event(c);
    RI_CHECK_HIP(hipEventRecord(a, s));
}

ProfScope::~ProfScope() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (hipEventRecord(b, s) == hipSuccess) c->prof_ev.push_back(ProfEvent{cat, a, b});
}

template <typename V>
static V *upload(ri_ctx *c, const V *host, size_t n) {
    V *d = (V *)dev_alloc(c, n * sizeof(V));
    RI_CHECK_HIP(hipMemcpy(d, host, n * sizeof(V), hipMemcpyHostToDevice));
    return d;
}

// Modified Bessel I0 by its defining power series (FP64).
static double bessel_i0(double x) {
    double q = 0.25 * x * x, t = 1.0, s = 1.0;
    for (int k = 1; k < 500; ++k) {
        t = t * q / ((double)k * k);
        s += t;
        if (t < 1e-17 * s) break;
    }
    return s;
}

// kappa_hat(nu) / (J / I0(beta)): sinh(a)/a, a^2 = beta^2 - (pi J nu)^2.
static double kb_transform(double nu, int J, double beta) {
    double z = M_PI * J * nu, a2 = beta * beta - z * z;
    double r = a2 > 0 ? std::sinh(std::sqrt(a2)) / std::sqrt(a2)
                      : (a2 < 0 ? std::sin(std::sqrt(-a2)) / std::sqrt(-a2) : 1.0);
    return J * r / bessel_i0(beta);
}

// ---------------------------------------------------------------------------
// w-kernel taps by least squares: find k[q], |q| <= h, minimising
//   sum_{n=-N/2}^{N/2-1} | exp(i pi w (n delta)^2) - sum_q k[q] e^{2 pi i q n / N'} |^2.
// The design matrix depends only on h, so it is factorised once per h by
// modified Gram-Schmidt applied twice (Q R with Q orthonormal columns).
// ---------------------------------------------------------------------------
namespace {
using zc = std::complex<double>;
struct QR {
    int K = 0, N = 0;
    std::vector<zc> Q;   // [K][N] columns
    std::vector<zc> R;   // [K][K] upper triangular
};

QR factor(int h, int N, int Np) {
    QR f;
    f.K = 2 * h + 1;
    f.N = N;
    f.Q.resize((size_t)f.K * N);
    f.R.assign((size_t)f.K * f.K, zc(0, 0));
    for (int j = 0; j < f.K; ++j) {
        int q = j - h;
        zc *col = &f.Q[(size_t)j * N];
        for (int i = 0; i < N; ++i) {
            double n = (double)(i - N / 2);
            double ph = 2.0 * M_PI * (double)q * n / (double)Np;
            col[i] = zc(std::cos(ph), std::sin(ph));
        }
        for (int pass = 0; pass < 2; ++pass) {
            for (int k = 0; k < j; ++k) {
                const zc *qk = &f.Q[(size_t)k * N];
                zc d(0, 0);
                for (int i = 0; i < N; ++i) d += std::conj(qk[i]) * col[i];
                for (int i = 0; i < N; ++i) col[i] -= d * qk[i];
                f.R[(size_t)k * f.K + j] += d;
            }
        }
        double nr = 0;
        for (int i = 0; i < N; ++i) nr += std::norm(col[i]);
        nr = std::sqrt(nr);
        for (int i = 0; i < N; ++i) col[i] /= nr;
        f.R[(size_t)j * f.K + j] = nr;
    }
    return f;
}

void solve_taps(const QR &f, double w, double cell, zc *out) {
    const int K = f.K, N = f.N;
    std::vector<zc> b(K, zc(0, 0));
    std::vector<zc> c(N);
    for (int i = 0; i < N; ++i) {
        double n = (double)(i - N / 2) * cell;
        double ph = M_PI * w * n * n;
        c[i] = zc(std::cos(ph), std::sin(ph));
    }
    for (int k = 0; k < K; ++k) {
        const zc *qk = &f.Q[(size_t)k * N];
        zc d(0, 0);
        for (int i = 0; i < N; ++i) d += std::conj(qk[i]) * c[i];
        b[k] = d;
    }
    for (int k = K - 1; k >= 0; --k) {      // back substitution R x = b
        zc s = b[k];
        for (int j = k + 1; j < K; ++j) s -= f.R[(size_t)k * K + j] * out[j];
        out[k] = s / f.R[(size_t)k * K + k];
    }
}

template <typename F>
void parallel_for(int64_t n, F fn) {
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 4096 || nt == 1) { fn(0, n); return; }
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t) {
        int64_t a = n * t / nt, b = n * (t + 1) / nt;
        th.emplace_back([=, &fn] { fn(a, b); });
    }
    for (auto &x : th) x.join();
}
}  // namespace

// ---------------------------------------------------------------------------
// Per-visibility quantities (caller order) and the w-plane tables.
// ---------------------------------------------------------------------------
void build_plan(ri_ctx *c, const double *uvw) {
    const ri_plan_desc &d = c->d;
    const int64_t M = c->M;
    const int P = d.n_wplanes, P_half = (P - 1) / 2;
    // w-stacks (appendix E hybrid): NS stacks of width 2W/NS; the plane table
    // then covers the residual w - w_s in [-W/NS, W/NS]
    const int NS = c->P;
    const double Wfull = d.w_max;
    const double W = NS > 1 ? Wfull / NS : Wfull;
    const double scale = (double)c->Np / (2.0 * M_PI);
    c->stack_w.assign(NS, 0.0);
    if (NS > 1)
        for (int k = 0; k < NS; ++k) c->stack_w[k] = -Wfull + (2.0 * k + 1.0) * Wfull / NS;

    c->pu.resize(M); c->pv.resize(M); c->cu.resize(M); c->cv.resize(M); c->plane.resize(M);
    c->stack.assign(M, 0);
    std::vector<int> bad(1, 0);
    parallel_for(M, [&](int64_t a, int64_t b) {
        for (int64_t m = a; m < b; ++m) {
            double ou = uvw[3 * m], ov = uvw[3 * m + 1], w = uvw[3 * m + 2];
            if (!std::isfinite(ou) || !std::isfinite(ov) || !std::isfinite(w) ||
                std::fabs(ou) >= M_PI || std::fabs(ov) >= M_PI) { bad[0] = 1; continue; }
            double pu = ou * scale, pv = ov * scale;
            double fu = std::floor(pu + 0.5), fv = std::floor(pv + 0.5);
            c->pu[m] = pu; c->pv[m] = pv;
            int64_t iu = (int64_t)fu, iv = (int64_t)fv;
            c->cu[m] = (int32_t)(((iu % c->Np) + c->Np) % c->Np);
            c->cv[m] = (int32_t)(((iv % c->Np) + c->Np) % c->Np);
            int j = 0;
            if (NS > 1) {
                double k = std::floor((w + Wfull) * NS / (2.0 * Wfull));
                const int st = (int)std::min(std::max(k, 0.0), (double)(NS - 1));
                c->stack[m] = st;
                w -= c->stack_w[st];
            }
            if (P_half > 0 && W != 0.0) {
                double dw = W / (double)P_half;
                double jj = std::floor(w / dw + 0.5);
                if (jj < -P_half) jj = -P_half;
                if (jj > P_half) jj = P_half;
                j = (int)jj + P_half;
            }
            c->plane[m] = j;
        }
    });
    if (bad[0]) throw Error(RI_EINVAL, "uvw holds a non-finite value or |omega| >= pi");

    // per-plane support and least-squares taps
    c->plane_h.assign(P, 0);
    const int K = 2 * c->hmax + 1;
    c->wtaps64.assign((size_t)P * K * 2, 0.0);
    std::vector<double> wj(P, 0.0);
    if (P_half > 0 && W != 0.0) {
        double dw = W / (double)P_half;
        for (int j = 0; j < P; ++j) wj[j] = (double)(j - P_half) * dw;
    }
    for (int j = 0; j < P; ++j) {
        if (wj[j] == 0.0) continue;
        double hex = std::fabs(wj[j]) * (double)d.oversample * (double)c->N * (double)c->N *
                     d.cell_rad * d.cell_rad * 0.5;
        c->plane_h[j] = std::min(c->hmax, (int)std::ceil(hex) + 1);
    }
    std::vector<char> used(P, 0);
    for (int64_t m = 0; m < M; ++m) used[c->plane[m]] = 1;
    std::vector<QR> fac(c->hmax + 1);
    std::vector<char> have(c->hmax + 1, 0);
    for (int j = 0; j < P; ++j)
        if (used[j]) have[c->plane_h[j]] = 1;
    for (int h = 0; h <= c->hmax; ++h)
        if (have[h]) fac[h] = factor(h, c->N, c->Np);
    parallel_for(P * 16, [&](int64_t a, int64_t b) {      // oversubscribe: planes are cheap
        for (int64_t jj = a; jj < b; ++jj) {
            if (jj % 16) continue;
            int j = (int)(jj / 16);
            if (!used[j]) continue;
            int h = c->plane_h[j];
            zc tap[16];
            if (wj[j] == 0.0) { for (int k = 0; k < 2 * h + 1; ++k) tap[k] = zc(k == h ? 1.0 : 0.0, 0.0); }
            else solve_taps(fac[h], wj[j], d.cell_rad, tap);
            for (int q = -h; q <= h; ++q) {
                size_t o = ((size_t)j * K + (q + c->hmax)) * 2;
                c->wtaps64[o] = tap[q + h].real();
                c->wtaps64[o + 1] = tap[q + h].imag();
            }
        }
    });
    c->d_plane_h = upload(c, c->plane_h.data(), (size_t)P);
}

// ---------------------------------------------------------------------------
// Tile sort: order visibilities by (block, uv tile, support, plane, index),
// cut each (block, tile) run into work items and sort the items by decreasing
// work so the persistent launch hands out the largest first.
// ---------------------------------------------------------------------------
void build_view(ri_ctx *c, View &v, int tile, int frac_bytes) {
    const int64_t M = c->M;
    const int Np = c->Np, nta = Np / tile;
    const int64_t ntiles = (int64_t)nta * nta;
    const int nb = (int)c->block_offsets.size() - 1;
    v.tile = tile;
    v.frac_bytes = frac_bytes;

    // Counting sort by (block, w-stack), then, inside each such segment, by uv
    // tile (the tile counters are reset only where a segment touched them, so
    // the work stays O(M + ntiles) however many blocks and stacks there are).
    const int NS = c->P;
    const int64_t nk1 = (int64_t)nb * NS;
    std::vector<int64_t> key1(M);
    std::vector<int64_t> c1(nk1 + 1, 0);
    for (int b = 0; b < nb; ++b)
        for (int64_t m = c->block_offsets[b]; m < c->block_offsets[b + 1]; ++m) {
            key1[m] = (int64_t)b * NS + c->stack[m];
            c1[key1[m] + 1]++;
        }
    for (int64_t i = 0; i < nk1; ++i) c1[i + 1] += c1[i];
    std::vector<int64_t> ord1(M);
    {
        std::vector<int64_t> pos(c1.begin(), c1.end() - 1);
        for (int64_t m = 0; m < M; ++m) ord1[pos[key1[m]]++] = m;   // stable
    }
    struct Bucket { int64_t k1, t, s, e; };
    std::vector<Bucket> buckets;
    std::vector<int64_t> order(M);
    std::vector<int64_t> ct(ntiles + 1, 0);
    for (int64_t k = 0; k < nk1; ++k) {
        const int64_t s0 = c1[k], e0 = c1[k + 1];
        if (s0 == e0) continue;
        auto tile_of = [&](int64_t m) { return (int64_t)(c->cv[m] / tile) * nta + c->cu[m] / tile; };
        for (int64_t i = s0; i < e0; ++i) ct[tile_of(ord1[i]) + 1]++;
        // prefix over the touched tiles only, in tile order
        std::vector<int64_t> touched;
        for (int64_t i = s0; i < e0; ++i) {
            const int64_t t = tile_of(ord1[i]);
            if (ct[t + 1] > 0) { touched.push_back(t); ct[t + 1] = -ct[t + 1]; }   // mark seen
        }
        std::sort(touched.begin(), touched.end());
        int64_t run = s0;
        std::vector<int64_t> start(touched.size());
        for (size_t q = 0; q < touched.size(); ++q) {
            const int64_t n = -ct[touched[q] + 1];
            start[q] = run;
            buckets.push_back({k, touched[q], run, run + n});
            ct[touched[q] + 1] = (int64_t)q;   // slot of this tile in `start`
            run += n;
        }
        for (int64_t i = s0; i < e0; ++i) {
            const int64_t m = ord1[i];
            order[start[ct[tile_of(m) + 1]]++] = m;   // stable within the tile
        }
        for (int64_t t : touched) ct[t + 1] = 0;
    }
    // inside each bucket: by (support, plane, caller index)
    parallel_for((int64_t)buckets.size(), [&](int64_t a, int64_t b) {
        for (int64_t k = a; k < b; ++k) {
            const int64_t s0 = buckets[k].s, e0 = buckets[k].e;
            if (e0 - s0 < 2) continue;
            std::sort(order.begin() + s0, order.begin() + e0, [&](int64_t x, int64_t y) {
                int hx = c->plane_h[c->plane[x]], hy = c->plane_h[c->plane[y]];
                if (hx != hy) return hx < hy;
                if (c->plane[x] != c->plane[y]) return c->plane[x] < c->plane[y];
                return x < y;
            });
        }
    });

    // work items (one bucket = one block, one stack, one uv tile; chunks of VMAX)
    const int64_t VMAX = c->d.item_vis > 0 ? c->d.item_vis : 2048;
    std::vector<TileItem> items;
    std::vector<int64_t> work;
    for (const Bucket &bk : buckets) {
        const int64_t s0 = bk.s, e0 = bk.e, t = bk.t;
        for (int64_t a = s0; a < e0; a += VMAX) {
            TileItem it;
            it.ty0 = (int32_t)(t / nta) * tile;
            it.tx0 = (int32_t)(t % nta) * tile;
            it.vb = (int32_t)a;
            it.vc = (int32_t)std::min(VMAX, e0 - a);
            int64_t wsum = 0;
            for (int64_t i = a; i < a + it.vc; ++i) {
                int S = 2 * c->plane_h[c->plane[order[i]]] + c->J;
                wsum += (int64_t)S * S;
            }
            items.push_back(it);
            work.push_back(wsum + 4 * (int64_t)(tile + 2 * c->H) * (tile + 2 * c->H));
        }
    }
    std::vector<int64_t> iord(items.size());
    std::iota(iord.begin(), iord.end(), 0);
    std::stable_sort(iord.begin(), iord.end(), [&](int64_t a, int64_t b) { return work[a] > work[b]; });
    std::vector<TileItem> sorted_items(items.size());
    v.max_item_vis = 0;
    for (size_t i = 0; i < items.size(); ++i) {
        sorted_items[i] = items[iord[i]];
        v.max_item_vis = std::max<int64_t>(v.max_item_vis, sorted_items[i].vc);
    }
    v.n_items = (int)sorted_items.size();

    // per-visibility arrays in internal order
    std::vector<int32_t> perm(M);
    std::vector<uint2> rec(M);
    std::vector<float> f32;
    std::vector<double> f64;
    if (frac_bytes == 4) f32.resize(2 * M); else f64.resize(2 * M);
    for (int64_t i = 0; i < M; ++i) {
        int64_t m = order[i];
        perm[i] = (int32_t)m;
        rec[i].x = ((uint32_t)c->cv[m] << 16) | (uint32_t)c->cu[m];
        rec[i].y = (uint32_t)c->plane[m] | ((uint32_t)c->plane_h[c->plane[m]] << 16) | ((uint32_t)c->stack[m] << 20);
        double fu = c->pu[m] - std::floor(c->pu[m] + 0.5);
        double fv = c->pv[m] - std::floor(c->pv[m] + 0.5);
        if (frac_bytes == 4) { f32[2 * i] = (float)fu; f32[2 * i + 1] = (float)fv; }
        else { f64[2 * i] = fu; f64[2 * i + 1] = fv; }
    }
    v.perm_host.assign(order.begin(), order.end());
    v.perm = upload(c, perm.data(), (size_t)M);
    v.rec = upload(c, rec.data(), (size_t)M);
    if (frac_bytes == 4) v.frac = upload(c, f32.data(), (size_t)(2 * M));
    else v.frac = upload(c, f64.data(), (size_t)(2 * M));
    v.items = upload(c, sorted_items.data(), sorted_items.size());
}

void free_view(ri_ctx *c, View &v) {
    dev_free(c, v.perm); dev_free(c, v.rec); dev_free(c, v.frac); dev_free(c, v.items);
    v = View();
}

// ---------------------------------------------------------------------------
// Tables and work buffers of one precision: 1/kappa_hat, twiddles, w-taps.
// ---------------------------------------------------------------------------
template <typename T>
void ensure_prec(ri_ctx *c, Prec<T> &p) {
    if (p.ready) return;
    const int N = c->N, Np = c->Np;
    std::vector<T> ic(N);
    for (int i = 0; i < N; ++i) ic[i] = (T)(1.0 / kb_transform((double)(i - N / 2) / Np, c->J, c->beta));
    p.icorr = upload(c, ic.data(), (size_t)N);
    std::vector<cx<T>> tw(Np);
    for (int k = 0; k < Np; ++k) {
        double a = -2.0 * M_PI * (double)k / (double)Np;
        tw[k] = mk<T>((T)std::cos(a), (T)std::sin(a));
    }
    p.tw = upload(c, tw.data(), (size_t)Np);
    const size_t nt = c->wtaps64.size() / 2;
    std::vector<cx<T>> wt(nt);
    for (size_t i = 0; i < nt; ++i) wt[i] = mk<T>((T)c->wtaps64[2 * i], (T)c->wtaps64[2 * i + 1]);
    p.wtaps = upload(c, wt.data(), nt);
    const size_t ng = (size_t)c->P * Np * Np;
    p.gridA = (cx<T> *)dev_alloc(c, sizeof(cx<T>) * ng);
    p.gridB = (cx<T> *)dev_alloc(c, sizeof(cx<T>) * ng);
    if (c->P > 1) {
        // phase screens c_s(n) = exp(-2 pi i w_s (sqrt(1 - l^2 - m^2) - 1)), FP64 arithmetic
        const double dl = c->d.cell_rad;
        std::vector<cx<T>> ch((size_t)c->P * N * N);
        parallel_for((int64_t)c->P * N, [&](int64_t a, int64_t b) {
            for (int64_t r = a; r < b; ++r) {
                const int st = (int)(r / N), iy = (int)(r % N);
                const double my = (iy - N / 2) * dl;
                for (int ix = 0; ix < N; ++ix) {
                    const double lx = (ix - N / 2) * dl;
                    const double ph = -2.0 * M_PI * c->stack_w[st] * (std::sqrt(1.0 - lx * lx - my * my) - 1.0);
                    ch[(size_t)r * N + ix] = mk<T>((T)std::cos(ph), (T)std::sin(ph));
                }
            }
        });
        p.chirp = upload(c, ch.data(), ch.size());
    }
    p.img0 = (T *)dev_alloc(c, sizeof(T) * (size_t)N * N);
    p.img1 = (T *)dev_alloc(c, sizeof(T) * (size_t)N * N);
    p.ydata = (cx<T> *)dev_alloc(c, sizeof(cx<T>) * (size_t)std::max<int64_t>(c->M, 1));
    p.ready = true;
}

template void ensure_prec<float>(ri_ctx *, Prec<float> &);
template void ensure_prec<double>(ri_ctx *, Prec<double> &);

}  // namespace ri
