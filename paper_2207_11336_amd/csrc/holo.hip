// Holographic form of Phi^dagger Phi (appendix E): with H = sum_p G_p^H G_p,
// Phi^dagger Phi = Z^dagger F^dagger H F Z, so one application costs an FFT
// pair and one banded product Y = H X on the fine grid, independent of the
// number of visibilities once H is built.
//
// Storage (struct Holo): the upper half of H's band per touched 32 x 32 tile,
// one contiguous 1024-cell plane per offset d = (dy, dx). The product runs one
// 1024-thread workgroup per stored tile, one thread per cell k: for each
// stored offset it reads H[k][k + d] once (coalesced, the only HBM stream),
// adds H[k][k + d] X[k + d] to its own sum and conj(H[k][k + d]) X[k] to
// Y[k + d] (the lower half). X and Y live in LDS over the tile's reach
// (rows ty0 .. ty0 + 31 + R, columns tx0 - R .. tx0 + 31 + R); Y accumulates in
// FP64 by LDS atomics and is flushed to the global grid by device atomics.
#include <algorithm>
#include <chrono>

#include "ri_internal.h"

namespace ri {

namespace {

template <typename T>
__device__ __forceinline__ void lds_add(T *p, T v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ void global_add(T *p, T v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int CHUNK = 8;   // offsets whose H loads are issued together

template <typename T>
__global__ void __launch_bounds__(1024) k_holo_apply(const cx<T> *__restrict__ H, const int64_t *__restrict__ off,
                                                     const int4 *__restrict__ tinfo, const cx<T> *__restrict__ X,
                                                     cx<T> *__restrict__ Y, int logNp) {
    extern __shared__ unsigned char smem_raw[];
    const int4 ti = tinfo[blockIdx.x];
    const int ty0 = ti.x, tx0 = ti.y, R = ti.z;
    const int RW = HOLO_T + 2 * R, RH = HOLO_T + R, RN = RW * RH;
    double *Yr = reinterpret_cast<double *>(smem_raw);
    double *Yi = Yr + RN;
    cx<T> *Xs = reinterpret_cast<cx<T> *>(Yi + RN);
    const int tid = threadIdx.x;
    const int Npm = (1 << logNp) - 1;
    for (int e = tid; e < RN; e += blockDim.x) {
        const int r = e / RW, cc = e - r * RW;
        Xs[e] = X[((size_t)((ty0 + r) & Npm) << logNp) + ((tx0 - R + cc) & Npm)];
        Yr[e] = 0.0;
        Yi[e] = 0.0;
    }
    __syncthreads();
    const int home = (tid >> 5) * RW + (tid & 31) + R;
    const cx<T> xk = Xs[home];
    cx<T> acc = mk<T>((T)0, (T)0);
    const cx<T> *hp = H + off[blockIdx.x] + tid;
    const int DW = 2 * R + 1;
    for (int dy = 0; dy <= R; ++dy) {
        const int dx0 = dy == 0 ? 0 : -R;
        const cx<T> *hrow = hp + ((size_t)(dy * DW + R) << 10);
        const int qrow = home + dy * RW;
        for (int dx = dx0; dx <= R; dx += CHUNK) {
            cx<T> hv[CHUNK];
#pragma unroll
            for (int j = 0; j < CHUNK; ++j)
                if (dx + j <= R) hv[j] = hrow[(ptrdiff_t)(dx + j) * 1024];
#pragma unroll
            for (int j = 0; j < CHUNK; ++j) {
                if (dx + j > R) break;
                const int q = qrow + dx + j;
                acc = acc + hv[j] * Xs[q];
                if (dy != 0 || dx + j != 0) {
                    const cx<T> v = mulc(xk, hv[j]);
                    lds_add(&Yr[q], (double)v.x);
                    lds_add(&Yi[q], (double)v.y);
                }
            }
        }
    }
    lds_add(&Yr[home], (double)acc.x);
    lds_add(&Yi[home], (double)acc.y);
    __syncthreads();
    for (int e = tid; e < RN; e += blockDim.x) {
        const double vr = Yr[e], vi = Yi[e];
        if (vr != 0.0 || vi != 0.0) {
            const int r = e / RW, cc = e - r * RW;
            cx<T> *dst = Y + ((size_t)((ty0 + r) & Npm) << logNp) + ((tx0 - R + cc) & Npm);
            global_add(&dst->x, (T)vr);
            global_add(&dst->y, (T)vi);
        }
    }
}

// ||Phi x - y||^2 = <x, Re Phi^dagger Phi x> - 2 <x, Re Phi^dagger y> + ||y||^2 from device scalars.
__global__ void k_holo_r2(double *out, const double *dots, const double *yy) {
    out[0] = dots[0] - 2.0 * dots[1] + yy[0];
}

template <typename T>
size_t apply_lds(int R) {
    const size_t RN = (size_t)(HOLO_T + 2 * R) * (HOLO_T + R);
    return RN * (2 * sizeof(double) + sizeof(cx<T>));
}

}  // namespace

void holo_free(ri_ctx *c) {
    Holo &h = c->holo;
    dev_free(c, h.tmap);
    dev_free(c, h.tinfo);
    dev_free(c, h.off);
    dev_free(c, h.val);
    h = Holo{};
}

// Tile reach from the plan (every window cell lies in a tile marked here, with
// R >= its window side - 1), slot layout, then the accumulation of G^H G.
void holo_build(ri_ctx *c, const View &v64, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    holo_free(c);
    Holo &h = c->holo;
    const int Np = c->Np, Npm = Np - 1, ntx = Np / HOLO_T;
    std::vector<int32_t> reach((size_t)ntx * ntx, -1);
    int64_t pairs = 0;
    for (int64_t m = 0; m < c->M; ++m) {
        const int hw = c->plane_h[c->plane[m]];
        const int S = 2 * hw + c->J;
        pairs += (int64_t)S * S * ((int64_t)S * S + 1) / 2;   // upper half of the S^2 x S^2 pairs
        const int ty[2] = {((c->cv[m] - hw - 3) & Npm) / HOLO_T, ((c->cv[m] + hw + 3) & Npm) / HOLO_T};
        const int tx[2] = {((c->cu[m] - hw - 3) & Npm) / HOLO_T, ((c->cu[m] + hw + 3) & Npm) / HOLO_T};
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                int32_t &r = reach[(size_t)ty[i] * ntx + tx[j]];
                r = std::max(r, S - 1);
            }
    }
    std::vector<int32_t> tmap((size_t)ntx * ntx, -1);
    std::vector<int4> tinfo;
    std::vector<int64_t> off;
    int64_t entries = 0;
    for (int t = 0; t < ntx * ntx; ++t) {
        const int R = reach[t];
        if (R < 0) continue;
        tmap[t] = (int32_t)tinfo.size();
        tinfo.push_back(make_int4((t / ntx) * HOLO_T, (t % ntx) * HOLO_T, R, 0));
        off.push_back(entries);
        entries += (int64_t)(R + 1) * (2 * R + 1) * HOLO_T * HOLO_T;
        h.max_R = std::max(h.max_R, R);
    }
    const size_t eb = c->d.precision == 64 ? sizeof(cx<double>) : sizeof(cx<float>);
    if (!tinfo.empty()) {
        const size_t need = c->d.precision == 64 ? apply_lds<double>(h.max_R) : apply_lds<float>(h.max_R);
        if (need > (size_t)c->dev.lds_per_block)
            throw Error(RI_EUNSUPPORTED, "holographic tile reach " + std::to_string(h.max_R) + " needs " +
                                             std::to_string(need) + " B of LDS per workgroup");
    }
    h.n_slots = (int)tinfo.size();
    h.entries = entries;
    h.pairs = pairs;
    h.tmap = (int32_t *)dev_alloc(c, sizeof(int32_t) * tmap.size());
    h.tinfo = (int4 *)dev_alloc(c, sizeof(int4) * std::max<size_t>(1, tinfo.size()));
    h.off = (int64_t *)dev_alloc(c, sizeof(int64_t) * std::max<size_t>(1, off.size()));
    h.val = dev_alloc(c, eb * (size_t)std::max<int64_t>(1, entries));
    RI_CHECK_HIP(hipMemcpyAsync(h.tmap, tmap.data(), sizeof(int32_t) * tmap.size(), hipMemcpyHostToDevice, s));
    if (!tinfo.empty()) {
        RI_CHECK_HIP(hipMemcpyAsync(h.tinfo, tinfo.data(), sizeof(int4) * tinfo.size(), hipMemcpyHostToDevice, s));
        RI_CHECK_HIP(hipMemcpyAsync(h.off, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice, s));
    }
    if (c->d.precision == 64) {
        fill_zero<double>((cx<double> *)h.val, entries, s);
        fill_holo<double>(c, v64, s);
    } else {
        fill_zero<float>((cx<float> *)h.val, entries, s);
        fill_holo<float>(c, v64, s);
    }
    RI_CHECK_HIP(hipStreamSynchronize(s));
    h.ready = true;
    h.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

template <typename T>
void holo_apply(ri_ctx *c, const cx<T> *X, cx<T> *Y, hipStream_t s) {
    const Holo &h = c->holo;
    fill_zero<T>(Y, (int64_t)c->Np * c->Np, s);
    if (h.n_slots == 0) return;
    ProfScope prof(c, PROF_TILES, s);
    hipLaunchKernelGGL(k_holo_apply<T>, dim3(h.n_slots), dim3(1024), apply_lds<T>(h.max_R), s, (const cx<T> *)h.val,
                       h.off, h.tinfo, X, Y, c->logNp);
    RI_CHECK_HIP(hipGetLastError());
}

template <typename T>
void holo_normal(ri_ctx *c, Prec<T> &p, const T *x, T *out, hipStream_t s) {
    fwd_zpad_fft<T>(c, p, x, s);
    holo_apply<T>(c, p.gridB, p.gridA, s);
    adj_fft_crop<T>(c, p, out, s);
}

void holo_residual(double *out, const double *dots, const double *yy, hipStream_t s) {
    hipLaunchKernelGGL(k_holo_r2, dim3(1), dim3(1), 0, s, out, dots, yy);
}

template void holo_normal<float>(ri_ctx *, Prec<float> &, const float *, float *, hipStream_t);
template void holo_normal<double>(ri_ctx *, Prec<double> &, const double *, double *, hipStream_t);
template void holo_apply<float>(ri_ctx *, const cx<float> *, cx<float> *, hipStream_t);
template void holo_apply<double>(ri_ctx *, const cx<double> *, cx<double> *, hipStream_t);

}  // namespace ri
