// G (degridding), G^H (gridding) and the fused degrid -> residual -> grid pass
// of the data-fidelity gradient (paper eq. 1 and appendix A; the per-block sum
// of eq. E2 is a loop over work items of one persistent launch).
//
// Row m of G (appendix E: interpolation kernel convolved row-wise with a small
// w-kernel) is separable: G_{m,(ky,kx)} = g_v[ay] g_u[ax] on the window of side
// S = 7 + 2h around the centre cell c = floor(p + 1/2), with per axis
//   g[a] = sum_{|q| <= h} k_w[q] kappa(f - a + h + 3 - q),  f = p - c,
// kappa the Kaiser-Bessel kernel (J = 7) and k_w the w-plane taps.
//
// Work item = one uv tile (T x T cells) of one data block, or a chunk of it.
// A workgroup stages the item's input subgrid X (T + 2H)^2 in LDS, walks the
// item's visibilities (one 16-lane group per visibility), accumulates the
// output subgrid Y and flushes it to the global grid with float atomics.
// Workgroups pull items from a global counter (persistent launch), largest
// items first. With G stored (CSR) the taps are spread over the lanes in row
// order; on the fly, or with the axis factors stored, lane c of the group owns
// window column c, holds g_u[c] and g_v[c] in registers and receives each row
// weight by a DPP broadcast, so the weights never pass through LDS.
// Y accumulates either in FP64 LDS planes by atomic adds (scatter form) or,
// for separable rows in FP32, in registers: every wave holds the whole
// subgrid and gathers its visibilities' outer products (gather form: on the
// VALU for subgrids up to 24 a side, on the matrix cores up to 32).
//
// The same row weights fill the stored G (k_fill_csr) and the holographic
// matrix H = G^H G of appendix E (k_fill_holo; its storage and banded product
// are in holo.hip).
#include <numeric>

#include "ri_internal.h"

namespace ri {

namespace {

constexpr int GROUPS = 16;         // visibilities in flight per 256-thread workgroup
constexpr int MAXI = 19;           // ceil(17^2 / 16): tap slots per lane
constexpr int SCR_KB = 16;         // per-group KB scratch (two axes x 8), T
constexpr int SCR_W = 12;          // per-group w-taps (2 hmax + 1 <= 11), cx<T>
constexpr int SCR_G = 36;          // per-group axis weights (two axes x 18), cx<T>
constexpr int KB_TERMS_MAX = 32;
#ifndef TILES_GA_WAVES
#define TILES_GA_WAVES 5           // waves per SIMD the gather-form kernels are compiled for
#endif
#ifndef TILES_CSR_WAVES
#define TILES_CSR_WAVES 4          // waves per SIMD the FP32 stored-G kernels are compiled for
#endif
#ifndef TILES_MF_WAVES
#define TILES_MF_WAVES 4           // waves per SIMD the matrix-core gather kernels are compiled for
#endif
constexpr int GB_MF = 16;          // gridding-form code of the matrix-core gather (16 x 16 tiles)
typedef float f32x4 __attribute__((ext_vector_type(4)));


template <typename T>
struct TileArgs {
    const TileItem *items;
    int n_items;
    int *counter;
    int tile, H, W, logNp, hmax, kb_terms;
    T kbc[KB_TERMS_MAX];           // kappa(t) = sum_k kbc[k] z^k, z = 1 - (2t/7)^2
    const uint2 *rec;              // per visibility: (cell, plane | h << 16 | w-stack << 20)
    const T *frac;
    const cx<T> *wtaps;
    const int32_t *perm;
    const int64_t *rowptr;
    const cx<T> *gval;
    const cx<T> *X;
    cx<T> *Y;
    const cx<T> *ysorted;
    const cx<T> *yuser;
    cx<T> *yout;
    double *r2part;
    const cx<T> *sepw;             // stored axis factors (RI_G_SEP): per visibility 17 (g_u, g_v) pairs
};

// The stored axis factors of visibility m (internal order): lane c < 16 takes
// (g_u[c], g_v[c]), every lane the pair of index 16; zero past the window.
template <typename T>
__device__ __forceinline__ void sep_load(const cx<T> *sepw, int m, int lane, cx<T> &gu, cx<T> &gv, cx<T> &gu16,
                                         cx<T> &gv16) {
    const cx<T> *p = sepw + (size_t)m * 34;
    gu = p[2 * lane];
    gv = p[2 * lane + 1];
    gu16 = p[32];
    gv16 = p[33];
}

// Kaiser-Bessel weight kappa(t) = I0(beta sqrt(z)) / I0(beta) with
// z = 1 - (2t/7)^2: the I0 power series is a power series in z, evaluated by
// Horner with coefficients kbc[k] = (beta^2/4)^k / (k!)^2 / I0(beta) computed
// in FP64 (22 terms reach FP32 rounding, 32 FP64; no square root needed).
template <typename T>
__device__ __forceinline__ T kb_weight(T t, const TileArgs<T> &a) {
    const T u = t * (T)(2.0 / 7.0);
    const T z = (T)1 - u * u;
    if (z < (T)0) return (T)0;
    constexpr int K = sizeof(T) == 4 ? 22 : 32;
    T p = a.kbc[K - 1];
#pragma unroll
    for (int k = K - 2; k >= 0; --k) p = p * z + a.kbc[k];
    return p;
}

// kappa(t) for |t| <= 7/2 (the window's taps): no branch, z clamped at 0.
template <typename T>
__device__ __forceinline__ T kb_weight_in(T t, const TileArgs<T> &a) {
    const T u = t * (T)(2.0 / 7.0);
    const T z = fmax((T)1 - u * u, (T)0);
    constexpr int K = sizeof(T) == 4 ? 22 : 32;
    T p = a.kbc[K - 1];
#pragma unroll
    for (int k = K - 2; k >= 0; --k) p = p * z + a.kbc[k];
    return p;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over the 16 lanes of a DPP row (quad swaps, then rotations by 4 and 8).
// Every control used here reads a lane inside the row, so bound_ctrl never
// applies; with it set (and old = 0) the compiler folds the move into the
// consuming VALU instruction (v_add_f32_dpp).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f(double v) {
    int2 p = __builtin_bit_cast(int2, v);
    p.x = __builtin_amdgcn_mov_dpp(p.x, CTRL, 0xF, 0xF, false);
    p.y = __builtin_amdgcn_mov_dpp(p.y, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, p);
}
template <typename T>
__device__ __forceinline__ T sum16(T v) {
    v += dpp_f<0xB1>(v);     // quad_perm(1,0,3,2)
    v += dpp_f<0x4E>(v);     // quad_perm(2,3,0,1)
    v += dpp_f<0x124>(v);    // row_ror:4
    v += dpp_f<0x128>(v);    // row_ror:8
    return v;
}

// Lane N of the caller's 16-lane DPP row, broadcast to the whole row
// (row_newbcast, which gfx950 also performs on 64-bit operands: one
// v_mov_b64_dpp per complex float or double).
template <int N>
__device__ __forceinline__ float row_share(float v) { return dpp_f<0x150 + N>(v); }
template <int N>
__device__ __forceinline__ long long row_share64(long long v) {
    return __builtin_amdgcn_mov_dpp(v, 0x150 + N, 0xF, 0xF, false);
}
template <int N>
__device__ __forceinline__ double row_share(double v) {
    return __builtin_bit_cast(double, row_share64<N>(__builtin_bit_cast(long long, v)));
}
template <int N>
__device__ __forceinline__ cx<float> row_share(cx<float> v) {
    static_assert(sizeof(cx<float>) == 8, "complex float is two packed floats");
    return __builtin_bit_cast(cx<float>, row_share64<N>(__builtin_bit_cast(long long, v)));
}
template <int N>
__device__ __forceinline__ cx<double> row_share(cx<double> v) { return mk<double>(row_share<N>(v.x), row_share<N>(v.y)); }

// f(integral_constant<int, i>) for i = 0 .. N-1, unrolled at compile time.
template <typename F, int... I>
__device__ __forceinline__ void static_for_(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) { static_for_(f, std::make_integer_sequence<int, N>{}); }

// acc + a b with the four products as FMAs.
template <typename T>
__device__ __forceinline__ cx<T> cmac(cx<T> acc, cx<T> a, cx<T> b) {
    acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
    return acc;
}

template <typename T>
__device__ __forceinline__ void lds_add(T *p, T v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ void global_add(T *p, T v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Axis weights of one G row into gg[0..S) (u) and gg[18..18+S) (v) by the 16
// lanes of a group: KB taps into kbg, the plane's w-taps into wk, then
//   g[a] = sum_q k_w[q] kappa(f - (a - h - 3) - q).
template <typename T>
__device__ __forceinline__ void axis_weights(const TileArgs<T> &a, int m, int pl, int h, int S, int lane, T *kbg,
                                             cx<T> *wk, cx<T> *gg) {
    const T fu = a.frac[2 * (size_t)m], fv = a.frac[2 * (size_t)m + 1];
    if (lane < 7) kbg[lane] = kb_weight<T>(fu - (T)(lane - 3), a);
    else if (lane >= 8 && lane < 15) kbg[lane] = kb_weight<T>(fv - (T)(lane - 11), a);
    if (lane <= 2 * h) wk[lane] = a.wtaps[(size_t)pl * (2 * a.hmax + 1) + a.hmax - h + lane];
    wave_sync();
    for (int idx = lane; idx < 2 * S; idx += 16) {
        const int axis = idx < S ? 0 : 1;
        const int ax = idx - axis * S;
        const int ap = ax - h - 3;
        const int qlo = max(-h, -3 - ap), qhi = min(h, 3 - ap);
        cx<T> acc = mk<T>((T)0, (T)0);
        for (int q = qlo; q <= qhi; ++q) acc = acc + scale(wk[q + h], kbg[axis * 8 + ap + q + 3]);
        gg[axis * 18 + ax] = acc;
    }
    wave_sync();
}

// Minimum waves per SIMD the register allocation must allow: the FP32
// scatter-form variants with separable rows fit 64 VGPRs without spilling (8
// waves), the VALU gather form 96 (TILES_GA_WAVES), the matrix-core gather
// and the FP32 stored-G kernels 128 (TILES_MF_WAVES, TILES_CSR_WAVES); FP64 is
// left free (1).
template <typename T, int GM, int GB>
constexpr int tiles_min_waves() {
    return GB == GB_MF ? TILES_MF_WAVES
           : GB > 0    ? TILES_GA_WAVES
                       : (std::is_same<T, float>::value ? (GM != RI_G_CSR ? 8 : TILES_CSR_WAVES) : 1);
}

// LDS of the gather form: per group a slot with the padded vectors P and g_v
// of its current visibility (complex arrays of LEN entries; the window's 17
// entries start at PAD = W - 7, the rest reads zero), then the window origins.
__host__ __device__ constexpr int ga_pad(int W) { return W - 7; }
// subgrid side the lanes cover: 8 GB on the VALU, two 16-cell tiles on the matrix cores
__host__ __device__ constexpr int ga_cover(int GB) { return GB == GB_MF ? 32 : 8 * GB; }
__host__ __device__ constexpr int ga_len(int W, int GB) { return (W - 7 + ga_cover(GB) + 1) & ~1; }
__host__ __device__ constexpr int ga_slot_cx(int W, int GB) { return 2 * ga_len(W, GB); }

// GM: RI_G_CSR (stored rows), RI_G_OTF (weights computed), RI_G_SEP (stored axis factors).
// GB = 0: scatter-form gridding (FP64 LDS atomics into the output subgrid).
// GB = 3: gather-form gridding on the VALU (3 x 3 output cells per lane);
// GB = GB_MF: gather-form gridding on the matrix cores (see the comments at
// the gather).
template <typename T, int OP, int GM, int GB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(tiles_min_waves<T, GM, GB>())))
k_tiles(TileArgs<T> a) {
    constexpr bool OTF = GM == RI_G_OTF, SEP = GM == RI_G_SEP, GA = GB > 0, MF = GB == GB_MF;
    static_assert(!GA || ((OP & OP_GRID) && GM != RI_G_CSR), "gather form: gridding with separable rows only");
    static_assert(!MF || std::is_same<T, float>::value, "matrix-core gather: FP32 only");
    // All LDS is dynamic and starts at byte 0: a static __shared__ variable
    // would shift the dynamic block by its size and misalign the 8-byte
    // atomics on the subgrid. Layout: Xs (input subgrid, T), Yr and Yi (output
    // subgrid, FP64 real and imaginary planes), then per group the w-taps,
    // then reduction slots and the item slot (every part a multiple of 16
    // bytes). The scatter form accumulates in FP64 for both precisions: on
    // gfx950 an LDS FP64 atomic add costs ~8 cycles per wave against ~190 for
    // FP32.
    // The gather form keeps X's region also when only gridding (it holds a
    // partial subgrid at the item's end) and has slots instead of Yr, Yi.
    extern __shared__ unsigned char smem_raw[];
    const int W = a.W, WW = W * W;
    // row stride of the staged X: with stored axis factors in the gather form
    // the covered side, a compile-time constant, so the degrid's row offsets
    // are immediates (on the fly that costs the kernel a spilled register); W
    // otherwise. The gather form's X region holds W x (covered side) entries.
    constexpr int XSC = (GA && SEP) ? ga_cover(GB) : 0;
    const int XS = XSC ? XSC : W;
    const int PAD = ga_pad(W), LEN = ga_len(W, GB), SLOT = ga_slot_cx(W, GB);
    cx<T> *Xs = reinterpret_cast<cx<T> *>(smem_raw);
    double *Yr = reinterpret_cast<double *>(Xs + (GA ? W * ga_cover(GB) : (OP & OP_DEGRID) ? WW : 0));
    double *Yi = Yr + ((!GA && (OP & OP_GRID)) ? WW : 0);
    cx<T> *slot = reinterpret_cast<cx<T> *>(Yi + ((!GA && (OP & OP_GRID)) ? WW : 0));
    int *sorg = reinterpret_cast<int *>(slot + (GA ? GROUPS * SLOT : 0));
    cx<T> *wks = reinterpret_cast<cx<T> *>(sorg + (GA ? GROUPS : 0));
    double *s_red = reinterpret_cast<double *>(wks + GROUPS * SCR_W);
    int &s_item = *reinterpret_cast<int *>(s_red + 4);
    const int tid = threadIdx.x, lane = tid & 15, grp = tid >> 4;
    cx<T> *wk = wks + grp * SCR_W;
    const int Npm = (1 << a.logNp) - 1;
    double r2 = 0.0;

    for (;;) {
        if (tid == 0) s_item = atomicAdd(a.counter, 1);
        __syncthreads();
        const int it = s_item;
        if (it >= a.n_items) break;
        const TileItem item = a.items[it];
        const int y0 = item.ty0 - a.H, x0 = item.tx0 - a.H;
        // all of an item's visibilities belong to one w-stack, whose grids follow
        const size_t goff = (size_t)(a.rec[item.vb].y >> 20) << (2 * a.logNp);
        const cx<T> *Xg = a.X + goff;
        cx<T> *Yg = a.Y + goff;
        if (OP & OP_DEGRID) {
            for (int e = tid; e < WW; e += blockDim.x) {
                const int r = e / W, cc = e - r * W;
                Xs[r * XS + cc] = Xg[((size_t)((y0 + r) & Npm) << a.logNp) + ((x0 + cc) & Npm)];
            }
        }
        if (!GA && (OP & OP_GRID)) {
            for (int e = tid; e < WW; e += blockDim.x) { Yr[e] = 0.0; Yi[e] = 0.0; }
        }
        if (GA) {   // the slots' padding must read zero (the item's end reuses them)
            for (int e = tid; e < GROUPS * SLOT; e += blockDim.x) slot[e] = mk<T>((T)0, (T)0);
        }
        __syncthreads();
        constexpr int NB = (GA && !MF) ? GB : 1;
        cx<T> gacc[NB][NB];
        f32x4 mre[2][2], mim[2][2];   // matrix-core gather: real and imaginary parts per tile
        if constexpr (MF) {
            static_for<2>([&](auto I) { static_for<2>([&](auto J) {
                mre[I][J] = f32x4{0.f, 0.f, 0.f, 0.f};
                mim[I][J] = f32x4{0.f, 0.f, 0.f, 0.f};
            }); });
        } else if (GA) {
            static_for<NB>([&](auto I) { static_for<NB>([&](auto J) { gacc[I][J] = mk<T>((T)0, (T)0); }); });
        }

        // the group's next record (and on the fly its fraction: lane l < 8 the
        // u one, 8.. the v one) is loaded one visibility ahead, with its data
        // value (subtracted when fused, gridded when gridding); with G stored
        // the data value is issued with the row instead, which keeps that
        // kernel's registers within four waves
        auto ydata = [&](int mm) -> cx<T> {
            if (OP == OP_GRID) return a.yuser[a.perm[mm]];
            if (a.ysorted) return a.ysorted[mm];
            if (a.yuser) return a.yuser[a.perm[mm]];
            return mk<T>((T)0, (T)0);
        };
        uint2 rec_n = make_uint2(0u, 0u);
        T f_n = (T)0;
        cx<T> su_n = mk<T>((T)0, (T)0), sv_n = su_n, su16_n = su_n, sv16_n = su_n, y_n = su_n;
        if (grp < item.vc) {
            rec_n = a.rec[item.vb + grp];
            if ((OP & OP_GRID) && GM != RI_G_CSR) y_n = ydata(item.vb + grp);
            if (OTF) f_n = a.frac[2 * (size_t)(item.vb + grp) + (lane >> 3)];
            if (SEP) sep_load(a.sepw, item.vb + grp, lane, su_n, sv_n, su16_n, sv16_n);
        }
        // The gather form steps whole waves (visibility vb + g for group g of
        // the wave) so that each wave can gather its four visibilities together.
        for (int vb = GA ? (grp & ~3) : grp; vb < item.vc; vb += GROUPS) {
          const int vi = GA ? vb + (grp & 3) : vb;
          if (!GA || vi < item.vc) {
            const int m = item.vb + vi;
            const uint2 rec = rec_n;
            const cx<T> yv = y_n;
            const T f = f_n;
            const int cu = (int)(rec.x & 0xFFFFu), cv = (int)(rec.x >> 16);
            const int pl = (int)(rec.y & 0xFFFFu), h = (int)((rec.y >> 16) & 0xFu);
            const int S = 2 * h + 7, SS = S * S;
            const int base = (cv - item.ty0 + a.H - h - 3) * XS + (cu - item.tx0 + a.H - h - 3);
            const int NI = (SS + 15) >> 4;
            cx<T> acc = mk<T>((T)0, (T)0);
            cx<T> r;
            if (OTF || SEP) {
                cx<T> gu = mk<T>((T)0, (T)0), gv = gu, gu16 = gu, gv16 = gu;
                if (SEP) {
                    // stored factors, loaded one visibility ahead
                    gu = su_n;
                    gv = sv_n;
                    gu16 = su16_n;
                    gv16 = sv16_n;
                    // (the item's last visibility again at its end: no branch,
                    // so no register copies for the not-loaded case)
                    {
                        const int mn = item.vb + min(vi + GROUPS, item.vc - 1);
                        rec_n = a.rec[mn];
                        if (OP & OP_GRID) y_n = ydata(mn);
                        sep_load(a.sepw, mn, lane, su_n, sv_n, su16_n, sv16_n);
                    }
                } else {
                // G row from its separable axis weights, all in registers:
                // lanes 0..6 hold the u-axis KB weights kappa(f_u - (j - 3)),
                // lanes 8..14 the v-axis ones; lane c then forms
                //   g[c] = sum_j kappa[j] k_w[2h + j - c]    (both axes, c < S),
                // with kappa[j] broadcast over the row by DPP. The last index
                // of a 17-wide window (c = 16, only k_w[0] kappa[6]) is kept by
                // lane 0. Lane c owns window column c and walks the rows; the
                // row weight g_v[ay] is broadcast from lane ay. For S = 17,
                // column 16 is taken row-wise (lane l: row l) and the corner
                // (16, 16) by lane 0, which keeps the 16 lanes balanced.
                // the plane's w-taps first, then the next visibility's record and
                // fraction (loads complete in order, so waiting for the taps
                // leaves the prefetch in flight)
                if (lane <= 2 * h) wk[lane] = a.wtaps[(size_t)pl * (2 * a.hmax + 1) + a.hmax - h + lane];
                if (vi + GROUPS < item.vc) {
                    rec_n = a.rec[m + GROUPS];
                    if (OP & OP_GRID) y_n = ydata(m + GROUPS);
                    f_n = a.frac[2 * (size_t)(m + GROUPS) + (lane >> 3)];
                }
                // one Horner series for all 14 taps (lanes 7 and 15 compute an
                // unused value): lane j < 8 evaluates kappa(f_u - (j - 3)),
                // lane 8 + j kappa(f_v - (j - 3))
                const T kbr = (lane & 7) < 7 ? kb_weight_in<T>(f - (T)((lane & 7) - 3), a) : (T)0;
                wave_sync();
                static_for<7>([&](auto J) {
                    constexpr int j = decltype(J)::value;
                    const T ku = row_share<j>(kbr), kv = row_share<8 + j>(kbr);
                    const int k = 2 * h + j - lane;
                    if (k >= 0 && k <= 2 * h) {
                        const cx<T> w = wk[k];
                        gu = gu + scale(w, ku);
                        gv = gv + scale(w, kv);
                    }
                });
                if (S == 17) {
                    const cx<T> w0 = wk[0];
                    gu16 = scale(w0, row_share<6>(kbr));
                    gv16 = scale(w0, row_share<14>(kbr));
                }
                }
                const bool col = lane < S;
                if (OP & OP_DEGRID) {
                    // Lanes c >= S read a cell inside the window and add it with
                    // weight g_u[c] = 0. Rows 0..6 exist for every S; the rest
                    // come in pairs (S is odd), so loads issue two at a time.
                    const cx<T> *xp = Xs + base + min(lane, S - 1);
                    cx<T> accv = mk<T>((T)0, (T)0);
                    // rows 0..6 in two batches of loads (4, then 3), which
                    // keeps the gather-form kernel's registers within 96
                    {
                        cx<T> xv[4];
                        static_for<4>([&](auto J) { xv[J] = xp[J * XS]; });
                        static_for<4>([&](auto J) { accv = cmac(accv, row_share<decltype(J)::value>(gv), xv[J]); });
                    }
                    {
                        cx<T> xv[3];
                        static_for<3>([&](auto J) { xv[J] = xp[(4 + J) * XS]; });
                        static_for<3>([&](auto J) { accv = cmac(accv, row_share<4 + decltype(J)::value>(gv), xv[J]); });
                    }
                    static_for<5>([&](auto P) {
                        constexpr int y0 = 7 + 2 * decltype(P)::value, y1 = y0 + 1;
                        if (y0 < S) {
                            const cx<T> x0 = xp[y0 * XS], x1 = xp[y1 * XS];
                            accv = cmac(accv, row_share<y0>(gv), x0);
                            accv = cmac(accv, y1 < 16 ? row_share<y1 & 15>(gv) : row_share<0>(gv16), x1);
                        }
                    });
                    acc = accv * gu;
                    if (S == 17) {
                        acc = cmac(acc, gv * row_share<0>(gu16), Xs[base + lane * XS + 16]);
                        if (lane == 0) acc = cmac(acc, gv16 * gu16, Xs[base + 16 * XS + 16]);
                    }
                    acc.x = sum16(acc.x);
                    acc.y = sum16(acc.y);
                }
                if (OP == OP_DEGRID) {
                    if (lane == 0) a.yout[a.perm[m]] = acc;
                } else if (OP == OP_FUSED) {
                    r = acc - yv;
                    if (lane == 0) r2 += (double)r.x * (double)r.x + (double)r.y * (double)r.y;
                } else {
                    r = yv;
                }
                if (GA) {
                    // publish P = r conj(g_u), g_v and the window origin in the
                    // group's slot (entries past the window are zero)
                    cx<T> *ps = slot + grp * SLOT + PAD;
                    ps[lane] = mulc(r, gu);
                    ps[LEN + lane] = gv;
                    if (lane == 0) {
                        ps[16] = mulc(r, gu16);
                        ps[LEN + 16] = gv16;
                        // where the gather reads: slot entries of P[-bx] and g_v[-by]
                        sorg[grp] = (grp * SLOT + PAD - (cu - item.tx0 + a.H - h - 3)) |
                                    ((grp * SLOT + LEN + PAD - (cv - item.ty0 + a.H - h - 3)) << 16);
                    }
                } else if (OP & OP_GRID) {
                    // Y[ay][c] += r conj(g_v[ay] g_u[c])
                    const cx<T> rc = mulc(r, gu);
                    double *yr = Yr + base + lane, *yi = Yi + base + lane;
                    if (col) {   // the row weights come from lanes ay < S, all active here
                        static_for<17>([&](auto J) {
                            constexpr int ay = decltype(J)::value;
                            if (ay < 7 || ay < S) {
                                const cx<T> gy = ay < 16 ? row_share<ay & 15>(gv) : row_share<0>(gv16);
                                const cx<T> v = mulc(rc, gy);
                                lds_add(yr + ay * W, (double)v.x);
                                lds_add(yi + ay * W, (double)v.y);
                            }
                        });
                    }
                    if (S == 17) {
                        const cx<T> v = mulc(mulc(r, row_share<0>(gu16)), gv);
                        const int o = base + lane * W + 16;
                        lds_add(&Yr[o], (double)v.x);
                        lds_add(&Yi[o], (double)v.y);
                        if (lane == 0) {
                            const cx<T> v2 = mulc(mulc(r, gu16), gv16);
                            const int o2 = base + 16 * W + 16;
                            lds_add(&Yr[o2], (double)v2.x);
                            lds_add(&Yi[o2], (double)v2.y);
                        }
                    }
                }
            } else {
                // stored row: lane l holds entries t = l + 16 i (row-major over the
                // window); its columns follow from the window. The window cell
                // (ay, ax) of entry t advances by 16 entries per slot without a
                // division: 16 = q16 S + (16 - q16 S), q16 = floor(16 / S).
                rec_n = a.rec[item.vb + min(vi + GROUPS, item.vc - 1)];
                // the data value is issued with the row, ahead of the sum
                const cx<T> ydv = (OP & OP_GRID) ? ydata(m) : mk<T>((T)0, (T)0);
                const cx<T> *gp = a.gval + a.rowptr[m];
                cx<T> wv[MAXI];
#pragma unroll
                for (int i = 0; i < MAXI; ++i) {
                    const int t = lane + 16 * i;
                    wv[i] = mk<T>((T)0, (T)0);
                    if (i < NI && t < SS) wv[i] = gp[t];
                }
                const int q16 = S <= 8 ? 2 : (S <= 16 ? 1 : 0);
                const int ay0 = (lane >= S) + (lane >= 2 * S), ax0 = lane - ay0 * S;
                if (OP & OP_DEGRID) {
                    int ay = ay0, ax = ax0;
#pragma unroll
                    for (int i = 0; i < MAXI; ++i) {
                        if (i < NI && lane + 16 * i < SS) acc = cmac(acc, wv[i], Xs[base + ay * W + ax]);
                        ax += 16 - q16 * S;
                        ay += q16;
                        if (ax >= S) { ax -= S; ++ay; }
                    }
                    acc.x = sum16(acc.x);
                    acc.y = sum16(acc.y);
                }
                if (OP == OP_DEGRID) {
                    if (lane == 0) a.yout[a.perm[m]] = acc;
                } else if (OP == OP_FUSED) {
                    r = acc - ydv;
                    if (lane == 0) r2 += (double)r.x * (double)r.x + (double)r.y * (double)r.y;
                } else {
                    r = ydv;
                }
                if (OP & OP_GRID) {
                    int ay = ay0, ax = ax0;
#pragma unroll
                    for (int i = 0; i < MAXI; ++i) {
                        if (i < NI && lane + 16 * i < SS) {
                            const cx<T> c = mulc(r, wv[i]);
                            const int o = base + ay * W + ax;
                            lds_add(&Yr[o], (double)c.x);
                            lds_add(&Yi[o], (double)c.y);
                        }
                        ax += 16 - q16 * S;
                        ay += q16;
                        if (ax >= S) { ax -= S; ++ay; }
                    }
                }
            }
            if (OTF && !GA) wave_sync();   // wk is rewritten by the group's next visibility
          } else if (GA) {
            // no visibility left for this group: its slot adds zeros
            cx<T> *ps = slot + grp * SLOT + PAD;
            ps[lane] = mk<T>((T)0, (T)0);
            if (lane == 0) {
                ps[16] = mk<T>((T)0, (T)0);
                sorg[grp] = (grp * SLOT) | ((grp * SLOT + LEN) << 16);
            }
          }
          if constexpr (MF) {
            // Gather-form gridding on the matrix cores: the same sum as below
            // as v_mfma_f32_16x16x4_f32 products with K = the wave's four
            // visibilities. Lane 16 v + c supplies visibility v (its own
            // group's slot): A[c][v] = g_v of subgrid row 16 ty + c and
            // B[v][c] = P of subgrid column 16 tx + c, so the product adds
            // sum_v g_v[y] P_v[x] to tile (ty, tx) of the subgrid; the real
            // part takes Re g Re P + Im g Im P, the imaginary part
            // Re g Im P - Im g Re P (P conj g_v). Two tiles a side cover 32
            // cells; 16 products per four visibilities, 4 LDS reads per lane.
            wave_sync();
            const int org = sorg[grp];
            const cx<T> *pp = slot + (org & 0xFFFF) + lane;
            const cx<T> *qq = slot + (org >> 16) + lane;
            const cx<T> p0 = pp[0], p1 = pp[16], q0 = qq[0], q1 = qq[16];
            static_for<2>([&](auto TY) {
                constexpr int ty = decltype(TY)::value;
                const cx<T> q = ty ? q1 : q0;
                const float nqy = -q.y;
                static_for<2>([&](auto TX) {
                    constexpr int tx = decltype(TX)::value;
                    const cx<T> p = tx ? p1 : p0;
                    mre[ty][tx] = __builtin_amdgcn_mfma_f32_16x16x4f32(q.x, p.x, mre[ty][tx], 0, 0, 0);
                    mim[ty][tx] = __builtin_amdgcn_mfma_f32_16x16x4f32(q.x, p.y, mim[ty][tx], 0, 0, 0);
                });
                static_for<2>([&](auto TX) {
                    constexpr int tx = decltype(TX)::value;
                    const cx<T> p = tx ? p1 : p0;
                    mre[ty][tx] = __builtin_amdgcn_mfma_f32_16x16x4f32(q.y, p.y, mre[ty][tx], 0, 0, 0);
                    mim[ty][tx] = __builtin_amdgcn_mfma_f32_16x16x4f32(nqy, p.x, mim[ty][tx], 0, 0, 0);
                });
            });
            wave_sync();   // the slots are rewritten by the next four visibilities
          } else if constexpr (GA) {
            // Gather-form gridding: each wave holds the whole output subgrid
            // in registers, lane l the GB x GB cells x = GB (l & 7) + j,
            // y = GB (l >> 3) + i, and adds for each of its four visibilities
            //   Y[y][x] += P[x - bx] conj(g_v[y - by])
            // with P and g_v read from the slot at offsets padded with zeros
            // (W - 7 entries before the window, the rest after it), so cells
            // outside a window add exact zeros without a test. No atomics: the
            // cost per visibility is 2 GB LDS reads per lane.
            wave_sync();
            const int wl = tid & 63, lx = wl & 7, ly = wl >> 3, sb = grp & ~3;
            const int4 o4 = *reinterpret_cast<const int4 *>(sorg + sb);
            // software-pipelined: the next slot's vectors load while this
            // slot's products accumulate
            cx<T> p[NB], q[NB];
            {
                const cx<T> *pp = slot + (o4.x & 0xFFFF) + NB * lx;
                const cx<T> *qq = slot + (o4.x >> 16) + NB * ly;
                static_for<NB>([&](auto J) { p[J] = pp[J]; q[J] = qq[J]; });
            }
            static_for<4>([&](auto S4) {
                constexpr int s4 = decltype(S4)::value;
                cx<T> pn[NB], qn[NB];
                if constexpr (s4 < 3) {
                    const int org = s4 == 0 ? o4.y : (s4 == 1 ? o4.z : o4.w);
                    const cx<T> *pp = slot + (org & 0xFFFF) + NB * lx;
                    const cx<T> *qq = slot + (org >> 16) + NB * ly;
                    static_for<NB>([&](auto J) { pn[J] = pp[J]; qn[J] = qq[J]; });
                }
                static_for<NB>([&](auto I) {
                    static_for<NB>([&](auto J) {
                        gacc[I][J].x = fma(p[J].x, q[I].x, fma(p[J].y, q[I].y, gacc[I][J].x));
                        gacc[I][J].y = fma(p[J].y, q[I].x, fma(-p[J].x, q[I].y, gacc[I][J].y));
                    });
                });
                if constexpr (s4 < 3) {
                    static_for<NB>([&](auto J) { p[J] = pn[J]; q[J] = qn[J]; });
                }
            });
            wave_sync();   // the slots are rewritten by the next four visibilities
          }
        }
        __syncthreads();
        if constexpr (GA) {
            // sum of the four waves' subgrids: waves 0 and 1 store theirs (in
            // X's region and the slots), waves 2 and 3 add theirs, then the
            // two partial sums are added and flushed
            const int w = tid >> 6, wl = tid & 63, lx = wl & 7, ly = wl >> 3;
            cx<T> *R = (w & 1) ? slot : Xs;
            if constexpr (MF) {
                // lane l holds rows 4 (l / 16) + e, column l % 16 of each tile
                auto put = [&](bool add) {
                    static_for<2>([&](auto TY) { static_for<2>([&](auto TX) { static_for<4>([&](auto E) {
                        constexpr int ty = decltype(TY)::value, tx = decltype(TX)::value, e = decltype(E)::value;
                        const int y = 16 * ty + 4 * (wl >> 4) + e, x = 16 * tx + (wl & 15);
                        if (x < W && y < W) {
                            const cx<T> v = mk<T>(mre[ty][tx][e], mim[ty][tx][e]);
                            R[y * W + x] = add ? R[y * W + x] + v : v;
                        }
                    }); }); });
                };
                if (w < 2) put(false);
                __syncthreads();
                if (w >= 2) put(true);
            } else {
            if (w < 2) {
                static_for<NB>([&](auto I) {
                    static_for<NB>([&](auto J) {
                        const int y = NB * ly + I, x = NB * lx + J;
                        if (x < W && y < W) R[y * W + x] = gacc[I][J];
                    });
                });
            }
            __syncthreads();
            if (w >= 2) {
                static_for<NB>([&](auto I) {
                    static_for<NB>([&](auto J) {
                        const int y = NB * ly + I, x = NB * lx + J;
                        if (x < W && y < W) R[y * W + x] = R[y * W + x] + gacc[I][J];
                    });
                });
            }
            }
            __syncthreads();
            for (int e = tid; e < WW; e += blockDim.x) {
                const cx<T> v = Xs[e] + slot[e];
                if (v.x != (T)0 || v.y != (T)0) {
                    const int r = e / W, cc = e - r * W;
                    cx<T> *dst = Yg + ((size_t)((y0 + r) & Npm) << a.logNp) + ((x0 + cc) & Npm);
                    global_add(&dst->x, v.x);
                    global_add(&dst->y, v.y);
                }
            }
        } else if constexpr ((OP & OP_GRID) != 0) {
            for (int e = tid; e < WW; e += blockDim.x) {
                const double vr = Yr[e], vi = Yi[e];
                if (vr != 0.0 || vi != 0.0) {
                    const int r = e / W, cc = e - r * W;
                    cx<T> *dst = Yg + ((size_t)((y0 + r) & Npm) << a.logNp) + ((x0 + cc) & Npm);
                    global_add(&dst->x, (T)vr);
                    global_add(&dst->y, (T)vi);
                }
            }
        }
    }
    if (OP == OP_FUSED) {
        for (int o = 32; o >= 1; o >>= 1) r2 += __shfl_xor(r2, o);
        if ((tid & 63) == 0) s_red[tid >> 6] = r2;
        __syncthreads();
        if (tid == 0) a.r2part[blockIdx.x] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
    }
}

// Stored G fill: per row the values of its S x S window in row-major window
// order (FP64 arithmetic, rounded to T); the columns follow from the window.
template <typename T>
__global__ void __launch_bounds__(256) k_fill_csr(TileArgs<double> a, int64_t M, const int64_t *rowptr,
                                                  cx<T> *val) {
    __shared__ double kbs[GROUPS * SCR_KB];
    __shared__ cx<double> wks[GROUPS * SCR_W];
    __shared__ cx<double> gs[GROUPS * SCR_G];
    const int tid = threadIdx.x, lane = tid & 15, grp = tid >> 4;
    double *kbg = kbs + grp * SCR_KB;
    cx<double> *wk = wks + grp * SCR_W;
    cx<double> *gg = gs + grp * SCR_G;
    for (int64_t m = (int64_t)blockIdx.x * GROUPS + grp; m < M; m += (int64_t)gridDim.x * GROUPS) {
        const uint2 rec = a.rec[m];
        const int pl = (int)(rec.y & 0xFFFFu), h = (int)((rec.y >> 16) & 0xFu);
        const int S = 2 * h + 7, SS = S * S;
        axis_weights<double>(a, (int)m, pl, h, S, lane, kbg, wk, gg);
        const int64_t rp = rowptr[m];
        for (int t = lane; t < SS; t += 16) {
            const int ay = t / S, ax = t - ay * S;
            const cx<double> w = gg[18 + ay] * gg[ax];
            val[rp + t] = mk<T>((T)w.x, (T)w.y);
        }
        wave_sync();
    }
}

// Axis-factor fill: per visibility its two axis weight vectors (FP64
// arithmetic, rounded to T), as pairs (g_u[c], g_v[c]) for c < 17, zero past S.
template <typename T>
__global__ void __launch_bounds__(256) k_fill_sep(TileArgs<double> a, int64_t M, cx<T> *out) {
    __shared__ double kbs[GROUPS * SCR_KB];
    __shared__ cx<double> wks[GROUPS * SCR_W];
    __shared__ cx<double> gs[GROUPS * SCR_G];
    const int tid = threadIdx.x, lane = tid & 15, grp = tid >> 4;
    double *kbg = kbs + grp * SCR_KB;
    cx<double> *wk = wks + grp * SCR_W;
    cx<double> *gg = gs + grp * SCR_G;
    for (int64_t m = (int64_t)blockIdx.x * GROUPS + grp; m < M; m += (int64_t)gridDim.x * GROUPS) {
        const uint2 rec = a.rec[m];
        const int pl = (int)(rec.y & 0xFFFFu), h = (int)((rec.y >> 16) & 0xFu);
        const int S = 2 * h + 7;
        axis_weights<double>(a, (int)m, pl, h, S, lane, kbg, wk, gg);
        cx<T> *o = out + (size_t)m * 34;
        for (int cidx = lane; cidx < 17; cidx += 16) {
            const cx<double> u = cidx < S ? gg[cidx] : mk<double>(0.0, 0.0);
            const cx<double> w = cidx < S ? gg[18 + cidx] : mk<double>(0.0, 0.0);
            o[2 * cidx] = mk<T>((T)u.x, (T)u.y);
            o[2 * cidx + 1] = mk<T>((T)w.x, (T)w.y);
        }
        wave_sync();
    }
}

// H = G^H G (appendix E), row by row of G: every pair of cells k, k + d of
// the window with d in the stored upper half (dy > 0, or dy = 0 and dx >= 0)
// adds conj(G[m, k]) G[m, k + d] = conj(g_v[ay] g_u[ax]) g_v[by] g_u[bx] to
// H[k][k + d] (FP64 products, added in T by device-scope atomics). The 16
// lanes of a group take consecutive window columns ax of one offset, so each
// atomic instruction lands on one or two cache lines of an offset plane.
// Visibility i of the launch is m = i * stride mod M (stride coprime to M):
// groups in flight work on windows far apart in the tile-sorted order and
// rarely add to the same entries at once.
template <typename T>
__global__ void __launch_bounds__(256) k_fill_holo(TileArgs<double> a, int64_t M, int64_t stride,
                                                   const int32_t *tmap, const int4 *tinfo, const int64_t *off,
                                                   cx<T> *H) {
    __shared__ double kbs[GROUPS * SCR_KB];
    __shared__ cx<double> wks[GROUPS * SCR_W];
    __shared__ cx<double> gs[GROUPS * SCR_G];
    const int tid = threadIdx.x, lane = tid & 15, grp = tid >> 4;
    double *kbg = kbs + grp * SCR_KB;
    cx<double> *wk = wks + grp * SCR_W;
    cx<double> *gg = gs + grp * SCR_G;
    const int Npm = (1 << a.logNp) - 1, ntx = 1 << (a.logNp - 5);
    for (int64_t i = (int64_t)blockIdx.x * GROUPS + grp; i < M; i += (int64_t)gridDim.x * GROUPS) {
        const int64_t m = (int64_t)((uint64_t)i * (uint64_t)stride % (uint64_t)M);   // M < 2^31
        const uint2 rec = a.rec[m];
        const int cu = (int)(rec.x & 0xFFFFu), cv = (int)(rec.x >> 16);
        const int pl = (int)(rec.y & 0xFFFFu), h = (int)((rec.y >> 16) & 0xFu);
        const int S = 2 * h + 7;
        axis_weights<double>(a, (int)m, pl, h, S, lane, kbg, wk, gg);
        for (int ay = 0; ay < S; ++ay) {
            const int ky = (cv + ay - h - 3) & Npm;
            const int trow = (ky >> 5) * ntx, cyl = (ky & 31) * 32;
            const cx<double> gva = conjg(gg[18 + ay]);
            for (int by = ay; by < S; ++by) {
                const cx<double> pv = gva * gg[18 + by];
                const int dy = by - ay;
                for (int dx = dy == 0 ? 0 : 1 - S; dx < S; ++dx) {
                    const int axlo = max(0, -dx), axhi = min(S, S - dx);
                    for (int ax = axlo + lane; ax < axhi; ax += 16) {
                        const int kx = (cu + ax - h - 3) & Npm;
                        const int slot = tmap[trow + (kx >> 5)];
                        const int R = tinfo[slot].z;
                        const cx<double> v = pv * mulc(gg[ax + dx], gg[ax]);
                        cx<T> *dst = H + off[slot] + ((int64_t)(dy * (2 * R + 1) + dx + R) << 10) + cyl + (kx & 31);
                        global_add(&dst->x, (T)v.x);
                        global_add(&dst->y, (T)v.y);
                    }
                }
            }
        }
        wave_sync();
    }
}

template <typename T>
TileArgs<T> make_args(ri_ctx *c, const View &v, Prec<T> &p) {
    TileArgs<T> a{};
    a.items = v.items;
    a.n_items = v.n_items;
    a.counter = c->d_counter;
    a.tile = v.tile;
    a.H = c->H;
    a.W = v.tile + 2 * c->H;
    a.logNp = c->logNp;
    a.hmax = c->hmax;
    // Horner coefficients of the KB kernel as a power series in z (FP64)
    double i0b = 1.0, t = 1.0, q = 0.25 * c->beta * c->beta;
    for (int k = 1; k < 500; ++k) { t = t * q / ((double)k * k); i0b += t; if (t < 1e-17 * i0b) break; }
    a.kb_terms = sizeof(T) == 4 ? 22 : 32;
    double ck = 1.0 / i0b;
    for (int k = 0; k < KB_TERMS_MAX; ++k) {
        a.kbc[k] = (T)ck;
        ck = ck * q / ((double)(k + 1) * (double)(k + 1));
    }
    a.rec = v.rec;
    a.frac = (const T *)v.frac;
    a.wtaps = p.wtaps;
    a.perm = v.perm;
    return a;
}

// Dynamic LDS of one k_tiles workgroup on a W x W subgrid (the layout at the
// kernel's top): X (cx<T>) when degridding, the FP64 real and imaginary planes
// when gridding, the groups' w-taps, the reduction slots and the item index.
// The gather form (GB > 0) has X's region (W rows of its covered side) in
// every case, the groups' slots and window origins in place of the FP64 planes.
size_t tiles_lds(size_t W, bool degrid, bool grid, size_t cx_bytes, int GB = 0) {
    const size_t WW = W * W;
    if (GB > 0)
        return cx_bytes * W * (size_t)ga_cover(GB) + cx_bytes * GROUPS * (size_t)ga_slot_cx((int)W, GB) +
               sizeof(int) * GROUPS +
               cx_bytes * GROUPS * SCR_W + 4 * sizeof(double) + 16;
    return cx_bytes * WW * (degrid ? 1 : 0) + 2 * sizeof(double) * WW * (grid ? 1 : 0) +
           cx_bytes * GROUPS * SCR_W + 4 * sizeof(double) + 16;
}

template <typename T, int OP, int GM, int GB>
void launch_op_gb(ri_ctx *c, TileArgs<T> &a, hipStream_t s) {
    // the gather form's subgrid fits the side its lanes cover, and its
    // reduction stores a W x W partial subgrid in the slots
    if (GB > 0 && (a.W > ga_cover(GB) || (size_t)a.W * a.W > (size_t)GROUPS * ga_slot_cx(a.W, GB)))
        throw Error(RI_EUNSUPPORTED, "gather-form tile kernel launched on a subgrid it does not cover");
    const size_t lds = tiles_lds((size_t)a.W, (OP & OP_DEGRID) != 0, (OP & OP_GRID) != 0, sizeof(cx<T>), GB);
    if (lds + 64 > (size_t)c->dev.lds_per_block)
        throw Error(RI_EUNSUPPORTED, "tile " + std::to_string(a.tile) + " needs " + std::to_string(lds) +
                                         " B of LDS per workgroup; device allows " +
                                         std::to_string(c->dev.lds_per_block));
    int per_cu = (int)std::max<size_t>(1, std::min<size_t>(8, (160 * 1024) / (lds + 1024)));
    int nwg = std::min(c->dev.cu_count * per_cu, std::max(1, a.n_items));
    if (nwg > c->n_partials) nwg = c->n_partials;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_tiles<T, OP, GM, GB>), dim3(nwg), dim3(256), lds, s, a);
    if (OP == OP_FUSED && nwg < c->n_partials) fill_zero_f64(a.r2part + nwg, c->n_partials - nwg, s);
}

// Gridding through separable rows in FP32 takes the gather form when the
// subgrid fits it unless the context asks for the scatter form: on the VALU
// up to 24 cells a side, on the matrix cores up to 32.
template <typename T, int OP, int GM>
void launch_op(ri_ctx *c, TileArgs<T> &a, hipStream_t s) {
    if constexpr (std::is_same<T, float>::value && GM != RI_G_CSR && (OP & OP_GRID) != 0) {
        if (c->d.grid_form == RI_GRID_GATHER && a.W <= 24) return launch_op_gb<T, OP, GM, 3>(c, a, s);
        if (c->d.grid_form == RI_GRID_GATHER && a.W <= 32) return launch_op_gb<T, OP, GM, GB_MF>(c, a, s);
    }
    launch_op_gb<T, OP, GM, 0>(c, a, s);
}

}  // namespace

int tiles_partials(ri_ctx *c) { return c->dev.cu_count * 8; }

size_t lds_for_tile(int tile, int H, int cx_bytes) { return tiles_lds((size_t)tile + 2 * H, true, true, cx_bytes); }

template <typename T, int GM>
void launch_mode(ri_ctx *c, TileArgs<T> &a, int op, hipStream_t s) {
    if (op == OP_DEGRID) launch_op<T, OP_DEGRID, GM>(c, a, s);
    else if (op == OP_GRID) launch_op<T, OP_GRID, GM>(c, a, s);
    else launch_op<T, OP_FUSED, GM>(c, a, s);
}

template <typename T>
void launch_tiles(ri_ctx *c, const View &v, Prec<T> &p, int op, int gm, const cx<T> *y_sorted,
                  const cx<T> *y_user, cx<T> *y_out_user, double *r2_partials, hipStream_t s, int32_t *counter) {
    if (c->M == 0 || v.n_items == 0) {
        if (op == OP_FUSED && r2_partials) fill_zero_f64(r2_partials, c->n_partials, s);
        return;
    }
    TileArgs<T> a = make_args<T>(c, v, p);
    a.X = p.gridB;
    a.Y = p.gridA;
    a.ysorted = y_sorted;
    a.yuser = y_user;
    a.yout = y_out_user;
    a.r2part = r2_partials;
    a.counter = counter ? counter : c->d_counter;
    if (gm == RI_G_CSR) {
        if (!c->csr.val || c->csr.val_bytes != (int)sizeof(cx<T>)) throw Error(RI_EINVAL, "no stored G of this precision");
        a.rowptr = c->csr.rowptr;
        a.gval = (const cx<T> *)c->csr.val;
    } else if (gm == RI_G_SEP) {
        if (!c->sep.w || c->sep.val_bytes != (int)sizeof(cx<T>))
            throw Error(RI_EINVAL, "no stored axis factors of this precision");
        a.sepw = (const cx<T> *)c->sep.w;
    }
    fill_zero_i32(a.counter, 1, s);
    ProfScope prof(c, PROF_TILES, s);
    if (gm == RI_G_OTF) launch_mode<T, RI_G_OTF>(c, a, op, s);
    else if (gm == RI_G_SEP) launch_mode<T, RI_G_SEP>(c, a, op, s);
    else launch_mode<T, RI_G_CSR>(c, a, op, s);
    RI_CHECK_HIP(hipGetLastError());
}

template <typename T>
void fill_csr(ri_ctx *c, hipStream_t s) {
    const View &v = c->view;
    if (v.frac_bytes != 8) throw Error(RI_EINVAL, "CSR fill needs FP64 fractions");
    // row pointers (internal order)
    std::vector<int64_t> rp(c->M + 1, 0);
    for (int64_t i = 0; i < c->M; ++i) {
        const int S = 2 * c->plane_h[c->plane[v.perm_host[i]]] + c->J;
        rp[i + 1] = rp[i] + (int64_t)S * S;
    }
    c->csr.nnz = rp[c->M];
    c->csr.val_bytes = (int)sizeof(cx<T>);
    c->csr.rowptr = (int64_t *)dev_alloc(c, sizeof(int64_t) * (c->M + 1));
    RI_CHECK_HIP(hipMemcpy(c->csr.rowptr, rp.data(), sizeof(int64_t) * (c->M + 1), hipMemcpyHostToDevice));
    c->csr.val = dev_alloc(c, sizeof(cx<T>) * (size_t)c->csr.nnz);
    ensure_prec<double>(c, c->p64);
    TileArgs<double> a = make_args<double>(c, v, c->p64);
    if (c->M > 0) {
        int nwg = (int)std::min<int64_t>((c->M + GROUPS - 1) / GROUPS, (int64_t)c->dev.cu_count * 16);
        hipLaunchKernelGGL(k_fill_csr<T>, dim3(nwg), dim3(256), 0, s, a, c->M, c->csr.rowptr,
                           (cx<T> *)c->csr.val);
        RI_CHECK_HIP(hipGetLastError());
    }
}

// Stored axis factors (RI_G_SEP): per visibility of the main view, in its
// internal order, the pairs (g_u[c], g_v[c]) for c = 0..16 (FP64 weights
// rounded to T, zero past the window), 34 complex values.
template <typename T>
void fill_sep(ri_ctx *c, hipStream_t s) {
    const View &v = c->view;
    if (v.frac_bytes != 8) throw Error(RI_EINVAL, "axis-factor fill needs FP64 fractions");
    c->sep.val_bytes = (int)sizeof(cx<T>);
    c->sep.w = dev_alloc(c, sizeof(cx<T>) * 34 * (size_t)std::max<int64_t>(1, c->M));
    ensure_prec<double>(c, c->p64);
    TileArgs<double> a = make_args<double>(c, v, c->p64);
    if (c->M > 0) {
        int nwg = (int)std::min<int64_t>((c->M + GROUPS - 1) / GROUPS, (int64_t)c->dev.cu_count * 16);
        hipLaunchKernelGGL(k_fill_sep<T>, dim3(nwg), dim3(256), 0, s, a, c->M, (cx<T> *)c->sep.w);
        RI_CHECK_HIP(hipGetLastError());
    }
}

template <typename T>
void fill_holo(ri_ctx *c, const View &v, hipStream_t s) {
    if (v.frac_bytes != 8) throw Error(RI_EINVAL, "holographic build needs FP64 fractions");
    ensure_prec<double>(c, c->p64);
    TileArgs<double> a = make_args<double>(c, v, c->p64);
    if (c->M > 0) {
        int nwg = (int)std::min<int64_t>((c->M + GROUPS - 1) / GROUPS, (int64_t)c->dev.cu_count * 16);
        int64_t stride = std::max<int64_t>(1, (int64_t)(0.6180339887498949 * (double)c->M));
        while (std::gcd(stride, c->M) != 1) ++stride;
        hipLaunchKernelGGL(k_fill_holo<T>, dim3(nwg), dim3(256), 0, s, a, c->M, stride, c->holo.tmap,
                           c->holo.tinfo, c->holo.off, (cx<T> *)c->holo.val);
        RI_CHECK_HIP(hipGetLastError());
    }
}

template void launch_tiles<float>(ri_ctx *, const View &, Prec<float> &, int, int, const cx<float> *,
                                  const cx<float> *, cx<float> *, double *, hipStream_t, int32_t *);
template void launch_tiles<double>(ri_ctx *, const View &, Prec<double> &, int, int, const cx<double> *,
                                   const cx<double> *, cx<double> *, double *, hipStream_t, int32_t *);
template void fill_sep<float>(ri_ctx *, hipStream_t);
template void fill_sep<double>(ri_ctx *, hipStream_t);
template void fill_csr<float>(ri_ctx *, hipStream_t);
template void fill_csr<double>(ri_ctx *, hipStream_t);
template void fill_holo<float>(ri_ctx *, const View &, hipStream_t);
template void fill_holo<double>(ri_ctx *, const View &, hipStream_t);

}  // namespace ri
