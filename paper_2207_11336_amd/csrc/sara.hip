// uSARA's denoiser (section "uSARA's handcrafted denoiser"): the prox of
// t ||w . Psi^dagger x||_1 + iota_+(x) for the SARA dictionary
// Psi = [Dirac, db1, ..., db8] / 3 (each basis an orthonormal 2D periodic
// wavelet transform with 4 levels), by sub-iterations of dual forward-backward
// with unit step (||Psi^dagger|| = 1):
//   x_k = max(0, z - Psi v_k),   v_{k+1} = clip(v_k + Psi^dagger x_k, -t w, t w),
// warm-started from the previous call's dual variable, and the reweighting of
// the log-sum penalty, w = rho / (rho + |Psi^dagger x|).
//
// Filters: the minimum-phase Daubechies low-pass filter with p vanishing
// moments (2p taps) is the spectral factor h(z) = sqrt(2) ((1+z)/2)^p Q(z)/Q(1)
// with Q's roots the roots outside the unit circle of z^{p-1} P_p((2-z-1/z)/4),
// P_p(y) = sum_{k<p} C(p-1+k, k) y^k; computed on the host (roots of P_p in y
// by Durand-Kerner in long double, then mapped to z) and checked for
// orthonormality before use. High-pass g[t] = (-1)^t h[L-1-t].
//
// Transform (per basis b = blockIdx.z, all 8 wavelet bases in one launch):
// one level on an n x n block (row stride N): rows then columns, each
// a[k] = sum_t h[t] x[(2k+t) mod n], d[k] = sum_t g[t] x[(2k+t) mod n],
// low half first; the top-left block goes on to the next level. The column
// pass writes only the low-low block for the next level and finalises every
// other coefficient in place: the dual update (clip), the new weight, or the
// plain coefficient. Synthesis runs the adjoint from the coarsest level, reading
// the coarse block from the previous level's result and the details from the
// coefficients; its last row pass sums the 8 bases and the Dirac part and
// applies max(0, z - .) with the Dirac dual update fused.
#include <cmath>
#include <complex>
#include <utility>

#include "ri_internal.h"

namespace ri {

namespace {

constexpr int NW = 8;          // wavelet bases (db1 .. db8)
constexpr int LEVELS = 4;
constexpr int LMAX = 16;

__constant__ double c_h64[NW][LMAX];
__constant__ double c_g64[NW][LMAX];
__constant__ float c_h32[NW][LMAX];
__constant__ float c_g32[NW][LMAX];

template <typename T> __device__ __forceinline__ T fh(int b, int t);
template <typename T> __device__ __forceinline__ T fg(int b, int t);
template <> __device__ __forceinline__ double fh<double>(int b, int t) { return c_h64[b][t]; }
template <> __device__ __forceinline__ double fg<double>(int b, int t) { return c_g64[b][t]; }
template <> __device__ __forceinline__ float fh<float>(int b, int t) { return c_h32[b][t]; }
template <> __device__ __forceinline__ float fg<float>(int b, int t) { return c_g32[b][t]; }

// f(integral_constant<int, i>) for i = 0 .. N-1, unrolled at compile time.
template <typename F, int... I>
__device__ __forceinline__ void static_for_(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) { static_for_(f, std::make_integer_sequence<int, N>{}); }

// 16 bytes of T as one LDS vector load.
template <typename T>
using vec16 = T __attribute__((ext_vector_type(16 / sizeof(T))));

enum { FIN_DUAL = 0, FIN_WEIGHT = 1, FIN_COEF = 2 };
enum { SYN_PROX = 0, SYN_PLAIN = 1 };

// Finalised coefficient val (unscaled) of basis slot j (1..8, 0 = Dirac) at flat index e.
template <typename T, int FIN>
__device__ __forceinline__ void finalise(T *dst9, const T *w9, size_t i9, T val, T scale, T par) {
    const T cval = val * scale;
    if (FIN == FIN_DUAL) {
        const T lim = par * w9[i9];
        dst9[i9] = fmin(fmax(dst9[i9] + cval, -lim), lim);
    } else if (FIN == FIN_WEIGHT) {
        dst9[i9] = par / (par + fabs(cval));
    } else {
        dst9[i9] = cval;
    }
}

// Column passes are register-blocked: a thread computes KB consecutive outputs
// of one column from one window of inputs held in registers (2 KB + L - 2
// inputs for analysis, KB + L/2 - 1 of each half for synthesis); KB is 8 on
// the finest level and smaller on the coarse ones, whose few columns would
// otherwise leave most of the device idle (col_block below). Row passes
// stage the row in LDS by coalesced loads; the analysis computes one output
// per lane per step, the synthesis 8 consecutive outputs per lane from
// 16-byte LDS windows (k_syn_rows, k_syn_final). The
// filter length L is a template parameter (one instantiation per basis, chosen
// from blockIdx.z).
// Column block of level side n: 8 outputs per thread at the finest levels, 4
// at n = 1024, 2 below (more workgroups for the small coarse levels).
inline int col_block(int n) { return n >= 2048 ? 8 : (n >= 1024 ? 4 : 2); }

// f(std::integral_constant<int, L>) for the filter length L = 2 (b + 1) of basis b.
template <typename F>
__device__ __forceinline__ void with_length(int b, F &&f) {
    switch (b) {
        case 0: f(std::integral_constant<int, 2>{}); break;
        case 1: f(std::integral_constant<int, 4>{}); break;
        case 2: f(std::integral_constant<int, 6>{}); break;
        case 3: f(std::integral_constant<int, 8>{}); break;
        case 4: f(std::integral_constant<int, 10>{}); break;
        case 5: f(std::integral_constant<int, 12>{}); break;
        case 6: f(std::integral_constant<int, 14>{}); break;
        default: f(std::integral_constant<int, 16>{}); break;
    }
}

// Row analysis of the n x n block of every basis: in (basis stride in_bs) -> tmp.
// Workgroup: one row of one basis, staged in LDS by coalesced loads; lane
// outputs k = tid, tid + 256, ... of both halves.
template <typename T>
__global__ void __launch_bounds__(256) k_ana_rows(const T *__restrict__ in, int64_t in_bs, T *__restrict__ tmp,
                                                  int N, int n) {
    extern __shared__ unsigned char smem_raw[];
    T *row_s = reinterpret_cast<T *>(smem_raw);
    const int b = blockIdx.z, row = blockIdx.y, half = n >> 1, m = n - 1;
    const T *src = in + b * in_bs + (size_t)row * N;
    for (int e = threadIdx.x; e < n; e += blockDim.x) row_s[e] = src[e];
    __syncthreads();
    T *dst = tmp + (size_t)b * N * N + (size_t)row * N;
    with_length(b, [&](auto Lc) {
        constexpr int L = decltype(Lc)::value;
        for (int k = threadIdx.x; k < half; k += blockDim.x) {
            T a = 0, d = 0;
#pragma unroll
            for (int t = 0; t < L; ++t) {
                const T v = row_s[(2 * k + t) & m];
                a += fh<T>(b, t) * v;
                d += fg<T>(b, t) * v;
            }
            dst[k] = a;
            dst[half + k] = d;
        }
    });
}

// Register-blocked row analysis (n a multiple of 8). The row is staged in LDS
// with a periodic tail, s[e] = row[e mod n] for e < n + AH; a lane computes the
// four output pairs k = 4 j .. 4 j + 3 from the window s[8 j .. 8 j + 24)
// (outputs need s[2 k + t], t < L <= 16) read as 16-byte vectors, and stores
// each half as one 4-element vector. ALLB: the eight bases share the input
// row (the finest level) and one workgroup computes all of them; otherwise
// one workgroup per row and basis (blockIdx.z).
constexpr int AH = 16;
constexpr int AWIN = 24;

template <typename T>
using vec4o = T __attribute__((ext_vector_type(4)));

template <typename T, int L>
__device__ __forceinline__ void ana_row_block(int b, const T *s, T (&a)[4], T (&d)[4]) {
    constexpr int E = 16 / sizeof(T);
    T w[AWIN];
#pragma unroll
    for (int i = 0; i < AWIN / E; ++i) {
        const vec16<T> v = reinterpret_cast<const vec16<T> *>(s)[i];
#pragma unroll
        for (int e = 0; e < E; ++e) w[i * E + e] = v[e];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        T aa = 0, dd = 0;
#pragma unroll
        for (int t = 0; t < L; ++t) {
            aa = fma(fh<T>(b, t), w[2 * u + t], aa);
            dd = fma(fg<T>(b, t), w[2 * u + t], dd);
        }
        a[u] = aa;
        d[u] = dd;
    }
}

template <typename T>
__device__ __forceinline__ void store4(T *p, const T (&v)[4]) {
    vec4o<T> o;
#pragma unroll
    for (int e = 0; e < 4; ++e) o[e] = v[e];
    *reinterpret_cast<vec4o<T> *>(p) = o;
}

template <typename T, int ALLB>
__global__ void __launch_bounds__(256) k_ana_rows_rb(const T *__restrict__ in, int64_t in_bs, T *__restrict__ tmp,
                                                     int N, int n) {
    extern __shared__ unsigned char smem_raw[];
    T *s = reinterpret_cast<T *>(smem_raw);
    const int row = blockIdx.y, half = n >> 1, m = n - 1, tid = threadIdx.x;
    const int b0 = ALLB ? 0 : (int)blockIdx.z;
    const T *src = in + b0 * in_bs + (size_t)row * N;
    for (int e = tid; e < n + AH; e += blockDim.x) s[e] = src[e & m];
    __syncthreads();
    const size_t NN = (size_t)N * N;
    auto basis = [&](int b, auto Lc) {
        constexpr int L = decltype(Lc)::value;
        T *dst = tmp + (size_t)b * NN + (size_t)row * N;
        for (int j = tid; 4 * j < half; j += blockDim.x) {
            T a[4], d[4];
            ana_row_block<T, L>(b, s + 8 * j, a, d);
            store4<T>(dst + 4 * j, a);
            store4<T>(dst + half + 4 * j, d);
        }
    };
    if (ALLB) {
        static_for<NW>([&](auto bc) {
            constexpr int b = decltype(bc)::value;
            basis(b, std::integral_constant<int, 2 * (b + 1)>{});
        });
    } else {
        with_length(b0, [&](auto Lc) { basis(b0, Lc); });
    }
}

// Column analysis: tmp -> low-low block into work (unless last) and every
// other coefficient finalised into dst9 (slot b + 1). Thread: column col,
// outputs k0 .. k0 + KB - 1 of both halves.
template <typename T, int FIN, int KB>
__global__ void __launch_bounds__(256) k_ana_cols(const T *__restrict__ tmp, T *__restrict__ work, T *dst9,
                                                  const T *__restrict__ w9, int N, int n, int last, T scale, T par) {
    const int b = blockIdx.z;
    const int col = blockIdx.x * 64 + (threadIdx.x & 63);
    const int k0 = (blockIdx.y * 4 + (threadIdx.x >> 6)) * KB, half = n >> 1, m = n - 1;
    if (col >= n || k0 >= half) return;
    const size_t NN = (size_t)N * N;
    const T *src = tmp + b * NN + col;
    const size_t base9 = (size_t)(b + 1) * NN;
    with_length(b, [&](auto Lc) {
        constexpr int L = decltype(Lc)::value, NR = 2 * KB + L - 2;
        T r[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j) r[j] = src[(size_t)((2 * k0 + j) & m) * N];
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
            const int k = k0 + kk;
            if (k >= half) break;
            T a = 0, d = 0;
#pragma unroll
            for (int t = 0; t < L; ++t) {
                a += fh<T>(b, t) * r[2 * kk + t];
                d += fg<T>(b, t) * r[2 * kk + t];
            }
            if (!last && col < half) work[b * NN + (size_t)k * N + col] = a;
            else finalise<T, FIN>(dst9, w9, base9 + (size_t)k * N + col, a, scale, par);
            finalise<T, FIN>(dst9, w9, base9 + (size_t)(half + k) * N + col, d, scale, par);
        }
    });
}

// Dirac slot of the analysis (weights or plain coefficients).
template <typename T, int FIN>
__global__ void k_ana_dirac(const T *__restrict__ x, T *dst9, int64_t n, T scale, T par) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        finalise<T, FIN>(dst9, nullptr, (size_t)i, x[i], scale, par);
}

// Synthesis of 2 KB consecutive outputs i0 .. i0 + 2 KB - 1 (i0 even) along one
// axis from the low half A and the high half D (element k at A[k * stride]):
// x[i] = sum_{t = i mod 2} h[t] A[k] + g[t] D[k], k = (i - t)/2 mod half.
template <typename T, int L, int KB>
__device__ __forceinline__ void syn_block(int b, const T *A, const T *D, size_t stride, int i0, int half, T *x) {
    constexpr int S2 = L / 2, NA = KB + S2 - 1;
    const int kb0 = (i0 >> 1) - S2 + 1, hm = half - 1;
    T ar[NA], dr[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) {
        const size_t k = (size_t)((kb0 + j) & hm);
        ar[j] = A[k * stride];
        dr[j] = D[k * stride];
    }
#pragma unroll
    for (int u = 0; u < KB; ++u) {
#pragma unroll
        for (int par = 0; par < 2; ++par) {
            T v = 0;
#pragma unroll
            for (int s2 = 0; s2 < S2; ++s2) {
                const int t = par + 2 * s2;
                v += fh<T>(b, t) * ar[u - s2 + S2 - 1] + fg<T>(b, t) * dr[u - s2 + S2 - 1];
            }
            x[2 * u + par] = v;
        }
    }
}

// Column synthesis of level block n: the coarse block (rows and columns < n/2)
// from work (or from the coefficients at the coarsest level), the rest from
// the coefficients v9 (slot b + 1) -> tmp. Thread: column col, rows i0 .. i0 + 2 KB - 1.
template <typename T, int KB>
__global__ void __launch_bounds__(256) k_syn_cols(const T *__restrict__ v9, const T *__restrict__ work,
                                                  T *__restrict__ tmp, int N, int n, int coarsest) {
    const int b = blockIdx.z;
    const int col = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i0 = (blockIdx.y * 4 + (threadIdx.x >> 6)) * 2 * KB, half = n >> 1;
    if (col >= n || i0 >= n) return;
    const size_t NN = (size_t)N * N;
    const T *cf = v9 + (size_t)(b + 1) * NN + col;
    const T *lo = (!coarsest && col < half) ? work + b * NN + col : cf;
    T x[2 * KB];
    with_length(b, [&](auto Lc) {
        syn_block<T, decltype(Lc)::value, KB>(b, lo, cf + (size_t)half * N, N, i0, half, x);
    });
    T *dst = tmp + b * NN + col;
#pragma unroll
    for (int u = 0; u < 2 * KB; ++u)
        if (i0 + u < n) dst[(size_t)(i0 + u) * N] = x[u];
}

// Row synthesis of one staged row (low half A = s[0, half), high half D =
// s[half, n)) at output j: sum_{t = j mod 2} h[t] A[k] + g[t] D[k], k = (j - t)/2 mod half.
// Used for the coarse levels with n < 8 only.
template <typename T, int L>
__device__ __forceinline__ T syn_row_at(int b, const T *row_s, int j, int half) {
    const int hm = half - 1, j2 = j >> 1, par = j & 1;
    T x = 0;
#pragma unroll
    for (int s2 = 0; s2 < L / 2; ++s2) {
        const int k = (j2 - s2) & hm;
        x += fh<T>(b, par + 2 * s2) * row_s[k] + fg<T>(b, par + 2 * s2) * row_s[half + k];
    }
    return x;
}

// Row synthesis of level block n < 8: tmp -> work. Workgroup: one row of one
// basis staged in LDS, one output per lane.
template <typename T>
__global__ void __launch_bounds__(64) k_syn_rows_small(const T *__restrict__ tmp, T *__restrict__ work, int N,
                                                       int n) {
    __shared__ T row_s[8];
    const int b = blockIdx.z, row = blockIdx.y, half = n >> 1;
    const size_t NN = (size_t)N * N;
    const T *src = tmp + b * NN + (size_t)row * N;
    if (threadIdx.x < n) row_s[threadIdx.x] = src[threadIdx.x];
    __syncthreads();
    T *dst = work + b * NN + (size_t)row * N;
    with_length(b, [&](auto Lc) {
        if (threadIdx.x < n) dst[threadIdx.x] = syn_row_at<T, decltype(Lc)::value>(b, row_s, threadIdx.x, half);
    });
}

// Register-blocked row synthesis (n >= 8). A row of one basis is staged in LDS
// with a periodic halo of RH elements in front of each half:
//   s[k] = A[(k - RH) mod half]  and  s[RH + half + k] = D[(k - RH) mod half],
// k < RH + half. A lane computes the 8 consecutive outputs x[2u + par],
// u = u0 .. u0 + 3 (u0 = 4 i for its block i), from the 12-element windows
// s[u0 .. u0 + 12) of both halves, read as 16-byte vectors: A[u - s2] is
// window element u - u0 + RH - s2 for s2 < L/2 <= 8.
constexpr int RH = 8;
constexpr int RWIN = 12;

template <typename T>
using vec8o = T __attribute__((ext_vector_type(8)));   // the 8 outputs of a lane block

// Element e < n + 2 RH of the staged row: its source index in the row (low half, then high half).
__device__ __forceinline__ int staged_src(int e, int half) {
    const int hs = e >= RH + half ? 1 : 0;
    const int k = e - hs * (RH + half);
    return hs * half + ((k - RH) & (half - 1));
}

template <typename T>
__device__ __forceinline__ void lds_window(const T *p, T (&w)[RWIN]) {
    constexpr int E = 16 / sizeof(T);
#pragma unroll
    for (int i = 0; i < RWIN / E; ++i) {
        const vec16<T> v = reinterpret_cast<const vec16<T> *>(p)[i];
#pragma unroll
        for (int e = 0; e < E; ++e) w[i * E + e] = v[e];
    }
}

// acc[2u + par] += sum_{s2 < L/2} h[par + 2 s2] A[u0 + u - s2] + g[par + 2 s2] D[u0 + u - s2].
template <typename T, int L>
__device__ __forceinline__ void syn_row_block(int b, const T *s, int half, int u0, T (&acc)[8]) {
    T wa[RWIN], wd[RWIN];
    lds_window<T>(s + u0, wa);
    lds_window<T>(s + RH + half + u0, wd);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int par = 0; par < 2; ++par) {
            T v = acc[2 * u + par];
#pragma unroll
            for (int s2 = 0; s2 < L / 2; ++s2) {
                v = fma(fh<T>(b, par + 2 * s2), wa[u + RH - s2], v);
                v = fma(fg<T>(b, par + 2 * s2), wd[u + RH - s2], v);
            }
            acc[2 * u + par] = v;
        }
    }
}

// 8 outputs to library-owned memory (the level buffers, 8-element aligned blocks).
template <typename T>
__device__ __forceinline__ void store8(T *p, const T (&v)[8]) {
    vec8o<T> o;
#pragma unroll
    for (int e = 0; e < 8; ++e) o[e] = v[e];
    *reinterpret_cast<vec8o<T> *>(p) = o;
}

// Row synthesis of level block n (8 <= n < N): tmp -> work. Workgroup: one
// row of one basis, n / 8 lanes (at least 64).
template <typename T>
__global__ void __launch_bounds__(256) k_syn_rows(const T *__restrict__ tmp, T *__restrict__ work, int N, int n) {
    extern __shared__ unsigned char smem_raw[];
    T *s = reinterpret_cast<T *>(smem_raw);
    const int b = blockIdx.z, row = blockIdx.y, half = n >> 1, tid = threadIdx.x;
    const size_t NN = (size_t)N * N;
    const T *src = tmp + b * NN + (size_t)row * N;
    for (int e = tid; e < n + 2 * RH; e += blockDim.x) s[e] = src[staged_src(e, half)];
    __syncthreads();
    if (8 * tid >= n) return;
    T acc[8] = {};
    with_length(b, [&](auto Lc) { syn_row_block<T, decltype(Lc)::value>(b, s, half, 4 * tid, acc); });
    store8<T>(work + b * NN + (size_t)row * N + 8 * tid, acc);
}

// Last row synthesis (n = N), summed over the 8 bases plus the Dirac slot:
// SYN_PLAIN: x = scale * s; SYN_PROX: x = max(0, z - scale * s) and the
// Dirac dual update v0 = clip(v0 + scale * x, -t w0, t w0). Workgroup: one
// row, 256 lanes, each with NB blocks of 8 outputs (8 (tid + 256 ib)); the 8
// bases' staged rows pass through LDS one after another, the next one loaded
// into registers while the current one is used.
template <typename T, int MODE, int NB>
__global__ void __launch_bounds__(256) k_syn_final(const T *__restrict__ tmp, T *v9, const T *__restrict__ w9,
                                                   const T *__restrict__ z, T *__restrict__ x, int N, T scale,
                                                   T thr) {
    extern __shared__ unsigned char smem_raw[];
    T *s = reinterpret_cast<T *>(smem_raw);
    constexpr int PQ = 8 * NB + 1;           // staged elements per lane: ceil((256 * 8 NB + 2 RH) / 256)
    const int row = blockIdx.y, half = N >> 1, tid = threadIdx.x, ns = N + 2 * RH;
    const size_t NN = (size_t)N * N;
    T acc[NB][8], pre[PQ];
    int src[PQ];                             // the staging sources, the same for every basis
#pragma unroll
    for (int ib = 0; ib < NB; ++ib)
#pragma unroll
        for (int e = 0; e < 8; ++e) acc[ib][e] = 0;
    const T *r0 = tmp + (size_t)row * N;
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
        const int e = tid + 256 * q;
        src[q] = e < ns ? staged_src(e, half) : 0;
        pre[q] = e < ns ? r0[src[q]] : (T)0;
    }
    static_for<NW>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PQ; ++q)
            if (tid + 256 * q < ns) s[tid + 256 * q] = pre[q];
        __syncthreads();
        if (b + 1 < NW) {
            const T *nxt = tmp + (b + 1) * NN + (size_t)row * N;
#pragma unroll
            for (int q = 0; q < PQ; ++q) {
                const int e = tid + 256 * q;
                if (e < ns) pre[q] = nxt[src[q]];
            }
        }
#pragma unroll
        for (int ib = 0; ib < NB; ++ib)
            if (8 * (tid + 256 * ib) < N) syn_row_block<T, 2 * (b + 1)>(b, s, half, 4 * (tid + 256 * ib), acc[ib]);
    });
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) {
        const int j0 = 8 * (tid + 256 * ib);
        if (j0 >= N) break;
        // element accesses: v9, z and x may be caller buffers of any element alignment
        const size_t p = (size_t)row * N + j0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const T tot = v9[p + e] + acc[ib][e];
            if (MODE == SYN_PLAIN) {
                x[p + e] = scale * tot;
            } else {
                const T xo = fmax((T)0, z[p + e] - scale * tot);
                x[p + e] = xo;
                const T lim = thr * w9[p + e];
                v9[p + e] = fmin(fmax(v9[p + e] + scale * xo, -lim), lim);
            }
        }
    }
}

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// Filters on the host
// ---------------------------------------------------------------------------
using cld = std::complex<long double>;

// Roots of sum_k a[k] y^k (degree d = a.size() - 1 >= 1) by Durand-Kerner.
std::vector<cld> poly_roots(const std::vector<long double> &a) {
    const int d = (int)a.size() - 1;
    std::vector<cld> r(d);
    const cld seed(0.4L, 0.9L);
    cld pw(1.0L, 0.0L);
    for (int i = 0; i < d; ++i) { r[i] = pw; pw *= seed; }
    auto eval = [&](cld y) {
        cld v = 0;
        for (int k = d; k >= 0; --k) v = v * y + a[k];
        return v / a[d];
    };
    for (int it = 0; it < 2000; ++it) {
        long double moved = 0;
        for (int i = 0; i < d; ++i) {
            cld den = 1;
            for (int j = 0; j < d; ++j)
                if (j != i) den *= (r[i] - r[j]);
            const cld step = eval(r[i]) / den;
            r[i] -= step;
            moved = std::max(moved, std::abs(step));
        }
        if (moved < 1e-24L) break;
    }
    return r;
}

std::vector<double> daubechies(int p) {
    std::vector<cld> q(1, cld(1.0L, 0.0L));   // Q(z), increasing powers
    if (p > 1) {
        std::vector<long double> a(p);
        long double binom = 1;                 // C(p-1+k, k)
        for (int k = 0; k < p; ++k) {
            a[k] = binom;
            binom = binom * (long double)(p + k) / (long double)(k + 1);
        }
        for (const cld &y : poly_roots(a)) {
            const cld bq = 1.0L - 2.0L * y;
            const cld disc = std::sqrt(bq * bq - 1.0L);
            const cld z = std::abs(bq + disc) > 1.0L ? bq + disc : bq - disc;
            std::vector<cld> nq(q.size() + 1, cld(0));
            for (size_t i = 0; i < q.size(); ++i) {
                nq[i + 1] += q[i];
                nq[i] -= z * q[i];
            }
            q.swap(nq);
        }
    }
    std::vector<long double> h(q.size());
    for (size_t i = 0; i < q.size(); ++i) h[i] = q[i].real();
    for (int k = 0; k < p; ++k) {              // times (1 + z) / 2, p times
        std::vector<long double> nh(h.size() + 1, 0.0L);
        for (size_t i = 0; i < h.size(); ++i) {
            nh[i] += 0.5L * h[i];
            nh[i + 1] += 0.5L * h[i];
        }
        h.swap(nh);
    }
    long double sum = 0;
    for (long double v : h) sum += v;
    std::vector<double> out(h.size());
    for (size_t i = 0; i < h.size(); ++i) out[i] = (double)(h[i] * std::sqrt(2.0L) / sum);
    // orthonormality check: sum_k h[k] h[k + 2m] = delta_m
    for (int m = 0; m < p; ++m) {
        long double dot = 0;
        for (size_t k = 0; k + 2 * m < out.size(); ++k) dot += (long double)out[k] * out[k + 2 * m];
        if (std::fabs((double)dot - (m == 0 ? 1.0 : 0.0)) > 1e-13)
            throw Error(RI_EDEVICE, "Daubechies filter " + std::to_string(p) + " failed its orthonormality check");
    }
    return out;
}

void upload_filters(ri_ctx *c) {
    double h64[NW][LMAX] = {}, g64[NW][LMAX] = {};
    float h32[NW][LMAX] = {}, g32[NW][LMAX] = {};
    for (int b = 0; b < NW; ++b) {
        const std::vector<double> h = daubechies(b + 1);
        const int L = (int)h.size();
        for (int t = 0; t < L; ++t) {
            h64[b][t] = h[t];
            g64[b][t] = (t & 1 ? -1.0 : 1.0) * h[L - 1 - t];
            h32[b][t] = (float)h64[b][t];
            g32[b][t] = (float)g64[b][t];
        }
    }
    RI_CHECK_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_h64), h64, sizeof(h64)));
    RI_CHECK_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_g64), g64, sizeof(g64)));
    RI_CHECK_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_h32), h32, sizeof(h32)));
    RI_CHECK_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_g32), g32, sizeof(g32)));
    (void)c;
}

// Psi^dagger x into dst9 (FIN selects the dual update, the weights or the plain coefficients).
template <typename T, int FIN>
void analysis(ri_ctx *c, const T *x, T *dst9, T par, bool dirac, hipStream_t s) {
    SaraState &st = c->sara;
    const int N = c->N;
    const T scale = (T)(1.0 / 3.0);
    T *work = (T *)st.work, *tmp = (T *)st.tmp;
    const T *w9 = (const T *)st.w;
    if (dirac)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ana_dirac<T, FIN>), dim3(1024), dim3(256), 0, s, x, dst9,
                           (int64_t)N * N, scale, par);
    for (int l = 0; l < LEVELS; ++l) {
        const int n = N >> l;
        const T *in = l == 0 ? x : work;
        const int64_t in_bs = l == 0 ? 0 : (int64_t)N * N;
        if (n % 8 != 0)
            hipLaunchKernelGGL(k_ana_rows<T>, dim3(1, n, NW), dim3(256), sizeof(T) * n, s, in, in_bs, tmp, N, n);
        else if (l == 0)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ana_rows_rb<T, 1>), dim3(1, n, 1), dim3(256),
                               sizeof(T) * (n + AH), s, in, in_bs, tmp, N, n);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ana_rows_rb<T, 0>), dim3(1, n, NW),
                               dim3(std::min(256, std::max(64, n / 8))), sizeof(T) * (n + AH), s, in, in_bs, tmp,
                               N, n);
        const int kb = col_block(n), last = l == LEVELS - 1 ? 1 : 0;
        const dim3 g(cdiv(n, 64), cdiv(n / 2, 4 * kb), NW);
        if (kb == 8)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ana_cols<T, FIN, 8>), g, dim3(256), 0, s, tmp, work, dst9, w9, N, n,
                               last, scale, par);
        else if (kb == 4)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ana_cols<T, FIN, 4>), g, dim3(256), 0, s, tmp, work, dst9, w9, N, n,
                               last, scale, par);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ana_cols<T, FIN, 2>), g, dim3(256), 0, s, tmp, work, dst9, w9, N, n,
                               last, scale, par);
    }
}

// Psi v9 (MODE SYN_PLAIN) or x = max(0, z - Psi v9) with the Dirac dual update (SYN_PROX).
template <typename T, int MODE>
void synthesis(ri_ctx *c, T *v9, const T *z, T *x, T thr, hipStream_t s) {
    SaraState &st = c->sara;
    const int N = c->N;
    const T scale = (T)(1.0 / 3.0);
    T *work = (T *)st.work, *tmp = (T *)st.tmp;
    for (int l = LEVELS - 1; l >= 0; --l) {
        const int n = N >> l;
        const int kb = col_block(n), coarsest = l == LEVELS - 1 ? 1 : 0;
        const dim3 g(cdiv(n, 64), cdiv(n, 4 * 2 * kb), NW);
        if (kb == 8)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_syn_cols<T, 8>), g, dim3(256), 0, s, v9, work, tmp, N, n, coarsest);
        else if (kb == 4)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_syn_cols<T, 4>), g, dim3(256), 0, s, v9, work, tmp, N, n, coarsest);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_syn_cols<T, 2>), g, dim3(256), 0, s, v9, work, tmp, N, n, coarsest);
        if (l > 0 && n >= 8)
            hipLaunchKernelGGL(k_syn_rows<T>, dim3(1, n, NW), dim3(std::max(64, n / 8)), sizeof(T) * (n + 2 * RH), s,
                               tmp, work, N, n);
        else if (l > 0)
            hipLaunchKernelGGL(k_syn_rows_small<T>, dim3(1, n, NW), dim3(64), 0, s, tmp, work, N, n);
    }
    const size_t lds = sizeof(T) * (N + 2 * RH);
    if (N <= 2048)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_syn_final<T, MODE, 1>), dim3(1, N), dim3(256), lds, s, tmp, v9,
                           (const T *)st.w, z, x, N, scale, thr);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_syn_final<T, MODE, 2>), dim3(1, N), dim3(256), lds, s, tmp, v9,
                           (const T *)st.w, z, x, N, scale, thr);
}

}  // namespace

void sara_free(ri_ctx *c) {
    SaraState &st = c->sara;
    dev_free(c, st.v);
    dev_free(c, st.w);
    dev_free(c, st.work);
    dev_free(c, st.tmp);
    const int sub = st.sub_iters;
    st = SaraState{};
    st.sub_iters = sub;
}

void sara_setup(ri_ctx *c, int sub_iters, hipStream_t s) {
    if (c->N % 16 != 0) throw Error(RI_EUNSUPPORTED, "the SARA dictionary needs N divisible by 16");
    SaraState &st = c->sara;
    if (sub_iters > 0) st.sub_iters = sub_iters;
    const size_t eb = c->d.precision == 64 ? sizeof(double) : sizeof(float);
    const size_t NN = (size_t)c->N * c->N;
    if (!st.ready) {
        upload_filters(c);
        st.v = dev_alloc(c, eb * 9 * NN);
        st.w = dev_alloc(c, eb * 9 * NN);
        st.work = dev_alloc(c, eb * NW * NN);
        st.tmp = dev_alloc(c, eb * NW * NN);
        st.ready = true;
    }
    sara_reset(c, s);
}

void sara_reset(ri_ctx *c, hipStream_t s) {
    SaraState &st = c->sara;
    const int64_t n9 = 9 * (int64_t)c->N * c->N;
    if (c->d.precision == 64) {
        fill_real<double>((double *)st.v, n9, 0.0, s);
        fill_real<double>((double *)st.w, n9, 1.0, s);
    } else {
        fill_real<float>((float *)st.v, n9, 0.0f, s);
        fill_real<float>((float *)st.w, n9, 1.0f, s);
    }
}

template <typename T>
void sara_prox(ri_ctx *c, const T *z, T thr, T *x_out, hipStream_t s) {
    SaraState &st = c->sara;
    ProfScope ps(c, PROF_PROX, s);
    T *v9 = (T *)st.v;
    for (int k = 0; k < st.sub_iters; ++k) {
        synthesis<T, SYN_PROX>(c, v9, z, x_out, thr, s);
        analysis<T, FIN_DUAL>(c, x_out, v9, thr, false, s);
    }
}

template <typename T>
void sara_reweight(ri_ctx *c, const T *x, T rho, hipStream_t s) {
    ProfScope ps(c, PROF_OTHER, s);
    analysis<T, FIN_WEIGHT>(c, x, (T *)c->sara.w, rho, true, s);
}

template <typename T>
void sara_analysis(ri_ctx *c, const T *x, T *coef9, hipStream_t s) {
    analysis<T, FIN_COEF>(c, x, coef9, (T)0, true, s);
}

template <typename T>
void sara_synthesis(ri_ctx *c, const T *coef9, T *x, hipStream_t s) {
    synthesis<T, SYN_PLAIN>(c, const_cast<T *>(coef9), nullptr, x, (T)0, s);
}

template void sara_prox<float>(ri_ctx *, const float *, float, float *, hipStream_t);
template void sara_prox<double>(ri_ctx *, const double *, double, double *, hipStream_t);
template void sara_reweight<float>(ri_ctx *, const float *, float, hipStream_t);
template void sara_reweight<double>(ri_ctx *, const double *, double, hipStream_t);
template void sara_analysis<float>(ri_ctx *, const float *, float *, hipStream_t);
template void sara_analysis<double>(ri_ctx *, const double *, double *, hipStream_t);
template void sara_synthesis<float>(ri_ctx *, const float *, float *, hipStream_t);
template void sara_synthesis<double>(ri_ctx *, const double *, double *, hipStream_t);

}  // namespace ri
