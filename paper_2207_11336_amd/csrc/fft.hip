// F and F^dagger on the N' x N' grid (paper eq. 1: F is the DFT on the fine
// grid), fused with Z (zero padding + 1/kappa_hat correction) on the way in
// and with Z^dagger (crop, correction, real part) on the way out.
//
// Layout: grid row-major [ky][kx], wrap-centred (pixel n at cell n mod N').
// Rows: one workgroup per image row, the whole N'-point row in LDS, Stockham
// radix-16 passes (natural order in and out, twiddles from an FP64-computed
// table); the first pass reads global memory and the last one writes it
// directly. Only the N non-zero rows are transformed on the way in, and only
// the N needed rows on the way out.
// Columns: four-step decomposition N' = N1 * N2 over stripes of adjacent
// columns, so every global access is a contiguous row segment:
//   pass A: N1-point transforms along rows n2 + N2*n1, times W_{N'}^{n2 k1};
//   pass B: N2-point transforms along rows N2*k1 + n2, written to row k1 + N1*k2.
// For N' = 4096 and 8192 each column's points stay in registers (a few lanes
// per column, see k_colpass_a_reg); for the other sizes a stripe of CW
// columns is transformed in LDS by Stockham passes.
#include <utility>

#include "ri_internal.h"

namespace ri {

namespace {

// exp(-2 pi i k / 16), k = 0..15 (exact constants of the 16th roots of unity)
__device__ __constant__ double kRoot16[16][2] = {
    {1.0, 0.0},
    {0.92387953251128675613, -0.38268343236508977173},
    {0.70710678118654752440, -0.70710678118654752440},
    {0.38268343236508977173, -0.92387953251128675613},
    {0.0, -1.0},
    {-0.38268343236508977173, -0.92387953251128675613},
    {-0.70710678118654752440, -0.70710678118654752440},
    {-0.92387953251128675613, -0.38268343236508977173},
    {-1.0, 0.0},
    {-0.92387953251128675613, 0.38268343236508977173},
    {-0.70710678118654752440, 0.70710678118654752440},
    {-0.38268343236508977173, 0.92387953251128675613},
    {0.0, 1.0},
    {0.38268343236508977173, 0.92387953251128675613},
    {0.70710678118654752440, 0.70710678118654752440},
    {0.92387953251128675613, 0.38268343236508977173}};

constexpr int brev(int k, int bits) {
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((k >> b) & 1) << (bits - 1 - b);
    return r;
}
constexpr int ilog2(int R) { return R <= 1 ? 0 : 1 + ilog2(R / 2); }

// In-register R-point DFT, natural order in and out:
// V[k] = sum_r v[r] exp(-+ 2 pi i r k / R).
template <typename T, int R>
__device__ __forceinline__ void dft_reg(cx<T> *v, bool inv) {
#pragma unroll
    for (int span = R / 2; span >= 1; span >>= 1) {
#pragma unroll
        for (int m = 0; m < R; ++m) {
            if (m & span) continue;
            const int mloc = m & (2 * span - 1);
            cx<T> a = v[m], b = v[m + span];
            v[m] = a + b;
            cx<T> d = a - b;
            const int e = mloc * (16 / (2 * span));
            if (e != 0) {
                cx<T> w = mk<T>((T)kRoot16[e][0], inv ? -(T)kRoot16[e][1] : (T)kRoot16[e][1]);
                d = d * w;
            }
            v[m + span] = d;
        }
    }
    cx<T> t[R];
#pragma unroll
    for (int k = 0; k < R; ++k) t[k] = v[brev(k, ilog2(R))];
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = t[k];
}

template <bool PAD>
__device__ __forceinline__ int pidx(int i) { return PAD ? i + (i >> 5) : i; }

// One Stockham radix-R pass over s[L][CW] (transform along the first index),
// in place: every thread loads its groups, barrier, computes, stores, barrier.
// Requires (L/R)*CW <= (16/R) * blockDim.x.
template <typename T, int R, bool PAD>
__device__ __forceinline__ void stockham_pass(cx<T> *s, int L, int logCW, int Ns, const cx<T> *__restrict__ tw,
                                              int tw_mul, bool inv) {
    constexpr int G = 16 / R;
    const int CW = 1 << logCW;
    const int ng = (L / R) << logCW;
    cx<T> v[G][R];
#pragma unroll
    for (int i = 0; i < G; ++i) {
        const int g = threadIdx.x + i * blockDim.x;
        if (g < ng) {
            const int col = g & (CW - 1), j = g >> logCW;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = s[pidx<PAD>(((j + r * (L / R)) << logCW) + col)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < G; ++i) {
        const int g = threadIdx.x + i * blockDim.x;
        if (g < ng) {
            const int col = g & (CW - 1), j = g >> logCW;
            const int jm = j & (Ns - 1);
            const int step = jm * tw_mul * (L / (Ns * R));
            if (jm != 0) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    cx<T> w = tw[step * r];
                    if (inv) w.y = -w.y;
                    v[i][r] = v[i][r] * w;
                }
            }
            dft_reg<T, R>(v[i], inv);
            const int idxD = (j - jm) * R + jm;
#pragma unroll
            for (int r = 0; r < R; ++r) s[pidx<PAD>(((idxD + r * Ns) << logCW) + col)] = v[i][r];
        }
    }
    __syncthreads();
}

// Full L-point transform of every column of s[L][CW]; caller syncs before.
template <typename T, bool PAD>
__device__ void fft_lds(cx<T> *s, int logL, int logCW, const cx<T> *__restrict__ tw, int tw_mul, bool inv) {
    const int L = 1 << logL;
    int Ns = 1, rem = logL;
    while (rem > 0) {
        if (rem >= 4) { stockham_pass<T, 16, PAD>(s, L, logCW, Ns, tw, tw_mul, inv); Ns <<= 4; rem -= 4; }
        else if (rem == 3) { stockham_pass<T, 8, PAD>(s, L, logCW, Ns, tw, tw_mul, inv); Ns <<= 3; rem -= 3; }
        else if (rem == 2) { stockham_pass<T, 4, PAD>(s, L, logCW, Ns, tw, tw_mul, inv); Ns <<= 2; rem -= 2; }
        else { stockham_pass<T, 2, PAD>(s, L, logCW, Ns, tw, tw_mul, inv); Ns <<= 1; rem -= 1; }
    }
}

__device__ __forceinline__ bool in_band(int r, int N, int Np) { return r < N / 2 || r >= Np - N / 2; }

// Row transforms (one row of L = N' points per workgroup) read their input
// straight into the first pass and write their output straight from the last:
// the first pass (radix 16, Ns = 1, no twiddles) takes inputs j + r L/16 of
// group j from ld(index) and leaves 16 j + r in LDS; the last pass (radix R,
// Ns = L/R, twiddle step j) hands outputs j + r Ns to st(index, value). Both
// index patterns run contiguously over j, so the global accesses coalesce; the
// passes between are the LDS Stockham passes. Same arithmetic as fft_lds.
template <typename T, bool PAD, typename Load>
__device__ __forceinline__ void row_first_pass(cx<T> *s, int L, bool inv, Load &&ld) {
    const int ng = L / 16;
    for (int j = threadIdx.x; j < ng; j += blockDim.x) {
        cx<T> v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = ld(j + r * ng);
        dft_reg<T, 16>(v, inv);
#pragma unroll
        for (int r = 0; r < 16; ++r) s[pidx<PAD>(16 * j + r)] = v[r];
    }
    __syncthreads();
}

template <typename T, int R, bool PAD, typename Store>
__device__ __forceinline__ void row_last_pass(const cx<T> *s, int L, const cx<T> *__restrict__ tw, bool inv,
                                              Store &&st) {
    const int Ns = L / R;
    for (int j = threadIdx.x; j < Ns; j += blockDim.x) {
        cx<T> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = s[pidx<PAD>(j + r * Ns)];
        if (j != 0) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                cx<T> w = tw[j * r];
                if (inv) w.y = -w.y;
                v[r] = v[r] * w;
            }
        }
        dft_reg<T, R>(v, inv);
#pragma unroll
        for (int r = 0; r < R; ++r) st(j + r * Ns, v[r]);
    }
}

// Whole row, logL >= 5: the first pass, radix-16 LDS passes, the last pass.
template <typename T, bool PAD, typename Load, typename Store>
__device__ __forceinline__ void row_fft(cx<T> *s, int logL, const cx<T> *__restrict__ tw, bool inv, Load &&ld,
                                        Store &&st) {
    const int L = 1 << logL;
    row_first_pass<T, PAD>(s, L, inv, ld);
    int Ns = 16, rem = logL - 4;
    while (rem > 4) {
        stockham_pass<T, 16, PAD>(s, L, 0, Ns, tw, 1, inv);
        Ns <<= 4;
        rem -= 4;
    }
    switch (rem) {
        case 4: row_last_pass<T, 16, PAD>(s, L, tw, inv, st); break;
        case 3: row_last_pass<T, 8, PAD>(s, L, tw, inv, st); break;
        case 2: row_last_pass<T, 4, PAD>(s, L, tw, inv, st); break;
        default: row_last_pass<T, 2, PAD>(s, L, tw, inv, st); break;
    }
}

// Z then the row DFT of image row iy (blockIdx.x), written to grid row (iy - N/2) mod N'.
// With a w-stack's phase screen (chirp != NULL) the padded image is x c_s.
template <typename T, bool PAD>
__global__ void k_zpad_rowfft(const T *__restrict__ x, cx<T> *__restrict__ grid, const T *__restrict__ icorr,
                              const cx<T> *__restrict__ tw, int N, int logNp, const cx<T> *__restrict__ chirp) {
    extern __shared__ unsigned char smem_raw[];
    cx<T> *s = reinterpret_cast<cx<T> *>(smem_raw);
    const int Np = 1 << logNp;
    const int iy = blockIdx.x;
    const T cy = icorr[iy];
    const T *xr = x + (size_t)iy * N;
    const cx<T> *chr = chirp ? chirp + (size_t)iy * N : nullptr;
    auto ld = [&](int gx) -> cx<T> {
        const int ix = (gx + N / 2) & (Np - 1);
        if (ix >= N) return mk<T>((T)0, (T)0);
        const T a = xr[ix] * icorr[ix] * cy;
        if (chr) {
            const cx<T> ch = chr[ix];
            return mk<T>(a * ch.x, a * ch.y);
        }
        return mk<T>(a, (T)0);
    };
    cx<T> *row = grid + (size_t)((iy - N / 2) & (Np - 1)) * Np;
    row_fft<T, PAD>(s, logNp, tw, false, ld, [&](int k, cx<T> v) { row[k] = v; });
}

// Inverse row DFT of grid row (iy - N/2) mod N', then crop, correction, real part:
// out[iy][ix] = Re{row[(ix - N/2) mod N']} / (kappa_hat_x kappa_hat_y). With a
// w-stack's phase screen the value is Re{conj(c_s) row[...]} (Z_s^dagger), added
// to out when accumulate != 0 (the sum over stacks).
template <typename T, bool PAD>
__global__ void k_irowfft_crop(const cx<T> *__restrict__ grid, T *__restrict__ out, const T *__restrict__ icorr,
                               const cx<T> *__restrict__ tw, int N, int logNp, const cx<T> *__restrict__ chirp,
                               int accumulate) {
    extern __shared__ unsigned char smem_raw[];
    cx<T> *s = reinterpret_cast<cx<T> *>(smem_raw);
    const int Np = 1 << logNp;
    const int iy = blockIdx.x;
    const cx<T> *row = grid + (size_t)((iy - N / 2) & (Np - 1)) * Np;
    const T cy = icorr[iy];
    T *orow = out + (size_t)iy * N;
    const cx<T> *chr = chirp ? chirp + (size_t)iy * N : nullptr;
    auto st = [&](int gx, cx<T> v) {
        const int ix = (gx + N / 2) & (Np - 1);   // the crop: image column ix < N
        if (ix >= N) return;
        T re = v.x;
        if (chr) {
            const cx<T> ch = chr[ix];
            re = v.x * ch.x + v.y * ch.y;
        }
        const T val = re * icorr[ix] * cy;
        if (accumulate) orow[ix] += val;
        else orow[ix] = val;
    };
    row_fft<T, PAD>(s, logNp, tw, true, [&](int k) { return row[k]; }, st);
}

// Four-step pass A (in place): rows n2 + N2*n1 of stripe [x0, x0+CW).
template <typename T>
__global__ void k_colpass_a(cx<T> *__restrict__ grid, const cx<T> *__restrict__ tw, int N, int logNp, int logN1,
                            int logN2, int logCW, int band_in, int inv) {
    extern __shared__ unsigned char smem_raw[];
    cx<T> *s = reinterpret_cast<cx<T> *>(smem_raw);
    const int Np = 1 << logNp, N1 = 1 << logN1, N2 = 1 << logN2, CW = 1 << logCW;
    const int x0 = blockIdx.x * CW, n2 = blockIdx.y;
    const int nel = N1 * CW;
    for (int e = threadIdx.x; e < nel; e += blockDim.x) {
        const int n1 = e >> logCW, c = e & (CW - 1);
        const int r = n2 + N2 * n1;
        cx<T> v = mk<T>((T)0, (T)0);
        if (!band_in || in_band(r, N, Np)) v = grid[(size_t)r * Np + x0 + c];
        s[e] = v;
    }
    __syncthreads();
    fft_lds<T, false>(s, logN1, logCW, tw, Np >> logN1, inv != 0);
    for (int e = threadIdx.x; e < nel; e += blockDim.x) {
        const int k1 = e >> logCW, c = e & (CW - 1);
        cx<T> w = tw[n2 * k1];
        if (inv) w.y = -w.y;
        grid[(size_t)(n2 + N2 * k1) * Np + x0 + c] = s[e] * w;
    }
}

// Four-step pass B (out of place): rows N2*k1 + n2 -> rows k1 + N1*k2.
template <typename T>
__global__ void k_colpass_b(const cx<T> *__restrict__ in, cx<T> *__restrict__ out, const cx<T> *__restrict__ tw,
                            int N, int logNp, int logN1, int logN2, int logCW, int band_out, int inv) {
    extern __shared__ unsigned char smem_raw[];
    cx<T> *s = reinterpret_cast<cx<T> *>(smem_raw);
    const int Np = 1 << logNp, N1 = 1 << logN1, N2 = 1 << logN2, CW = 1 << logCW;
    const int x0 = blockIdx.x * CW, k1 = blockIdx.y;
    const int nel = N2 * CW;
    for (int e = threadIdx.x; e < nel; e += blockDim.x) {
        const int n2 = e >> logCW, c = e & (CW - 1);
        s[e] = in[(size_t)(N2 * k1 + n2) * Np + x0 + c];
    }
    __syncthreads();
    fft_lds<T, false>(s, logN2, logCW, tw, Np >> logN2, inv != 0);
    for (int e = threadIdx.x; e < nel; e += blockDim.x) {
        const int k2 = e >> logCW, c = e & (CW - 1);
        const int r = k1 + N1 * k2;
        if (!band_out || in_band(r, N, Np)) out[(size_t)r * Np + x0 + c] = s[e];
    }
}

// ---------------------------------------------------------------------------
// Column passes of the 4096- and 8192-point transforms (N1 = 64 or 128,
// N2 = 64) in registers: a one-wave workgroup takes 64/Q adjacent columns, Q
// lanes per column so that a lane holds at most 512 bytes of points (64 FP32
// or 32 FP64 complex values), so every load and store of the wave is a
// contiguous 512-byte row segment and no LDS or barrier is involved. Radix-2
// decimation in frequency, natural order in, bit-reversed out; twiddles come
// from the FP64-computed table.
// ---------------------------------------------------------------------------
template <typename F, int... I>
__device__ __forceinline__ void static_for_(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) { static_for_(f, std::make_integer_sequence<int, N>{}); }

template <typename T, int P>
__device__ __forceinline__ void fftp_reg(cx<T> *v, const cx<T> *__restrict__ tw, int tw_mul, bool inv) {
    static_for<ilog2(P)>([&](auto St) {
        constexpr int span = (P / 2) >> decltype(St)::value;
        static_for<P>([&](auto J) {
            constexpr int j = decltype(J)::value;
            if constexpr ((j & span) == 0) {
                const cx<T> a = v[j], b = v[j + span];
                v[j] = a + b;
                cx<T> d = a - b;
                constexpr int e = (j & (span - 1)) * ((P / 2) / span);
                if constexpr (e != 0) {
                    cx<T> w = tw[e * tw_mul];
                    if (inv) w.y = -w.y;
                    d = d * w;
                }
                v[j + span] = d;
            }
        });
    });
}

// L-point transform of a column held by Q lanes (lane half h = 0 .. Q-1 holds
// points h P .. h P + P - 1, P = L / Q, the lanes of one column CPB = 64 / Q
// apart): the first log2 Q decimation-in-frequency stages pair lanes h and
// h ^ (s / P) by shuffles (span s = L/2 .. P), the rest run in registers.
// Afterwards point i of lane h holds frequency brev_P(i) Q + brev_Q(h).
template <typename T, int L, int Q>
__device__ __forceinline__ void fft_lanes(cx<T> *v, int h, const cx<T> *__restrict__ tw, int Np, bool inv) {
    constexpr int P = L / Q, CPB = 64 / Q;
    static_for<ilog2(Q)>([&](auto St) {
        constexpr int s = (L / 2) >> decltype(St)::value;   // span in points, >= P
        constexpr int hs = s / P;                            // partner distance in lane halves
        const bool upper = (h & hs) != 0;
        static_for<P>([&](auto I) {
            constexpr int i = decltype(I)::value;
            cx<T> o;
            o.x = __shfl_xor(v[i].x, hs * CPB);
            o.y = __shfl_xor(v[i].y, hs * CPB);
            if (!upper) {
                v[i] = v[i] + o;
            } else {
                cx<T> d = o - v[i];
                const int e = ((h * P + i) & (s - 1)) * ((L / 2) / s);   // W_{2s}^{j mod s} = W_L^{...}
                if (e != 0) {
                    cx<T> w = tw[e * (Np / L)];
                    if (inv) w.y = -w.y;
                    d = d * w;
                }
                v[i] = d;
            }
        });
    });
    fftp_reg<T, P>(v, tw, Np / P, inv);
}

// Pass A in place: rows n2 + N2 n1 -> L = N1-point transforms over n1, times W_{N'}^{n2 k1}, rows n2 + N2 k1.
template <typename T, int L, int Q>
__global__ void __launch_bounds__(64) k_colpass_a_reg(cx<T> *__restrict__ grid, const cx<T> *__restrict__ tw, int N,
                                                      int logNp, int band_in, int inv) {
    constexpr int P = L / Q, CPB = 64 / Q;
    const int Np = 1 << logNp, N2 = Np / L;
    const int h = threadIdx.x / CPB, c = blockIdx.x * CPB + threadIdx.x % CPB, n2 = blockIdx.y;
    cx<T> v[P];
    static_for<P>([&](auto I) {
        const int r = n2 + N2 * (h * P + decltype(I)::value);
        v[I] = (!band_in || in_band(r, N, Np)) ? grid[(size_t)r * Np + c] : mk<T>((T)0, (T)0);
    });
    fft_lanes<T, L, Q>(v, h, tw, Np, inv != 0);
    const int hb = brev(h, ilog2(Q));
    static_for<P>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const int k1 = brev(i, ilog2(P)) * Q + hb;
        cx<T> w = tw[n2 * k1];
        if (inv) w.y = -w.y;
        grid[(size_t)(n2 + N2 * k1) * Np + c] = v[i] * w;
    });
}

// Pass B: rows L k1 + n2 (L = N2) -> L-point transforms over n2 -> rows k1 + N1 k2.
template <typename T, int L, int Q>
__global__ void __launch_bounds__(64) k_colpass_b_reg(const cx<T> *__restrict__ in, cx<T> *__restrict__ out,
                                                      const cx<T> *__restrict__ tw, int N, int logNp, int band_out,
                                                      int inv) {
    constexpr int P = L / Q, CPB = 64 / Q;
    const int Np = 1 << logNp, N1 = Np / L;
    const int h = threadIdx.x / CPB, c = blockIdx.x * CPB + threadIdx.x % CPB, k1 = blockIdx.y;
    cx<T> v[P];
    static_for<P>([&](auto I) { v[I] = in[(size_t)(L * k1 + h * P + decltype(I)::value) * Np + c]; });
    fft_lanes<T, L, Q>(v, h, tw, Np, inv != 0);
    const int hb = brev(h, ilog2(Q));
    static_for<P>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const int r = k1 + N1 * (brev(i, ilog2(P)) * Q + hb);
        if (!band_out || in_band(r, N, Np)) out[(size_t)r * Np + c] = v[i];
    });
}

template <typename T, int L>
constexpr int lanes_per_column() { return (L * (int)sizeof(cx<T>)) / 512 < 1 ? 1 : (L * (int)sizeof(cx<T>)) / 512; }

int threads_for(int L, int CW) { return L * CW / 16 < 64 ? 64 : L * CW / 16; }

template <typename T>
void colfft(ri_ctx *c, cx<T> *grid_io, cx<T> *grid_out, const cx<T> *tw, bool inv, bool band_in, bool band_out,
            hipStream_t s) {
    const int logNp = c->logNp, Np = c->Np;
    const int logN1 = (logNp + 1) / 2, logN2 = logNp / 2;
    if (logNp == 12 || logNp == 13) {
        // 4096 = 64 x 64 and 8192 = 128 x 64: both column passes in registers,
        // at most 64 complex FP32 (32 FP64) points per lane
        constexpr int QA4 = lanes_per_column<T, 64>(), QA8 = lanes_per_column<T, 128>();
        constexpr int QB = lanes_per_column<T, 64>();
        if (logNp == 12)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_colpass_a_reg<T, 64, QA4>), dim3(Np / (64 / QA4), 64), dim3(64), 0,
                               s, grid_io, tw, c->N, logNp, band_in ? 1 : 0, inv ? 1 : 0);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_colpass_a_reg<T, 128, QA8>), dim3(Np / (64 / QA8), 64), dim3(64), 0,
                               s, grid_io, tw, c->N, logNp, band_in ? 1 : 0, inv ? 1 : 0);
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_colpass_b_reg<T, 64, QB>), dim3(Np / (64 / QB), Np / 64), dim3(64), 0, s,
                           (const cx<T> *)grid_io, grid_out, tw, c->N, logNp, band_out ? 1 : 0, inv ? 1 : 0);
        return;
    }
    int logCW = sizeof(T) == 4 ? 6 : 5;
    if ((1 << logCW) > Np) logCW = logNp;
    const int CW = 1 << logCW;
    {
        const int L = 1 << logN1;
        dim3 grid(Np / CW, 1 << logN2);
        size_t lds = sizeof(cx<T>) * (size_t)L * CW;
        hipLaunchKernelGGL(k_colpass_a<T>, grid, dim3(threads_for(L, CW)), lds, s, grid_io, tw, c->N, logNp, logN1,
                           logN2, logCW, band_in ? 1 : 0, inv ? 1 : 0);
    }
    {
        const int L = 1 << logN2;
        dim3 grid(Np / CW, 1 << logN1);
        size_t lds = sizeof(cx<T>) * (size_t)L * CW;
        hipLaunchKernelGGL(k_colpass_b<T>, grid, dim3(threads_for(L, CW)), lds, s, grid_io, grid_out, tw, c->N,
                           logNp, logN1, logN2, logCW, band_out ? 1 : 0, inv ? 1 : 0);
    }
}

}  // namespace

// x (N x N) -> F Z_s x in p.gridB[s] for every w-stack s (row FFT into gridA band rows,
// columns A in place, B into gridB[s])
// Row transforms pad LDS by one element per 32 (fewer bank conflicts) when it fits.
template <typename T>
bool row_pad(ri_ctx *c) { return sizeof(cx<T>) * (size_t)(c->Np + c->Np / 32) <= (size_t)c->dev.lds_per_block; }

template <typename T>
size_t row_lds(ri_ctx *c) { return sizeof(cx<T>) * (size_t)(row_pad<T>(c) ? c->Np + c->Np / 32 : c->Np); }

template <typename T>
void fwd_zpad_fft(ri_ctx *c, Prec<T> &p, const T *x, hipStream_t s) {
    const int Np = c->Np;
    ProfScope prof(c, PROF_FFT, s);
    if (sizeof(cx<T>) * (size_t)Np > (size_t)c->dev.lds_per_block)
        throw Error(RI_EUNSUPPORTED, "grid row does not fit the workgroup LDS");
    // one FFT per w-stack (a single one without stacking); gridA is the scratch
    for (int st = 0; st < c->P; ++st) {
        const cx<T> *ch = c->P > 1 ? p.chirp + (size_t)st * c->N * c->N : nullptr;
        if (row_pad<T>(c))
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_zpad_rowfft<T, true>), dim3(c->N), dim3(threads_for(Np, 1)),
                               row_lds<T>(c), s, x, p.gridA, p.icorr, p.tw, c->N, c->logNp, ch);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_zpad_rowfft<T, false>), dim3(c->N), dim3(threads_for(Np, 1)),
                               row_lds<T>(c), s, x, p.gridA, p.icorr, p.tw, c->N, c->logNp, ch);
        colfft<T>(c, p.gridA, p.gridB + (size_t)st * Np * Np, p.tw, false, true, false, s);
    }
}

// p.gridA (Y_s = G_s^H r, one full grid per w-stack) -> Re sum_s Z_s^dagger F^dagger Y_s
// into x (N x N); gridA is clobbered and gridB[0] serves as the scratch.
template <typename T>
void adj_fft_crop(ri_ctx *c, Prec<T> &p, T *x, hipStream_t s) {
    const int Np = c->Np;
    ProfScope prof(c, PROF_FFT, s);
    for (int st = 0; st < c->P; ++st) {
        const cx<T> *ch = c->P > 1 ? p.chirp + (size_t)st * c->N * c->N : nullptr;
        colfft<T>(c, p.gridA + (size_t)st * Np * Np, p.gridB, p.tw, true, false, true, s);
        if (row_pad<T>(c))
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_irowfft_crop<T, true>), dim3(c->N), dim3(threads_for(Np, 1)),
                               row_lds<T>(c), s, p.gridB, x, p.icorr, p.tw, c->N, c->logNp, ch, st > 0 ? 1 : 0);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_irowfft_crop<T, false>), dim3(c->N), dim3(threads_for(Np, 1)),
                               row_lds<T>(c), s, p.gridB, x, p.icorr, p.tw, c->N, c->logNp, ch, st > 0 ? 1 : 0);
    }
}

template void fwd_zpad_fft<float>(ri_ctx *, Prec<float> &, const float *, hipStream_t);
template void fwd_zpad_fft<double>(ri_ctx *, Prec<double> &, const double *, hipStream_t);
template void adj_fft_crop<float>(ri_ctx *, Prec<float> &, float *, hipStream_t);
template void adj_fft_crop<double>(ri_ctx *, Prec<double> &, double *, hipStream_t);

}  // namespace ri
