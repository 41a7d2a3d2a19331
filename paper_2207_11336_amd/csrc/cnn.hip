// Residual CNN denoiser D(z) = z - net(z) (paper appendix C), forward and
// backward, on gfx950; facet-wise application (appendix D).
//
// Activations: bfloat16, NHWC with 64 channels (128 B per pixel).
// 64 -> 64 layers: implicit GEMM on v_mfma_f32_16x16x32_bf16. A persistent
// workgroup of four waves keeps the layer's packed weights in LDS and walks
// 32 x 16 pixel blocks; for each block it stages the 34 x 18 input patch in
// LDS (channel stride padded to 144 B) and every wave computes eight pixel
// rows for all 64 output channels: output channels are the MFMA rows (A =
// weights, pre-packed in lane order so each lane reads one 16-byte chunk),
// pixels the MFMA columns (B = the patch), K = 9 taps x 64 input channels in
// steps of 32; a patch row fragment serves the three row taps.
// Lane l holds A[l%16][8(l/16)..+7], B[8(l/16)..+7][l%16] and receives
// D[4(l/16)..+3][l%16], so the epilogue stores four consecutive channels of
// one pixel. The next block's patch is loaded into registers while the
// current one is computed. Blocks are dealt to XCDs in contiguous ranges so
// neighbouring blocks (which share halo rows) meet in the same L2.
// The same kernel computes the backward data pass with the weights flipped in
// space and transposed in channels, and a ReLU-mask epilogue.
// Weight gradients: MFMA with K = pixels; the output gradient and the input
// activations are staged transposed in LDS (the activations in three copies
// shifted by one column so every 16-byte read is aligned).
// First and last layers (1 -> 64, 64 -> 1) are FP32 VALU kernels; the last is
// fused with the residual subtraction.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "ri_internal.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace ri {

namespace {

constexpr int CH = 64;
constexpr int PADC = 72;                 // LDS channel stride of a pixel (144 B)
constexpr int WPK = 9 * 2 * 4 * 64;      // 16-byte chunks of one packed 64x64x3x3 layer
constexpr int PATCH_CHUNKS = 18 * 18 * 8;   // 16-byte chunks of an 18 x 18 x 64 patch
constexpr int DT_STRIDE = 256 + 8;       // LDS stride of one channel in the transposed gradient block
constexpr int AT_STRIDE = 18 * 16 + 8;   // LDS stride of one channel in a shifted activation copy
constexpr int N_XCD = 8;

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float bfround(float f) { return bf2f(f2bf(f)); }

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ int4 valid_rect(const CnnGeo &g, int b, int h, int w) {
    if (g.N == 0) return make_int4(0, h, 0, w);
    const int f = g.first + b, fy = f / g.nfx, fx = f - fy * g.nfx;
    const int oy = fy * g.core - g.halo, ox = fx * g.core - g.halo, ext = g.core + 2 * g.halo;
    return make_int4(max(0, -oy), min(min(h, ext), g.N - oy), max(0, -ox), min(min(w, ext), g.N - ox));
}

// Blocks of the persistent walk of workgroup `wg`: workgroups are dealt to the
// 8 XCDs round-robin, so XCD x = wg % 8 takes the contiguous range
// [x nb / 8, (x+1) nb / 8) and its nwg / 8 workgroups stride through it.
struct BlockWalk {
    int begin, end, step;
    __device__ BlockWalk(int wg, int nwg, int nb) {
        const int per = nwg / N_XCD;
        if (per == 0 || nwg % N_XCD) { begin = wg; end = nb; step = nwg; return; }
        const int x = wg % N_XCD;
        begin = (int)((int64_t)nb * x / N_XCD) + wg / N_XCD;
        end = (int)((int64_t)nb * (x + 1) / N_XCD);
        step = per;
    }
};

// ---------------------------------------------------------------------------
// Weight packing (FP32 master -> bfloat16 MFMA lane order)
//   fwd: chunk ((t*2 + kb)*4 + mi)*64 + lane, element e:
//        W[o = mi*16 + lane%16][c = kb*32 + 8(lane/16) + e][t]
//   bwd (flipped, transposed): W[o = kb*32 + 8(lane/16) + e][c = mi*16 + lane%16][8 - t]
// ---------------------------------------------------------------------------
__global__ void k_pack(const float *__restrict__ w, uint16_t *__restrict__ fwd, uint16_t *__restrict__ bwd) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= WPK * 8) return;
    const int e = idx & 7, chunk = idx >> 3;
    const int lane = chunk & 63, mi = (chunk >> 6) & 3, kb = (chunk >> 8) & 1, t = chunk >> 9;
    const int r = mi * 16 + (lane & 15), k = kb * 32 + 8 * (lane >> 4) + e;
    fwd[idx] = f2bf(w[(r * CH + k) * 9 + t]);
    bwd[idx] = f2bf(w[(k * CH + r) * 9 + (8 - t)]);
}

// Output-layer weights as a zero-padded 16-row MFMA A operand (rows = taps):
// chunk kb * 64 + lane, element e: bf16(W[0][c = 32 kb + 8(lane/16) + e][t = lane%16]), 0 for t >= 9.
__global__ void k_pack_proj(const float *__restrict__ w, uint16_t *__restrict__ proj) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 2 * 64 * 8) return;
    const int e = idx & 7, lane = (idx >> 3) & 63, kb = idx >> 9;
    const int t = lane & 15, c = kb * 32 + 8 * (lane >> 4) + e;
    proj[idx] = t < 9 ? f2bf(w[c * 9 + t]) : (uint16_t)0;
}

__device__ __forceinline__ void block_origin(int blk, int nbx, int nby, int rows, int &b, int &y0, int &x0) {
    b = blk / (nbx * nby);
    const int rem = blk - b * nbx * nby, by = rem / nbx;
    y0 = by * rows;
    x0 = (rem - by * nbx) * 16;
}

// 64 -> 64 convolution blocks: 32 rows x 16 columns, input patch 34 x 18.
constexpr int CB_ROWS = 32;
constexpr int CP_ROWS = CB_ROWS + 2, CP_COLS = 18;
constexpr int CP_CHUNKS = CP_ROWS * CP_COLS * 8;          // 16-byte chunks of the patch

// Buffer resource over one batch item's activations (bytes < 2^32): loads at
// an offset past the end return zeros and stores there are dropped, which is
// how patch halos outside the image and rows past H are handled without
// branches.
constexpr unsigned OOB = 0xFFFFFFF0u;
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t item_rsrc(const uint16_t *base, int H, int W) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)((unsigned)H * (unsigned)W * (CH * 2u)),
                                             0x00020000);
}
// Byte offset of channel c of pixel p (p < 2^25) in an item.
__device__ __forceinline__ unsigned px_off(int p, int c) { return (unsigned)p * (CH * 2u) + (unsigned)c * 2u; }

constexpr int CNW = 8;                                   // waves per workgroup (2 per SIMD)
constexpr int CNT = 64 * CNW;                             // threads per workgroup
constexpr int CRW = CB_ROWS / CNW;                        // block rows per wave
constexpr int CPRE8 = (CP_CHUNKS + CNT - 1) / CNT;        // patch chunks per thread

__device__ __forceinline__ void conv_patch_fetch(uint4 (&pre)[CPRE8], const uint16_t *__restrict__ in, int blk,
                                                 int nbx, int nby, int H, int W, int tid) {
    int b, y0, x0;
    block_origin(blk, nbx, nby, CB_ROWS, b, y0, x0);
    const __amdgpu_buffer_rsrc_t rs = item_rsrc(in + (size_t)b * H * W * CH, H, W);
#pragma unroll
    for (int k = 0; k < CPRE8; ++k) {
        const int e = tid + k * CNT;
        const int pix = e >> 3, ch = e & 7;
        const int py = pix / CP_COLS, px = pix - py * CP_COLS;
        const int y = y0 - 1 + py, x = x0 - 1 + px;
        const bool ok = e < CP_CHUNKS && (unsigned)y < (unsigned)H && (unsigned)x < (unsigned)W;
        const unsigned off = ok ? px_off(y * W + x, ch * 8) : OOB;
        pre[k] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
    }
}

// Scheduling hint for a K step of NMF MFMAs that also loads NRD fragments of
// the next step: alternate MFMA and LDS read, then the remaining MFMAs.
template <int NRD, int NMF>
__device__ __forceinline__ void sched_interleave() {
#pragma unroll
    for (int k = 0; k < NRD; ++k) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS read
    }
    if constexpr (NMF - NRD > 0) __builtin_amdgcn_sched_group_barrier(0x008, NMF - NRD, 0);
}

// ---------------------------------------------------------------------------
// 64 -> 64 convolution, persistent. MODE 0: out = relu(conv + bias), zero
// outside the batch item's valid rectangle. MODE 1 (backward data): out =
// conv * [mask_act > 0] (mask_act: the post-ReLU activation the gradient
// flows into). MODE 2: as MODE 0, but the activations are projected onto the
// nine taps of the 64 -> 1 output layer instead of being stored.
// Eight waves (two per SIMD); blocks of 32 x 16 pixels (nbx x nby per item,
// the last block row may reach past H); wave w computes block rows
// 4w..4w+3 for all 64 output channels: 4 x 4 accumulator tiles (initialised
// with the bias). The K loop runs as 18 steps (dx, kb, dy): the six patch
// rows of a (dx, kb) pair are loaded once and serve the three row taps, and
// each step's fragments are loaded while the previous step's MFMAs run. The
// results go through LDS (the patch area, swizzled) so that every lane
// stores 16 contiguous bytes and a wave writes whole pixel rows.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ void __launch_bounds__(CNT) k_conv64(const uint16_t *__restrict__ in, uint16_t *__restrict__ out,
                                                const uint4 *__restrict__ wpk, const float *__restrict__ bias,
                                                const uint16_t *__restrict__ mask_act, CnnGeo geo, int H, int W,
                                                int nbx, int nby, int nblocks, const uint4 *__restrict__ wproj,
                                                float *__restrict__ S, int64_t plane) {
    extern __shared__ uint4 smem4[];
    uint16_t *patch = reinterpret_cast<uint16_t *>(smem4);                 // [34*18][PADC]
    uint4 *wl = smem4 + (CP_ROWS * CP_COLS * PADC * 2) / 16;                // [WPK]
    float *bs = reinterpret_cast<float *>(wl + WPK);                        // [64]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, j = lane & 15;
    for (int e = tid; e < WPK; e += CNT) wl[e] = wpk[e];
    if (tid < CH) bs[tid] = MODE != 1 ? bias[tid] : 0.f;
    const BlockWalk walk(blockIdx.x, gridDim.x, nblocks);
    uint4 pre[CPRE8];
    if (walk.begin < walk.end) conv_patch_fetch(pre, in, walk.begin, nbx, nby, H, W, tid);
    for (int blk = walk.begin; blk < walk.end; blk += walk.step) {
        __syncthreads();   // the previous block's patch and staging reads are done
#pragma unroll
        for (int k = 0; k < CPRE8; ++k) {
            const int e = tid + k * CNT;
            if (e < CP_CHUNKS) *reinterpret_cast<uint4 *>(patch + (e >> 3) * PADC + (e & 7) * 8) = pre[k];
        }
        __syncthreads();
        if (blk + walk.step < walk.end) conv_patch_fetch(pre, in, blk + walk.step, nbx, nby, H, W, tid);
        floatx4 acc[4][CRW];
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) {
            const float4 bb = *reinterpret_cast<const float4 *>(bs + mi * 16 + 4 * g);
#pragma unroll
            for (int ni = 0; ni < CRW; ++ni) acc[mi][ni] = floatx4{bb.x, bb.y, bb.z, bb.w};
        }
        const uint16_t *pw = patch + (wave * CRW * CP_COLS + j) * PADC + 8 * g;
        bf16x8 bcur[CRW + 2], bnext[CRW + 2], acur[4], anext[4];
#pragma unroll
        for (int r = 0; r < CRW + 2; ++r) bcur[r] = as_bf16x8(*reinterpret_cast<const uint4 *>(pw + r * CP_COLS * PADC));
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) acur[mi] = as_bf16x8(wl[mi * 64 + lane]);
#pragma unroll
        for (int st = 0; st < 18; ++st) {            // st = (2 dx + kb) * 3 + dy, tap t = 3 dy + dx
            const int dy = st % 3;
            if (st + 1 < 18) {
                const int grp1 = (st + 1) / 3, dy1 = (st + 1) % 3, dx1 = grp1 / 2, kb1 = grp1 % 2;
                const int t1 = dy1 * 3 + dx1;
#pragma unroll
                for (int mi = 0; mi < 4; ++mi) anext[mi] = as_bf16x8(wl[((t1 * 2 + kb1) * 4 + mi) * 64 + lane]);
                if (dy == 2) {
#pragma unroll
                    for (int r = 0; r < CRW + 2; ++r)
                        bnext[r] = as_bf16x8(
                            *reinterpret_cast<const uint4 *>(pw + (r * CP_COLS + dx1) * PADC + kb1 * 32));
                }
            }
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < CRW; ++ni)
                    acc[mi][ni] =
                        __builtin_amdgcn_mfma_f32_16x16x32_bf16(acur[mi], bcur[ni + dy], acc[mi][ni], 0, 0, 0);
            if (st + 1 < 18) {
                if (dy == 2) sched_interleave<4 + CRW + 2, 4 * CRW>();
                else sched_interleave<4, 4 * CRW>();
            }
#pragma unroll
            for (int mi = 0; mi < 4; ++mi) acur[mi] = anext[mi];
            if (dy == 2) {
#pragma unroll
                for (int r = 0; r < CRW + 2; ++r) bcur[r] = bnext[r];
            }
        }
        int b, y0, x0;
        block_origin(blk, nbx, nby, CB_ROWS, b, y0, x0);
        const size_t img = (size_t)b * H * W * CH;
        bool all_in = true, x_in = true;
        int4 vr = make_int4(0, H, 0, W);
        if (MODE != 1 && geo.N != 0) {
            vr = valid_rect(geo, b, H, W);
            x_in = x0 + j >= vr.z && x0 + j < vr.w;
            all_in = y0 >= vr.x && y0 + CB_ROWS <= vr.y && x0 >= vr.z && x0 + 16 <= vr.w;
        }
        __amdgpu_buffer_rsrc_t ms;
        if (MODE == 1) ms = item_rsrc(mask_act + img, H, W);
        // bf16 results: pk[ni][mi] = channels 16 mi + 4 g .. +3 of pixel (row ni, column j)
        uint2 pk[CRW][4];
#pragma unroll
        for (int ni = 0; ni < CRW; ++ni) {
            const int y = y0 + wave * CRW + ni;
            const bool inside = all_in || (x_in && y >= vr.x && y < vr.y);
#pragma unroll
            for (int mi = 0; mi < 4; ++mi) {
                float v[4];
                if (MODE != 1) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] = inside ? fmaxf(acc[mi][ni][r], 0.f) : 0.f;
                } else {
                    // the gradient flows where the post-ReLU activation is > 0
                    const unsigned off = y < H ? px_off(y * W + x0 + j, mi * 16 + 4 * g) : OOB;
                    const uint2 mv = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(ms, off, 0, 0));
                    const int16_t m4[4] = {(int16_t)(mv.x & 0xFFFFu), (int16_t)(mv.x >> 16),
                                           (int16_t)(mv.y & 0xFFFFu), (int16_t)(mv.y >> 16)};
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] = m4[r] > 0 ? acc[mi][ni][r] : 0.f;
                }
                const bf16x2 lo = {(__bf16)v[0], (__bf16)v[1]}, hi = {(__bf16)v[2], (__bf16)v[3]};
                pk[ni][mi] = make_uint2(__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi));
            }
        }
        if (MODE == 2) {
            // last hidden layer: project the block's activations onto the nine
            // taps of the 64 -> 1 output layer, s_t[p] = sum_c W[c][t] act[p][c]
            // (MFMA rows t < 9 of a zero-padded 16-row A), instead of storing
            // them. The activations go through LDS (the patch area, swizzled by
            // pixel) to reach the MFMA operand layout.
            __syncthreads();   // every wave is done with the patch
            uint16_t *stg = patch + wave * (CRW * 16 * 64);                // [CRW rows][16 px][64 ch]
#pragma unroll
            for (int ni = 0; ni < CRW; ++ni)
#pragma unroll
                for (int mi = 0; mi < 4; ++mi) {
                    const int q = (2 * mi + (g >> 1)) ^ (j & 7);
                    *reinterpret_cast<uint2 *>(stg + (ni * 16 + j) * 64 + q * 8 + (g & 1) * 4) = pk[ni][mi];
                }
            __builtin_amdgcn_wave_barrier();   // the wave reads back what its other lanes staged
            const bf16x8 ap0 = as_bf16x8(wproj[lane]), ap1 = as_bf16x8(wproj[64 + lane]);
#pragma unroll
            for (int ni = 0; ni < CRW; ++ni) {
                const int y = y0 + wave * CRW + ni;
                const uint16_t *sp = stg + (ni * 16 + j) * 64;
                const bf16x8 b0 = as_bf16x8(*reinterpret_cast<const uint4 *>(sp + ((g ^ (j & 7)) * 8)));
                const bf16x8 b1 = as_bf16x8(*reinterpret_cast<const uint4 *>(sp + (((4 + g) ^ (j & 7)) * 8)));
                floatx4 pr = floatx4{0.f, 0.f, 0.f, 0.f};
                pr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap0, b0, pr, 0, 0, 0);
                pr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap1, b1, pr, 0, 0, 0);
                if (y < H) {
                    float *sq = S + (size_t)b * H * W + (size_t)y * W + x0 + j;
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (4 * g + r < 9) sq[(size_t)(4 * g + r) * plane] = pr[r];
                }
            }
            continue;
        }
        // Direct 16-byte stores: lane rows g and g ^ 1 (lanes l and l ^ 16)
        // exchange halves with v_permlane16_swap so that a lane holds eight
        // consecutive channels. For the tile pair (mi, mi + 1): even rows keep
        // tile mi (their 4 channels + the odd row's 4), odd rows take tile
        // mi + 1; a lane then owns 16-byte chunk 2 (mi + (g & 1)) + (g >> 1).
        const __amdgpu_buffer_rsrc_t os = item_rsrc(out + img, H, W);
#pragma unroll
        for (int ni = 0; ni < CRW; ++ni) {
            const int y = y0 + wave * CRW + ni;
#pragma unroll
            for (int mp = 0; mp < 4; mp += 2) {
                uint2 a = pk[ni][mp], c = pk[ni][mp + 1];
                const auto sx = __builtin_amdgcn_permlane16_swap(a.x, c.x, false, false);
                const auto sy = __builtin_amdgcn_permlane16_swap(a.y, c.y, false, false);
                const u32x4 v = {sx[0], sy[0], sx[1], sy[1]};
                const int q = 2 * (mp + (g & 1)) + (g >> 1);
                const unsigned off = y < H ? px_off(y * W + x0 + j, q * 8) : OOB;
                __builtin_amdgcn_raw_buffer_store_b128(v, os, off, 0, 0);
            }
        }
    }
}

// First layer: FP32 input, FP32 weights W0[64][9], bias; relu, valid mask,
// bfloat16 out. A 16 x 16 block in eight passes of 32 pixels; thread t
// computes channels 8 (t % 8) .. +7 of one pixel, so a wave stores eight
// whole pixels (1 KB contiguous). Tangent mode (mask_act != NULL, b0 NULL):
// out = [mask_act > 0] (W0 * z), the layer's Jacobian applied to z.
__global__ void __launch_bounds__(256) k_conv_in(const float *__restrict__ z, uint16_t *__restrict__ out,
                                                 const float *__restrict__ w0, const float *__restrict__ b0,
                                                 CnnGeo geo, int H, int W, const uint16_t *__restrict__ mask_act) {
    __shared__ float zp[18][18];
    __shared__ float ws[9][CH];
    __shared__ float bs[CH];
    const int b = blockIdx.z, y0 = blockIdx.y * 16, x0 = blockIdx.x * 16, tid = threadIdx.x;
    const size_t img = (size_t)b * H * W;
    for (int e = tid; e < 18 * 18; e += 256) {
        const int py = e / 18, px = e - py * 18, y = y0 - 1 + py, x = x0 - 1 + px;
        zp[py][px] = (y >= 0 && y < H && x >= 0 && x < W) ? z[img + (size_t)y * W + x] : 0.f;
    }
    for (int e = tid; e < CH * 9; e += 256) ws[e % 9][e / 9] = w0[e];
    if (tid < CH) bs[tid] = b0 ? b0[tid] : 0.f;
    __syncthreads();
    const int4 vr = valid_rect(geo, b, H, W);
    const int q = tid & 7;
    float wr[9][8], br[8];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int e = 0; e < 8; ++e) wr[t][e] = ws[t][8 * q + e];
#pragma unroll
    for (int e = 0; e < 8; ++e) br[e] = bs[8 * q + e];
#pragma unroll 2
    for (int pass = 0; pass < 8; ++pass) {
        const int p = pass * 32 + (tid >> 3), ty = p >> 4, tx = p & 15, y = y0 + ty, x = x0 + tx;
        const bool inside = y >= vr.x && y < vr.y && x >= vr.z && x < vr.w;
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = br[e];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const float zz = zp[ty + t / 3][tx + t % 3];
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] += wr[t][e] * zz;
        }
        uint32_t o[4];
        if (mask_act) {
            const uint4 mv = *reinterpret_cast<const uint4 *>(mask_act + (img + (size_t)y * W + x) * CH + 8 * q);
            const uint32_t mu[4] = {mv.x, mv.y, mv.z, mv.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bf16x2 pr = {(__bf16)((int16_t)(mu[e] & 0xFFFFu) > 0 ? v[2 * e] : 0.f),
                                   (__bf16)((int16_t)(mu[e] >> 16) > 0 ? v[2 * e + 1] : 0.f)};
                o[e] = __builtin_bit_cast(uint32_t, pr);
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bf16x2 pr = {(__bf16)(inside ? fmaxf(v[2 * e], 0.f) : 0.f),
                                   (__bf16)(inside ? fmaxf(v[2 * e + 1], 0.f) : 0.f)};
                o[e] = __builtin_bit_cast(uint32_t, pr);
            }
        }
        *reinterpret_cast<uint4 *>(out + (img + (size_t)y * W + x) * CH + 8 * q) = make_uint4(o[0], o[1], o[2], o[3]);
    }
}

__device__ __forceinline__ void load_patch_lds(uint16_t *patch, const uint16_t *__restrict__ act, size_t img, int y0,
                                               int x0, int H, int W, int tid) {
    for (int e = tid; e < PATCH_CHUNKS; e += 256) {
        const int pix = e >> 3, ch = e & 7, py = pix / 18, px = pix - py * 18;
        const int y = y0 - 1 + py, x = x0 - 1 + px;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (y >= 0 && y < H && x >= 0 && x < W)
            v = reinterpret_cast<const uint4 *>(act + (img + (size_t)y * W + x) * CH)[ch];
        *reinterpret_cast<uint4 *>(patch + pix * PADC + ch * 8) = v;
    }
}

// Last layer + residual: D = z - (b + sum_{t,c} bf16(W[0][c][t]) act[p + t - centre][c]) in FP32;
// z == NULL and bl == NULL give the layer without bias or residual (its
// Jacobian). FLIP: the transposed first layer, D[p] = sum_{t,c} W0[c][t]
// act[p - (t - centre)][c] with FP32 weights (the input gradient).
template <bool FLIP>
__global__ void __launch_bounds__(256) k_conv_out(const uint16_t *__restrict__ act, const float *__restrict__ z,
                                                  float *__restrict__ D, const float *__restrict__ wl_,
                                                  const float *__restrict__ bl, int H, int W) {
    extern __shared__ uint4 smem4[];
    uint16_t *patch = reinterpret_cast<uint16_t *>(smem4);          // [18*18][PADC]
    float *ws = reinterpret_cast<float *>(patch + 18 * 18 * PADC);  // [9][64]
    const int b = blockIdx.z, y0 = blockIdx.y * 16, x0 = blockIdx.x * 16, tid = threadIdx.x;
    const size_t img = (size_t)b * H * W;
    load_patch_lds(patch, act, img, y0, x0, H, W, tid);
    for (int e = tid; e < CH * 9; e += 256) {
        const int c = e / 9, t = e - c * 9;
        ws[t * CH + c] = FLIP ? wl_[e] : bfround(wl_[e]);
    }
    __syncthreads();
    const int ty = tid >> 4, tx = tid & 15;
    float acc = (!FLIP && bl) ? bl[0] : 0.f;
    for (int t = 0; t < 9; ++t) {
        const int oy = FLIP ? 2 - t / 3 : t / 3, ox = FLIP ? 2 - t % 3 : t % 3;
        const uint16_t *pp = patch + ((ty + oy) * 18 + tx + ox) * PADC;
        const float *wt = ws + t * CH;
#pragma unroll
        for (int c8 = 0; c8 < CH; c8 += 8) {
            const uint4 v = *reinterpret_cast<const uint4 *>(pp + c8);
            const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                acc += wt[c8 + 2 * q] * __uint_as_float(u[q] << 16);
                acc += wt[c8 + 2 * q + 1] * __uint_as_float(u[q] & 0xFFFF0000u);
            }
        }
    }
    const size_t o = img + (size_t)(y0 + ty) * W + x0 + tx;
    D[o] = (!FLIP && z) ? z[o] - acc : acc;
}

// Output layer from the tap projections: D = z - (b + sum_t s_t[p + (t - centre)]).
__global__ void k_conv_sum(const float *__restrict__ S, const float *__restrict__ z, float *__restrict__ D,
                           const float *__restrict__ bl, int B, int H, int W) {
    const int64_t plane = (int64_t)B * H * W;
    const float b0 = bl[0];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < plane; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t item = i / ((int64_t)H * W);
        const int r = (int)(i - item * H * W), y = r / W, x = r - y * W;
        float acc = b0;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
            if (yy >= 0 && yy < H && xx >= 0 && xx < W) acc += S[t * plane + item * H * W + (int64_t)yy * W + xx];
        }
        D[i] = z[i] - acc;
    }
}

// l1 loss gradient with respect to net(z): g = -sign(D - u) / numel; partials of mean|D - u|.
__global__ void k_l1(const float *__restrict__ D, const float *__restrict__ u, float *__restrict__ g, int64_t n,
                     double *part) {
    __shared__ double s_red[4];
    double acc = 0.0;
    const float inv = 1.f / (float)n;
    const double invd = 1.0 / (double)n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float d = D[i] - u[i];
        g[i] = d > 0.f ? -inv : (d < 0.f ? inv : 0.f);
        acc += fabs((double)d) * invd;
    }
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
}

// Backward of the last layer. dpre[p][c] = [mask[p][c] > 0] sum_t bf16(W[0][c][t]) g[p - (t - centre)]
// with mask = mask_act if given, else act;
// this block's share of dW[c][t] = sum_p act[p + (t - centre)][c] g[p] and db = sum_p g[p] goes to
// row `block` of part (577 floats), summed over blocks by k_reduce_rows.
__global__ void __launch_bounds__(256) k_out_backward(const float *__restrict__ g, const uint16_t *__restrict__ act,
                                                      const float *__restrict__ wl_, uint16_t *__restrict__ dpre,
                                                      float *__restrict__ part, int H, int W,
                                                      const uint16_t *__restrict__ mask_act) {
    extern __shared__ uint4 smem4[];
    uint16_t *patch = reinterpret_cast<uint16_t *>(smem4);          // act patch [18*18][PADC]
    float *gp = reinterpret_cast<float *>(patch + 18 * 18 * PADC);  // g patch [18][18]
    float *ws = gp + 18 * 18;                                       // [64][9]
    float *red = ws + CH * 9;                                       // [4]
    const int b = blockIdx.z, y0 = blockIdx.y * 16, x0 = blockIdx.x * 16, tid = threadIdx.x;
    const size_t img = (size_t)b * H * W;
    float *prow = part + ((size_t)(blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * (CH * 9 + 1);
    load_patch_lds(patch, act, img, y0, x0, H, W, tid);
    for (int e = tid; e < 18 * 18; e += 256) {
        const int py = e / 18, px = e - py * 18, y = y0 - 1 + py, x = x0 - 1 + px;
        gp[e] = (y >= 0 && y < H && x >= 0 && x < W) ? g[img + (size_t)y * W + x] : 0.f;
    }
    for (int e = tid; e < CH * 9; e += 256) ws[e] = bfround(wl_[e]);
    __syncthreads();
    const int ty = tid >> 4, tx = tid & 15;
    float gg[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) gg[t] = gp[(ty + 2 - t / 3) * 18 + tx + 2 - t % 3];
    // the ReLU mask comes from mask_act (the activations at z) when the layer
    // input act is a tangent, else from act itself
    const uint16_t *ac = mask_act ? mask_act + (img + (size_t)(y0 + ty) * W + x0 + tx) * CH
                                  : patch + ((ty + 1) * 18 + tx + 1) * PADC;
    uint16_t *dst = dpre + (img + (size_t)(y0 + ty) * W + x0 + tx) * CH;
    for (int c8 = 0; c8 < CH; c8 += 8) {
        uint32_t o[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            float v = 0.f;
#pragma unroll
            for (int t = 0; t < 9; ++t) v += ws[(c8 + e) * 9 + t] * gg[t];
            o[e] = (int16_t)ac[c8 + e] > 0 ? f2bf(v) : 0u;
        }
        *reinterpret_cast<uint4 *>(dst + c8) =
            make_uint4(o[0] | (o[1] << 16), o[2] | (o[3] << 16), o[4] | (o[5] << 16), o[6] | (o[7] << 16));
    }
    for (int pr = tid; pr < CH * 9; pr += 256) {
        const int c = pr / 9, t = pr - c * 9, dy = t / 3, dx = t % 3;
        float s = 0.f;
        for (int py = 0; py < 16; ++py)
            for (int px = 0; px < 16; ++px)
                s += bf2f(patch[((py + dy) * 18 + px + dx) * PADC + c]) * gp[(py + 1) * 18 + px + 1];
        prow[pr] = s;
    }
    float sg = gp[(ty + 1) * 18 + tx + 1];
    for (int o = 32; o >= 1; o >>= 1) sg += __shfl_xor(sg, o);
    if ((tid & 63) == 0) red[tid >> 6] = sg;
    __syncthreads();
    if (tid == 0) prow[CH * 9] = red[0] + red[1] + red[2] + red[3];
}

// Weight and bias gradients of a 64 -> 64 layer:
//   dW[o][c][t] += sum_p dpre[p][o] act[p + (t - centre)][c],  db[o] += sum_p dpre[p][o].
// A workgroup walks 16x16 pixel blocks and accumulates all 9 x 64 x 64
// outputs in MFMA accumulators (wave w: output channels 16w..16w+15).
constexpr int DW_PART = 9 * 4 * 4 * 256 + 64;    // per-workgroup partials: accumulators + bias sums

__global__ void __launch_bounds__(256) k_dw64(const uint16_t *__restrict__ dpre, const uint16_t *__restrict__ act,
                                              float *__restrict__ part, int H, int W, int nbx, int nby, int nblocks) {
    extern __shared__ uint4 smem4[];
    uint16_t *dT = reinterpret_cast<uint16_t *>(smem4);   // [64][DT_STRIDE]   dpre transposed
    uint16_t *aT = dT + CH * DT_STRIDE;                   // [3][64][AT_STRIDE] act transposed, shifted by dx
    float *red = reinterpret_cast<float *>(aT + 3 * CH * AT_STRIDE);   // [256]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, j = lane & 15;
    floatx4 acc[9][4];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[t][n] = floatx4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    const BlockWalk walk(blockIdx.x, gridDim.x, nblocks);
    for (int blk = walk.begin; blk < walk.end; blk += walk.step) {
        int b, y0, x0;
        block_origin(blk, nbx, nby, 16, b, y0, x0);
        const size_t img = (size_t)b * H * W;
        __syncthreads();
        for (int e = tid; e < 256 * 8; e += 256) {
            const int pix = e >> 3, ch = e & 7;
            const uint4 v = reinterpret_cast<const uint4 *>(
                dpre + (img + (size_t)(y0 + (pix >> 4)) * W + x0 + (pix & 15)) * CH)[ch];
            const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                dT[(ch * 8 + 2 * q) * DT_STRIDE + pix] = (uint16_t)(u[q] & 0xFFFFu);
                dT[(ch * 8 + 2 * q + 1) * DT_STRIDE + pix] = (uint16_t)(u[q] >> 16);
            }
        }
        for (int e = tid; e < PATCH_CHUNKS; e += 256) {
            const int pix = e >> 3, ch = e & 7, py = pix / 18, px = pix - py * 18;
            const int y = y0 - 1 + py, x = x0 - 1 + px;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (y >= 0 && y < H && x >= 0 && x < W)
                v = reinterpret_cast<const uint4 *>(act + (img + (size_t)y * W + x) * CH)[ch];
            const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int cc = px - dx;
                if (cc < 0 || cc >= 16) continue;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    aT[(dx * CH + ch * 8 + 2 * q) * AT_STRIDE + py * 16 + cc] = (uint16_t)(u[q] & 0xFFFFu);
                    aT[(dx * CH + ch * 8 + 2 * q + 1) * AT_STRIDE + py * 16 + cc] = (uint16_t)(u[q] >> 16);
                }
            }
        }
        __syncthreads();
        {
            const int o = tid & 63, q0 = (tid >> 6) * 64;
            for (int p = q0; p < q0 + 64; ++p) bsum += bf2f(dT[o * DT_STRIDE + p]);
        }
        for (int ks = 0; ks < 8; ++ks) {
            const int pr = 2 * ks;
            const bf16x8 a =
                as_bf16x8(*reinterpret_cast<const uint4 *>(dT + (wave * 16 + j) * DT_STRIDE + pr * 16 + 8 * g));
            const int row = pr + (g >> 1), col = 8 * (g & 1);
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int dy = t / 3, dx = t - dy * 3;
#pragma unroll
                for (int n = 0; n < 4; ++n) {
                    const bf16x8 bv = as_bf16x8(*reinterpret_cast<const uint4 *>(
                        aT + (dx * CH + n * 16 + j) * AT_STRIDE + (row + dy) * 16 + col));
                    acc[t][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv, acc[t][n], 0, 0, 0);
                }
            }
        }
    }
    // this workgroup's partial sums, in accumulator order (coalesced; reduced by k_dw64_reduce)
    float *pp = part + (size_t)blockIdx.x * DW_PART;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) pp[((t * 4 + n) * 4 + r) * 256 + tid] = acc[t][n][r];
    red[tid] = bsum;
    __syncthreads();
    if (tid < CH) pp[9 * 4 * 4 * 256 + tid] = red[tid] + red[tid + 64] + red[tid + 128] + red[tid + 192];
}

// dW[o][c][t] and db[o] from the per-workgroup partials of k_dw64, in a fixed order.
__global__ void k_dw64_reduce(const float *__restrict__ part, int nwg, float *__restrict__ dW, float *__restrict__ db) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 9 * 4 * 4 * 256 + CH) return;
    float s8[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};      // eight independent loads in flight
    int w = 0;
    for (; w + 8 <= nwg; w += 8)
#pragma unroll
        for (int k = 0; k < 8; ++k) s8[k] += part[(size_t)(w + k) * DW_PART + e];
    for (; w < nwg; ++w) s8[0] += part[(size_t)w * DW_PART + e];
    const float s = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
    if (e < 9 * 4 * 4 * 256) {
        const int tid = e & 255, r = (e >> 8) & 3, n = (e >> 10) & 3, t = e >> 12;
        const int wave = tid >> 6, lane = tid & 63, o = wave * 16 + 4 * (lane >> 4) + r, c = n * 16 + (lane & 15);
        dW[(o * CH + c) * 9 + t] = s;
    } else {
        db[e - 9 * 4 * 4 * 256] = s;
    }
}

// Weight and bias gradients of the first layer, this block's share: dW0[c][t] = sum_p z[p + (t - centre)]
// dpre[p][c] and db0[c] = sum_p dpre[p][c] into row `block` of part (640 floats, parameter order).
__global__ void __launch_bounds__(256) k_dw_in(const float *__restrict__ z, const uint16_t *__restrict__ dpre,
                                               float *__restrict__ part, int H, int W) {
    __shared__ float zp[18][18];
    __shared__ uint16_t dp[256][CH + 2];
    const int b = blockIdx.z, y0 = blockIdx.y * 16, x0 = blockIdx.x * 16, tid = threadIdx.x;
    const size_t img = (size_t)b * H * W;
    for (int e = tid; e < 18 * 18; e += 256) {
        const int py = e / 18, px = e - py * 18, y = y0 - 1 + py, x = x0 - 1 + px;
        zp[py][px] = (y >= 0 && y < H && x >= 0 && x < W) ? z[img + (size_t)y * W + x] : 0.f;
    }
    for (int e = tid; e < 256 * CH; e += 256) {
        const int pix = e >> 6, c = e & 63;
        dp[pix][c] = dpre[(img + (size_t)(y0 + (pix >> 4)) * W + x0 + (pix & 15)) * CH + c];
    }
    __syncthreads();
    for (int pr = tid; pr < CH * 9 + CH; pr += 256) {
        float s = 0.f;
        if (pr < CH * 9) {
            const int c = pr / 9, t = pr - c * 9, dy = t / 3, dx = t % 3;
            for (int p = 0; p < 256; ++p) s += zp[(p >> 4) + dy][(p & 15) + dx] * bf2f(dp[p][c]);
        } else {
            const int c = pr - CH * 9;
            for (int p = 0; p < 256; ++p) s += bf2f(dp[p][c]);
        }
        part[((size_t)(blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * (CH * 9 + CH) + pr] = s;
    }
}

// out[e] = sum over rows r < nrows of part[r * stride + e], e < count (fixed order).
__global__ void k_reduce_rows(const float *__restrict__ part, int nrows, int stride, int count, float *__restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    float s8[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int r = 0;
    for (; r + 8 <= nrows; r += 8)
#pragma unroll
        for (int k = 0; k < 8; ++k) s8[k] += part[(size_t)(r + k) * stride + e];
    for (; r < nrows; ++r) s8[0] += part[(size_t)r * stride + e];
    out[e] = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
}

// Adam (beta1 0.9, beta2 0.999, eps 1e-8) with the bias corrections
// c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t) from the host (FP64). The
// weights 1 - beta are written as their own FP32 constants: 1.f - 0.999f
// would carry the rounding of 0.999f (1.3e-5 of the result) into every
// second-moment update.
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ gr, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float c1, float c2) {
    const float b1 = 0.9f, omb1 = 0.1f, b2 = 0.999f, omb2 = 0.001f, eps = 1e-8f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = gr[i];
        const float mi = b1 * m[i] + omb1 * gi;
        const float vi = b2 * v[i] + omb2 * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    }
}

// Counter-based standard normals: splitmix64 of (seed, index), Box-Muller.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ float normal_at(uint64_t seed, uint64_t i) {
    const uint64_t r = mix64(seed * 0xD1B54A32D192ED03ull + i);
    const float u1 = ((float)(r >> 40) + 0.5f) * (1.0f / 16777216.0f);
    const float u2 = (float)((r >> 16) & 0xFFFFFFull) * (1.0f / 16777216.0f);
    return sqrtf(-2.f * logf(u1)) * cospif(2.f * u2);
}

__global__ void k_noisy(const float *__restrict__ clean, float *__restrict__ noisy, int64_t n, float sigma,
                        uint64_t seed) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        noisy[i] = clean[i] + sigma * normal_at(seed, (uint64_t)i);
}

// Seeded standard normal vector (the start of the FNE power iteration).
__global__ void k_normal(float *__restrict__ v, int64_t n, uint64_t seed) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = normal_at(seed, (uint64_t)i);
}

// Training batch from a resident pool of patches: item b is patch
// p = (d >> 3) mod n_pool in orientation d & 7 (bit 0: transpose, bit 1: rows
// reversed, bit 2: columns reversed; the eight symmetries of the square),
// d = mix64 of (seed, b). Training images have no preferred orientation.
__global__ void k_sample_batch(const float *__restrict__ pool, int64_t n_pool, int side, int batch, uint64_t seed,
                               float *__restrict__ out) {
    const int64_t per = (int64_t)side * side, n = per * batch;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(i / per);
        const int r = (int)(i - (int64_t)b * per), y = r / side, x = r - y * side;
        const uint64_t d = mix64(seed * 0x9E6C63D0676A9A99ull + (uint64_t)b);
        const int64_t p = (int64_t)((d >> 3) % (uint64_t)n_pool);
        int sy = y, sx = x;
        if (d & 1) { const int t = sy; sy = sx; sx = t; }
        if (d & 2) sy = side - 1 - sy;
        if (d & 4) sx = side - 1 - sx;
        out[i] = pool[p * per + (int64_t)sy * side + sx];
    }
}

// out = rho_b clean + (1 - rho_b) D over item b of a batch (per_item pixels
// each), rho_b uniform in [0, 1) from mix64 of (seed, b): the points between
// the clean images and their denoised noisy versions where the relaxed
// firm-nonexpansiveness penalty evaluates the Jacobian.
__global__ void k_mix(const float *__restrict__ clean, const float *__restrict__ D, float *__restrict__ out,
                      int64_t n, int64_t per_item, uint64_t seed) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t b = (uint64_t)(i / per_item);
        const float rho = (float)(mix64(seed * 0xA24BAED4963EE407ull + b) >> 40) * (1.0f / 16777216.0f);
        out[i] = rho * clean[i] + (1.f - rho) * D[i];
    }
}

// out = a - 2 t (the map I - 2 J_net applied through its Jacobian product t).
__global__ void k_minus2(const float *__restrict__ a, const float *__restrict__ t, float *__restrict__ out,
                         int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a[i] - 2.f * t[i];
}

// grads[i] += coef grads2[i] over [0, n) with coef = -4 lambda when the
// squared Jacobian norm ss[0] exceeds 1 - eps, else 0 (the gradient of
// lambda max(||J_{2D - I}||^2, 1 - eps) through u^T J_net v, u the unnormalised
// image of the unit v).
__global__ void k_fne_combine(float *__restrict__ grads, const float *__restrict__ grads2, int64_t n,
                              const double *__restrict__ ss, float lambda, float eps) {
    const float coef = ss[0] > 1.0 - (double)eps ? -4.f * lambda : 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        grads[i] += coef * grads2[i];
}

// v /= sqrt(ss[0]) (FP64 squared norm from the reduction).
__global__ void k_scale_rsqrt(float *__restrict__ v, int64_t n, const double *__restrict__ ss) {
    const float k = (float)(1.0 / sqrt(ss[0]));
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] *= k;
}

__global__ void k_init_params(float *p, const int64_t *offs, const float *stds, int nl, int64_t total, uint64_t seed) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        int l = 0;
        while (l + 1 < 2 * nl && i >= offs[l + 1]) ++l;
        p[i] = (l & 1) ? 0.f : stds[l >> 1] * normal_at(seed, (uint64_t)i);   // odd segments: biases
    }
}

// Facet tiles: z_tile[b][ty][tx] = z[oy + ty][ox + tx] inside the valid
// rectangle, 0 elsewhere.
template <typename T>
__global__ void k_facet_extract(const T *__restrict__ z, float *__restrict__ zt, CnnGeo geo, int B, int h, int w) {
    const int64_t n = (int64_t)B * h * w;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(i / ((int64_t)h * w)), r = (int)(i - (int64_t)b * h * w), ty = r / w, tx = r - ty * w;
        const int4 vr = valid_rect(geo, b, h, w);
        const int f = geo.first + b, fy = f / geo.nfx, fx = f - fy * geo.nfx;
        float v = 0.f;
        if (ty >= vr.x && ty < vr.y && tx >= vr.z && tx < vr.w)
            v = (float)z[(size_t)(fy * geo.core - geo.halo + ty) * geo.N + (fx * geo.core - geo.halo + tx)];
        zt[i] = v;
    }
}

// out[y][x] = D_tile[b][halo + cy][halo + cx] for the core pixels of each facet.
template <typename T>
__global__ void k_facet_insert(const float *__restrict__ Dt, T *__restrict__ out, CnnGeo geo, int B, int h, int w) {
    const int64_t cc = (int64_t)geo.core * geo.core;
    const int64_t n = (int64_t)B * cc;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(i / cc), r = (int)(i - (int64_t)b * cc), cy = r / geo.core, cx = r - cy * geo.core;
        const int f = geo.first + b, fy = f / geo.nfx, fx = f - fy * geo.nfx;
        const int y = fy * geo.core + cy, x = fx * geo.core + cx;
        if (y < geo.N && x < geo.N)
            out[(size_t)y * geo.N + x] = (T)Dt[((size_t)b * h + geo.halo + cy) * w + geo.halo + cx];
    }
}

inline int gridn(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

}  // namespace

}  // namespace ri

using namespace ri;

struct ri_cnn {
    int L = 10, maxB = 0, maxH = 0, maxW = 0, training = 0, n_cu = 256;
    int64_t P = 0;
    std::vector<int64_t> off;          // [2L+1]: weight, bias offsets of each layer
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
    uint16_t *wfwd = nullptr, *wbwd = nullptr;   // packed hidden layers [L-2][WPK*8]
    uint16_t *wproj = nullptr;         // output layer as an MFMA operand [2][64][8]
    float *S = nullptr;                // inference: tap projections of the last hidden layer [9][pixels]
    std::vector<uint16_t *> act;       // training: L-1 activation buffers; inference: 2
    uint16_t *dpre[2] = {nullptr, nullptr};
    float *D = nullptr, *g = nullptr, *zin = nullptr;
    float *dwpart = nullptr;           // training: per-workgroup weight-gradient partials
    float *blkpart = nullptr;          // training: per-block partials of the first / last layer
    double *part = nullptr;
    double *scal = nullptr;            // FP64 scalars of the Jacobian-norm iteration
    std::vector<uint16_t *> tan;       // tangents of the layers (allocated on first use)
    float *grads2 = nullptr;           // parameter gradient of u^T J_net v
    float *fv = nullptr;               // power-iteration vector of the penalised training
    bool fv_ready = false;
    int64_t step = 0;
    std::string err;
    std::vector<void *> allocs;
};

namespace {

void *cnn_alloc(ri_cnn *n, size_t bytes) {
    void *p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess) {
        (void)hipGetLastError();
        throw Error(RI_ENOMEM, "hipMalloc failed for the CNN (" + std::to_string(bytes) + " B)");
    }
    n->allocs.push_back(p);
    return p;
}

size_t conv64_lds() { return (size_t)CP_ROWS * CP_COLS * PADC * 2 + (size_t)WPK * 16 + CH * 4; }
size_t convout_lds() { return (size_t)18 * 18 * PADC * 2 + 9 * CH * 4; }
size_t outbwd_lds() { return (size_t)18 * 18 * PADC * 2 + 18 * 18 * 4 + CH * 9 * 4 + 16; }
size_t dw64_lds() { return ((size_t)CH * DT_STRIDE + 3 * CH * AT_STRIDE) * 2 + 256 * 4; }

void check_shape(const ri_cnn *n, int B, int h, int w) {
    if (B < 1 || h < 16 || w < 16 || h % 16 || w % 16 || h > n->maxH || w > n->maxW || B > n->maxB)
        throw Error(RI_EINVAL, "batch/size outside the network's buffers or not multiples of 16");
}

void repack(ri_cnn *n, hipStream_t s) {
    for (int l = 1; l <= n->L - 2; ++l)
        hipLaunchKernelGGL(k_pack, dim3((WPK * 8 + 255) / 256), dim3(256), 0, s, n->params + n->off[2 * l],
                           n->wfwd + (size_t)(l - 1) * WPK * 8, n->wbwd + (size_t)(l - 1) * WPK * 8);
    hipLaunchKernelGGL(k_pack_proj, dim3(4), dim3(256), 0, s, n->params + n->off[2 * (n->L - 1)], n->wproj);
}

int persistent_grid(const ri_cnn *n, int nblocks) {
    const int g = std::min(nblocks, n->n_cu);
    return g >= N_XCD ? g - g % N_XCD : g;
}

// Forward through all layers. Training: hidden activations into act[0..L-2],
// then the output layer reads act[L-2]. Inference: ping-pong act[0], act[1];
// the last hidden layer is not stored but projected onto the output layer's
// nine taps inside its kernel, and a stencil pass forms D.
void forward(ri_cnn *n, const float *z, float *D, int B, int h, int w, const CnnGeo &geo, hipStream_t s) {
    dim3 grid(w / 16, h / 16, B);
    const int L = n->L, nbx = w / 16, nby = (h + CB_ROWS - 1) / CB_ROWS, nb = nbx * nby * B;
    const int64_t plane = (int64_t)B * h * w;
    auto A = [&](int l) { return n->training ? n->act[l] : n->act[l & 1]; };
    hipLaunchKernelGGL(k_conv_in, grid, dim3(256), 0, s, z, A(0), n->params + n->off[0], n->params + n->off[1], geo,
                       h, w, (const uint16_t *)nullptr);
    for (int l = 1; l <= L - 2; ++l) {
        const uint4 *wl = reinterpret_cast<const uint4 *>(n->wfwd + (size_t)(l - 1) * WPK * 8);
        if (n->training || l < L - 2)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_conv64<0>), dim3(persistent_grid(n, nb)), dim3(CNT), conv64_lds(), s,
                               A(l - 1), A(l), wl, n->params + n->off[2 * l + 1], (const uint16_t *)nullptr, geo, h,
                               w, nbx, nby, nb, (const uint4 *)nullptr, (float *)nullptr, plane);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_conv64<2>), dim3(persistent_grid(n, nb)), dim3(CNT), conv64_lds(), s,
                               A(l - 1), (uint16_t *)nullptr, wl, n->params + n->off[2 * l + 1],
                               (const uint16_t *)nullptr, geo, h, w, nbx, nby, nb,
                               reinterpret_cast<const uint4 *>(n->wproj), n->S, plane);
    }
    if (n->training)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_conv_out<false>), grid, dim3(256), convout_lds(), s, A(L - 2), z, D,
                           n->params + n->off[2 * (L - 1)], n->params + n->off[2 * (L - 1) + 1], h, w);
    else
        hipLaunchKernelGGL(k_conv_sum, dim3(std::min<int64_t>((plane + 255) / 256, 8192)), dim3(256), 0, s, n->S, z,
                           D, n->params + n->off[2 * (L - 1) + 1], B, h, w);
    RI_CHECK_HIP(hipGetLastError());
}

// Parameter gradients of sum(g * f) into grads (zeroed here), where f is the
// network (ins = the activations of forward(), zin = z) or its linearisation
// at z applied to a tangent (ins = the tangents of jvp_store(), zin = the
// tangent v): the same passes, the layer inputs taken from ins while the ReLU
// masks stay those of the activations at z.
void backward_core(ri_cnn *n, const float *zin, const float *g, const std::vector<uint16_t *> &ins, float *grads,
                   int B, int h, int w, hipStream_t s) {
    const int L = n->L;
    dim3 grid(w / 16, h / 16, B);
    fill_real<float>(grads, n->P, 0.f, s);
    const int nblk16 = (w / 16) * (h / 16) * B;
    hipLaunchKernelGGL(k_out_backward, grid, dim3(256), outbwd_lds(), s, g, ins[L - 2],
                       n->params + n->off[2 * (L - 1)], n->dpre[0], n->blkpart, h, w, n->act[L - 2]);
    hipLaunchKernelGGL(k_reduce_rows, dim3((CH * 9 + 1 + 255) / 256), dim3(256), 0, s, n->blkpart, nblk16, CH * 9 + 1,
                       CH * 9 + 1, grads + n->off[2 * (L - 1)]);
    int cur = 0;
    const int nbx = w / 16, nby = h / 16, nb = nbx * nby * B;                  // 16 x 16 blocks (weight gradients)
    const int cby = (h + CB_ROWS - 1) / CB_ROWS, cnb = nbx * cby * B;         // 32 x 16 blocks (convolutions)
    const CnnGeo full;
    for (int l = L - 2; l >= 1; --l) {
        const int nwg = persistent_grid(n, nb);
        hipLaunchKernelGGL(k_dw64, dim3(nwg), dim3(256), dw64_lds(), s, n->dpre[cur], ins[l - 1], n->dwpart, h, w,
                           nbx, nby, nb);
        hipLaunchKernelGGL(k_dw64_reduce, dim3((9 * 4 * 4 * 256 + CH + 255) / 256), dim3(256), 0, s, n->dwpart, nwg,
                           grads + n->off[2 * l], grads + n->off[2 * l + 1]);
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_conv64<1>), dim3(persistent_grid(n, cnb)), dim3(CNT), conv64_lds(), s,
                           n->dpre[cur], n->dpre[cur ^ 1],
                           reinterpret_cast<const uint4 *>(n->wbwd + (size_t)(l - 1) * WPK * 8),
                           (const float *)nullptr, n->act[l - 1], full, h, w, nbx, cby, cnb, (const uint4 *)nullptr,
                           (float *)nullptr, (int64_t)0);
        cur ^= 1;
    }
    hipLaunchKernelGGL(k_dw_in, grid, dim3(256), 0, s, zin, n->dpre[cur], n->blkpart, h, w);
    hipLaunchKernelGGL(k_reduce_rows, dim3((CH * 9 + CH + 255) / 256), dim3(256), 0, s, n->blkpart, nblk16,
                       CH * 9 + CH, CH * 9 + CH, grads + n->off[0]);
    RI_CHECK_HIP(hipGetLastError());
}

// Gradients of sum(g * net(z)) into n->grads; activations from forward().
void backward(ri_cnn *n, const float *z, const float *g, int B, int h, int w, hipStream_t s) {
    backward_core(n, z, g, n->act, n->grads, B, h, w, s);
}

// J_net(z) v into out, with the activations of forward(z) (training mode):
// tangents through the first layer (masked, no bias), the hidden layers
// (MODE 1 with the forward weights: conv * [activation > 0]) and the output
// layer without bias or residual. Tangent activations in bfloat16.
void jvp(ri_cnn *n, const float *v, float *out, int B, int h, int w, hipStream_t s) {
    const int L = n->L;
    dim3 grid(w / 16, h / 16, B);
    const int nbx = w / 16, cby = (h + CB_ROWS - 1) / CB_ROWS, cnb = nbx * cby * B;
    const CnnGeo full;
    hipLaunchKernelGGL(k_conv_in, grid, dim3(256), 0, s, v, n->dpre[0], n->params + n->off[0], (const float *)nullptr,
                       full, h, w, n->act[0]);
    int cur = 0;
    for (int l = 1; l <= L - 2; ++l) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_conv64<1>), dim3(persistent_grid(n, cnb)), dim3(CNT), conv64_lds(), s,
                           n->dpre[cur], n->dpre[cur ^ 1],
                           reinterpret_cast<const uint4 *>(n->wfwd + (size_t)(l - 1) * WPK * 8),
                           (const float *)nullptr, n->act[l], full, h, w, nbx, cby, cnb, (const uint4 *)nullptr,
                           (float *)nullptr, (int64_t)0);
        cur ^= 1;
    }
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_conv_out<false>), grid, dim3(256), convout_lds(), s, n->dpre[cur],
                       (const float *)nullptr, out, n->params + n->off[2 * (L - 1)], (const float *)nullptr, h, w);
    RI_CHECK_HIP(hipGetLastError());
}

void ensure_tangent(ri_cnn *n) {
    if (!n->tan.empty()) return;
    const size_t npix = (size_t)n->maxB * n->maxH * n->maxW;
    for (int l = 0; l < n->L - 1; ++l) n->tan.push_back((uint16_t *)cnn_alloc(n, sizeof(uint16_t) * npix * CH));
    n->grads2 = (float *)cnn_alloc(n, sizeof(float) * n->P);
    n->fv = (float *)cnn_alloc(n, sizeof(float) * npix);
}

// jvp() keeping every layer's tangent in n->tan (the layer inputs of the
// tangent backward pass).
void jvp_store(ri_cnn *n, const float *v, float *out, int B, int h, int w, hipStream_t s) {
    const int L = n->L;
    dim3 grid(w / 16, h / 16, B);
    const int nbx = w / 16, cby = (h + CB_ROWS - 1) / CB_ROWS, cnb = nbx * cby * B;
    const CnnGeo full;
    hipLaunchKernelGGL(k_conv_in, grid, dim3(256), 0, s, v, n->tan[0], n->params + n->off[0], (const float *)nullptr,
                       full, h, w, n->act[0]);
    for (int l = 1; l <= L - 2; ++l)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_conv64<1>), dim3(persistent_grid(n, cnb)), dim3(CNT), conv64_lds(), s,
                           n->tan[l - 1], n->tan[l],
                           reinterpret_cast<const uint4 *>(n->wfwd + (size_t)(l - 1) * WPK * 8),
                           (const float *)nullptr, n->act[l], full, h, w, nbx, cby, cnb, (const uint4 *)nullptr,
                           (float *)nullptr, (int64_t)0);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_conv_out<false>), grid, dim3(256), convout_lds(), s, n->tan[L - 2],
                       (const float *)nullptr, out, n->params + n->off[2 * (L - 1)], (const float *)nullptr, h, w);
    RI_CHECK_HIP(hipGetLastError());
}

// Parameter gradient of u^T J_net(z) v into n->grads2 (weights; the bias
// entries, which the shared passes fill with sums of the adjoints, are
// cleared: the Jacobian does not depend on the biases). Needs forward(z).
void jvp_grad(ri_cnn *n, const float *v, const float *u, float *tscratch, int B, int h, int w, hipStream_t s) {
    ensure_tangent(n);
    jvp_store(n, v, tscratch, B, h, w, s);
    backward_core(n, v, u, n->tan, n->grads2, B, h, w, s);
    for (int l = 0; l < n->L; ++l)
        fill_real<float>(n->grads2 + n->off[2 * l + 1], n->off[2 * l + 2] - n->off[2 * l + 1], 0.f, s);
}

// J_net(z)^T u into out: the backward data pass of backward() without the
// weight gradients, then the transposed first layer (FP32 weights).
void vjp(ri_cnn *n, const float *u, float *out, int B, int h, int w, hipStream_t s) {
    const int L = n->L;
    dim3 grid(w / 16, h / 16, B);
    const int nbx = w / 16, cby = (h + CB_ROWS - 1) / CB_ROWS, cnb = nbx * cby * B;
    const CnnGeo full;
    hipLaunchKernelGGL(k_out_backward, grid, dim3(256), outbwd_lds(), s, u, n->act[L - 2],
                       n->params + n->off[2 * (L - 1)], n->dpre[0], n->blkpart, h, w, n->act[L - 2]);
    int cur = 0;
    for (int l = L - 2; l >= 1; --l) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_conv64<1>), dim3(persistent_grid(n, cnb)), dim3(CNT), conv64_lds(), s,
                           n->dpre[cur], n->dpre[cur ^ 1],
                           reinterpret_cast<const uint4 *>(n->wbwd + (size_t)(l - 1) * WPK * 8),
                           (const float *)nullptr, n->act[l - 1], full, h, w, nbx, cby, cnb, (const uint4 *)nullptr,
                           (float *)nullptr, (int64_t)0);
        cur ^= 1;
    }
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_conv_out<true>), grid, dim3(256), convout_lds(), s, n->dpre[cur],
                       (const float *)nullptr, out, n->params + n->off[0], (const float *)nullptr, h, w);
    RI_CHECK_HIP(hipGetLastError());
}

template <typename F>
ri_status cnn_guard(const ri_cnn *n, F &&fn) {
    try {
        fn();
        return RI_OK;
    } catch (const Error &e) {
        if (n) const_cast<ri_cnn *>(n)->err = e.msg;
        return e.code;
    } catch (const std::exception &e) {
        if (n) const_cast<ri_cnn *>(n)->err = e.what();
        return RI_EDEVICE;
    }
}

thread_local std::string g_cnn_err;

void offsets_for(int L, std::vector<int64_t> &off, std::vector<float> *stds) {
    off.assign(2 * L + 1, 0);
    if (stds) stds->resize(L);
    for (int l = 0; l < L; ++l) {
        const int ci = l == 0 ? 1 : CH, co = l == L - 1 ? 1 : CH;
        off[2 * l + 1] = off[2 * l] + (int64_t)co * ci * 9;
        off[2 * l + 2] = off[2 * l + 1] + co;
        if (stds) (*stds)[l] = std::sqrt(2.0f / (9.0f * ci));
    }
}

ri_cnn *create(const ri_cnn_desc &d, uint64_t seed) {
    if (d.layers < 3 || d.layers > 64 || d.channels != CH || d.max_batch < 1 || d.max_h < 16 || d.max_w < 16 ||
        d.max_h % 16 || d.max_w % 16 || (int64_t)d.max_h * d.max_w > (int64_t)4096 * 4096)
        throw Error(RI_EINVAL, "CNN: 3 <= layers <= 64, channels == 64, sides multiples of 16, "
                               "at most 4096 x 4096 pixels per image");
    int dev = 0;
    RI_CHECK_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    RI_CHECK_HIP(hipGetDeviceProperties(&prop, dev));
    const size_t need = std::max(conv64_lds(), dw64_lds());
    if (need > (size_t)prop.sharedMemPerBlock)
        throw Error(RI_EUNSUPPORTED, "CNN kernels need " + std::to_string(need) +
                                         " B of LDS per workgroup; the device allows " +
                                         std::to_string(prop.sharedMemPerBlock));
    ri_cnn *n = new ri_cnn();
    try {
        n->n_cu = prop.multiProcessorCount;
        n->L = d.layers; n->maxB = d.max_batch; n->maxH = d.max_h; n->maxW = d.max_w; n->training = d.training;
        std::vector<float> stds;
        offsets_for(n->L, n->off, &stds);
        n->P = n->off[2 * n->L];
        n->params = (float *)cnn_alloc(n, sizeof(float) * n->P);
        n->wfwd = (uint16_t *)cnn_alloc(n, sizeof(uint16_t) * (size_t)(n->L - 2) * WPK * 8);
        n->wbwd = (uint16_t *)cnn_alloc(n, sizeof(uint16_t) * (size_t)(n->L - 2) * WPK * 8);
        n->wproj = (uint16_t *)cnn_alloc(n, sizeof(uint16_t) * 2 * 64 * 8);
        const size_t npix = (size_t)n->maxB * n->maxH * n->maxW;
        const int nact = n->training ? n->L - 1 : 2;
        for (int i = 0; i < nact; ++i) n->act.push_back((uint16_t *)cnn_alloc(n, sizeof(uint16_t) * npix * CH));
        n->D = (float *)cnn_alloc(n, sizeof(float) * npix);
        n->zin = (float *)cnn_alloc(n, sizeof(float) * npix);
        n->part = (double *)cnn_alloc(n, sizeof(double) * 1024);
        n->scal = (double *)cnn_alloc(n, sizeof(double) * 16);
        if (!n->training) n->S = (float *)cnn_alloc(n, sizeof(float) * 9 * npix);
        if (n->training) {
            n->grads = (float *)cnn_alloc(n, sizeof(float) * n->P);
            n->dwpart = (float *)cnn_alloc(n, sizeof(float) * (size_t)DW_PART * n->n_cu);
            n->blkpart = (float *)cnn_alloc(n, sizeof(float) * (npix / 256) * (CH * 9 + CH));
            n->dpre[0] = (uint16_t *)cnn_alloc(n, sizeof(uint16_t) * npix * CH);
            n->dpre[1] = (uint16_t *)cnn_alloc(n, sizeof(uint16_t) * npix * CH);
            n->g = (float *)cnn_alloc(n, sizeof(float) * npix);
            n->m = (float *)cnn_alloc(n, sizeof(float) * n->P);
            n->v = (float *)cnn_alloc(n, sizeof(float) * n->P);
            fill_real<float>(n->m, n->P, 0.f, nullptr);
            fill_real<float>(n->v, n->P, 0.f, nullptr);
        }
        int64_t *doffs = (int64_t *)cnn_alloc(n, sizeof(int64_t) * n->off.size());
        float *dstd = (float *)cnn_alloc(n, sizeof(float) * n->L);
        RI_CHECK_HIP(hipMemcpy(doffs, n->off.data(), sizeof(int64_t) * n->off.size(), hipMemcpyHostToDevice));
        RI_CHECK_HIP(hipMemcpy(dstd, stds.data(), sizeof(float) * n->L, hipMemcpyHostToDevice));
        hipLaunchKernelGGL(k_init_params, dim3(gridn(n->P)), dim3(256), 0, nullptr, n->params, doffs, dstd, n->L, n->P,
                           seed);
        repack(n, nullptr);
        RI_CHECK_HIP(hipGetLastError());
        RI_CHECK_HIP(hipDeviceSynchronize());
    } catch (...) {
        ri::cnn_destroy(n);
        throw;
    }
    return n;
}

}  // namespace

namespace ri {

ri_cnn *cnn_create_inference(int layers, int max_batch, int side) {
    ri_cnn_desc d{};
    d.layers = layers;
    d.channels = CH;
    d.max_batch = max_batch;
    d.max_h = side;
    d.max_w = side;
    d.training = 0;
    return create(d, 0);
}

void cnn_destroy(ri_cnn *n) {
    if (!n) return;
    (void)hipDeviceSynchronize();
    for (void *p : n->allocs) (void)hipFree(p);
    delete n;
}

int64_t cnn_param_count_for(int layers) {
    std::vector<int64_t> off;
    offsets_for(layers, off, nullptr);
    return off.back();
}

int cnn_layers(const ri_cnn *n) { return n->L; }

void cnn_load_params(ri_cnn *n, const float *params, hipStream_t s) {
    RI_CHECK_HIP(hipMemcpyAsync(n->params, params, sizeof(float) * n->P, hipMemcpyDeviceToDevice, s));
    repack(n, s);
    RI_CHECK_HIP(hipGetLastError());
}

int cnn_tile_side(int N, int core, int halo) {
    const bool whole = core <= 0 || core >= N;
    return ((whole ? N : core + 2 * halo) + 15) / 16 * 16;
}

template <typename T>
void cnn_denoise(ri_cnn *n, const T *z, T *out, int N, int core, int halo, hipStream_t s) {
    const bool whole = core <= 0 || core >= N;
    CnnGeo geo;
    geo.N = N;
    geo.core = whole ? N : core;
    geo.halo = whole ? 0 : halo;
    geo.nfx = (N + geo.core - 1) / geo.core;
    const int side = cnn_tile_side(N, core, halo);
    const int nf = geo.nfx * geo.nfx;
    if (side > n->maxH || side > n->maxW) throw Error(RI_EINVAL, "facet tile larger than the network's buffers");
    const int per = std::min(nf, n->maxB);
    for (int f0 = 0; f0 < nf; f0 += per) {
        const int B = std::min(per, nf - f0);
        geo.first = f0;
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_facet_extract<T>), dim3(gridn((int64_t)B * side * side)), dim3(256), 0,
                           s, z, n->zin, geo, B, side, side);
        forward(n, n->zin, n->D, B, side, side, geo, s);
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_facet_insert<T>), dim3(gridn((int64_t)B * geo.core * geo.core)),
                           dim3(256), 0, s, n->D, out, geo, B, side, side);
    }
    RI_CHECK_HIP(hipGetLastError());
}
template void cnn_denoise<float>(ri_cnn *, const float *, float *, int, int, int, hipStream_t);
template void cnn_denoise<double>(ri_cnn *, const double *, double *, int, int, int, hipStream_t);

}  // namespace ri

extern "C" {

ri_status ri_cnn_create(const ri_cnn_desc *d, uint64_t seed, ri_cnn **out) {
    if (!out || !d) {
        g_cnn_err = "desc or out is NULL";
        return RI_EINVAL;
    }
    *out = nullptr;
    try {
        *out = create(*d, seed);
        return RI_OK;
    } catch (const Error &e) {
        g_cnn_err = e.msg;
        return e.code;
    } catch (const std::exception &e) {
        g_cnn_err = e.what();
        return RI_EDEVICE;
    }
}

void ri_cnn_destroy(ri_cnn *n) { ri::cnn_destroy(n); }

const char *ri_cnn_last_error(const ri_cnn *n) { return n ? n->err.c_str() : g_cnn_err.c_str(); }

int64_t ri_cnn_param_count(const ri_cnn *n) { return n ? n->P : 0; }

ri_status ri_cnn_set_params(ri_cnn *n, const float *params, ri_stream stream) {
    if (!n || !params) return RI_EINVAL;
    return cnn_guard(n, [&] { cnn_load_params(n, params, reinterpret_cast<hipStream_t>(stream)); });
}

ri_status ri_cnn_get_params(const ri_cnn *n, float *params, ri_stream stream) {
    if (!n || !params) return RI_EINVAL;
    return cnn_guard(n, [&] {
        RI_CHECK_HIP(hipMemcpyAsync(params, n->params, sizeof(float) * n->P, hipMemcpyDeviceToDevice,
                                    reinterpret_cast<hipStream_t>(stream)));
    });
}

ri_status ri_cnn_forward(ri_cnn *n, const float *z, float *out, int32_t B, int32_t h, int32_t w, ri_stream stream) {
    if (!n || !z || !out) return RI_EINVAL;
    return cnn_guard(n, [&] {
        check_shape(n, B, h, w);
        forward(n, z, out, B, h, w, CnnGeo(), reinterpret_cast<hipStream_t>(stream));
    });
}

ri_status ri_cnn_grad(ri_cnn *n, const float *z, const float *g, int32_t B, int32_t h, int32_t w, float *grads,
                      ri_stream stream) {
    if (!n || !z || !g || !grads) return RI_EINVAL;
    return cnn_guard(n, [&] {
        if (!n->training) throw Error(RI_EINVAL, "network created without training buffers");
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        check_shape(n, B, h, w);
        forward(n, z, n->D, B, h, w, CnnGeo(), s);
        backward(n, z, g, B, h, w, s);
        RI_CHECK_HIP(hipMemcpyAsync(grads, n->grads, sizeof(float) * n->P, hipMemcpyDeviceToDevice, s));
    });
}

ri_status ri_cnn_sample_batch(ri_cnn *n, const float *pool, int64_t n_pool, int32_t side, int32_t batch,
                              uint64_t seed, float *out, ri_stream stream) {
    if (!n || !pool || !out) return RI_EINVAL;
    return cnn_guard(n, [&] {
        if (n_pool < 1 || side < 1 || batch < 1) throw Error(RI_EINVAL, "n_pool, side and batch must be >= 1");
        const int64_t total = (int64_t)batch * side * side;
        hipLaunchKernelGGL(k_sample_batch, dim3(gridn(total)), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                           pool, n_pool, (int)side, (int)batch, seed, out);
        RI_CHECK_HIP(hipGetLastError());
    });
}

ri_status ri_cnn_train_step(ri_cnn *n, const float *clean, int32_t B, int32_t h, int32_t w, float sigma,
                            uint64_t seed, float lr, double *loss, ri_stream stream) {
    if (!n || !clean) return RI_EINVAL;
    return cnn_guard(n, [&] {
        if (!n->training) throw Error(RI_EINVAL, "network created without training buffers");
        if (!(sigma >= 0.f) || !(lr > 0.f)) throw Error(RI_EINVAL, "sigma >= 0 and lr > 0 required");
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        check_shape(n, B, h, w);
        const int64_t npix = (int64_t)B * h * w;
        hipLaunchKernelGGL(k_noisy, dim3(gridn(npix)), dim3(256), 0, s, clean, n->zin, npix, sigma, seed);
        forward(n, n->zin, n->D, B, h, w, CnnGeo(), s);
        hipLaunchKernelGGL(k_l1, dim3(1024), dim3(256), 0, s, n->D, clean, n->g, npix, n->part);
        if (loss) reduce_partials(n->part, 1024, 1, 1, loss, s);
        backward(n, n->zin, n->g, B, h, w, s);
        n->step++;
        const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)n->step)));
        const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)n->step)));
        hipLaunchKernelGGL(k_adam, dim3(gridn(n->P)), dim3(256), 0, s, n->params, n->grads, n->m, n->v, n->P, lr, c1,
                           c2);
        repack(n, s);
        RI_CHECK_HIP(hipGetLastError());
    });
}

ri_status ri_cnn_jvp(ri_cnn *n, const float *z, const float *v, float *out, int32_t B, int32_t h, int32_t w,
                     ri_stream stream) {
    if (!n || !z || !v || !out) return RI_EINVAL;
    return cnn_guard(n, [&] {
        if (!n->training) throw Error(RI_EINVAL, "network created without training buffers");
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        check_shape(n, B, h, w);
        forward(n, z, n->D, B, h, w, CnnGeo(), s);
        jvp(n, v, out, B, h, w, s);
    });
}

ri_status ri_cnn_vjp(ri_cnn *n, const float *z, const float *u, float *out, int32_t B, int32_t h, int32_t w,
                     ri_stream stream) {
    if (!n || !z || !u || !out) return RI_EINVAL;
    return cnn_guard(n, [&] {
        if (!n->training) throw Error(RI_EINVAL, "network created without training buffers");
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        check_shape(n, B, h, w);
        forward(n, z, n->D, B, h, w, CnnGeo(), s);
        vjp(n, u, out, B, h, w, s);
    });
}

ri_status ri_cnn_fne_norm(ri_cnn *n, const float *z, int32_t B, int32_t h, int32_t w, int32_t iters, uint64_t seed,
                          double *norm_out, ri_stream stream) {
    if (!n || !z || !norm_out) return RI_EINVAL;
    return cnn_guard(n, [&] {
        if (!n->training) throw Error(RI_EINVAL, "network created without training buffers");
        if (iters < 1) throw Error(RI_EINVAL, "iters must be >= 1");
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        check_shape(n, B, h, w);
        const int64_t np = (int64_t)B * h * w;
        forward(n, z, n->D, B, h, w, CnnGeo(), s);
        float *v = n->zin, *t = n->D, *a = n->g;
        hipLaunchKernelGGL(k_normal, dim3(gridn(np)), dim3(256), 0, s, v, np, seed);
        dot_partials<float>(v, v, np, n->part, s);
        reduce_partials(n->part, 1024, 1, 1, n->scal, s);
        hipLaunchKernelGGL(k_scale_rsqrt, dim3(gridn(np)), dim3(256), 0, s, v, np, n->scal);
        for (int it = 0; it < iters; ++it) {
            jvp(n, v, t, B, h, w, s);                                                   // t = J_net v
            hipLaunchKernelGGL(k_minus2, dim3(gridn(np)), dim3(256), 0, s, v, t, a, np);   // a = (I - 2 J_net) v
            dot_partials<float>(a, a, np, n->part, s);
            reduce_partials(n->part, 1024, 1, 1, n->scal + 1, s);                       // ||a||^2, v unit
            vjp(n, a, t, B, h, w, s);                                                   // t = J_net^T a
            hipLaunchKernelGGL(k_minus2, dim3(gridn(np)), dim3(256), 0, s, a, t, v, np);   // v = (I - 2 J_net)^T a
            dot_partials<float>(v, v, np, n->part, s);
            reduce_partials(n->part, 1024, 1, 1, n->scal, s);
            hipLaunchKernelGGL(k_scale_rsqrt, dim3(gridn(np)), dim3(256), 0, s, v, np, n->scal);
        }
        double ss = 0.0;
        RI_CHECK_HIP(hipMemcpyAsync(&ss, n->scal + 1, sizeof(double), hipMemcpyDeviceToHost, s));
        RI_CHECK_HIP(hipStreamSynchronize(s));
        *norm_out = std::sqrt(ss);
    });
}

ri_status ri_cnn_jvp_grad(ri_cnn *n, const float *z, const float *v, const float *u, int32_t B, int32_t h, int32_t w,
                          float *grads, ri_stream stream) {
    if (!n || !z || !v || !u || !grads) return RI_EINVAL;
    return cnn_guard(n, [&] {
        if (!n->training) throw Error(RI_EINVAL, "network created without training buffers");
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        check_shape(n, B, h, w);
        forward(n, z, n->D, B, h, w, CnnGeo(), s);
        jvp_grad(n, v, u, n->D, B, h, w, s);
        RI_CHECK_HIP(hipMemcpyAsync(grads, n->grads2, sizeof(float) * n->P, hipMemcpyDeviceToDevice, s));
    });
}

ri_status ri_cnn_train_step_fne(ri_cnn *n, const float *clean, int32_t B, int32_t h, int32_t w, float sigma,
                                uint64_t seed, float lr, float lambda, float eps, int32_t power_iters, int32_t point,
                                double *loss, double *fne_sq, ri_stream stream) {
    if (!n || !clean) return RI_EINVAL;
    return cnn_guard(n, [&] {
        if (!n->training) throw Error(RI_EINVAL, "network created without training buffers");
        if (!(sigma >= 0.f) || !(lr > 0.f) || !(lambda >= 0.f) || !(eps >= 0.f && eps < 1.f) || power_iters < 0)
            throw Error(RI_EINVAL, "sigma >= 0, lr > 0, lambda >= 0, 0 <= eps < 1, power_iters >= 0 required");
        if (point != RI_FNE_AT_INPUT && point != RI_FNE_AT_MIX) throw Error(RI_EINVAL, "point must be 0 or 1");
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        check_shape(n, B, h, w);
        ensure_tangent(n);
        const int64_t np = (int64_t)B * h * w;
        // the l1 loss and its gradient, as in ri_cnn_train_step
        hipLaunchKernelGGL(k_noisy, dim3(gridn(np)), dim3(256), 0, s, clean, n->zin, np, sigma, seed);
        forward(n, n->zin, n->D, B, h, w, CnnGeo(), s);
        hipLaunchKernelGGL(k_l1, dim3(1024), dim3(256), 0, s, n->D, clean, n->g, np, n->part);
        if (loss) reduce_partials(n->part, 1024, 1, 1, loss, s);
        backward(n, n->zin, n->g, B, h, w, s);
        if (point == RI_FNE_AT_MIX) {
            // the Jacobian at rho u + (1 - rho) D(u + sigma n): the network's
            // activations there (the l1 gradients above are already taken)
            hipLaunchKernelGGL(k_mix, dim3(gridn(np)), dim3(256), 0, s, clean, n->D, n->zin, np, (int64_t)h * w,
                               seed ^ 0x5851F42D4C957F2Dull);
            forward(n, n->zin, n->D, B, h, w, CnnGeo(), s);
        }
        // ||J_{2D - I}(z)||_S at z (the training input, or the mixed point) by
        // power iterations on J^T J, warm-started from the previous step's vector
        float *v = n->fv, *t = n->D, *a = n->g;
        if (!n->fv_ready) {
            hipLaunchKernelGGL(k_normal, dim3(gridn(np)), dim3(256), 0, s, v, np, seed ^ 0x9E3779B97F4A7C15ull);
            n->fv_ready = true;
        }
        auto normalise = [&](float *x) {
            dot_partials<float>(x, x, np, n->part, s);
            reduce_partials(n->part, 1024, 1, 1, n->scal, s);
            hipLaunchKernelGGL(k_scale_rsqrt, dim3(gridn(np)), dim3(256), 0, s, x, np, n->scal);
        };
        normalise(v);
        for (int it = 0; it < power_iters; ++it) {
            jvp(n, v, t, B, h, w, s);
            hipLaunchKernelGGL(k_minus2, dim3(gridn(np)), dim3(256), 0, s, v, t, a, np);
            vjp(n, a, t, B, h, w, s);
            hipLaunchKernelGGL(k_minus2, dim3(gridn(np)), dim3(256), 0, s, a, t, v, np);
            normalise(v);
        }
        // a = (I - 2 J_net) v, ||a||^2 (v unit), and d(a^T J_net v)/dtheta
        jvp_store(n, v, t, B, h, w, s);
        hipLaunchKernelGGL(k_minus2, dim3(gridn(np)), dim3(256), 0, s, v, t, a, np);
        dot_partials<float>(a, a, np, n->part, s);
        reduce_partials(n->part, 1024, 1, 1, n->scal + 1, s);
        backward_core(n, v, a, n->tan, n->grads2, B, h, w, s);
        for (int l = 0; l < n->L; ++l)   // weights only: the penalty does not depend on the biases
            hipLaunchKernelGGL(k_fne_combine, dim3(gridn(n->off[2 * l + 1] - n->off[2 * l])), dim3(256), 0, s,
                               n->grads + n->off[2 * l], n->grads2 + n->off[2 * l], n->off[2 * l + 1] - n->off[2 * l],
                               n->scal + 1, lambda, eps);
        if (fne_sq) RI_CHECK_HIP(hipMemcpyAsync(fne_sq, n->scal + 1, sizeof(double), hipMemcpyDeviceToDevice, s));
        n->step++;
        const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)n->step)));
        const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)n->step)));
        hipLaunchKernelGGL(k_adam, dim3(gridn(n->P)), dim3(256), 0, s, n->params, n->grads, n->m, n->v, n->P, lr, c1,
                           c2);
        repack(n, s);
        RI_CHECK_HIP(hipGetLastError());
    });
}

}  // extern "C"
