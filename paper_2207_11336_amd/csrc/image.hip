// Image-domain kernels: the Haar-l1 + positivity prox (paper appendices A and
// B: soft-thresholding is the closed-form prox of the l1 norm; the threshold
// is gamma lambda = tau / sqrt(2L)), fused with the gradient step of eq. (A2),
// FP64 reductions for the stopping test and the power method, and small
// fill / permutation kernels (fills instead of memset so any sequence can be
// captured in a graph).
#include "ri_internal.h"

namespace ri {

namespace {

constexpr int RED_WG = 1024;   // fixed grid of the FP64 reductions -> deterministic sums

template <typename V>
__global__ void k_fill(V *p, int64_t n, V v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

template <typename T>
__global__ void k_permute(const cx<T> *__restrict__ yu, cx<T> *__restrict__ yi, const int32_t *__restrict__ perm,
                          int64_t M) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x)
        yi[i] = yu[perm[i]];
}

__device__ __forceinline__ double block_sum(double v, double *s_red) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) t += s_red[w];
    return t;   // valid in thread 0
}

template <typename T>
__device__ __forceinline__ T soft(T c, T t) {
    const T a = fabs(c) - t;
    return a > (T)0 ? copysign(a, c) : (T)0;
}

// Four levels of the orthonormal 2D Haar transform act on each 16 x 16
// aligned block on its own, so the prox runs block by block: 4 blocks per
// 256-thread workgroup, the block in LDS, analysis with every detail
// coefficient thresholded as it is produced, the coarsest coefficient
// thresholded, synthesis, positivity. z = zdirect, or x - gamma g.
template <typename T>
__global__ void __launch_bounds__(256) k_haar_prox(const T *__restrict__ x, const T *__restrict__ g, T gamma,
                                                   const T *__restrict__ zdirect, T thr, T *__restrict__ out,
                                                   double *__restrict__ part, int N) {
    __shared__ T a[4][16][17];
    __shared__ double s_red[8];
    const int nbx = N / 16, nb = nbx * nbx;
    const int sub = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int b = blockIdx.x * 4 + sub;
    const bool active = b < nb;
    const int by = active ? (b / nbx) * 16 : 0, bx = active ? (b % nbx) * 16 : 0;
    // load: each lane 4 pixels (a 2x2 quad)
    const int qy = (l >> 3) * 2, qx = (l & 7) * 2;
    if (active) {
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const int yy = qy + (d >> 1), xx = qx + (d & 1);
            const size_t o = (size_t)(by + yy) * N + bx + xx;
            a[sub][yy][xx] = zdirect ? zdirect[o] : x[o] - gamma * g[o];
        }
    }
    __syncthreads();
    // analysis: level s = 1, 2, 4, 8 (quad spacing)
    for (int s = 1; s <= 8; s <<= 1) {
        const int nq = 16 / (2 * s);                 // quads per side
        if (active && l < nq * nq) {
            const int y = (l / nq) * 2 * s, xx = (l % nq) * 2 * s;
            const T x00 = a[sub][y][xx], x01 = a[sub][y][xx + s];
            const T x10 = a[sub][y + s][xx], x11 = a[sub][y + s][xx + s];
            const T ll = (x00 + x01 + x10 + x11) * (T)0.5;
            const T lh = (x00 - x01 + x10 - x11) * (T)0.5;
            const T hl = (x00 + x01 - x10 - x11) * (T)0.5;
            const T hh = (x00 - x01 - x10 + x11) * (T)0.5;
            a[sub][y][xx] = s == 8 ? soft(ll, thr) : ll;
            a[sub][y][xx + s] = soft(lh, thr);
            a[sub][y + s][xx] = soft(hl, thr);
            a[sub][y + s][xx + s] = soft(hh, thr);
        }
        __syncthreads();
    }
    // synthesis
    for (int s = 8; s >= 1; s >>= 1) {
        const int nq = 16 / (2 * s);
        if (active && l < nq * nq) {
            const int y = (l / nq) * 2 * s, xx = (l % nq) * 2 * s;
            const T ll = a[sub][y][xx], lh = a[sub][y][xx + s];
            const T hl = a[sub][y + s][xx], hh = a[sub][y + s][xx + s];
            a[sub][y][xx] = (ll + lh + hl + hh) * (T)0.5;
            a[sub][y][xx + s] = (ll - lh + hl - hh) * (T)0.5;
            a[sub][y + s][xx] = (ll + lh - hl - hh) * (T)0.5;
            a[sub][y + s][xx + s] = (ll - lh - hl + hh) * (T)0.5;
        }
        __syncthreads();
    }
    double dx2 = 0.0, x2 = 0.0;
    if (active) {
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const int yy = qy + (d >> 1), xx = qx + (d & 1);
            const size_t o = (size_t)(by + yy) * N + bx + xx;
            T v = a[sub][yy][xx];
            v = v > (T)0 ? v : (T)0;
            out[o] = v;
            if (part) {
                const double dv = (double)v - (x ? (double)x[o] : 0.0);
                dx2 += dv * dv;
                x2 += (double)v * (double)v;
            }
        }
    }
    if (part) {
        const double s1 = block_sum(dx2, s_red);
        const double s2 = block_sum(x2, s_red);
        if (threadIdx.x == 0) { part[2 * blockIdx.x] = s1; part[2 * blockIdx.x + 1] = s2; }
    }
}

template <typename T>
__global__ void k_dot(const T *__restrict__ a, const T *__restrict__ b, int64_t n, double *part) {
    __shared__ double s_red[4];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += (double)a[i] * (double)b[i];
    const double t = block_sum(acc, s_red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <typename T>
__global__ void k_diff2(const T *__restrict__ a, T alpha, const T *__restrict__ b, int64_t n, double *part) {
    __shared__ double s_red[4];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double d = (double)alpha * (double)a[i] - (double)b[i];
        acc += d * d;
    }
    const double t = block_sum(acc, s_red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <typename T>
__global__ void k_max(const T *__restrict__ a, int64_t n, double *part) {
    __shared__ double s_red[4];
    double m = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = fmax(m, (double)a[i]);
    for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(s_red[0], s_red[1]), fmax(s_red[2], s_red[3]));
}

__global__ void k_reduce_max(const double *part, int n, double *out) {
    __shared__ double s_red[4];
    double m = -INFINITY;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, part[i]);
    for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = fmax(fmax(s_red[0], s_red[1]), fmax(s_red[2], s_red[3]));
}

// out[k] = sum_i part[i * stride + k], i < n (fixed order).
__global__ void k_reduce(const double *part, int n, int stride, int count, double *out) {
    __shared__ double s_red[4];
    for (int k = 0; k < count; ++k) {
        double acc = 0.0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[(size_t)i * stride + k];
        const double t = block_sum(acc, s_red);
        if (threadIdx.x == 0) out[k] = t;
        __syncthreads();
    }
}

template <typename T>
__global__ void k_axpby(T *out, const T *a, T alpha, const T *b, T beta, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = alpha * a[i] + (b ? beta * b[i] : (T)0);
}

__global__ void k_scale_inv_sqrt(double *x, const double *sumsq, int64_t n) {
    const double s = 1.0 / sqrt(sumsq[0]);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] *= s;
}

template <typename Tin, typename Tout>
__global__ void k_convert(const Tin *in, Tout *out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (Tout)in[i];
}

inline int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

}  // namespace

template <typename T>
void fill_zero(cx<T> *p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<cx<T>>, dim3(grid_for(n)), dim3(256), 0, s, p, n, mk<T>((T)0, (T)0));
}
template <typename T>
void fill_real(T *p, int64_t n, T v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
}
template void fill_real<float>(float *, int64_t, float, hipStream_t);
template void fill_real<double>(double *, int64_t, double, hipStream_t);

void fill_zero_i32(int32_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(n)), dim3(256), 0, s, p, n, 0);
}
void fill_zero_f64(double *p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n)), dim3(256), 0, s, p, n, 0.0);
}

template <typename T>
void permute_to_internal(const cx<T> *y_user, cx<T> *y_int, const int32_t *perm, int64_t M, hipStream_t s) {
    if (M <= 0) return;
    hipLaunchKernelGGL(k_permute<T>, dim3(grid_for(M)), dim3(256), 0, s, y_user, y_int, perm, M);
}

int image_partials(ri_ctx *c) {
    const int nb = (c->N / 16) * (c->N / 16);
    return std::max(RED_WG, (nb + 3) / 4) * 2;
}

template <typename T>
void haar_prox(ri_ctx *c, const T *x_in, const T *g, T gamma, const T *z_direct, T thr, T *out,
               double *norm_partials, hipStream_t s) {
    const int nb = (c->N / 16) * (c->N / 16);
    const int nwg = (nb + 3) / 4;
    ProfScope prof(c, PROF_PROX, s);
    hipLaunchKernelGGL(k_haar_prox<T>, dim3(nwg), dim3(256), 0, s, x_in, g, gamma, z_direct, thr, out,
                       norm_partials, c->N);
}

void reduce_partials(const double *partials, int n, int stride, int count, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, partials, n, stride, count, out);
}

template <typename T>
void dot_partials(const T *a, const T *b, int64_t n, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_dot<T>, dim3(RED_WG), dim3(256), 0, s, a, b, n, partials);
}

template <typename T>
void max_value(const T *a, int64_t n, double *partials, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_max<T>, dim3(RED_WG), dim3(256), 0, s, a, n, partials);
    hipLaunchKernelGGL(k_reduce_max, dim3(1), dim3(256), 0, s, partials, RED_WG, out);
}
template void max_value<float>(const float *, int64_t, double *, double *, hipStream_t);
template void max_value<double>(const double *, int64_t, double *, double *, hipStream_t);

template <typename T>
void diff2_partials(const T *a, T alpha, const T *b, int64_t n, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_diff2<T>, dim3(RED_WG), dim3(256), 0, s, a, alpha, b, n, partials);
}
template void diff2_partials<float>(const float *, float, const float *, int64_t, double *, hipStream_t);
template void diff2_partials<double>(const double *, double, const double *, int64_t, double *, hipStream_t);

template <typename T>
void axpby(T *out, const T *a, T alpha, const T *b, T beta, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby<T>, dim3(grid_for(n)), dim3(256), 0, s, out, a, alpha, b, beta, n);
}

void scale_by_inv_sqrt(double *x, const double *sumsq, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_inv_sqrt, dim3(grid_for(n)), dim3(256), 0, s, x, sumsq, n);
}

template <typename Tin, typename Tout>
void convert(const Tin *in, Tout *out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_convert<Tin, Tout>), dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
}

template void fill_zero<float>(cx<float> *, int64_t, hipStream_t);
template void fill_zero<double>(cx<double> *, int64_t, hipStream_t);
template void permute_to_internal<float>(const cx<float> *, cx<float> *, const int32_t *, int64_t, hipStream_t);
template void permute_to_internal<double>(const cx<double> *, cx<double> *, const int32_t *, int64_t, hipStream_t);
template void haar_prox<float>(ri_ctx *, const float *, const float *, float, const float *, float, float *,
                               double *, hipStream_t);
template void haar_prox<double>(ri_ctx *, const double *, const double *, double, const double *, double, double *,
                                double *, hipStream_t);
template void dot_partials<float>(const float *, const float *, int64_t, double *, hipStream_t);
template void dot_partials<double>(const double *, const double *, int64_t, double *, hipStream_t);
template void axpby<float>(float *, const float *, float, const float *, float, int64_t, hipStream_t);
template void axpby<double>(double *, const double *, double, const double *, double, int64_t, hipStream_t);
template void convert<float, double>(const float *, double *, int64_t, hipStream_t);
template void convert<double, float>(const double *, float *, int64_t, hipStream_t);
template void convert<double, double>(const double *, double *, int64_t, hipStream_t);

}  // namespace ri
