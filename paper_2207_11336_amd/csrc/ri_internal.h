// Internal declarations of libri.so (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ri.h"
#include "../../include/ri_cnn.h"

namespace ri {

// --------------------------------------------------------------------------
// Complex helpers (interleaved re/im, 8- or 16-byte aligned)
// --------------------------------------------------------------------------
template <typename T> struct cx;
template <> struct alignas(8) cx<float> { float x, y; };
template <> struct alignas(16) cx<double> { double x, y; };

template <typename T> __host__ __device__ inline cx<T> mk(T a, T b) { cx<T> r; r.x = a; r.y = b; return r; }
template <typename T> __host__ __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __host__ __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __host__ __device__ inline cx<T> operator*(cx<T> a, cx<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> __host__ __device__ inline cx<T> scale(cx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
template <typename T> __host__ __device__ inline cx<T> conjg(cx<T> a) { return mk<T>(a.x, -a.y); }
// a * conj(b)
template <typename T> __host__ __device__ inline cx<T> mulc(cx<T> a, cx<T> b) {
    return mk<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// --------------------------------------------------------------------------
// Work item of the tile launches: one uv tile of one data block, or a chunk
// of it when the tile holds many visibilities.
// --------------------------------------------------------------------------
struct alignas(16) TileItem {
    int32_t ty0, tx0;   // tile origin (grid cells)
    int32_t vb, vc;     // first visibility (internal order) and count
};

// Sorted per-visibility data of one tile size and fraction precision.
struct View {
    int tile = 0;                 // T
    int n_items = 0;
    int64_t max_item_vis = 0;
    int32_t *perm = nullptr;      // internal -> caller index
    uint2 *rec = nullptr;         // per visibility: ((c_v << 16) | c_u, plane | h << 16 | stack << 20)
    void *frac = nullptr;         // float[2] or double[2] per visibility (f_u, f_v)
    int frac_bytes = 0;           // 4 or 8
    TileItem *items = nullptr;
    std::vector<int64_t> perm_host;  // kept for tests (caller index of each internal slot)
};

// Stored G: row m (internal order) holds the S x S values of its window in
// row-major window order; the columns follow from the row's window (centre
// cell and support in the view's record), so none are stored.
struct CSR {
    int64_t nnz = 0;
    int64_t *rowptr = nullptr;    // [M+1], internal order
    void *val = nullptr;          // cx<T>[nnz]
    int val_bytes = 0;
};

// G stored as its separable axis factors (RI_G_SEP): per visibility, in the
// main view's internal order, 17 pairs (g_u[c], g_v[c]) of complex weights.
struct Sep {
    void *w = nullptr;            // cx<T>[M][17][2]
    int val_bytes = 0;
};

// Tables and work buffers of one precision.
template <typename T> struct Prec {
    bool ready = false;
    T *icorr = nullptr;           // [N]  1 / kappa_hat((i - N/2) / N')
    cx<T> *tw = nullptr;          // [N'] exp(-2 pi i k / N')
    cx<T> *wtaps = nullptr;       // [n_wplanes][2*hmax+1]
    cx<T> *gridA = nullptr, *gridB = nullptr;   // [w-stacks][N'][N']
    cx<T> *chirp = nullptr;       // [w-stacks][N][N] phase screens (stacking only)
    T *img0 = nullptr, *img1 = nullptr;         // N x N scratch images
    cx<T> *ydata = nullptr;       // stored data, internal order
};

// Holographic matrix H = G^H G on the fine grid (appendix E), kept for the
// 32 x 32-cell tiles of the grid that some window touches. Slot s (tile
// origin ty0, tx0) stores the upper half of H's band, offsets d = (dy, dx)
// with dy in [0, R_s], dx in [-R_s, R_s] (R_s + 1 = the largest window side
// over the visibilities touching the tile; dy = 0, dx < 0 stays zero since
// H[k + d][k] = conj H[k][k + d]), one 1024-cell plane per offset:
//   H[k][k + d] at off[s] + ((dy (2 R_s + 1) + dx + R_s) << 10) + (ky & 31) * 32 + (kx & 31).
constexpr int HOLO_T = 32;
struct Holo {
    bool ready = false;
    int n_slots = 0;
    int64_t entries = 0;          // stored complex entries
    int64_t pairs = 0;            // window-cell pairs accumulated by the build
    int32_t *tmap = nullptr;      // [(N'/32)^2] slot of each tile, -1 when untouched
    int4 *tinfo = nullptr;        // [slot] (ty0, tx0, R, 0)
    int64_t *off = nullptr;       // [slot] first entry
    void *val = nullptr;          // cx<T>[entries], T the context precision
    int max_R = 0;
    double build_ms = 0.0;
};

// uSARA's denoiser state (sara.hip): dual variable and weights over the nine
// bases of the dictionary, [9][N][N] each (slot 0 the Dirac basis), and two
// [8][N][N] transform work arrays.
struct SaraState {
    bool ready = false;
    int sub_iters = 10;           // dual forward-backward sub-iterations per prox
    void *v = nullptr, *w = nullptr, *work = nullptr, *tmp = nullptr;
};

enum { PROF_TILES = 0, PROF_FFT = 1, PROF_PROX = 2, PROF_OTHER = 3, PROF_N = 4 };
struct ProfEvent {
    int cat;
    hipEvent_t a, b;
};

struct DeviceInfo {
    int cu_count = 256;
    int lds_per_block = 65536;
};

}  // namespace ri

struct ri_ctx {
    ri_plan_desc d{};
    std::vector<int64_t> block_offsets;
    int N = 0, Np = 0, logNp = 0, J = 7, jh = 3, hmax = 0, H = 3;
    double beta = 0.0;
    int64_t M = 0;
    int device = 0;
    ri::DeviceInfo dev;
    std::string err;

    // host-side plan copies (caller order)
    std::vector<double> pu, pv;           // FP64 grid positions
    std::vector<int32_t> cu, cv;          // window centres mod N'
    std::vector<int32_t> plane;           // w-plane per visibility (of the residual w with stacking)
    int P = 1;                            // w-stacks
    std::vector<double> stack_w;          // [P] stack centres w_p
    std::vector<int32_t> stack;           // stack per visibility
    std::vector<int32_t> plane_h;         // [n_wplanes]
    std::vector<double> wtaps64;          // [n_wplanes][2*hmax+1][2]

    int32_t *d_plane_h = nullptr;

    ri::View view;                        // operator view (context precision, desc tile)
    ri::View view64;                      // FP64 OTF view for the power iteration (if needed)
    bool view64_is_main = false;
    ri::CSR csr;
    ri::Sep sep;
    ri::Holo holo;
    ri::SaraState sara;

    ri::Prec<float> p32;
    ri::Prec<double> p64;

    int32_t *d_counter = nullptr;         // persistent-launch work counters
    double *d_partials = nullptr;         // FP64 reduction partials
    int n_partials = 0;
    double *d_scalars = nullptr;          // small FP64 scratch
    double *h_pinned = nullptr;           // pinned host scalars

    // CNN denoiser (inference network sized for this context's facets)
    ri_cnn *cnn = nullptr;

    bool has_data = false;
    bool prof_on = false;
    std::vector<ri::ProfEvent> prof_ev;
    std::vector<hipEvent_t> prof_pool;
    int64_t device_bytes = 0;
    double plan_ms = 0.0;
    std::vector<std::pair<int, float>> tune_ms;   // autotuner: (tile, ms per fused pass)
    std::vector<std::pair<void *, size_t>> allocs;
};

namespace ri {

#define RI_CHECK_HIP(expr)                                                          \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess) {                                                     \
            throw ::ri::Error(RI_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
        }                                                                           \
    } while (0)

struct Error {
    ri_status code;
    std::string msg;
    Error(ri_status c, std::string m) : code(c), msg(std::move(m)) {}
};

// Records a start event at construction and a stop event at destruction on
// stream s when profiling is enabled on the context.
struct ProfScope {
    ri_ctx *c;
    int cat;
    hipStream_t s;
    hipEvent_t a = nullptr;
    ProfScope(ri_ctx *c, int cat, hipStream_t s);
    ~ProfScope();
};

void *dev_alloc(ri_ctx *c, size_t bytes);
void dev_free(ri_ctx *c, void *p);

// plan.cpp
void build_plan(ri_ctx *c, const double *uvw);
void build_view(ri_ctx *c, View &v, int tile, int frac_bytes);
void free_view(ri_ctx *c, View &v);
template <typename T> void ensure_prec(ri_ctx *c, Prec<T> &p);

// fft.hip
template <typename T> void fwd_zpad_fft(ri_ctx *c, Prec<T> &p, const T *x, hipStream_t s);
template <typename T> void adj_fft_crop(ri_ctx *c, Prec<T> &p, T *x, hipStream_t s);

// gridding.hip
enum { OP_DEGRID = 1, OP_GRID = 2, OP_FUSED = 3 };
// The persistent uv-tile launch with G in mode g_mode (RI_G_CSR, RI_G_OTF or
// RI_G_SEP; the stored forms must exist in T). OP_FUSED subtracts y_sorted (internal order)
// or else y_user (caller's order, read through the view's permutation), or
// nothing when both are NULL. counter: the launch's work counter (NULL: the
// context's).
template <typename T> void launch_tiles(ri_ctx *c, const View &v, Prec<T> &p, int op, int g_mode,
                                        const cx<T> *y_sorted, const cx<T> *y_user,
                                        cx<T> *y_out_user, double *r2_partials, hipStream_t s,
                                        int32_t *counter = nullptr);
template <typename T> void fill_csr(ri_ctx *c, hipStream_t s);
template <typename T> void fill_sep(ri_ctx *c, hipStream_t s);
// Accumulate G^H G of the visibilities of v (FP64 fractions) into c->holo.val (zeroed).
template <typename T> void fill_holo(ri_ctx *c, const View &v, hipStream_t s);

// sara.hip: uSARA's prox, reweighting and dictionary transforms (context precision T)
void sara_setup(ri_ctx *c, int sub_iters, hipStream_t s);   // allocate on first use; v = 0, w = 1
void sara_reset(ri_ctx *c, hipStream_t s);
void sara_free(ri_ctx *c);
template <typename T> void sara_prox(ri_ctx *c, const T *z, T thr, T *x_out, hipStream_t s);
template <typename T> void sara_reweight(ri_ctx *c, const T *x, T rho, hipStream_t s);
template <typename T> void sara_analysis(ri_ctx *c, const T *x, T *coef9, hipStream_t s);
template <typename T> void sara_synthesis(ri_ctx *c, const T *coef9, T *x, hipStream_t s);

// holo.hip
void holo_build(ri_ctx *c, const View &v64, hipStream_t s);
void holo_free(ri_ctx *c);
// Y = H X on the N' x N' grid (Y is overwritten).
template <typename T> void holo_apply(ri_ctx *c, const cx<T> *X, cx<T> *Y, hipStream_t s);
// out = Re{Z^dagger F^dagger H F Z} x (uses p.gridA and p.gridB).
template <typename T> void holo_normal(ri_ctx *c, Prec<T> &p, const T *x, T *out, hipStream_t s);
// out[0] = dots[0] - 2 dots[1] + yy[0] (the residual norm from the normal operator).
void holo_residual(double *out, const double *dots, const double *yy, hipStream_t s);
int tiles_partials(ri_ctx *c);
// Dynamic LDS bytes of a fused tile-kernel workgroup at tile side `tile` (subgrid tile + 2 H),
// cx_bytes = 8 (FP32) or 16 (FP64).
size_t lds_for_tile(int tile, int H, int cx_bytes);

// noalloc.hip: the allocation-free gradient's workspace
void noalloc_init_device(int device);          // once per device, with it current (ri_create)
size_t noalloc_scratch_bytes(const ri_ctx *c); // workspace bytes the context's gradient needs

// image.hip
template <typename T> void fill_zero(cx<T> *p, int64_t n, hipStream_t s);
template <typename T> void fill_real(T *p, int64_t n, T v, hipStream_t s);
void fill_zero_i32(int32_t *p, int64_t n, hipStream_t s);
void fill_zero_f64(double *p, int64_t n, hipStream_t s);
template <typename T> void permute_to_internal(const cx<T> *y_user, cx<T> *y_int, const int32_t *perm,
                                               int64_t M, hipStream_t s);
template <typename T> void haar_prox(ri_ctx *c, const T *x_in, const T *g, T gamma_or_zero, const T *z_direct,
                                     T thr, T *out, double *norm_partials, hipStream_t s);
int image_partials(ri_ctx *c);
void reduce_partials(const double *partials, int n, int stride, int count, double *out, hipStream_t s);
template <typename T> void dot_partials(const T *a, const T *b, int64_t n, double *partials, hipStream_t s);
template <typename T> void diff2_partials(const T *a, T alpha, const T *b, int64_t n, double *partials,
                                          hipStream_t s);
template <typename T> void axpby(T *out, const T *a, T alpha, const T *b, T beta, int64_t n, hipStream_t s);
// out[0] = max_i a[i] (FP64), via RED_WG partials.
template <typename T> void max_value(const T *a, int64_t n, double *partials, double *out, hipStream_t s);
void scale_by_inv_sqrt(double *x, const double *sumsq, int64_t n, hipStream_t s);
template <typename Tin, typename Tout> void convert(const Tin *in, Tout *out, int64_t n, hipStream_t s);

// cnn.hip: the residual CNN denoiser seen from the imaging context.
// Facet geometry of a batch: item b is facet first + b of an N x N image cut
// into core x core facets (nfx per row) with a halo; its tile holds image rows
// fy*core - halo ... (N == 0: every item is a whole image, nothing masked).
struct CnnGeo {
    int N = 0, core = 0, halo = 0, nfx = 1, first = 0;
};
ri_cnn *cnn_create_inference(int layers, int max_batch, int side);
void cnn_destroy(ri_cnn *n);
int64_t cnn_param_count_for(int layers);
int cnn_layers(const ri_cnn *n);
void cnn_load_params(ri_cnn *n, const float *params, hipStream_t s);
// out = D(z) facet by facet (appendix D): core x core facets with a halo,
// all facets of a batch in one launch per layer. z, out: N x N, type T.
template <typename T> void cnn_denoise(ri_cnn *n, const T *z, T *out, int N, int core, int halo, hipStream_t s);
int cnn_tile_side(int N, int core, int halo);

}  // namespace ri
