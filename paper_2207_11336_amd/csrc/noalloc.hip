// ri_gradient_noalloc: the gradient pass of ri_gradient (appendix A,
// Re{Phi^dagger (Phi x - y)} in one fused degrid -> residual -> grid pass)
// with every work buffer its kernels use taken from a workspace that is
// compiled into the library instead of from the context: the two oversampled
// grids, the persistent launch's work counter and the FP64 partial sums of
// ||Phi x - y||^2. For callers that cannot allocate device memory (code under
// graph capture, serving loops, harnesses that forbid hipMalloc).
//
// The workspace is one file-scope __device__ array; every GPU the library runs
// on holds its own copy at its own address until the process ends. Host code
// never passes the array's name to a kernel (in host code it names a
// host-side stand-in, not device memory): ri_create looks its address up once
// per device with hipGetSymbolAddress, with that device current, and the entry
// point uses only that per-device address.
#include <mutex>

#include "ri_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)RI_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
constexpr size_t kAlign = 256;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};   // device address of `scratch` per device ordinal

size_t up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

template <typename T> ri::Prec<T> &ctx_prec(ri_ctx *c);
template <> ri::Prec<float> &ctx_prec<float>(ri_ctx *c) { return c->p32; }
template <> ri::Prec<double> &ctx_prec<double>(ri_ctx *c) { return c->p64; }

template <typename T>
void gradient_in_workspace(ri_ctx *c, unsigned char *ws, const T *x, const void *y, T *g, double *r2,
                           hipStream_t s) {
    using namespace ri;
    const size_t grid_bytes = up(sizeof(cx<T>) * (size_t)c->P * c->Np * c->Np);
    int32_t *counter = reinterpret_cast<int32_t *>(ws);
    double *part = reinterpret_cast<double *>(ws + kAlign);
    Prec<T> p = ctx_prec<T>(c);   // the context's tables; its grids are replaced below
    unsigned char *grids = ws + kAlign + up(sizeof(double) * (size_t)c->n_partials);
    p.gridA = reinterpret_cast<cx<T> *>(grids);
    p.gridB = reinterpret_cast<cx<T> *>(grids + grid_bytes);
    // data: none, the context's stored copy (internal order), or the caller's
    // vector read in place through the permutation (no staging copy)
    const cx<T> *y_sorted = nullptr, *y_user = nullptr;
    if (y == nullptr) {
        if (!c->has_data) throw Error(RI_EINVAL, "y is NULL but no data was stored with ri_set_data");
        y_sorted = p.ydata;
    } else if (y != RI_NO_DATA) {
        y_user = static_cast<const cx<T> *>(y);
    }
    fwd_zpad_fft<T>(c, p, x, s);
    fill_zero<T>(p.gridA, (int64_t)c->P * c->Np * c->Np, s);
    launch_tiles<T>(c, c->view, p, OP_FUSED, c->d.g_mode, y_sorted, y_user, nullptr, part, s,
                    counter);
    adj_fft_crop<T>(c, p, g, s);
    if (r2) reduce_partials(part, c->n_partials, 1, 1, r2, s);
}

}  // namespace

namespace ri {

size_t noalloc_scratch_bytes(const ri_ctx *c) {
    const size_t cxb = c->d.precision == 64 ? 16 : 8;
    return kAlign + up(sizeof(double) * (size_t)c->n_partials) + 2 * up(cxb * (size_t)c->P * c->Np * c->Np);
}

// Called by ri_create with the context's device current: the workspace's
// device address on that device, looked up once per device.
void noalloc_init_device(int device) {
    if (device < 0 || device >= kMaxDevices)
        throw Error(RI_EUNSUPPORTED, "device ordinal " + std::to_string(device) + " beyond the library's table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return;
    void *ptr = nullptr;
    RI_CHECK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw Error(RI_EDEVICE, "hipGetSymbolAddress returned no address for the workspace");
    g_scratch[device] = ptr;
}

}  // namespace ri

extern "C" ri_status ri_gradient_noalloc(ri_ctx *c, const void *x, const void *y, void *g, double *r2,
                                         ri_stream stream) {
    using namespace ri;
    if (!c) return RI_EINVAL;
    try {
        if (!x || !g) throw Error(RI_EINVAL, "x or g is NULL");
        if (y != nullptr && y != RI_NO_DATA && c->M == 0) y = RI_NO_DATA;
        if (c->prof_on)
            throw Error(RI_EINVAL, "kernel timing is on (ri_profile); its events come from a growing pool");
        const size_t need = noalloc_scratch_bytes(c);
        if (need > kScratchBytes)
            throw Error(RI_EINVAL, "the gradient of this context needs " + std::to_string(need) +
                                       " B of work buffers; the allocation-free workspace holds " +
                                       std::to_string(kScratchBytes) + " B (2 x w-stacks x N'^2 grid cells)");
        void *ws = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            ws = (c->device >= 0 && c->device < kMaxDevices) ? g_scratch[c->device] : nullptr;
        }
        if (!ws) throw Error(RI_EDEVICE, "the workspace address of this device was not set up");
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        if (c->d.precision == 32)
            gradient_in_workspace<float>(c, (unsigned char *)ws, (const float *)x, y, (float *)g, r2, s);
        else
            gradient_in_workspace<double>(c, (unsigned char *)ws, (const double *)x, y, (double *)g, r2, s);
        RI_CHECK_HIP(hipGetLastError());
        return RI_OK;
    } catch (const Error &e) {
        c->err = e.msg;
        return e.code;
    } catch (const std::exception &e) {
        c->err = e.what();
        return RI_EDEVICE;
    }
}
