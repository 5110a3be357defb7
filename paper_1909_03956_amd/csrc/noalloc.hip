// The allocation-free form of the adjoint, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).  Its
// per-chunk partial sums live in one fixed file-scope device array instead of
// a context workspace.
//
// `scratch` below is a device variable: in host code its name is only a
// host-side stand-in, so every host use goes through the device address that
// hipGetSymbolAddress returns for the current device (each GPU holds its own
// copy of the array, at its own address).  The addresses are looked up once
// per device, at context creation, and cached.
#include <map>
#include <mutex>

#include "api_internal.h"

namespace swv {

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;   // 32 MiB per device

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device id -> device address of `scratch`

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

int noalloc_scratch(int device, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return SWV_OK;
    }
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        *out = nullptr;
        return fail(SWV_EHIP, "scratch address on device %d: %s", device, hipGetErrorString(e));
    }
    g_scratch_ptr[device] = p;
    *out = p;
    return SWV_OK;
}

}  // namespace swv

using namespace swv;

extern "C" int swv_adjoint_noalloc(swv_ctx ctx, int64_t n_vis, const double* u, const double* v,
                                   const double* w, const void* y, int64_t n_pix, const double* l,
                                   const double* m, const double* nm1, int sign, int prec,
                                   void* img_out) {
    int rc = check_adjoint_args("swv_adjoint_noalloc", ctx, n_vis, u, v, w, y, n_pix, l, m, nm1,
                                sign, prec, img_out);
    if (rc) return rc;
    if (n_pix == 0) return SWV_OK;
    try {
        DeviceGuard guard(ctx->device);
        if (!guard.ok)
            return fail(SWV_EHIP, "swv_adjoint_noalloc: cannot select device %d", ctx->device);
        const AdjointShape sh = adjoint_shape(ctx, n_vis, n_pix, prec);
        const size_t need = adjoint_partial_bytes(sh, n_pix);
        if (need > kScratchBytes)
            return fail(SWV_ENOMEM,
                        "swv_adjoint_noalloc: %lld pixels x %lld row chunks need %zu bytes of "
                        "partial sums; the fixed scratch holds %zu",
                        (long long)n_pix, (long long)sh.n_chunks, need, kScratchBytes);
        void* p = ctx->scratch;
        if (!p) {
            rc = noalloc_scratch(ctx->device, &p);
            if (rc) return rc;
            ctx->scratch = p;
        }
        const hipError_t e = launch_adjoint(ctx->stream, prec, sh.ppl, sh.block, sh.chunk, n_vis,
                                            u, v, w, y, n_pix, l, m, nm1, sign, p, img_out);
        if (e != hipSuccess) return hip_fail(e, "swv_adjoint_noalloc");
        return SWV_OK;
    } catch (...) {
        return fail(SWV_EINVAL, "swv_adjoint_noalloc: internal error");
    }
}
