// Host-runtime internals shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "launch.h"
#include "tree.h"

namespace swv {

// Kernel families of the tuning table.
enum { kFamDirect64 = 0, kFamDirect32 = 1, kFamTree = 2, kFamAdjoint = 3, kFamGrad = 4, kFamilies = 5 };

struct DevBuf {
    void* p = nullptr;
    size_t n = 0;
};

struct DeviceGuard {
    int prev = 0;
    bool ok = false;
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
};

}  // namespace swv

struct swv_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    swv::DevBuf comp;       // packed components
    swv::DevBuf partial;    // per-chunk partial sums (adjoint, gradients)
    swv::DevBuf partial2;   // per-block chi^2 partials
    swv::DevBuf grid;       // image-grid directions and adjoint output (dirty images)
    swv::DevBuf ones;       // unit visibilities (dirty beam)
    swv::DevBuf degrid;     // w planes and image scratch of the degridding predictor
    swv::DevBuf hog;        // per-workgroup peaks of the grid-wide Hogbom cycle
    void* fft_plan = nullptr;   // batched 2-D FFT plan of the degridding predictor
    void* scratch = nullptr;    // device address of the allocation-free entry points' array
    int fft_shape[3] = {0, 0, 0};
    int* d_status = nullptr;  // deferred-error bits raised by kernels
    int n_cu = 256;
    int per_lane[swv::kFamilies][2];
    int block[swv::kFamilies][2];
    // plans that point at this context; the context is freed when it has
    // been destroyed and the last plan has gone
    int refs = 1;
};

namespace swv {
// Drops one reference to the context and frees it when none is left.
void ctx_release(swv_ctx ctx);
}  // namespace swv

namespace swv {

int hip_fail(hipError_t e, const char* what);
int ensure(swv_ctx ctx, DevBuf& b, size_t bytes);
void tune_defaults(swv_ctx ctx);
int size_class(int64_t rows);
// Rows per chunk of the adjoint (image) and gradient reductions: enough
// (chunk, tile) blocks for one full round of resident blocks, `blocks_per_cu`
// on each compute unit.
int64_t choose_chunk(int64_t n_rows, int64_t tiles, int n_cu, int blocks_per_cu);
int check_sign_prec(int sign, int prec, bool allow_f32);
bool tune_valid(int family, int per_lane, int block);
int upload_tree(swv_ctx ctx, swv_tree t, const TRec** out);
TreeArgs tree_args(swv_tree t, const TRec* d_rec);
// Traversal for tree t given the tuned choice (1 level walker, 2 branch
// walker): 0 level walker, 1 branch walker, -1 if no compiled one fits.
int tree_walker(swv_tree t, int preferred);
// Releases a plan made by the degridding predictor (no-op on NULL).
void destroy_fft_plan(void* plan);

// Argument checks shared by the adjoint entry points (status code).
int check_adjoint_args(const char* who, swv_ctx ctx, int64_t n_vis, const double* u,
                       const double* v, const double* w, const void* y, int64_t n_pix,
                       const double* l, const double* m, const double* nm1, int sign, int prec,
                       const void* img_out);
// Tile shape and row chunking of the adjoint for a problem size; the chunk
// count fixes the summation order, so two calls with the same shape give the
// same bits.
struct AdjointShape {
    int ppl = 1, block = 64;
    int64_t chunk = 1, n_chunks = 0;
};
AdjointShape adjoint_shape(swv_ctx ctx, int64_t n_vis, int64_t n_pix, int prec);
// Bytes of per-chunk partial sums the adjoint needs (complex128 per chunk and pixel).
size_t adjoint_partial_bytes(const AdjointShape& sh, int64_t n_pix);

// Device address of the fixed scratch array of the allocation-free entry
// points on `device`, which must be the current device; looked up once per
// device (hipGetSymbolAddress) and cached.
int noalloc_scratch(int device, void** out);
// Its size in bytes.
size_t noalloc_scratch_bytes();

}  // namespace swv
