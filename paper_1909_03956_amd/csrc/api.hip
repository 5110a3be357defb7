// C ABI of libswvis: argument checks, context and workspace management, tree
// upload and kernel dispatch.  No exception crosses this file's functions.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "api_internal.h"
#include "sphere.h"

using namespace swv;

namespace swv {

DeviceGuard::DeviceGuard(int dev) {
    ok = hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess;
}
DeviceGuard::~DeviceGuard() {
    if (ok) (void)hipSetDevice(prev);
}

int hip_fail(hipError_t e, const char* what) {
    return fail(SWV_EHIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

int ensure(swv_ctx ctx, DevBuf& b, size_t bytes) {
    if (b.n >= bytes && b.p) return SWV_OK;
    size_t want = bytes < 256 ? 256 : bytes;
    want = want + want / 4;  // headroom against regrowth
    if (b.p) {
        // the old buffer may still be read by queued work
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        (void)hipFree(b.p);
        b.p = nullptr;
        b.n = 0;
    }
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(SWV_ENOMEM, "device allocation of %zu bytes failed: %s", want,
                    hipGetErrorString(e));
    }
    b.n = want;
    return SWV_OK;
}

void tune_defaults(swv_ctx ctx) {
    // (per_lane, block) per family, both size classes; see swv_tune_get.  The
    // fastest shapes measured on MI355X for a few thousand components, a
    // thousand pixels and 10^6 - 10^7 rows.
    const int pl[kFamilies][2] = {{2, 64}, {1, 256}, {1, 64}, {4, 128}, {4, 128}};
    for (int f = 0; f < kFamilies; ++f)
        for (int c = 0; c < 2; ++c) {
            ctx->per_lane[f][c] = pl[f][0];
            ctx->block[f][c] = pl[f][1];
        }
    // adjoint over 2^20 rows or more: 256-thread blocks of 4 pixels per lane
    // cover a thousand pixels in one tile, so every row chunk is read by one
    // block: the same time as 128 threads, with 1.0x the rows' bytes fetched
    // from memory instead of 1.4x
    ctx->block[kFamAdjoint][1] = 256;
    // FP32-compensated direct sum under 2^20 rows: two rows per lane share
    // each component's scalar loads (0.230 against 0.264 ms for 1 per lane in
    // the autotuner's small case, 2^18 rows; the two tie on its 2^22 rows)
    ctx->per_lane[kFamDirect32][0] = 2;
}

int size_class(int64_t rows) { return rows < (int64_t(1) << 20) ? 0 : 1; }

// Rows per chunk.  Chunks come in groups of 8 with one chunk of each group on
// each XCD (the block order of the row-chunked kernels), so the chunk count is
// 8q: an XCD then runs q x tiles blocks in rounds of n_cu x blocks_per_cu / 8,
// each block doing 1/(8q) of the rows, and the time goes as rounds / q.  q is
// the smallest minimiser of that, searched up to about 8 rounds per XCD
// (which also bounds the partial sums, one set per chunk) or one full round,
// whichever is more.  A count that is not a multiple of 8 would leave the last
// group's chunks on some XCDs only.
int64_t choose_chunk(int64_t n_rows, int64_t tiles, int n_cu, int blocks_per_cu) {
    if (n_rows <= 0) return 1;
    if (tiles < 1) tiles = 1;
    const int64_t per_xcd = std::max<int64_t>(1, (int64_t)n_cu * blocks_per_cu / 8);
    const int64_t q_fill = (per_xcd + tiles - 1) / tiles;           // one round or more
    const int64_t q_rounds = 8 * per_xcd / tiles;                   // about 8 rounds
    const int64_t q_rows = std::max<int64_t>(1, n_rows / (8 * 64));  // chunks of >= 64 rows
    const int64_t q_max = std::min<int64_t>(std::max<int64_t>(q_fill, q_rounds), q_rows);
    int64_t best_q = 1, best_rounds = (tiles + per_xcd - 1) / per_xcd;
    for (int64_t q = 2; q <= q_max; ++q) {
        const int64_t rounds = (q * tiles + per_xcd - 1) / per_xcd;
        if (rounds * best_q < best_rounds * q) {   // rounds / q < best_rounds / best_q
            best_q = q;
            best_rounds = rounds;
        }
    }
    const int64_t want = 8 * best_q;
    int64_t chunk = (n_rows + want - 1) / want;
    if (chunk < 64) chunk = 64;
    if (chunk > (int64_t(1) << 30)) chunk = int64_t(1) << 30;  // rows per chunk fit an int
    return chunk;
}

bool tune_valid(int family, int per_lane, int block) {
    if (family < 0 || family >= kFamilies) return false;
    const bool pl_ok = per_lane == 1 || per_lane == 2 || per_lane == 4;
    const bool bl_ok = block == 64 || block == 128 || block == 256;
    // tree: per_lane selects the traversal (1 by depth and shape, 2 branch
    // walker, 4 level walker where it fits)
    if (family == kFamTree) return (per_lane == 1 || per_lane == 2 || per_lane == 4) && bl_ok;
    if (family == kFamGrad) return pl_ok && block == 128;
    return pl_ok && bl_ok;
}

int check_sign_prec(int sign, int prec, bool allow_f32) {
    if (sign != 1 && sign != -1) return fail(SWV_EDOMAIN, "sign must be +1 or -1 (got %d)", sign);
    if (prec != SWV_FP64 && !(allow_f32 && prec == SWV_F32C))
        return fail(allow_f32 ? SWV_EINVAL : SWV_ENOTSUP, "unsupported precision %d", prec);
    return SWV_OK;
}

int upload_tree(swv_ctx ctx, swv_tree t, const TRec** out) {
    auto it = t->device_records.find(ctx->device);
    if (it != t->device_records.end()) {
        *out = (const TRec*)it->second;
        return SWV_OK;
    }
    void* p = nullptr;
    const size_t bytes = t->records.size() * sizeof(TRec);
    if (bytes > kMaxRecordBytes)
        return fail(SWV_ENOTSUP, "tree upload: a record stream of %zu bytes exceeds the traversal's "
                    "%zu-byte limit", bytes, (size_t)kMaxRecordBytes);
    hipError_t e = hipMalloc(&p, bytes < 32 ? 32 : bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SWV_ENOMEM, "tree upload: %s", hipGetErrorString(e));
    }
    if (bytes) {
        e = hipMemcpy(p, t->records.data(), bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(p);
            return hip_fail(e, "tree upload");
        }
    }
    t->device_records[ctx->device] = p;
    *out = (const TRec*)p;
    return SWV_OK;
}

static std::vector<Comp> packed_leaves(swv_tree t) {
    const size_t n = t->leaf_pix.size();
    std::vector<Comp> c(n);
    for (size_t k = 0; k < n; ++k)
        c[k] = Comp{t->leaf_l[k], t->leaf_m[k], t->leaf_nm1[k], t->leaf_flux[k]};
    return c;
}

static int upload_leaves(swv_ctx ctx, swv_tree t, const Comp** out) {
    auto it = t->device_leaves.find(ctx->device);
    if (it != t->device_leaves.end()) {
        *out = (const Comp*)it->second;
        return SWV_OK;
    }
    const std::vector<Comp> c = packed_leaves(t);
    void* p = nullptr;
    const size_t bytes = c.size() * sizeof(Comp);
    hipError_t e = hipMalloc(&p, bytes < 32 ? 32 : bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SWV_ENOMEM, "tree leaves upload: %s", hipGetErrorString(e));
    }
    if (bytes) {
        e = hipMemcpy(p, c.data(), bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(p);
            return hip_fail(e, "tree leaves upload");
        }
    }
    t->device_leaves[ctx->device] = p;
    *out = (const Comp*)p;
    return SWV_OK;
}

int tree_walker(swv_tree t, int preferred) {
    const bool level_ok = t->J <= kTreeMaxJ;
    const bool branch_ok = t->max_branching + 1 <= kTreeMaxSeg;
    if (preferred == 2 && branch_ok) return 1;
    if (!level_ok) return branch_ok ? 1 : -1;
    if (preferred == 4 || t->J <= kTreeLevelAlwaysJ || !branch_ok) return 0;
    // a thresholded tree (leaves at many levels) keeps the branch walker: by
    // levels, the sweep track's J = 16 tree at 0.5 % retained took 0.48 ms,
    // 2.4 times its time at 1 %
    if (t->thresholded) return 1;
    // deeper trees: runs of one-child nodes cost the branch walker less (cfg2's
    // 2,000 components at J = 11, 12, 53-62 % of the internal nodes with one
    // child: 10.8 and 18.1 ms by levels against 14.9 and 23.3 ms by branchings;
    // 140 sparse components at J = 12-16, 89-94 %: 0.75-0.98 ms by branchings
    // against 1.49-1.99 ms by levels)
    int64_t internal = 0;
    for (int j = 1; j < t->J; ++j) internal += (int64_t)t->levels[j - 1].pix.size();
    return 4 * t->n_one_child > 3 * internal ? 1 : 0;
}

TreeArgs tree_args(swv_tree t, const TRec* d_rec) {
    TreeArgs a;
    a.rec = d_rec;
    a.n_roots = (int)t->n_roots;
    a.J = t->J;
    a.seg_depth = t->max_branching + 1;
    a.pruned = t->thresholded ? 1 : 0;
    return a;
}

int check_adjoint_args(const char* who, swv_ctx ctx, int64_t n_vis, const double* u,
                       const double* v, const double* w, const void* y, int64_t n_pix,
                       const double* l, const double* m, const double* nm1, int sign, int prec,
                       const void* img_out) {
    if (!ctx) return fail(SWV_EINVAL, "%s: null context", who);
    if (n_vis < 0 || n_pix < 0) return fail(SWV_EINVAL, "%s: negative size", who);
    if (n_vis > 0 && (!u || !v || !w || !y))
        return fail(SWV_EINVAL, "%s: null visibility pointer", who);
    if (n_pix > 0 && (!l || !m || !nm1 || !img_out))
        return fail(SWV_EINVAL, "%s: null pixel pointer", who);
    if (sign != 1 && sign != -1) return fail(SWV_EDOMAIN, "sign must be +1 or -1 (got %d)", sign);
    if (prec != SWV_FP64 && prec != SWV_F32C)
        return fail(SWV_EINVAL, "%s: unsupported precision %d", who, prec);
    return SWV_OK;
}

AdjointShape adjoint_shape(swv_ctx ctx, int64_t n_vis, int64_t n_pix, int prec) {
    AdjointShape sh;
    const int sc = size_class(n_vis);
    sh.ppl = ctx->per_lane[kFamAdjoint][sc];
    sh.block = ctx->block[kFamAdjoint][sc];
    const int64_t tiles = (n_pix + (int64_t)sh.ppl * sh.block - 1) / ((int64_t)sh.ppl * sh.block);
    sh.chunk = choose_chunk(n_vis, tiles, ctx->n_cu, adjoint_blocks_per_cu(prec, sh.ppl, sh.block));
    sh.n_chunks = n_vis > 0 ? (n_vis + sh.chunk - 1) / sh.chunk : 0;
    return sh;
}

size_t adjoint_partial_bytes(const AdjointShape& sh, int64_t n_pix) {
    return 16 * (size_t)n_pix * (size_t)(sh.n_chunks > 0 ? sh.n_chunks : 1);
}

void ctx_release(swv_ctx ctx) {
    if (--ctx->refs > 0) return;
    {
        DeviceGuard g(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        for (DevBuf* b : {&ctx->comp, &ctx->partial, &ctx->partial2, &ctx->grid, &ctx->ones,
                          &ctx->degrid, &ctx->hog})
            if (b->p) (void)hipFree(b->p);
        destroy_fft_plan(ctx->fft_plan);
        if (ctx->d_status) (void)hipFree(ctx->d_status);
    }
    delete ctx;
}

}  // namespace swv

#define CHECK_CTX(ctx)                                                   \
    do {                                                                 \
        if (!(ctx)) return fail(SWV_EINVAL, "%s: null context", __func__); \
    } while (0)

#define GUARD(ctx)                                                              \
    DeviceGuard guard_((ctx)->device);                                          \
    if (!guard_.ok) return fail(SWV_EHIP, "%s: cannot select device %d", __func__, (ctx)->device)

#define HIPCALL(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

#define NEED(ptr, n)                                                                   \
    do {                                                                               \
        if ((n) > 0 && !(ptr)) return fail(SWV_EINVAL, "%s: %s is null", __func__, #ptr); \
    } while (0)

#define TRY_BEGIN try {
#define TRY_END                                                          \
    }                                                                    \
    catch (const std::bad_alloc&) {                                      \
        return fail(SWV_ENOMEM, "%s: host allocation failed", __func__); \
    }                                                                    \
    catch (...) {                                                        \
        return fail(SWV_EINVAL, "%s: internal error", __func__);         \
    }

extern "C" {

// ------------------------------------------------------------ contexts ---
int swv_ctx_create(int device, void* stream, swv_ctx* out) {
    if (!out) return fail(SWV_EINVAL, "swv_ctx_create: null out");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= n)
        return fail(SWV_EINVAL, "swv_ctx_create: device %d not in [0, %d)", device, n);
    TRY_BEGIN
    DeviceGuard g(device);
    if (!g.ok) return fail(SWV_EHIP, "swv_ctx_create: cannot select device %d", device);
    auto* c = new swv_ctx_s();
    c->device = device;
    c->stream = (hipStream_t)stream;
    e = hipMalloc(&c->d_status, sizeof(int));
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "hipMalloc(status)");
    }
    e = hipMemset(c->d_status, 0, sizeof(int));
    if (e != hipSuccess) {
        (void)hipFree(c->d_status);
        delete c;
        return hip_fail(e, "hipMemset(status)");
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
    // the fixed scratch of swv_adjoint_noalloc on this device (the device is
    // current here); a failure is reported by that entry point instead
    if (noalloc_scratch(device, &c->scratch) != SWV_OK) c->scratch = nullptr;
    tune_defaults(c);
    if (const char* path = getenv("SWV_TUNE_CACHE")) {
        if (path[0] && swv_tune_load(c, path) != SWV_OK) tune_defaults(c);
    }
    *out = c;
    clear_error();
    return SWV_OK;
    TRY_END
}

int swv_ctx_set_stream(swv_ctx ctx, void* stream) {
    CHECK_CTX(ctx);
    ctx->stream = (hipStream_t)stream;
    return SWV_OK;
}

int swv_ctx_synchronize(swv_ctx ctx) {
    CHECK_CTX(ctx);
    GUARD(ctx);
    HIPCALL(hipStreamSynchronize(ctx->stream));
    int st = 0;
    HIPCALL(hipMemcpy(&st, ctx->d_status, sizeof(int), hipMemcpyDeviceToHost));
    if (st) {
        HIPCALL(hipMemset(ctx->d_status, 0, sizeof(int)));
        if (st & kStatusDomain)
            return fail(SWV_EDOMAIN, "a kernel saw a component with l^2 + m^2 >= 1");
        return fail(SWV_EDOMAIN, "a kernel saw a non-finite input");
    }
    clear_error();
    return SWV_OK;
}

int swv_ctx_destroy(swv_ctx ctx) {
    if (!ctx) return SWV_OK;
    ctx_release(ctx);
    return SWV_OK;
}

// ------------------------------------------------------- direct route ---
int swv_predict_direct(swv_ctx ctx, int64_t n_vis, const double* u, const double* v,
                       const double* w, int64_t n_comp, const double* l, const double* m,
                       const double* flux, int sign, int prec, void* vis_out) {
    CHECK_CTX(ctx);
    if (n_vis < 0 || n_comp < 0) return fail(SWV_EINVAL, "swv_predict_direct: negative size");
    if (n_comp > INT32_MAX) return fail(SWV_EINVAL, "swv_predict_direct: n_comp > 2^31 - 1");
    NEED(u, n_vis); NEED(v, n_vis); NEED(w, n_vis); NEED(vis_out, n_vis);
    NEED(l, n_comp); NEED(m, n_comp); NEED(flux, n_comp);
    int rc = check_sign_prec(sign, prec, true);
    if (rc) return rc;
    if (n_vis == 0) return SWV_OK;
    TRY_BEGIN
    GUARD(ctx);
    rc = ensure(ctx, ctx->comp, sizeof(Comp) * (size_t)(n_comp > 0 ? n_comp : 1));
    if (rc) return rc;
    Comp* comp = (Comp*)ctx->comp.p;
    HIPCALL(launch_ingest(ctx->stream, n_comp, l, m, flux, comp, ctx->d_status));
    const int fam = prec == SWV_FP64 ? kFamDirect64 : kFamDirect32;
    const int sc = size_class(n_vis);
    HIPCALL(launch_direct(ctx->stream, prec, ctx->per_lane[fam][sc], ctx->block[fam][sc], n_vis,
                          u, v, w, comp, n_comp, sign, vis_out, ctx->d_status));
    return SWV_OK;
    TRY_END
}

// --------------------------------------------------------- tree route ---
static int check_components_host(int64_t n, const double* l, const double* m, const double* f) {
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(l[i]) || !std::isfinite(m[i]) || !std::isfinite(f[i]))
            return fail(SWV_EDOMAIN, "component %lld is not finite", (long long)i);
        if (!(l[i] * l[i] + m[i] * m[i] < 1.0))
            return fail(SWV_EDOMAIN, "component %lld has l^2 + m^2 >= 1", (long long)i);
    }
    return SWV_OK;
}

static int check_level(int J) {
    if (J < 1 || J > SWV_MAX_LEVEL) return fail(SWV_EDOMAIN, "J = %d outside [1, 29]", J);
    return SWV_OK;
}

int swv_tree_build(int J, double ra_p, double dec_p, int64_t n_comp, const double* l,
                   const double* m, const double* flux, swv_tree* out) {
    if (!out) return fail(SWV_EINVAL, "swv_tree_build: null out");
    *out = nullptr;
    int rc = check_level(J);
    if (rc) return rc;
    if (n_comp < 0) return fail(SWV_EINVAL, "swv_tree_build: negative n_comp");
    NEED(l, n_comp); NEED(m, n_comp); NEED(flux, n_comp);
    if (!std::isfinite(ra_p) || !std::isfinite(dec_p))
        return fail(SWV_EDOMAIN, "swv_tree_build: non-finite phase centre");
    rc = check_components_host(n_comp, l, m, flux);
    if (rc) return rc;
    TRY_BEGIN
    auto* t = new swv_tree_s();
    rc = build_tree(J, ra_p, dec_p, n_comp, l, m, flux, t);
    if (rc) {
        delete t;
        return rc;
    }
    *out = t;
    clear_error();
    return SWV_OK;
    TRY_END
}

int swv_tree_stats(swv_tree t, swv_tree_stats_t* out) {
    if (!t || !out) return fail(SWV_EINVAL, "swv_tree_stats: null argument");
    std::memset(out, 0, sizeof *out);
    out->J = t->J;
    out->n_comp = t->n_comp;
    out->n_leaves = (int64_t)t->leaf_pix.size();
    for (int j = 1; j <= t->J; ++j) out->n_nodes[j] = (int64_t)t->levels[j - 1].pix.size();
    int64_t internal = 0;
    for (int j = 1; j < t->J; ++j) internal += out->n_nodes[j];
    // a thresholded tree has leaves above level J too
    out->n_internal = t->thresholded ? t->n_alive : internal;
    out->n_records = (int64_t)t->records.size();
    out->sparsity = (double)out->n_leaves / (double)n_pixels(t->J);
    out->build_seconds = t->build_seconds;
    out->max_branching = t->max_branching;
    return SWV_OK;
}

int swv_tree_leaves(swv_tree t, int64_t* pix, double* l, double* m, double* nm1, double* flux) {
    if (!t) return fail(SWV_EINVAL, "swv_tree_leaves: null tree");
    if (t->thresholded)
        return fail(SWV_ENOTSUP, "swv_tree_leaves: defined on an unthresholded tree only");
    const size_t n = t->leaf_pix.size();
    if (pix) std::memcpy(pix, t->leaf_pix.data(), n * sizeof(int64_t));
    if (l) std::memcpy(l, t->leaf_l.data(), n * sizeof(double));
    if (m) std::memcpy(m, t->leaf_m.data(), n * sizeof(double));
    if (nm1) std::memcpy(nm1, t->leaf_nm1.data(), n * sizeof(double));
    if (flux) std::memcpy(flux, t->leaf_flux.data(), n * sizeof(double));
    return SWV_OK;
}

int swv_tree_level(swv_tree t, int j, int64_t* pix, int32_t* child_mask, double* lambda,
                   double* gamma) {
    if (!t) return fail(SWV_EINVAL, "swv_tree_level: null tree");
    if (t->thresholded)
        return fail(SWV_ENOTSUP, "swv_tree_level: defined on an unthresholded tree only");
    if (j < 1 || j > t->J) return fail(SWV_EINVAL, "swv_tree_level: level %d not in [1, %d]", j, t->J);
    const TreeLevel& L = t->levels[j - 1];
    const size_t n = L.pix.size();
    if (pix) std::memcpy(pix, L.pix.data(), n * sizeof(int64_t));
    if (child_mask) std::memcpy(child_mask, L.mask.data(), n * sizeof(int32_t));
    if (lambda) std::memcpy(lambda, L.lambda.data(), n * sizeof(double));
    if (gamma) std::memcpy(gamma, L.gamma.data(), 3 * n * sizeof(double));
    return SWV_OK;
}

int swv_tree_set_flux(swv_tree t, const double* leaf_flux) {
    if (!t) return fail(SWV_EINVAL, "swv_tree_set_flux: null tree");
    if (t->thresholded)
        return fail(SWV_ENOTSUP, "swv_tree_set_flux: defined on an unthresholded tree only");
    const size_t n = t->leaf_pix.size();
    if (n > 0 && !leaf_flux) return fail(SWV_EINVAL, "swv_tree_set_flux: null leaf_flux");
    for (size_t k = 0; k < n; ++k)
        if (!std::isfinite(leaf_flux[k]))
            return fail(SWV_EDOMAIN, "swv_tree_set_flux: flux %zu is not finite", k);
    TRY_BEGIN
    for (auto* copies : {&t->device_records, &t->device_leaves})
        for (auto& kv : *copies) {   // device copies may still be read
            DeviceGuard g(kv.first);
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        }
    const size_t n_rec = t->records.size();
    std::copy(leaf_flux, leaf_flux + n, t->leaf_flux.begin());
    build_coefficients(t);
    if (t->records.size() != n_rec) return fail(SWV_EINVAL, "swv_tree_set_flux: internal error");
    for (auto& kv : t->device_records) {   // same structure: refresh in place
        DeviceGuard g(kv.first);
        hipError_t e = hipMemcpy(kv.second, t->records.data(), n_rec * sizeof(TRec),
                                 hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "swv_tree_set_flux upload");
    }
    if (!t->device_leaves.empty()) {
        const std::vector<Comp> c = packed_leaves(t);
        for (auto& kv : t->device_leaves) {
            DeviceGuard g(kv.first);
            hipError_t e = hipMemcpy(kv.second, c.data(), c.size() * sizeof(Comp),
                                     hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_fail(e, "swv_tree_set_flux upload");
        }
    }
    return SWV_OK;
    TRY_END
}

int swv_predict_tree(swv_ctx ctx, swv_tree t, int64_t n_vis, const double* u, const double* v,
                     const double* w, int sign, int prec, void* vis_out) {
    CHECK_CTX(ctx);
    if (!t) return fail(SWV_EINVAL, "swv_predict_tree: null tree");
    if (n_vis < 0) return fail(SWV_EINVAL, "swv_predict_tree: negative n_vis");
    NEED(u, n_vis); NEED(v, n_vis); NEED(w, n_vis); NEED(vis_out, n_vis);
    int rc = check_sign_prec(sign, prec, true);
    if (rc) return rc;
    const int sc = size_class(n_vis);
    const int walker = tree_walker(t, ctx->per_lane[kFamTree][sc]);
    if (walker < 0)
        return fail(SWV_ENOTSUP,
                    "swv_predict_tree: J = %d with %d nested branchings on one path: above the "
                    "compiled maxima (J %d, or %d branchings)",
                    t->J, t->max_branching, kTreeMaxJ, kTreeMaxSeg - 1);
    if (n_vis == 0) return SWV_OK;
    TRY_BEGIN
    GUARD(ctx);
    const TRec* rec = nullptr;
    rc = upload_tree(ctx, t, &rec);
    if (rc) return rc;
    const TreeArgs a = tree_args(t, rec);
    HIPCALL(launch_tree(ctx->stream, walker, ctx->block[kFamTree][sc], prec, a, n_vis, u, v, w,
                        sign, vis_out, ctx->d_status));
    return SWV_OK;
    TRY_END
}

int swv_predict_tree_leaves(swv_ctx ctx, swv_tree t, int64_t n_vis, const double* u,
                            const double* v, const double* w, int sign, int prec,
                            void* vis_out) {
    CHECK_CTX(ctx);
    if (!t) return fail(SWV_EINVAL, "swv_predict_tree_leaves: null tree");
    if (t->thresholded)
        return fail(SWV_ENOTSUP,
                    "swv_predict_tree_leaves: a thresholded tree has no Eq. 16 form (its dropped "
                    "coefficients do not collapse onto leaves)");
    if (n_vis < 0) return fail(SWV_EINVAL, "swv_predict_tree_leaves: negative n_vis");
    NEED(u, n_vis); NEED(v, n_vis); NEED(w, n_vis); NEED(vis_out, n_vis);
    int rc = check_sign_prec(sign, prec, true);
    if (rc) return rc;
    if (n_vis == 0) return SWV_OK;
    TRY_BEGIN
    GUARD(ctx);
    const Comp* comp = nullptr;
    rc = upload_leaves(ctx, t, &comp);
    if (rc) return rc;
    const int fam = prec == SWV_FP64 ? kFamDirect64 : kFamDirect32;
    const int sc = size_class(n_vis);
    HIPCALL(launch_direct(ctx->stream, prec, ctx->per_lane[fam][sc], ctx->block[fam][sc], n_vis,
                          u, v, w, comp, (int64_t)t->leaf_pix.size(), sign, vis_out,
                          ctx->d_status));
    return SWV_OK;
    TRY_END
}

int swv_tree_destroy(swv_tree t) {
    if (!t) return SWV_OK;
    if (--t->refs > 0) return SWV_OK;   // a plan still reads its device records
    for (auto* copies : {&t->device_records, &t->device_leaves})
        for (auto& kv : *copies) {
            DeviceGuard g(kv.first);
            (void)hipDeviceSynchronize();
            (void)hipFree(kv.second);
        }
    delete t;
    return SWV_OK;
}

int swv_tree_threshold(swv_tree t, double fraction, swv_tree* out) {
    if (!out) return fail(SWV_EINVAL, "swv_tree_threshold: null out");
    *out = nullptr;
    if (!t) return fail(SWV_EINVAL, "swv_tree_threshold: null tree");
    if (t->thresholded) return fail(SWV_ENOTSUP, "swv_tree_threshold: tree already thresholded");
    if (!(fraction >= 0.0 && fraction <= 1.0))
        return fail(SWV_EDOMAIN, "swv_tree_threshold: fraction must be in [0, 1]");
    TRY_BEGIN
    auto* p = new swv_tree_s();
    const int rc = prune_tree(*t, retain_fraction(*t, fraction), p);
    if (rc) {
        delete p;
        return rc;
    }
    *out = p;
    return SWV_OK;
    TRY_END
}

int swv_tree_prune(swv_tree t, int64_t n_kept, const int64_t* kept, swv_tree* out) {
    if (!out) return fail(SWV_EINVAL, "swv_tree_prune: null out");
    *out = nullptr;
    if (!t) return fail(SWV_EINVAL, "swv_tree_prune: null tree");
    if (t->thresholded) return fail(SWV_ENOTSUP, "swv_tree_prune: tree already thresholded");
    if (n_kept < 0 || (n_kept > 0 && !kept)) return fail(SWV_EINVAL, "swv_tree_prune: bad list");
    TRY_BEGIN
    std::vector<int64_t> k(kept, kept + n_kept);
    for (int64_t i = 1; i < n_kept; ++i)
        if (k[i] <= k[i - 1])
            return fail(SWV_EINVAL, "swv_tree_prune: indices must increase");
    auto* p = new swv_tree_s();
    const int rc = prune_tree(*t, k, p);
    if (rc) {
        delete p;
        return rc;
    }
    *out = p;
    return SWV_OK;
    TRY_END
}

int swv_tree_kept(swv_tree t, int64_t cap, int64_t* kept, int64_t* n_kept, int64_t* n_coeffs) {
    if (!t || !n_kept || !n_coeffs || cap < 0 || (cap > 0 && !kept))
        return fail(SWV_EINVAL, "swv_tree_kept: bad argument");
    if (!t->thresholded) return fail(SWV_EINVAL, "swv_tree_kept: tree not thresholded");
    *n_kept = (int64_t)t->kept.size();
    *n_coeffs = t->n_coeffs;
    const int64_t nw = std::min<int64_t>(cap, *n_kept);
    if (nw > 0) std::memcpy(kept, t->kept.data(), (size_t)nw * sizeof(int64_t));
    return SWV_OK;
}

// ------------------------------------------------------ sphere pixels ---
int swv_ang2pix(int J, double ra_p, double dec_p, int64_t n, const double* l, const double* m,
                int64_t* pix) {
    int rc = check_level(J);
    if (rc) return rc;
    if (n < 0) return fail(SWV_EINVAL, "swv_ang2pix: negative n");
    NEED(l, n); NEED(m, n); NEED(pix, n);
    const Frame F = make_frame(ra_p, dec_p);
    for (int64_t i = 0; i < n; ++i) {
        if (!(l[i] * l[i] + m[i] * m[i] < 1.0) || !std::isfinite(l[i]) || !std::isfinite(m[i]))
            return fail(SWV_EDOMAIN, "swv_ang2pix: direction %lld outside the unit disk",
                        (long long)i);
        ld xyz[3];
        lm_to_xyz(F, l[i], m[i], xyz);
        pix[i] = ang2pix(J, xyz);
    }
    return SWV_OK;
}

int swv_pixel_centres(int J, double ra_p, double dec_p, int64_t n, const int64_t* pix, double* l,
                      double* m, double* nm1) {
    int rc = check_level(J);
    if (rc) return rc;
    if (n < 0) return fail(SWV_EINVAL, "swv_pixel_centres: negative n");
    NEED(pix, n); NEED(l, n); NEED(m, n); NEED(nm1, n);
    const Frame F = make_frame(ra_p, dec_p);
    const int64_t np = n_pixels(J);
    for (int64_t i = 0; i < n; ++i) {
        if (pix[i] < 0 || pix[i] >= np)
            return fail(SWV_EINVAL, "swv_pixel_centres: pixel %lld out of range", (long long)pix[i]);
        ld xyz[3];
        pix2xyz(J, pix[i], xyz);
        xyz_to_lmn(F, xyz, &l[i], &m[i], &nm1[i]);
    }
    return SWV_OK;
}

int swv_pixels_in_disk(int J, double ra_p, double dec_p, double radius, int64_t cap,
                       int64_t* pix, double* l, double* m, double* nm1, int64_t* n_out) {
    int rc = check_level(J);
    if (rc) return rc;
    if (!n_out) return fail(SWV_EINVAL, "swv_pixels_in_disk: null n_out");
    if (cap < 0) return fail(SWV_EINVAL, "swv_pixels_in_disk: negative cap");
    if (!(radius >= 0) || !std::isfinite(radius))
        return fail(SWV_EDOMAIN, "swv_pixels_in_disk: bad radius");
    NEED(pix, cap); NEED(l, cap); NEED(m, cap); NEED(nm1, cap);
    TRY_BEGIN
    const Frame F = make_frame(ra_p, dec_p);
    // phase centre in xyz
    ld pc[3];
    lm_to_xyz(F, 0.0, 0.0, pc);
    const ld cosr = cosl((ld)radius);
    // descend the hierarchy keeping pixels whose extent can reach the disk
    // (a level-j pixel lies within 2 sqrt(A_j) of its centre)
    std::vector<int64_t> cand, next;
    for (int64_t k = 0; k < 12; ++k) cand.push_back(k);
    for (int j = 1; j <= J; ++j) {
        next.clear();
        const ld reach = (j < J) ? 2.0L * sqrtl((ld)pixel_area(j)) : 0.0L;
        const ld cos_reach = (ld)radius + reach >= 3.1415926535L ? -2.0L : cosl((ld)radius + reach);
        for (int64_t k : cand) {
            ld c[3];
            pix2xyz(j, k, c);
            const ld dot = pc[0] * c[0] + pc[1] * c[1] + pc[2] * c[2];
            if (j < J) {
                if (dot >= cos_reach)
                    for (int64_t ch = 0; ch < 4; ++ch) next.push_back(4 * k + ch);
            } else if (dot >= cosr) {
                next.push_back(k);
            }
        }
        cand.swap(next);
    }
    std::sort(cand.begin(), cand.end());
    *n_out = (int64_t)cand.size();
    const int64_t nw = cap < *n_out ? cap : *n_out;
    for (int64_t i = 0; i < nw; ++i) {
        pix[i] = cand[i];
        ld xyz[3];
        pix2xyz(J, cand[i], xyz);
        xyz_to_lmn(F, xyz, &l[i], &m[i], &nm1[i]);
    }
    return SWV_OK;
    TRY_END
}

// ---------------------------------------------- subtract, image, grads ---
int swv_residual_chi2(swv_ctx ctx, int64_t n_vis, const void* vis_obs, const void* vis_model,
                      double inv_sigma2, void* resid_out, double* chi2_out) {
    CHECK_CTX(ctx);
    if (n_vis < 0) return fail(SWV_EINVAL, "swv_residual_chi2: negative n_vis");
    NEED(vis_obs, n_vis); NEED(vis_model, n_vis); NEED(resid_out, n_vis);
    if (!chi2_out) return fail(SWV_EINVAL, "swv_residual_chi2: null chi2_out");
    if (!std::isfinite(inv_sigma2)) return fail(SWV_EDOMAIN, "swv_residual_chi2: bad inv_sigma2");
    TRY_BEGIN
    GUARD(ctx);
    int rc = ensure(ctx, ctx->partial2, sizeof(double) * (size_t)residual_blocks(n_vis));
    if (rc) return rc;
    HIPCALL(launch_residual(ctx->stream, n_vis, vis_obs, vis_model, inv_sigma2, resid_out,
                            (double*)ctx->partial2.p, chi2_out));
    return SWV_OK;
    TRY_END
}


int swv_adjoint(swv_ctx ctx, int64_t n_vis, const double* u, const double* v, const double* w,
                const void* y, int64_t n_pix, const double* l, const double* m,
                const double* nm1, int sign, int prec, void* img_out) {
    int rc = check_adjoint_args("swv_adjoint", ctx, n_vis, u, v, w, y, n_pix, l, m, nm1, sign,
                                prec, img_out);
    if (rc) return rc;
    if (n_pix == 0) return SWV_OK;
    TRY_BEGIN
    GUARD(ctx);
    const AdjointShape sh = adjoint_shape(ctx, n_vis, n_pix, prec);
    rc = ensure(ctx, ctx->partial, adjoint_partial_bytes(sh, n_pix));
    if (rc) return rc;
    HIPCALL(launch_adjoint(ctx->stream, prec, sh.ppl, sh.block, sh.chunk, n_vis, u, v, w, y,
                           n_pix, l, m, nm1, sign, ctx->partial.p, img_out));
    return SWV_OK;
    TRY_END
}

int swv_grad_direct(swv_ctx ctx, int64_t n_vis, const double* u, const double* v,
                    const double* w, const void* y, int64_t n_comp, const double* l,
                    const double* m, const double* flux, int sign, double alpha,
                    double* d_flux, double* d_l, double* d_m) {
    CHECK_CTX(ctx);
    if (n_vis < 0 || n_comp < 0) return fail(SWV_EINVAL, "swv_grad_direct: negative size");
    NEED(u, n_vis); NEED(v, n_vis); NEED(w, n_vis); NEED(y, n_vis);
    NEED(l, n_comp); NEED(m, n_comp); NEED(flux, n_comp);
    NEED(d_flux, n_comp); NEED(d_l, n_comp); NEED(d_m, n_comp);
    int rc = check_sign_prec(sign, SWV_FP64, false);
    if (rc) return rc;
    if (!std::isfinite(alpha)) return fail(SWV_EDOMAIN, "swv_grad_direct: bad alpha");
    if (n_comp == 0) return SWV_OK;
    TRY_BEGIN
    GUARD(ctx);
    rc = ensure(ctx, ctx->comp, sizeof(Comp) * (size_t)n_comp);
    if (rc) return rc;
    Comp* comp = (Comp*)ctx->comp.p;
    HIPCALL(launch_ingest(ctx->stream, n_comp, l, m, flux, comp, ctx->d_status));
    const int cpl = ctx->per_lane[kFamGrad][size_class(n_vis)];
    int gblock = 128;
    int64_t tiles = 1;
    grad_tiling(cpl, n_comp, &gblock, &tiles);
    const int64_t chunk = choose_chunk(n_vis, tiles, ctx->n_cu, grad_blocks_per_cu(cpl, gblock));
    const int64_t n_chunks = n_vis > 0 ? (n_vis + chunk - 1) / chunk : 0;
    rc = ensure(ctx, ctx->partial, 32 * (size_t)n_comp * (size_t)(n_chunks > 0 ? n_chunks : 1));
    if (rc) return rc;
    HIPCALL(launch_grad(ctx->stream, cpl, chunk, n_vis, u, v, w, y, comp, n_comp, sign, alpha,
                        (double*)ctx->partial.p, d_flux, d_l, d_m));
    return SWV_OK;
    TRY_END
}

// -------------------------------------------------------------- tuning ---
int swv_tune_get(swv_ctx ctx, int family, int size_class_, int* per_lane, int* block) {
    CHECK_CTX(ctx);
    if (family < 0 || family >= kFamilies || size_class_ < 0 || size_class_ > 1 || !per_lane ||
        !block)
        return fail(SWV_EINVAL, "swv_tune_get: bad argument");
    *per_lane = ctx->per_lane[family][size_class_];
    *block = ctx->block[family][size_class_];
    return SWV_OK;
}

int swv_tune_set(swv_ctx ctx, int family, int size_class_, int per_lane, int block) {
    CHECK_CTX(ctx);
    if (size_class_ < 0 || size_class_ > 1 || !tune_valid(family, per_lane, block))
        return fail(SWV_EINVAL, "swv_tune_set: no compiled shape (%d, %d) for family %d",
                    per_lane, block, family);
    ctx->per_lane[family][size_class_] = per_lane;
    ctx->block[family][size_class_] = block;
    return SWV_OK;
}

}  // extern "C"
