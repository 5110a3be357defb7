// Clean loop (sections 2.1, 2.2, 3.5): image grids, dirty images and the
// dirty beam from the exact adjoint, the Hogbom minor cycle (Eqs. 4, 5), the
// clean image (Eq. 6) and the major-cycle driver around the tree predictor.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <vector>

#include "api_internal.h"
#include "clean.h"
#include "sphere.h"
#include "tree.h"

namespace swv {

namespace {

constexpr int kGridBlock = 256;

// Direction of grid pixel p (SIN projection); off the unit disk: zeros.
__device__ __forceinline__ bool grid_direction(int64_t p, int nx, int cx, int cy, double cell,
                                               double& l, double& m, double& nm1) {
    const int64_t iy = p / nx, ix = p - iy * nx;
    l = (double)(ix - cx) * cell;
    m = (double)(iy - cy) * cell;
    const double r2 = l * l + m * m;
    const bool in = r2 < 1.0;
    nm1 = in ? -r2 / (1.0 + sqrt(1.0 - r2)) : 0.0;
    if (!in) l = m = 0.0;
    return in;
}

__global__ __launch_bounds__(kGridBlock) void k_grid(int64_t n, int nx, int cx, int cy,
                                                     double cell, double* __restrict__ l,
                                                     double* __restrict__ m,
                                                     double* __restrict__ nm1) {
    const int64_t p = (int64_t)blockIdx.x * kGridBlock + threadIdx.x;
    if (p >= n) return;
    double a, b, c;
    grid_direction(p, nx, cx, cy, cell, a, b, c);
    l[p] = a;
    m[p] = b;
    nm1[p] = c;
}

__global__ __launch_bounds__(kGridBlock) void k_fill_unit(int64_t n, double2* __restrict__ y) {
    const int64_t j = (int64_t)blockIdx.x * kGridBlock + threadIdx.x;
    if (j < n) y[j] = make_double2(1.0, 0.0);
}

// img[p] = Re x[p] / n_vis on the disk, 0 off it.
__global__ __launch_bounds__(kGridBlock) void k_real_image(int64_t n, const double2* __restrict__ x,
                                                           int nx, int cx, int cy, double cell,
                                                           double n_vis,
                                                           double* __restrict__ img) {
    const int64_t p = (int64_t)blockIdx.x * kGridBlock + threadIdx.x;
    if (p >= n) return;
    double l, m, nm1;
    const bool in = grid_direction(p, nx, cx, cy, cell, l, m, nm1);
    img[p] = in ? x[p].x / n_vis : 0.0;
}

// ---------------------------------------------------------------- Hogbom ---
// One workgroup runs the whole minor cycle.  Thread t owns pixels t, t + 1024,
// ... for the whole cycle, so a pixel is only ever read and written by its
// owner.  Each iteration: the owners' running peaks are reduced to the block's
// peak (largest key, lowest pixel id on ties: a total order, so the result
// does not depend on the reduction's shape), and one pass over the pixels
// subtracts the shifted beam and finds the next running peaks.  One barrier
// per iteration: the per-wave results alternate between two LDS slots.
constexpr int kHogBlock = 1024;
constexpr int kHogWaves = kHogBlock / 64;
constexpr int kHogBatch = 8;

__device__ __forceinline__ bool ahead(double k1, int i1, double k2, int i2) {
    return k1 > k2 || (k1 == k2 && i1 < i2);
}

template <bool ABS>
__global__ __launch_bounds__(kHogBlock) void k_hogbom(
    double* __restrict__ img, const double* __restrict__ beam, int nx, int ny, double gain,
    double threshold, int64_t max_iter, int64_t* __restrict__ comp_pix,
    double* __restrict__ comp_val, int64_t* __restrict__ n_found) {
    __shared__ double s_key[2][kHogWaves], s_val[2][kHogWaves];
    __shared__ int s_idx[2][kHogWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = nx * ny;
    const int64_t bw = 2 * (int64_t)nx - 1;
    // the thread's first pixel and the stride as (rows, columns)
    const int y0 = tid / nx, x0 = tid - (tid / nx) * nx;
    const int sy = kHogBlock / nx, sx = kHogBlock - sy * nx;

    double key = -HUGE_VAL, val = 0.0;
    int idx = INT_MAX;
    for (int p = tid; p < n; p += kHogBlock) {
        const double x = img[p];
        const double k = ABS ? fabs(x) : x;
        if (k > key) {
            key = k;
            val = x;
            idx = p;
        }
    }
    int64_t it = 0;
    for (int buf = 0;; buf ^= 1) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double k2 = __shfl_xor(key, off, 64);
            const double v2 = __shfl_xor(val, off, 64);
            const int i2 = __shfl_xor(idx, off, 64);
            if (ahead(k2, i2, key, idx)) {
                key = k2;
                val = v2;
                idx = i2;
            }
        }
        if (lane == 0) {
            s_key[buf][wave] = key;
            s_val[buf][wave] = val;
            s_idx[buf][wave] = idx;
        }
        __syncthreads();
        key = s_key[buf][0];
        val = s_val[buf][0];
        idx = s_idx[buf][0];
        for (int q = 1; q < kHogWaves; ++q) {
            if (ahead(s_key[buf][q], s_idx[buf][q], key, idx)) {
                key = s_key[buf][q];
                val = s_val[buf][q];
                idx = s_idx[buf][q];
            }
        }
        // the same decision in every thread
        if (it >= max_iter || !(key > threshold)) break;
        const double gc = gain * val;
        if (tid == 0) {
            comp_pix[it] = idx;
            comp_val[it] = gc;
        }
        ++it;
        const int py = idx / nx, px = idx - (idx / nx) * nx;
        const double* B = beam + (int64_t)(ny - 1 - py) * bw + (nx - 1 - px);
        key = -HUGE_VAL;
        val = 0.0;
        idx = INT_MAX;
        int y = y0, x = x0;
        // kHogBatch pixels per step: their loads are all in flight together
        for (int p0 = tid; p0 < n; p0 += kHogBatch * kHogBlock) {
            double iv[kHogBatch], bv[kHogBatch];
#pragma unroll
            for (int b = 0; b < kHogBatch; ++b) {
                const int p = p0 + b * kHogBlock;
                if (p < n) {
                    iv[b] = img[p];
                    bv[b] = B[(int64_t)y * bw + x];
                }
                x += sx;
                y += sy;
                if (x >= nx) {
                    x -= nx;
                    ++y;
                }
            }
#pragma unroll
            for (int b = 0; b < kHogBatch; ++b) {
                const int p = p0 + b * kHogBlock;
                if (p < n) {
                    const double t = gc * bv[b];
                    const double r = iv[b] - t;
                    img[p] = r;
                    const double k = ABS ? fabs(r) : r;
                    if (k > key) {
                        key = k;
                        val = r;
                        idx = p;
                    }
                }
            }
        }
    }
    if (tid == 0) *n_found = it;
}

// The same minor cycle spread over G workgroups, all resident at once (a
// cooperative launch: the runtime refuses a grid that could not be).  Global
// thread g owns pixels g, g + G B, ...  Each iteration a workgroup publishes
// its peak in its slot (key, value, index, then the iteration number with
// release order) and gathers every workgroup's slot of that iteration
// (acquire loads of the iteration number, then the data): the gather is the
// barrier, with no shared counter.  Every workgroup reduces the G peaks in
// the same total order, so all take the same decision.  Slots alternate
// between two buffers: a workgroup can only reuse a buffer after every other
// one has published the next iteration, i.e. finished reading it.  Every wait
// is bounded: after kHogSpinLimit polls the workgroup gives up, the cycle
// ends and *n_found is set to -1.
constexpr int kHogGridBlock = 256;
constexpr int kHogGridWaves = kHogGridBlock / 64;
constexpr int kHogSpinLimit = 1 << 22;

// Block-wide best (key, val, idx): wave butterflies, then every thread
// reduces the per-wave results in wave order.
__device__ __forceinline__ void block_best(double& key, double& val, int& idx, double* sk,
                                           double* sv, int* si) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double k2 = __shfl_xor(key, off, 64);
        const double v2 = __shfl_xor(val, off, 64);
        const int i2 = __shfl_xor(idx, off, 64);
        if (ahead(k2, i2, key, idx)) {
            key = k2;
            val = v2;
            idx = i2;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();   // the previous reader of these slots is done
    if (lane == 0) {
        sk[wave] = key;
        sv[wave] = val;
        si[wave] = idx;
    }
    __syncthreads();
    key = sk[0];
    val = sv[0];
    idx = si[0];
    for (int q = 1; q < kHogGridWaves; ++q)
        if (ahead(sk[q], si[q], key, idx)) {
            key = sk[q];
            val = sv[q];
            idx = si[q];
        }
}

// slot layout: [buffer][workgroup][key, val, idx, iteration + 1] as 64-bit words
__device__ __forceinline__ void publish(unsigned long long* slot, double key, double val,
                                        int idx, int64_t it) {
    __hip_atomic_store(slot + 0, (unsigned long long)__double_as_longlong(key), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(slot + 1, (unsigned long long)__double_as_longlong(val), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(slot + 2, (unsigned long long)(unsigned)idx, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(slot + 3, (unsigned long long)(it + 1), __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
}

template <bool ABS>
__global__ __launch_bounds__(kHogGridBlock) void k_hogbom_grid(
    double* __restrict__ img, const double* __restrict__ beam, int nx, int ny, double gain,
    double threshold, int64_t max_iter, int64_t* __restrict__ comp_pix,
    double* __restrict__ comp_val, int64_t* __restrict__ n_found,
    unsigned long long* __restrict__ slots) {
    __shared__ double sk[kHogGridWaves], sv[kHogGridWaves];
    __shared__ int si[kHogGridWaves];
    __shared__ int s_timeout;
    const int G = (int)gridDim.x;
    const int n = nx * ny;
    const int64_t bw = 2 * (int64_t)nx - 1;
    const int stride = G * kHogGridBlock;
    const int g0 = (int)blockIdx.x * kHogGridBlock + (int)threadIdx.x;
    const int y0 = g0 / nx, x0 = g0 - (g0 / nx) * nx;
    const int sy = stride / nx, sx = stride - sy * nx;
    if (threadIdx.x == 0) s_timeout = 0;

    double key = -HUGE_VAL, val = 0.0;
    int idx = INT_MAX;
    for (int p = g0; p < n; p += stride) {
        const double x = img[p];
        const double k = ABS ? fabs(x) : x;
        if (k > key) {
            key = k;
            val = x;
            idx = p;
        }
    }
    int64_t it = 0;   // the peaks being exchanged belong to the image after `it` components
    for (;;) {
        block_best(key, val, idx, sk, sv, si);
        unsigned long long* buf = slots + (size_t)(it & 1) * 4 * G;
        if (threadIdx.x == 0) publish(buf + 4 * (size_t)blockIdx.x, key, val, idx, it);
        // gather: thread b waits for workgroup b's slot of this iteration
        key = -HUGE_VAL;
        val = 0.0;
        idx = INT_MAX;
        for (int b = threadIdx.x; b < G; b += kHogGridBlock) {
            const unsigned long long* sl = buf + 4 * (size_t)b;
            int spins = 0;
            while (__hip_atomic_load(sl + 3, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) !=
                   (unsigned long long)(it + 1)) {
                if (++spins > kHogSpinLimit) {
                    s_timeout = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            const double k2 = __longlong_as_double(
                (long long)__hip_atomic_load(sl + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            const double v2 = __longlong_as_double(
                (long long)__hip_atomic_load(sl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            const int i2 = (int)(unsigned)__hip_atomic_load(sl + 2, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
            if (ahead(k2, i2, key, idx)) {
                key = k2;
                val = v2;
                idx = i2;
            }
        }
        block_best(key, val, idx, sk, sv, si);   // its barriers also publish s_timeout
        if (s_timeout) {
            if (threadIdx.x == 0) *n_found = -1;
            return;
        }
        if (it >= max_iter || !(key > threshold)) break;   // the same in every workgroup
        const double gc = gain * val;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            comp_pix[it] = idx;
            comp_val[it] = gc;
        }
        ++it;
        const int py = idx / nx, px = idx - (idx / nx) * nx;
        const double* B = beam + (int64_t)(ny - 1 - py) * bw + (nx - 1 - px);
        key = -HUGE_VAL;
        val = 0.0;
        idx = INT_MAX;
        int y = y0, x = x0;
        for (int p = g0; p < n; p += stride) {
            const double t = gc * B[(int64_t)y * bw + x];
            const double r = img[p] - t;
            img[p] = r;
            const double k = ABS ? fabs(r) : r;
            if (k > key) {
                key = k;
                val = r;
                idx = p;
            }
            x += sx;
            y += sy;
            while (x >= nx) {
                x -= nx;
                ++y;
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *n_found = it;
}

// --------------------------------------------------------------- restore ---
// Components are staged through LDS in tiles (pixel split into row and
// column once per component); each thread sums its pixel's terms in list
// order.
constexpr int kRestTile = 256;

__global__ __launch_bounds__(kGridBlock) void k_restore(
    int nx, int64_t n, int64_t n_comp, const int64_t* __restrict__ comp_pix,
    const double* __restrict__ comp_val, double a, double b, double c,
    const double* __restrict__ residual, double* __restrict__ out) {
    __shared__ double s_x[kRestTile], s_y[kRestTile], s_g[kRestTile];
    const int64_t p = (int64_t)blockIdx.x * kGridBlock + threadIdx.x;
    const int64_t pc = p < n ? p : n - 1;
    const double iy = (double)(pc / nx), ix = (double)(pc - (pc / nx) * nx);
    const double b2 = 2.0 * b;
    double s = 0.0;
    for (int64_t t0 = 0; t0 < n_comp; t0 += kRestTile) {
        const int nt = (int)(n_comp - t0 < kRestTile ? n_comp - t0 : kRestTile);
        __syncthreads();
        for (int i = threadIdx.x; i < nt; i += kGridBlock) {
            const int64_t q = comp_pix[t0 + i];
            s_y[i] = (double)(q / nx);
            s_x[i] = (double)(q - (q / nx) * nx);
            s_g[i] = comp_val[t0 + i];
        }
        __syncthreads();
        for (int i = 0; i < nt; ++i) {
            const double dx = ix - s_x[i], dy = iy - s_y[i];
            s += s_g[i] * exp(-(a * dx * dx + b2 * dx * dy + c * dy * dy));
        }
    }
    if (p < n) out[p] = residual ? s + residual[p] : s;
}

unsigned grid_blocks(int64_t n) { return (unsigned)((n + kGridBlock - 1) / kGridBlock); }

__global__ void k_zero_u64(int64_t n, unsigned long long* p) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Below this many pixels one workgroup is as fast as an exchange per iteration.
constexpr int kHogGridMinPixels = 16384;
constexpr int kHogGridMaxBlocks = 64;

bool coop_supported(int device) {
    int v = 0;
    return hipDeviceGetAttribute(&v, hipDeviceAttributeCooperativeLaunch, device) == hipSuccess &&
           v != 0;
}

int check_grid(int nx, int ny, double cell) {
    if (nx < 1 || ny < 1 || nx > 32768 || ny > 32768 || (int64_t)nx * ny > (1 << 30))
        return fail(SWV_EINVAL, "grid %d x %d outside 1 .. 32768 per side, 2^30 pixels", nx, ny);
    if (!(cell > 0.0) || !std::isfinite(cell))
        return fail(SWV_EDOMAIN, "grid cell must be positive and finite");
    return SWV_OK;
}

}  // namespace

}  // namespace swv

using namespace swv;

#define CLEAN_CHECK_CTX(ctx) \
    if (!(ctx)) return fail(SWV_EINVAL, "%s: null context", __func__)
#define CLEAN_GUARD(ctx)                   \
    DeviceGuard guard_((ctx)->device);     \
    if (!guard_.ok) return fail(SWV_EHIP, "%s: cannot select device %d", __func__, (ctx)->device)
#define CLEAN_HIP(expr)                                      \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);    \
    } while (0)
#define CLEAN_RC(expr)          \
    do {                        \
        const int rc_ = (expr); \
        if (rc_) return rc_;    \
    } while (0)

extern "C" int swv_image_grid(swv_ctx ctx, int nx, int ny, int cx, int cy, double cell,
                              double* l, double* m, double* nm1) {
    CLEAN_CHECK_CTX(ctx);
    CLEAN_RC(check_grid(nx, ny, cell));
    if (!l || !m || !nm1) return fail(SWV_EINVAL, "swv_image_grid: null output");
    CLEAN_GUARD(ctx);
    const int64_t n = (int64_t)nx * ny;
    k_grid<<<grid_blocks(n), kGridBlock, 0, ctx->stream>>>(n, nx, cx, cy, cell, l, m, nm1);
    CLEAN_HIP(hipGetLastError());
    return SWV_OK;
}

extern "C" int swv_dirty_image(swv_ctx ctx, int64_t n_vis, const double* u, const double* v,
                               const double* w, const void* y, int nx, int ny, int cx, int cy,
                               double cell, int sign, int prec, double* img_out) {
    CLEAN_CHECK_CTX(ctx);
    CLEAN_RC(check_grid(nx, ny, cell));
    if (n_vis < 1) return fail(SWV_EINVAL, "swv_dirty_image: no visibilities");
    if (!u || !v || !w || !img_out) return fail(SWV_EINVAL, "swv_dirty_image: null argument");
    if (sign != 1 && sign != -1) return fail(SWV_EDOMAIN, "sign must be +1 or -1 (got %d)", sign);
    if (prec != SWV_FP64 && prec != SWV_F32C)
        return fail(SWV_EINVAL, "swv_dirty_image: unsupported precision %d", prec);
    CLEAN_GUARD(ctx);
    const int64_t n = (int64_t)nx * ny;
    CLEAN_RC(ensure(ctx, ctx->grid, 40 * (size_t)n));
    // the complex adjoint output first, so that it is 16-byte aligned for any n
    double2* gx = (double2*)ctx->grid.p;
    double* gl = (double*)(gx + n);
    double* gm = gl + n;
    double* gn = gm + n;
    const double2* yy = (const double2*)y;
    if (!yy) {
        if (ctx->ones.n < 16 * (size_t)n_vis) {
            CLEAN_RC(ensure(ctx, ctx->ones, 16 * (size_t)n_vis));
            // fill the whole buffer: later calls with fewer rows reuse it
            const int64_t cap = (int64_t)(ctx->ones.n / 16);
            k_fill_unit<<<grid_blocks(cap), kGridBlock, 0, ctx->stream>>>(cap, (double2*)ctx->ones.p);
            CLEAN_HIP(hipGetLastError());
        }
        yy = (const double2*)ctx->ones.p;
    }
    k_grid<<<grid_blocks(n), kGridBlock, 0, ctx->stream>>>(n, nx, cx, cy, cell, gl, gm, gn);
    CLEAN_HIP(hipGetLastError());
    CLEAN_RC(swv_adjoint(ctx, n_vis, u, v, w, yy, n, gl, gm, gn, sign, prec, gx));
    k_real_image<<<grid_blocks(n), kGridBlock, 0, ctx->stream>>>(n, gx, nx, cx, cy, cell,
                                                                 (double)n_vis, img_out);
    CLEAN_HIP(hipGetLastError());
    return SWV_OK;
}

extern "C" int swv_hogbom(swv_ctx ctx, int nx, int ny, double* image, const double* beam,
                          double gain, double threshold, int64_t max_iter, int flags,
                          int64_t* comp_pix, double* comp_val, int64_t* n_found) {
    CLEAN_CHECK_CTX(ctx);
    CLEAN_RC(check_grid(nx, ny, 1.0));
    if (!image || !beam || !n_found) return fail(SWV_EINVAL, "swv_hogbom: null argument");
    if (max_iter < 0) return fail(SWV_EINVAL, "swv_hogbom: negative max_iter");
    if (max_iter > 0 && (!comp_pix || !comp_val))
        return fail(SWV_EINVAL, "swv_hogbom: null component arrays");
    if (!std::isfinite(gain) || std::isnan(threshold))
        return fail(SWV_EDOMAIN, "swv_hogbom: gain must be finite, threshold a number");
    if (flags & ~(SWV_HOGBOM_ABS | SWV_HOGBOM_SINGLE))
        return fail(SWV_EINVAL, "swv_hogbom: unknown flags %d", flags);
    CLEAN_GUARD(ctx);
    const int n = nx * ny;
    if (n >= kHogGridMinPixels && !(flags & SWV_HOGBOM_SINGLE) && coop_supported(ctx->device)) {
        // about four pixels per thread, at most kHogGridMaxBlocks workgroups: the
        // exchange (every workgroup polls every slot) grows with their square
        int G = (n + 4 * kHogGridBlock - 1) / (4 * kHogGridBlock);
        G = G < kHogGridMaxBlocks ? G : kHogGridMaxBlocks;
        G = G < ctx->n_cu ? G : ctx->n_cu;
        CLEAN_RC(ensure(ctx, ctx->hog, 64 * (size_t)G));
        unsigned long long* slots = (unsigned long long*)ctx->hog.p;
        // iteration numbers start from a clean slate (a fill kernel, no memset)
        k_zero_u64<<<(unsigned)((8 * G + 255) / 256), 256, 0, ctx->stream>>>(8 * (int64_t)G, slots);
        CLEAN_HIP(hipGetLastError());
        void* args[] = {&image, (void*)&beam, &nx, &ny, &gain, &threshold, &max_iter, &comp_pix,
                        &comp_val, &n_found, &slots};
        const void* fn = (flags & SWV_HOGBOM_ABS) ? (const void*)k_hogbom_grid<true>
                                                  : (const void*)k_hogbom_grid<false>;
        const hipError_t e = hipLaunchCooperativeKernel(fn, dim3(G), dim3(kHogGridBlock), args, 0,
                                                        ctx->stream);
        if (e == hipSuccess) return SWV_OK;
        // a grid that cannot be resident at once is refused before it starts
        (void)hipGetLastError();
    }
    if (flags & SWV_HOGBOM_ABS)
        k_hogbom<true><<<1, kHogBlock, 0, ctx->stream>>>(image, beam, nx, ny, gain, threshold,
                                                         max_iter, comp_pix, comp_val, n_found);
    else
        k_hogbom<false><<<1, kHogBlock, 0, ctx->stream>>>(image, beam, nx, ny, gain, threshold,
                                                          max_iter, comp_pix, comp_val, n_found);
    CLEAN_HIP(hipGetLastError());
    return SWV_OK;
}

extern "C" int swv_cross_reference(int J, double ra_p, double dec_p, int nx, int ny, double cell,
                                   int64_t* pix) {
    if (J < 1 || J > SWV_MAX_LEVEL) return fail(SWV_EDOMAIN, "J = %d outside [1, 29]", J);
    CLEAN_RC(check_grid(nx, ny, cell));
    if (!pix) return fail(SWV_EINVAL, "swv_cross_reference: null pix");
    if (!std::isfinite(ra_p) || !std::isfinite(dec_p))
        return fail(SWV_EDOMAIN, "swv_cross_reference: non-finite phase centre");
    CLEAN_RC(cross_reference(J, ra_p, dec_p, nx, ny, cell, pix));
    clear_error();
    return SWV_OK;
}

extern "C" int swv_tree_build_pixels(int J, double ra_p, double dec_p, int64_t n,
                                     const int64_t* pix, const double* flux, swv_tree* out) {
    if (!out) return fail(SWV_EINVAL, "swv_tree_build_pixels: null out");
    *out = nullptr;
    if (J < 1 || J > SWV_MAX_LEVEL) return fail(SWV_EDOMAIN, "J = %d outside [1, 29]", J);
    if (n < 0) return fail(SWV_EINVAL, "swv_tree_build_pixels: negative n");
    if (n > 0 && (!pix || !flux)) return fail(SWV_EINVAL, "swv_tree_build_pixels: null array");
    if (!std::isfinite(ra_p) || !std::isfinite(dec_p))
        return fail(SWV_EDOMAIN, "swv_tree_build_pixels: non-finite phase centre");
    const int64_t np = n_pixels(J);
    for (int64_t i = 0; i < n; ++i) {
        if (pix[i] < 0 || pix[i] >= np)
            return fail(SWV_EDOMAIN, "swv_tree_build_pixels: pixel %lld outside level %d",
                        (long long)pix[i], J);
        if (!std::isfinite(flux[i]))
            return fail(SWV_EDOMAIN, "swv_tree_build_pixels: non-finite flux at %lld",
                        (long long)i);
    }
    try {
        auto* t = new swv_tree_s();
        const int rc = build_tree_pixels(J, ra_p, dec_p, n, pix, flux, t);
        if (rc) {
            delete t;
            return rc;
        }
        *out = t;
    } catch (const std::bad_alloc&) {
        return fail(SWV_ENOMEM, "swv_tree_build_pixels: host allocation failed");
    }
    clear_error();
    return SWV_OK;
}

extern "C" int swv_fit_clean_beam(int nbx, int nby, const double* beam, double* abc) {
    if (nbx < 1 || nby < 1 || !beam || !abc) return fail(SWV_EINVAL, "swv_fit_clean_beam: bad argument");
    for (int64_t i = 0; i < (int64_t)nbx * nby; ++i)
        if (!std::isfinite(beam[i])) return fail(SWV_EDOMAIN, "swv_fit_clean_beam: non-finite beam");
    try {
        CLEAN_RC(fit_clean_beam(nbx, nby, beam, abc));
    } catch (const std::bad_alloc&) {
        return fail(SWV_ENOMEM, "swv_fit_clean_beam: host allocation failed");
    }
    clear_error();
    return SWV_OK;
}

extern "C" int swv_restore(swv_ctx ctx, int nx, int ny, int64_t n_comp, const int64_t* comp_pix,
                           const double* comp_val, const double* abc, const double* residual,
                           double* out) {
    CLEAN_CHECK_CTX(ctx);
    CLEAN_RC(check_grid(nx, ny, 1.0));
    if (n_comp < 0) return fail(SWV_EINVAL, "swv_restore: negative n_comp");
    if (!abc || !out || (n_comp > 0 && (!comp_pix || !comp_val)))
        return fail(SWV_EINVAL, "swv_restore: null argument");
    if (!std::isfinite(abc[0]) || !std::isfinite(abc[1]) || !std::isfinite(abc[2]))
        return fail(SWV_EDOMAIN, "swv_restore: non-finite beam parameters");
    CLEAN_GUARD(ctx);
    const int64_t n = (int64_t)nx * ny;
    k_restore<<<grid_blocks(n), kGridBlock, 0, ctx->stream>>>(nx, n, n_comp, comp_pix, comp_val,
                                                              abc[0], abc[1], abc[2], residual, out);
    CLEAN_HIP(hipGetLastError());
    return SWV_OK;
}

namespace {

// Owns the per-call device scratch and events of swv_wavelet_clean.
struct CleanScratch {
    void* p[5] = {};
    hipEvent_t ev[2] = {};
    swv_tree tree = nullptr;
    ~CleanScratch() {
        for (void* q : p)
            if (q) (void)hipFree(q);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (tree) (void)swv_tree_destroy(tree);
    }
};

}  // namespace

extern "C" int swv_wavelet_clean(swv_ctx ctx, const swv_clean_params_t* P, int64_t n_vis,
                                 const double* u, const double* v, const double* w,
                                 const void* vis_obs, double* beam, double* residual,
                                 void* vis_model, int64_t cap, int64_t* comp_pix,
                                 double* comp_val, int64_t* n_comp, swv_clean_stats_t* stats) {
    CLEAN_CHECK_CTX(ctx);
    if (!P) return fail(SWV_EINVAL, "swv_wavelet_clean: null params");
    CLEAN_RC(check_grid(P->nx, P->ny, P->cell));
    if (P->J < 1 || P->J > SWV_MAX_LEVEL) return fail(SWV_EDOMAIN, "J = %d outside [1, 29]", P->J);
    if (n_vis < 1 || !u || !v || !w || !vis_obs || !beam || !residual || !vis_model || !n_comp)
        return fail(SWV_EINVAL, "swv_wavelet_clean: null argument or no visibilities");
    if (P->minor_iter < 0 || P->n_major < 0 || P->n_major > SWV_CLEAN_MAX_CYCLES)
        return fail(SWV_EINVAL, "swv_wavelet_clean: minor_iter >= 0, 0 <= n_major <= %d",
                    SWV_CLEAN_MAX_CYCLES);
    const int64_t need = P->minor_iter * (int64_t)P->n_major;
    if (cap < need || (need > 0 && (!comp_pix || !comp_val)))
        return fail(SWV_EINVAL, "swv_wavelet_clean: component arrays hold %lld, need %lld",
                    (long long)cap, (long long)need);
    if (P->sign != 1 && P->sign != -1) return fail(SWV_EDOMAIN, "sign must be +1 or -1");
    if (P->predictor != SWV_PREDICT_TREE && P->predictor != SWV_PREDICT_DEGRID &&
        P->predictor != SWV_PREDICT_DIRECT)
        return fail(SWV_EINVAL, "swv_wavelet_clean: unknown predictor %d", P->predictor);
    if (P->image_prec != SWV_FP64 && P->image_prec != SWV_F32C)
        return fail(SWV_EINVAL, "swv_wavelet_clean: unsupported image precision %d",
                    P->image_prec);
    if (P->predictor == SWV_PREDICT_DEGRID && (P->support < 2 || P->support > 16))
        return fail(SWV_EINVAL, "swv_wavelet_clean: support %d outside 2 .. 16", P->support);
    if (!std::isfinite(P->gain) || std::isnan(P->threshold))
        return fail(SWV_EDOMAIN, "swv_wavelet_clean: gain must be finite, threshold a number");
    const int nx = P->nx, ny = P->ny;
    const int64_t n_pix = (int64_t)nx * ny;
    *n_comp = 0;
    if (stats) *stats = swv_clean_stats_t{};
    try {
        // cross-reference table: once per run, before cleaning (section 3.5)
        std::vector<int64_t> xref((size_t)n_pix);
        CLEAN_RC(cross_reference(P->J, P->ra_p, P->dec_p, nx, ny, P->cell, xref.data()));
        CLEAN_GUARD(ctx);
        const hipStream_t s = ctx->stream;
        CleanScratch S;
        const int64_t ncap = need > 0 ? need : 1;
        CLEAN_HIP(hipMalloc(&S.p[0], 8 * (size_t)ncap));   // component pixels
        CLEAN_HIP(hipMalloc(&S.p[1], 8 * (size_t)ncap));   // component values
        CLEAN_HIP(hipMalloc(&S.p[2], 16 * (size_t)n_vis));  // residual visibilities
        CLEAN_HIP(hipMalloc(&S.p[3], 256));                 // n_found, chi^2
        CLEAN_HIP(hipEventCreate(&S.ev[0]));
        CLEAN_HIP(hipEventCreate(&S.ev[1]));
        int64_t* d_pix = (int64_t*)S.p[0];
        double* d_val = (double*)S.p[1];
        int64_t* d_found = (int64_t*)S.p[3];
        double* d_chi2 = (double*)S.p[3] + 1;
        const auto lap = [&](double* ms) -> int {
            CLEAN_HIP(hipEventRecord(S.ev[1], s));
            CLEAN_HIP(hipEventSynchronize(S.ev[1]));
            float t = 0.f;
            CLEAN_HIP(hipEventElapsedTime(&t, S.ev[0], S.ev[1]));
            if (ms) *ms = t;
            CLEAN_HIP(hipEventRecord(S.ev[0], s));
            return SWV_OK;
        };
        double scratch_ms = 0.0;
        CLEAN_HIP(hipEventRecord(S.ev[0], s));
        // the beam once, in the images' precision
        CLEAN_RC(swv_dirty_image(ctx, n_vis, u, v, w, nullptr, 2 * nx - 1, 2 * ny - 1, nx - 1,
                                 ny - 1, P->cell, P->sign, P->image_prec, beam));
        CLEAN_RC(lap(stats ? &stats->ms_beam : &scratch_ms));
        CLEAN_RC(swv_dirty_image(ctx, n_vis, u, v, w, vis_obs, nx, ny, nx / 2, ny / 2, P->cell,
                                 P->sign, P->image_prec, residual));
        CLEAN_RC(lap(stats ? &stats->ms_dirty : &scratch_ms));
        CLEAN_HIP(hipMemsetAsync(vis_model, 0, 16 * (size_t)n_vis, s));
        int64_t total = 0;
        std::vector<int64_t> kj;
        std::vector<double> model, ml, mm, mf;
        double* d_model = nullptr;
        if (P->predictor != SWV_PREDICT_TREE) {
            model.assign((size_t)n_pix, 0.0);
            CLEAN_HIP(hipMalloc(&S.p[4], 24 * (size_t)n_pix));
            d_model = (double*)S.p[4];
        }
        for (int cyc = 0; cyc < P->n_major; ++cyc) {
            CLEAN_RC(swv_hogbom(ctx, nx, ny, residual, beam, P->gain, P->threshold, P->minor_iter,
                                P->flags, d_pix + total, d_val + total, d_found));
            int64_t found = 0;
            CLEAN_HIP(hipMemcpyAsync(&found, d_found, 8, hipMemcpyDeviceToHost, s));
            double ms_minor = 0.0;
            CLEAN_RC(lap(&ms_minor));   // synchronises: `found` is valid
            if (found < 0)
                return fail(SWV_EHIP, "swv_wavelet_clean: the grid-wide minor cycle timed out");
            if (found == 0) break;
            CLEAN_HIP(hipMemcpyAsync(comp_pix + total, d_pix + total, 8 * (size_t)found,
                                     hipMemcpyDeviceToHost, s));
            CLEAN_HIP(hipMemcpyAsync(comp_val + total, d_val + total, 8 * (size_t)found,
                                     hipMemcpyDeviceToHost, s));
            CLEAN_HIP(hipStreamSynchronize(s));
            total += found;
            const auto t0 = std::chrono::steady_clock::now();
            int64_t leaves = 0;
            if (P->predictor == SWV_PREDICT_TREE) {
                // the model tree of every component so far, from the cross-referenced pixels
                kj.resize((size_t)total);
                for (int64_t i = 0; i < total; ++i) kj[(size_t)i] = xref[(size_t)comp_pix[i]];
                if (S.tree) {
                    (void)swv_tree_destroy(S.tree);   // the stream is idle here
                    S.tree = nullptr;
                }
                CLEAN_RC(swv_tree_build_pixels(P->J, P->ra_p, P->dec_p, total, kj.data(),
                                               comp_val, &S.tree));
                swv_tree_stats_t ts;
                (void)swv_tree_stats(S.tree, &ts);
                leaves = ts.n_leaves;
            } else {
                // the model image: components summed per pixel in list order
                std::fill(model.begin(), model.end(), 0.0);
                for (int64_t i = 0; i < total; ++i) model[(size_t)comp_pix[i]] += comp_val[i];
                if (P->predictor == SWV_PREDICT_DIRECT) {
                    ml.clear();
                    mm.clear();
                    mf.clear();
                    for (int64_t p = 0; p < n_pix; ++p)
                        if (model[(size_t)p] != 0.0) {
                            const int64_t iy = p / nx, ix = p - iy * nx;
                            ml.push_back((double)(ix - nx / 2) * P->cell);
                            mm.push_back((double)(iy - ny / 2) * P->cell);
                            mf.push_back(model[(size_t)p]);
                        }
                    leaves = (int64_t)mf.size();
                    for (const auto* a : {&ml, &mm, &mf}) {
                        const size_t k = (a == &ml ? 0 : a == &mm ? 1 : 2);
                        CLEAN_HIP(hipMemcpyAsync(d_model + k * (size_t)n_pix, a->data(),
                                                 8 * a->size(), hipMemcpyHostToDevice, s));
                    }
                } else {
                    for (int64_t p = 0; p < n_pix; ++p) leaves += model[(size_t)p] != 0.0;
                    CLEAN_HIP(hipMemcpyAsync(d_model, model.data(), 8 * (size_t)n_pix,
                                             hipMemcpyHostToDevice, s));
                }
            }
            const double ms_build =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                    .count();
            CLEAN_HIP(hipEventRecord(S.ev[0], s));
            if (P->predictor == SWV_PREDICT_TREE)
                CLEAN_RC(swv_predict_tree(ctx, S.tree, n_vis, u, v, w, P->sign, SWV_FP64,
                                          vis_model));
            else if (P->predictor == SWV_PREDICT_DEGRID)
                CLEAN_RC(swv_predict_degrid(ctx, nx, ny, P->cell, d_model, n_vis, u, v, w,
                                            P->support, P->sign, vis_model, nullptr));
            else
                CLEAN_RC(swv_predict_direct(ctx, n_vis, u, v, w, leaves, d_model,
                                            d_model + n_pix, d_model + 2 * n_pix, P->sign,
                                            SWV_FP64, vis_model));
            double ms_predict = 0.0, ms_image = 0.0;
            CLEAN_RC(lap(&ms_predict));
            CLEAN_RC(swv_residual_chi2(ctx, n_vis, vis_obs, vis_model, 1.0, S.p[2], d_chi2));
            CLEAN_RC(swv_dirty_image(ctx, n_vis, u, v, w, S.p[2], nx, ny, nx / 2, ny / 2,
                                     P->cell, P->sign, P->image_prec, residual));
            double chi2 = 0.0;
            CLEAN_HIP(hipMemcpyAsync(&chi2, d_chi2, 8, hipMemcpyDeviceToHost, s));
            CLEAN_RC(lap(&ms_image));
            if (stats) {
                stats->found[cyc] = found;
                stats->leaves[cyc] = leaves;
                stats->chi2[cyc] = chi2;
                stats->ms_minor[cyc] = ms_minor;
                stats->ms_build[cyc] = ms_build;
                stats->ms_predict[cyc] = ms_predict;
                stats->ms_image[cyc] = ms_image;
                stats->n_cycles = cyc + 1;
            }
        }
        *n_comp = total;
        CLEAN_HIP(hipStreamSynchronize(s));
    } catch (const std::bad_alloc&) {
        return fail(SWV_ENOMEM, "swv_wavelet_clean: host allocation failed");
    }
    clear_error();
    return SWV_OK;
}
