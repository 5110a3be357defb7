// The conventional predictor the wavelet route is compared against (section
// 2.2, first step of the major cycle: a forward FFT of the model image, then
// degridding with an anti-aliasing kernel and a w correction).  Written as a
// type-2 non-uniform FFT in (u, v, w):
//   * the model image is divided by the Fourier transform of the kernel in
//     all three directions, multiplied per w plane by exp(s 2 pi i w_q (n - 1 - c)),
//     zero-padded twofold and transformed (one batched hipFFT over the planes);
//   * every visibility then gathers W x W cells from each of the W planes
//     around it, weighted by the "exponential of semicircle" kernel
//     phi(z) = exp(beta (sqrt(1 - z^2) - 1)) (Barnett, Magland & af Klinteberg
//     2019), the w planes being interpolated like u and v (the improved
//     w-stacking of Ye et al. 2021).
// The result approximates the direct sum over the image pixels to about
// 10^(1 - W).
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <vector>

#include "api_internal.h"
#include "device_math.h"

namespace swv {

namespace {

constexpr int kDgBlock = 256;
constexpr int kQuad = 100;           // Gauss-Legendre nodes of the kernel transform
constexpr int kMaxSupport = 16;
constexpr double kBetaPerW = 2.3;
constexpr double kTwoPi = 6.283185307179586476925286766559;

// Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on P_n, with
// P_n from the three-term recurrence k P_k = (2k - 1) z P_{k-1} - (k - 1) P_{k-2}
// and P_n' = n (z P_n - P_{n-1}) / (z^2 - 1); weights 2 / ((1 - z^2) P_n'^2).
void gauss_legendre(int n, double* x, double* wt) {
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double pn = 0, dpn = 1;
        for (int it = 0; it < 12; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            pn = p1;
            dpn = n * (z * p1 - p0) / (z * z - 1.0);
            z -= pn / dpn;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dpn = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        x[n - 1 - i] = z;
        wt[i] = wt[n - 1 - i] = 2.0 / ((1.0 - z * z) * dpn * dpn);
    }
}

__host__ __device__ __forceinline__ double es_phi(double z, double beta) {
    const double t = 1.0 - z * z;
    return t >= 0.0 ? exp(beta * (sqrt(t) - 1.0)) : 0.0;
}

// phi_hat(f) = sum_k coef_k cos(2 pi f x_k): Gauss-Legendre in theta with
// x = (W / 2) sin(theta), coef_k = exp(beta (cos theta_k - 1)) cos theta_k w_k (pi / 2) (W / 2)
__device__ double es_hat(double f, const double* __restrict__ xk,
                         const double* __restrict__ coef) {
    double s = 0.0;
    for (int k = 0; k < kQuad; ++k) s += coef[k] * cos(kTwoPi * f * xk[k]);
    return s;
}

__global__ __launch_bounds__(kDgBlock) void k_hat_1d(int n, const double* __restrict__ f,
                                                     const double* __restrict__ xk,
                                                     const double* __restrict__ coef,
                                                     double* __restrict__ out) {
    const int i = blockIdx.x * kDgBlock + threadIdx.x;
    if (i < n) out[i] = es_hat(f[i], xk, coef);
}

// base[p] = I[p] / (hy hx hw), sn[p] = n_p - 1 - c
__global__ __launch_bounds__(kDgBlock) void k_degrid_prep(
    int nx, int ny, double cell, double c, double dw, const double* __restrict__ image,
    const double* __restrict__ hx, const double* __restrict__ hy, const double* __restrict__ xk,
    const double* __restrict__ coef, double* __restrict__ base, double* __restrict__ sn) {
    const int64_t p = (int64_t)blockIdx.x * kDgBlock + threadIdx.x;
    if (p >= (int64_t)nx * ny) return;
    const int iy = (int)(p / nx), ix = (int)(p - (int64_t)iy * nx);
    const double l = (double)(ix - nx / 2) * cell, m = (double)(iy - ny / 2) * cell;
    const double r2 = l * l + m * m;
    const double s = -r2 / (1.0 + sqrt(1.0 - r2)) - c;
    const double hw = es_hat(dw * s, xk, coef);
    base[p] = image[p] / (hy[iy] * hx[ix] * hw);
    sn[p] = s;
}

// Plane q, padded cell (ky, kx): the image pixel at offset t = k (k below the
// image's positive half) or t = k - N (the wrapped negative half), else 0.
__global__ __launch_bounds__(kDgBlock) void k_fill_planes(
    int nx, int ny, int Nx, int Ny, int64_t n_planes, double w0, double dw, int sign,
    const double* __restrict__ base, const double* __restrict__ sn, double2* __restrict__ G) {
    const int64_t cells = (int64_t)Nx * Ny;
    const int64_t i = (int64_t)blockIdx.x * kDgBlock + threadIdx.x;
    if (i >= n_planes * cells) return;
    const int64_t q = i / cells;
    const int64_t r = i - q * cells;
    const int ky = (int)(r / Nx), kx = (int)(r - (int64_t)ky * Nx);
    const int cx = nx / 2, cy = ny / 2;
    int ty = ky <= ny - 1 - cy ? ky : (ky >= Ny - cy ? ky - Ny : INT_MIN);
    int tx = kx <= nx - 1 - cx ? kx : (kx >= Nx - cx ? kx - Nx : INT_MIN);
    double2 out = make_double2(0.0, 0.0);
    if (ty != INT_MIN && tx != INT_MIN) {
        const int64_t p = (int64_t)(ty + cy) * nx + (tx + cx);
        const double wq = w0 + (double)q * dw;
        const double t = wq * sn[p];
        double cs, q4;
        cis2pi_q(t - rint(t), cs, q4);
        const double b = base[p];
        out = make_double2(b * cs, b * (sign * 4.0 * q4));
    }
    G[i] = out;
}

// One visibility per thread.  T = W + 1 cells per direction starting at
// ceil(x - W/2): the last one lies outside the support unless x - W/2 is an
// integer, and then takes weight phi(+-1) like the first; outside it the
// weight is exactly 0.
template <int W>
__global__ __launch_bounds__(kDgBlock) void k_degrid(
    int64_t n_vis, const double* __restrict__ u, const double* __restrict__ v,
    const double* __restrict__ w, int Nx, int Ny, int64_t n_planes, double cell, double w0,
    double dw, double c, double beta, int sign, const double2* __restrict__ G,
    double2* __restrict__ out) {
    constexpr int T = W + 1;
    const int64_t j = (int64_t)blockIdx.x * kDgBlock + threadIdx.x;
    if (j >= n_vis) return;
    const double h = 0.5 * W;
    const double xi = u[j] * Nx * cell, zeta = v[j] * Ny * cell, eta = (w[j] - w0) / dw;
    // non-finite or absurd coordinates give NaN, never an index
    if (!(fabs(xi) < 0x1p50 && fabs(zeta) < 0x1p50 && eta >= 0.0 && eta <= (double)n_planes)) {
        out[j] = make_double2(NAN, NAN);
        return;
    }
    const int64_t x0 = (int64_t)ceil(xi - h), y0 = (int64_t)ceil(zeta - h);
    const int64_t q0 = (int64_t)ceil(eta - h);
    double fx[T], fy[T];
    int cxk[T];
#pragma unroll
    for (int a = 0; a < T; ++a) {
        fx[a] = es_phi((xi - (double)(x0 + a)) / h, beta);
        fy[a] = es_phi((zeta - (double)(y0 + a)) / h, beta);
        int64_t k = (x0 + a) % Nx;
        cxk[a] = (int)(k < 0 ? k + Nx : k);
    }
    double vr = 0.0, vi = 0.0;
#pragma unroll 1
    for (int b3 = 0; b3 < T; ++b3) {
        const int64_t q = q0 + b3;
        if (q < 0 || q >= n_planes) continue;
        const double fq = es_phi((eta - (double)q) / h, beta);
        if (fq == 0.0) continue;
        const double2* Gq = G + q * (int64_t)Nx * Ny;
        double pr = 0.0, pi = 0.0;
#pragma unroll 1
        for (int b = 0; b < T; ++b) {
            int64_t ky = (y0 + b) % Ny;
            ky = ky < 0 ? ky + Ny : ky;
            const double2* row = Gq + ky * Nx;
            double rr = 0.0, ri = 0.0;
#pragma unroll
            for (int a = 0; a < T; ++a) {
                const double2 g = row[cxk[a]];
                rr = fma(fx[a], g.x, rr);
                ri = fma(fx[a], g.y, ri);
            }
            pr = fma(fy[b], rr, pr);
            pi = fma(fy[b], ri, pi);
        }
        vr = fma(fq, pr, vr);
        vi = fma(fq, pi, vi);
    }
    const double t = w[j] * c;
    double cs, q4;
    cis2pi_q(t - rint(t), cs, q4);
    const double sn = sign * 4.0 * q4;
    out[j] = make_double2(vr * cs - vi * sn, vr * sn + vi * cs);
}

template <int W>
void launch_degrid_w(hipStream_t s, int64_t n_vis, const double* u, const double* v,
                     const double* w, int Nx, int Ny, int64_t nq, double cell, double w0,
                     double dw, double c, double beta, int sign, const double2* G, double2* out) {
    k_degrid<W><<<(unsigned)((n_vis + kDgBlock - 1) / kDgBlock), kDgBlock, 0, s>>>(
        n_vis, u, v, w, Nx, Ny, nq, cell, w0, dw, c, beta, sign, G, out);
}

using DegridFn = void (*)(hipStream_t, int64_t, const double*, const double*, const double*, int,
                          int, int64_t, double, double, double, double, double, int,
                          const double2*, double2*);
constexpr DegridFn kDegrid[] = {
    nullptr, nullptr, launch_degrid_w<2>, launch_degrid_w<3>, launch_degrid_w<4>,
    launch_degrid_w<5>, launch_degrid_w<6>, launch_degrid_w<7>, launch_degrid_w<8>,
    launch_degrid_w<9>, launch_degrid_w<10>, launch_degrid_w<11>, launch_degrid_w<12>,
    launch_degrid_w<13>, launch_degrid_w<14>, launch_degrid_w<15>, launch_degrid_w<16>};

// w range: kMinmaxBlocks partial (min, max) pairs, then one block combines them.
constexpr int kMinmaxBlocks = 512;

__device__ __forceinline__ void block_minmax(double& lo, double& hi, double* smin,
                                             double* smax) {
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int s = kDgBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
        }
        __syncthreads();
    }
    lo = smin[0];
    hi = smax[0];
}

__global__ __launch_bounds__(kDgBlock) void k_minmax_partial(int64_t n,
                                                             const double* __restrict__ x,
                                                             double* __restrict__ part) {
    __shared__ double smin[kDgBlock], smax[kDgBlock];
    double lo = HUGE_VAL, hi = -HUGE_VAL;
    for (int64_t i = (int64_t)blockIdx.x * kDgBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kDgBlock) {
        lo = fmin(lo, x[i]);
        hi = fmax(hi, x[i]);
    }
    block_minmax(lo, hi, smin, smax);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = lo;
        part[2 * blockIdx.x + 1] = hi;
    }
}

__global__ __launch_bounds__(kDgBlock) void k_minmax_final(int n_part,
                                                           const double* __restrict__ part,
                                                           double* __restrict__ out) {
    __shared__ double smin[kDgBlock], smax[kDgBlock];
    double lo = HUGE_VAL, hi = -HUGE_VAL;
    for (int i = threadIdx.x; i < n_part; i += kDgBlock) {
        lo = fmin(lo, part[2 * i]);
        hi = fmax(hi, part[2 * i + 1]);
    }
    block_minmax(lo, hi, smin, smax);
    if (threadIdx.x == 0) {
        out[0] = lo;
        out[1] = hi;
    }
}

unsigned blocks_of(int64_t n) { return (unsigned)((n + kDgBlock - 1) / kDgBlock); }

}  // namespace

void destroy_fft_plan(void* plan) {
    if (plan) (void)hipfftDestroy((hipfftHandle)plan);
}

}  // namespace swv

using namespace swv;

extern "C" int swv_predict_degrid(swv_ctx ctx, int nx, int ny, double cell, const double* image,
                                  int64_t n_vis, const double* u, const double* v,
                                  const double* w, int support, int sign, void* vis_out,
                                  swv_degrid_stats_t* stats) {
    if (!ctx) return fail(SWV_EINVAL, "swv_predict_degrid: null context");
    if (nx < 1 || ny < 1 || nx > 16384 || ny > 16384)
        return fail(SWV_EINVAL, "swv_predict_degrid: grid %d x %d outside 1 .. 16384", nx, ny);
    if (!(cell > 0.0) || !std::isfinite(cell))
        return fail(SWV_EDOMAIN, "swv_predict_degrid: cell must be positive and finite");
    if (support < 2 || support > kMaxSupport)
        return fail(SWV_EINVAL, "swv_predict_degrid: support %d outside 2 .. 16", support);
    if (sign != 1 && sign != -1) return fail(SWV_EDOMAIN, "sign must be +1 or -1 (got %d)", sign);
    if (n_vis < 0) return fail(SWV_EINVAL, "swv_predict_degrid: negative n_vis");
    if (!image || (n_vis > 0 && (!u || !v || !w || !vis_out)))
        return fail(SWV_EINVAL, "swv_predict_degrid: null argument");
    // n - 1 over the grid: 0 at the centre pixel, lowest at the farthest corner
    const int cx = nx / 2, cy = ny / 2;
    double lo = 0.0;
    for (int ix : {0, nx - 1})
        for (int iy : {0, ny - 1}) {
            const double l = (double)(ix - cx) * cell, m = (double)(iy - cy) * cell;
            const double r2 = l * l + m * m;
            if (!(r2 < 1.0)) return fail(SWV_EDOMAIN, "swv_predict_degrid: grid leaves the unit disk");
            lo = std::fmin(lo, -r2 / (1.0 + std::sqrt(1.0 - r2)));
        }
    const double hi = 0.0;
    const double extent = std::fmax(hi - lo, 1e-300);
    const double c = 0.5 * (lo + hi);
    const double dw = 1.0 / (2.0 * extent);
    const int Nx = 2 * nx, Ny = 2 * ny;
    const double beta = kBetaPerW * support;
    if (stats) *stats = swv_degrid_stats_t{};
    if (n_vis == 0) return SWV_OK;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(SWV_EHIP, "swv_predict_degrid: cannot select device");
    const hipStream_t s = ctx->stream;
    const auto t0 = std::chrono::steady_clock::now();
    // w range of the rows
    int rc = ensure(ctx, ctx->partial2, 16 * (kMinmaxBlocks + 1));
    if (rc) return rc;
    double* d_mm = (double*)ctx->partial2.p;
    const int nb = (int)std::min<int64_t>(kMinmaxBlocks, (n_vis + kDgBlock - 1) / kDgBlock);
    k_minmax_partial<<<nb, kDgBlock, 0, s>>>(n_vis, w, d_mm + 2);
    k_minmax_final<<<1, kDgBlock, 0, s>>>(nb, d_mm + 2, d_mm);
    double mm[2];
    hipError_t e = hipMemcpyAsync(mm, d_mm, 16, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "swv_predict_degrid: w range");
    if (!std::isfinite(mm[0]) || !std::isfinite(mm[1]))
        return fail(SWV_EDOMAIN, "swv_predict_degrid: non-finite w");
    const double w0 = mm[0] - 0.5 * support * dw;
    const double nq_f = std::floor((mm[1] - w0) / dw + 0.5 * support) + 1.0;
    const int64_t cells = (int64_t)Nx * Ny;
    if (!(nq_f * (double)cells * 16.0 <= 64.0 * (1ull << 30)))
        return fail(SWV_ENOMEM,
                    "swv_predict_degrid: %.0f w planes of %d x %d cells exceed 64 GiB "
                    "(field too wide for the w range)", nq_f, Nx, Ny);
    const int64_t nq = (int64_t)nq_f;
    // scratch: planes, then base, sn, hx, hy, quadrature
    const int64_t n_pix = (int64_t)nx * ny;
    const size_t plane_bytes = 16 * (size_t)(nq * cells);
    const size_t extra = 8 * (size_t)(2 * n_pix + 2 * (nx + ny) + 2 * kQuad) + 256;
    rc = ensure(ctx, ctx->degrid, plane_bytes + extra);
    if (rc) return rc;
    double2* G = (double2*)ctx->degrid.p;
    double* base = (double*)((char*)ctx->degrid.p + plane_bytes);
    double* sn = base + n_pix;
    double* hx = sn + n_pix;
    double* hy = hx + nx;
    double* fxy = hy + ny;              // nx + ny transform arguments
    double* xk = fxy + nx + ny;
    double* coef = xk + kQuad;
    {
        std::vector<double> z(kQuad), wt(kQuad), hx_k(kQuad), hc(kQuad), f((size_t)(nx + ny));
        gauss_legendre(kQuad, z.data(), wt.data());
        // x = (W / 2) sin(theta), theta = (pi / 2) z: a smooth integrand
        for (int k = 0; k < kQuad; ++k) {
            const double th = 0.5 * M_PI * z[k];
            hx_k[k] = 0.5 * support * std::sin(th);
            hc[k] = std::exp(beta * (std::cos(th) - 1.0)) * std::cos(th) * wt[k] * (0.5 * M_PI) *
                    (0.5 * support);
        }
        for (int i = 0; i < nx; ++i) f[i] = (double)(i - cx) / Nx;
        for (int i = 0; i < ny; ++i) f[nx + i] = (double)(i - cy) / Ny;
        e = hipMemcpyAsync(xk, hx_k.data(), 8 * kQuad, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(coef, hc.data(), 8 * kQuad, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(fxy, f.data(), 8 * (size_t)(nx + ny), hipMemcpyHostToDevice, s);
        // the host vectors must outlive the copies
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "swv_predict_degrid: upload");
    }
    k_hat_1d<<<blocks_of(nx + ny), kDgBlock, 0, s>>>(nx + ny, fxy, xk, coef, hx);
    k_degrid_prep<<<blocks_of(n_pix), kDgBlock, 0, s>>>(nx, ny, cell, c, dw, image, hx, hy, xk,
                                                        coef, base, sn);
    k_fill_planes<<<blocks_of(nq * cells), kDgBlock, 0, s>>>(nx, ny, Nx, Ny, nq, w0, dw, sign,
                                                             base, sn, G);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "swv_predict_degrid: plane fill");
    // batched 2-D transform of every plane (plan cached per context and shape)
    if (!ctx->fft_plan || ctx->fft_shape[0] != Nx || ctx->fft_shape[1] != Ny ||
        ctx->fft_shape[2] != nq) {
        destroy_fft_plan(ctx->fft_plan);
        ctx->fft_plan = nullptr;
        hipfftHandle plan = nullptr;
        int n2[2] = {Ny, Nx};
        if (hipfftPlanMany(&plan, 2, n2, nullptr, 1, (int)cells, nullptr, 1, (int)cells,
                           HIPFFT_Z2Z, (int)nq) != HIPFFT_SUCCESS)
            return fail(SWV_EHIP, "swv_predict_degrid: hipfftPlanMany failed");
        ctx->fft_plan = (void*)plan;
        ctx->fft_shape[0] = Nx;
        ctx->fft_shape[1] = Ny;
        ctx->fft_shape[2] = (int)nq;
    }
    hipfftHandle plan = (hipfftHandle)ctx->fft_plan;
    if (hipfftSetStream(plan, s) != HIPFFT_SUCCESS ||
        hipfftExecZ2Z(plan, (hipfftDoubleComplex*)G, (hipfftDoubleComplex*)G,
                      sign < 0 ? HIPFFT_FORWARD : HIPFFT_BACKWARD) != HIPFFT_SUCCESS)
        return fail(SWV_EHIP, "swv_predict_degrid: hipfftExecZ2Z failed");
    kDegrid[support](s, n_vis, u, v, w, Nx, Ny, nq, cell, w0, dw, c, beta, sign, G,
                     (double2*)vis_out);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "swv_predict_degrid: degrid");
    if (stats) {
        stats->n_planes = nq;
        stats->grid_nx = Nx;
        stats->grid_ny = Ny;
        stats->w0 = w0;
        stats->dw = dw;
        stats->c = c;
        stats->plane_bytes = (int64_t)plane_bytes;
        stats->host_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                .count();
    }
    clear_error();
    return SWV_OK;
}
