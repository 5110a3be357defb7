// Measured ceilings of the arithmetic the path is built from, on the device
// at hand: FP64 FMA, FP32 FMA (unpacked), the FP32 hardware sine/cosine and
// the FP64 phasor of device_math.h.  Each kernel runs independent dependency
// chains per lane, enough of them and long enough (5-20 ms a launch) that issue
// rate, not latency, is what is measured.  The engine clock ramps up over the
// first tens of milliseconds of a heavy kernel that follows lighter work: four
// back-to-back 15 ms FP64 FMA launches after the direct kernel ran at 2.04,
// 2.23, 2.36 and 2.37 GHz (busy cycles over duration, averaged over the eight
// dies).  Each ceiling is therefore timed after at least 50 ms of warm-up
// launches of the same kernel, as the fastest of five launches.  The results
// scale the published peaks to what a kernel of this library can reach on the
// part.
#include <algorithm>

#include "api_internal.h"
#include "device_math.h"
#include "launch.h"

namespace swv {

constexpr int kPeakBlock = 256;

template <int CHAINS>
__global__ __launch_bounds__(kPeakBlock) void k_peak_fma_f64(double* out, int iters) {
    const int t = blockIdx.x * kPeakBlock + threadIdx.x;
    double x[CHAINS];
#pragma unroll
    for (int k = 0; k < CHAINS; ++k) x[k] = 1.0 + 1e-9 * (t + k);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int k = 0; k < CHAINS; ++k) x[k] = fma(x[k], 0.9999999, 1e-8);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < CHAINS; ++k) s += x[k];
    out[t] = s;
}

template <int CHAINS>
__global__ __launch_bounds__(kPeakBlock) void k_peak_fma_f32(double* out, int iters) {
    const int t = blockIdx.x * kPeakBlock + threadIdx.x;
    float x[CHAINS];
#pragma unroll
    for (int k = 0; k < CHAINS; ++k) x[k] = 1.0f + 1e-6f * (float)((t + k) & 255);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int k = 0; k < CHAINS; ++k) x[k] = fmaf(x[k], 0.999f, 1e-3f);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < CHAINS; ++k) s += x[k];
    out[t] = s;
}

template <int CHAINS>
__global__ __launch_bounds__(kPeakBlock) void k_peak_sincos_f32(double* out, int iters) {
    const int t = blockIdx.x * kPeakBlock + threadIdx.x;
    float x[CHAINS];
#pragma unroll
    for (int k = 0; k < CHAINS; ++k) x[k] = 1e-3f * (float)((t + k) & 255);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int k = 0; k < CHAINS; ++k) {
                float c, s;
                cis2pi_f32(x[k], c, s);
                x[k] = c - s;   // stays within [-2, 2] revolutions
            }
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < CHAINS; ++k) s += x[k];
    out[t] = s;
}

template <int CHAINS>
__global__ __launch_bounds__(kPeakBlock) void k_peak_cis2pi_f64(double* out, int iters) {
    const int t = blockIdx.x * kPeakBlock + threadIdx.x;
    double x[CHAINS];
#pragma unroll
    for (int k = 0; k < CHAINS; ++k) x[k] = 1e-4 * ((t + k) & 1023);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < CHAINS; ++k) {
            double c, q;
            cis2pi_q(x[k], c, q);
            x[k] = fma(0.25, c, q);   // |x| <= 1/2: a valid reduced phase again
        }
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < CHAINS; ++k) s += x[k];
    out[t] = s;
}

namespace {

// Times `launch(iters)`: warm-up launches until 50 ms have run (at most 16),
// then the fastest of five, in seconds.
template <class F>
int time_kernel(hipStream_t s, F&& launch, int iters, double* seconds) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(SWV_EHIP, "swv_measure_peaks: event creation failed");
    }
    auto once = [&](float& ms) {
        (void)hipEventRecord(e0, s);
        launch(iters);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        return e;
    };
    hipError_t e = hipSuccess;
    float warm = 0.0f, best = 0.0f;
    for (int r = 0; r < 16 && warm < 50.0f && e == hipSuccess; ++r) {
        float ms = 0.0f;
        e = once(ms);
        warm += ms;
    }
    for (int r = 0; r < 5 && e == hipSuccess; ++r) {
        float ms = 0.0f;
        e = once(ms);
        if (e == hipSuccess) best = r == 0 ? ms : std::min(best, ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "swv_measure_peaks");
    *seconds = 1e-3 * best;
    return SWV_OK;
}

}  // namespace

}  // namespace swv

using namespace swv;

extern "C" int swv_measure_peaks(swv_ctx ctx, swv_peaks_t* out) {
    if (!ctx || !out) return fail(SWV_EINVAL, "swv_measure_peaks: null argument");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(SWV_EHIP, "swv_measure_peaks: cannot select device");
    const hipStream_t s = ctx->stream;
    // 32 waves per CU: enough to hide every latency at any occupancy
    const int blocks = ctx->n_cu * 8;
    const double lanes = (double)blocks * kPeakBlock;
    double* buf = nullptr;
    if (hipMalloc(&buf, sizeof(double) * (size_t)blocks * kPeakBlock) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SWV_ENOMEM, "swv_measure_peaks: scratch allocation failed");
    }
    constexpr int C64 = 8, C32 = 16, CS = 8, CP = 4;
    int rc = SWV_OK;
    double t = 0.0;
    const int it64 = 16384, it32 = 8192, itsc = 2048, itcp = 8192;   // ~5-20 ms each
    rc = time_kernel(s, [&](int n) {
        k_peak_fma_f64<C64><<<dim3(blocks), dim3(kPeakBlock), 0, s>>>(buf, n);
    }, it64, &t);
    if (!rc) out->fp64_fma_tflops = lanes * it64 * 8.0 * C64 * 2.0 / t / 1e12;
    if (!rc) rc = time_kernel(s, [&](int n) {
        k_peak_fma_f32<C32><<<dim3(blocks), dim3(kPeakBlock), 0, s>>>(buf, n);
    }, it32, &t);
    if (!rc) out->fp32_fma_tflops = lanes * it32 * 8.0 * C32 * 2.0 / t / 1e12;
    if (!rc) rc = time_kernel(s, [&](int n) {
        k_peak_sincos_f32<CS><<<dim3(blocks), dim3(kPeakBlock), 0, s>>>(buf, n);
    }, itsc, &t);
    if (!rc) out->sincos_f32_gops = lanes * itsc * 4.0 * CS / t / 1e9;
    if (!rc) rc = time_kernel(s, [&](int n) {
        k_peak_cis2pi_f64<CP><<<dim3(blocks), dim3(kPeakBlock), 0, s>>>(buf, n);
    }, itcp, &t);
    if (!rc) out->cis2pi_f64_gops = lanes * itcp * (double)CP / t / 1e9;
    (void)hipFree(buf);
    if (!rc) clear_error();
    return rc;
}
