// Direct component sum (section 3.3, Eq. 12) on gfx950.
//
// Mapping: each lane owns VPL visibility rows (coalesced FP64 loads of u, v,
// w); every lane of a wave walks the same component list, so a component
// record (l, m, n-1, I; 32 B) is one scalar load into SGPRs and enters the
// FMAs as the instruction's scalar operand.  The sum over components is a
// per-lane running sum: no cross-lane reduction, no atomics, a fixed order,
// bit-reproducible.  VPL independent rows give the FP64 pipeline ILP.
//
// Work per (row, component): phase 3 ops, reduction 2, phasor 20, MAC 2.
#include "device_math.h"
#include "launch.h"

namespace swv {

__global__ void k_ingest(int64_t n, const double* __restrict__ l, const double* __restrict__ m,
                         const double* __restrict__ flux, Comp* __restrict__ out,
                         int* __restrict__ status) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double L = l[k], M = m[k], I = flux[k];
    const double r2 = L * L + M * M;
    int bad = 0;
    if (!(r2 < 1.0)) bad |= kStatusDomain;
    if (!isfinite(L) || !isfinite(M) || !isfinite(I)) bad |= kStatusNonFinite;
    if (bad) {
        atomicOr(status, bad);
        out[k] = Comp{0.0, 0.0, 0.0, 0.0};
        return;
    }
    // n - 1 = -(l^2 + m^2) / (1 + n), free of cancellation
    out[k] = Comp{L, M, -r2 / (1.0 + sqrt(1.0 - r2)), I};
}

hipError_t launch_ingest(hipStream_t s, int64_t n, const double* l, const double* m,
                         const double* flux, Comp* out, int* status) {
    if (n <= 0) return hipSuccess;
    const int b = 256;
    k_ingest<<<dim3((unsigned)((n + b - 1) / b)), dim3(b), 0, s>>>(n, l, m, flux, out, status);
    return hipGetLastError();
}

template <int VPL, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_direct_f64(const double* __restrict__ u,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ w, int64_t n_vis,
                                                      const Comp* __restrict__ comp, int n_comp,
                                                      double sgn, double2* __restrict__ out,
                                                      int* __restrict__ status) {
    const int64_t base = (int64_t)blockIdx.x * (BLOCK * VPL) + threadIdx.x;
    double U[VPL], V[VPL], W[VPL], re[VPL], iq[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
        int64_t j = base + (int64_t)i * BLOCK;
        j = j < n_vis ? j : n_vis - 1;
        U[i] = u[j];
        V[i] = v[j];
        W[i] = w[j];
        re[i] = 0.0;
        iq[i] = 0.0;
    }
    const auto* cp = uniform_ptr(comp);
    for (int k = 0; k < n_comp; ++k) {
        const Comp cur{cp[k].l, cp[k].m, cp[k].nm1, cp[k].I};
#pragma unroll
        for (int i = 0; i < VPL; ++i) {
            double c, q;
            cis2pi_q(reduced_phase(U[i], V[i], W[i], cur.l, cur.m, cur.nm1), c, q);
            re[i] = fma(cur.I, c, re[i]);
            iq[i] = fma(cur.I, q, iq[i]);
        }
    }
    const double s4 = 4.0 * sgn;
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
        const int64_t j = base + (int64_t)i * BLOCK;
        if (j < n_vis) {
            if (!isfinite(U[i] + V[i] + W[i])) atomicOr(status, kStatusNonFinite);
            out[j] = make_double2(re[i], s4 * iq[i]);
        }
    }
}

// FP64 phase and reduction; FP32 phasor, products and Kahan-compensated sums.
template <int VPL, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_direct_f32c(const double* __restrict__ u,
                                                       const double* __restrict__ v,
                                                       const double* __restrict__ w,
                                                       int64_t n_vis,
                                                       const Comp* __restrict__ comp, int n_comp,
                                                       float sgn, float2* __restrict__ out,
                                                       int* __restrict__ status) {
    const int64_t base = (int64_t)blockIdx.x * (BLOCK * VPL) + threadIdx.x;
    double U[VPL], V[VPL], W[VPL];
    float sr[VPL], cr[VPL], si[VPL], ci[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
        int64_t j = base + (int64_t)i * BLOCK;
        j = j < n_vis ? j : n_vis - 1;
        U[i] = u[j];
        V[i] = v[j];
        W[i] = w[j];
        sr[i] = cr[i] = si[i] = ci[i] = 0.0f;
    }
    const auto* cp = uniform_ptr(comp);
    for (int k = 0; k < n_comp; ++k) {
        const Comp cur{cp[k].l, cp[k].m, cp[k].nm1, cp[k].I};
        const float cI = (float)cur.I;
#pragma unroll
        for (int i = 0; i < VPL; ++i) {
            const float r = (float)reduced_phase(U[i], V[i], W[i], cur.l, cur.m, cur.nm1);
            float c, s;
            cis2pi_f32(r, c, s);
            kahan_add(cI * c, sr[i], cr[i]);
            kahan_add(cI * s, si[i], ci[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
        const int64_t j = base + (int64_t)i * BLOCK;
        if (j < n_vis) {
            if (!isfinite(U[i] + V[i] + W[i])) atomicOr(status, kStatusNonFinite);
            out[j] = make_float2(sr[i], sgn * si[i]);
        }
    }
}

template <int VPL, int BLOCK>
static hipError_t run_direct(hipStream_t s, int prec, int64_t n_vis, const double* u,
                             const double* v, const double* w, const Comp* comp, int64_t n_comp,
                             int sign, void* out, int* status) {
    const int64_t rows = (int64_t)BLOCK * VPL;
    const dim3 grid((unsigned)((n_vis + rows - 1) / rows)), blk(BLOCK);
    if (prec == SWV_FP64)
        k_direct_f64<VPL, BLOCK><<<grid, blk, 0, s>>>(u, v, w, n_vis, comp, (int)n_comp,
                                                       (double)sign, (double2*)out, status);
    else
        k_direct_f32c<VPL, BLOCK><<<grid, blk, 0, s>>>(u, v, w, n_vis, comp, (int)n_comp,
                                                        (float)sign, (float2*)out, status);
    return hipGetLastError();
}

template <int VPL>
static hipError_t run_direct_b(hipStream_t s, int prec, int block, int64_t n_vis,
                               const double* u, const double* v, const double* w,
                               const Comp* comp, int64_t n_comp, int sign, void* out,
                               int* status) {
    switch (block) {
        case 64: return run_direct<VPL, 64>(s, prec, n_vis, u, v, w, comp, n_comp, sign, out, status);
        case 128: return run_direct<VPL, 128>(s, prec, n_vis, u, v, w, comp, n_comp, sign, out, status);
        case 256: return run_direct<VPL, 256>(s, prec, n_vis, u, v, w, comp, n_comp, sign, out, status);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_direct(hipStream_t s, int prec, int vpl, int block, int64_t n_vis,
                         const double* u, const double* v, const double* w, const Comp* comp,
                         int64_t n_comp, int sign, void* out, int* status) {
    if (n_vis <= 0) return hipSuccess;
    switch (vpl) {
        case 1: return run_direct_b<1>(s, prec, block, n_vis, u, v, w, comp, n_comp, sign, out, status);
        case 2: return run_direct_b<2>(s, prec, block, n_vis, u, v, w, comp, n_comp, sign, out, status);
        case 4: return run_direct_b<4>(s, prec, block, n_vis, u, v, w, comp, n_comp, sign, out, status);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace swv
