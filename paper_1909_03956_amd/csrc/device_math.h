// Per-term arithmetic of every kernel: the reduced phase and its complex
// exponential.
//
// Phase (section 3.3, Eq. 12 with P = [0, 0, 1]), in cycles:
//     phi = u l + v m + w (n - 1)
// evaluated with two FMAs and one multiply, then reduced exactly to
// r = phi - rint(phi) in [-1/2, 1/2] (the subtraction is exact).
//
// Phasor: with x = (pi/2) r, |x| <= pi/4, s = sin x and c = cos x come from
// the fitted polynomials of sincos_coeffs.h, and the full angle 4x = 2 pi r
// from the identities
//     cos 4x = 1 - 8 (s c)^2,      sin 4x = 4 (s c)(c^2 - s^2).
// cis2pi_q returns cos(2 pi r) and q = sin(2 pi r) / 4: callers fold the
// factor 4 (a power of two, so exactly) into their accumulators.
//
// Operation count per phasor: 1 (r^2) + 7 (sine polynomial) + 6 (cosine
// polynomial) + 6 (the 4x identities) = 20 VALU instructions, 14 of them FMAs.
#pragma once

#include <hip/hip_runtime.h>

#include "sincos_coeffs.h"

namespace swv {

__host__ __device__ __forceinline__ double reduced_phase(double u, double v, double w, double l,
                                                         double m, double nm1) {
    const double ph = fma(u, l, fma(v, m, w * nm1));
    return ph - rint(ph);
}

// The same phase reduced to [0, 1) by the hardware fract, one FP64
// instruction against rint and a subtraction, and exact as well (|phase| is
// far below 2^52). For the FP32 phasor only: its sine and cosine take any
// angle in [-256, 256] revolutions, and the conversion of r to FP32 then
// rounds by at most 2^-25 cycles.
__device__ __forceinline__ double fract_phase(double u, double v, double w, double l, double m,
                                              double nm1) {
    return __builtin_amdgcn_fract(fma(u, l, fma(v, m, w * nm1)));
}

// Fused multiply-add as one 3-operand v_fma_f64 on VGPRs: the same rounding
// as fma(), but never the two-address form (a copy of the addend into the
// destination, then v_fmac_f64) that the compiler picks when the addend is a
// value it keeps, such as a polynomial coefficient held in a register across
// loops.
__device__ __forceinline__ double fma_v(double a, double b, double c) {
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

template <bool VOP3>
__host__ __device__ __forceinline__ double fma_sel(double a, double b, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (VOP3) return fma_v(a, b, c);
#endif
    return fma(a, b, c);
}

template <bool VOP3>
__host__ __device__ __forceinline__ void cis2pi_q_impl(double r, double& c, double& q) {
    const double t = r * r;
    double ps = kS64[6];
    ps = fma_sel<VOP3>(ps, t, kS64[5]);
    ps = fma_sel<VOP3>(ps, t, kS64[4]);
    ps = fma_sel<VOP3>(ps, t, kS64[3]);
    ps = fma_sel<VOP3>(ps, t, kS64[2]);
    ps = fma_sel<VOP3>(ps, t, kS64[1]);
    ps = fma_sel<VOP3>(ps, t, kS64[0]);
    double pc = kC64[5];
    pc = fma_sel<VOP3>(pc, t, kC64[4]);
    pc = fma_sel<VOP3>(pc, t, kC64[3]);
    pc = fma_sel<VOP3>(pc, t, kC64[2]);
    pc = fma_sel<VOP3>(pc, t, kC64[1]);
    pc = fma_sel<VOP3>(pc, t, kC64[0]);
    const double s1 = r * ps;
    const double c1 = fma(pc, t, 1.0);
    const double p = s1 * c1;
    const double d = fma(c1, c1, -(s1 * s1));
    c = fma(-8.0 * p, p, 1.0);
    q = p * d;
}

__host__ __device__ __forceinline__ void cis2pi_q(double r, double& c, double& q) {
    cis2pi_q_impl<false>(r, c, q);
}

// The same phasor with every polynomial step a 3-operand FMA (for kernels
// whose coefficients live in VGPRs; bitwise equal to cis2pi_q).
__host__ __device__ __forceinline__ void cis2pi_q_vop3(double r, double& c, double& q) {
    cis2pi_q_impl<true>(r, c, q);
}

// FP32 phasor of a reduced phase r in cycles (the callers pass r in [0, 1)):
// cos(2 pi r), sin(2 pi r) from the hardware transcendental unit (v_cos_f32 /
// v_sin_f32 take the angle in revolutions and are valid on [-256, 256]).
__device__ __forceinline__ void cis2pi_f32(float r, float& c, float& s) {
    c = __builtin_amdgcn_cosf(r);
    s = __builtin_amdgcn_sinf(r);
}

// One Kahan step: y is the next addend with the running compensation already
// subtracted; the rounding error of sum + y becomes the new compensation (the
// compensated total is sum - comp).
__host__ __device__ __forceinline__ void kahan_step(float y, float& sum, float& comp) {
    const float t = sum + y;
    comp = (t - sum) - y;
    sum = t;
}

// Kahan-compensated accumulation of the product a b into (sum, comp); the
// product is rounded once, inside the FMA that removes the compensation.
__host__ __device__ __forceinline__ void kahan_add_prod(float a, float b, float& sum,
                                                        float& comp) {
    kahan_step(fmaf(a, b, -comp), sum, comp);
}

}  // namespace swv
