// Per-row device code of the direct component sum (section 3.3, Eq. 12),
// shared by the single-instance kernels and the persistent batched kernel.
//
// A lane owns VPL visibility rows j[0..VPL) (rows >= limit are computed on a
// clamped index and not stored); every lane of a wave walks the same
// component list, so a component record (l, m, n-1, I; 32 B) is one scalar
// load into SGPRs that enters the FMAs as the scalar operand.  The sum over
// components is a per-lane running sum in a fixed order: bit-reproducible,
// no atomics.  Work per (row, component): phase 3 ops, reduction 2,
// phasor 20, MAC 2.
#pragma once

#include "device_math.h"
#include "launch.h"

namespace swv {

// One packed component: n - 1 = -(l^2 + m^2) / (1 + n), free of cancellation.
// Written with an explicit FMA so every kernel that packs components rounds
// identically.  Sets bits of `bad` for out-of-domain or non-finite input (the
// record is then zero).
__device__ __forceinline__ Comp pack_component(double L, double M, double I, int& bad) {
    const double r2 = fma(L, L, M * M);
    bad = 0;
    if (!(r2 < 1.0)) bad |= kStatusDomain;
    if (!isfinite(L) || !isfinite(M) || !isfinite(I)) bad |= kStatusNonFinite;
    if (bad) return Comp{0.0, 0.0, 0.0, 0.0};
    return Comp{L, M, -r2 / (1.0 + sqrt(1.0 - r2)), I};
}

template <int VPL>
__device__ __forceinline__ void direct_rows_f64(const int64_t (&j)[VPL], int64_t limit,
                                                const double* __restrict__ u,
                                                const double* __restrict__ v,
                                                const double* __restrict__ w,
                                                const Comp* __restrict__ comp, int n_comp,
                                                double sgn, double2* __restrict__ out,
                                                int* __restrict__ status) {
    double U[VPL], V[VPL], W[VPL], re[VPL], iq[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
        const int64_t jj = j[i] < limit ? j[i] : limit - 1;
        U[i] = u[jj];
        V[i] = v[jj];
        W[i] = w[jj];
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
        if (j[i] < limit) {
            if (!isfinite(U[i] + V[i] + W[i])) atomicOr(status, kStatusNonFinite);
            out[j[i]] = make_double2(re[i], s4 * iq[i]);
        }
    }
}

// FP64 phase and reduction; FP32 phasor, products and Kahan-compensated sums.
template <int VPL>
__device__ __forceinline__ void direct_rows_f32c(const int64_t (&j)[VPL], int64_t limit,
                                                 const double* __restrict__ u,
                                                 const double* __restrict__ v,
                                                 const double* __restrict__ w,
                                                 const Comp* __restrict__ comp, int n_comp,
                                                 float sgn, float2* __restrict__ out,
                                                 int* __restrict__ status) {
    double U[VPL], V[VPL], W[VPL];
    float sr[VPL], cr[VPL], si[VPL], ci[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
        const int64_t jj = j[i] < limit ? j[i] : limit - 1;
        U[i] = u[jj];
        V[i] = v[jj];
        W[i] = w[jj];
        sr[i] = cr[i] = si[i] = ci[i] = 0.0f;
    }
    const auto* cp = uniform_ptr(comp);
    // components in pairs: the pair's two products and the running
    // compensation meet in two FMAs, then one Kahan step, so a component costs
    // half a step (the pair's roundings stay within 2 x 2^-24 of its terms);
    // an odd last component enters alone
    const int npair = n_comp & ~1;
    for (int k = 0; k < npair; k += 2) {
        const Comp a{cp[k].l, cp[k].m, cp[k].nm1, cp[k].I};
        const Comp b{cp[k + 1].l, cp[k + 1].m, cp[k + 1].nm1, cp[k + 1].I};
        const float aI = (float)a.I, bI = (float)b.I;
#pragma unroll
        for (int i = 0; i < VPL; ++i) {
            const float ra = (float)fract_phase(U[i], V[i], W[i], a.l, a.m, a.nm1);
            const float rb = (float)fract_phase(U[i], V[i], W[i], b.l, b.m, b.nm1);
            float ca, sa, cb, sb;
            cis2pi_f32(ra, ca, sa);
            cis2pi_f32(rb, cb, sb);
            kahan_step(fmaf(aI, ca, fmaf(bI, cb, -cr[i])), sr[i], cr[i]);
            kahan_step(fmaf(aI, sa, fmaf(bI, sb, -ci[i])), si[i], ci[i]);
        }
    }
    if (npair < n_comp) {
        const Comp cur{cp[npair].l, cp[npair].m, cp[npair].nm1, cp[npair].I};
        const float cI = (float)cur.I;
#pragma unroll
        for (int i = 0; i < VPL; ++i) {
            const float r = (float)fract_phase(U[i], V[i], W[i], cur.l, cur.m, cur.nm1);
            float c, s;
            cis2pi_f32(r, c, s);
            kahan_add_prod(cI, c, sr[i], cr[i]);
            kahan_add_prod(cI, s, si[i], ci[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
        if (j[i] < limit) {
            if (!isfinite(U[i] + V[i] + W[i])) atomicOr(status, kStatusNonFinite);
            out[j[i]] = make_float2(sr[i], sgn * si[i]);
        }
    }
}

}  // namespace swv
