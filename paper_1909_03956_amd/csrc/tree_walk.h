// Depth-first traversal of the wavelet tree for one visibility row per
// lane, shared by the single-instance and the persistent batched kernels.
// The algorithm is described in k_tree.hip.
#pragma once

#include "device_math.h"
#include "launch.h"

namespace swv {

using RecPtr = const __attribute__((address_space(4))) TRec*;

template <int LVL, int JMAX>
__device__ __forceinline__ void walk(RecPtr rec, int& pos, const int J, const TreeArgs& ta,
                                     const double u, const double v, const double w, double& er,
                                     double& ei, double& Vr, double& Vi) {
    const int me = pos++;
    if (LVL == JMAX || LVL == J) {
        // leaf: eta_{J,k} = exp(2 pi i B . (s_k - P))
        double c, q;
        cis2pi_q(reduced_phase(u, v, w, rec[me].a, rec[me].b, rec[me].c), c, q);
        er = c;
        ei = q;
        return;
    }
    if constexpr (LVL < JMAX) {
        unsigned mask = (unsigned)rec[me].meta;
        double Sr = 0.0, Si = 0.0, D0r = 0.0, D0i = 0.0, D1r = 0.0, D1i = 0.0, D2r = 0.0,
               D2i = 0.0;
        while (mask) {
            const int c = __builtin_ctz(mask);
            mask &= mask - 1;
            double xr, xi;
            walk<LVL + 1, JMAX>(rec, pos, J, ta, u, v, w, xr, xi, Vr, Vi);
            // Eq. 10 signs of child c: gamma^0 (+-+-), gamma^1 (++--), gamma^2 (+--+)
            const double s0 = (c & 1) ? -1.0 : 1.0;
            const double s1 = (c & 2) ? -1.0 : 1.0;
            const double s2 = s0 * s1;
            Sr += xr;
            Si += xi;
            D0r = fma(s0, xr, D0r);
            D0i = fma(s0, xi, D0i);
            D1r = fma(s1, xr, D1r);
            D1i = fma(s1, xi, D1i);
            D2r = fma(s2, xr, D2r);
            D2i = fma(s2, xi, D2i);
        }
        // eta_j (Eq. 9 on the plane wave) goes up to the parent
        er = 0.25 * Sr;
        ei = 0.25 * Si;
        // sigma^m_j (Eq. 10 on the plane wave), then gamma^m_j sigma^m_j (Eq. 17)
        const double a = ta.scale[LVL];
        const double g0 = rec[me].a, g1 = rec[me].b, g2 = rec[me].c;
        const double s0r = a * D0r, s0i = a * D0i;
        const double s1r = a * D1r, s1i = a * D1i;
        const double s2r = a * D2r, s2i = a * D2i;
        Vr = fma(g0, s0r, Vr);
        Vi = fma(g0, s0i, Vi);
        Vr = fma(g1, s1r, Vr);
        Vi = fma(g1, s1i, Vi);
        Vr = fma(g2, s2r, Vr);
        Vi = fma(g2, s2i, Vi);
    }
}

// V (real, imaginary / 4) of one row: the root loop of the traversal.
template <int JMAX>
__device__ __forceinline__ void tree_row(const TRec* recs, int n_roots, int J,
                                         const TreeArgs& ta, double U, double V, double W,
                                         double& Vr, double& Vi) {
    const RecPtr rec = uniform_ptr(recs);
    Vr = 0.0;
    Vi = 0.0;
    int pos = 0;
    for (int r = 0; r < n_roots; ++r) {
        const int root = pos++;
        double er, ei;
        walk<1, JMAX>(rec, pos, J, ta, U, V, W, er, ei, Vr, Vi);
        const double A1lam = rec[root].a;  // A_1 lambda_1
        Vr = fma(A1lam, er, Vr);
        Vi = fma(A1lam, ei, Vi);
    }
}

}  // namespace swv
