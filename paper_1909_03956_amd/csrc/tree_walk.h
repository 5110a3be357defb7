// Depth-first traversal of the wavelet tree for one visibility row per
// lane, shared by the single-instance and the persistent batched kernels.
// The algorithm is described in k_tree.hip.
#pragma once

#include "device_math.h"
#include "launch.h"

namespace swv {

using RecPtr = const __attribute__((address_space(4))) TRec*;
using LdsPtr = __attribute__((address_space(3))) double*;

// Open levels (segments) whose running sums stay in registers; the ones above
// them are kept in LDS (see slot_put).
constexpr int kTreeRegLevels = 6;

// Running sums of an open node at level j over its finished children, whose
// values are T_{j+1,c} = 4^(J-j-1) eta_{j+1,c} (the plain sums of the leaf
// phasors below them, see close_node), the D^m taken relative to the node's
// first child c0:
//   S = sum_c T_{j+1,c},   D^m = s^m_{c0} sum_c s^m_c T_{j+1,c}   (m = 0, 1, 2),
// so the first child's value enters every sum as it is, and the sign
// s^m_{c0} moves to the node's scale factor when it closes.  With s = +-1 and
// rounding symmetric in sign, each value is the plain sum times s^m_{c0}
// exactly, so sigma comes out the same bit for bit.  (The branch walker
// passes c0 = 0 and starts its sums at zero.)
struct NodeSums {
    double Sr, Si, D0r, D0i, D1r, D1i, D2r, D2i;
};

// Eq. 10 signs: gamma^0 (+-+-), gamma^1 (++--), gamma^2 (+--+) over the
// children c = 0..3; s^m_c s^m_{c0} is the sign of child c ^ c0.
__device__ __forceinline__ double sign0(int c) { return (c & 1) ? -1.0 : 1.0; }
__device__ __forceinline__ double sign1(int c) { return (c & 2) ? -1.0 : 1.0; }
__device__ __forceinline__ double sign2(int c) { return ((c ^ (c >> 1)) & 1) ? -1.0 : 1.0; }

// Takes child c's value x = T_{j+1,c} into the sums of a node whose first
// child is c0: the first child sets them all to x, later ones add with the
// signs of c ^ c0.  `first` is the same for every lane, so this is
// a scalar branch, and no sums need zeroing.
__device__ __forceinline__ void add_child(NodeSums& n, int c, int c0, double xr, double xi,
                                          bool first) {
    if (first) {
        n.Sr = n.D0r = n.D1r = n.D2r = xr;
        n.Si = n.D0i = n.D1i = n.D2i = xi;
    } else {
        const int r = c ^ c0;
        const double s0 = sign0(r), s1 = sign1(r), s2 = sign2(r);
        n.Sr += xr;
        n.Si += xi;
        n.D0r = fma(s0, xr, n.D0r);
        n.D0i = fma(s0, xi, n.D0i);
        n.D1r = fma(s1, xr, n.D1r);
        n.D1i = fma(s1, xi, n.D1i);
        n.D2r = fma(s2, xr, n.D2r);
        n.D2i = fma(s2, xi, n.D2i);
    }
}

// Closes a node at level j whose first child is c0 (g = gamma^m_j): its sum
// T_j goes to the parent, sigma^m_j = s^m_{c0} a D^m (Eq. 10 on the plane
// wave) is formed with a = (sqrt(A_j)/4) 4^-(J-j-1) (the children's sums are
// T_{j+1} = 4^(J-j-1) eta_{j+1}) and gamma^m_j sigma^m_j added to V (Eq. 17).
// Passing T_j = sum over the leaves below of eta_J instead of eta_j = T_j /
// 4^(J-j) (Eq. 9 on the plane wave) moves every quarter into the scale
// factors as exact powers of two: the same sigma bit for bit, two fewer
// products per node.
__device__ __forceinline__ void close_node(const NodeSums& n, int c0, double a, double g0,
                                           double g1, double g2, double& er, double& ei,
                                           double& Vr, double& Vi) {
    // sign choices on a wave-uniform value: scalar selects, no arithmetic
    const double a0 = (c0 & 1) ? -a : a;
    const double a1 = (c0 & 2) ? -a : a;
    const double a2 = ((c0 ^ (c0 >> 1)) & 1) ? -a : a;
    er = n.Sr;
    ei = n.Si;
    const double s0r = a0 * n.D0r, s0i = a0 * n.D0i;
    const double s1r = a1 * n.D1r, s1i = a1 * n.D1i;
    const double s2r = a2 * n.D2r, s2i = a2 * n.D2i;
    Vr = fma(g0, s0r, Vr);
    Vi = fma(g0, s0i, Vi);
    Vr = fma(g1, s1r, Vr);
    Vi = fma(g1, s1i, Vi);
    Vr = fma(g2, s2r, Vr);
    Vi = fma(g2, s2i, Vi);
}

// Open nodes of the top LDSL levels (level walker) or segments (branch
// walker) keep their children's plane-wave coefficients in LDS rather than
// running sums in registers: such a node is touched only when one of its few
// children finishes, and its registers would otherwise stay allocated through
// every subtree below it, which limits how many waves share a SIMD.  A node
// holds at most three finished children while its last one is walked, so a
// slot is three complex values (6 doubles, against 8 for the four running
// sums); the sums are formed when the last child is back, in child order, so
// they equal the register levels' bit for bit.  Layout [slot][6][BLOCK]:
// lane-contiguous, so the accesses are free of bank conflicts.
// The accesses are volatile: otherwise the compiler, seeing the whole inlined
// walk, forwards each stored value to its reload and keeps it in registers.
constexpr int kSlotDoubles = 6;

template <int BLOCK>
__device__ __forceinline__ void slot_put(LdsPtr lds, int slot, int k, double xr, double xi) {
    volatile __attribute__((address_space(3))) double* p =
        lds + (slot * kSlotDoubles + 2 * k) * BLOCK + threadIdx.x;
    p[0] = xr;
    p[BLOCK] = xi;
}

template <int BLOCK>
__device__ __forceinline__ void slot_get(LdsPtr lds, int slot, int k, double& xr, double& xi) {
    const volatile __attribute__((address_space(3))) double* p =
        lds + (slot * kSlotDoubles + 2 * k) * BLOCK + threadIdx.x;
    xr = p[0];
    xi = p[BLOCK];
}

// Adds the k children kept in a slot to n, in child order, relative to
// child c0; `all` is the node's child mask, whose k lowest set bits name them.
template <int BLOCK>
__device__ __forceinline__ void slot_replay(LdsPtr lds, int slot, int k, unsigned all, int c0,
                                            NodeSums& n, bool& first) {
    for (int q = 0; q < k; ++q) {
        const int c = __builtin_ctz(all);
        all &= all - 1;
        double xr, xi;
        slot_get<BLOCK>(lds, slot, q, xr, xi);
        add_child(n, c, c0, xr, xi, first);
        first = false;
    }
}

// a 2^e for a normal a and a normal result: e is added to the exponent
// field, an exact operation that stays on the scalar unit for wave-uniform
// operands.
__device__ __forceinline__ double pow2_scale(double a, int e) {
    return __longlong_as_double(__double_as_longlong(a) + ((long long)e << 52));
}

// The scale a of close_node at level j of a depth-J tree:
// (sqrt(A_j)/4) 4^-(J-j-1) = (sqrt(A_1)/4) 2^(j+3-2J), from the level-1 factor
// the host stores (sqrt(A_j)/4 halves from level to level) with no load that
// waits on the record.
__device__ __forceinline__ double level_factor(const TreeArgs& ta, int j, int J) {
    return pow2_scale(ta.scale[1], j + 3 - 2 * J);
}

// Closes a node whose only child c returned its sum x: T_j = x and
// sigma^m_j = (s^m_c a) x -- close_node after add_child with c0 = c, the
// same operations -- then gamma^m_j sigma^m_j is added to V.
__device__ __forceinline__ void close_single(int c, double a, double g0, double g1, double g2,
                                             double& er, double& ei, double& Vr, double& Vi) {
    const double xr = er, xi = ei;
    const double a0 = (c & 1) ? -a : a;
    const double a1 = (c & 2) ? -a : a;
    const double a2 = ((c ^ (c >> 1)) & 1) ? -a : a;
    const double s0r = a0 * xr, s0i = a0 * xi;
    const double s1r = a1 * xr, s1i = a1 * xi;
    const double s2r = a2 * xr, s2i = a2 * xi;
    Vr = fma(g0, s0r, Vr);
    Vi = fma(g0, s0i, Vi);
    Vr = fma(g1, s1r, Vr);
    Vi = fma(g1, s1i, Vi);
    Vr = fma(g2, s2r, Vr);
    Vi = fma(g2, s2i, Vi);
}

// Leaf: eta_{J,k} = exp(2 pi i B . (s_k - P)) (imaginary part / 4).  VOP3
// selects the phasor whose polynomial steps are 3-operand FMAs (same values);
// F32 the precision form: the FP64 phase, reduced exactly in FP64, then the
// FP32 hardware sine and cosine (everything after the leaf stays FP64).
template <bool VOP3, bool F32>
__device__ __forceinline__ void leaf_wave(RecPtr rec, int me, double u, double v, double w,
                                          double& er, double& ei) {
    const double r = reduced_phase(u, v, w, rec[me].a, rec[me].b, rec[me].c);
    if constexpr (F32) {
        float c32, s32;
        cis2pi_f32((float)r, c32, s32);
        er = (double)c32;
        ei = 0.25 * (double)s32;
    } else {
        double c, q;
        if constexpr (VOP3)
            cis2pi_q_vop3(r, c, q);
        else
            cis2pi_q(r, c, q);
        er = c;
        ei = q;
    }
}

// Leaf at level j < J, which only a thresholded tree has: a node none of whose
// coefficients at or below it is retained, walked as a leaf at its pixel
// centre.  The traversal hands up plain sums T_j = 4^(J-j) eta_j (see
// close_node), so its plane wave is scaled by that exact power of two.  Only
// the PRUNED instantiations of the walkers test for such leaves.
template <bool F32>
__device__ __forceinline__ void leaf_above(RecPtr rec, int me, int j, int J, double u,
                                           double v, double w, double& er, double& ei) {
    leaf_wave<false, F32>(rec, me, u, v, w, er, ei);
    const double s = pow2_scale(1.0, 2 * (J - j));
    er *= s;
    ei *= s;
}

// Level walker: one register set per level, the level a template parameter
// (levels <= LDSL keep theirs in LDS).
template <int LVL, int JMAX, int LDSL, int BLOCK, bool F32, bool PRUNED>
__device__ __forceinline__ void walk(RecPtr rec, int& pos, const int J, const TreeArgs& ta,
                                     LdsPtr lds, const double u, const double v, const double w,
                                     double& er, double& ei, double& Vr, double& Vi) {
    const int me = pos++;
    if (LVL == JMAX || LVL == J) {
        leaf_wave<true, F32>(rec, me, u, v, w, er, ei);
        return;
    }
    if constexpr (LVL < JMAX) {
        const unsigned all = meta_mask(rec[me].meta);
        if constexpr (PRUNED) {
            if (all == 0) {   // a node collapsed by thresholding
                leaf_above<F32>(rec, me, LVL, J, u, v, w, er, ei);
                return;
            }
        }
        const int c0 = __builtin_ctz(all);
        unsigned mask = all;
        NodeSums n;
        bool first = true;
        if constexpr (LVL <= LDSL) {
            // every child but the last waits in the slot (stored when the
            // next one starts); only the last one's value leaves the loop
            int k = 0, c = 0;
            double xr = 0.0, xi = 0.0;
            while (mask) {
                if (mask != all) slot_put<BLOCK>(lds, LVL - 1, k++, xr, xi);
                c = __builtin_ctz(mask);
                mask &= mask - 1;
                walk<LVL + 1, JMAX, LDSL, BLOCK, F32, PRUNED>(rec, pos, J, ta, lds, u, v, w, xr, xi, Vr,
                                                      Vi);
            }
            slot_replay<BLOCK>(lds, LVL - 1, k, all, c0, n, first);
            add_child(n, c, c0, xr, xi, first);
        } else {
            while (mask) {
                const int c = __builtin_ctz(mask);
                mask &= mask - 1;
                double xr, xi;
                walk<LVL + 1, JMAX, LDSL, BLOCK, F32, PRUNED>(rec, pos, J, ta, lds, u, v, w, xr, xi, Vr,
                                                      Vi);
                add_child(n, c, c0, xr, xi, first);
                first = false;
            }
        }
        close_node(n, c0, level_factor(ta, LVL, J), rec[me].a, rec[me].b, rec[me].c, er, ei,
                   Vr, Vi);
    }
}

// Branch walker: one register set per open BRANCHING node, so any J.  A
// segment is a run of one-child nodes (possibly empty) and the leaf or
// branching node below it; the run keeps no state while the part below is
// walked, and is closed bottom-up afterwards with the same arithmetic a
// one-child node gets in the level walker.  D counts segments from the root;
// the host launches DMAX >= 1 + the tree's largest branching count on a path.
template <int D, int DMAX, int LDSL, int BLOCK, bool F32, bool PRUNED>
__device__ __forceinline__ void seg_walk(RecPtr rec, int& pos, const int J, const TreeArgs& ta,
                                         LdsPtr lds, const double u, const double v,
                                         const double w, double& er, double& ei, double& Vr,
                                         double& Vi) {
    const int first = pos;
    const int run = meta_chain(rec[first].meta);
    const int term = first + run;
    pos = term + 1;
    const unsigned long long mt = rec[term].meta;
    er = 0.0;
    ei = 0.0;
    if (meta_level(mt) == J) {
        leaf_wave<false, F32>(rec, term, u, v, w, er, ei);
    } else if (PRUNED && meta_mask(mt) == 0) {
        // a node collapsed by thresholding
        leaf_above<F32>(rec, term, meta_level(mt), J, u, v, w, er, ei);
    } else {
        if constexpr (D < DMAX) {
            // a terminal node has two or more children.  Its sums start at
            // zero and take every child with its own signs (c0 = 0: the
            // plain sums); the level walker's first-child form costs this
            // walker more in scalar registers than it saves
            const unsigned all = meta_mask(mt);
            unsigned mask = all;
            NodeSums n{};
            bool first = false;
            if constexpr (D <= LDSL) {
                // as in the level walker: all children but the last wait in
                // the slot, and the sums are formed at the end
                int k = 0, c = 0;
                double xr = 0.0, xi = 0.0;
                while (mask) {
                    if (mask != all) slot_put<BLOCK>(lds, D - 1, k++, xr, xi);
                    c = __builtin_ctz(mask);
                    mask &= mask - 1;
                    seg_walk<D + 1, DMAX, LDSL, BLOCK, F32, PRUNED>(rec, pos, J, ta, lds, u, v, w, xr,
                                                            xi, Vr, Vi);
                }
                slot_replay<BLOCK>(lds, D - 1, k, all, 0, n, first);
                add_child(n, c, 0, xr, xi, false);
            } else {
                while (mask) {
                    const int c = __builtin_ctz(mask);
                    mask &= mask - 1;
                    double xr, xi;
                    seg_walk<D + 1, DMAX, LDSL, BLOCK, F32, PRUNED>(rec, pos, J, ta, lds, u, v, w, xr,
                                                            xi, Vr, Vi);
                    add_child(n, c, 0, xr, xi, false);
                }
            }
            close_node(n, 0, level_factor(ta, meta_level(mt), J), rec[term].a, rec[term].b,
                       rec[term].c, er, ei, Vr, Vi);
        }
    }
    // the run, bottom-up
    for (int i = run - 1; i >= 0; --i) {
        const int me = first + i;
        const unsigned long long mm = rec[me].meta;
        close_single(__builtin_ctz(meta_mask(mm)), level_factor(ta, meta_level(mm), J), rec[me].a,
                     rec[me].b, rec[me].c, er, ei, Vr, Vi);
    }
}

// Levels (segments) of a traversal compiled to depth JMAX whose sums go to
// LDS: all but the deepest kTreeRegLevels, within 64 KB per block.
template <int JMAX, int BLOCK>
constexpr int tree_lds_levels() {
    constexpr int want = JMAX > kTreeRegLevels ? JMAX - kTreeRegLevels : 0;
    constexpr int cap = (64 * 1024) / (kSlotDoubles * 8 * BLOCK);
    return want < cap ? want : cap;
}

// V (real, imaginary / 4) of one row: the root loop of the traversal.
// WALKER 0: level walker up to level JMAX; 1: branch walker up to JMAX segments.
// lds: the block's [LDSL][6][BLOCK] child slots.  F32: FP32 phasors at the leaves.
// PRUNED: the tree may hold leaves above level J (coefficient thresholding).
template <int JMAX, int WALKER, int LDSL, int BLOCK, bool F32 = false, bool PRUNED = false>
__device__ __forceinline__ void tree_row(const TRec* recs, int n_roots, int J,
                                         const TreeArgs& ta, LdsPtr lds, double U, double V,
                                         double W, double& Vr, double& Vi) {
    const RecPtr rec = uniform_ptr(recs);
    Vr = 0.0;
    Vi = 0.0;
    int pos = 0;
    for (int r = 0; r < n_roots; ++r) {
        const int root = pos++;
        double er, ei;
        if constexpr (WALKER == 0)
            walk<1, JMAX, LDSL, BLOCK, F32, PRUNED>(rec, pos, J, ta, lds, U, V, W, er, ei, Vr, Vi);
        else
            seg_walk<1, JMAX, LDSL, BLOCK, F32, PRUNED>(rec, pos, J, ta, lds, U, V, W, er, ei, Vr,
                                                         Vi);
        // A_1 lambda_1 eta_1 with eta_1 = T_1 / 4^(J-1); ldexp, as A_1 lambda_1
        // may be zero
        const double A1lam = ldexp(rec[root].a, -2 * (J - 1));
        Vr = fma(A1lam, er, Vr);
        Vi = fma(A1lam, ei, Vi);
    }
}

}  // namespace swv
