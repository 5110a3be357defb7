// Depth-first traversal of the wavelet tree for one visibility row per
// lane, shared by the single-instance and the persistent batched kernels.
// The algorithm is described in k_tree.hip.
#pragma once

#include "device_math.h"
#include "launch.h"

namespace swv {

using RecPtr = const __attribute__((address_space(4))) TRec*;

// The walkers address the record stream by byte offset (a 32-bit scalar that
// steps by 32), so a record's address is one 64-bit add to the base; the host
// keeps streams below 4 GiB.
constexpr unsigned kRecBytes = sizeof(TRec);
__device__ __forceinline__ RecPtr rec_at(RecPtr base, unsigned off) {
    return (RecPtr)((const __attribute__((address_space(4))) char*)base + off);
}
using LdsPtr = __attribute__((address_space(3))) double*;
using PrivPtr = __attribute__((address_space(5))) double*;

// Branch walker, open segment levels 1 .. DMAX-1 (DMAX: the compiled
// branching depth): the deepest branch_reg_levels keep their running sums in
// registers, the branch_lds_levels above them keep their children in LDS (see
// slot_put; within 64 KB per block), the rest in private memory; compiled for
// branch_waves waves per SIMD (1: left to the compiler).  Measured (one
// MI355X, median of seven) with 3 + 3 levels at 4 waves against the earlier
// 5 register levels and every level above in LDS (2-3 waves): the run-time
// sweep's 140 components at J = 12, 16, 20, 25 0.76, 0.96, 1.20, 1.43 ms
// against 0.83, 1.09, 1.37, 1.66; cfg2 at J = 11, 12 14.9 and 23.4 ms against
// 17.5 and 27.4; 4 + 2 at 4 waves within 3 %, 2-3 register levels at 5 waves
// 1-8 % slower than 3 + 3.
template <int DMAX>
constexpr int branch_reg_levels() { return 3; }
template <int DMAX>
constexpr int branch_lds_levels() { return 3; }
template <int DMAX>
constexpr int branch_waves() { return DMAX >= 5 ? 4 : 1; }
// Level walker, open levels 1 .. JMAX-1 (level JMAX holds the leaves): the
// deepest level_reg_levels in registers, the level_lds_levels above them in
// LDS, the rest in private memory, compiled for level_waves waves per SIMD (1:
// left to the compiler).  Chosen by measurement at cfg2 J = 8, 9, 10 (one
// MI355X, median of nine launches): 3 register and 2 LDS levels at 5 waves
// per SIMD (96 VGPRs, 6 KB of LDS per wave) give 1.13, 2.98 and 6.02 ms;
// 2 + 2 levels 1.15, 3.04 and 6.31 ms (J = 8, 9 at 3 + 3 and 4 waves); 4 + 2
// at 4 waves 1.14, 3.03 and 6.28 ms.  Before the depth was a compile-time
// constant and the first child's signs sat in the records, 2 + 2 at 5 waves
// was the best at J = 10 and one register set per level at 3 waves took
// 8.67 ms.
template <int JMAX>
constexpr int level_reg_levels() { return 3; }
template <int JMAX>
constexpr int level_lds_levels() { return 2; }
template <int JMAX>
constexpr int level_waves() { return JMAX >= 8 ? 5 : 1; }

// Running sums of an open node at level j over its finished children, whose
// values are T_{j+1,c} = 4^(J-j-1) eta_{j+1,c} (the plain sums of the leaf
// phasors below them, see close_node), the D^m taken relative to the node's
// first child c0:
//   S = sum_c T_{j+1,c},   D^m = s^m_{c0} sum_c s^m_c T_{j+1,c}   (m = 0, 1, 2),
// so the first child's value enters every sum as it is, and the sign
// s^m_{c0} sits in the node's coefficient, which the host stores multiplied
// by it.  With s = +-1 and rounding symmetric in sign, each value is the
// plain sum times s^m_{c0} exactly, so the result comes out the same bit for
// bit.  (The branch walker starts its sums at zero.)
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
// signs of c ^ c0.  `first` is the same for every lane, so this is a scalar
// branch, and no sums need zeroing.
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

// Closes a node at level j.  The record carries the node's coefficients
// already multiplied by its scale and by the signs of its first child c0,
//   h^m = s^m_{c0} gamma^m_j a,   a = (sqrt(A_j)/4) 4^-(J-j-1),
// so gamma^m_j sigma^m_j (Eq. 10 on the plane wave, then Eq. 17) is h^m D^m
// with the sums relative to c0, one FMA per part and no per-row sign work:
// sigma^m_j = sqrt(A_j)/4 sum_c s^m_c eta_{j+1,c} and the children's sums are
// T_{j+1} = 4^(J-j-1) eta_{j+1}.  Passing T_j = sum over the leaves below of
// eta_J instead of eta_j = T_j / 4^(J-j) (Eq. 9 on the plane wave) keeps every
// quarter out of the per-row work.  T_j goes to the parent.
__device__ __forceinline__ void close_node(const NodeSums& n, double h0, double h1, double h2,
                                           double& er, double& ei, double& Vr, double& Vi) {
    er = n.Sr;
    ei = n.Si;
    Vr = fma(h0, n.D0r, Vr);
    Vi = fma(h0, n.D0i, Vi);
    Vr = fma(h1, n.D1r, Vr);
    Vi = fma(h1, n.D1i, Vi);
    Vr = fma(h2, n.D2r, Vr);
    Vi = fma(h2, n.D2i, Vi);
}

// Adds gamma^m_j sigma^m_j of a node whose only child returned the sum x
// (T_j = x, D^m relative to that child = x): close_node's arithmetic.
__device__ __forceinline__ void close_single(double h0, double h1, double h2, double xr,
                                             double xi, double& Vr, double& Vi) {
    Vr = fma(h0, xr, Vr);
    Vi = fma(h0, xi, Vi);
    Vr = fma(h1, xr, Vr);
    Vi = fma(h1, xi, Vi);
    Vr = fma(h2, xr, Vr);
    Vi = fma(h2, xi, Vi);
}

// Open nodes above the register levels (level walker) or segments (branch
// walker) keep their children's plane-wave coefficients in a slot (LDS, or
// for the level walker's topmost levels the lane's private memory) rather
// than running sums in registers: such a node is touched only when one of its
// few children finishes, and its registers would otherwise stay allocated
// through every subtree below it, which limits how many waves share a SIMD.  A node
// holds at most three finished children while its last one is walked, so a
// slot is three complex values (6 doubles, against 8 for the four running
// sums); the sums are formed when the last child is back, in child order, so
// they equal the register levels' bit for bit.  Layout [slot][6][BLOCK]:
// lane-contiguous, so the accesses are free of bank conflicts; private
// slots are [slot][6] per lane.  The accesses are volatile: otherwise the
// compiler, seeing the whole inlined walk, forwards each stored value to its
// reload and keeps it in registers.
constexpr int kSlotDoubles = 6;

//
// Private slots hold the level walker's topmost levels, whose slots are
// touched least (once per child of a node there: at cfg2 J = 10 levels 1-5
// take 22 values per row, levels 6-7 117, levels 8-9 804).
template <int BLOCK, bool PRIV>
__device__ __forceinline__ void slot_put(LdsPtr lds, PrivPtr priv, int slot, int k, double xr,
                                         double xi) {
    if constexpr (PRIV) {
        volatile __attribute__((address_space(5))) double* p = priv + slot * kSlotDoubles + 2 * k;
        p[0] = xr;
        p[1] = xi;
    } else {
        volatile __attribute__((address_space(3))) double* p =
            lds + (slot * kSlotDoubles + 2 * k) * BLOCK + threadIdx.x;
        p[0] = xr;
        p[BLOCK] = xi;
    }
}

template <int BLOCK, bool PRIV>
__device__ __forceinline__ void slot_get(LdsPtr lds, PrivPtr priv, int slot, int k, double& xr,
                                         double& xi) {
    if constexpr (PRIV) {
        const volatile __attribute__((address_space(5))) double* p =
            priv + slot * kSlotDoubles + 2 * k;
        xr = p[0];
        xi = p[1];
    } else {
        const volatile __attribute__((address_space(3))) double* p =
            lds + (slot * kSlotDoubles + 2 * k) * BLOCK + threadIdx.x;
        xr = p[0];
        xi = p[BLOCK];
    }
}

// Adds the k children kept in a slot to n, in child order, relative to
// child c0; `all` is the node's child mask, whose k lowest set bits name them.
template <int BLOCK, bool PRIV>
__device__ __forceinline__ void slot_replay(LdsPtr lds, PrivPtr priv, int slot, int k,
                                            unsigned all, int c0, NodeSums& n, bool& first) {
    for (int q = 0; q < k; ++q) {
        const int c = __builtin_ctz(all);
        all &= all - 1;
        double xr, xi;
        slot_get<BLOCK, PRIV>(lds, priv, slot, q, xr, xi);
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

// Leaf: eta_{J,k} = exp(2 pi i B . (s_k - P)) (imaginary part / 4).  VOP3
// selects the phasor whose polynomial steps are 3-operand FMAs (same values);
// F32 the precision form: the FP64 phase, reduced exactly in FP64, then the
// FP32 hardware sine and cosine (everything after the leaf stays FP64).
template <bool VOP3, bool F32>
__device__ __forceinline__ void leaf_wave(RecPtr rec, unsigned me, double u, double v, double w,
                                          double& er, double& ei) {
    const RecPtr q = rec_at(rec, me);
    if constexpr (F32) {
        float c32, s32;
        cis2pi_f32((float)fract_phase(u, v, w, q->a, q->b, q->c), c32, s32);
        er = (double)c32;
        ei = 0.25 * (double)s32;
    } else {
        const double r = reduced_phase(u, v, w, q->a, q->b, q->c);
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
__device__ __forceinline__ void leaf_above(RecPtr rec, unsigned me, int j, int J, double u,
                                           double v, double w, double& er, double& ei) {
    leaf_wave<false, F32>(rec, me, u, v, w, er, ei);
    const double s = pow2_scale(1.0, 2 * (J - j));
    er *= s;
    ei *= s;
}

// Level walker: one register set per level, the level a template parameter
// (levels <= PRIVL keep theirs in private memory, the next LDSL in LDS).
template <int LVL, int JMAX, int LDSL, int PRIVL, int BLOCK, bool F32, bool PRUNED>
__device__ __forceinline__ void walk(RecPtr rec, unsigned& pos, const int J, LdsPtr lds,
                                     PrivPtr priv, const double u, const double v,
                                     const double w, double& er, double& ei, double& Vr,
                                     double& Vi) {
    const unsigned me = pos;
    pos += kRecBytes;
    if (LVL == JMAX || LVL == J) {
        leaf_wave<true, F32>(rec, me, u, v, w, er, ei);
        return;
    }
    if constexpr (LVL < JMAX) {
        const unsigned all = meta_mask(rec_at(rec, me)->meta);
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
        if constexpr (LVL <= PRIVL + LDSL) {
            // every child but the last waits in the slot (stored when the
            // next one starts); only the last one's value leaves the loop
            constexpr bool PRIV = LVL <= PRIVL;
            constexpr int SLOT = PRIV ? LVL - 1 : LVL - PRIVL - 1;
            int k = 0, c = 0;
            double xr = 0.0, xi = 0.0;
            while (mask) {
                if (mask != all) slot_put<BLOCK, PRIV>(lds, priv, SLOT, k++, xr, xi);
                c = __builtin_ctz(mask);
                mask &= mask - 1;
                walk<LVL + 1, JMAX, LDSL, PRIVL, BLOCK, F32, PRUNED>(rec, pos, J, lds, priv, u, v,
                                                                     w, xr, xi, Vr, Vi);
            }
            slot_replay<BLOCK, PRIV>(lds, priv, SLOT, k, all, c0, n, first);
            add_child(n, c, c0, xr, xi, first);
        } else {
            while (mask) {
                const int c = __builtin_ctz(mask);
                mask &= mask - 1;
                double xr, xi;
                walk<LVL + 1, JMAX, LDSL, PRIVL, BLOCK, F32, PRUNED>(rec, pos, J, lds, priv, u, v,
                                                                     w, xr, xi, Vr, Vi);
                add_child(n, c, c0, xr, xi, first);
                first = false;
            }
        }
        const RecPtr q = rec_at(rec, me);
        close_node(n, q->a, q->b, q->c, er, ei, Vr, Vi);
    }
}

// Branch walker: one register set per open BRANCHING node, so any J.  A
// segment is a run of one-child nodes (possibly empty) and the leaf or
// branching node below it; the run keeps no state while the part below is
// walked, and is closed bottom-up afterwards with the same arithmetic a
// one-child node gets in the level walker.  D counts segments from the root;
// the host launches DMAX >= 1 + the tree's largest branching count on a path.
template <int D, int DMAX, int LDSL, int PRIVL, int BLOCK, bool F32, bool PRUNED>
__device__ __forceinline__ void seg_walk(RecPtr rec, unsigned& pos, const int J, LdsPtr lds,
                                         PrivPtr priv, const double u, const double v,
                                         const double w, double& er, double& ei, double& Vr,
                                         double& Vi) {
    const unsigned first = pos;
    const int run = meta_chain(rec_at(rec, first)->meta);
    const unsigned term = first + (unsigned)run * kRecBytes;
    pos = term + kRecBytes;
    const unsigned long long mt = rec_at(rec, term)->meta;
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
            // zero and take every child with the signs of c ^ c0 (relative
            // to its first child, as the record's coefficients are); the
            // level walker's first-child seeding costs this walker more in
            // scalar registers than it saves
            const unsigned all = meta_mask(mt);
            const int c0 = __builtin_ctz(all);
            unsigned mask = all;
            NodeSums n{};
            bool first = false;
            if constexpr (D <= PRIVL + LDSL) {
                // as in the level walker: all children but the last wait in
                // the slot, and the sums are formed at the end
                constexpr bool PRIV = D <= PRIVL;
                constexpr int SLOT = PRIV ? D - 1 : D - PRIVL - 1;
                int k = 0, c = 0;
                double xr = 0.0, xi = 0.0;
                while (mask) {
                    if (mask != all) slot_put<BLOCK, PRIV>(lds, priv, SLOT, k++, xr, xi);
                    c = __builtin_ctz(mask);
                    mask &= mask - 1;
                    seg_walk<D + 1, DMAX, LDSL, PRIVL, BLOCK, F32, PRUNED>(rec, pos, J, lds, priv,
                                                                           u, v, w, xr, xi, Vr,
                                                                           Vi);
                }
                slot_replay<BLOCK, PRIV>(lds, priv, SLOT, k, all, c0, n, first);
                add_child(n, c, c0, xr, xi, false);
            } else {
                while (mask) {
                    const int c = __builtin_ctz(mask);
                    mask &= mask - 1;
                    double xr, xi;
                    seg_walk<D + 1, DMAX, LDSL, PRIVL, BLOCK, F32, PRUNED>(rec, pos, J, lds, priv,
                                                                           u, v, w, xr, xi, Vr,
                                                                           Vi);
                    add_child(n, c, c0, xr, xi, false);
                }
            }
            const RecPtr q = rec_at(rec, term);
            close_node(n, q->a, q->b, q->c, er, ei, Vr, Vi);
        }
    }
    // the run, bottom-up
    for (int i = run - 1; i >= 0; --i) {
        const RecPtr q = rec_at(rec, first + (unsigned)i * kRecBytes);
        close_single(q->a, q->b, q->c, er, ei, Vr, Vi);
    }
}

// Levels (segments) of a traversal compiled to depth JMAX whose children go
// to LDS: for the level walker the level_lds_levels above its register levels,
// for the branch walker the branch_lds_levels above its register levels, within
// 64 KB per block.
template <int JMAX, int WALKER, int BLOCK>
constexpr int tree_lds_levels() {
    constexpr int above =
        JMAX - 1 - (WALKER == 0 ? level_reg_levels<JMAX>() : branch_reg_levels<JMAX>());
    constexpr int want = WALKER == 0 ? level_lds_levels<JMAX>() : branch_lds_levels<JMAX>();
    constexpr int block_cap = (64 * 1024) / (kSlotDoubles * 8 * BLOCK);
    constexpr int cap = want < block_cap ? want : block_cap;
    return above <= 0 ? 0 : (above < cap ? above : cap);
}

// Top levels (segments) whose children go to private memory: those above the
// register and LDS levels.
template <int JMAX, int WALKER, int BLOCK>
constexpr int tree_priv_levels() {
    constexpr int above =
        JMAX - 1 - (WALKER == 0 ? level_reg_levels<JMAX>() : branch_reg_levels<JMAX>()) -
        tree_lds_levels<JMAX, WALKER, BLOCK>();
    return above <= 0 ? 0 : above;
}

// Waves per SIMD a traversal is compiled for (the kernels' amdgpu_waves_per_eu).
template <int JMAX, int WALKER>
constexpr int tree_waves_per_simd() {
    return WALKER == 0 ? level_waves<JMAX>() : branch_waves<JMAX>();
}

// V (real, imaginary / 4) of one row: the root loop of the traversal.
// WALKER 0: level walker up to level JMAX; 1: branch walker up to JMAX segments.
// lds: the block's [LDSL][6][BLOCK] child slots.  F32: FP32 phasors at the leaves.
// PRUNED: the tree may hold leaves above level J (coefficient thresholding).
template <int JMAX, int WALKER, int LDSL, int BLOCK, bool F32 = false, bool PRUNED = false>
__device__ __forceinline__ void tree_row(const TRec* recs, int n_roots, int J, LdsPtr lds,
                                         double U, double V, double W, double& Vr, double& Vi) {
    const RecPtr rec = uniform_ptr(recs);
    constexpr int PRIVL = tree_priv_levels<JMAX, WALKER, BLOCK>();
    double slots[PRIVL > 0 ? PRIVL * kSlotDoubles : 1];
    const PrivPtr priv = (PrivPtr)slots;
    Vr = 0.0;
    Vi = 0.0;
    unsigned pos = 0;
    for (int r = 0; r < n_roots; ++r) {
        const unsigned root = pos;
        pos += kRecBytes;
        double er, ei;
        if constexpr (WALKER == 0)
            walk<1, JMAX, LDSL, PRIVL, BLOCK, F32, PRUNED>(rec, pos, J, lds, priv, U, V, W, er, ei,
                                                           Vr, Vi);
        else
            seg_walk<1, JMAX, LDSL, PRIVL, BLOCK, F32, PRUNED>(rec, pos, J, lds, priv, U, V, W, er,
                                                               ei, Vr, Vi);
        // A_1 lambda_1 eta_1 with eta_1 = T_1 / 4^(J-1); ldexp, as A_1 lambda_1
        // may be zero
        const double A1lam = ldexp(rec_at(rec, root)->a, -2 * (J - 1));
        Vr = fma(A1lam, er, Vr);
        Vi = fma(A1lam, ei, Vi);
    }
}

}  // namespace swv
