// Wavelet-tree route (section 3.3, Eqs. 14-17; section 3.5) on gfx950: the
// kernel and its launch, instantiated per precision in k_tree.hip (FP64) and
// k_tree_f32c.hip (FP32 leaf phasors).
//
// Per visibility row (one per lane) the paper's work is: the plane wave at
// the leaves (eta_J), the plane-wave coefficients up the tree (eta_j and
// sigma^m_j by Eqs. 9 and 10 applied to the plane wave), and the
// reconstruction sum of Eq. 17.  Every lane traverses the same tree, so the
// traversal is wave-uniform: the tree comes as one pre-order stream of
// 32-byte records read with scalar loads, and the branches on child masks
// are scalar branches.
//
// Depth-first order keeps the live state O(J) per lane: while a subtree is
// walked, each open ancestor at level j holds its running sums
//     S = sum_c eta_{j+1,c},   D^m = sum_c s^m_c eta_{j+1,c}   (m = 0, 1, 2)
// over the children finished so far (4 complex FP64 values).  When the last
// child returns, the node forms eta_j = S / 4 and sigma^m_j = sqrt(A_j)/4 D^m,
// adds gamma^m_j sigma^m_j to V, and hands eta_j to its parent.  The level is
// a template parameter, so each open level's sums live in their own
// registers (the deepest levels; the ones above keep their finished children
// in LDS or private-memory slots); one call site per level (inside a loop
// over the set bits of the child mask) keeps the code linear in J.  Roots add
// A_1 lambda_1 eta_1.
// Three rewritings cut the arithmetic (see tree_walk.h): nodes hand up
// T_j = 4^(J-j) eta_j, the plain sum of the leaf phasors below, with the
// quarters moved into the node constants as exact powers of two; the level
// walker keeps D^m relative to a node's first child, which then enters every
// sum without a sign product (both exact); and a node's record carries
// gamma^m_j times its constant sqrt(A_j)/4 4^-(J-j-1), multiplied once per
// tree on the host, so gamma^m_j sigma^m_j costs one FMA per part per row.
//
// Deep trees are mostly runs of one-child nodes, so a second traversal (the
// branch walker) keeps a register set only for open BRANCHING nodes: a run of
// one-child nodes holds nothing while the subtree below it is walked and is
// closed bottom-up afterwards.  Its depth parameter is the number of nested
// branchings, which stays small (a few to a dozen) at any J, so it serves
// J = 1 .. 29; both traversals give the same values bit for bit (up to the
// sign of an exactly-zero intermediate).
//
// Imaginary parts are carried divided by 4 (cis2pi_q's convention; every step
// is linear) and scaled back once at the end.
#pragma once

#include "tree_walk.h"

namespace swv {

// PREC: SWV_FP64 (complex128 out) or SWV_F32C (FP32 leaf phasors, complex64 out).
template <int JMAX, int BLOCK, int WALKER, int PREC, bool PRUNED = false>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(tree_waves_per_simd<JMAX, WALKER>()))) void k_tree(TreeArgs ta, const double* __restrict__ u,
                                                const double* __restrict__ v,
                                                const double* __restrict__ w, int64_t n_vis,
                                                double sgn, void* __restrict__ out,
                                                int* __restrict__ status) {
    const int64_t jrow = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t j = jrow < n_vis ? jrow : n_vis - 1;
    const double U = u[j], V = v[j], W = w[j];
    constexpr int LDSL = tree_lds_levels<JMAX, WALKER, BLOCK>();
    __shared__ double sums[LDSL > 0 ? LDSL * kSlotDoubles * BLOCK : 1];
    double Vr, Vi;
    // the level walker is launched for the tree's own J (JMAX = J), which
    // the compiler then folds into every level test
    const int J = WALKER == 0 ? JMAX : ta.J;
    tree_row<JMAX, WALKER, LDSL, BLOCK, PREC == SWV_F32C, PRUNED>(ta.rec, ta.n_roots, J,
                                                                  (LdsPtr)sums, U, V, W, Vr, Vi);
    if (jrow < n_vis) {
        if (!isfinite(U + V + W)) atomicOr(status, kStatusNonFinite);
        if constexpr (PREC == SWV_F32C)
            ((float2*)out)[jrow] = make_float2((float)Vr, (float)(4.0 * sgn * Vi));
        else
            ((double2*)out)[jrow] = make_double2(Vr, 4.0 * sgn * Vi);
    }
}

template <int JMAX, int WALKER, int PREC>
static hipError_t run_tree_p(hipStream_t s, int block, const TreeArgs& t, int64_t n_vis,
                             const double* u, const double* v, const double* w, int sign,
                             void* out, int* status) {
    const double sg = (double)sign;
    if (t.pruned) {
        // thresholded trees: one block shape
        k_tree<JMAX, 64, WALKER, PREC, true><<<dim3((unsigned)((n_vis + 63) / 64)), dim3(64), 0, s>>>(
            t, u, v, w, n_vis, sg, out, status);
        return hipGetLastError();
    }
    switch (block) {
        case 64:
            k_tree<JMAX, 64, WALKER, PREC><<<dim3((unsigned)((n_vis + 63) / 64)), dim3(64), 0, s>>>(
                t, u, v, w, n_vis, sg, out, status);
            break;
        case 128:
            k_tree<JMAX, 128, WALKER, PREC><<<dim3((unsigned)((n_vis + 127) / 128)), dim3(128), 0, s>>>(
                t, u, v, w, n_vis, sg, out, status);
            break;
        case 256:
            k_tree<JMAX, 256, WALKER, PREC><<<dim3((unsigned)((n_vis + 255) / 256)), dim3(256), 0, s>>>(
                t, u, v, w, n_vis, sg, out, status);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#define SWV_TREE_CASE(N, W) \
    case N: return run_tree_p<N, W, PREC>(s, block, t, n_vis, u, v, w, sign, out, status);

// Launch of the traversal compiled for this tree's depth, in precision PREC.
template <int PREC>
hipError_t launch_tree_prec(hipStream_t s, int walker, int block, const TreeArgs& t,
                            int64_t n_vis, const double* u, const double* v, const double* w,
                            int sign, void* out, int* status) {
    if (n_vis <= 0) return hipSuccess;
    if (walker == 0) {
        // the compiled traversal depth is the tree's J: register use grows with it
        switch (t.J) {
            SWV_TREE_CASE(1, 0) SWV_TREE_CASE(2, 0) SWV_TREE_CASE(3, 0) SWV_TREE_CASE(4, 0)
            SWV_TREE_CASE(5, 0) SWV_TREE_CASE(6, 0) SWV_TREE_CASE(7, 0) SWV_TREE_CASE(8, 0)
            SWV_TREE_CASE(9, 0) SWV_TREE_CASE(10, 0) SWV_TREE_CASE(11, 0) SWV_TREE_CASE(12, 0)
            SWV_TREE_CASE(13, 0) SWV_TREE_CASE(14, 0) SWV_TREE_CASE(15, 0) SWV_TREE_CASE(16, 0)
            default: return hipErrorInvalidValue;
        }
    }
    // branch walker: compiled for the tree's number of nested segments
    switch (t.seg_depth) {
        SWV_TREE_CASE(1, 1) SWV_TREE_CASE(2, 1) SWV_TREE_CASE(3, 1) SWV_TREE_CASE(4, 1)
        SWV_TREE_CASE(5, 1) SWV_TREE_CASE(6, 1) SWV_TREE_CASE(7, 1) SWV_TREE_CASE(8, 1)
        SWV_TREE_CASE(9, 1) SWV_TREE_CASE(10, 1) SWV_TREE_CASE(11, 1) SWV_TREE_CASE(12, 1)
        SWV_TREE_CASE(13, 1) SWV_TREE_CASE(14, 1) SWV_TREE_CASE(15, 1) SWV_TREE_CASE(16, 1)
        default: return hipErrorInvalidValue;
    }
}

#undef SWV_TREE_CASE

}  // namespace swv
