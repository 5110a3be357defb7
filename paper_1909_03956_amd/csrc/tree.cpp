// Host construction of the sparse spherical-Haar coefficient tree.
//
// Model side, once per major cycle (section 3.6.1):
//   * each component is rotated to xyz (Eq. 18) and assigned its level-J
//     nested pixel (section 3.5's cross-reference);
//   * components in one pixel are summed (the distinct components of
//     section 3.3); the leaf sits at the pixel centre;
//   * lambda_J = F / A_J, and for every existing node of levels J-1 .. 1
//     lambda_j = 1/4 sum_c lambda_{j+1,4k+c}            (Eq. 9)
//     gamma^m_j = sqrt(A_j)/4 sum_c s^m_c lambda_{j+1}  (Eq. 10)
//     with ancestors k_j = k_J >> 2(J - j) (section 3.5).
// The levels are kept as sorted, level-ordered arrays.  For the per-visibility
// traversal the tree is also written as one depth-first (pre-order) record
// stream: a root record per level-1 node, then node records, each followed by
// its children's subtrees in child order, with leaf records at level J.
// Runs of one-child nodes are marked in the stream, and the largest number of
// branching nodes on a path is recorded, for a traversal that keeps state
// only for branching ancestors.
#include "tree.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>

#include "sphere.h"

namespace swv {

// Eq. 10 sign pattern s^m_c (row m, column c).
static const double kSign[3][4] = {{+1, -1, +1, -1}, {+1, +1, -1, -1}, {+1, -1, -1, +1}};

static void emit(const swv_tree_s& t, int j, int64_t idx, std::vector<TRec>& out) {
    if (j == t.J) {
        out.push_back(TRec{t.leaf_l[idx], t.leaf_m[idx], t.leaf_nm1[idx], make_meta(0, j, 0)});
        return;
    }
    const TreeLevel& L = t.levels[j - 1];
    out.push_back(TRec{L.gamma[3 * idx], L.gamma[3 * idx + 1], L.gamma[3 * idx + 2],
                       make_meta((unsigned)L.mask[idx], j, L.chain[idx])});
    int64_t child = L.first_child[idx];
    for (int c = 0; c < 4; ++c)
        if (L.mask[idx] & (1 << c)) emit(t, j + 1, child++, out);
}

void build_coefficients(swv_tree_s* t) {
    const int J = t->J;
    const int64_t nl = (int64_t)t->leaf_pix.size();
    // levels J .. 1
    t->levels.assign(J, TreeLevel());
    TreeLevel& top = t->levels[J - 1];
    top.pix = t->leaf_pix;
    top.mask.assign(nl, 0);
    top.first_child.assign(nl, -1);
    top.gamma.assign(3 * nl, 0.0);
    top.lambda.resize(nl);
    const double AJ = pixel_area(J);
    for (int64_t k = 0; k < nl; ++k) top.lambda[k] = t->leaf_flux[k] / AJ;

    for (int j = J - 1; j >= 1; --j) {
        const TreeLevel& below = t->levels[j];
        TreeLevel& L = t->levels[j - 1];
        const double a = std::sqrt(pixel_area(j)) / 4.0;
        const int64_t nb = (int64_t)below.pix.size();
        for (int64_t s = 0; s < nb;) {
            const int64_t parent = below.pix[s] >> 2;
            int32_t mask = 0;
            double lam = 0.0, g[3] = {0.0, 0.0, 0.0};
            int64_t e = s;
            for (; e < nb && (below.pix[e] >> 2) == parent; ++e) {
                const int c = (int)(below.pix[e] & 3);
                mask |= 1 << c;
                const double x = below.lambda[e];
                lam += x;
                for (int mm = 0; mm < 3; ++mm) g[mm] += kSign[mm][c] * x;
            }
            L.pix.push_back(parent);
            L.mask.push_back(mask);
            L.first_child.push_back(s);
            L.lambda.push_back(0.25 * lam);
            for (int mm = 0; mm < 3; ++mm) L.gamma.push_back(a * g[mm]);
            s = e;
        }
    }
    // sqrt(A_j)/4; A_j = A_1 4^(1-j), so every level's factor is the level-1
    // factor times an exact power of two (the device forms it that way too)
    for (int j = 1; j <= SWV_MAX_LEVEL; ++j) t->level_scale[j] = level_scale(j);

    // one-child runs and branching depth, bottom-up
    std::vector<int> depth_below(nl, 0);   // branching nodes strictly below, per node
    top.chain.assign(nl, 0);
    for (int j = J - 1; j >= 1; --j) {
        TreeLevel& L = t->levels[j - 1];
        const TreeLevel& below = t->levels[j];
        const int64_t n = (int64_t)L.pix.size();
        L.chain.assign(n, 0);
        std::vector<int> depth(n, 0);
        for (int64_t k = 0; k < n; ++k) {
            const int nch = __builtin_popcount((unsigned)L.mask[k]);
            const int64_t c0 = L.first_child[k];
            int d = 0;
            for (int i = 0; i < nch; ++i) d = std::max(d, depth_below[c0 + i]);
            depth[k] = d + (nch >= 2 ? 1 : 0);
            if (nch == 1) L.chain[k] = 1 + (j + 1 < J ? below.chain[c0] : 0);
        }
        depth_below.swap(depth);
    }
    t->max_branching = 0;
    for (int d : depth_below) t->max_branching = std::max(t->max_branching, d);

    // depth-first record stream
    t->records.clear();
    const TreeLevel& L1 = t->levels[0];
    const double A1 = pixel_area(1);
    t->n_roots = (int64_t)L1.pix.size();
    for (int64_t r = 0; r < t->n_roots; ++r) {
        t->records.push_back(TRec{A1 * L1.lambda[r], 0.0, 0.0, 0ull});
        emit(*t, 1, r, t->records);
    }
}

int build_tree_pixels(int J, double ra_p, double dec_p, int64_t n, const int64_t* kJ,
                      const double* flux, swv_tree_s* t) {
    const auto t0 = std::chrono::steady_clock::now();
    const Frame F = make_frame(ra_p, dec_p);
    std::vector<int64_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return kJ[a] < kJ[b]; });

    t->J = J;
    t->ra_p = ra_p;
    t->dec_p = dec_p;
    t->n_comp = n;
    t->leaf_pix.clear();
    t->leaf_flux.clear();
    for (int64_t s = 0; s < n;) {
        int64_t e = s;
        double f = 0.0;
        while (e < n && kJ[order[e]] == kJ[order[s]]) f += flux[order[e++]];
        t->leaf_pix.push_back(kJ[order[s]]);
        t->leaf_flux.push_back(f);
        s = e;
    }
    const int64_t nl = (int64_t)t->leaf_pix.size();
    t->leaf_l.resize(nl);
    t->leaf_m.resize(nl);
    t->leaf_nm1.resize(nl);
    for (int64_t k = 0; k < nl; ++k) {
        ld xyz[3];
        pix2xyz(J, t->leaf_pix[k], xyz);
        xyz_to_lmn(F, xyz, &t->leaf_l[k], &t->leaf_m[k], &t->leaf_nm1[k]);
    }

    build_coefficients(t);
    t->build_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return SWV_OK;
}

int build_tree(int J, double ra_p, double dec_p, int64_t n, const double* l, const double* m,
               const double* flux, swv_tree_s* t) {
    const auto t0 = std::chrono::steady_clock::now();
    const Frame F = make_frame(ra_p, dec_p);
    // pixel of every component
    std::vector<int64_t> kJ(n);
    for (int64_t i = 0; i < n; ++i) {
        ld xyz[3];
        lm_to_xyz(F, l[i], m[i], xyz);
        kJ[i] = ang2pix(J, xyz);
    }
    const int rc = build_tree_pixels(J, ra_p, dec_p, n, kJ.data(), flux, t);
    t->build_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

}  // namespace swv
