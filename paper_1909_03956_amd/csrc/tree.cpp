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

// The factor a node record's coefficients carry for the traversal:
// gamma^m_j sigma^m_j = gamma^m_j (sqrt(A_j)/4) sum_c s^m_c eta_{j+1,c}, and the
// traversal hands up T_{j+1} = 4^(J-j-1) eta_{j+1} and forms the sums relative
// to the node's first child c0 (times s^m_{c0}), so the record holds
// h^m = s^m_{c0} gamma^m_j (sqrt(A_j)/4) 4^-(J-j-1) and the row's work for the
// node's part of Eq. 17 is one product per coefficient.
static double record_factor(int j, int J) { return std::ldexp(level_scale(j), -2 * (J - j - 1)); }

static void record_coefficients(double a, unsigned mask, const double* gamma, const bool* keep,
                                double* h) {
    const int c0 = mask ? __builtin_ctz(mask) : 0;
    for (int m = 0; m < 3; ++m) h[m] = keep[m] ? kSign[m][c0] * (a * gamma[m]) : 0.0;
}

static void emit(const swv_tree_s& t, int j, int64_t idx, std::vector<TRec>& out) {
    if (j == t.J) {
        out.push_back(TRec{t.leaf_l[idx], t.leaf_m[idx], t.leaf_nm1[idx], make_meta(0, j, 0)});
        return;
    }
    const TreeLevel& L = t.levels[j - 1];
    const bool all[3] = {true, true, true};
    double h[3];
    record_coefficients(record_factor(j, t.J), (unsigned)L.mask[idx], &L.gamma[3 * idx], all, h);
    out.push_back(TRec{h[0], h[1], h[2], make_meta((unsigned)L.mask[idx], j, L.chain[idx])});
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

    // one-child runs and branching depth, bottom-up
    std::vector<int> depth_below(nl, 0);   // branching nodes strictly below, per node
    top.chain.assign(nl, 0);
    t->n_one_child = 0;
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
            if (nch == 1) {
                L.chain[k] = 1 + (j + 1 < J ? below.chain[c0] : 0);
                ++t->n_one_child;
            }
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

// ------------------------------------------------------------ thresholding --
// Hard thresholding of the wavelet coefficients, the retention of a fixed
// proportion that section 1 cites (the paper itself keeps every non-zero
// coefficient).  The coefficients of Eq. 10 are orthonormal (sqrt(A_j)/4), so
// their magnitudes rank across levels.

std::vector<int64_t> retain_fraction(const swv_tree_s& t, double fraction) {
    std::vector<double> mag;
    for (int j = 1; j < t.J; ++j)
        for (double g : t.levels[j - 1].gamma) mag.push_back(std::fabs(g));
    const int64_t n = (int64_t)mag.size();
    std::vector<int64_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    // largest first, ties to the lower flat index
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return mag[a] > mag[b]; });
    int64_t keep = (int64_t)std::floor(fraction * (double)n + 0.5);
    keep = std::max<int64_t>(0, std::min<int64_t>(n, keep));
    std::vector<int64_t> kept(order.begin(), order.begin() + keep);
    std::sort(kept.begin(), kept.end());
    return kept;
}

namespace {

struct Pruner {
    const swv_tree_s& t;
    const Frame F;
    std::vector<int64_t> off;                    // flat offset of level j's coefficients
    std::vector<uint8_t> keep;                   // per flat index
    std::vector<std::vector<uint8_t>> alive;     // [j - 1][k], levels < J
    std::vector<std::vector<int32_t>> chain;     // one-child runs of the pruned tree
    std::vector<std::vector<int32_t>> depth;     // branching nodes at and below
    swv_tree_s* out;

    Pruner(const swv_tree_s& tt, swv_tree_s* o) : t(tt), F(make_frame(tt.ra_p, tt.dec_p)), out(o) {}

    void emit(int j, int64_t idx) {
        if (j == t.J) {
            out->records.push_back(
                TRec{t.leaf_l[idx], t.leaf_m[idx], t.leaf_nm1[idx], make_meta(0, j, 0)});
            out->levels[j - 1].pix.push_back(t.leaf_pix[idx]);
            out->leaf_pix.push_back(t.leaf_pix[idx]);
            return;
        }
        const TreeLevel& L = t.levels[j - 1];
        if (!alive[j - 1][idx]) {
            // nothing retained here or below: a leaf at its own level, the
            // plane wave sampled at its pixel centre
            ld xyz[3];
            double l, m, nm1;
            pix2xyz(j, L.pix[idx], xyz);
            xyz_to_lmn(F, xyz, &l, &m, &nm1);
            out->records.push_back(TRec{l, m, nm1, make_meta(0, j, 0)});
            out->levels[j - 1].pix.push_back(L.pix[idx]);
            out->leaf_pix.push_back(L.pix[idx]);
            return;
        }
        const int64_t f = off[j - 1] + 3 * idx;
        const bool kept3[3] = {keep[f] != 0, keep[f + 1] != 0, keep[f + 2] != 0};
        double h[3];
        record_coefficients(record_factor(j, t.J), (unsigned)L.mask[idx], &L.gamma[3 * idx], kept3,
                            h);
        out->records.push_back(
            TRec{h[0], h[1], h[2], make_meta((unsigned)L.mask[idx], j, chain[j - 1][idx])});
        out->levels[j - 1].pix.push_back(L.pix[idx]);
        ++out->n_alive;
        if (__builtin_popcount((unsigned)L.mask[idx]) == 1) ++out->n_one_child;
        int64_t child = L.first_child[idx];
        for (int c = 0; c < 4; ++c)
            if (L.mask[idx] & (1 << c)) emit(j + 1, child++);
    }
};

}  // namespace

int prune_tree(const swv_tree_s& t, const std::vector<int64_t>& kept, swv_tree_s* out) {
    const auto t0 = std::chrono::steady_clock::now();
    const int J = t.J;
    Pruner P(t, out);
    P.off.assign(J, 0);
    for (int j = 1; j < J; ++j) P.off[j] = P.off[j - 1] + 3 * (int64_t)t.levels[j - 1].pix.size();
    const int64_t n_coeffs = J > 1 ? P.off[J - 1] : 0;
    P.keep.assign((size_t)n_coeffs, 0);
    for (int64_t f : kept) {
        if (f < 0 || f >= n_coeffs)
            return fail(SWV_EINVAL, "coefficient index %lld outside [0, %lld)", (long long)f,
                        (long long)n_coeffs);
        P.keep[(size_t)f] = 1;
    }
    // bottom-up: whether a node keeps a coefficient at or below it, its
    // one-child run and its branching depth in the pruned tree
    P.alive.assign(J, {});
    P.chain.assign(J, {});
    P.depth.assign(J, {});
    for (int j = J - 1; j >= 1; --j) {
        const TreeLevel& L = t.levels[j - 1];
        const int64_t n = (int64_t)L.pix.size();
        P.alive[j - 1].assign(n, 0);
        P.chain[j - 1].assign(n, 0);
        P.depth[j - 1].assign(n, 0);
        for (int64_t k = 0; k < n; ++k) {
            const int64_t f = P.off[j - 1] + 3 * k;
            bool a = P.keep[f] || P.keep[f + 1] || P.keep[f + 2];
            const int nch = __builtin_popcount((unsigned)L.mask[k]);
            const int64_t c0 = L.first_child[k];
            int d = 0;
            if (j + 1 < J)
                for (int i = 0; i < nch; ++i)
                    if (P.alive[j][c0 + i]) {
                        a = true;
                        d = std::max(d, P.depth[j][c0 + i]);
                    }
            P.alive[j - 1][k] = a;
            P.depth[j - 1][k] = d + (nch >= 2 ? 1 : 0);
            if (nch == 1)
                P.chain[j - 1][k] =
                    1 + ((j + 1 < J && P.alive[j][c0]) ? P.chain[j][c0] : 0);
        }
    }
    out->J = J;
    out->ra_p = t.ra_p;
    out->dec_p = t.dec_p;
    out->n_comp = t.n_comp;
    out->thresholded = true;
    out->n_coeffs = n_coeffs;
    out->kept = kept;
    out->levels.assign(J, TreeLevel());
    out->records.clear();
    out->leaf_pix.clear();
    out->n_alive = 0;
    out->n_one_child = 0;
    out->max_branching = 0;
    const TreeLevel& L1 = t.levels[0];
    const double A1 = pixel_area(1);
    out->n_roots = (int64_t)L1.pix.size();
    for (int64_t r = 0; r < out->n_roots; ++r) {
        out->records.push_back(TRec{A1 * L1.lambda[r], 0.0, 0.0, 0ull});
        P.emit(1, r);
        if (J > 1 && P.alive[0][r]) out->max_branching = std::max(out->max_branching, P.depth[0][r]);
    }
    out->build_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return SWV_OK;
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
