// Sparse spherical-Haar coefficient tree (sections 3.2-3.5), host side.
#pragma once

#include <cstdint>
#include <map>
#include <vector>

#include "common.h"

namespace swv {

// One level of the tree: the existing nodes in increasing pixel order.
struct TreeLevel {
    std::vector<int64_t> pix;         // nested ids, sorted
    std::vector<int32_t> mask;        // bit c set if child 4k + c exists (level < J)
    std::vector<int64_t> first_child; // index of the first child in the next level
    std::vector<double> lambda;       // lambda_{j,k}
    std::vector<double> gamma;        // gamma^m_{j,k} at [3 k + m] (level < J)
    std::vector<int32_t> chain;       // one-child run starting here (see TRec)
};

}  // namespace swv

struct swv_tree_s {
    int J = 0;
    double ra_p = 0, dec_p = 0;
    int64_t n_comp = 0;
    // leaves (level J), sorted by pixel id
    std::vector<int64_t> leaf_pix;
    std::vector<double> leaf_l, leaf_m, leaf_nm1, leaf_flux;
    std::vector<swv::TreeLevel> levels;  // levels[j - 1] is level j
    // depth-first record stream consumed by the device traversal
    std::vector<swv::TRec> records;
    int64_t n_roots = 0;
    // most nodes with two or more children on one root-to-leaf path
    int max_branching = 0;
    double build_seconds = 0;
    // device copies of `records`, one per HIP device id
    std::map<int, void*> device_records;
    // device copies of the leaves packed as direct-sum components (l, m, n - 1,
    // flux), one per HIP device id (swv_predict_tree_leaves)
    std::map<int, void*> device_leaves;
    // the caller's handle plus one per plan that reads the device records; the
    // tree is freed when the last of them is released
    int refs = 1;
    // coefficient thresholding (swv_tree_threshold / swv_tree_prune): the tree
    // is a pruned copy whose record stream has leaves at several levels;
    // `levels[j - 1].pix` then lists the nodes present at level j and
    // `leaf_pix` the leaves of every level
    bool thresholded = false;
    int64_t n_alive = 0;                 // internal nodes of the pruned tree
    int64_t n_one_child = 0;             // internal nodes with a single child
    int64_t n_coeffs = 0;                // wavelet coefficients of the source tree
    std::vector<int64_t> kept;           // retained ones, flat indices, increasing
};

namespace swv {

// (Re)computes levels, coefficients and the record stream from the leaves.
void build_coefficients(swv_tree_s* t);

// Builds the tree; returns a status code (message via fail()).
int build_tree(int J, double ra_p, double dec_p, int64_t n, const double* l, const double* m,
               const double* flux, swv_tree_s* out);

// The same from the components' level-J pixel ids (the cross-referenced form).
int build_tree_pixels(int J, double ra_p, double dec_p, int64_t n, const int64_t* kJ,
                      const double* flux, swv_tree_s* out);

// Flat index of gamma^m_{j,k}: 3 x (nodes at levels < j) + 3 k + m.  The
// retained coefficients of a proportion `fraction`: the round(fraction N)
// largest |gamma|, ties to the lower flat index; returned increasing.
std::vector<int64_t> retain_fraction(const swv_tree_s& t, double fraction);

// The thresholded tree of `t` keeping the coefficients `kept` (flat indices,
// increasing, each below 3 x internal nodes): nodes with nothing retained at or
// below them become leaves at their own level (their pixel centre), dropped
// coefficients of the other nodes are zero.  Status code.
int prune_tree(const swv_tree_s& t, const std::vector<int64_t>& kept, swv_tree_s* out);

}  // namespace swv
