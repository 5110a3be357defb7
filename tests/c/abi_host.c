/* A C program that uses libswvis.so through include/swvis.h alone (no
 * Python, no C++): the host-side entry points.  Prints one line per check
 * and exits non-zero on the first failure. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "swvis.h"

static const double kPi = 3.14159265358979323846;

#define CHECK(cond, what)                                           \
    do {                                                            \
        if (!(cond)) {                                              \
            printf("FAIL %s: %s\n", what, swv_last_error());        \
            return 1;                                               \
        }                                                           \
        printf("ok %s\n", what);                                    \
    } while (0)

int main(void) {
    int major = -1, minor = -1;
    CHECK(swv_version(&major, &minor) == SWV_OK && major >= 1, "version");

    /* the phase centre's own direction lies in one level-9 pixel, whose centre
       maps back into the same pixel */
    const double ra = 3.14159265358979, dec = 0.785398163397448;
    double l0 = 0.0, m0 = 0.0, lc, mc, nc;
    int64_t pix = -1, pix2 = -1;
    CHECK(swv_ang2pix(9, ra, dec, 1, &l0, &m0, &pix) == SWV_OK && pix >= 0 &&
              pix < 12 * (1LL << 16), "ang2pix");
    CHECK(swv_pixel_centres(9, ra, dec, 1, &pix, &lc, &mc, &nc) == SWV_OK, "pixel centre");
    CHECK(swv_ang2pix(9, ra, dec, 1, &lc, &mc, &pix2) == SWV_OK && pix2 == pix, "round trip");

    /* a three-component tree: stats and leaves */
    double l[3] = {0.01, 0.01, -0.02}, m[3] = {0.002, 0.002, 0.01}, f[3] = {1.0, 2.0, 0.5};
    swv_tree t = NULL;
    CHECK(swv_tree_build(12, ra, dec, 3, l, m, f, &t) == SWV_OK && t, "tree build");
    swv_tree_stats_t st;
    CHECK(swv_tree_stats(t, &st) == SWV_OK && st.n_leaves == 2 && st.J == 12, "tree stats");
    double lf[2];
    CHECK(swv_tree_leaves(t, NULL, NULL, NULL, NULL, lf) == SWV_OK &&
              fabs(lf[0] + lf[1] - 3.5) < 1e-15, "leaf fluxes");
    /* level 1 carries the whole flux: lambda_j A_j = sum of lambda_{j+1} A_{j+1}
       (Eq. 9 with A_j = 4 A_{j+1}), and level J has no children */
    const double A1 = 4.0 * kPi / 12.0;
    int64_t pix1[12];
    double lam1[12], lamJ[2];
    int32_t maskJ[2];
    CHECK(st.n_nodes[1] >= 1 && st.n_nodes[1] <= 12 &&
              swv_tree_level(t, 1, pix1, NULL, lam1, NULL) == SWV_OK, "tree level 1");
    double s1 = 0.0;
    for (int k = 0; k < st.n_nodes[1]; ++k) s1 += lam1[k] * A1;
    CHECK(fabs(s1 - 3.5) < 1e-13, "level-1 flux");
    CHECK(swv_tree_level(t, 12, NULL, maskJ, lamJ, NULL) == SWV_OK && maskJ[0] == 0 &&
              maskJ[1] == 0, "leaf level masks");

    /* new leaf fluxes on the same pixels */
    const double nf[2] = {2.0, 4.0};
    CHECK(swv_tree_set_flux(t, nf) == SWV_OK && swv_tree_leaves(t, NULL, NULL, NULL, NULL, lf) ==
              SWV_OK && lf[0] == 2.0 && lf[1] == 4.0, "set flux");
    CHECK(swv_tree_level(t, 1, NULL, NULL, lam1, NULL) == SWV_OK, "level 1 after set flux");
    s1 = 0.0;
    for (int k = 0; k < st.n_nodes[1]; ++k) s1 += lam1[k] * A1;
    CHECK(fabs(s1 - 6.0) < 1e-13, "level-1 flux after set flux");

    /* thresholding: every coefficient kept, none kept, and an empty prune */
    swv_tree all = NULL, none = NULL, pr = NULL;
    int64_t n_kept = -1, n_coeffs = -1;
    CHECK(swv_tree_threshold(t, 1.0, &all) == SWV_OK && all, "threshold 1");
    /* sized by a first call with cap = 0 */
    CHECK(swv_tree_kept(all, 0, NULL, &n_kept, &n_coeffs) == SWV_OK &&
              n_coeffs == 3 * st.n_internal && n_kept == n_coeffs, "all kept");
    int64_t* kept = malloc(sizeof(int64_t) * (size_t)n_kept);
    int64_t n_again = -1;
    CHECK(kept && swv_tree_kept(all, n_kept, kept, &n_again, &n_coeffs) == SWV_OK &&
              n_again == n_kept, "kept indices");
    int increasing = 1;
    for (int64_t k = 1; k < n_kept; ++k) increasing &= kept[k] > kept[k - 1];
    CHECK(increasing && kept[0] == 0 && kept[n_kept - 1] == n_coeffs - 1,
          "kept indices increase");
    CHECK(swv_tree_threshold(t, 0.0, &none) == SWV_OK &&
              swv_tree_kept(none, n_kept, kept, &n_again, &n_coeffs) == SWV_OK && n_again == 0,
          "none kept");
    free(kept);
    swv_tree_stats_t sn, sp;
    CHECK(swv_tree_stats(none, &sn) == SWV_OK && sn.n_internal == 0 &&
              sn.n_leaves == st.n_nodes[1], "collapsed to level 1");
    CHECK(swv_tree_prune(t, 0, NULL, &pr) == SWV_OK && swv_tree_stats(pr, &sp) == SWV_OK &&
              sp.n_leaves == sn.n_leaves && sp.n_records == sn.n_records, "empty prune");
    CHECK(swv_tree_leaves(none, NULL, NULL, NULL, NULL, lf) == SWV_ENOTSUP,
          "leaves of a thresholded tree refused");
    swv_tree_destroy(pr);
    swv_tree_destroy(none);
    swv_tree_destroy(all);
    CHECK(swv_tree_destroy(t) == SWV_OK, "tree destroy");

    /* the level-9 pixels within 2 deg: sized, filled, sorted, inside the disk */
    const double rad = 2.0 * kPi / 180.0;
    int64_t n_disk = -1;
    CHECK(swv_pixels_in_disk(9, ra, dec, rad, 0, NULL, NULL, NULL, NULL, &n_disk) == SWV_OK &&
              n_disk > 0, "disk count");
    int64_t* dp = malloc(sizeof(int64_t) * (size_t)n_disk);
    double* dl = malloc(sizeof(double) * (size_t)n_disk);
    double* dm = malloc(sizeof(double) * (size_t)n_disk);
    double* dn = malloc(sizeof(double) * (size_t)n_disk);
    n_again = -1;
    CHECK(dp && dl && dm && dn &&
              swv_pixels_in_disk(9, ra, dec, rad, n_disk, dp, dl, dm, dn, &n_again) == SWV_OK &&
              n_again == n_disk,
          "disk fill");
    int inside = 1, sorted = 1;
    for (int64_t k = 0; k < n_disk; ++k) {
        inside &= 1.0 + dn[k] >= cos(rad) - 1e-15;
        if (k) sorted &= dp[k] > dp[k - 1];
    }
    free(dp);
    free(dl);
    free(dm);
    free(dn);
    CHECK(inside && sorted, "disk pixels sorted and inside");

    /* cross reference of a small image grid, and the tree from its pixels */
    int64_t xref[12];
    CHECK(swv_cross_reference(10, ra, dec, 4, 3, 0.002, xref) == SWV_OK, "cross reference");
    double ones[2] = {1.0, 1.0};
    int64_t two[2] = {xref[0], xref[11]};
    CHECK(swv_tree_build_pixels(10, ra, dec, 2, two, ones, &t) == SWV_OK, "tree from pixels");
    swv_tree_destroy(t);

    /* clean beam of a sampled Gaussian */
    enum { NB = 21 };
    double beam[NB * NB], abc[3];
    for (int y = 0; y < NB; ++y)
        for (int x = 0; x < NB; ++x) {
            const double dx = x - NB / 2, dy = y - NB / 2;
            beam[y * NB + x] = exp(-(0.1 * dx * dx + 2 * 0.02 * dx * dy + 0.15 * dy * dy));
        }
    CHECK(swv_fit_clean_beam(NB, NB, beam, abc) == SWV_OK && fabs(abc[0] - 0.1) < 1e-12 &&
              fabs(abc[1] - 0.02) < 1e-12 && fabs(abc[2] - 0.15) < 1e-12, "clean beam fit");

    /* errors come back as codes with a message */
    CHECK(swv_tree_build(30, ra, dec, 3, l, m, f, &t) == SWV_EDOMAIN && t == NULL,
          "bad J rejected");
    CHECK(swv_predict_direct(NULL, 0, NULL, NULL, NULL, 0, NULL, NULL, NULL, -1, SWV_FP64,
                             NULL) == SWV_EINVAL,
          "null context rejected");
    printf("all host checks passed\n");
    return 0;
}
