/* A C program that uses libswvis.so through include/swvis.h alone (no
 * Python, no C++): the host-side entry points.  Prints one line per check
 * and exits non-zero on the first failure. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "swvis.h"

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
    CHECK(swv_tree_destroy(t) == SWV_OK, "tree destroy");

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
