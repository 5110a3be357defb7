/* A C program that drives the device entry points of libswvis.so through
 * include/swvis.h, with device memory from the HIP runtime's C API: a unit
 * source at the phase centre gives V = 1 on every row, the tree of one
 * component equals its direct sum and its leaf sum, the adjoint of V = 1 at
 * the centre pixel is the row count (also without allocation), the residual
 * against a zero model is V with chi^2 = N / 2, and the gradients of a unit
 * source at the centre are (N, 0, 0). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "swvis.h"

#define CHECK(cond, what)                                           \
    do {                                                            \
        if (!(cond)) {                                              \
            printf("FAIL %s: %s\n", what, swv_last_error());        \
            return 1;                                               \
        }                                                           \
        printf("ok %s\n", what);                                    \
    } while (0)

enum { N = 5000 };

int main(void) {
    swv_ctx ctx = NULL;
    CHECK(swv_ctx_create(0, NULL, &ctx) == SWV_OK, "context");
    double* h = (double*)malloc(sizeof(double) * 3 * N);
    for (int j = 0; j < 3 * N; ++j) h[j] = 2e4 * sin(0.37 * j + 0.1);
    double *d_uvw = NULL, *d_c = NULL, *d_v1 = NULL, *d_v2 = NULL, *d_img = NULL;
    CHECK(hipMalloc((void**)&d_uvw, sizeof(double) * 3 * N) == hipSuccess &&
              hipMalloc((void**)&d_c, sizeof(double) * 6) == hipSuccess &&
              hipMalloc((void**)&d_v1, 16 * N) == hipSuccess &&
              hipMalloc((void**)&d_v2, 16 * N) == hipSuccess &&
              hipMalloc((void**)&d_img, 16) == hipSuccess,
          "device memory");
    CHECK(hipMemcpy(d_uvw, h, sizeof(double) * 3 * N, hipMemcpyHostToDevice) == hipSuccess,
          "upload rows");
    const double comp[6] = {0.0, 0.0, 1.0, 0.0, 0.0, 0.0};   /* l, m, flux; pixel l, m, n - 1 */
    CHECK(hipMemcpy(d_c, comp, sizeof comp, hipMemcpyHostToDevice) == hipSuccess,
          "upload component");
    const double *u = d_uvw, *v = d_uvw + N, *w = d_uvw + 2 * N;
    CHECK(swv_predict_direct(ctx, N, u, v, w, 1, d_c, d_c + 1, d_c + 2, -1, SWV_FP64, d_v1) ==
              SWV_OK,
          "direct launch");
    double* vis = (double*)malloc(16 * N);
    CHECK(swv_ctx_synchronize(ctx) == SWV_OK &&
              hipMemcpy(vis, d_v1, 16 * N, hipMemcpyDeviceToHost) == hipSuccess,
          "direct result");
    double e = 0.0;
    for (int j = 0; j < N; ++j) e = fmax(e, fabs(vis[2 * j] - 1.0) + fabs(vis[2 * j + 1]));
    CHECK(e == 0.0, "unit source at the phase centre gives V = 1");

    const double l = 0.013, m = -0.004, f = 0.7, ra = 1.0, dec = 0.5;
    swv_tree t = NULL;
    CHECK(swv_tree_build(14, ra, dec, 1, &l, &m, &f, &t) == SWV_OK, "tree build");
    double ll, lm, lnm1, lflux;
    CHECK(swv_tree_leaves(t, NULL, &ll, &lm, &lnm1, &lflux) == SWV_OK, "leaf");
    const double leaf[3] = {ll, lm, lflux};
    CHECK(hipMemcpy(d_c, leaf, sizeof leaf, hipMemcpyHostToDevice) == hipSuccess, "leaf up");
    CHECK(swv_predict_tree(ctx, t, N, u, v, w, -1, SWV_FP64, d_v1) == SWV_OK &&
              swv_predict_direct(ctx, N, u, v, w, 1, d_c, d_c + 1, d_c + 2, -1, SWV_FP64,
                                 d_v2) == SWV_OK,
          "tree and direct launches");
    double* vd = (double*)malloc(16 * N);
    CHECK(swv_ctx_synchronize(ctx) == SWV_OK &&
              hipMemcpy(vis, d_v1, 16 * N, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(vd, d_v2, 16 * N, hipMemcpyDeviceToHost) == hipSuccess,
          "tree result");
    e = 0.0;
    for (int j = 0; j < 2 * N; ++j) e = fmax(e, fabs(vis[j] - vd[j]));
    CHECK(e <= 1e-12 * f, "one-component tree equals its direct sum");
    /* the same model visibilities as the direct sum over the tree's leaves (Eq. 16) */
    CHECK(swv_predict_tree_leaves(ctx, t, N, u, v, w, -1, SWV_FP64, d_v2) == SWV_OK &&
              swv_ctx_synchronize(ctx) == SWV_OK &&
              hipMemcpy(vd, d_v2, 16 * N, hipMemcpyDeviceToHost) == hipSuccess,
          "leaf-sum launch");
    e = 0.0;
    for (int j = 0; j < 2 * N; ++j) e = fmax(e, fabs(vis[j] - vd[j]));
    CHECK(e <= 1e-12 * f, "leaf sum equals the traversal");
    swv_tree_destroy(t);

    /* adjoint of the unit-source visibilities at the centre pixel: N */
    CHECK(swv_predict_direct(ctx, N, u, v, w, 1, d_c + 3, d_c + 4, d_c + 2, -1, SWV_FP64, d_v1) ==
              SWV_OK,
          "direct again");
    const double px[3] = {0.0, 0.0, 0.0};
    CHECK(hipMemcpy(d_c + 3, px, sizeof px, hipMemcpyHostToDevice) == hipSuccess, "pixel up");
    const double one = 1.0;
    CHECK(hipMemcpy(d_c + 2, &one, 8, hipMemcpyHostToDevice) == hipSuccess, "flux up");
    CHECK(swv_predict_direct(ctx, N, u, v, w, 1, d_c + 3, d_c + 4, d_c + 2, -1, SWV_FP64,
                             d_v1) == SWV_OK &&
              swv_adjoint(ctx, N, u, v, w, d_v1, 1, d_c + 3, d_c + 4, d_c + 5, -1, SWV_FP64,
                          d_img) == SWV_OK,
          "adjoint launch");
    double img[2];
    CHECK(swv_ctx_synchronize(ctx) == SWV_OK &&
              hipMemcpy(img, d_img, 16, hipMemcpyDeviceToHost) == hipSuccess,
          "adjoint result");
    CHECK(img[0] == (double)N && img[1] == 0.0, "adjoint of V = 1 at the centre is N");

    /* the allocation-free adjoint gives the same bits */
    double *d_img2 = NULL, *d_r = NULL, *d_chi2 = NULL, *d_g = NULL;
    CHECK(hipMalloc((void**)&d_img2, 16) == hipSuccess && hipMalloc((void**)&d_r, 16 * N) ==
              hipSuccess && hipMalloc((void**)&d_chi2, 8) == hipSuccess &&
              hipMalloc((void**)&d_g, 24) == hipSuccess,
          "more device memory");
    double img2[2];
    CHECK(swv_adjoint_noalloc(ctx, N, u, v, w, d_v1, 1, d_c + 3, d_c + 4, d_c + 5, -1,
                              SWV_FP64, d_img2) == SWV_OK &&
              swv_ctx_synchronize(ctx) == SWV_OK &&
              hipMemcpy(img2, d_img2, 16, hipMemcpyDeviceToHost) == hipSuccess,
          "allocation-free adjoint");
    CHECK(img2[0] == img[0] && img2[1] == img[1], "allocation-free adjoint equals the adjoint");

    /* residual of V = 1 against a zero model: 1 on every row, chi^2 = N / 2 */
    double chi2 = -1.0;
    CHECK(hipMemset(d_v2, 0, 16 * N) == hipSuccess &&
              swv_residual_chi2(ctx, N, d_v1, d_v2, 0.5, d_r, d_chi2) == SWV_OK &&
              swv_ctx_synchronize(ctx) == SWV_OK &&
              hipMemcpy(vd, d_r, 16 * N, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(&chi2, d_chi2, 8, hipMemcpyDeviceToHost) == hipSuccess,
          "residual launch");
    e = 0.0;
    for (int j = 0; j < N; ++j) e = fmax(e, fabs(vd[2 * j] - 1.0) + fabs(vd[2 * j + 1]));
    CHECK(e == 0.0 && chi2 == 0.5 * N, "residual and chi^2");

    /* gradients of Re sum conj(y) V at a unit source at the centre with y = 1:
       every term is exactly 1, so d_flux = N and d_l = d_m = 0 */
    double g[3] = {-1.0, -1.0, -1.0};
    CHECK(swv_grad_direct(ctx, N, u, v, w, d_v1, 1, d_c + 3, d_c + 4, d_c + 2, -1, 1.0, d_g,
                          d_g + 1, d_g + 2) == SWV_OK &&
              swv_ctx_synchronize(ctx) == SWV_OK &&
              hipMemcpy(g, d_g, 24, hipMemcpyDeviceToHost) == hipSuccess,
          "gradient launch");
    CHECK(g[0] == (double)N && g[1] == 0.0 && g[2] == 0.0, "gradients at the centre");
    hipFree(d_img2);
    hipFree(d_r);
    hipFree(d_chi2);
    hipFree(d_g);
    CHECK(swv_ctx_destroy(ctx) == SWV_OK, "context destroy");
    hipFree(d_uvw);
    hipFree(d_c);
    hipFree(d_v1);
    hipFree(d_v2);
    hipFree(d_img);
    free(h);
    free(vis);
    free(vd);
    printf("all device checks passed\n");
    return 0;
}
