/* A C program that drives the device entry points of libswvis.so through
 * include/swvis.h, with device memory from the HIP runtime's C API: a unit
 * source at the phase centre gives V = 1 on every row, the tree of one
 * component equals its direct sum and its leaf sum, the adjoint of V = 1 at
 * the centre pixel is the row count (also without allocation), the residual
 * against a zero model is V with chi^2 = N / 2, and the gradients of a unit
 * source at the centre are (N, 0, 0); a batched plan over two direct
 * instances and a tree instance, run and replayed as a captured graph, gives
 * the single calls' bits. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

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
    /* batched: two direct instances of different lengths and one tree instance in
       one plan; the run and a replay of its captured graph give the single calls'
       bits */
    {
        const double hb[9] = {0.013, -0.02, -0.004, 0.01, 0.7, 1.3, 0.0, 0.0, 1.0};
        const int64_t nb = N - 1234, off = 1000;
        double *d_cb = NULL, *d_o = NULL, *d_s = NULL;
        CHECK(hipMalloc((void**)&d_cb, sizeof hb) == hipSuccess &&
                  hipMalloc((void**)&d_o, 3 * 16 * N) == hipSuccess &&
                  hipMalloc((void**)&d_s, 3 * 16 * N) == hipSuccess &&
                  hipMemcpy(d_cb, hb, sizeof hb, hipMemcpyHostToDevice) == hipSuccess,
              "batched buffers");
        swv_tree tb = NULL;
        CHECK(swv_tree_build(12, ra, dec, 2, hb, hb + 2, hb + 4, &tb) == SWV_OK, "batched tree");
        CHECK(swv_predict_direct(ctx, N, u, v, w, 2, d_cb, d_cb + 2, d_cb + 4, -1, SWV_FP64,
                                 d_s) == SWV_OK &&
                  swv_predict_direct(ctx, nb, u + off, v + off, w + off, 1, d_cb + 6, d_cb + 7,
                                     d_cb + 8, -1, SWV_FP64, d_s + 2 * N) == SWV_OK &&
                  swv_predict_tree(ctx, tb, N, u, v, w, -1, SWV_FP64, d_s + 4 * N) == SWV_OK,
              "single calls");
        swv_instance in[3];
        memset(in, 0, sizeof in);
        in[0].route = SWV_ROUTE_DIRECT; in[0].prec = SWV_FP64; in[0].sign = -1;
        in[0].n_vis = N; in[0].u = u; in[0].v = v; in[0].w = w;
        in[0].n_comp = 2; in[0].l = d_cb; in[0].m = d_cb + 2; in[0].flux = d_cb + 4;
        in[0].vis_out = d_o;
        in[1] = in[0];
        in[1].n_vis = nb; in[1].u = u + off; in[1].v = v + off; in[1].w = w + off;
        in[1].n_comp = 1; in[1].l = d_cb + 6; in[1].m = d_cb + 7; in[1].flux = d_cb + 8;
        in[1].vis_out = d_o + 2 * N;
        in[2] = in[0];
        in[2].route = SWV_ROUTE_TREE; in[2].n_comp = 0; in[2].l = in[2].m = in[2].flux = NULL;
        in[2].tree = tb; in[2].vis_out = d_o + 4 * N;
        swv_plan plan = NULL;
        swv_plan_stats_t ps;
        CHECK(swv_batch_plan(ctx, 3, in, &plan) == SWV_OK && plan &&
                  swv_plan_stats(plan, &ps) == SWV_OK && ps.n_instances == 3 && ps.n_items > 0,
              "batch plan");
        double* a = (double*)malloc(3 * 16 * N);
        double* b = (double*)malloc(3 * 16 * N);
        const size_t sizes[3] = {16 * (size_t)N, 16 * (size_t)nb, 16 * (size_t)N};
        CHECK(swv_batch_run(plan) == SWV_OK && swv_ctx_synchronize(ctx) == SWV_OK &&
                  hipMemcpy(a, d_o, 3 * 16 * N, hipMemcpyDeviceToHost) == hipSuccess &&
                  hipMemcpy(b, d_s, 3 * 16 * N, hipMemcpyDeviceToHost) == hipSuccess,
              "batch run");
        int same = 1;
        for (int k = 0; k < 3; ++k) same &= memcmp(a + 2 * N * k, b + 2 * N * k, sizes[k]) == 0;
        CHECK(same, "batched equals single calls bit for bit");
        swv_graph g = NULL;
        CHECK(hipMemset(d_o, 0, 3 * 16 * N) == hipSuccess && hipDeviceSynchronize() == hipSuccess &&
                  swv_graph_capture(plan, &g) == SWV_OK && g &&
                  swv_graph_launch(g) == SWV_OK && swv_ctx_synchronize(ctx) == SWV_OK &&
                  hipMemcpy(a, d_o, 3 * 16 * N, hipMemcpyDeviceToHost) == hipSuccess,
              "graph capture and replay");
        same = 1;
        for (int k = 0; k < 3; ++k) same &= memcmp(a + 2 * N * k, b + 2 * N * k, sizes[k]) == 0;
        CHECK(same, "graph replay equals single calls bit for bit");
        CHECK(swv_graph_destroy(g) == SWV_OK && swv_plan_destroy(plan) == SWV_OK &&
                  swv_tree_destroy(tb) == SWV_OK,
              "batched objects destroyed");
        free(a);
        free(b);
        hipFree(d_cb);
        hipFree(d_o);
        hipFree(d_s);
    }
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
