/*
 * swvis.h -- C ABI of libswvis.so: model-visibility prediction on MI355X
 * (gfx950) by the direct component sum and by the spherical-Haar-wavelet
 * tree of Skipper, Scaife & McEwen (2019), plus the exact adjoint and the
 * chi^2 gradients of the direct sum, and the wavelet clean loop around them
 * (Hogbom minor cycles, major cycles with the tree predictor).
 *
 * Notation.  A visibility row j has baseline B_j = (u_j, v_j, w_j) in
 * wavelengths; a component k has direction cosines (l_k, m_k), n_k =
 * sqrt(1 - l_k^2 - m_k^2), and flux I_k.  The phase in cycles is
 *     phi_jk = u_j l_k + v_j m_k + w_j (n_k - 1)
 * (section 3.3, Eq. 12 with the phase centre at [0, 0, 1]) and
 *     e_jk = exp(s 2 pi i phi_jk),  s = `sign` in {-1, +1}.
 * The paper prints s = +1; the conventional default is s = -1.
 *
 * Conventions of every entry point.
 *  - Return value: SWV_OK (0) or a negative status; swv_last_error() then
 *    holds a message (thread-local, valid until the next call on the thread).
 *    No C++ exception and no abort crosses this boundary.
 *  - Pointers marked DEVICE are caller-owned device memory (e.g. a torch
 *    tensor's data_ptr()) on the context's device; they must stay valid until
 *    the context's stream has reached the work.  Pointers marked HOST are
 *    caller-owned host memory, read or written before the call returns.  The
 *    library never frees caller memory.
 *  - Arrays are contiguous.  FP64 unless stated.  Complex values are
 *    interleaved (re, im): complex128 = 2 x FP64 (16 B), complex64 = 2 x FP32.
 *  - Device work is enqueued asynchronously on the context's stream.  Errors
 *    the kernels detect (non-finite or out-of-domain inputs) and HIP faults
 *    are reported by the next swv_ctx_synchronize() on that context.
 *  - Library objects (swv_ctx, swv_tree, swv_plan, swv_graph, swv_cycle)
 *    follow create/destroy pairs.  A plan or cycle keeps its context alive, a
 *    plan its trees and a graph its plan, so they may be destroyed in any order (memory is
 *    released with the last of them); a handle must not be used after its
 *    destroy call.  A context may be used from one thread at a time; calls
 *    that overlap on one stream are ordered by the stream.
 *  - Destroy every object before the process exits: the destroy calls wait
 *    for the streams and release device memory while the HIP runtime (and
 *    any tool attached to it) is still up.
 *  - n = 0 is valid everywhere and enqueues nothing (outputs untouched,
 *    except reductions, which write zero).
 */
#ifndef SWVIS_H
#define SWVIS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SWV_VERSION_MAJOR 1
#define SWV_VERSION_MINOR 0

/* Status codes. */
#define SWV_OK        0
#define SWV_EINVAL   (-1)  /* null pointer, negative size, bad enum, bad handle */
#define SWV_EDOMAIN  (-2)  /* l^2 + m^2 >= 1, J outside [1, 29], |sign| != 1, non-finite input */
#define SWV_ENOMEM   (-3)  /* host or device allocation failed */
#define SWV_EHIP     (-4)  /* a HIP runtime call failed; the message holds the HIP error text */
#define SWV_ENOTSUP  (-5)  /* valid request the library does not support */

/* Arithmetic forms. */
#define SWV_FP64  0  /* phase, sincos and sums in FP64; output complex128 */
#define SWV_F32C  1  /* phase and its reduction mod 1 in FP64; sincos (the hardware
                        v_sin_f32 / v_cos_f32, which take revolutions), products and
                        Kahan-compensated sums in FP32; output complex64 */

/* Routes of a batched instance. */
#define SWV_ROUTE_DIRECT 0
#define SWV_ROUTE_TREE   1

#define SWV_MAX_LEVEL 29

typedef struct swv_ctx_s* swv_ctx;
typedef struct swv_tree_s* swv_tree;
typedef struct swv_plan_s* swv_plan;
typedef struct swv_graph_s* swv_graph;

/* ------------------------------------------------------------ basics --- */

/* Library version (SWV_VERSION_MAJOR, SWV_VERSION_MINOR). */
int swv_version(int* major, int* minor);

/* Message of the last failing call on this thread ("" if none). */
const char* swv_last_error(void);

/* Creates a context bound to HIP device `device` and the HIP stream `stream`
 * (a hipStream_t; NULL = the legacy default stream).  The context owns its
 * workspaces and its tuning table.  If the environment variable
 * SWV_TUNE_CACHE names a file written by swv_autotune, it is loaded. */
int swv_ctx_create(int device, void* stream, swv_ctx* out);

/* Rebinds the context to another stream of the same device. */
int swv_ctx_set_stream(swv_ctx ctx, void* stream);

/* Waits for the context's stream; returns the first deferred error since the
 * previous call: SWV_EDOMAIN if a kernel saw an out-of-domain or non-finite
 * input, SWV_EHIP on a HIP failure. */
int swv_ctx_synchronize(swv_ctx ctx);

/* Frees the context's workspaces (after waiting for its stream). */
int swv_ctx_destroy(swv_ctx ctx);

/* ------------------------------------------------------- direct route --- */

/* Direct component sum (section 3.3, Eq. 12):
 *     vis_out[j] = sum_k flux[k] * e_jk,   j < n_vis.
 * u, v, w [n_vis] DEVICE; l, m, flux [n_comp] DEVICE (l^2 + m^2 < 1);
 * vis_out [n_vis] DEVICE complex128 (SWV_FP64) or complex64 (SWV_F32C).
 * n - 1 is formed as -(l^2 + m^2) / (1 + n).  Work: n_vis * n_comp terms.
 * Uses a context workspace of 32 * n_comp bytes (the packed components). */
int swv_predict_direct(swv_ctx ctx, int64_t n_vis, const double* u, const double* v,
                       const double* w, int64_t n_comp, const double* l, const double* m,
                       const double* flux, int sign, int prec, void* vis_out);

/* --------------------------------------------------------- tree route --- */

typedef struct {
    int J;                                   /* finest level */
    int64_t n_comp;                          /* components given */
    int64_t n_leaves;                        /* distinct level-J pixels (N~_C) */
    int64_t n_internal;                      /* existing nodes at levels 1..J-1 */
    int64_t n_nodes[SWV_MAX_LEVEL + 1];      /* n_nodes[j] = existing nodes at level j */
    int64_t n_records;                       /* length of the depth-first record stream */
    double sparsity;                         /* n_leaves / N_J */
    double build_seconds;                    /* host time of swv_tree_build */
    int max_branching;                       /* most nodes with >= 2 children on one
                                                root-to-leaf path */
} swv_tree_stats_t;

/* Builds the sparse coefficient tree of a component list (sections 3.2-3.5),
 * on the host:
 *  1. [l, m, n] (SIN projection) is rotated to the equatorial xyz frame by
 *     R_uvw->xyz = R_y(ra_p) R_x(-dec_p) (section 3.4, Eq. 18);
 *  2. assigned to its level-J nested pixel of the 12 * 4^(J-1)-pixel
 *     equal-area (HEALPix NESTED) pixelisation (section 3.2);
 *  3. components sharing a pixel are summed into one leaf; the leaf position
 *     is the pixel centre rotated back to uvw (section 3.5);
 *  4. lambda_J = flux / A_J, and for existing nodes at j = J-1 .. 1
 *     lambda_j = 1/4 sum_c lambda_{j+1,4k+c} (Eq. 9) and
 *     gamma^m_j = sqrt(A_j)/4 sum_c s^m_c lambda_{j+1,4k+c} (Eq. 10);
 *     ancestors are k_j = k_J >> 2(J - j) (section 3.5).
 * Geometry is evaluated in extended precision and rounded once to FP64.
 * l, m, flux [n_comp] HOST.  1 <= J <= 29.  ra_p, dec_p in radians. */
int swv_tree_build(int J, double ra_p, double dec_p, int64_t n_comp, const double* l,
                   const double* m, const double* flux, swv_tree* out);

/* Sizes of a tree (HOST struct). */
int swv_tree_stats(swv_tree tree, swv_tree_stats_t* out);

/* Copies the leaves, sorted by pixel id, to HOST arrays of n_leaves entries:
 * nested pixel id, centre (l, m, n - 1) in the uvw frame, summed flux.
 * Any pointer may be NULL to skip that array. */
int swv_tree_leaves(swv_tree tree, int64_t* pix, double* l, double* m, double* nm1,
                    double* flux);

/* Copies level j (1 <= j <= J) of the tree to HOST arrays of n_nodes[j]
 * entries: sorted pixel ids, 4-bit child masks (bit c set if child 4k+c
 * exists; 0 at level J), lambda_j, and gamma^0..2 as [n][3] (zeros at level
 * J).  Any pointer may be NULL. */
int swv_tree_level(swv_tree tree, int j, int64_t* pix, int32_t* child_mask, double* lambda,
                   double* gamma);

/* Replaces the flux of every leaf (HOST array of n_leaves entries, in leaf
 * order) and recomputes lambda and gamma on the same pixel set; the tree's
 * device copies are refreshed in place, so plans and captured graphs that use
 * the tree predict the new model.  Waits for the devices holding copies. */
int swv_tree_set_flux(swv_tree tree, const double* leaf_flux);

/* Model visibilities by the wavelet route (section 3.3, Eqs. 14-17; the
 * per-visibility work of section 3.6.1): for every row, the plane wave
 * eta_{J,k} = exp(s 2 pi i B . (s_k - P)) at the leaf centres, then per
 * existing node eta_j = 1/4 sum_c eta_{j+1} and
 * sigma^m_j = sqrt(A_j)/4 sum_c s^m_c eta_{j+1} (Eqs. 9, 10 applied to the
 * plane wave), and
 *     vis_out = A_1 sum_k lambda_1 eta_1 + sum_{j<J} sum_k sum_m gamma^m sigma^m
 * (Eq. 17 with lambda_J a flux density; equal to the direct sum over the
 * pixel-snapped leaves, Eq. 16).  u, v, w [n_vis] DEVICE; vis_out DEVICE
 * complex128 (SWV_FP64) or complex64 (SWV_F32C: the leaf phase in FP64,
 * reduced exactly, then the FP32 hardware sine and cosine; the node
 * arithmetic stays FP64).  The tree is copied to the device on first use with
 * this context's device.
 * Two traversals compute the same operations in the same order (bitwise equal
 * results): one keeps a state set per level (J <= 16), the other one per open
 * node with two or more children (any J, up to 15 such nodes on one
 * root-to-leaf path, see swv_tree_stats_t.max_branching).  By default the
 * first serves J <= 10, and J <= 16 unless more than three in four internal
 * nodes have a single child; the tuning table can force either (swv_tune_set).
 * SWV_ENOTSUP if neither fits, or if the tree's record stream (32 bytes per
 * record) exceeds 4 GiB - 32. */
int swv_predict_tree(swv_ctx ctx, swv_tree tree, int64_t n_vis, const double* u,
                     const double* v, const double* w, int sign, int prec, void* vis_out);

/* The same model visibilities in the form of Eq. 16: the direct sum over the
 * tree's merged leaves at their pixel centres,
 *     vis_out[j] = sum_k F_k exp(s 2 pi i B_j . (s_k - P)),
 * which Eq. 17 equals exactly (the wavelet terms of every level collapse onto
 * the leaves they were built from).  One term per leaf instead of one per
 * node; SWV_FP64 or SWV_F32C as in swv_predict_direct.  The leaves are copied
 * to the device on first use with this context's device (32 bytes each) and
 * refreshed by swv_tree_set_flux.  Arguments as swv_predict_tree. */
int swv_predict_tree_leaves(swv_ctx ctx, swv_tree tree, int64_t n_vis, const double* u,
                            const double* v, const double* w, int sign, int prec,
                            void* vis_out);

/* Coefficient thresholding: the retention of a fixed proportion of the wavelet
 * coefficients that section 1 cites (McEwen 2008), an approximation the paper
 * itself does not use (it keeps every non-zero coefficient).  Writes a new,
 * thresholded tree:
 *  - ranked are the wavelet coefficients gamma^m_{j,k} of every node at levels
 *    1 .. J-1 (Eq. 10 gives them orthonormal, so |gamma| compares across
 *    levels); the level-1 scaling coefficients are always kept;
 *  - the round(fraction N) largest |gamma| are retained (N = 3 x internal
 *    nodes; ties to the lower flat index, below), the rest set to zero;
 *  - a node with nothing retained at or below it becomes a leaf at its own
 *    level: the plane wave is sampled at its pixel centre, as at the level-J
 *    leaves, and nothing below it is visited.
 * swv_predict_tree then evaluates Eq. 17 over the thresholded tree (FP64 or
 * F32C); fraction 1 gives the exact tree route.  The thresholded tree works
 * with swv_predict_tree (64-thread blocks), swv_tree_stats (n_leaves counts the
 * leaves of every level, n_internal the remaining internal nodes) and batched
 * plans (which then walk every tree with the traversal per branching node);
 * swv_tree_leaves, swv_tree_level, swv_tree_set_flux, swv_predict_tree_leaves
 * and swv_cycle_set_tree return SWV_ENOTSUP for it.  0 <= fraction <= 1. */
int swv_tree_threshold(swv_tree tree, double fraction, swv_tree* out);

/* The same with the retained coefficients given: kept [n_kept] HOST, flat
 * indices increasing, where gamma^m_{j,k} has flat index
 * 3 x (nodes at levels < j) + 3 k + m (k in the level's pixel order, as
 * swv_tree_level lists it). */
int swv_tree_prune(swv_tree tree, int64_t n_kept, const int64_t* kept, swv_tree* out);

/* The retained coefficients of a thresholded tree: up to cap flat indices to
 * kept (HOST), their count to *n_kept and the number of coefficients of the
 * source tree to *n_coeffs. */
int swv_tree_kept(swv_tree tree, int64_t cap, int64_t* kept, int64_t* n_kept,
                  int64_t* n_coeffs);

/* Releases the caller's handle.  A plan made with the tree holds its own
 * reference (its device records stay valid until the plan and its graphs are
 * destroyed); the tree is freed with the last reference. */
int swv_tree_destroy(swv_tree tree);

/* ------------------------------------------------------ sphere pixels --- */

/* Level-J nested pixel of each SIN-projected direction (l, m) for the phase
 * centre (ra_p, dec_p) (sections 3.2, 3.4, 3.5).  l, m [n] HOST, pix [n] HOST. */
int swv_ang2pix(int J, double ra_p, double dec_p, int64_t n, const double* l, const double* m,
                int64_t* pix);

/* Centres of level-J pixels as (l, m, n - 1) in the uvw frame of (ra_p, dec_p).
 * pix, l, m, nm1 [n] HOST.  For a centre behind the phase centre's
 * hemisphere n - 1 < -1. */
int swv_pixel_centres(int J, double ra_p, double dec_p, int64_t n, const int64_t* pix,
                      double* l, double* m, double* nm1);

/* Sorted level-J pixels whose centres lie within `radius` radians of the
 * phase centre, with their centres (l, m, n - 1).  At most `cap` entries are
 * written to the HOST arrays, all four of which are required when cap > 0
 * (SWV_EINVAL otherwise); *n_out receives the full count (call with cap = 0
 * and null arrays to size them). */
int swv_pixels_in_disk(int J, double ra_p, double dec_p, double radius, int64_t cap,
                       int64_t* pix, double* l, double* m, double* nm1, int64_t* n_out);

/* -------------------------------------------- major cycle: subtract, image --- */

/* Subtract step of the major cycle (section 2.2):
 *     resid_out[j] = vis_obs[j] - vis_model[j],
 *     *chi2_out = inv_sigma2 * sum_j |resid_out[j]|^2   (deterministic order).
 * vis_obs, vis_model, resid_out [n_vis] DEVICE complex128 (resid_out may alias
 * vis_obs); chi2_out DEVICE, one FP64. */
int swv_residual_chi2(swv_ctx ctx, int64_t n_vis, const void* vis_obs, const void* vis_model,
                      double inv_sigma2, void* resid_out, double* chi2_out);

/* Exact adjoint of the direct sum on a pixel set (the residual image on the
 * sphere pixels; replaces the grid + inverse FFT of section 2.2's third
 * step):
 *     img_out[p] = sum_j conj(e_jp) * y[j].
 * u, v, w, y [n_vis] DEVICE (y complex128); l, m, nm1 [n_pix] DEVICE (pixel
 * centres, n - 1 given explicitly); img_out [n_pix] DEVICE complex128 for
 * both precisions (SWV_F32C: FP32 sincos and products, Kahan sums per
 * visibility chunk).  Deterministic: fixed chunking and summation order.
 * Uses a workspace of 16 * n_pix * ceil(n_vis / chunk) bytes; the chunk
 * count is a multiple of 8 (a chunk of every group of 8 per XCD) chosen for
 * whole rounds of resident blocks on each XCD, at most about 8 rounds, which
 * keeps the workspace under 128 * (pixels per block) * (resident blocks)
 * bytes (about 240 MB at the default tiling). */
int swv_adjoint(swv_ctx ctx, int64_t n_vis, const double* u, const double* v, const double* w,
                const void* y, int64_t n_pix, const double* l, const double* m,
                const double* nm1, int sign, int prec, void* img_out);

/* swv_adjoint for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, the same result bit for bit (the same tiling, row
 * chunks and summation order), but the per-chunk partial sums live in a fixed
 * 32 MiB device array that the library holds on every device it runs on
 * until the process ends, instead of a context workspace.  The call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 * SWV_ENOMEM, before any work is enqueued, if the partial sums,
 * 16 * n_pix * (row chunks of swv_adjoint) bytes, exceed 32 MiB (e.g. about
 * 2,000,000 pixel-chunks: 955 pixels over 8.36M rows need 15.6 MB).  All
 * calls on one device share the array and every call overwrites the part it
 * uses before reading it: calls that overlap on one device (other streams,
 * other contexts, other threads) race and must be ordered by the caller. */
int swv_adjoint_noalloc(swv_ctx ctx, int64_t n_vis, const double* u, const double* v,
                        const double* w, const void* y, int64_t n_pix, const double* l,
                        const double* m, const double* nm1, int sign, int prec,
                        void* img_out);

/* Gradient of  alpha * Re sum_j conj(y_j) V_j(theta)  with respect to the real
 * parameters theta = (flux_k, l_k, m_k) of the direct sum (Eq. 12):
 *     d_flux[k] = alpha Re sum_j conj(y_j) e_jk
 *     d_l[k]    = alpha Re sum_j conj(y_j) flux_k s 2 pi i (u_j - w_j l_k / n_k) e_jk
 *     d_m[k]    = alpha Re sum_j conj(y_j) flux_k s 2 pi i (v_j - w_j m_k / n_k) e_jk
 * y = residuals and alpha = -2/sigma^2 give d(chi^2); y = dL/dV* and alpha = 1
 * give the backward of a real loss.  All arrays DEVICE; FP64.  Deterministic.
 * Per component only four real sums over the rows are formed:
 * Re sum conj(y) e and Im sum {u, v, w} conj(y) e.  Uses a workspace of
 * 32 * n_comp * ceil(n_vis / chunk) bytes plus the packed components. */
int swv_grad_direct(swv_ctx ctx, int64_t n_vis, const double* u, const double* v,
                    const double* w, const void* y, int64_t n_comp, const double* l,
                    const double* m, const double* flux, int sign, double alpha,
                    double* d_flux, double* d_l, double* d_m);

/* ------------------------------------------------------- clean loop --- */
/* Cotton-Schwab cleaning with the wavelet predictor (sections 2.1, 2.2, 3.5).
 * Images are row-major (ny, nx) FP64 grids: pixel p = iy * nx + ix at the
 * SIN-projected direction l = (ix - cx) cell, m = (iy - cy) cell,
 * n - 1 = -(l^2 + m^2) / (1 + sqrt(1 - l^2 - m^2)).  An image grid has its
 * phase centre at (cx, cy) = (nx / 2, ny / 2) (integer division); a beam grid
 * is (2 ny - 1, 2 nx - 1) pixel offsets with the zero offset at
 * (nx - 1, ny - 1). */

#define SWV_HOGBOM_ABS 1     /* take the peak of |I| instead of I */
#define SWV_HOGBOM_SINGLE 2  /* run the cycle in one workgroup (the grid-wide form is
                                otherwise used from 16,384 pixels where the device
                                supports cooperative launches) */

/* Directions of a grid: l, m, nm1 [nx * ny] DEVICE.  cx, cy is the pixel of
 * the phase centre.  Directions off the unit disk (l^2 + m^2 >= 1) get
 * l = m = nm1 = 0.  cell > 0 in direction cosines. */
int swv_image_grid(swv_ctx ctx, int nx, int ny, int cx, int cy, double cell, double* l,
                   double* m, double* nm1);

/* Dirty image from visibilities (section 2.1, first two steps, as the exact
 * adjoint of Eq. 12 instead of gridding and an inverse FFT):
 *     img_out[p] = (1 / n_vis) Re sum_j conj(e_jp) y[j]
 * on the grid (nx, ny, cx, cy, cell); a unit source on a pixel gives 1 there.
 * Pixels whose direction is off the unit disk are 0.  y [n_vis] DEVICE
 * complex128; img_out [nx * ny] DEVICE FP64.  With y = NULL the visibilities
 * are all 1: on the beam grid (cx = nx' - 1 of an nx' image) that is the
 * dirty beam B_D, the image of a unit source at the phase centre.  prec is
 * the adjoint's: SWV_FP64, or SWV_F32C (FP32 phasors and Kahan sums, about
 * twice as fast, relative error up to ~1e-6).  Uses 40 * nx * ny bytes of
 * device scratch plus the adjoint's workspace. */
int swv_dirty_image(swv_ctx ctx, int64_t n_vis, const double* u, const double* v,
                    const double* w, const void* y, int nx, int ny, int cx, int cy,
                    double cell, int sign, int prec, double* img_out);

/* Hogbom minor cycle (section 2.1, Eqs. 4 and 5) on image [ny][nx] (DEVICE,
 * updated in place to the residual) with beam [2 ny - 1][2 nx - 1] (DEVICE,
 * zero offset at its centre).  Iteration n takes the peak pixel p_n, the first
 * in row-major order holding the largest value (largest |value| with
 * SWV_HOGBOM_ABS), with value C_n; stops if the peak is not above `threshold`
 * or after max_iter components; else records comp_pix[n] = p_n and
 * comp_val[n] = gain * C_n and subtracts comp_val[n] * beam shifted to p_n from
 * every pixel (one product, one subtraction: the result does not depend on
 * the device).  comp_pix, comp_val [max_iter] DEVICE; *n_found DEVICE
 * receives the number of components.  Image and beam must be finite.  From
 * 16,384 pixels up to 64 workgroups (about four pixels per thread, more
 * beyond 262,144 pixels) run the cycle under a cooperative launch, the workgroups exchanging
 * their peaks once per iteration (SWV_HOGBOM_SINGLE, or a device that cannot
 * launch cooperatively, keeps it in one workgroup); both give the same bits.
 * Every wait in the exchange is bounded: should one ever run out, the cycle
 * stops and *n_found is -1 (the image is then partly updated).  Uses 64 bytes
 * per workgroup of context workspace.  The call does not synchronise. */
int swv_hogbom(swv_ctx ctx, int nx, int ny, double* image, const double* beam, double gain,
               double threshold, int64_t max_iter, int flags, int64_t* comp_pix,
               double* comp_val, int64_t* n_found);

/* Cross-reference table of an image grid (section 3.5): the level-J nested
 * sphere pixel of every image pixel's direction (the grid's l, m rotated to
 * the equatorial frame as in swv_tree_build).  pix [nx * ny] HOST.
 * SWV_EDOMAIN if a grid direction is off the unit disk. */
int swv_cross_reference(int J, double ra_p, double dec_p, int nx, int ny, double cell,
                        int64_t* pix);

/* swv_tree_build from the components' level-J pixel ids (the cross-referenced
 * form of section 3.5): pix [n] HOST in [0, 12 * 4^(J-1)), flux [n] HOST. */
int swv_tree_build_pixels(int J, double ra_p, double dec_p, int64_t n, const int64_t* pix,
                          const double* flux, swv_tree* out);

/* Clean beam B_C (section 2.1, third step): the rotated 2-D Gaussian
 *     B_C(dx, dy) = exp(-(a dx^2 + 2 b dx dy + c dy^2)),  offsets in pixels,
 * whose logarithm is the least-squares fit of ln B_D over the main lobe: the
 * 8-connected region of beam >= 1/2 around the centre.  beam [nby][nbx] HOST
 * with its zero offset at (nbx / 2, nby / 2); abc[3] HOST receives (a, b, c).
 * SWV_EDOMAIN if the centre is below 1/2, the lobe does not determine the
 * three parameters or the fit is not a peaked Gaussian. */
int swv_fit_clean_beam(int nbx, int nby, const double* beam, double* abc);

/* Clean image (Eq. 6): out[p] = sum_i comp_val[i] B_C(p - comp_pix[i]), the
 * terms added in list order, plus residual[p] if residual is not NULL.
 * comp_pix, comp_val [n_comp] DEVICE; residual, out [nx * ny] DEVICE;
 * abc HOST as from swv_fit_clean_beam. */
int swv_restore(swv_ctx ctx, int nx, int ny, int64_t n_comp, const int64_t* comp_pix,
                const double* comp_val, const double* abc, const double* residual, double* out);

typedef struct {
    int nx, ny;           /* image grid, phase centre at (nx / 2, ny / 2) */
    double cell;          /* pixel size in direction cosines */
    int J;                /* wavelet resolution of the model */
    double ra_p, dec_p;   /* phase centre, radians */
    double gain;          /* Hogbom loop gain g */
    double threshold;     /* minor cycles stop at a peak not above this */
    int64_t minor_iter;   /* Hogbom iterations per major cycle */
    int n_major;          /* major cycles */
    int flags;            /* SWV_HOGBOM_ABS */
    int sign;             /* phase sign of Eq. 12, +1 or -1 */
    int predictor;        /* SWV_PREDICT_TREE (the wavelet clean), SWV_PREDICT_DEGRID or
                             SWV_PREDICT_DIRECT */
    int support;          /* kernel width W of SWV_PREDICT_DEGRID */
    int image_prec;       /* precision of the dirty beam, the dirty image and every
                             residual image: SWV_FP64 or SWV_F32C (see
                             swv_dirty_image) */
} swv_clean_params_t;

/* Model-visibility predictor of the major cycles.  TREE: the tree of every
 * component so far at level J (the wavelet clean).  DEGRID: the model image
 * (components summed per pixel, in list order) by swv_predict_degrid, the
 * conventional clean's FFT + degridding.  DIRECT: the direct sum over the
 * image pixels holding components (exact for the pixelated model). */
#define SWV_PREDICT_TREE 0
#define SWV_PREDICT_DEGRID 1
#define SWV_PREDICT_DIRECT 2

#define SWV_CLEAN_MAX_CYCLES 64

typedef struct {
    int n_cycles;                            /* major cycles run */
    int64_t found[SWV_CLEAN_MAX_CYCLES];     /* components found per cycle */
    int64_t leaves[SWV_CLEAN_MAX_CYCLES];    /* distinct level-J pixels after it */
    double chi2[SWV_CLEAN_MAX_CYCLES];       /* sum |V - V_model|^2 after it */
    double ms_minor[SWV_CLEAN_MAX_CYCLES];   /* Hogbom kernel */
    double ms_build[SWV_CLEAN_MAX_CYCLES];   /* host tree build */
    double ms_predict[SWV_CLEAN_MAX_CYCLES]; /* tree prediction */
    double ms_image[SWV_CLEAN_MAX_CYCLES];   /* subtract + residual image */
    double ms_beam, ms_dirty;                /* dirty beam, first dirty image */
} swv_clean_stats_t;

/* The whole wavelet clean (sections 2.2 and 3.5): the dirty beam and the
 * cross-reference table once, the dirty image, then per major cycle up to
 * minor_iter Hogbom iterations, the tree of every component found so far
 * (swv_tree_build_pixels on the cross-referenced pixels), the model
 * visibilities by the tree route (FP64), the residual visibilities and the new
 * residual image.  With params->predictor DEGRID or DIRECT the same loop runs
 * with that predictor instead of the tree (ms_build then times the host
 * model-image or component-list step).  Stops after n_major cycles (<= SWV_CLEAN_MAX_CYCLES) or
 * when a minor cycle finds nothing.
 * u, v, w, vis_obs [n_vis] DEVICE (vis_obs complex128).  Outputs: beam
 * [(2 ny - 1)(2 nx - 1)] DEVICE, residual [nx * ny] DEVICE, vis_model [n_vis]
 * DEVICE complex128, comp_pix / comp_val [cap] HOST (all components in the
 * order found; cap >= minor_iter * n_major), *n_comp HOST, stats HOST (may be
 * NULL).  Allocates its scratch for the call and synchronises the stream. */
int swv_wavelet_clean(swv_ctx ctx, const swv_clean_params_t* params, int64_t n_vis,
                      const double* u, const double* v, const double* w, const void* vis_obs,
                      double* beam, double* residual, void* vis_model, int64_t cap,
                      int64_t* comp_pix, double* comp_val, int64_t* n_comp,
                      swv_clean_stats_t* stats);

/* ------------------------------------------- degridding comparator --- */

typedef struct {
    int64_t n_planes;     /* w planes */
    int grid_nx, grid_ny; /* padded uv grid (2 nx, 2 ny) */
    double w0, dw;        /* w of plane 0, plane spacing (wavelengths) */
    double c;             /* the centre of the image's n - 1 range */
    int64_t plane_bytes;  /* device memory of the planes */
    double host_ms;       /* wall time of the call up to the last launch */
} swv_degrid_stats_t;

/* The conventional predictor that section 2.2's major cycle uses and the
 * wavelet route replaces: a forward FFT of the model image and degridding
 * with an anti-aliasing kernel, plus a correction for the w-term.  Written as
 * a type-2 non-uniform FFT in (u, v, w) with the exponential-of-semicircle
 * kernel phi(z) = exp(beta (sqrt(1 - z^2) - 1)), beta = 2.3 W, over W cells in
 * each of u, v and w (Barnett, Magland & af Klinteberg 2019; w planes
 * interpolated as in the improved w-stacking of Ye et al. 2021):
 *   uv grid 2 nx x 2 ny cells of 1 / (2 nx cell) wavelengths; w planes
 *   dw = 1 / (2 E) apart, E the extent of n - 1 over the image and c its
 *   midpoint, from w_0 = min w - (W / 2) dw;
 *   plane q = FFT of the padded image I_p exp(s 2 pi i w_q (n_p - 1 - c))
 *   divided by the kernel's Fourier transform in l, m and (n - 1 - c) dw
 *   (100-node Gauss-Legendre quadrature in theta, x = (W / 2) sin theta);
 *   V_j = exp(s 2 pi i w_j c) sum over the W (or W + 1) nearest planes, rows
 *   and columns of kernel weight x plane value.
 * V_j approximates sum_p image[p] e^{s 2 pi i (u l_p + v m_p + w (n_p - 1))}
 * over the image grid of swv_image_grid (phase centre (nx / 2, ny / 2)) to
 * about 10^(1 - W) of sum |image|.  image [ny][nx] DEVICE FP64; u, v, w
 * [n_vis] DEVICE; vis_out [n_vis] DEVICE complex128 (NaN for a row with
 * non-finite coordinates); support W in 2 .. 16; stats HOST or NULL.
 * Synchronises once (for the w range); uses a context workspace of
 * 16 n_planes (4 nx ny) bytes plus the image, and a cached FFT plan.
 * SWV_ENOMEM if the planes would exceed 64 GiB. */
int swv_predict_degrid(swv_ctx ctx, int nx, int ny, double cell, const double* image,
                       int64_t n_vis, const double* u, const double* v, const double* w,
                       int support, int sign, void* vis_out, swv_degrid_stats_t* stats);

/* ------------------------------------------------------------ batched --- */

/* One prediction instance (a channel x pointing), all pointers DEVICE except
 * `tree`.  route SWV_ROUTE_DIRECT uses (n_comp, l, m, flux); SWV_ROUTE_TREE
 * uses `tree`.  vis_out is complex128 (SWV_FP64) or complex64 (SWV_F32C,
 * either route; the library cannot check the buffer's type: a complex64
 * buffer under SWV_FP64 is written past its end). */
typedef struct {
    int route;
    int prec;
    int sign;
    int64_t n_vis;
    const double* u;
    const double* v;
    const double* w;
    int64_t n_comp;
    const double* l;
    const double* m;
    const double* flux;
    swv_tree tree;
    void* vis_out;
} swv_instance;

typedef struct {
    int64_t n_instances;
    int64_t n_items;          /* (instance, visibility tile) work items */
    int64_t total_terms;      /* sum over instances of n_vis * terms */
    int tile_rows;            /* visibilities per work item */
    int grid_blocks;          /* persistent blocks launched */
    int block_threads;
} swv_plan_stats_t;

/* Plans one persistent launch per route (and, for trees, per precision) over
 * many instances: packs every
 * instance's components (direct) and uploads every tree, splits each
 * instance into visibility tiles and orders the (instance, tile) work items
 * by decreasing cost (longest-processing-time first).  Workgroups take items
 * from a device counter, so uneven instances balance across the chip.  The
 * tile shape comes from the context's tuning table.  `inst` [n] HOST; the
 * device buffers they name must outlive the plan. */
int swv_batch_plan(swv_ctx ctx, int n, const swv_instance* inst, swv_plan* out);

int swv_plan_stats(swv_plan plan, swv_plan_stats_t* out);

/* Enqueues the planned prediction on the context's stream. */
int swv_batch_run(swv_plan plan);

/* Captures the planned prediction (counter reset by a kernel, then the
 * persistent launches) into a HIP graph on the context's stream. */
int swv_graph_capture(swv_plan plan, swv_graph* out);

/* Replays a captured graph on the context's stream. */
int swv_graph_launch(swv_graph graph);

int swv_graph_destroy(swv_graph graph);
int swv_plan_destroy(swv_plan plan);

/* ------------------------------------------------------ major cycles --- */

typedef struct swv_cycle_s* swv_cycle;

/* One instance (a channel x pointing) of a captured major cycle.  All
 * pointers DEVICE; FP64 throughout.  route SWV_ROUTE_DIRECT predicts with the
 * component list set by swv_cycle_set_components, SWV_ROUTE_TREE with the tree
 * set by swv_cycle_set_tree. */
typedef struct {
    int route;
    int sign;                   /* +1 or -1 */
    int64_t n_vis;
    const double* u;            /* [n_vis] */
    const double* v;
    const double* w;
    const void* vis_obs;        /* [n_vis] complex128, observed visibilities */
    void* vis_model;            /* [n_vis] complex128, written: model visibilities */
    void* resid;                /* [n_vis] complex128, written: vis_obs - vis_model */
    double* chi2;               /* one FP64, written: inv_sigma2 * sum |resid|^2 */
    double inv_sigma2;
    int64_t n_pix;              /* pixel set of the residual image (0: no image) */
    const double* pix_l;        /* [n_pix] pixel centres, n - 1 given explicitly */
    const double* pix_m;
    const double* pix_nm1;
    void* image;                /* [n_pix] complex128, written: sum_j conj(e_jp) resid_j */
    int64_t comp_cap;           /* direct: most components a model may have; tree: most
                                   leaves */
    int tree_level_cap;         /* tree: largest J of a model (1 .. 29) */
    double* d_flux;             /* direct, optional (all three or none): [comp_cap]
                                   d chi^2 / d(flux, l, m) of the model's components */
    double* d_l;
    double* d_m;
} swv_cycle_instance;

/* A major cycle over many instances (section 2.2 steps 1-3, with the chi^2
 * gradients beside them), runnable eagerly or as one captured HIP graph:
 *   1. the model visibilities of every instance in one persistent launch per
 *      route (as swv_batch_plan: direct sums and wavelet trees, FP64);
 *   2. per instance the subtract step with chi^2 (swv_residual_chi2), the
 *      residual image on its pixel set (swv_adjoint of the residuals) and,
 *      for a direct instance with gradient outputs, the chi^2 gradients of its
 *      components (swv_grad_direct of the residuals with alpha = -2 inv_sigma2).
 * The model of each instance may change between cycles within the stated
 * capacities: its size, pointers and tree records are read on the device, so
 * a captured graph replays the new model without a new capture.  Grids and
 * tilings follow the capacities: results are bitwise the same eager and
 * replayed, and agree with the single calls to their tolerances (the
 * gradients' summation order follows comp_cap).  The cycle holds a tree
 * record buffer of 32 (comp_cap J_cap + 12) bytes per tree instance (at most
 * 4 GiB - 32 each, else SWV_ENOTSUP) and workspaces for the largest image and
 * gradient step.  The buffers named by `inst` must outlive the cycle.  Until a
 * model is set an instance predicts zero. */
int swv_cycle_create(swv_ctx ctx, int n, const swv_cycle_instance* inst, swv_cycle* out);

/* Sets the component list of direct instance k for the following cycles:
 * l, m, flux [n_comp] DEVICE (read on every run), n_comp <= comp_cap.
 * Gradient entries past n_comp are left untouched. */
int swv_cycle_set_components(swv_cycle cycle, int k, int64_t n_comp, const double* l,
                             const double* m, const double* flux);

/* Sets the tree of tree instance k for the following cycles: its records are
 * copied into the instance's buffer (after the work already on the context's
 * stream, which this call waits for), so the tree may be destroyed afterwards.
 * SWV_EINVAL if J exceeds tree_level_cap or the records the capacity;
 * SWV_ENOTSUP if the cycle's traversal cannot walk the tree. */
int swv_cycle_set_tree(swv_cycle cycle, int k, swv_tree tree);

/* Enqueues one cycle on the context's stream (uploading changed models first). */
int swv_cycle_run(swv_cycle cycle);

/* Captures the cycle as a HIP graph held by the cycle (replacing an earlier
 * one); capture needs no model to be set. */
int swv_cycle_capture(swv_cycle cycle);

/* Replays the captured graph on the context's stream, after uploading changed
 * models; SWV_EINVAL if nothing was captured. */
int swv_cycle_launch(swv_cycle cycle);

int swv_cycle_destroy(swv_cycle cycle);

/* ------------------------------------------------------ measured peaks --- */

typedef struct {
    double fp64_fma_tflops;   /* FP64 FMA stream, flop/s (FMA = 2) */
    double fp32_fma_tflops;   /* FP32 FMA stream, unpacked instructions */
    double sincos_f32_gops;   /* hardware FP32 sine + cosine pairs per second */
    double cis2pi_f64_gops;   /* FP64 phasors (the polynomial of every FP64
                                 kernel) per second */
} swv_peaks_t;

/* Measures the arithmetic ceilings of the device of `ctx` with
 * microbenchmarks of independent dependency chains (one warm-up launch, then
 * the median of three, tens of milliseconds each; about 0.3 s in all).  The
 * published peak is an upper bound the part reaches only at full clock; these
 * figures are what this library's kernels can reach.  Allocates and frees a
 * scratch buffer; synchronises the context's stream. */
int swv_measure_peaks(swv_ctx ctx, swv_peaks_t* out);

/* ------------------------------------------------------------- tuning --- */

/* Times every compiled tile shape of each kernel family (direct FP64,
 * direct F32C, tree, adjoint, gradients) on synthetic inputs of the two size
 * classes (2^18 and 2^22 rows), keeps
 * the fastest per (family, size class) in the context's tuning table and, if
 * `cache_path` is not NULL, writes the table there as JSON.  flags: 0 =
 * full sweep, 1 = quick sweep (fewer repetitions). */
int swv_autotune(swv_ctx ctx, const char* cache_path, int flags);

/* Loads a tuning table written by swv_autotune into the context. */
int swv_tune_load(swv_ctx ctx, const char* cache_path);

/* Tile shape the context uses per kernel family and size class.  Families:
 * 0 direct FP64, 1 direct F32C, 2 tree, 3 adjoint, 4 gradients.  Size class
 * 0 is fewer than 2^20 visibility rows, 1 the rest.  per_lane is rows per lane
 * (direct), pixels per lane (adjoint) or components per lane (gradients), in
 * {1, 2, 4}; for the tree it selects the traversal (1: by depth and shape as
 * swv_predict_tree describes; 2: per branching node where it fits; 4: per
 * level where J <= 16).  block is threads per block in {64, 128, 256}; the
 * gradients' entries hold 128 (swv_tune_set rejects any other value for them):
 * their launches take the narrowest block of 128 .. 1024 threads that holds
 * every component at per_lane (else 1024).  Results do not depend on the
 * shape except for the summation order of the adjoint and gradients. */
int swv_tune_get(swv_ctx ctx, int family, int size_class, int* per_lane, int* block);

/* Sets one entry of the context's tuning table (SWV_EINVAL for a shape that is
 * not compiled). */
int swv_tune_set(swv_ctx ctx, int family, int size_class, int per_lane, int block);

#ifdef __cplusplus
}
#endif

#endif /* SWVIS_H */
