// Major-cycle kernels around the prediction: the subtract step with chi^2
// (section 2.2), the exact adjoint of the direct sum (the residual image on
// sphere pixels), and the chi^2 gradients of the direct sum.
//
// Adjoint and gradients swap the roles of the direct kernel: lanes own the
// outputs (pixels or components) and every lane of the wave walks the same
// visibility rows (the adjoint reads them with scalar loads, the gradients
// stage them through LDS).  The visibility axis is split
// into fixed chunks; each (chunk, tile) block writes its partial sums, and a
// second kernel adds the chunks in index order -- deterministic and free of
// atomics.
//
// Block order (1-D grid): workgroups are dealt to the 8 XCDs round-robin by
// linear id, and blocks sharing a chunk read the same rows.  Ids therefore
// walk groups of 8 chunks -- one per XCD -- and, inside a group, all tiles in
// consecutive dispatch rounds: every tile of a chunk runs on the same XCD at
// about the same time and the chunk's rows come from HBM into one L2 once.
#include "device_math.h"
#include "launch.h"

namespace swv {

// Chunk count rounded up to a whole number of XCD rounds.
static int64_t xcd_padded(int64_t n_chunks) { return (n_chunks + 7) / 8 * 8; }

// (chunk, tile) of linear block id `bid` in the order described above.
__device__ __forceinline__ void chunk_tile(int64_t bid, int64_t tiles, int64_t& chunk,
                                           int64_t& tile) {
    const int64_t per_group = 8 * tiles;
    const int64_t g = bid / per_group;
    const int64_t r = bid - g * per_group;
    tile = r >> 3;
    chunk = g * 8 + (r & 7);
}

// Launches `total` blocks as 1-D grids of at most 2^30 blocks, passing the
// first linear id of each.
template <class F>
static void launch_slabs(int64_t total, F&& launch) {
    constexpr int64_t kSlab = int64_t(1) << 30;
    for (int64_t b0 = 0; b0 < total; b0 += kSlab)
        launch(b0, (unsigned)(total - b0 < kSlab ? total - b0 : kSlab));
}

// ---------------------------------------------------------------- adjoint --
// img[p] = sum_j conj(e_jp) y_j, e = exp(s 2 pi i phi).  With e = c + i s S:
// conj(e) y = (c yr + s S yi) + i (c yi - s S yr), S = 4 q.
// One lane's G pixels q0, q0 + 64, ... over the rows of chunk chunk_id.
template <int G, int PREC>
__device__ __forceinline__ void adjoint_lane(
    const double* __restrict__ u, const double* __restrict__ v, const double* __restrict__ w,
    const double2* __restrict__ y, int64_t n_vis, int64_t chunk, const double* __restrict__ pl,
    const double* __restrict__ pm, const double* __restrict__ pn, int64_t n_pix, double sgn,
    int64_t chunk_id, int64_t q0, double2* __restrict__ partial) {
    double L[G], M[G], N[G];
    double ar[G], ai[G];
    float sr[G], cr[G], si[G], ci[G];
#pragma unroll
    for (int i = 0; i < G; ++i) {
        int64_t p = q0 + (int64_t)i * 64;
        p = p < n_pix ? p : n_pix - 1;
        L[i] = pl[p];
        M[i] = pm[p];
        N[i] = pn[p];
        ar[i] = ai[i] = 0.0;
        sr[i] = cr[i] = si[i] = ci[i] = 0.0f;
    }
    const int64_t j0 = chunk_id * chunk;
    const int64_t j1 = j0 + chunk < n_vis ? j0 + chunk : n_vis;
    // wave-uniform trip count, kept in scalar registers
    const int nrow = __builtin_amdgcn_readfirstlane((int)(j1 - j0));
    const auto* U = uniform_ptr(u + j0);
    const auto* V = uniform_ptr(v + j0);
    const auto* W = uniform_ptr(w + j0);
    const auto* Y = uniform_ptr(y + j0);
    if constexpr (PREC == SWV_FP64) {
#pragma unroll 4
        for (int j = 0; j < nrow; ++j) {
            const double uj = U[j], vj = V[j], wj = W[j];
            const double yr = Y[j].x, yi = Y[j].y;
            const double y4r = 4.0 * sgn * yr, y4i = 4.0 * sgn * yi;
#pragma unroll
            for (int i = 0; i < G; ++i) {
                double c, q;
                cis2pi_q(reduced_phase(uj, vj, wj, L[i], M[i], N[i]), c, q);
                ar[i] = fma(c, yr, ar[i]);
                ar[i] = fma(q, y4i, ar[i]);
                ai[i] = fma(c, yi, ai[i]);
                ai[i] = fma(-q, y4r, ai[i]);
            }
        }
    } else {
        // rows in pairs: the pair's four products and the running compensation
        // meet in one chain of FMAs, then one Kahan step, so a row costs half a
        // step (the chain's roundings stay within a few 2^-24 of the pair's
        // terms); an odd last row enters alone
        // sgn is +-1, so fsg * (float)y is (float)(sgn * y) bit for bit
        const float fsg = (float)sgn;
        const auto cis = [&](double uj, double vj, double wj, int i, float& c, float& s) {
            cis2pi_f32((float)fract_phase(uj, vj, wj, L[i], M[i], N[i]), c, s);
        };
        const int npair = nrow & ~1;
#pragma unroll 2
        for (int j = 0; j < npair; j += 2) {
            const double u0 = U[j], v0 = V[j], w0 = W[j], yr0 = Y[j].x, yi0 = Y[j].y;
            const double u1 = U[j + 1], v1 = V[j + 1], w1 = W[j + 1];
            const double yr1 = Y[j + 1].x, yi1 = Y[j + 1].y;
            const float fyr0 = (float)yr0, fyi0 = (float)yi0;
            const float fsyr0 = fsg * fyr0, fsyi0 = fsg * fyi0;
            const float fyr1 = (float)yr1, fyi1 = (float)yi1;
            const float fsyr1 = fsg * fyr1, fsyi1 = fsg * fyi1;
#pragma unroll
            for (int i = 0; i < G; ++i) {
                float c0, s0, c1, s1;
                cis(u0, v0, w0, i, c0, s0);
                cis(u1, v1, w1, i, c1, s1);
                kahan_step(fmaf(c0, fyr0, fmaf(s0, fsyi0, fmaf(c1, fyr1, fmaf(s1, fsyi1, -cr[i])))),
                           sr[i], cr[i]);
                kahan_step(fmaf(c0, fyi0, fmaf(-s0, fsyr0, fmaf(c1, fyi1, fmaf(-s1, fsyr1, -ci[i])))),
                           si[i], ci[i]);
            }
        }
        if (npair < nrow) {
            const int j = npair;
            const double yr = Y[j].x, yi = Y[j].y;
            const float fyr = (float)yr, fyi = (float)yi;
            const float fsyr = fsg * fyr, fsyi = fsg * fyi;
#pragma unroll
            for (int i = 0; i < G; ++i) {
                float c, s;
                cis(U[j], V[j], W[j], i, c, s);
                kahan_step(fmaf(c, fyr, fmaf(s, fsyi, -cr[i])), sr[i], cr[i]);
                kahan_step(fmaf(c, fyi, fmaf(-s, fsyr, -ci[i])), si[i], ci[i]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < G; ++i) {
        const int64_t p = q0 + (int64_t)i * 64;
        if (p < n_pix) {
            double2 o;
            if constexpr (PREC == SWV_FP64)
                o = make_double2(ar[i], ai[i]);
            else
                o = make_double2((double)sr[i] - (double)cr[i], (double)si[i] - (double)ci[i]);
            partial[chunk_id * n_pix + p] = o;
        }
    }
}

// Each wave of a tile owns PPL consecutive groups of 64 pixels (lane l of the
// wave takes pixel l of each group), so the pixels past the last one gather
// in whole groups at the end of the last tile, which are not computed (the
// 955-pixel image of the major cycle in one 1,024-pixel tile: 64 of its 69
// idle slots).  A pixel's sum is the same whichever lane takes it.
template <int PPL, int BLOCK, int PREC>
__global__ __launch_bounds__(BLOCK) void k_adjoint(
    const double* __restrict__ u, const double* __restrict__ v, const double* __restrict__ w,
    const double2* __restrict__ y, int64_t n_vis, int64_t chunk, const double* __restrict__ pl,
    const double* __restrict__ pm, const double* __restrict__ pn, int64_t n_pix, double sgn,
    int64_t n_chunks, int64_t tiles, int64_t bid0, double2* __restrict__ partial) {
    int64_t chunk_id, tile;
    chunk_tile(bid0 + blockIdx.x, tiles, chunk_id, tile);
    if (chunk_id >= n_chunks) return;   // padding of the last XCD group
    static_assert(BLOCK % 64 == 0, "whole waves");
    const int wave = (int)(threadIdx.x / 64), lane = (int)(threadIdx.x % 64);
    const int64_t g0 = tile * (BLOCK * PPL) + (int64_t)wave * (64 * PPL);
    const int64_t left = n_pix - g0;   // the same for every lane of the wave
    const int groups = __builtin_amdgcn_readfirstlane(
        left <= 0 ? 0 : (left >= 64 * PPL ? PPL : (int)((left + 63) / 64)));
    const int64_t q0 = g0 + lane;
    if (groups >= PPL) {
        adjoint_lane<PPL, PREC>(u, v, w, y, n_vis, chunk, pl, pm, pn, n_pix, sgn, chunk_id, q0,
                                partial);
    } else if constexpr (PPL >= 2) {
        if (groups == 1)
            adjoint_lane<1, PREC>(u, v, w, y, n_vis, chunk, pl, pm, pn, n_pix, sgn, chunk_id, q0,
                                  partial);
        if constexpr (PPL >= 4) {
            if (groups == 2)
                adjoint_lane<2, PREC>(u, v, w, y, n_vis, chunk, pl, pm, pn, n_pix, sgn, chunk_id,
                                      q0, partial);
            if (groups == 3)
                adjoint_lane<3, PREC>(u, v, w, y, n_vis, chunk, pl, pm, pn, n_pix, sgn, chunk_id,
                                      q0, partial);
        }
    }
}

// out[p] = sum over chunks c of partial[c][p].
// Chunk reductions: a block owns kSumCols consecutive outputs (coalesced along
// x); its kSumQ rows of threads each add the chunks q, q + kSumQ, ... in order,
// and the kSumQ subtotals are then added by a fixed binary tree in LDS.  The
// order depends only on the chunk count, so results are run-to-run identical.
constexpr int kSumCols = 64;
constexpr int kSumQ = 16;

__global__ __launch_bounds__(kSumCols * kSumQ) void k_sum_chunks_c128(
    const double2* __restrict__ partial, int64_t n_chunks, int64_t n, double2* __restrict__ out) {
    __shared__ double red_r[kSumQ][kSumCols], red_i[kSumQ][kSumCols];
    const int tx = threadIdx.x % kSumCols, q = threadIdx.x / kSumCols;
    const int64_t p = (int64_t)blockIdx.x * kSumCols + tx;
    double re = 0.0, im = 0.0;
    if (p < n) {
        for (int64_t c = q; c < n_chunks; c += kSumQ) {
            const double2 x = partial[c * n + p];
            re += x.x;
            im += x.y;
        }
    }
    red_r[q][tx] = re;
    red_i[q][tx] = im;
    __syncthreads();
    for (int h = kSumQ / 2; h > 0; h >>= 1) {
        if (q < h) {
            red_r[q][tx] += red_r[q + h][tx];
            red_i[q][tx] += red_i[q + h][tx];
        }
        __syncthreads();
    }
    if (q == 0 && p < n) out[p] = make_double2(red_r[0][tx], red_i[0][tx]);
}

template <int PPL, int BLOCK, int PREC>
static void run_adjoint(hipStream_t s, int64_t tiles, int64_t chunk, int64_t n_vis,
                        const double* u, const double* v, const double* w, const void* y,
                        int64_t n_pix, const double* l, const double* m, const double* nm1,
                        int sign, void* partial) {
    const int64_t n_chunks = (n_vis + chunk - 1) / chunk;
    launch_slabs(xcd_padded(n_chunks) * tiles, [&](int64_t b0, unsigned nb) {
        k_adjoint<PPL, BLOCK, PREC><<<dim3(nb), dim3(BLOCK), 0, s>>>(
            u, v, w, (const double2*)y, n_vis, chunk, l, m, nm1, n_pix, (double)sign, n_chunks,
            tiles, b0, (double2*)partial);
    });
}

template <int PPL, int PREC>
static hipError_t run_adjoint_b(hipStream_t s, int block, int64_t grid, int64_t chunk,
                                int64_t n_vis, const double* u, const double* v, const double* w,
                                const void* y, int64_t n_pix, const double* l, const double* m,
                                const double* nm1, int sign, void* partial) {
    switch (block) {
        case 64: run_adjoint<PPL, 64, PREC>(s, grid, chunk, n_vis, u, v, w, y, n_pix, l, m, nm1, sign, partial); break;
        case 128: run_adjoint<PPL, 128, PREC>(s, grid, chunk, n_vis, u, v, w, y, n_pix, l, m, nm1, sign, partial); break;
        case 256: run_adjoint<PPL, 256, PREC>(s, grid, chunk, n_vis, u, v, w, y, n_pix, l, m, nm1, sign, partial); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Blocks of one kernel shape that fit on a compute unit at once (registers,
// LDS, waves), from the runtime's occupancy calculator; cached per shape.
template <class K>
static int resident_blocks(K kernel, int block) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, block, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return nb > 0 ? nb : 1;
}

template <int PPL, int BLOCK, int PREC>
static int adjoint_occ() {
    static const int v = resident_blocks(k_adjoint<PPL, BLOCK, PREC>, BLOCK);
    return v;
}

int adjoint_blocks_per_cu(int prec, int ppl, int block) {
#define SWV_OCC_A(P, B)                                                                   \
    if (ppl == P && block == B)                                                           \
        return prec == SWV_FP64 ? adjoint_occ<P, B, SWV_FP64>() : adjoint_occ<P, B, SWV_F32C>();
    SWV_OCC_A(1, 64) SWV_OCC_A(1, 128) SWV_OCC_A(1, 256)
    SWV_OCC_A(2, 64) SWV_OCC_A(2, 128) SWV_OCC_A(2, 256)
    SWV_OCC_A(4, 64) SWV_OCC_A(4, 128) SWV_OCC_A(4, 256)
#undef SWV_OCC_A
    return 1;
}

hipError_t launch_adjoint(hipStream_t s, int prec, int ppl, int block, int64_t chunk,
                          int64_t n_vis, const double* u, const double* v, const double* w,
                          const void* y, int64_t n_pix, const double* l, const double* m,
                          const double* nm1, int sign, void* partial, void* out) {
    if (n_pix <= 0) return hipSuccess;
    const int64_t n_chunks = n_vis > 0 ? (n_vis + chunk - 1) / chunk : 0;
    if (n_chunks > 0) {
        const int64_t per_block = (int64_t)block * ppl;
        const int64_t grid = (n_pix + per_block - 1) / per_block;   // pixel tiles
        hipError_t e;
        if (prec == SWV_FP64) {
            switch (ppl) {
                case 1: e = run_adjoint_b<1, SWV_FP64>(s, block, grid, chunk, n_vis, u, v, w, y, n_pix, l, m, nm1, sign, partial); break;
                case 2: e = run_adjoint_b<2, SWV_FP64>(s, block, grid, chunk, n_vis, u, v, w, y, n_pix, l, m, nm1, sign, partial); break;
                case 4: e = run_adjoint_b<4, SWV_FP64>(s, block, grid, chunk, n_vis, u, v, w, y, n_pix, l, m, nm1, sign, partial); break;
                default: return hipErrorInvalidValue;
            }
        } else {
            switch (ppl) {
                case 1: e = run_adjoint_b<1, SWV_F32C>(s, block, grid, chunk, n_vis, u, v, w, y, n_pix, l, m, nm1, sign, partial); break;
                case 2: e = run_adjoint_b<2, SWV_F32C>(s, block, grid, chunk, n_vis, u, v, w, y, n_pix, l, m, nm1, sign, partial); break;
                case 4: e = run_adjoint_b<4, SWV_F32C>(s, block, grid, chunk, n_vis, u, v, w, y, n_pix, l, m, nm1, sign, partial); break;
                default: return hipErrorInvalidValue;
            }
        }
        if (e != hipSuccess) return e;
    }
    k_sum_chunks_c128<<<dim3((unsigned)((n_pix + kSumCols - 1) / kSumCols)),
                        dim3(kSumCols * kSumQ), 0, s>>>((const double2*)partial, n_chunks, n_pix,
                                                       (double2*)out);
    return hipGetLastError();
}

// -------------------------------------------------------------- gradients --
// The gradients need four real sums per component k (CPL per lane) and chunk
// of rows, with z = conj(y) e:
//   Z0 = Re sum z                    (flux:      dchi2/dI ~ Re A^H r)
//   Zu, Zv, Zw = Im sum {u, v, w} z  (positions: d phi/dl = u - w l / n, ...)
// conj(y) e = (yr - i yi)(c + i s S) = (yr c + yi s S) + i (yr s S - yi c),
// S = 4 q; the products 4 s y are formed once per row for all CPL components.
//
// Rows are staged through LDS in tiles of kGradRowTile: the block loads each
// tile once with coalesced vector loads and forms 4 s y there, once per row;
// every wave then reads the rows as LDS broadcasts.  The block is as wide as
// the component list needs (up to 1024 threads), so that one block covers
// every component of a chunk and each row is fetched from memory once.
constexpr int kGradRowTile = 256;

// n_comp_dev, if not null, holds the number of components on the device (a
// captured major cycle whose model changes between replays): the grid is then
// sized for n_comp, the capacity, and blocks past the actual count leave.
template <int CPL, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_grad_partial(
    const double* __restrict__ u, const double* __restrict__ v, const double* __restrict__ w,
    const double2* __restrict__ y, int64_t n_vis, int64_t chunk, const Comp* __restrict__ comp,
    int64_t n_comp, const int* __restrict__ n_comp_dev, double sgn, int64_t n_chunks,
    int64_t tiles, int64_t bid0, double* __restrict__ partial) {
    // one row: u, v, w, yr, yi, 4 s yr, 4 s yi, (pad) -- 64 bytes
    __shared__ double2 rows[kGradRowTile][4];
    int64_t chunk_id, tile;
    chunk_tile(bid0 + blockIdx.x, tiles, chunk_id, tile);
    if (chunk_id >= n_chunks) return;   // padding of the last XCD group (whole block)
    if (n_comp_dev) n_comp = *n_comp_dev;
    if (tile * (BLOCK * CPL) >= n_comp) return;   // no component in this tile (whole block)
    const int64_t k0 = tile * (BLOCK * CPL) + threadIdx.x;
    double L[CPL], M[CPL], N[CPL];
    double z0[CPL], zu[CPL], zv[CPL], zw[CPL];
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
        int64_t k = k0 + (int64_t)i * BLOCK;
        k = k < n_comp ? k : n_comp - 1;
        L[i] = comp[k].l;
        M[i] = comp[k].m;
        N[i] = comp[k].nm1;
        z0[i] = zu[i] = zv[i] = zw[i] = 0.0;
    }
    const int64_t j0 = chunk_id * chunk;
    const int64_t j1 = j0 + chunk < n_vis ? j0 + chunk : n_vis;
    const double s4 = 4.0 * sgn;
    for (int64_t t0 = j0; t0 < j1; t0 += kGradRowTile) {
        const int nt = (int)(j1 - t0 < kGradRowTile ? j1 - t0 : kGradRowTile);
        __syncthreads();   // the previous tile has been read by every wave
        for (int r = threadIdx.x; r < nt; r += BLOCK) {
            const int64_t j = t0 + r;
            const double2 yj = y[j];
            rows[r][0] = make_double2(u[j], v[j]);
            rows[r][1] = make_double2(w[j], yj.x);
            rows[r][2] = make_double2(yj.y, s4 * yj.x);
            rows[r][3] = make_double2(s4 * yj.y, 0.0);
        }
        __syncthreads();
        // wave-uniform trip count, kept in scalar registers
        const int nrow = __builtin_amdgcn_readfirstlane(nt);
        // the next row's LDS reads are issued before this row's arithmetic,
        // so their latency is hidden behind it (the last row reads itself
        // again, in bounds)
        double2 na = rows[0][0], nb = rows[0][1], nc = rows[0][2], nd = rows[0][3];
#pragma unroll 1
        for (int r = 0; r < nrow; ++r) {
            const double2 a = na, b = nb, c2 = nc, d = nd;
            const int rn = r + 1 < nrow ? r + 1 : r;
            na = rows[rn][0];
            nb = rows[rn][1];
            nc = rows[rn][2];
            nd = rows[rn][3];
            const double uj = a.x, vj = a.y, wj = b.x;
            const double yr = b.y, yi = c2.x, y4r = c2.y, y4i = d.x;
#pragma unroll
            for (int i = 0; i < CPL; ++i) {
                double c, q;
                cis2pi_q(reduced_phase(uj, vj, wj, L[i], M[i], N[i]), c, q);
                // Re z goes straight into its sum: two FMAs, no product of its own
                z0[i] = fma(c, yr, fma(q, y4i, z0[i]));
                const double zi = fma(q, y4r, -(yi * c));
                zu[i] = fma(uj, zi, zu[i]);
                zv[i] = fma(vj, zi, zv[i]);
                zw[i] = fma(wj, zi, zw[i]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
        const int64_t k = k0 + (int64_t)i * BLOCK;
        if (k < n_comp) {
            double* o = partial + (chunk_id * 4) * n_comp + k;
            o[0 * n_comp] = z0[i];
            o[1 * n_comp] = zu[i];
            o[2 * n_comp] = zv[i];
            o[3 * n_comp] = zw[i];
        }
    }
}

__global__ __launch_bounds__(kSumCols * kSumQ) void k_grad_finish(
    const double* __restrict__ partial, int64_t n_chunks, const Comp* __restrict__ comp,
    int64_t n_comp, const int* __restrict__ n_comp_dev, double sgn, double alpha,
    double* __restrict__ d_flux, double* __restrict__ d_l, double* __restrict__ d_m) {
    __shared__ double red[4][kSumQ][kSumCols];
    if (n_comp_dev) n_comp = *n_comp_dev;
    if ((int64_t)blockIdx.x * kSumCols >= n_comp) return;   // whole block past the count
    const int tx = threadIdx.x % kSumCols, q = threadIdx.x / kSumCols;
    const int64_t k = (int64_t)blockIdx.x * kSumCols + tx;
    double z[4] = {0, 0, 0, 0};
    if (k < n_comp) {
        for (int64_t c = q; c < n_chunks; c += kSumQ)
            for (int t = 0; t < 4; ++t) z[t] += partial[(c * 4 + t) * n_comp + k];
    }
    for (int t = 0; t < 4; ++t) red[t][q][tx] = z[t];
    __syncthreads();
    for (int h = kSumQ / 2; h > 0; h >>= 1) {
        if (q < h)
            for (int t = 0; t < 4; ++t) red[t][q][tx] += red[t][q + h][tx];
        __syncthreads();
    }
    if (q != 0 || k >= n_comp) return;
    const double z0 = red[0][0][tx], zu = red[1][0][tx], zv = red[2][0][tx],
                 zw = red[3][0][tx];
    const double n = 1.0 + comp[k].nm1;
    const double f = -alpha * comp[k].I * sgn * 2.0 * M_PI;
    d_flux[k] = alpha * z0;
    d_l[k] = f * (zu - (comp[k].l / n) * zw);
    d_m[k] = f * (zv - (comp[k].m / n) * zw);
}

template <int CPL, int BLOCK>
static int grad_occ() {
    static const int v = resident_blocks(k_grad_partial<CPL, BLOCK>, BLOCK);
    return v;
}

void grad_tiling(int cpl, int64_t n_comp, int* block, int64_t* tiles) {
    int b = 128;
    while (b < 1024 && (int64_t)b * cpl < n_comp) b *= 2;
    *block = b;
    *tiles = n_comp > 0 ? (n_comp + (int64_t)b * cpl - 1) / ((int64_t)b * cpl) : 1;
}

int grad_blocks_per_cu(int cpl, int block) {
#define SWV_OCC_G(C, B) if (cpl == C && block == B) return grad_occ<C, B>();
    SWV_OCC_G(1, 128) SWV_OCC_G(1, 256) SWV_OCC_G(1, 512) SWV_OCC_G(1, 1024)
    SWV_OCC_G(2, 128) SWV_OCC_G(2, 256) SWV_OCC_G(2, 512) SWV_OCC_G(2, 1024)
    SWV_OCC_G(4, 128) SWV_OCC_G(4, 256) SWV_OCC_G(4, 512) SWV_OCC_G(4, 1024)
#undef SWV_OCC_G
    return 1;
}

hipError_t launch_grad(hipStream_t s, int cpl, int64_t chunk, int64_t n_vis, const double* u,
                       const double* v, const double* w, const void* y, const Comp* comp,
                       int64_t n_comp, int sign, double alpha, double* partial, double* d_flux,
                       double* d_l, double* d_m, const int* n_comp_dev) {
    if (n_comp <= 0) return hipSuccess;
    if (cpl != 1 && cpl != 2 && cpl != 4) return hipErrorInvalidValue;
    const int64_t n_chunks = n_vis > 0 ? (n_vis + chunk - 1) / chunk : 0;
    if (n_chunks > 0) {
        int block = 128;
        int64_t tiles = 1;
        grad_tiling(cpl, n_comp, &block, &tiles);
        const double sg = (double)sign;
        const double2* yy = (const double2*)y;
        launch_slabs(xcd_padded(n_chunks) * tiles, [&](int64_t b0, unsigned nb) {
#define SWV_RUN_G(C, B)                                                                      \
    if (cpl == C && block == B)                                                              \
        k_grad_partial<C, B><<<dim3(nb), dim3(B), 0, s>>>(u, v, w, yy, n_vis, chunk, comp, n_comp, \
                                                          n_comp_dev, sg, n_chunks, tiles, b0,  \
                                                          partial);
            SWV_RUN_G(1, 128) SWV_RUN_G(1, 256) SWV_RUN_G(1, 512) SWV_RUN_G(1, 1024)
            SWV_RUN_G(2, 128) SWV_RUN_G(2, 256) SWV_RUN_G(2, 512) SWV_RUN_G(2, 1024)
            SWV_RUN_G(4, 128) SWV_RUN_G(4, 256) SWV_RUN_G(4, 512) SWV_RUN_G(4, 1024)
#undef SWV_RUN_G
        });
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_grad_finish<<<dim3((unsigned)((n_comp + kSumCols - 1) / kSumCols)), dim3(kSumCols * kSumQ),
                    0, s>>>(partial, n_chunks, comp, n_comp, n_comp_dev, (double)sign, alpha,
                            d_flux, d_l, d_m);
    return hipGetLastError();
}

// ------------------------------------------------------ residual and chi^2 --
constexpr int kResBlock = 256;
constexpr int kResMaxBlocks = 2048;

int residual_blocks(int64_t n_vis) {
    const int64_t b = (n_vis + kResBlock * 8 - 1) / (kResBlock * 8);
    return (int)(b < 1 ? 1 : (b > kResMaxBlocks ? kResMaxBlocks : b));
}

__global__ __launch_bounds__(kResBlock) void k_residual(const double2* __restrict__ obs,
                                                        const double2* __restrict__ model,
                                                        int64_t n, double2* __restrict__ resid,
                                                        double* __restrict__ partial) {
    __shared__ double red[kResBlock];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kResBlock;
    for (int64_t j = (int64_t)blockIdx.x * kResBlock + threadIdx.x; j < n; j += stride) {
        const double2 a = obs[j], b = model[j];
        const double rr = a.x - b.x, ri = a.y - b.y;
        resid[j] = make_double2(rr, ri);
        acc = fma(rr, rr, fma(ri, ri, acc));
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kResBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// One block: thread t adds partials t, t + kResBlock, ... in order, then a
// fixed binary tree in LDS.
__global__ __launch_bounds__(kResBlock) void k_chi2_finish(const double* __restrict__ partial,
                                                           int nb, double inv_sigma2,
                                                           double* __restrict__ chi2) {
    __shared__ double red[kResBlock];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kResBlock) s += partial[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kResBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *chi2 = red[0] * inv_sigma2;
}

hipError_t launch_residual(hipStream_t s, int64_t n_vis, const void* obs, const void* model,
                           double inv_sigma2, void* resid, double* partial, double* chi2) {
    const int nb = n_vis > 0 ? residual_blocks(n_vis) : 0;
    if (nb > 0) {
        k_residual<<<dim3(nb), dim3(kResBlock), 0, s>>>((const double2*)obs,
                                                        (const double2*)model, n_vis,
                                                        (double2*)resid, partial);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_chi2_finish<<<1, kResBlock, 0, s>>>(partial, nb, inv_sigma2, chi2);
    return hipGetLastError();
}

}  // namespace swv
