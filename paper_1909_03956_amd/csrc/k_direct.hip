// Direct component sum (section 3.3, Eq. 12) on gfx950: the component
// ingest and the single-instance kernels.  Rows of a block are strided by
// the block size so each of a lane's VPL loads is coalesced.
#include "direct_rows.h"

namespace swv {

__global__ void k_ingest(int64_t n, const double* __restrict__ l, const double* __restrict__ m,
                         const double* __restrict__ flux, Comp* __restrict__ out,
                         int* __restrict__ status) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int bad;
    out[k] = pack_component(l[k], m[k], flux[k], bad);
    if (bad) atomicOr(status, bad);
}

hipError_t launch_ingest(hipStream_t s, int64_t n, const double* l, const double* m,
                         const double* flux, Comp* out, int* status) {
    if (n <= 0) return hipSuccess;
    const int b = 256;
    k_ingest<<<dim3((unsigned)((n + b - 1) / b)), dim3(b), 0, s>>>(n, l, m, flux, out, status);
    return hipGetLastError();
}

template <int VPL, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_direct_f64(const double* __restrict__ u,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ w, int64_t n_vis,
                                                      const Comp* __restrict__ comp, int n_comp,
                                                      double sgn, double2* __restrict__ out,
                                                      int* __restrict__ status) {
    const int64_t base = (int64_t)blockIdx.x * (BLOCK * VPL) + threadIdx.x;
    int64_t j[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) j[i] = base + (int64_t)i * BLOCK;
    direct_rows_f64<VPL>(j, n_vis, u, v, w, comp, n_comp, sgn, out, status);
}

template <int VPL, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_direct_f32c(const double* __restrict__ u,
                                                       const double* __restrict__ v,
                                                       const double* __restrict__ w,
                                                       int64_t n_vis,
                                                       const Comp* __restrict__ comp, int n_comp,
                                                       float sgn, float2* __restrict__ out,
                                                       int* __restrict__ status) {
    const int64_t base = (int64_t)blockIdx.x * (BLOCK * VPL) + threadIdx.x;
    int64_t j[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) j[i] = base + (int64_t)i * BLOCK;
    direct_rows_f32c<VPL>(j, n_vis, u, v, w, comp, n_comp, sgn, out, status);
}

template <int VPL, int BLOCK>
static hipError_t run_direct(hipStream_t s, int prec, int64_t n_vis, const double* u,
                             const double* v, const double* w, const Comp* comp, int64_t n_comp,
                             int sign, void* out, int* status) {
    const int64_t rows = (int64_t)BLOCK * VPL;
    const dim3 grid((unsigned)((n_vis + rows - 1) / rows)), blk(BLOCK);
    if (prec == SWV_FP64)
        k_direct_f64<VPL, BLOCK><<<grid, blk, 0, s>>>(u, v, w, n_vis, comp, (int)n_comp,
                                                       (double)sign, (double2*)out, status);
    else
        k_direct_f32c<VPL, BLOCK><<<grid, blk, 0, s>>>(u, v, w, n_vis, comp, (int)n_comp,
                                                        (float)sign, (float2*)out, status);
    return hipGetLastError();
}

template <int VPL>
static hipError_t run_direct_b(hipStream_t s, int prec, int block, int64_t n_vis,
                               const double* u, const double* v, const double* w,
                               const Comp* comp, int64_t n_comp, int sign, void* out,
                               int* status) {
    switch (block) {
        case 64: return run_direct<VPL, 64>(s, prec, n_vis, u, v, w, comp, n_comp, sign, out, status);
        case 128: return run_direct<VPL, 128>(s, prec, n_vis, u, v, w, comp, n_comp, sign, out, status);
        case 256: return run_direct<VPL, 256>(s, prec, n_vis, u, v, w, comp, n_comp, sign, out, status);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_direct(hipStream_t s, int prec, int vpl, int block, int64_t n_vis,
                         const double* u, const double* v, const double* w, const Comp* comp,
                         int64_t n_comp, int sign, void* out, int* status) {
    if (n_vis <= 0) return hipSuccess;
    switch (vpl) {
        case 1: return run_direct_b<1>(s, prec, block, n_vis, u, v, w, comp, n_comp, sign, out, status);
        case 2: return run_direct_b<2>(s, prec, block, n_vis, u, v, w, comp, n_comp, sign, out, status);
        case 4: return run_direct_b<4>(s, prec, block, n_vis, u, v, w, comp, n_comp, sign, out, status);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace swv
