// Persistent batched prediction: many instances (channels x pointings) of
// uneven size in one launch per route.
//
// The host splits every instance into row tiles and orders the (instance,
// tile) work items by decreasing cost, largest first.  Each wave of a
// grid sized to stay resident takes the next item from a device counter
// (one atomic per item, on lane 0), so long and short instances balance
// across the chip without a second launch; a wave leaves when the counter
// passes the item count, so every wave exits.  The row arithmetic is the
// single-instance kernels' (direct_rows.h, tree_walk.h).
#include "direct_rows.h"
#include "tree_walk.h"

namespace swv {

// Packs the components of every direct instance: block row y is instance y.
__global__ void k_batch_ingest(const BatchInst* __restrict__ inst, Comp* __restrict__ pack,
                               int* __restrict__ status) {
    const BatchInst I = inst[blockIdx.y];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= I.n_comp) return;
    int bad;
    pack[I.comp_offset + k] = pack_component(I.l[k], I.m[k], I.flux[k], bad);
    if (bad) atomicOr(status, bad);
}

hipError_t launch_batch_ingest(hipStream_t s, const BatchInst* inst, int n_inst, int max_comp,
                               Comp* pack, int* status) {
    if (n_inst <= 0 || max_comp <= 0) return hipSuccess;
    k_batch_ingest<<<dim3((unsigned)((max_comp + 255) / 256), (unsigned)n_inst), dim3(256), 0,
                     s>>>(inst, pack, status);
    return hipGetLastError();
}

// Work-counter reset as a kernel, so a captured graph re-arms itself on
// every replay without a memset node.
__global__ void k_reset_counters(unsigned* counters, int n) {
    if ((int)threadIdx.x < n) counters[threadIdx.x] = 0u;
}

hipError_t launch_reset_counters(hipStream_t s, unsigned* counters, int n) {
    k_reset_counters<<<1, 64, 0, s>>>(counters, n);
    return hipGetLastError();
}

__device__ __forceinline__ unsigned next_item(unsigned* counter) {
    unsigned it = 0;
    if ((threadIdx.x & 63) == 0) it = atomicAdd(counter, 1u);
    return __builtin_amdgcn_readfirstlane(it);
}

template <int VPL, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_batch_direct(const BatchInst* __restrict__ inst,
                                                        const Comp* __restrict__ pack,
                                                        const WorkItem* __restrict__ items,
                                                        unsigned n_items,
                                                        unsigned* __restrict__ counter,
                                                        int* __restrict__ status) {
    const int lane = threadIdx.x & 63;
    const auto* IT = uniform_ptr(items);
    const auto* IN = uniform_ptr(inst);
    for (;;) {
        const unsigned it = next_item(counter);
        if (it >= n_items) break;
        const int64_t row0 = IT[it].row0;
        const int nrows = IT[it].nrows;
        const int ii = IT[it].inst;
        const int64_t n_vis = IN[ii].n_vis;
        const int64_t limit = row0 + nrows < n_vis ? row0 + nrows : n_vis;
        const double* u = IN[ii].u;
        const double* v = IN[ii].v;
        const double* w = IN[ii].w;
        void* out = IN[ii].out;
        const Comp* comp = pack + IN[ii].comp_offset;
        const int n_comp = IN[ii].n_comp;
        const double sgn = IN[ii].sgn;
        const bool f64 = IN[ii].prec == SWV_FP64;
        for (int sub = 0; sub < nrows; sub += 64 * VPL) {
            int64_t j[VPL];
#pragma unroll
            for (int i = 0; i < VPL; ++i) j[i] = row0 + sub + i * 64 + lane;
            if (f64)
                direct_rows_f64<VPL>(j, limit, u, v, w, comp, n_comp, sgn, (double2*)out, status);
            else
                direct_rows_f32c<VPL>(j, limit, u, v, w, comp, n_comp, (float)sgn, (float2*)out,
                                      status);
        }
    }
}

// One row of an instance whose depth J is read per work item (level walker):
// the depths JD, JD - 1, ..., JD - K are compiled with J folded in, as the
// single-tree kernel is, and smaller depths go through the walk of the
// kernel's JMAX with J tested at run time.  J is the same for every lane, so
// the choice is a scalar branch; every path does the same operations in the
// same order.
template <int JD, int K, int JMAX, int LDSL, bool F32>
__device__ __forceinline__ void batch_row_folded(const TRec* rec, int n_roots, int J, LdsPtr lds,
                                                 double U, double V, double W, double& Vr,
                                                 double& Vi) {
    if (J == JD) {
        // a shallower walk needs no more LDS levels than the kernel holds
        constexpr int L = tree_lds_levels<JD, 0, kBatchTreeBlock>();
        static_assert(L <= LDSL, "LDS levels grow with the depth");
        tree_row<JD, 0, L, kBatchTreeBlock, F32, false>(rec, n_roots, JD, lds, U, V, W, Vr, Vi);
    } else if constexpr (K > 0 && JD > 1) {
        batch_row_folded<JD - 1, K - 1, JMAX, LDSL, F32>(rec, n_roots, J, lds, U, V, W, Vr, Vi);
    } else {
        tree_row<JMAX, 0, LDSL, kBatchTreeBlock, F32, false>(rec, n_roots, J, lds, U, V, W, Vr,
                                                             Vi);
    }
}

// Depths below JMAX compiled with J folded in.
constexpr int kBatchFoldedDepths = 3;

// PREC: SWV_FP64 (complex128 out) or SWV_F32C (FP32 leaf phasors, complex64
// out), exactly as the single-instance tree kernel writes them.
template <int JMAX, int WALKER, int PREC, bool PRUNED = false>
__global__ __launch_bounds__(kBatchTreeBlock)
__attribute__((amdgpu_waves_per_eu(tree_waves_per_simd<JMAX, WALKER>()))) void k_batch_tree(
    const BatchInst* __restrict__ inst, const WorkItem* __restrict__ items,
    unsigned n_items, unsigned* __restrict__ counter, int* __restrict__ status) {
    const int lane = threadIdx.x & 63;
    const auto* IT = uniform_ptr(items);
    const auto* IN = uniform_ptr(inst);
    constexpr int LDSL = tree_lds_levels<JMAX, WALKER, kBatchTreeBlock>();
    __shared__ double sums[LDSL > 0 ? LDSL * kSlotDoubles * kBatchTreeBlock : 1];
    for (;;) {
        const unsigned it = next_item(counter);
        if (it >= n_items) break;
        const int64_t row0 = IT[it].row0;
        const int nrows = IT[it].nrows;
        const int ii = IT[it].inst;
        const int64_t n_vis = IN[ii].n_vis;
        const int64_t limit = row0 + nrows < n_vis ? row0 + nrows : n_vis;
        const double* u = IN[ii].u;
        const double* v = IN[ii].v;
        const double* w = IN[ii].w;
        void* out = IN[ii].out;
        const TRec* rec = IN[ii].rec;
        const int n_roots = IN[ii].n_roots, J = IN[ii].J;
        const double s4 = 4.0 * IN[ii].sgn;
        for (int sub = 0; sub < nrows; sub += 64) {
            const int64_t jr = row0 + sub + lane;
            const int64_t j = jr < limit ? jr : limit - 1;
            const double U = u[j], V = v[j], W = w[j];
            double Vr, Vi;
            if constexpr (WALKER == 0 && !PRUNED)
                batch_row_folded<JMAX, kBatchFoldedDepths, JMAX, LDSL, PREC == SWV_F32C>(
                    rec, n_roots, J, (LdsPtr)sums, U, V, W, Vr, Vi);
            else
                tree_row<JMAX, WALKER, LDSL, kBatchTreeBlock, PREC == SWV_F32C, PRUNED>(
                    rec, n_roots, J, (LdsPtr)sums, U, V, W, Vr, Vi);
            if (jr < limit) {
                if (!isfinite(U + V + W)) atomicOr(status, kStatusNonFinite);
                if constexpr (PREC == SWV_F32C)
                    ((float2*)out)[jr] = make_float2((float)Vr, (float)(s4 * Vi));
                else
                    ((double2*)out)[jr] = make_double2(Vr, s4 * Vi);
            }
        }
    }
}

template <int VPL, int BLOCK>
static int direct_occupancy() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_direct<VPL, BLOCK>, BLOCK, 0) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

int batch_direct_blocks_per_cu(int vpl, int block) {
#define SWV_OCC(V, B) if (vpl == V && block == B) return direct_occupancy<V, B>();
    SWV_OCC(1, 64) SWV_OCC(1, 128) SWV_OCC(1, 256)
    SWV_OCC(2, 64) SWV_OCC(2, 128) SWV_OCC(2, 256)
    SWV_OCC(4, 64) SWV_OCC(4, 128) SWV_OCC(4, 256)
#undef SWV_OCC
    return 1;
}

template <int JMAX, int WALKER, int PREC, bool PRUNED = false>
static int tree_occupancy() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_tree<JMAX, WALKER, PREC, PRUNED>,
                                                     kBatchTreeBlock, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

int batch_tree_pruned_blocks_per_cu(int prec) {
    return prec == SWV_F32C ? tree_occupancy<kTreeMaxSeg, 1, SWV_F32C, true>()
                            : tree_occupancy<kTreeMaxSeg, 1, SWV_FP64, true>();
}

// Instantiates X(depth, walker) for every compiled traversal.
#define SWV_TREE_SHAPES(X)                                                            \
    X(1, 0) X(2, 0) X(3, 0) X(4, 0) X(5, 0) X(6, 0) X(7, 0) X(8, 0) X(9, 0) X(10, 0)  \
    X(1, 1) X(2, 1) X(3, 1) X(4, 1) X(5, 1) X(6, 1) X(7, 1) X(8, 1) X(9, 1) X(10, 1)  \
    X(11, 1) X(12, 1) X(13, 1) X(14, 1) X(15, 1) X(16, 1)

int batch_tree_blocks_per_cu(int walker, int depth, int prec) {
#define SWV_OCC_T(D, W)                                                                  \
    if (walker == W && depth == D)                                                       \
        return prec == SWV_F32C ? tree_occupancy<D, W, SWV_F32C>() : tree_occupancy<D, W, SWV_FP64>();
    SWV_TREE_SHAPES(SWV_OCC_T)
#undef SWV_OCC_T
    return 1;
}

hipError_t launch_batch_direct(hipStream_t s, int vpl, int block, int grid,
                               const BatchInst* inst, const Comp* pack, const WorkItem* items,
                               unsigned n_items, unsigned* counter, int* status) {
    if (n_items == 0) return hipSuccess;
#define SWV_RUN(V, B)                                                                     \
    if (vpl == V && block == B) {                                                         \
        k_batch_direct<V, B><<<dim3(grid), dim3(B), 0, s>>>(inst, pack, items, n_items,    \
                                                            counter, status);             \
        return hipGetLastError();                                                         \
    }
    SWV_RUN(1, 64) SWV_RUN(1, 128) SWV_RUN(1, 256)
    SWV_RUN(2, 64) SWV_RUN(2, 128) SWV_RUN(2, 256)
    SWV_RUN(4, 64) SWV_RUN(4, 128) SWV_RUN(4, 256)
#undef SWV_RUN
    return hipErrorInvalidValue;
}

hipError_t launch_batch_tree(hipStream_t s, int walker, int depth, int prec, int grid,
                             const BatchInst* inst,
                             const WorkItem* items, unsigned n_items, unsigned* counter,
                             int* status, bool pruned) {
    if (n_items == 0) return hipSuccess;
    const dim3 g(grid), b(kBatchTreeBlock);
    if (pruned) {
        if (walker != 1 || depth != kTreeMaxSeg) return hipErrorInvalidValue;
        if (prec == SWV_F32C)
            k_batch_tree<kTreeMaxSeg, 1, SWV_F32C, true><<<g, b, 0, s>>>(inst, items, n_items,
                                                                       counter, status);
        else
            k_batch_tree<kTreeMaxSeg, 1, SWV_FP64, true><<<g, b, 0, s>>>(inst, items, n_items,
                                                                       counter, status);
        return hipGetLastError();
    }
#define SWV_RUN_T(D, W)                                                                    \
    if (walker == W && depth == D) {                                                       \
        if (prec == SWV_F32C)                                                              \
            k_batch_tree<D, W, SWV_F32C><<<g, b, 0, s>>>(inst, items, n_items,     \
                                                         counter, status);                 \
        else                                                                               \
            k_batch_tree<D, W, SWV_FP64><<<g, b, 0, s>>>(inst, items, n_items,     \
                                                         counter, status);                 \
        return hipGetLastError();                                                          \
    }
    SWV_TREE_SHAPES(SWV_RUN_T)
#undef SWV_RUN_T
    return hipErrorInvalidValue;
}

#undef SWV_TREE_SHAPES

}  // namespace swv
