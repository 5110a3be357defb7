// Host-side launchers of the gfx950 kernels (internal to libswvis).
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace swv {

// Reads through the constant address space: a wave-uniform index then
// compiles to a scalar (SMEM) load whose result lands in SGPRs and feeds
// every lane's arithmetic for free.  Only for memory no kernel writes while
// the reading kernel runs.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* uniform_ptr(const T* p) {
    return (const __attribute__((address_space(4))) T*)p;
}

// Tile shapes compiled for each kernel family.
constexpr int kPerLaneOptions[3] = {1, 2, 4};
constexpr int kBlockOptions[3] = {64, 128, 256};

hipError_t launch_ingest(hipStream_t s, int64_t n, const double* l, const double* m,
                         const double* flux, Comp* out, int* status);

hipError_t launch_direct(hipStream_t s, int prec, int vpl, int block, int64_t n_vis,
                         const double* u, const double* v, const double* w, const Comp* comp,
                         int64_t n_comp, int sign, void* out, int* status);

struct TreeArgs {
    const TRec* rec;
    int n_roots;
    int J;
    int seg_depth;                    // 1 + most branching nodes on a root-to-leaf path
    int pruned;                       // leaves above level J (coefficient thresholding)
};

// Largest J of the level walker (one state set per level) in the single-tree
// kernel, and in the batched and cycle kernels; beyond them the branch walker,
// whose state follows the branching depth.
constexpr int kTreeMaxJ = 16;
constexpr int kBatchTreeMaxJ = 10;
// Depth up to which the single-tree kernel takes the level walker for every
// tree; above it (up to kTreeMaxJ) only for trees in which at most three in
// four internal nodes have a single child.
constexpr int kTreeLevelAlwaysJ = 10;
// Largest segment depth of the branch walker (one register set per branching
// node); it serves every J.
constexpr int kTreeMaxSeg = 16;
// The traversals address a record stream by 32-bit byte offsets.
constexpr size_t kMaxRecordBytes = 0xFFFFFFE0u;

// walker 0: level walker (t.J <= kTreeMaxJ); 1: branch walker
// (t.seg_depth <= kTreeMaxSeg).  prec SWV_FP64 (complex128 out) or SWV_F32C
// (FP32 leaf phasors, complex64 out).  A thresholded tree (t.pruned) runs the
// traversals compiled for leaves above level J, at 64-thread blocks.
hipError_t launch_tree(hipStream_t s, int walker, int block, int prec, const TreeArgs& t,
                       int64_t n_vis, const double* u, const double* v, const double* w,
                       int sign, void* out, int* status);

hipError_t launch_adjoint(hipStream_t s, int prec, int ppl, int block, int64_t chunk,
                          int64_t n_vis, const double* u, const double* v, const double* w,
                          const void* y, int64_t n_pix, const double* l, const double* m,
                          const double* nm1, int sign, void* partial, void* out);

// Resident blocks per compute unit of the adjoint and gradient kernels.
int adjoint_blocks_per_cu(int prec, int ppl, int block);
// Gradient kernel block (128 .. 1024 threads, the smallest that holds every
// component at cpl per lane, else 1024) and the component tiles it leaves.
void grad_tiling(int cpl, int64_t n_comp, int* block, int64_t* tiles);
int grad_blocks_per_cu(int cpl, int block);

// n_comp_dev (optional): the actual component count on the device, at most
// n_comp, which then only sizes the grid (see k_grad_partial).
hipError_t launch_grad(hipStream_t s, int cpl, int64_t chunk, int64_t n_vis, const double* u,
                       const double* v, const double* w, const void* y, const Comp* comp,
                       int64_t n_comp, int sign, double alpha, double* partial, double* d_flux,
                       double* d_l, double* d_m, const int* n_comp_dev = nullptr);

hipError_t launch_residual(hipStream_t s, int64_t n_vis, const void* obs, const void* model,
                           double inv_sigma2, void* resid, double* partial, double* chi2);

// Number of blocks launch_residual uses (its partial buffer holds that many doubles).
int residual_blocks(int64_t n_vis);

// ------------------------------------------------------------ batched --
// One prediction instance as the persistent kernels read it.
struct BatchInst {
    const double* u;
    const double* v;
    const double* w;
    void* out;
    const double* l;      // direct: caller's components, packed by the batched ingest
    const double* m;
    const double* flux;
    const TRec* rec;      // tree: record stream on the device
    int64_t n_vis;
    int64_t comp_offset;  // direct: first packed component of this instance
    int n_comp;
    int n_roots;
    int J;
    int prec;
    double sgn;
};

// A tile of rows [row0, row0 + nrows) of one instance.
struct WorkItem {
    int64_t row0;
    int inst;
    int nrows;
};

hipError_t launch_batch_ingest(hipStream_t s, const BatchInst* inst, int n_inst, int max_comp,
                               Comp* pack, int* status);
hipError_t launch_reset_counters(hipStream_t s, unsigned* counters, int n);
// Blocks per CU that stay resident for the persistent kernels.
int batch_direct_blocks_per_cu(int vpl, int block);
// walker / depth as for launch_tree: depth is the largest J (walker 0) or
// segment depth (walker 1) over the plan's trees.
int batch_tree_blocks_per_cu(int walker, int depth, int prec);
hipError_t launch_batch_direct(hipStream_t s, int vpl, int block, int grid,
                               const BatchInst* inst, const Comp* pack, const WorkItem* items,
                               unsigned n_items, unsigned* counter, int* status);
// prec: the precision of every instance the work items refer to.  pruned: some
// tree holds leaves above level J; only the branch walker at depth kTreeMaxSeg
// is compiled for that.
hipError_t launch_batch_tree(hipStream_t s, int walker, int depth, int prec, int grid,
                             const BatchInst* inst, const WorkItem* items,
                             unsigned n_items, unsigned* counter, int* status,
                             bool pruned = false);
int batch_tree_pruned_blocks_per_cu(int prec);
constexpr int kBatchTreeBlock = 64;

}  // namespace swv
