// The tree route in the precision form (FP64 phase, FP32 leaf phasors), in a
// translation unit of its own so that the two precisions compile in parallel.
#include "tree_kernel.h"

namespace swv {

hipError_t launch_tree_f32c(hipStream_t s, int walker, int block, const TreeArgs& t,
                            int64_t n_vis, const double* u, const double* v, const double* w,
                            int sign, void* out, int* status) {
    return launch_tree_prec<SWV_F32C>(s, walker, block, t, n_vis, u, v, w, sign, out, status);
}

}  // namespace swv
