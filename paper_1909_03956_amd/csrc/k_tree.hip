// Wavelet-tree route (section 3.3, Eqs. 14-17; section 3.5) on gfx950: the
// FP64 instantiations and the launch entry for both precisions.  The kernel
// and the traversal it runs are described in tree_kernel.h and tree_walk.h.
#include "tree_kernel.h"

namespace swv {

hipError_t launch_tree_f32c(hipStream_t s, int walker, int block, const TreeArgs& t,
                            int64_t n_vis, const double* u, const double* v, const double* w,
                            int sign, void* out, int* status);

hipError_t launch_tree(hipStream_t s, int walker, int block, int prec, const TreeArgs& t,
                       int64_t n_vis, const double* u, const double* v, const double* w,
                       int sign, void* out, int* status) {
    if (prec == SWV_F32C)
        return launch_tree_f32c(s, walker, block, t, n_vis, u, v, w, sign, out, status);
    return launch_tree_prec<SWV_FP64>(s, walker, block, t, n_vis, u, v, w, sign, out, status);
}

}  // namespace swv
