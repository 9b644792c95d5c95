// Kernel instantiations for d = 3, N = 9 (large cells: per-cell arrays in global slots).
#include "adg_kernels_impl.h"

namespace adg {

const Ops *ops_3d_9(int N) {
    static const Ops ops = make_ops<3, 9>();
    return N == 9 ? &ops : nullptr;
}

}  // namespace adg
