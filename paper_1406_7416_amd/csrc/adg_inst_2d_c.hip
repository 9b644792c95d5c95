// Kernel instantiations for d = 2, N = 6..7.
#include "adg_kernels_impl.h"

namespace adg {

const Ops *ops_2d_c(int N) {
    static const Ops ops[2] = {make_ops<2, 6>(), make_ops<2, 7>()};
    return (N >= 6 && N <= 7) ? &ops[N - 6] : nullptr;
}

}  // namespace adg
