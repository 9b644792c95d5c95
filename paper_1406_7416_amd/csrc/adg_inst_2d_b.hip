// Kernel instantiations for d = 2, N = 4..5.
#include "adg_kernels_impl.h"

namespace adg {

const Ops *ops_2d_b(int N) {
    static const Ops ops[2] = {make_ops<2, 4>(), make_ops<2, 5>()};
    return (N >= 4 && N <= 5) ? &ops[N - 4] : nullptr;
}

}  // namespace adg
