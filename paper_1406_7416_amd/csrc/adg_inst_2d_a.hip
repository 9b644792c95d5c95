// Kernel instantiations for d = 2, N = 1..3.
#include "adg_kernels_impl.h"

namespace adg {

const Ops *ops_2d_a(int N) {
    static const Ops ops[3] = {make_ops<2, 1>(), make_ops<2, 2>(), make_ops<2, 3>()};
    return (N >= 1 && N <= 3) ? &ops[N - 1] : nullptr;
}

}  // namespace adg
