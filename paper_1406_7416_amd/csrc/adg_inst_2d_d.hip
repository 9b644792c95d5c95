// Kernel instantiations for d = 2, N = 8..9.
#include "adg_kernels_impl.h"

namespace adg {

const Ops *ops_2d_d(int N) {
    static const Ops ops[2] = {make_ops<2, 8>(), make_ops<2, 9>()};
    return (N >= 8 && N <= 9) ? &ops[N - 8] : nullptr;
}

}  // namespace adg
