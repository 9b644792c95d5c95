// Kernel instantiations for d = 3, N = 1..3.
#include "adg_kernels_impl.h"

namespace adg {

const Ops *ops_3d(int N) {
    static const Ops ops[3] = {make_ops<3, 1>(), make_ops<3, 2>(), make_ops<3, 3>()};
    return (N >= 1 && N <= 3) ? &ops[N - 1] : nullptr;
}

}  // namespace adg
