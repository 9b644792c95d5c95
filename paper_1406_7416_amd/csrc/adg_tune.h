// Compile-time tile parameters per (d, N, working precision).  The defaults below are
// overridden per class by the generated header <adg_tuning.h> when the build provides it:
// build.py writes it from paper_1406_7416_amd/tuning.json, which the offline sweep
// (paper_1406_7416_amd/tune.py) fills with the fastest measured values.
#pragma once

namespace adg {

template <int DIM, int N, bool F32>
struct TuneDefault {
    // predictor: thread budget of a workgroup (cells per block = pred_tb / n^d) and the
    // waves per SIMD its register budget is held to
    static constexpr int pred_tb = 256;
    static constexpr int pred_wps = F32 ? 4 : 2;
    // corrector + detection: cells per workgroup while a cell has at most 128 subcells
    static constexpr int corr_cpb = 4;
    // subcell recompute: workgroups per CU (= waves per SIMD of its 256-thread workgroups)
    static constexpr int sub_wps = (DIM == 2 && N <= 5) ? 3 : 2;
};

template <int DIM, int N, bool F32>
struct Tune : TuneDefault<DIM, N, F32> {};

}  // namespace adg

#if __has_include(<adg_tuning.h>)
#include <adg_tuning.h>
#endif
