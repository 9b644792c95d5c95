// Dispatch of the step's kernels over the (d, N) instantiations, and the launches that do
// not depend on (d, N).
#include "adg_kernels_impl.h"

namespace adg {

static const Ops *ops_for(int dim, int N) {
    if (dim == 2 && N >= 1 && N <= 3) return ops_2d_a(N);
    if (dim == 2 && N >= 4 && N <= 5) return ops_2d_b(N);
    if (dim == 2 && N >= 6 && N <= 7) return ops_2d_c(N);
    if (dim == 2 && N >= 8 && N <= 9) return ops_2d_d(N);
    if (dim == 3 && N >= 1 && N <= 3) return ops_3d(N);
    if (dim == 3 && N == 9) return ops_3d_9(N);
    return nullptr;
}

bool supported(int dim, int N) { return ops_for(dim, N) != nullptr; }
int64_t big_slot_doubles(int dim, int N) { return ops_for(dim, N)->big_slot; }
int positions_per_cell(int dim, int N) { return ops_for(dim, N)->npos; }
int subcell_workgroups(int dim, int N, int precision) {
    return ops_for(dim, N)->sub_wgs[precision != ADG_FP64 ? 1 : 0];
}

void launch_bounds(const StepCtx &C) { ops_for(C.P.dim, C.P.N)->bounds(C); }
void launch_predictor(const StepCtx &C) { ops_for(C.P.dim, C.P.N)->predictor(C); }
void launch_faces(const StepCtx &C) { ops_for(C.P.dim, C.P.N)->faces(C); }
void launch_corrector_detect(const StepCtx &C) { ops_for(C.P.dim, C.P.N)->corrector_detect(C); }
void launch_compact(const StepCtx &C) {
    const int nblk = (int)((C.P.ncell + CBS - 1) / CBS);
    hipLaunchKernelGGL(k_compact_count, dim3(nblk), dim3(CBS), 0, C.stream, C.P, C.B, C.capacity);
    hipLaunchKernelGGL(k_compact_scatter, dim3(nblk), dim3(CBS), 0, C.stream, C.P, C.B, C.capacity);
}
void launch_subcell(const StepCtx &C, int redo) { ops_for(C.P.dim, C.P.N)->subcell(C, redo); }
void launch_fluxcorr(const StepCtx &C, int count, int advance) {
    ops_for(C.P.dim, C.P.N)->fluxcorr(C, count, advance);
}
void launch_lambda(const StepCtx &C, const double *u, double factor) {
    ops_for(C.P.dim, C.P.N)->lambda(C, u, factor);
}
int64_t stage_blocks(int stage, const Prob &P, int precision, int64_t *kb1, int64_t *kb2) {
    if (stage == BSTAGE_COMPACT) return (P.ncell + CBS - 1) / CBS;
    return ops_for(P.dim, P.N)->blocks(stage, P, precision, kb1, kb2);
}
void launch_batched(int dim, int N, int stage, const BatchLaunch &L) { ops_for(dim, N)->batched(stage, L); }
void predictor_args(const StepCtx &C, PredArgs<float> *pf, PredArgs<double> *pd) {
    ops_for(C.P.dim, C.P.N)->pred_args(C, pf, pd);
}
void launch_set_scalar(const StepCtx &C, int idx, double val) {
    hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, C.stream, C.B.scal, idx, val);
}
__global__ void k_copy_scalar(const double *src, double *dst) { dst[0] = src[0]; }
void launch_copy_scalar(const double *src, double *dst, hipStream_t stream) {
    hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, stream, src, dst);
}
void launch_advance_time(const StepCtx &C) {
    hipLaunchKernelGGL(k_advance_time, dim3(1), dim3(1), 0, C.stream, C.B.scal);
}

}  // namespace adg
