// Launch interface between the C ABI and the kernels.
#pragma once
#include "adg_internal.h"

namespace adg {

struct StepCtx {
    Prob P;
    Bufs B;
    const Tables *tab;     // device copy
    hipStream_t stream;
    int cur;               // index of the current state buffer
    int limiter;
    int picard_iters;
    int64_t capacity;      // pool slots
    int lam_blocks;        // blocks of the lambda reduction
    int precision;         // ADG_FP64 or ADG_MIXED
    int ring_only;         // bounds pass over the ghost ring only
    int64_t nring;         // ghost-ring cells
    int subcell_grid;      // workgroups (= scratch slots) of the subcell recompute
    int mood;              // MOOD layer after the subcell scheme
};

bool supported(int dim, int N);
int positions_per_cell(int dim, int N);
void build_tables(int N, int Ns, Tables *T);
void gl_nodes(int n, double *x01, double *w01);
void lagrange_values(int n, const double *xi, double t, double *phi);

void launch_bounds(const StepCtx &C);
void launch_predictor(const StepCtx &C);
void launch_faces(const StepCtx &C);
void launch_corrector_detect(const StepCtx &C);
void launch_compact(const StepCtx &C);
// redo = 0: the subcell scheme; 1: the MOOD layer's recompute
void launch_subcell(const StepCtx &C, int redo);
// advance != 0: the launch also advances t by dt (the step's last kernel)
void launch_fluxcorr(const StepCtx &C, int count, int advance);
void launch_lambda(const StepCtx &C, const double *u, double factor);
void launch_set_scalar(const StepCtx &C, int idx, double val);
void launch_advance_time(const StepCtx &C);
void launch_copy_scalar(const double *src, double *dst, hipStream_t stream);

}  // namespace adg
