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
    int precision;         // ADG_FP64, ADG_MIXED or ADG_MIXED_DEV
    int ring_only;         // bounds pass over the ghost ring only
    int64_t nring;         // ghost-ring cells
    int subcell_grid;      // workgroups (= scratch slots) of the subcell recompute
    int mood;              // MOOD layer after the subcell scheme
};

// Scratch of the subcell scheme, one slot per workgroup (sidx): reconstructed nodal values,
// predictor traces, the 3D halo and the per-point boundary fluxes.
struct SubScratch {
    double *Y, *strace, *halo, *fpts;
    double *big;           // large cells: slots of the update's sub-face fluxes and subcell arrays
};

// Workgroups (= global scratch slots) of the kernels of large cells, whose per-cell arrays
// exceed the LDS of a CU and live in a slot of global memory instead (3D, N = 9).
constexpr int BIG_WG = 512;

// Stages of one step in a batch, each one batched launch (or a few) per (d, N) class.
enum {
    BSTAGE_DT = 0,         // wave speed reduction and dt (eq. (cfl))
    BSTAGE_BOUNDS,         // old-time bounds of the ghost ring
    BSTAGE_PREDICTOR,      // predictor + volume term + face traces
    BSTAGE_FACE,           // face fluxes
    BSTAGE_CORRECTOR,      // corrector + scatter + detection
    BSTAGE_COMPACT,        // compaction + the class's global worklist offsets
    BSTAGE_SUBCELL,        // subcell ADER-WENO3 over the global troubled worklist (+ MOOD layer)
    BSTAGE_FLUXCORR,       // flux correction over the global list of corrected neighbours
    BSTAGE_ADVANCE,        // t += dt
    BSTAGE_COUNT
};

// One (d, N) class of a batch at one buffer parity (device pointers).
struct BatchLaunch {
    const Tables *T;       // the class's operator tables (they depend on (N, Ns) only)
    const BatchEntry *E;
    int np;
    const BTile *t_lambda, *t_bounds, *t_pred, *t_face, *t_corr, *t_compact;
    int n_lambda, n_bounds, n_pred, n_face, n_corr, n_compact;
    int *off_t, *off_c;    // np + 1 each: global troubled / corrected worklist offsets
    SubScratch S;          // sub_grid scratch slots for the subcell scheme
    int sub_grid, fc_grid;
    int precision, mood;
    hipStream_t stream;
};

bool supported(int dim, int N);
// doubles per global scratch slot of a large-cell class (0: the class works in LDS)
int64_t big_slot_doubles(int dim, int N);
int positions_per_cell(int dim, int N);
// workgroups (= scratch slots) of the persistent subcell launch that fill MI355X's 256 CUs
int subcell_workgroups(int dim, int N, int precision);
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
// blocks of one problem's launch of a batch stage (predictor, face, corrector, compaction)
int64_t stage_blocks(int stage, const Prob &P, int precision, int64_t *kb1, int64_t *kb2);
void launch_batched(int dim, int N, int stage, const BatchLaunch &L);
// the predictor's launch arguments of C in both precisions (batch entries)
void predictor_args(const StepCtx &C, PredArgs<float> *pf, PredArgs<double> *pd);

}  // namespace adg
