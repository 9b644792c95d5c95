/*
 * adg.h -- C ABI of the MI355X (gfx950) ADER-DG step with the a-posteriori subcell
 * limiter for the compressible Euler equations on uniform Cartesian grids.
 *
 * Method: Dumbser, Zanotti, Loubere, Diot, "A posteriori subcell limiting of the
 * discontinuous Galerkin finite element method for hyperbolic conservation laws",
 * J. Comput. Phys. 2014 (arXiv 1406.7416).  One call of adg_step performs the five
 * steps of Sec. 4.4: unlimited ADER-DG candidate (Sec. 2.2 predictor eq. (pde.nc.dg2),
 * Sec. 2.3 corrector eq. (pde.nc.gw2) with the Rusanov flux), scatter onto Ns^d
 * subcells (eq. (subcell.p)), detection by PAD + relaxed DMP (eqs. (positivity),
 * (relax), (dmp)), subcell ADER-WENO3 recompute of troubled cells (eqs. (aderweno),
 * (ader.icbc)) with flux correction of their unlimited neighbours, and gather
 * (eq. (subcell.r)).
 *
 * Conventions
 *  - Every function returns ADG_OK (0) or a negative error code; adg_last_error()
 *    gives a thread-local message for the last failure.  Nothing throws or exits.
 *  - State layout (device or host, double): [var][cell][node] with var = (rho, rho u,
 *    rho v, [rho w], rho E); cells row-major with x fastest; nodes the tensor
 *    Gauss-Legendre points of the cell (N+1 per axis), x fastest.  Nodal values are the
 *    DG degrees of freedom (Sec. 2.1).
 *  - Subcell layout: [var][cell][subcell], Ns per axis, x fastest.
 *  - Memory: the caller owns all device memory and the stream.  adg_workspace_bytes
 *    says how much one problem needs; adg_bind hands in one device allocation of at
 *    least that size (256-byte aligned) and a hipStream_t.  The library keeps only host
 *    tables and the plan; adg_destroy frees host memory only.
 *  - Calls on one problem are not thread-safe; work is enqueued on the bound stream.
 *    Functions marked "synchronising" wait for that stream.
 */
#ifndef ADG_H
#define ADG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ADG_OK = 0,
    ADG_EINVAL = -1,      /* bad argument or unsupported configuration */
    ADG_ENOMEM = -2,      /* host allocation failed or workspace too small */
    ADG_EDEVICE = -3,     /* a HIP call failed (message names it) */
    ADG_ECAPACITY = -4,   /* more troubled cells than the subcell pool holds */
    ADG_ENONPHYSICAL = -5,/* a subcell recompute produced rho <= 0 or p <= 0 (count via stats) */
    ADG_ESTATE = -6       /* call order (e.g. step before bind/set_state) */
};

enum { ADG_PERIODIC = 0, ADG_TRANSMISSIVE = 1, ADG_REFLECTIVE = 2, ADG_DIRICHLET = 3 };
/* Precision forms.  ADG_FP64: every operation in FP64.  ADG_MIXED: the predictor, its volume
 * term and traces, the face fluxes and face increments, and the subcell scheme's
 * reconstruction, predictor and sub-face fluxes in FP32; the state, the update additions,
 * projection/reconstruction, detection, time step and the subcell halo and update in FP64.
 * ADG_MIXED_DEV: as ADG_MIXED, with the predictor, traces and face fluxes carried as
 * deviations from each cell's reference state (its first nodal value of u^n rounded to FP32)
 * and the fluxes evaluated as F(c + dq) - F(c) in a form whose terms all have the size of dq,
 * so that FP32 rounding is relative to the deviation rather than to the state (for smooth
 * flows, where the mixed form's error would otherwise not fall with the mesh size);
 * Rusanov flux only. */
enum { ADG_FP64 = 0, ADG_MIXED = 1, ADG_MIXED_DEV = 2 };

/* One side of one axis.  Where the coordinate along split_axis is below
 * split0 + split_speed * t, (kind[0], state[0]) applies, else (kind[1], state[1]);
 * split_axis = -1: no split.  States are conserved variables (unused entries ignored).
 * Ghost states (the paper names its boundary conditions without formulas): transmissive
 * copies the interior state, reflective negates the normal momentum, Dirichlet takes
 * the prescribed state; subcell ghosts mirror the interior subcells first.  Periodic
 * must be set on both sides of an axis. */
typedef struct {
    int kind[2];
    int split_axis;
    double split0, split_speed;
    double state[2][5];
} adg_bc;

/* Uniform Cartesian grid on [lo, hi] with n[k] cells along axis k (k < dim). */
typedef struct {
    int dim;              /* 2 or 3 */
    int64_t n[3];
    double lo[3], hi[3];
    adg_bc bc[3][2];      /* [axis][0: low side, 1: high side] */
} adg_grid_desc;

typedef struct {
    int Ns;               /* subcells per axis; 0 -> 2N+1.  Sec. 4.5 allows any Ns >= N+1 and shows 2N+1
                             to be the optimum (the subgrid FV scheme is then stable at the DG time step
                             of eq. (cfl) and resolves as finely as the DG polynomial); the kernels are
                             specialised at compile time on Ns = 2N+1, so any other value gives
                             ADG_EINVAL */
    int picard_iters;     /* 0 -> N+1 sweeps of the predictor (reading: fixed count) */
    int precision;        /* ADG_FP64, ADG_MIXED or ADG_MIXED_DEV */
    int limiter;          /* 1: subcell limiter on (default), 0: unlimited ADER-DG */
    double eps;           /* eq. (relax) epsilon; 0 -> 1e-3 */
    double delta0;        /* absolute floor of delta; 0 -> 1e-4 (reading: not in the paper) */
    int64_t pool_capacity;/* troubled cells the subcell pool holds; 0 -> all cells */
    int mood;             /* 1: one more MOOD layer after the subcell WENO3 scheme (Sec. 6, Fig.
                             algo2): subcells whose WENO3 result fails PAD or the relaxed DMP
                             against their cell's bounds get the first-order flux of the subcell
                             averages on all their sub-faces (reading); 0: off (default) */
    int flux;             /* numerical flux at element faces and sub-faces (Sec. 2.3): 0 Rusanov
                             (default), 1 Osher-type in the universal form (straight path, 3-point
                             Gauss-Legendre, |A| from the Euler eigen-split; reading); the
                             first-order fallbacks of the subcell scheme stay Rusanov */
} adg_params;

typedef struct adg_problem adg_problem;

const char *adg_last_error(void);

/* Creates a problem (host side only).  N in 1..9 for dim 2; 1..3 and 9 for dim 3 (the
 * degrees of the paper's 3D runs; at N = 9, 19^3 subcells per cell, the per-cell arrays of the
 * corrector, bounds, subcell and flux-correction kernels live in 512 per-workgroup slots of
 * about 1.4 MB of the workspace instead of LDS); gamma > 1.  p may be NULL for defaults.
 * Errors: ADG_EINVAL (other degrees included). */
int adg_create(const adg_grid_desc *g, int N, double gamma, const adg_params *p, adg_problem **out);
int adg_destroy(adg_problem *pb);

/* Bytes of device workspace (including the state) this problem needs. */
size_t adg_workspace_bytes(const adg_problem *pb);

/* Binds a caller-owned device allocation (>= adg_workspace_bytes, 256-byte aligned) and
 * a hipStream_t (NULL: the null stream), uploads the operator tables.  The DG state is
 * part of this one allocation (two copies, current and next, swapped by every step), so
 * there is no separate state argument: adg_state_device_ptr gives the current copy in
 * place, adg_set_state / adg_get_state copy from and to caller buffers.  Errors:
 * ADG_ENOMEM (too small), ADG_EDEVICE. */
int adg_bind(adg_problem *pb, void *dev_workspace, size_t bytes, void *hip_stream);

/* Device address of the current DG state inside the workspace (state layout above),
 * valid until the next step or adg_set_state; read it on the bound stream.  Errors:
 * ADG_EINVAL, ADG_ESTATE (no state). */
int adg_state_device_ptr(const adg_problem *pb, const double **u);

/* Physical coordinates along `axis` of the points where initial data is sampled:
 * m = 0: the DG nodes, out[(i*(N+1) + a)] for cell i, node a;
 * m > 0: m-point Gauss-Legendre points of every subcell, out[(i*Ns + s)*m + q].
 * Host memory, n[axis]*(N+1) or n[axis]*Ns*m doubles. */
int adg_axis_points(const adg_problem *pb, int axis, int m, double *out);

/* Host-side projection of samples taken on the tensor grid of adg_axis_points(m):
 * samples[var][z][y][x].  m = 0: nodal interpolation (u only).  m > 0: L2 projection
 * onto the DG basis by the composite m-point rule on every subcell, and (if v != NULL)
 * the subcell averages of the samples.  u, v: host, state / subcell layouts.  Runs on
 * host threads (OMP_NUM_THREADS if set, else the hardware's, at most 16). */
int adg_project_samples(const adg_problem *pb, const double *samples, int m, double *u, double *v);

/* Sets the DG state u (layout above; device pointer if on_device, else host) and time 0.
 * If v_exact (host, subcell layout) is given, applies the initial detection of Sec. 4.4:
 * PAD + DMP of P(u) against the bounds of v_exact over each cell's neighbourhood;
 * troubled cells start from v_exact and u := R(v_exact).  The detection runs on host
 * threads like adg_project_samples; the pool must hold every cell it flags
 * (ADG_ECAPACITY otherwise).  Synchronising. */
int adg_set_state(adg_problem *pb, const double *u, int on_device, const double *v_exact);

/* Masked geometry (Sec. 5, forward-facing step: a rectangle is removed from the domain and
 * its faces are reflective walls).  mask: host, one byte per cell (x fastest), nonzero =
 * solid; NULL removes the mask.  A solid cell keeps whatever state adg_set_state gave it,
 * is never updated, troubled or corrected and takes no part in the time step; a face
 * between a fluid and a solid cell is a reflective wall for the DG face fluxes and for the
 * subcell scheme's sub-faces.  Where the subcell halo or the neighbourhood bounds V_i of
 * eq. (dmp) reach a solid cell, it holds the mirror image of the fluid across its walls:
 * along each axis with a fluid face neighbour (the lower one if both are fluid) the
 * neighbour's subcells, reversed along that axis with that axis's momentum negated (at a
 * convex corner of the obstacle, mirrored along both axes).  Call it before
 * adg_set_state (whose initial detection uses it); it may be called before or after
 * adg_bind.  Errors: ADG_EINVAL (every cell solid), ADG_ESTATE (the problem belongs to a
 * batch), ADG_EDEVICE.  Synchronising when bound. */
int adg_set_mask(adg_problem *pb, const uint8_t *mask);

/* Copies the DG state out (device pointer if to_device).  Synchronising for host copies. */
int adg_get_state(const adg_problem *pb, double *u, int to_device);

/* Eq. (cfl): dt = cfl * min_k h_k / (d (2N+1) max |v_k| + c) from the current state.
 * Synchronising. */
int adg_cfl_dt(adg_problem *pb, double cfl, double *dt_out);

/* One full step with the given dt, enqueued on the bound stream without any host wait
 * (the troubled-cell count stays on the device).  Errors: ADG_ESTATE (no state, or the
 * problem belongs to a batch), ADG_EDEVICE; ADG_ECAPACITY once an earlier step found more
 * troubled cells than the pool holds (detected asynchronously; the state is then not
 * advanced correctly; sticky until the next adg_set_state).
 * ADG_ENONPHYSICAL is a warning, not a failure: this step was enqueued normally, and the
 * counter of subcell ADER-WENO3 results that fail the positivity test of eq. (positivity)
 * (Sec. 6 notes that the WENO3 scheme need not preserve positivity) has risen since the last
 * report, as read from the asynchronous counter copy of an earlier step; the count is in
 * adg_get_stats. */
int adg_step(adg_problem *pb, double dt);

/* As adg_step with dt from eq. (cfl) computed on the device from the current state. */
int adg_step_cfl(adg_problem *pb, double cfl);

/* Current time (synchronising). */
int adg_time(const adg_problem *pb, double *t);

/* Troubled-cell map of the last step (or of the initial detection): the flag
 * beta_i^{n+1} of Sec. 4.4 (step 3 of the five), 1 byte per cell, host memory;
 * *count = number of troubled cells.  Synchronising. */
int adg_get_troubled(const adg_problem *pb, uint8_t *beta, int64_t *count);

/* Signed normalised detection margin per cell of the last detection (Sec. 4.3: the
 * smallest slack of the candidate's subcell averages to the relaxed DMP bounds of eqs.
 * (dmp), (relax) and to the positivity thresholds of eq. (positivity), each divided by
 * the variable's scale; negative: a test failed).  Host memory, float per cell.
 * Synchronising. */
int adg_get_margin(const adg_problem *pb, float *margin);

/* Subcell data v_h of troubled cells, the alternative representation that Sec. 4.4 stores
 * only in troubled cells (the result of the subcell scheme, eq. (aderweno)) and that
 * eq. (ader.icbc) takes as the next step's data there (subcell layout, host; entries of
 * untroubled cells are left untouched).  Synchronising. */
int adg_get_subcells(const adg_problem *pb, double *v);

/* Statistics of the last step: out[0] troubled cells, out[1] corrected neighbours,
 * out[2] cumulative subcell results failing PAD, out[3] steps taken.  Synchronising. */
int adg_get_stats(const adg_problem *pb, int64_t *out4);

/* MOOD layer of the last step (adg_params.mood): subcells whose WENO3 result failed the
 * detection, and troubled cells recomputed.  Synchronising. */
int adg_get_mood_stats(const adg_problem *pb, int64_t *flagged, int64_t *redone);

/* Per-kernel timing with hipEvents recorded on the bound stream around each kernel
 * group.  Groups: 0 old-time bounds, 1 predictor, 2 face fluxes, 3 corrector + detection,
 * 4 compaction, 5 subcell ADER-WENO3, 6 flux correction, 7 time-step reduction.
 * adg_profile(pb, mask) clears the totals and times the groups whose bit is set in mask
 * (bit g: group g; 0xFF: all; each timed group adds two event records per step);
 * adg_profile(pb, 0) stops.  adg_profile_read fills ms[g] (total milliseconds) and
 * launches[g] for g < ngroups (<= 8).  Synchronising. */
int adg_profile(adg_problem *pb, int enable);
int adg_profile_read(adg_problem *pb, double *ms, int64_t *launches, int ngroups);

/* Batching of independent problems (not in the paper): the problems (each created and
 * bound as above, with a state set, all on the current device, none in another batch,
 * sharing precision, limiter and MOOD layer; grids, degrees, boundaries, flux and Picard
 * sweeps may differ; 3D problems of degree 9 are refused with ADG_EINVAL: they are stepped
 * one by one) advance together; while the batch exists they are not stepped or set on their
 * own (adg_step, adg_step_cfl, adg_set_state return ADG_ESTATE).
 * The problems are grouped into classes of equal (dim, N).  Every stage of the step is one
 * launch per class over all its problems: a tile table maps each workgroup to (problem,
 * block of that problem's own grid) for the time step, ghost-ring bounds, predictor, face
 * fluxes, corrector + detection and compaction; the subcell ADER-WENO3 recompute and the
 * flux correction run over one global worklist per class (the troubled cells, resp. their
 * corrected neighbours, of all its problems, from per-problem offsets computed on the
 * device after the compaction).  Each problem's arithmetic is that of its own step, so
 * the batch is bitwise equal to stepping the problems one by one.
 * adg_batch_workspace_bytes / adg_batch_bind: the batch's device memory (launch tables of
 * both buffer parities, worklist offsets, the subcell scratch of each class: about 0.1-0.2
 * GB per 2D class with N <= 5), owned by the caller, 256-byte aligned, and the caller's
 * stream (NULL: the null stream), whose pending work each batch step waits for; the batch
 * captures and replays on a stream of its own (created by adg_batch_create).
 * adg_batch_step_cfl: the first call (or a call with another cfl) takes one ordinary step
 * per problem, then captures one step of every problem (dt from eq. (cfl) per problem, on
 * the device; stage after stage, the classes one after another) into two hipGraphs (the two
 * buffer parities) and from then on replays them: one hipGraphLaunch per batch step.  Synchronises the batch stream before returning.
 * Errors: ADG_EINVAL, ADG_ESTATE (not bound), ADG_EDEVICE; ADG_ECAPACITY if any problem's
 * troubled cells exceeded its pool capacity (the message names the first such problem);
 * ADG_ENONPHYSICAL (a warning, as for adg_step) if a problem's count of non-physical
 * subcell results rose.
 * adg_batch_profile(b, 1) clears the stage timing; while it is on, each batch step
 * enqueues the graph's launches directly on the batch stream (the same kernels in the same
 * order) with a HIP event before every launch group (stage, class) and one at the end of
 * the step (stages: 0 time step, 1 ghost-ring bounds, 2 predictor, 3 face fluxes,
 * 4 corrector + detection, 5 compaction + worklist offsets, 6 subcell ADER-WENO3 (+ MOOD
 * layer), 7 flux correction, 8 time advance); adg_batch_profile(b, 0) returns to graph
 * replays.  adg_batch_classes returns the number of classes and fills their dim and N (up
 * to max_classes); adg_batch_profile_read fills ms[stage * nclasses + class] (total
 * milliseconds; 9 x nclasses entries) and *steps (timed batch steps).
 * adg_batch_dt: per-problem dt of the last batch step (host memory, count doubles).
 * Synchronising. */
typedef struct adg_batch adg_batch;
int adg_batch_create(adg_problem *const *ps, int count, adg_batch **out);
size_t adg_batch_workspace_bytes(const adg_batch *b);
int adg_batch_bind(adg_batch *b, void *dev_workspace, size_t bytes, void *hip_stream);
int adg_batch_step_cfl(adg_batch *b, double cfl, int nsteps);
int adg_batch_profile(adg_batch *b, int enable);
int adg_batch_classes(const adg_batch *b, int *dims, int *Ns, int max_classes);
int adg_batch_profile_read(adg_batch *b, double *ms, int64_t *steps);
int adg_batch_dt(adg_batch *b, double *dts);
int adg_batch_destroy(adg_batch *b);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops or harnesses that forbid hipMalloc): the time step of adg_cfl_dt for a state the
 * caller holds, computed by the same kernels with no problem handle and no workspace.
 * The reduction's partial maxima and scalars live in a static device array of the library
 * (ADG_STATIC_PARTIALS + 8 doubles, about 8 KB), one per device, held until the process
 * ends; nothing is allocated.
 *   dev_u   device, state layout above: ncell cells of degree N in dim dimensions
 *           (read only; owned by the caller);
 *   gamma   ratio of specific heats; hmin the smallest cell edge; cfl the Courant factor:
 *           dt = cfl * hmin / (dim (2N+1) max over cells, nodes, axes of |v_k| + c);
 *   dev_dt  device, one double, written (owned by the caller);
 *   hip_stream the stream to enqueue on (NULL: the null stream); no host wait.
 * Every call on one device shares that device's array: calls that overlap on one device
 * (different streams or threads) race and must be serialised by the caller.
 * Errors: ADG_EINVAL (null pointer, dim/N not supported, ncell outside
 * 1..ADG_STATIC_MAX_CELLS, gamma <= 1, hmin or cfl <= 0), ADG_EDEVICE. */
#define ADG_STATIC_PARTIALS 1024
#define ADG_STATIC_MAX_CELLS ((int64_t)1 << 34)
int adg_cfl_dt_static(const double *dev_u, int dim, int N, int64_t ncell, double gamma, double hmin, double cfl,
                      double *dev_dt, void *hip_stream);

/* Debug hook: cells with mask[c] != 0 are flagged troubled at every following detection
 * (NULL clears).  Host memory, one byte per cell. */
int adg_debug_force_troubled(adg_problem *pb, const uint8_t *mask);

/* Debug hook for the a-posteriori detection (Sec. 4.3, 4.4): at the next step only, every
 * node of variable var (0..dim+1) of cell's unlimited candidate is set to value (NaN, a
 * negative density, ...) before the detection tests it.  Errors: ADG_EINVAL (cell or var
 * out of range), ADG_ESTATE.  Synchronising. */
int adg_debug_poison(adg_problem *pb, int64_t cell, int var, double value);

#ifdef __cplusplus
}
#endif
#endif
