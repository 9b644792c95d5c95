/*
 * FP64 CPU oracle for one ADER-DG time step with the a-posteriori subcell (MOOD)
 * limiter, after Dumbser, Zanotti, Loubere, Diot, "A posteriori subcell limiting of
 * the discontinuous Galerkin finite element method for hyperbolic conservation laws"
 * (J. Comput. Phys. 2014, arXiv 1406.7416).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or calls
 * this code; only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no source with the GPU library: its own quadrature
 * (Golub-Welsch eigen-solve), its own operator tables, its own loops.
 *
 * Layouts (all arrays are plain host memory owned by the caller unless stated):
 *   state u      [var][cell][node]   var = (rho, rho u, rho v, [rho w], rho E)
 *   cells        row-major, x fastest;  nodes: tensor Gauss-Legendre, x fastest
 *   subcells     [var][cell][subcell], subcell index x fastest (Ns per axis)
 */
#ifndef ADG_ORACLE_H
#define ADG_ORACLE_H
#include <stdint.h>

#define OR_MAXN 10      /* up to N = 9 */
#define OR_MAXNS 32     /* subcells per axis */

enum { OR_PERIODIC = 0, OR_TRANSMISSIVE = 1, OR_REFLECTIVE = 2, OR_DIRICHLET = 3 };

/* One side of one axis.  Where the coordinate along split_axis is below
 * split0 + split_speed * t the pair (kind[0], state[0]) applies, else (kind[1], state[1]).
 * split_axis < 0 means no split: (kind[0], state[0]) everywhere. */
typedef struct {
    int kind[2];
    int split_axis;
    double split0, split_speed;
    double state[2][5];   /* conserved Dirichlet states */
} or_bc;

typedef struct {
    int dim;              /* 2 or 3 */
    int N;                /* polynomial degree, 1..9 */
    int Ns;               /* subcells per axis (>= N+1, >= 3) */
    int picard_iters;     /* Picard sweeps of the local space-time predictor */
    int limiter;          /* 1: a-posteriori subcell limiter on, 0: unlimited ADER-DG */
    int ncell[3];
    double lo[3], hi[3];
    double gamma, eps, delta0;
    or_bc bc[3][2];
    int mood;             /* 1: one more MOOD layer after the subcell WENO3 scheme (first order) */
    int flux;             /* 0: Rusanov, 1: Osher-type (universal form) */
} or_config;

typedef struct or_solver or_solver;

or_solver *or_create(const or_config *c);
void or_destroy(or_solver *s);

/* Reference-element operators for n = N+1 Gauss-Legendre nodes on [0,1]. */
void or_basis(int n, double *xi, double *w, double *D, double *L, double *R, double *Kw);
/* Subcell projection P (Ns x n) and reconstruction R (n x Ns), 1D factors. */
void or_subcell_ops(int N, int Ns, double *P, double *R);

void or_axis_points(const or_solver *s, int axis, int m, double *out);
void or_project(const or_solver *s, const double *samples, int m, double *u, double *v);

int or_set_state(or_solver *s, const double *u, const double *v_exact);
void or_get_state(const or_solver *s, double *u);
void or_get_troubled(const or_solver *s, uint8_t *beta);
void or_get_margin(const or_solver *s, double *margin);
void or_get_subcells(const or_solver *s, double *v);
void or_get_bounds(const or_solver *s, double *bmin, double *bmax);
void or_force_troubled(or_solver *s, const uint8_t *mask);
/* Masked geometry: mask[c] = 1 marks a solid cell (copied; NULL clears).  Set it before
 * or_set_state. */
void or_set_mask(or_solver *s, const uint8_t *mask);
int or_poison(or_solver *s, long cell, int var, double value);
/* MOOD layer of the last step: subcells whose WENO3 candidate failed, cells recomputed. */
void or_mood_stats(const or_solver *s, long *flagged, long *redone);
/* Test entries: numerical flux (0 Rusanov, 1 Osher-type) along axis k, and |A(Q)| dQ. */
void or_numerical_flux(int d, int k, double g, int flux, const double *qL, const double *qR, double *G);
void or_abs_jacobian(int d, int k, double g, const double *Q, const double *dQ, double *out);
double or_time(const or_solver *s);
void or_set_time(or_solver *s, double t);
double or_cfl_dt(const or_solver *s, double cfl);
int or_step(or_solver *s, double dt);
long or_nonphysical(const or_solver *s);
void or_set_threads(int nthreads);
int or_get_threads(void);

/* Pieces exposed for the pin tests. */
void or_predictor(int dim, int N, double gamma, const double *dt_over_h, int iters,
                  const double *u_cell, double *q);
void or_weno3(const double *avg5, double *out3);
void or_exact_riemann(double rl, double ul, double pl, double rr, double ur, double pr,
                      double gamma, const double *s, int m, double *out, double *pstar_ustar);

#endif
