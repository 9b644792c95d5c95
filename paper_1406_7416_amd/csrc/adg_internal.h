// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "adg.h"
#include "adg_tune.h"

namespace adg {

constexpr int MAXN = 10;     // nodes per axis (N <= 9)
constexpr int MAXNS = 19;    // subcells per axis (2N+1)

// Operator tables, built on the host in FP64 (Newton Gauss-Legendre, barycentric
// Lagrange) and uploaded once per problem.
struct Tables {
    double xi[MAXN], w[MAXN];
    double D[MAXN][MAXN];        // D[a][b] = phi_b'(xi_a)
    double L[MAXN], R[MAXN];     // phi_b(0), phi_b(1)
    double Kw[MAXN][MAXN];       // K1^{-1} diag(w), time operator of the predictor
    double Dvol[MAXN][MAXN];     // w_b D[b][a] / w_a : volume-term operator
    double P[MAXNS][MAXN];       // subcell projection, eq. (subcell.p)
    double Rg[MAXN][MAXNS];      // subcell reconstruction (gather), eq. (subcell.r)
    double Pq[3 * MAXNS][MAXN];  // (w3_g / Ns) phi_a((s + xi3_g) / Ns) / w_a at row s*3+g:
                                 // sub-face quadrature of phi_a over the face weight w_a
    // degree-2 subcell scheme (3 Gauss-Legendre nodes)
    double xi3[3], w3[3];
    double D3[MAXN][MAXN], L3[MAXN], R3[MAXN], Kw3[MAXN][MAXN];
    double weno[3][3][3];        // [stencil][monomial][cell]: averages -> coefficients
    float fweno[3][3][3];        // the same in FP32 (mixed form)
    // Even / odd parts of D on the symmetric nodes, where D[n-1-a][n-1-b] = -D[a][b]:
    //   DE[a][b] = (D[a][b] + D[a][n-1-b]) / 2,  DO[a][b] = (D[a][b] - D[a][n-1-b]) / 2
    // for a, b < n/2; odd n adds DE[a][n/2] = D[a][n/2] and the middle row DO[n/2][b] = D[n/2][b].
    double DE[MAXN / 2][MAXN / 2 + 1], DO[MAXN / 2 + 1][MAXN / 2];
    // FP32 copies for the mixed-precision predictor and face fluxes
    float fD[MAXN][MAXN], fKw[MAXN][MAXN], fDvol[MAXN][MAXN], fL[MAXN], fR[MAXN], fw[MAXN];
    float fDE[MAXN / 2][MAXN / 2 + 1], fDO[MAXN / 2 + 1][MAXN / 2];
    // FP32 copies of the degree-2 subcell operators (mixed form)
    float fD3[3][3], fKw3[3][3], fL3[3], fR3[3], fw3[3], fxi3[3];
};

struct BCDev {
    int kind[2];
    int split_axis;
    double split0, split_speed;
    double state[2][5];
};

// Everything a kernel needs to know about one problem.
struct Prob {
    int dim, N, n, nv, Ns;
    int nc[3];
    int64_t ncell;
    double lo[3], h[3];
    double gamma, eps, delta0;
    BCDev bc[3][2];
    int periodic[3];
    int flux;              // 0 Rusanov, 1 Osher-type
};

// Device buffers of one problem, carved out of the caller's workspace.
struct Bufs {
    Tables *tab;
    double *u[2];          // [v][cell][node] current / next
    double *ext_min[2], *ext_max[2];   // [v][ext cell] per-cell subcell min/max incl. ghost ring:
                                       // [0] this step's old-time data, [1] the next step's
    double *trace;         // [cell][2d][v][nfn*n]
    double *gbar;          // [cell][2d][v][nfn]
    uint8_t *beta[2];      // [cell] old / new
    uint8_t *force;        // [cell] forced troubled mask
    const uint8_t *mask;   // [cell] masked geometry, 1 = solid cell (null: no solid cells)
    uint8_t *mflag;        // [slot][subcell] MOOD flags of the troubled cells' WENO3 results
    float *margin;         // [cell]
    int *tlist, *clist;    // troubled cells, corrected cells
    int *slot[2];          // cell -> pool slot (old / new), -1 if none
    double *pool[2];       // [slot][v][sub]
    double *sflux;         // [slot][2d][v][n^(d-1)] subcell fluxes integrated against the face basis
    double *fpts;          // [chunk][2d][v][(3 Ns)^(d-1)] time-averaged sub-face fluxes per point
    int *blk;              // block partial counts for compaction [2][nblk]
    int *counts;           // [0] troubled [1] corrected [2] nonphysical cumulative [3] capacity overflow
                           // [4] block ticket of the compaction [5] MOOD-flagged subcells
                           // [6] cells recomputed by the MOOD layer
    double *scal;          // [0] dt [1] t [2] lambda_max [4] poison armed [5] cell [6] var [7] value
    double *lam_part;      // per-block lambda partials
    int64_t *ring;         // extended-grid indices of the ghost ring
    // subcell chunk scratch
    double *halo;          // [chunk][v][(Ns+6)^d]
    double *Y;             // [chunk][pos][v][3^d] reconstructed nodal values (float in the mixed form)
    double *strace;        // [chunk][pos][2d][v][3^(d-1)*3]
    // large cells (3D, N = 9): per-workgroup slots of the arrays that exceed LDS
    double *big;           // [BIG_WG][BigCell slot]
};

// Arguments of one launch of the space-time predictor.
template <typename R>
struct PredArgs {
    const double *in;      // input nodal values
    int64_t in_cstride;    // stride between cells
    int64_t in_vstride;    // stride between variables
    R *trace;              // [cell][2d][v][nfn*n]
    double *vol_out;       // candidate with volume term [v][cell][node] (main scheme only)
    int64_t ncell;         // cells (or subcell positions) in this launch
    int64_t cell0;         // first cell index (for vol_out addressing)
    int iters;
    double dth[3];         // dt/h_k multipliers (without dt)
    const double *dt;      // device scalar
    // operators of the n-node basis used by this launch (row stride MAXN)
    const R *D, *Kw, *Lb, *Rb, *w, *Dvol;
    const R *DE, *DO;      // even / odd parts of D (row strides MAXN/2 + 1 and MAXN/2)
    // if set, the number of cells is min(*dcount, dcap) * dmult (read on the device)
    const int *dcount;
    int64_t dcap;
    int dmult;
};

// Batched launches: one launch per stage of the step covers every problem of one (d, N)
// class.  A BatchEntry holds what the per-problem launch passes as arguments (one entry
// per problem and buffer parity, in device memory); a BTile names the problem and the
// block within that problem's own grid for one workgroup of a batched launch.
struct BatchEntry {
    const Tables *T;
    Prob P;
    Bufs B;
    int cur;               // current state buffer
    int limiter;
    int64_t cap;           // pool slots
    int64_t kb1, kb2;      // face kernel: first block of axis 1 and of axis 2
    int lam_nb;            // blocks of the wave-speed reduction
    double factor;         // dt = factor / lambda_max  (cfl * hmin / (d (2N+1)))
    const int64_t *ring;   // ghost-ring cells of the extended grid (null: every extended cell)
    PredArgs<float> pf;    // predictor arguments in the mixed form
    PredArgs<double> pd;   // and in the FP64 form
};

struct BTile {
    int p;                 // problem within the class
    int b;                 // block index within that problem's grid
    int n;                 // that problem's grid size for this stage
};

int64_t ipow64(int64_t b, int e);

}  // namespace adg
