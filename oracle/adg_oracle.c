/*
 * FP64 CPU oracle: one ADER-DG step with the a-posteriori subcell (MOOD) limiter.
 *
 * TEST INFRASTRUCTURE ONLY (see adg_oracle.h).  Written as plain loops that follow
 * the paper step by step, with no blocking, fusion or sum-factorisation beyond what
 * the formulas state, so that each function can be checked against the paper by eye.
 *
 * Section references are to Dumbser, Zanotti, Loubere, Diot (2014):
 *   Sec. 2.1  data representation (tensor Gauss-Legendre nodal basis)
 *   Sec. 2.2  local space-time predictor, eq. (pde.nc.dg2)
 *   Sec. 2.3  one-step corrector, eq. (pde.nc.gw2), Rusanov flux
 *   Sec. 2.4  time step, eq. (cfl)
 *   Sec. 4.2  subcell projection P, eq. (subcell.p); reconstruction R, eqs. (subcell.r),
 *             (subcell.r.constraint), (rid)
 *   Sec. 4.3  PAD eq. (positivity), relaxed DMP eqs. (dmp.org), (relax), (dmp),
 *             subcell ADER-WENO3 eq. (aderweno), its initial/boundary data eq. (ader.icbc)
 *   Sec. 4.4  five-step summary, flux correction of unlimited neighbours, initial detection
 *   Sec. 5    Euler equations and ideal-gas EOS
 * Where the paper is silent the reading taken is named in a comment ("reading: ...").
 */
#include "adg_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXN OR_MAXN
#define MAXNS OR_MAXNS

typedef struct {
    int n;
    double xi[MAXN], w[MAXN];
    double D[MAXN][MAXN];   /* D[a][b] = phi_b'(xi_a) */
    double L[MAXN], R[MAXN];/* phi_b(0), phi_b(1) */
    double Kw[MAXN][MAXN];  /* K1^{-1} diag(w) */
} basis_t;

struct or_solver {
    or_config c;
    int d, nv, n, nn, nst, nfn, Ns, nsub, nsubf;
    long ncell;
    int nc[3];
    double h[3];
    basis_t B, B3;
    double P[MAXNS][MAXN], R[MAXN][MAXNS];
    double wenoinv[3][3][3];
    double *u, *vstore, *margin, *bmin, *bmax;
    uint8_t *beta, *force;
    uint8_t *solid;            /* masked geometry: 1 = solid cell (NULL: none) */
    double t;
    long nonphys;
    long poison_cell;          /* test hook: cell whose next candidate is overwritten (-1: none) */
    long mood_flagged, mood_redone;   /* MOOD layer of the last step: flagged subcells, recomputed cells */
    int poison_var;
    double poison_value;
};

/* ------------------------------------------------------------------ helpers */
static int ipow(int b, int e) { int r = 1; while (e-- > 0) r *= b; return r; }

static void unflat(int idx, int n, int d, int *m) {
    for (int k = 0; k < d; k++) { m[k] = idx % n; idx /= n; }
}
static int flat(const int *m, int n, int d) {
    int r = 0;
    for (int k = d - 1; k >= 0; k--) r = r * n + m[k];
    return r;
}
/* index of a node with its axis-k coordinate removed (axes kept in increasing order) */
static int strip_axis(const int *m, int k, int n, int d) {
    int r = 0;
    for (int j = d - 1; j >= 0; j--) if (j != k) r = r * n + m[j];
    return r;
}

/* Gauss-Jordan inverse with partial pivoting of a dense n x n matrix (row major). */
static int invert(int n, const double *A, double *Ainv) {
    double M[2 * MAXNS * MAXNS];
    int w2 = 2 * n;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < w2; j++)
            M[i * w2 + j] = j < n ? A[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int col = 0; col < n; col++) {
        int piv = col;
        for (int r = col + 1; r < n; r++)
            if (fabs(M[r * w2 + col]) > fabs(M[piv * w2 + col])) piv = r;
        if (M[piv * w2 + col] == 0.0) return -1;
        if (piv != col)
            for (int j = 0; j < w2; j++) { double t = M[col * w2 + j]; M[col * w2 + j] = M[piv * w2 + j]; M[piv * w2 + j] = t; }
        double p = M[col * w2 + col];
        for (int j = 0; j < w2; j++) M[col * w2 + j] /= p;
        for (int r = 0; r < n; r++) {
            if (r == col) continue;
            double f = M[r * w2 + col];
            if (f != 0.0) for (int j = 0; j < w2; j++) M[r * w2 + j] -= f * M[col * w2 + j];
        }
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) Ainv[i * n + j] = M[i * w2 + n + j];
    return 0;
}

/* ------------------------------------------------- Sec. 2.1: quadrature and basis */
/* Gauss-Legendre nodes/weights on [0,1] by Golub-Welsch: eigen-decomposition of the
 * symmetric tridiagonal Jacobi matrix of the Legendre recurrence, done here with the
 * cyclic Jacobi rotation method (small n, plainly convergent). */
static void gauss_legendre(int n, double *xi, double *w) {
    double A[MAXNS][MAXNS], V[MAXNS][MAXNS];
    memset(A, 0, sizeof A);
    for (int i = 0; i < n; i++) for (int j = 0; j < n; j++) V[i][j] = (i == j);
    for (int k = 1; k < n; k++) {
        double b = k / sqrt(4.0 * k * k - 1.0);
        A[k - 1][k] = A[k][k - 1] = b;
    }
    for (int sweep = 0; sweep < 100; sweep++) {
        double off = 0;
        for (int p = 0; p < n; p++) for (int q = p + 1; q < n; q++) off += A[p][q] * A[p][q];
        if (off < 1e-34) break;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) {
                if (fabs(A[p][q]) < 1e-300) continue;
                double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; k++) {      /* A <- A J */
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; k++) {      /* A <- J^T A */
                    double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; k++) {      /* V <- V J */
                    double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
    double x[MAXNS], ww[MAXNS];
    for (int i = 0; i < n; i++) {
        double nrm = 0;
        for (int k = 0; k < n; k++) nrm += V[k][i] * V[k][i];
        x[i] = A[i][i];
        ww[i] = V[0][i] * V[0][i] / nrm;   /* weights on [-1,1] are 2 v0^2; on [0,1] halve */
    }
    for (int i = 0; i < n; i++)            /* sort ascending */
        for (int j = i + 1; j < n; j++)
            if (x[j] < x[i]) { double t = x[i]; x[i] = x[j]; x[j] = t; t = ww[i]; ww[i] = ww[j]; ww[j] = t; }
    for (int i = 0; i < n; i++) { xi[i] = 0.5 * (x[i] + 1.0); w[i] = ww[i]; }
}

static double lagrange(int n, const double *xi, int b, double x) {
    double r = 1;
    for (int m = 0; m < n; m++) if (m != b) r *= (x - xi[m]) / (xi[b] - xi[m]);
    return r;
}
static double lagrange_d(int n, const double *xi, int b, double x) {
    double s = 0;
    for (int j = 0; j < n; j++) {
        if (j == b) continue;
        double r = 1.0 / (xi[b] - xi[j]);
        for (int m = 0; m < n; m++) if (m != b && m != j) r *= (x - xi[m]) / (xi[b] - xi[m]);
        s += r;
    }
    return s;
}

/* Operators of eq. (pde.nc.dg2) in nodal form.  Time part of
 * [theta_k,theta_l]^1 - <d_tau theta_k, theta_l> with GL quadrature:
 *   K1[k][l] = R_k R_l - w_l D[l][k];  the spatial mass factor cancels. */
static void make_basis(int n, basis_t *B) {
    B->n = n;
    gauss_legendre(n, B->xi, B->w);
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++) B->D[a][b] = lagrange_d(n, B->xi, b, B->xi[a]);
    for (int b = 0; b < n; b++) {
        B->L[b] = lagrange(n, B->xi, b, 0.0);
        B->R[b] = lagrange(n, B->xi, b, 1.0);
    }
    double K1[MAXN * MAXN], K1i[MAXN * MAXN];
    for (int k = 0; k < n; k++)
        for (int l = 0; l < n; l++) K1[k * n + l] = B->R[k] * B->R[l] - B->w[l] * B->D[l][k];
    invert(n, K1, K1i);
    for (int s = 0; s < n; s++)
        for (int t = 0; t < n; t++) B->Kw[s][t] = K1i[s * n + t] * B->w[t];
}

void or_basis(int n, double *xi, double *w, double *D, double *L, double *R, double *Kw) {
    basis_t B;
    make_basis(n, &B);
    for (int a = 0; a < n; a++) {
        xi[a] = B.xi[a]; w[a] = B.w[a]; L[a] = B.L[a]; R[a] = B.R[a];
        for (int b = 0; b < n; b++) { D[a * n + b] = B.D[a][b]; Kw[a * n + b] = B.Kw[a][b]; }
    }
}

/* Sec. 4.2, eq. (subcell.p): P[s][l] = Ns * integral over subinterval s of phi_l,
 * evaluated exactly with n-point GL on the subinterval (degree N integrand).
 * eqs. (subcell.r)+(subcell.r.constraint): with equal subcells and an unweighted
 * residual the least-squares solution already conserves the cell mean (constants lie
 * in range(P), so the residual is orthogonal to the ones vector); R = (P^T P)^{-1} P^T.
 * reading: unweighted least squares; the tests cross-check against a KKT solve. */
static void make_subcell_ops(const basis_t *B, int Ns, double P[MAXNS][MAXN], double R[MAXN][MAXNS]) {
    int n = B->n;
    for (int s = 0; s < Ns; s++)
        for (int l = 0; l < n; l++) {
            double acc = 0;
            for (int q = 0; q < n; q++) acc += B->w[q] * lagrange(n, B->xi, l, (s + B->xi[q]) / Ns);
            P[s][l] = acc;
        }
    double PtP[MAXN * MAXN], PtPi[MAXN * MAXN];
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            double acc = 0;
            for (int s = 0; s < Ns; s++) acc += P[s][i] * P[s][j];
            PtP[i * n + j] = acc;
        }
    invert(n, PtP, PtPi);
    for (int i = 0; i < n; i++)
        for (int s = 0; s < Ns; s++) {
            double acc = 0;
            for (int j = 0; j < n; j++) acc += PtPi[i * n + j] * P[s][j];
            R[i][s] = acc;
        }
}

void or_subcell_ops(int N, int Ns, double *P, double *R) {
    basis_t B;
    double Pm[MAXNS][MAXN], Rm[MAXN][MAXNS];
    make_basis(N + 1, &B);
    make_subcell_ops(&B, Ns, Pm, Rm);
    for (int s = 0; s < Ns; s++)
        for (int l = 0; l <= N; l++) { P[s * (N + 1) + l] = Pm[s][l]; R[l * Ns + s] = Rm[l][s]; }
}

/* ---------------------------------------------------- Sec. 5: Euler, ideal gas */
static double pressure(int d, double g, const double *Q) {
    double ke = 0;
    for (int j = 0; j < d; j++) ke += Q[1 + j] * Q[1 + j];
    return (g - 1.0) * (Q[d + 1] - 0.5 * ke / Q[0]);
}
static void euler_flux(int d, int k, double g, const double *Q, double *F) {
    double p = pressure(d, g, Q);
    double un = Q[1 + k] / Q[0];
    F[0] = Q[1 + k];
    for (int j = 0; j < d; j++) F[1 + j] = Q[1 + j] * un + (j == k ? p : 0.0);
    F[d + 1] = un * (Q[d + 1] + p);
}
/* Sec. 2.3: Rusanov flux; reading: wave speed taken per quadrature node as the larger
 * of |u_n| + c on the two sides. */
static void rusanov(int d, int k, double g, const double *qL, const double *qR, double *G) {
    double FL[5], FR[5];
    euler_flux(d, k, g, qL, FL);
    euler_flux(d, k, g, qR, FR);
    double sL = fabs(qL[1 + k] / qL[0]) + sqrt(g * pressure(d, g, qL) / qL[0]);
    double sR = fabs(qR[1 + k] / qR[0]) + sqrt(g * pressure(d, g, qR) / qR[0]);
    double s = fmax(sL, sR);
    for (int v = 0; v < d + 2; v++) G[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * s * (qR[v] - qL[v]);
}

/* |A(Q)| dQ for the Euler flux Jacobian A along axis k: dQ is split into the waves of A at
 * Q (acoustic, entropy, shear) and each part scaled by the modulus of its eigenvalue
 * (u_k - c, u_k, u_k + c). */
void or_abs_jacobian(int d, int k, double g, const double *Q, const double *dQ, double *out) {
    int nv = d + 2;
    double rho = Q[0], u[3] = {0, 0, 0}, q2 = 0;
    for (int j = 0; j < d; j++) { u[j] = Q[1 + j] / rho; q2 += u[j] * u[j]; }
    double p = pressure(d, g, Q), c2 = g * p / rho, c = sqrt(c2), H = (Q[d + 1] + p) / rho, un = u[k];
    /* primitive increments of dQ at Q */
    double drho = dQ[0], du[3] = {0, 0, 0}, mdq = 0;
    for (int j = 0; j < d; j++) { du[j] = (dQ[1 + j] - u[j] * drho) / rho; mdq += u[j] * dQ[1 + j]; }
    double dp = (g - 1.0) * (dQ[d + 1] - mdq + 0.5 * q2 * drho);
    double a1 = (dp - rho * c * du[k]) / (2.0 * c2), a5 = (dp + rho * c * du[k]) / (2.0 * c2);
    double a2 = drho - dp / c2;
    double l1 = fabs(un - c), l2 = fabs(un), l5 = fabs(un + c);
    for (int v = 0; v < nv; v++) out[v] = 0.0;
    /* acoustic waves r = (1, u -+ c e_k, H -+ c u_k) */
    out[0] += l1 * a1 + l5 * a5;
    for (int j = 0; j < d; j++) out[1 + j] += l1 * a1 * (u[j] - (j == k ? c : 0.0)) + l5 * a5 * (u[j] + (j == k ? c : 0.0));
    out[d + 1] += l1 * a1 * (H - c * un) + l5 * a5 * (H + c * un);
    /* entropy wave r = (1, u, |u|^2/2) and shear waves r = (0, e_j, u_j), j != k */
    out[0] += l2 * a2;
    for (int j = 0; j < d; j++) out[1 + j] += l2 * a2 * u[j];
    out[d + 1] += l2 * a2 * 0.5 * q2;
    for (int j = 0; j < d; j++) {
        if (j == k) continue;
        double at = rho * du[j];
        out[1 + j] += l2 * at;
        out[d + 1] += l2 * at * u[j];
    }
}

/* Osher-type flux of the universal form (reading: the paper names the flux of its
 * reference without giving formulas): G = (F(qL) + F(qR))/2 - 1/2 int_0^1 |A(psi(s))| ds
 * (qR - qL) along the straight path psi(s) = qL + s (qR - qL), integrated with the
 * 3-point Gauss-Legendre rule (xi3, w3). */
static void osher(int d, int k, double g, const double *xi3, const double *w3, const double *qL, const double *qR,
                  double *G) {
    int nv = d + 2;
    double FL[5], FR[5], dQ[5], acc[5] = {0, 0, 0, 0, 0};
    euler_flux(d, k, g, qL, FL);
    euler_flux(d, k, g, qR, FR);
    for (int v = 0; v < nv; v++) dQ[v] = qR[v] - qL[v];
    for (int j = 0; j < 3; j++) {
        double psi[5], o[5];
        for (int v = 0; v < nv; v++) psi[v] = qL[v] + xi3[j] * dQ[v];
        or_abs_jacobian(d, k, g, psi, dQ, o);
        for (int v = 0; v < nv; v++) acc[v] += w3[j] * o[v];
    }
    for (int v = 0; v < nv; v++) G[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * acc[v];
}

/* Numerical flux of the scheme: Rusanov (0) or Osher-type (1). */
static void num_flux(const or_solver *S, int k, const double *qL, const double *qR, double *G) {
    if (S->c.flux == 1) osher(S->d, k, S->c.gamma, S->B3.xi, S->B3.w, qL, qR, G);
    else rusanov(S->d, k, S->c.gamma, qL, qR, G);
}

/* Test entry: the numerical flux with the 3-point rule computed here. */
void or_numerical_flux(int d, int k, double g, int flux, const double *qL, const double *qR, double *G) {
    if (flux == 1) {
        double xi[3], w[3];
        gauss_legendre(3, xi, w);
        osher(d, k, g, xi, w, qL, qR, G);
    } else {
        rusanov(d, k, g, qL, qR, G);
    }
}

/* --------------------------------------------------------- boundary conditions */
/* reading: the paper names its boundary conditions without formulas.  A ghost state
 * is made from the interior state at the same point: transmissive copies it,
 * reflective negates the normal momentum, Dirichlet takes the prescribed state. */
static void bc_ghost(const or_solver *S, int k, int side, const double *qin, const double *x, double t,
                     double *qout) {
    const or_bc *b = &S->c.bc[k][side];
    int which = 0;
    if (b->split_axis >= 0) which = (x[b->split_axis] < b->split0 + b->split_speed * t) ? 0 : 1;
    int kind = b->kind[which];
    int nv = S->nv;
    if (kind == OR_DIRICHLET) {
        for (int v = 0; v < nv; v++) qout[v] = b->state[which][v];
        return;
    }
    for (int v = 0; v < nv; v++) qout[v] = qin[v];
    if (kind == OR_REFLECTIVE) qout[1 + k] = -qout[1 + k];
}

/* ----------------------------------------------- Sec. 2.2: space-time predictor */
/* Nodal form of eq. (pde.nc.dg2) for one cell (dividing out the spatial weights):
 *   q^{r+1}_{a,s} = (K1^{-1} L)_s u_a - sum_t (K1^{-1} diag w)_{st} sum_k (dt/h_k)
 *                   sum_b D[a_k][b] F_k(q^r at node a with a_k <- b, time t)
 * with K1^{-1} L = 1 (checked in the tests).  reading: initial guess q^0 = u (constant
 * in time) and a fixed number of sweeps.
 * u0[v*nn + a];  q[v*nst + a + nn*s]. */
static void predictor(const basis_t *B, int d, int nv, double g, const double *dth, int iters,
                      const double *u0, double *q, double *F, double *V) {
    int n = B->n, nn = ipow(n, d), nst = nn * n;
    for (int v = 0; v < nv; v++)
        for (int s = 0; s < n; s++)
            for (int a = 0; a < nn; a++) q[v * nst + a + nn * s] = u0[v * nn + a];
    for (int r = 0; r < iters; r++) {
        for (int i = 0; i < nv * nst; i++) V[i] = 0;
        for (int k = 0; k < d; k++) {
            for (int p = 0; p < nst; p++) {
                double Q[5], Fk[5];
                for (int v = 0; v < nv; v++) Q[v] = q[v * nst + p];
                euler_flux(d, k, g, Q, Fk);
                for (int v = 0; v < nv; v++) F[v * nst + p] = Fk[v];
            }
            for (int s = 0; s < n; s++)
                for (int a = 0; a < nn; a++) {
                    int m[3];
                    unflat(a, n, d, m);
                    int ak = m[k];
                    for (int v = 0; v < nv; v++) {
                        double acc = 0;
                        for (int b = 0; b < n; b++) {
                            m[k] = b;
                            acc += B->D[ak][b] * F[v * nst + flat(m, n, d) + nn * s];
                        }
                        m[k] = ak;
                        V[v * nst + a + nn * s] += dth[k] * acc;
                    }
                }
        }
        for (int v = 0; v < nv; v++)
            for (int a = 0; a < nn; a++)
                for (int s = 0; s < n; s++) {
                    double acc = 0;
                    for (int t = 0; t < n; t++) acc += B->Kw[s][t] * V[v * nst + a + nn * t];
                    q[v * nst + a + nn * s] = u0[v * nn + a] - acc;
                }
    }
}

/* Face traces of the predictor: q at xi_k = 0 (side 0) or 1 (side 1), per tangential node
 * and time node.  tr[((2k+side)*nv + v)*nfn*n + ap + nfn*s] */
static void traces(const basis_t *B, int d, int nv, const double *q, double *tr) {
    int n = B->n, nn = ipow(n, d), nst = nn * n, nfn = ipow(n, d - 1);
    for (int k = 0; k < d; k++)
        for (int side = 0; side < 2; side++)
            for (int v = 0; v < nv; v++)
                for (int s = 0; s < n; s++)
                    for (int ap = 0; ap < nfn; ap++) {
                        /* rebuild the full index with axis k free */
                        int m[3], mp[3], j2 = 0;
                        unflat(ap, n, d - 1, mp);
                        for (int j = 0; j < d; j++) m[j] = (j == k) ? 0 : mp[j2++];
                        double acc = 0;
                        for (int b = 0; b < n; b++) {
                            m[k] = b;
                            acc += (side ? B->R[b] : B->L[b]) * q[v * nst + flat(m, n, d) + nn * s];
                        }
                        tr[((2 * k + side) * nv + v) * nfn * n + ap + nfn * s] = acc;
                    }
}

void or_predictor(int dim, int N, double gamma, const double *dt_over_h, int iters,
                  const double *u_cell, double *q) {
    basis_t B;
    make_basis(N + 1, &B);
    int n = N + 1, nv = dim + 2, nst = ipow(n, dim + 1);
    double *F = malloc(sizeof(double) * nv * nst), *V = malloc(sizeof(double) * nv * nst);
    predictor(&B, dim, nv, gamma, dt_over_h, iters, u_cell, q, F, V);
    free(F); free(V);
}

/* --------------------------------------------------------------- subcell WENO3 */
/* reading (the paper defers the scheme to its references): polynomial WENO of degree 2
 * on conserved variables, one dimension at a time.  Three stencils {j-2..j}, {j-1..j+1},
 * {j..j+2}; each quadratic matches its three averages exactly.  Oscillation indicator
 * sigma = int_0^1 (p')^2 + (p'')^2 in the subcell's unit coordinate; weights
 * lambda / (sigma + 1e-14)^8 with lambda = 1e5 for the central stencil and 1 else. */
static const double WENO_LAMBDA[3] = {1.0, 1.0e5, 1.0};
static const double WENO_EPS = 1e-14;

static void make_weno(double inv[3][3][3]) {
    for (int st = 0; st < 3; st++) {
        double A[9], Ai[9];
        for (int m = 0; m < 3; m++) {
            double o = st - 2 + m;
            for (int pw = 0; pw < 3; pw++) A[m * 3 + pw] = (pow(o + 1, pw + 1) - pow(o, pw + 1)) / (pw + 1);
        }
        invert(3, A, Ai);
        for (int i = 0; i < 9; i++) inv[st][i / 3][i % 3] = Ai[i];
    }
}

/* a[0..4] averages at offsets -2..2; out: reconstructed values at the 3 GL nodes xi3 */
static void weno3_1d(const double inv[3][3][3], const double *xi3, const double *a, double *out) {
    double c[3][3], wt[3], sum = 0;
    for (int st = 0; st < 3; st++) {
        for (int pw = 0; pw < 3; pw++) {
            double acc = 0;
            for (int m = 0; m < 3; m++) acc += inv[st][pw][m] * a[st + m];
            c[st][pw] = acc;
        }
        double sig = c[st][1] * c[st][1] + 2.0 * c[st][1] * c[st][2] + (16.0 / 3.0) * c[st][2] * c[st][2];
        wt[st] = WENO_LAMBDA[st] / pow(sig + WENO_EPS, 8);
        sum += wt[st];
    }
    for (int q = 0; q < 3; q++) {
        double x = xi3[q], acc = 0;
        for (int st = 0; st < 3; st++) acc += (wt[st] / sum) * (c[st][0] + c[st][1] * x + c[st][2] * x * x);
        out[q] = acc;
    }
}

void or_weno3(const double *avg5, double *out3) {
    double inv[3][3][3], xi[3], w[3];
    make_weno(inv);
    gauss_legendre(3, xi, w);
    weno3_1d(inv, xi, avg5, out3);
}

/* -------------------------------------------------------------- solver set-up */
or_solver *or_create(const or_config *c) {
    if (c->dim < 2 || c->dim > 3 || c->N < 1 || c->N + 1 > MAXN || c->Ns < c->N + 1 || c->Ns < 3 ||
        c->Ns > MAXNS)
        return NULL;
    or_solver *S = calloc(1, sizeof *S);
    S->c = *c;
    S->poison_cell = -1;
    S->d = c->dim; S->nv = c->dim + 2; S->n = c->N + 1; S->Ns = c->Ns;
    S->nn = ipow(S->n, S->d); S->nst = S->nn * S->n; S->nfn = ipow(S->n, S->d - 1);
    S->nsub = ipow(S->Ns, S->d); S->nsubf = ipow(S->Ns, S->d - 1);
    S->ncell = 1;
    for (int k = 0; k < 3; k++) {
        S->nc[k] = k < S->d ? c->ncell[k] : 1;
        S->ncell *= S->nc[k];
        S->h[k] = k < S->d ? (c->hi[k] - c->lo[k]) / c->ncell[k] : 1.0;
    }
    make_basis(S->n, &S->B);
    make_basis(3, &S->B3);
    make_subcell_ops(&S->B, S->Ns, S->P, S->R);
    make_weno(S->wenoinv);
    S->u = calloc((size_t)S->nv * S->ncell * S->nn, sizeof(double));
    S->vstore = calloc((size_t)S->nv * S->ncell * S->nsub, sizeof(double));
    S->margin = calloc(S->ncell, sizeof(double));
    S->bmin = calloc((size_t)S->nv * S->ncell, sizeof(double));
    S->bmax = calloc((size_t)S->nv * S->ncell, sizeof(double));
    S->beta = calloc(S->ncell, 1);
    S->force = calloc(S->ncell, 1);
    return S;
}

void or_destroy(or_solver *S) {
    if (!S) return;
    free(S->u); free(S->vstore); free(S->margin); free(S->bmin); free(S->bmax);
    free(S->beta); free(S->force); free(S->solid); free(S);
}

/* Masked geometry (reading: the paper's forward-facing step removes a rectangle from the
 * domain and names its faces reflective walls, without saying how the scheme treats them):
 * solid cells carry a fixed state, are never updated, troubled or corrected, and take no
 * part in the time step; a face between a fluid and a solid cell is a reflective wall. */
void or_set_mask(or_solver *S, const uint8_t *mask) {
    free(S->solid);
    S->solid = NULL;
    if (!mask) return;
    S->solid = malloc(S->ncell);
    memcpy(S->solid, mask, S->ncell);
}

void or_set_threads(int nt) {
#ifdef _OPENMP
    omp_set_num_threads(nt);
#else
    (void)nt;
#endif
}
int or_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static long cell_index(const or_solver *S, const int *ci) {
    return ci[0] + (long)S->nc[0] * (ci[1] + (long)S->nc[1] * ci[2]);
}
static void cell_coords(const or_solver *S, long c, int *ci) {
    ci[0] = (int)(c % S->nc[0]);
    ci[1] = (int)((c / S->nc[0]) % S->nc[1]);
    ci[2] = (int)(c / ((long)S->nc[0] * S->nc[1]));
}

/* ------------------------------------------------------- projection utilities */
/* P applied to one cell's nodal values: plain tensor sum over all nodes. */
static void apply_P(const or_solver *S, const double *ucell /*[v][nn] stride nn*/, long ustride,
                    double *vcell /*[v][nsub] stride vstride*/, long vstride) {
    int d = S->d, n = S->n, Ns = S->Ns;
    for (int v = 0; v < S->nv; v++)
        for (int sg = 0; sg < S->nsub; sg++) {
            int ms[3];
            unflat(sg, Ns, d, ms);
            double acc = 0;
            for (int a = 0; a < S->nn; a++) {
                int ma[3];
                unflat(a, n, d, ma);
                double wgt = 1;
                for (int k = 0; k < d; k++) wgt *= S->P[ms[k]][ma[k]];
                acc += wgt * ucell[v * ustride + a];
            }
            vcell[v * vstride + sg] = acc;
        }
}
static void apply_R(const or_solver *S, const double *vcell, long vstride, double *ucell, long ustride) {
    int d = S->d, n = S->n, Ns = S->Ns;
    for (int v = 0; v < S->nv; v++)
        for (int a = 0; a < S->nn; a++) {
            int ma[3];
            unflat(a, n, d, ma);
            double acc = 0;
            for (int sg = 0; sg < S->nsub; sg++) {
                int ms[3];
                unflat(sg, Ns, d, ms);
                double wgt = 1;
                for (int k = 0; k < d; k++) wgt *= S->R[ma[k]][ms[k]];
                acc += wgt * vcell[v * vstride + sg];
            }
            ucell[v * ustride + a] = acc;
        }
}

/* 1 if the cell at global coordinates g (possibly outside the domain) is solid: outside a
 * periodic axis it wraps; outside another axis it is the cell whose interior it mirrors. */
static int solid_at(const or_solver *S, const int *g) {
    if (!S->solid) return 0;
    int ci[3] = {0, 0, 0};
    for (int k = 0; k < S->d; k++) {
        int x = g[k], nk = S->nc[k];
        if (x < 0 || x >= nk) {
            if (S->c.bc[k][x >= nk].kind[0] == OR_PERIODIC) x = ((x % nk) + nk) % nk;
            else x = x >= nk ? 2 * nk - 1 - x : -1 - x;
        }
        ci[k] = x;
    }
    return S->solid[cell_index(S, ci)];
}

/* Subcell value at global (cell, subcell) position, where the cell index may lie one
 * or more cells outside the domain.  reading (the paper is silent on boundaries of the
 * subgrid data): periodic axes wrap; other axes mirror the interior subcells across the
 * boundary and then apply the boundary rule at the ghost subcell centre (time t).
 * A solid cell (masked geometry) holds the mirror image of the fluid across its walls: for
 * every axis along which it has a fluid face neighbour (the lower one if both are fluid)
 * its data is that neighbour's, mirrored along the axis (subcell index reversed, the axis's
 * momentum negated); a solid cell at a convex corner of the obstacle, with fluid face
 * neighbours along two axes, mirrors along both (the point reflection through the corner).
 * The image depends on the solid cell alone, not on the cell that reads it, so two troubled
 * cells see the same data and compute the same sub-face fluxes.
 * vn is [v][cell][sub]. */
static void subcell_value(const or_solver *S, const double *vn, const int *gci_in, const int *gs_in, double t,
                          double *out) {
    int d = S->d, Ns = S->Ns, nv = S->nv;
    int gci[3] = {gci_in[0], gci_in[1], gci_in[2]}, gs[3] = {gs_in[0], gs_in[1], gs_in[2]};
    int wall[3] = {0, 0, 0};
    if (S->solid && solid_at(S, gci)) {
        int step[3] = {0, 0, 0};
        for (int k = 0; k < d; k++) {
            int lo[3] = {gci[0], gci[1], gci[2]}, hi[3] = {gci[0], gci[1], gci[2]};
            lo[k] -= 1;
            hi[k] += 1;
            if (!solid_at(S, lo)) step[k] = -1;
            else if (!solid_at(S, hi)) step[k] = 1;
        }
        for (int k = 0; k < d; k++)
            if (step[k]) { wall[k] = 1; gci[k] += step[k]; gs[k] = Ns - 1 - gs[k]; }
    }
    int ci[3] = {0, 0, 0}, si[3] = {0, 0, 0};
    int ghost_axis[3], ghost_side[3], ng = 0;
    for (int k = 0; k < d; k++) {
        ci[k] = gci[k]; si[k] = gs[k];
        int nk = S->nc[k];
        if (ci[k] < 0 || ci[k] >= nk) {
            int side = ci[k] >= nk;
            if (S->c.bc[k][side].kind[0] == OR_PERIODIC) {
                ci[k] = ((ci[k] % nk) + nk) % nk;
            } else {
                ci[k] = side ? 2 * nk - 1 - ci[k] : -1 - ci[k];
                si[k] = Ns - 1 - si[k];
                ghost_axis[ng] = k; ghost_side[ng] = side; ng++;
            }
        }
    }
    long c = cell_index(S, ci);
    int sg = flat(si, Ns, d);
    double q[5];
    for (int v = 0; v < nv; v++) q[v] = vn[((long)v * S->ncell + c) * S->nsub + sg];
    if (ng) {
        double x[3];
        for (int k = 0; k < d; k++)
            x[k] = S->c.lo[k] + S->h[k] * (gci[k] + (gs[k] + 0.5) / Ns);
        for (int g = 0; g < ng; g++) {
            double qo[5];
            bc_ghost(S, ghost_axis[g], ghost_side[g], q, x, t, qo);
            for (int v = 0; v < nv; v++) q[v] = qo[v];
        }
    }
    for (int k = 0; k < d; k++)
        if (wall[k]) q[1 + k] = -q[1 + k];
    for (int v = 0; v < nv; v++) out[v] = q[v];
}

/* Sec. 4.3: M_i, m_i of eq. (dmp): componentwise max/min of the subcell data v over the
 * Voronoi neighbourhood V_i (the 3^d block of cells sharing a node with T_i). */
static void neighbourhood_bounds(const or_solver *S, const double *vn, double t, double *bmin, double *bmax) {
    int d = S->d, Ns = S->Ns, nv = S->nv;
    long ncell = S->ncell;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < ncell; c++) {
        int ci[3];
        cell_coords(S, c, ci);
        double lo[5], hi[5];
        for (int v = 0; v < nv; v++) { lo[v] = INFINITY; hi[v] = -INFINITY; }
        int nblk = ipow(3, d);
        for (int o = 0; o < nblk; o++) {
            int off[3], gci[3] = {0, 0, 0};
            unflat(o, 3, d, off);
            for (int k = 0; k < d; k++) gci[k] = ci[k] + off[k] - 1;
            for (int sg = 0; sg < S->nsub; sg++) {
                int gs[3] = {0, 0, 0};
                unflat(sg, Ns, d, gs);
                double q[5];
                subcell_value(S, vn, gci, gs, t, q);
                for (int v = 0; v < nv; v++) { lo[v] = fmin(lo[v], q[v]); hi[v] = fmax(hi[v], q[v]); }
            }
        }
        for (int v = 0; v < nv; v++) { bmin[v * ncell + c] = lo[v]; bmax[v * ncell + c] = hi[v]; }
    }
}

/* PAD eq. (positivity) + relaxed DMP eqs. (relax),(dmp) on one cell's candidate subcell
 * averages.  reading: PAD is checked on the candidate subcell averages (the detection runs
 * subcell by subcell), plus a finiteness check; delta = max(delta0, eps (M - m)).
 * Returns 1 if troubled; *margin = smallest normalised slack over all tests. */
static int detect_cell(const or_solver *S, const double *vstar /*[v][nsub]*/, const double *m,
                       const double *M, double *margin) {
    int nv = S->nv, d = S->d;
    double g = S->c.gamma;
    int bad = 0;
    double mg = INFINITY;
    for (int sg = 0; sg < S->nsub; sg++) {
        double q[5];
        int finite = 1;
        for (int v = 0; v < nv; v++) { q[v] = vstar[v * S->nsub + sg]; if (!isfinite(q[v])) finite = 0; }
        if (!finite) { bad = 1; mg = -INFINITY; continue; }
        double p = pressure(d, g, q);
        if (!(q[0] > 0.0) || !(p > 0.0)) bad = 1;
        double sr = fmax(fabs(M[0]), fabs(m[0]));
        double se = fmax(fabs(M[d + 1]), fabs(m[d + 1]));
        mg = fmin(mg, q[0] / (sr > 0 ? sr : 1.0));
        mg = fmin(mg, p / (se > 0 ? se : 1.0));
        for (int v = 0; v < nv; v++) {
            double delta = fmax(S->c.delta0, S->c.eps * (M[v] - m[v]));
            double lo = m[v] - delta, hi = M[v] + delta;
            if (q[v] < lo || q[v] > hi) bad = 1;
            double sc = fmax(fabs(M[v]), fabs(m[v]));
            double slack = fmin(q[v] - lo, hi - q[v]) / (sc > 0 ? sc : 1.0);
            mg = fmin(mg, slack);
        }
    }
    *margin = mg;
    return bad;
}

/* v^n of eq. (ader.icbc) for every cell: stored subcell data for cells troubled at the
 * previous step, P(u^n) for all others. */
static double *old_subcell_data(const or_solver *S) {
    double *vn = malloc(sizeof(double) * S->nv * S->ncell * S->nsub);
    long ncell = S->ncell;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < ncell; c++) {
        if (S->beta[c]) {
            for (int v = 0; v < S->nv; v++)
                memcpy(vn + ((long)v * ncell + c) * S->nsub, S->vstore + ((long)v * ncell + c) * S->nsub,
                       sizeof(double) * S->nsub);
        } else {
            apply_P(S, S->u + c * S->nn, ncell * S->nn, vn + c * S->nsub, ncell * S->nsub);
        }
    }
    return vn;
}

/* ------------------------------------------------------------- state I/O */
void or_axis_points(const or_solver *S, int axis, int m, double *out) {
    double lo = S->c.lo[axis], h = S->h[axis];
    int nk = S->nc[axis];
    if (m == 0) {
        for (int i = 0; i < nk; i++)
            for (int a = 0; a < S->n; a++) out[i * S->n + a] = lo + h * (i + S->B.xi[a]);
        return;
    }
    double xi[MAXNS], w[MAXNS];
    gauss_legendre(m, xi, w);
    for (int i = 0; i < nk; i++)
        for (int s = 0; s < S->Ns; s++)
            for (int q = 0; q < m; q++) out[((long)i * S->Ns + s) * m + q] = lo + h * (i + (s + xi[q]) / S->Ns);
}

/* Initial data (Sec. 4.4, last paragraph): L2 projection onto the DG basis by a composite
 * rule (m-point GL on every subcell), and the subcell averages of the same samples.
 * m = 0: samples are point values at the DG nodes (nodal interpolation); v untouched. */
void or_project(const or_solver *S, const double *samples, int m, double *u, double *v) {
    int d = S->d, n = S->n, Ns = S->Ns, nv = S->nv;
    long ncell = S->ncell;
    long ext[3] = {1, 1, 1};
    int per = (m == 0) ? n : Ns * m;
    for (int k = 0; k < d; k++) ext[k] = (long)S->nc[k] * per;
    long npts = ext[0] * ext[1] * ext[2];
    if (m == 0) {
#pragma omp parallel for schedule(static)
        for (long c = 0; c < ncell; c++) {
            int ci[3];
            cell_coords(S, c, ci);
            for (int a = 0; a < S->nn; a++) {
                int ma[3] = {0, 0, 0};
                unflat(a, n, d, ma);
                long gi[3];
                for (int k = 0; k < 3; k++) gi[k] = (long)ci[k] * per + (k < d ? ma[k] : 0);
                long pidx = gi[0] + ext[0] * (gi[1] + ext[1] * gi[2]);
                for (int vv = 0; vv < nv; vv++) u[((long)vv * ncell + c) * S->nn + a] = samples[vv * npts + pidx];
            }
        }
        return;
    }
    double xm[MAXNS], wm[MAXNS];
    gauss_legendre(m, xm, wm);
    int nq = ipow(m, d);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < ncell; c++) {
        int ci[3];
        cell_coords(S, c, ci);
        double acc[5][MAXN * MAXN * MAXN];
        for (int vv = 0; vv < nv; vv++) for (int a = 0; a < S->nn; a++) acc[vv][a] = 0;
        for (int sg = 0; sg < S->nsub; sg++) {
            int ms[3] = {0, 0, 0};
            unflat(sg, Ns, d, ms);
            double avg[5] = {0, 0, 0, 0, 0};
            for (int qi = 0; qi < nq; qi++) {
                int mq[3] = {0, 0, 0};
                unflat(qi, m, d, mq);
                long gi[3] = {0, 0, 0};
                double wq = 1, xref[3];
                for (int k = 0; k < d; k++) {
                    gi[k] = ((long)ci[k] * Ns + ms[k]) * m + mq[k];
                    wq *= wm[mq[k]];
                    xref[k] = (ms[k] + xm[mq[k]]) / Ns;
                }
                long pidx = gi[0] + ext[0] * (gi[1] + ext[1] * gi[2]);
                for (int vv = 0; vv < nv; vv++) avg[vv] += wq * samples[vv * npts + pidx];
                for (int a = 0; a < S->nn; a++) {
                    int ma[3];
                    unflat(a, n, d, ma);
                    double phi = 1;
                    for (int k = 0; k < d; k++) phi *= lagrange(n, S->B.xi, ma[k], xref[k]);
                    for (int vv = 0; vv < nv; vv++) acc[vv][a] += wq * phi * samples[vv * npts + pidx];
                }
            }
            if (v)
                for (int vv = 0; vv < nv; vv++) v[((long)vv * ncell + c) * S->nsub + sg] = avg[vv];
        }
        for (int a = 0; a < S->nn; a++) {
            int ma[3];
            unflat(a, n, d, ma);
            double W = 1;
            for (int k = 0; k < d; k++) W *= S->B.w[ma[k]];
            for (int vv = 0; vv < nv; vv++)
                u[((long)vv * ncell + c) * S->nn + a] = acc[vv][a] / (W * S->nsub);
        }
    }
}

/* Sets u^0.  With v_exact (subcell averages of the exact initial condition) the
 * detection is applied to P(u^0) against the exact data, and troubled cells start from
 * the exact subcell averages: u^0 := R(v_exact) (reading: the paper is silent on which
 * data a cell flagged at t = 0 carries).  Returns the number of troubled cells. */
int or_set_state(or_solver *S, const double *u, const double *v_exact) {
    long ncell = S->ncell;
    memcpy(S->u, u, sizeof(double) * S->nv * ncell * S->nn);
    memset(S->beta, 0, ncell);
    S->nonphys = 0;
    if (!v_exact) return 0;
    neighbourhood_bounds(S, v_exact, S->t, S->bmin, S->bmax);
    int count = 0;
#pragma omp parallel for schedule(static) reduction(+ : count)
    for (long c = 0; c < ncell; c++) {
        double *vs = malloc(sizeof(double) * S->nv * S->nsub);
        apply_P(S, S->u + c * S->nn, ncell * S->nn, vs, S->nsub);
        double m[5], M[5];
        for (int v = 0; v < S->nv; v++) { m[v] = S->bmin[v * ncell + c]; M[v] = S->bmax[v * ncell + c]; }
        int bad = detect_cell(S, vs, m, M, &S->margin[c]);
        if (S->solid && S->solid[c]) { bad = 0; S->margin[c] = INFINITY; }
        if (bad) {
            S->beta[c] = 1;
            count++;
            for (int v = 0; v < S->nv; v++)
                memcpy(S->vstore + ((long)v * ncell + c) * S->nsub, v_exact + ((long)v * ncell + c) * S->nsub,
                       sizeof(double) * S->nsub);
            apply_R(S, S->vstore + c * S->nsub, ncell * S->nsub, S->u + c * S->nn, ncell * S->nn);
        }
        free(vs);
    }
    return count;
}

void or_get_state(const or_solver *S, double *u) { memcpy(u, S->u, sizeof(double) * S->nv * S->ncell * S->nn); }
void or_get_troubled(const or_solver *S, uint8_t *beta) { memcpy(beta, S->beta, S->ncell); }
void or_get_margin(const or_solver *S, double *m) { memcpy(m, S->margin, sizeof(double) * S->ncell); }
void or_get_subcells(const or_solver *S, double *v) { memcpy(v, S->vstore, sizeof(double) * S->nv * S->ncell * S->nsub); }
void or_get_bounds(const or_solver *S, double *bmin, double *bmax) {
    memcpy(bmin, S->bmin, sizeof(double) * S->nv * S->ncell);
    memcpy(bmax, S->bmax, sizeof(double) * S->nv * S->ncell);
}
/* Test hook: at the next step, every node of variable `var` of cell `cell`'s candidate is
 * set to `value` before the detection of Sec. 4.3 sees it (one step only). */
void or_mood_stats(const or_solver *S, long *flagged, long *redone) {
    *flagged = S->mood_flagged;
    *redone = S->mood_redone;
}

int or_poison(or_solver *S, long cell, int var, double value) {
    if (cell < 0 || cell >= S->ncell || var < 0 || var >= S->nv) return -1;
    S->poison_cell = cell;
    S->poison_var = var;
    S->poison_value = value;
    return 0;
}

void or_force_troubled(or_solver *S, const uint8_t *mask) {
    if (mask) memcpy(S->force, mask, S->ncell); else memset(S->force, 0, S->ncell);
}
double or_time(const or_solver *S) { return S->t; }
void or_set_time(or_solver *S, double t) { S->t = t; }
long or_nonphysical(const or_solver *S) { return S->nonphys; }

/* Sec. 2.4, eq. (cfl): dt = CFL h / (d (2N+1) |lambda_max|).  reading: h is the smallest
 * cell edge and |lambda_max| the largest |v_k| + c over all cells, nodes and axes. */
double or_cfl_dt(const or_solver *S, double cfl) {
    double lam = 0;
    long ncell = S->ncell;
    int d = S->d;
    for (long c = 0; c < ncell; c++)
        for (int a = 0; a < S->nn; a++) {
            if (S->solid && S->solid[c]) break;   /* solid cells take no part in the time step */
            double q[5];
            for (int v = 0; v < S->nv; v++) q[v] = S->u[((long)v * ncell + c) * S->nn + a];
            double cs = sqrt(S->c.gamma * pressure(d, S->c.gamma, q) / q[0]);
            for (int k = 0; k < d; k++) lam = fmax(lam, fabs(q[1 + k] / q[0]) + cs);
        }
    double h = S->h[0];
    for (int k = 1; k < d; k++) h = fmin(h, S->h[k]);
    return cfl * h / (d * (2.0 * S->c.N + 1.0) * lam);
}

/* ---------------------------------------------- subcell ADER-WENO3 (operator A) */
/* Working storage for one troubled cell. */
typedef struct {
    double *halo;   /* [v][(Ns+6)^d]                   subcell averages v^n, 3-deep halo */
    double *tr;     /* [(Ns+2)^d][2d][v][3^{d-1}*3]     subcell predictor face traces */
    uint8_t *have;  /* [(Ns+2)^d]                       trace computed */
    double *F;      /* [d][(Ns+1)][Ns^{d-1}][v]         time/face averaged sub-face fluxes */
    double *Fq;     /* [d][(Ns+1)][Ns^{d-1}][3^{d-1}][v] time-averaged flux at each tangential point */
} sc_work;

static void sc_alloc(const or_solver *S, sc_work *W) {
    int d = S->d, Ns = S->Ns, nv = S->nv;
    W->halo = malloc(sizeof(double) * nv * ipow(Ns + 6, d));
    W->tr = malloc(sizeof(double) * ipow(Ns + 2, d) * 2 * d * nv * ipow(3, d));
    W->have = malloc(ipow(Ns + 2, d));
    W->F = malloc(sizeof(double) * d * (Ns + 1) * ipow(Ns, d - 1) * nv);
    W->Fq = malloc(sizeof(double) * d * (Ns + 1) * ipow(Ns, d - 1) * ipow(3, d - 1) * nv);
}
static void sc_free(sc_work *W) { free(W->halo); free(W->tr); free(W->have); free(W->F); free(W->Fq); }

/* 1 if every point of q[v*npts + i] has finite values, rho > 0 and p > 0 */
static int all_physical(int d, double g, const double *q, int npts) {
    for (int i = 0; i < npts; i++) {
        double Q[5];
        for (int v = 0; v < d + 2; v++) {
            Q[v] = q[v * npts + i];
            if (!isfinite(Q[v])) return 0;
        }
        if (!(Q[0] > 0.0) || !(pressure(d, g, Q) > 0.0)) return 0;
    }
    return 1;
}

static int floordiv(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

/* Operator A of eq. (aderweno) for troubled cell c:
 *   1. initial/boundary data of eq. (ader.icbc) on the cell and on V_i (3-deep halo);
 *   2. WENO3 reconstruction, dimension by dimension, to nodal values at 3^d GL points;
 *   3. degree-2 local space-time predictor (same scheme as Sec. 2.2 with h/Ns);
 *   4. Rusanov on every sub-face at 3 GL points per tangential axis x 3 in time;
 *   5. one-step FV update of the subcell averages.
 * reading (scheme details are given in the paper's references, not in the paper):
 * steps 2-4 as stated; sub-faces on the domain boundary take the boundary ghost state of
 * the DG scheme.  Outputs vnew [v][nsub] and, on the cell's own faces, the time-averaged
 * flux at each tangential quadrature point of each sub-face,
 * sf[(2k+side)][v][nsubf][3^{d-1}] (consumed by the flux correction of Sec. 4.4). */
/* 1 if subcell (global cell gci, local subcell ms) carries a MOOD flag; cells outside a
 * non-periodic boundary and untroubled cells carry none. */
static int mood_flag(const or_solver *S, const uint8_t *flag, const uint8_t *troubled, const int *gci, const int *ms) {
    int ci[3] = {gci[0], gci[1], gci[2]};
    for (int k = 0; k < S->d; k++) {
        if (ci[k] < 0 || ci[k] >= S->nc[k]) {
            if (S->c.bc[k][0].kind[0] != OR_PERIODIC) return 0;
            ci[k] = (ci[k] + S->nc[k]) % S->nc[k];
        }
    }
    long cn = cell_index(S, ci);
    if (!troubled[cn]) return 0;
    return flag[cn * S->nsub + flat(ms, S->Ns, S->d)];
}

static void subcell_update(const or_solver *S, const double *vn, long c, double dt, sc_work *W, double *vnew,
                           double *sf, const uint8_t *flag, const uint8_t *troubled) {
    int d = S->d, Ns = S->Ns, nv = S->nv;
    double g = S->c.gamma, t = S->t;
    int ci[3];
    cell_coords(S, c, ci);
    int HN = Ns + 6, hsz = ipow(HN, d);
    /* 1. halo of subcell averages, local subcell coordinate L in [-3, Ns+2] */
    for (int hidx = 0; hidx < hsz; hidx++) {
        int hl[3] = {0, 0, 0}, gci[3] = {0, 0, 0}, gs[3] = {0, 0, 0};
        unflat(hidx, HN, d, hl);
        for (int k = 0; k < d; k++) {
            int L = hl[k] - 3;
            int off = floordiv(L, Ns);
            gci[k] = ci[k] + off;
            gs[k] = L - off * Ns;
        }
        double q[5];
        subcell_value(S, vn, gci, gs, t, q);
        for (int v = 0; v < nv; v++) W->halo[v * hsz + hidx] = q[v];
    }
    /* 2-3. reconstruction + predictor on the cell's subcells and the face-adjacent ring */
    int PN = Ns + 2, psz = ipow(PN, d);
    int nn3 = ipow(3, d), nfn3 = ipow(3, d - 1);
    int trsz = 2 * d * nv * nfn3 * 3;
    memset(W->have, 0, psz);
    double Y[5 * 27], q3[5 * 81], Fw[5 * 81], Vw[5 * 81];
    double dth[3];
    for (int k = 0; k < d; k++) dth[k] = dt * Ns / S->h[k];
    for (int pidx = 0; pidx < psz; pidx++) {
        int pl[3] = {0, 0, 0};
        unflat(pidx, PN, d, pl);
        int nout = 0, oax = -1, oside = 0;
        for (int k = 0; k < d; k++) {
            int L = pl[k] - 1;
            if (L < 0 || L >= Ns) { nout++; oax = k; oside = L >= Ns; }
        }
        if (nout > 1) continue;
        if (nout == 1) {
            int nb = ci[oax] + (oside ? 1 : -1);
            if ((nb < 0 || nb >= S->nc[oax]) && S->c.bc[oax][oside].kind[0] != OR_PERIODIC) continue;
            int f[3] = {ci[0], ci[1], ci[2]};
            f[oax] = nb;
            if (solid_at(S, f)) continue;   /* a wall: no subcells beyond it */
        }
        /* dimension-by-dimension WENO: work array with axes < k reconstructed (size 3,
         * node index) and axes >= k still stencil offsets (size 5). */
        double work[2][5 * 125];
        int cur = 0;
        for (int v = 0; v < nv; v++)
            for (int e = 0; e < ipow(5, d); e++) {
                int mo[3] = {0, 0, 0}, hl[3] = {0, 0, 0};
                unflat(e, 5, d, mo);
                for (int k = 0; k < d; k++) hl[k] = (pl[k] - 1) + (mo[k] - 2) + 3;
                work[0][v * 125 + e] = W->halo[v * hsz + flat(hl, HN, d)];
            }
        for (int k = 0; k < d; k++) {
            /* dims before: axes < k size 3, axes >= k size 5 ; after: axis k size 3 */
            int dimsb[3], dimsa[3];
            for (int j = 0; j < d; j++) { dimsb[j] = j < k ? 3 : 5; dimsa[j] = j <= k ? 3 : 5; }
            int na = 1;
            for (int j = 0; j < d; j++) na *= dimsa[j];
            for (int v = 0; v < nv; v++)
                for (int e = 0; e < na; e++) {
                    int ma[3] = {0, 0, 0}, r = e;
                    for (int j = 0; j < d; j++) { ma[j] = r % dimsa[j]; r /= dimsa[j]; }
                    if (ma[k] != 0) continue;  /* handle each line once */
                    double a5[5], o3[3];
                    for (int o = 0; o < 5; o++) {
                        int mb[3] = {ma[0], ma[1], ma[2]};
                        mb[k] = o;
                        int ib = 0;
                        for (int j = d - 1; j >= 0; j--) ib = ib * dimsb[j] + mb[j];
                        a5[o] = work[cur][v * 125 + ib];
                    }
                    weno3_1d(S->wenoinv, S->B3.xi, a5, o3);
                    for (int qn = 0; qn < 3; qn++) {
                        int mc[3] = {ma[0], ma[1], ma[2]};
                        mc[k] = qn;
                        int ic = 0;
                        for (int j = d - 1; j >= 0; j--) ic = ic * dimsa[j] + mc[j];
                        work[1 - cur][v * 125 + ic] = o3[qn];
                    }
                }
            cur = 1 - cur;
        }
        for (int v = 0; v < nv; v++)
            for (int a = 0; a < nn3; a++) Y[v * nn3 + a] = work[cur][v * 125 + a];
        predictor(&S->B3, d, nv, g, dth, 3, Y, q3, Fw, Vw);
        traces(&S->B3, d, nv, q3, W->tr + (long)pidx * trsz);
        W->have[pidx] = 1;
    }
    /* 4. sub-face fluxes */
    int nsf = S->nsubf;
    for (int k = 0; k < d; k++)
        for (int f = 0; f <= Ns; f++)
            for (int sp = 0; sp < nsf; sp++) {
                int mp[3] = {0, 0, 0};
                unflat(sp, Ns, d - 1, mp);
                int pL[3] = {0, 0, 0}, pR[3] = {0, 0, 0}, j2 = 0;
                for (int j = 0; j < d; j++) {
                    if (j == k) { pL[j] = f - 1 + 1; pR[j] = f + 1; }
                    else { pL[j] = pR[j] = mp[j2++] + 1; }
                }
                int iL = flat(pL, PN, d), iR = flat(pR, PN, d);
                int bside = -1, bwall = 0;
                if (f == 0 && !W->have[iL]) bside = 0;
                if (f == Ns && !W->have[iR]) bside = 1;
                if (bside >= 0) {
                    int fc[3] = {ci[0], ci[1], ci[2]};
                    fc[k] += bside ? 1 : -1;
                    const int inside = (fc[k] >= 0 && fc[k] < S->nc[k]) || S->c.bc[k][bside].kind[0] == OR_PERIODIC;
                    bwall = inside && solid_at(S, fc);
                }
                const double *trL = W->tr + (long)iL * trsz + (long)(2 * k + 1) * nv * nfn3 * 3;
                const double *trR = W->tr + (long)iR * trsz + (long)(2 * k + 0) * nv * nfn3 * 3;
                /* subcell averages on both sides (halo coordinates) */
                double avL[5], avR[5];
                {
                    int hL[3], hR[3];
                    for (int j = 0; j < d; j++) { hL[j] = pL[j] - 1 + 3; hR[j] = pR[j] - 1 + 3; }
                    for (int v = 0; v < nv; v++) {
                        avL[v] = W->halo[v * hsz + flat(hL, HN, d)];
                        avR[v] = W->halo[v * hsz + flat(hR, HN, d)];
                    }
                }
                /* reading (positivity safeguard; the paper leaves the subcell scheme to its
                 * references and notes that WENO3 may fail positivity): if any predictor
                 * trace on either side of the sub-face is not a physical state, the
                 * sub-face takes the first-order flux of the two subcell averages.
                 * MOOD layer (Sec. 6, Fig. algo2): a sub-face next to a subcell whose WENO3
                 * candidate failed the detection takes that first-order flux too. */
                int low = 0;
                if (flag) {
                    int gL[3] = {ci[0], ci[1], ci[2]}, gR[3] = {ci[0], ci[1], ci[2]};
                    int mL[3] = {0, 0, 0}, mR[3] = {0, 0, 0};
                    for (int j = 0; j < d; j++) { mL[j] = pL[j] - 1; mR[j] = pR[j] - 1; }
                    if (mL[k] < 0) { gL[k] -= 1; mL[k] += Ns; }
                    if (mR[k] >= Ns) { gR[k] += 1; mR[k] -= Ns; }
                    low = mood_flag(S, flag, troubled, gL, mL) || mood_flag(S, flag, troubled, gR, mR);
                }
                double Fbar[5] = {0, 0, 0, 0, 0};
                double *Fq = W->Fq + (((long)k * (Ns + 1) + f) * nsf + sp) * nfn3 * nv;
                for (int pass = low; pass < 2; pass++) {
                    int ok = 1;
                    for (int v = 0; v < nv; v++) Fbar[v] = 0.0;
                    for (int i = 0; i < nfn3 * nv; i++) Fq[i] = 0.0;
                    for (int s = 0; s < 3 && ok; s++)
                        for (int ap = 0; ap < nfn3; ap++) {
                            double qL[5], qR[5], G[5];
                            int ma[3] = {0, 0, 0};
                            unflat(ap, 3, d - 1, ma);
                            double wt = S->B3.w[s];
                            double x[3];
                            int j3 = 0;
                            for (int j = 0; j < d; j++) {
                                if (j == k) x[j] = S->c.lo[j] + S->h[j] * (ci[j] + (double)f / Ns);
                                else {
                                    int sj = mp[j3];
                                    wt *= S->B3.w[ma[j3]];
                                    x[j] = S->c.lo[j] + S->h[j] * (ci[j] + (sj + S->B3.xi[ma[j3]]) / Ns);
                                    j3++;
                                }
                            }
                            double tn = t + S->B3.xi[s] * dt;
                            for (int v = 0; v < nv; v++) {
                                qL[v] = pass ? avL[v] : trL[v * nfn3 * 3 + ap + nfn3 * s];
                                qR[v] = pass ? avR[v] : trR[v * nfn3 * 3 + ap + nfn3 * s];
                            }
                            if (bwall) {   /* reflective wall of the masked geometry */
                                double *qg = bside ? qR : qL;
                                const double *qi = bside ? qL : qR;
                                for (int v = 0; v < nv; v++) qg[v] = qi[v];
                                qg[1 + k] = -qg[1 + k];
                            } else if (bside == 0) bc_ghost(S, k, 0, qR, x, tn, qL);
                            else if (bside == 1) bc_ghost(S, k, 1, qL, x, tn, qR);
                            if (!pass && !(all_physical(d, g, qL, 1) && all_physical(d, g, qR, 1))) { ok = 0; break; }
                            /* the scheme's flux on the traces; first-order fallbacks use Rusanov */
                            if (pass) rusanov(d, k, g, qL, qR, G);
                            else num_flux(S, k, qL, qR, G);
                            for (int v = 0; v < nv; v++) {
                                Fbar[v] += wt * G[v];
                                Fq[ap * nv + v] += S->B3.w[s] * G[v];
                            }
                        }
                    if (ok) break;
                }
                for (int v = 0; v < nv; v++) W->F[(((long)k * (Ns + 1) + f) * nsf + sp) * nv + v] = Fbar[v];
            }
    /* 5. FV update */
    for (int sg = 0; sg < S->nsub; sg++) {
        int ms[3] = {0, 0, 0};
        unflat(sg, Ns, d, ms);
        for (int v = 0; v < nv; v++) {
            int hl[3];
            for (int k = 0; k < d; k++) hl[k] = ms[k] + 3;
            double acc = W->halo[v * hsz + flat(hl, HN, d)];
            for (int k = 0; k < d; k++) {
                int sp = strip_axis(ms, k, Ns, d);
                double Fp = W->F[(((long)k * (Ns + 1) + ms[k] + 1) * nsf + sp) * nv + v];
                double Fm = W->F[(((long)k * (Ns + 1) + ms[k]) * nsf + sp) * nv + v];
                acc -= dth[k] * (Fp - Fm);
            }
            vnew[v * S->nsub + sg] = acc;
        }
    }
    for (int k = 0; k < d; k++)
        for (int side = 0; side < 2; side++)
            for (int v = 0; v < nv; v++)
                for (int sp = 0; sp < nsf; sp++)
                    for (int ap = 0; ap < nfn3; ap++)
                        sf[(((2 * k + side) * nv + v) * nsf + sp) * nfn3 + ap] =
                            W->Fq[((((long)k * (Ns + 1) + (side ? Ns : 0)) * nsf + sp) * nfn3 + ap) * nv + v];
}

/* --------------------------------------------------------------- the step */
/* Sec. 4.4, the five steps: (1) unlimited ADER-DG candidate, (2) scatter P, (3) detection,
 * (4) subcell ADER-WENO3 recompute of troubled cells with flux correction of their
 * unlimited neighbours, (5) gather R.  Returns the number of troubled cells. */
int or_step(or_solver *S, double dt) {
    int d = S->d, n = S->n, nv = S->nv, nn = S->nn, nst = S->nst, nfn = S->nfn, Ns = S->Ns;
    long ncell = S->ncell;
    double g = S->c.gamma, t = S->t;
    double dth[3];
    for (int k = 0; k < d; k++) dth[k] = dt / S->h[k];
    const basis_t *B = &S->B;

    /* old-time subcell data and DMP bounds */
    double *vn = old_subcell_data(S);
    if (S->c.limiter) neighbourhood_bounds(S, vn, t, S->bmin, S->bmax);

    /* predictor, volume term, traces */
    long trsz = 2L * d * nv * nfn * n;
    double *tr = malloc(sizeof(double) * ncell * trsz);
    double *ustar = malloc(sizeof(double) * nv * ncell * nn);
#pragma omp parallel
    {
        double *ucell = malloc(sizeof(double) * nv * nn);
        double *q = malloc(sizeof(double) * nv * nst);
        double *F = malloc(sizeof(double) * nv * nst);
        double *V = malloc(sizeof(double) * nv * nst);
#pragma omp for schedule(dynamic, 4)
        for (long c = 0; c < ncell; c++) {
            for (int v = 0; v < nv; v++)
                for (int a = 0; a < nn; a++) ucell[v * nn + a] = S->u[((long)v * ncell + c) * nn + a];
            if (S->solid && S->solid[c]) {   /* solid: state kept, traces never read */
                for (int v = 0; v < nv; v++)
                    for (int a = 0; a < nn; a++) ustar[((long)v * ncell + c) * nn + a] = ucell[v * nn + a];
                continue;
            }
            predictor(B, d, nv, g, dth, S->c.picard_iters, ucell, q, F, V);
            traces(B, d, nv, q, tr + c * trsz);
            /* volume term of eq. (pde.nc.gw2), divided by the diagonal mass h^d W_a:
             *   (dt/h_k)(1/w_{a_k}) sum_s w_s sum_b w_b D[b][a_k] F_k(q at a with a_k<-b, s) */
            for (int v = 0; v < nv; v++)
                for (int a = 0; a < nn; a++) ustar[((long)v * ncell + c) * nn + a] = ucell[v * nn + a];
            for (int k = 0; k < d; k++)
                for (int s = 0; s < n; s++)
                    for (int a = 0; a < nn; a++) {
                        int m[3];
                        unflat(a, n, d, m);
                        int ak = m[k];
                        double acc[5] = {0, 0, 0, 0, 0};
                        for (int b = 0; b < n; b++) {
                            m[k] = b;
                            double Q[5], Fk[5];
                            int p = flat(m, n, d) + nn * s;
                            for (int v = 0; v < nv; v++) Q[v] = q[v * nst + p];
                            euler_flux(d, k, g, Q, Fk);
                            for (int v = 0; v < nv; v++) acc[v] += B->w[b] * B->D[b][ak] * Fk[v];
                        }
                        m[k] = ak;
                        for (int v = 0; v < nv; v++)
                            ustar[((long)v * ncell + c) * nn + a] += dth[k] / B->w[ak] * B->w[s] * acc[v];
                    }
        }
        free(ucell); free(q); free(F); free(V);
    }

    /* face fluxes, time-integrated: gbar[c][2k+side][v][a_perp] = sum_s w_s G */
    long gsz = 2L * d * nv * nfn;
    double *gbar = malloc(sizeof(double) * ncell * gsz);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < ncell; c++) {
        int ci[3];
        cell_coords(S, c, ci);
        for (int k = 0; k < d; k++) {
            /* the k- face of c; and the k+ face too when it is a non-periodic boundary */
            for (int side = 0; side < 2; side++) {
                int nb[3] = {ci[0], ci[1], ci[2]};
                nb[k] += side ? 1 : -1;
                int boundary = nb[k] < 0 || nb[k] >= S->nc[k];
                int periodic = S->c.bc[k][side].kind[0] == OR_PERIODIC;
                if (S->solid && S->solid[c]) continue;
                if (boundary && periodic) nb[k] = (nb[k] + S->nc[k]) % S->nc[k];
                /* a fluid cell's face toward a solid cell is a reflective wall (masked geometry) */
                const int wall = !(boundary && !periodic) && S->solid && S->solid[cell_index(S, nb)];
                if (side == 1 && !(boundary && !periodic) && !wall) continue;
                long cn = (boundary && !periodic) || wall ? -1 : cell_index(S, nb);
                for (int ap = 0; ap < nfn; ap++) {
                    double acc[5] = {0, 0, 0, 0, 0};
                    int mp[3] = {0, 0, 0};
                    unflat(ap, n, d - 1, mp);
                    for (int s = 0; s < n; s++) {
                        double qin[5], qout[5], G[5];
                        /* trace of c on this face */
                        for (int v = 0; v < nv; v++)
                            qin[v] = tr[c * trsz + ((2 * k + side) * nv + v) * nfn * n + ap + nfn * s];
                        if (wall) {
                            for (int v = 0; v < nv; v++) qout[v] = qin[v];
                            qout[1 + k] = -qout[1 + k];
                        } else if (cn < 0) {
                            double x[3];
                            int j2 = 0;
                            for (int j = 0; j < d; j++)
                                x[j] = (j == k) ? S->c.lo[j] + S->h[j] * (ci[j] + side)
                                                : S->c.lo[j] + S->h[j] * (ci[j] + B->xi[mp[j2++]]);
                            bc_ghost(S, k, side, qin, x, t + B->xi[s] * dt, qout);
                        } else {
                            for (int v = 0; v < nv; v++)
                                qout[v] = tr[cn * trsz + ((2 * k + 1 - side) * nv + v) * nfn * n + ap + nfn * s];
                        }
                        if (side == 0) num_flux(S, k, qout, qin, G);
                        else num_flux(S, k, qin, qout, G);
                        for (int v = 0; v < nv; v++) acc[v] += B->w[s] * G[v];
                    }
                    for (int v = 0; v < nv; v++) gbar[c * gsz + ((2 * k + side) * nv + v) * nfn + ap] = acc[v];
                }
            }
        }
    }
    /* copy each interior face flux to the other cell (its k+ face) */
#pragma omp parallel for schedule(static)
    for (long c = 0; c < ncell; c++) {
        int ci[3];
        cell_coords(S, c, ci);
        for (int k = 0; k < d; k++) {
            int nb[3] = {ci[0], ci[1], ci[2]};
            nb[k] += 1;
            int boundary = nb[k] >= S->nc[k];
            int periodic = S->c.bc[k][1].kind[0] == OR_PERIODIC;
            if (boundary && !periodic) continue;
            if (boundary) nb[k] = 0;
            long cn = cell_index(S, nb);
            if (S->solid && (S->solid[c] || S->solid[cn])) continue;   /* wall: computed by c itself */
            for (int v = 0; v < nv; v++)
                for (int ap = 0; ap < nfn; ap++)
                    gbar[c * gsz + ((2 * k + 1) * nv + v) * nfn + ap] = gbar[cn * gsz + ((2 * k + 0) * nv + v) * nfn + ap];
        }
    }
    /* candidate: face terms of eq. (pde.nc.gw2) with the diagonal mass divided out */
#pragma omp parallel for schedule(static)
    for (long c = 0; c < ncell; c++)
        for (int a = 0; a < nn; a++) {
            if (S->solid && S->solid[c]) break;
            int m[3];
            unflat(a, n, d, m);
            for (int k = 0; k < d; k++) {
                int ap = strip_axis(m, k, n, d);
                int ak = m[k];
                for (int v = 0; v < nv; v++) {
                    double Gm = gbar[c * gsz + ((2 * k + 0) * nv + v) * nfn + ap];
                    double Gp = gbar[c * gsz + ((2 * k + 1) * nv + v) * nfn + ap];
                    ustar[((long)v * ncell + c) * nn + a] += dth[k] / B->w[ak] * (B->L[ak] * Gm - B->R[ak] * Gp);
                }
            }
        }

    if (S->poison_cell >= 0) {
        for (int a = 0; a < nn; a++) ustar[((long)S->poison_var * ncell + S->poison_cell) * nn + a] = S->poison_value;
        S->poison_cell = -1;
    }

    if (!S->c.limiter) {
        memcpy(S->u, ustar, sizeof(double) * nv * ncell * nn);
        free(vn); free(tr); free(ustar); free(gbar);
        S->t += dt;
        return 0;
    }

    /* scatter + detection (steps 2 and 3) */
    uint8_t *bnew = malloc(ncell);
    int count = 0;
#pragma omp parallel
    {
        double *vs = malloc(sizeof(double) * nv * S->nsub);
#pragma omp for schedule(static) reduction(+ : count)
        for (long c = 0; c < ncell; c++) {
            apply_P(S, ustar + c * nn, ncell * nn, vs, S->nsub);
            double m[5], M[5];
            for (int v = 0; v < nv; v++) { m[v] = S->bmin[v * ncell + c]; M[v] = S->bmax[v * ncell + c]; }
            int bad = detect_cell(S, vs, m, M, &S->margin[c]);
            bnew[c] = (uint8_t)(bad || S->force[c]);
            if (S->solid && S->solid[c]) { bnew[c] = 0; S->margin[c] = INFINITY; }
            count += bnew[c];
        }
        free(vs);
    }

    /* step 4: subcell recompute */
    long nsf = S->nsubf;
    const int nfn3 = ipow(3, d - 1);
    const long sfsz = 2L * d * nv * nsf * nfn3;   /* per cell: [2d][v][sub-face][tangential point] */
    double *vnew = malloc(sizeof(double) * nv * ncell * S->nsub);
    double *sf = malloc(sizeof(double) * ncell * sfsz);
    long nonphys = 0;
#pragma omp parallel
    {
        sc_work W;
        sc_alloc(S, &W);
        double *vc = malloc(sizeof(double) * nv * S->nsub);
#pragma omp for schedule(dynamic, 1)
        for (long c = 0; c < ncell; c++) {
            if (!bnew[c]) continue;
            subcell_update(S, vn, c, dt, &W, vc, sf + c * sfsz, NULL, NULL);
            for (int v = 0; v < nv; v++)
                memcpy(vnew + ((long)v * ncell + c) * S->nsub, vc + v * S->nsub, sizeof(double) * S->nsub);
        }
        free(vc);
        sc_free(&W);
    }

    /* MOOD layer after the subcell scheme (Sec. 6, Fig. algo2).  reading: the WENO3
     * candidate of a troubled cell is tested subcell by subcell with the criteria of Sec.
     * 4.3 (PAD, and the relaxed DMP against that cell's bounds of eq. (dmp)); every
     * troubled cell with a flagged subcell on or next to its sub-faces is recomputed with
     * the first-order flux of the subcell averages on each sub-face adjacent to a flagged
     * subcell (adjacent troubled cells then agree on their shared sub-faces: conservative). */
    if (S->c.mood) {
        const int nsub = S->nsub;
        uint8_t *flag = calloc((size_t)ncell * nsub, 1);
        uint8_t *redo = calloc((size_t)ncell, 1);
#pragma omp parallel for schedule(static)
        for (long c = 0; c < ncell; c++) {
            if (!bnew[c]) continue;
            for (int sg = 0; sg < nsub; sg++) {
                double q[5];
                int bad = 0;
                for (int v = 0; v < nv; v++) {
                    q[v] = vnew[((long)v * ncell + c) * nsub + sg];
                    if (!isfinite(q[v])) bad = 1;
                }
                if (!bad && (!(q[0] > 0) || !(pressure(d, g, q) > 0))) bad = 1;
                for (int v = 0; v < nv && !bad; v++) {
                    double m = S->bmin[v * ncell + c], M = S->bmax[v * ncell + c];
                    double delta = fmax(S->c.delta0, S->c.eps * (M - m));
                    if (q[v] < m - delta || q[v] > M + delta) bad = 1;
                }
                flag[c * nsub + sg] = (uint8_t)bad;
            }
        }
        /* cells to recompute: a flagged subcell of their own or on a neighbour's face layer */
#pragma omp parallel for schedule(static)
        for (long c = 0; c < ncell; c++) {
            if (!bnew[c]) continue;
            int any = 0;
            for (int sg = 0; sg < nsub && !any; sg++) any = flag[c * nsub + sg];
            int ci[3];
            cell_coords(S, c, ci);
            for (int k = 0; k < d && !any; k++)
                for (int side = 0; side < 2 && !any; side++) {
                    int gci[3] = {ci[0], ci[1], ci[2]};
                    gci[k] += side ? 1 : -1;
                    for (int sp = 0; sp < S->nsubf && !any; sp++) {
                        int mp[3] = {0, 0, 0}, ms[3] = {0, 0, 0}, j2 = 0;
                        unflat(sp, Ns, d - 1, mp);
                        for (int j = 0; j < d; j++) ms[j] = (j == k) ? (side ? 0 : Ns - 1) : mp[j2++];
                        any = mood_flag(S, flag, bnew, gci, ms);
                    }
                }
            redo[c] = (uint8_t)any;
        }
#pragma omp parallel
        {
            sc_work W;
            sc_alloc(S, &W);
            double *vc = malloc(sizeof(double) * nv * nsub);
#pragma omp for schedule(dynamic, 1)
            for (long c = 0; c < ncell; c++) {
                if (!redo[c]) continue;
                subcell_update(S, vn, c, dt, &W, vc, sf + c * sfsz, flag, bnew);
                for (int v = 0; v < nv; v++)
                    memcpy(vnew + ((long)v * ncell + c) * nsub, vc + v * nsub, sizeof(double) * nsub);
            }
            free(vc);
            sc_free(&W);
        }
        long nf = 0, nr = 0;
        for (long i = 0; i < ncell * (long)nsub; i++) nf += flag[i];
        for (long c = 0; c < ncell; c++) nr += redo[c];
        S->mood_flagged = nf;
        S->mood_redone = nr;
        free(flag);
        free(redo);
    }
    /* subcell results that fail PAD (counted, not corrected) */
    for (long c = 0; c < ncell; c++) {
        if (!bnew[c]) continue;
        for (int sg = 0; sg < S->nsub; sg++) {
            double q[5];
            for (int v = 0; v < nv; v++) q[v] = vnew[((long)v * ncell + c) * S->nsub + sg];
            if (!(q[0] > 0) || !(pressure(d, g, q) > 0)) { nonphys++; break; }
        }
    }
    S->nonphys += nonphys;

    /* flux correction of unlimited cells next to troubled cells (Sec. 4.4): the DG face
     * integral becomes the sum of the integrals over the sub-faces, with the subcell
     * scheme's flux.  Remove the DG face flux and add, for each basis function, the
     * integral over each sub-face of the subcell flux times that basis function: the flux
     * at the 3 Gauss-Legendre points per tangential axis (time-averaged) times the
     * tangential basis there, with the quadrature weights (w3/Ns per axis).  The mean
     * moment receives the sub-face averages that the troubled cell's update used, so the
     * step stays conservative. */
    double phi3[MAXNS][3][MAXN];   /* phi3[sigma][g][m] = phi_m((sigma + xi3_g)/Ns) */
    for (int sg = 0; sg < Ns; sg++)
        for (int gq = 0; gq < 3; gq++)
            for (int m = 0; m < n; m++) phi3[sg][gq][m] = lagrange(n, B->xi, m, (sg + S->B3.xi[gq]) / Ns);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < ncell; c++) {
        if (bnew[c] || (S->solid && S->solid[c])) continue;
        int ci[3];
        cell_coords(S, c, ci);
        for (int k = 0; k < d; k++)
            for (int side = 0; side < 2; side++) {
                int nb[3] = {ci[0], ci[1], ci[2]};
                nb[k] += side ? 1 : -1;
                if (nb[k] < 0 || nb[k] >= S->nc[k]) {
                    if (S->c.bc[k][side].kind[0] != OR_PERIODIC) continue;
                    nb[k] = (nb[k] + S->nc[k]) % S->nc[k];
                }
                long cn = cell_index(S, nb);
                if (!bnew[cn]) continue;
                const double *fs = sf + cn * sfsz + (long)(2 * k + (1 - side)) * nv * nsf * nfn3;
                for (int a = 0; a < nn; a++) {
                    int m[3];
                    unflat(a, n, d, m);
                    int ap = strip_axis(m, k, n, d);
                    int ak = m[k];
                    for (int v = 0; v < nv; v++) {
                        double Fsub = 0;
                        for (int sp = 0; sp < nsf; sp++) {
                            int ms[3] = {0, 0, 0};
                            unflat(sp, Ns, d - 1, ms);
                            for (int gp = 0; gp < nfn3; gp++) {
                                int mg[3] = {0, 0, 0};
                                unflat(gp, 3, d - 1, mg);
                                double wgt = 1;
                                int j2 = 0;
                                for (int j = 0; j < d; j++) {
                                    if (j == k) continue;
                                    wgt *= S->B3.w[mg[j2]] / Ns * phi3[ms[j2]][mg[j2]][m[j]] / B->w[m[j]];
                                    j2++;
                                }
                                Fsub += wgt * fs[(v * nsf + sp) * nfn3 + gp];
                            }
                        }
                        double Gdg = gbar[c * gsz + ((2 * k + side) * nv + v) * nfn + ap];
                        double corr = side ? dth[k] * B->R[ak] / B->w[ak] * (Gdg - Fsub)
                                           : dth[k] * B->L[ak] / B->w[ak] * (Fsub - Gdg);
                        ustar[((long)v * ncell + c) * nn + a] += corr;
                    }
                }
            }
    }

    /* step 5: gather; store the subcell data of troubled cells for the next step */
#pragma omp parallel for schedule(static)
    for (long c = 0; c < ncell; c++) {
        if (!bnew[c]) continue;
        apply_R(S, vnew + c * S->nsub, ncell * S->nsub, ustar + c * nn, ncell * nn);
        for (int v = 0; v < nv; v++)
            memcpy(S->vstore + ((long)v * ncell + c) * S->nsub, vnew + ((long)v * ncell + c) * S->nsub,
                   sizeof(double) * S->nsub);
    }
    memcpy(S->u, ustar, sizeof(double) * nv * ncell * nn);
    memcpy(S->beta, bnew, ncell);
    S->t += dt;
    free(vn); free(tr); free(ustar); free(gbar); free(bnew); free(vnew); free(sf);
    return count;
}

/* ----------------------------------------------- exact Riemann solver (tests) */
/* Exact solution of the 1D Riemann problem for the ideal-gas Euler equations by the
 * pressure-function Newton method of Toro's textbook (cited by the paper for the shock
 * tubes of Sec. 5).  out[3*i..] = (rho, u, p) at similarity coordinate s[i] = x/t. */
static void rp_f(double p, double rk, double pk, double ck, double g, double *f, double *df) {
    if (p > pk) {
        double A = 2.0 / ((g + 1.0) * rk), Bk = (g - 1.0) / (g + 1.0) * pk;
        double sq = sqrt(A / (p + Bk));
        *f = (p - pk) * sq;
        *df = sq * (1.0 - 0.5 * (p - pk) / (p + Bk));
    } else {
        double pr = p / pk;
        *f = 2.0 * ck / (g - 1.0) * (pow(pr, (g - 1.0) / (2.0 * g)) - 1.0);
        *df = 1.0 / (rk * ck) * pow(pr, -(g + 1.0) / (2.0 * g));
    }
}

void or_exact_riemann(double rl, double ul, double pl, double rr, double ur, double pr, double g,
                      const double *s, int m, double *out, double *ps_us) {
    double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
    /* two-rarefaction initial guess */
    double z = (g - 1.0) / (2.0 * g);
    double p = pow((cl + cr - 0.5 * (g - 1.0) * (ur - ul)) / (cl / pow(pl, z) + cr / pow(pr, z)), 1.0 / z);
    if (!(p > 1e-12)) p = 1e-12;
    for (int it = 0; it < 200; it++) {
        double fl, dfl, fr, dfr;
        rp_f(p, rl, pl, cl, g, &fl, &dfl);
        rp_f(p, rr, pr, cr, g, &fr, &dfr);
        double f = fl + fr + (ur - ul);
        double pn = p - f / (dfl + dfr);
        if (pn < 1e-14) pn = 1e-14;
        double ch = 2.0 * fabs(pn - p) / (pn + p);
        p = pn;
        if (ch < 1e-15) break;
    }
    double fl, dfl, fr, dfr;
    rp_f(p, rl, pl, cl, g, &fl, &dfl);
    rp_f(p, rr, pr, cr, g, &fr, &dfr);
    double us = 0.5 * (ul + ur) + 0.5 * (fr - fl);
    if (ps_us) { ps_us[0] = p; ps_us[1] = us; }
    double gm = (g - 1.0) / (g + 1.0);
    for (int i = 0; i < m; i++) {
        double S = s[i], rho, u, pp;
        if (S <= us) {  /* left of contact */
            if (p > pl) {
                double SL = ul - cl * sqrt((g + 1.0) / (2.0 * g) * p / pl + (g - 1.0) / (2.0 * g));
                if (S <= SL) { rho = rl; u = ul; pp = pl; }
                else { rho = rl * ((p / pl + gm) / (gm * p / pl + 1.0)); u = us; pp = p; }
            } else {
                double SHL = ul - cl, cls = cl * pow(p / pl, z), STL = us - cls;
                if (S <= SHL) { rho = rl; u = ul; pp = pl; }
                else if (S > STL) { rho = rl * pow(p / pl, 1.0 / g); u = us; pp = p; }
                else {
                    u = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + S);
                    double c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - S));
                    rho = rl * pow(c / cl, 2.0 / (g - 1.0));
                    pp = pl * pow(c / cl, 2.0 * g / (g - 1.0));
                }
            }
        } else {        /* right of contact */
            if (p > pr) {
                double SR = ur + cr * sqrt((g + 1.0) / (2.0 * g) * p / pr + (g - 1.0) / (2.0 * g));
                if (S >= SR) { rho = rr; u = ur; pp = pr; }
                else { rho = rr * ((p / pr + gm) / (gm * p / pr + 1.0)); u = us; pp = p; }
            } else {
                double SHR = ur + cr, crs = cr * pow(p / pr, z), STR = us + crs;
                if (S >= SHR) { rho = rr; u = ur; pp = pr; }
                else if (S < STR) { rho = rr * pow(p / pr, 1.0 / g); u = us; pp = p; }
                else {
                    u = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + S);
                    double c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - S));
                    rho = rr * pow(c / cr, 2.0 / (g - 1.0));
                    pp = pr * pow(c / cr, 2.0 * g / (g - 1.0));
                }
            }
        }
        out[3 * i] = rho; out[3 * i + 1] = u; out[3 * i + 2] = pp;
    }
}
