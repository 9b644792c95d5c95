// Host-side operator tables in FP64 (Sec. 2.1, 2.2, 4.2 and the subcell WENO3 scheme).
// Gauss-Legendre points by Newton iteration on the Legendre three-term recurrence;
// Lagrange basis in barycentric form.
#include <cmath>
#include <cstring>
#include "adg_internal.h"

namespace adg {

int64_t ipow64(int64_t b, int e) {
    int64_t r = 1;
    while (e-- > 0) r *= b;
    return r;
}

// Gauss-Legendre nodes and weights on [0,1], ascending.
static void gl_newton(int n, double *x01, double *w01) {
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; i++) {
        double x = std::cos(pi * (n - i - 0.25) / (n + 0.5));  // ascending initial guesses
        double dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double pn = (n == 1) ? x : p1, pnm1 = (n == 1) ? 1.0 : p0;
            dp = n * (x * pn - pnm1) / (x * x - 1.0);
            double dx = pn / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-17) break;
        }
        // refresh derivative at the converged point
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; k++) {
            double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        double pn = (n == 1) ? x : p1, pnm1 = (n == 1) ? 1.0 : p0;
        dp = n * (x * pn - pnm1) / (x * x - 1.0);
        x01[i] = 0.5 * (x + 1.0);
        w01[i] = 1.0 / ((1.0 - x * x) * dp * dp);  // 2/((1-x^2)P'^2) halved for [0,1]
    }
}

struct Bary {
    int n;
    double x[MAXN], lam[MAXN];
    void init(int nn, const double *xs) {
        n = nn;
        for (int b = 0; b < n; b++) {
            x[b] = xs[b];
            double p = 1.0;
            for (int m = 0; m < n; m++)
                if (m != b) p *= (xs[b] - xs[m]);
            lam[b] = 1.0 / p;
        }
    }
    // values of all basis functions at t
    void eval(double t, double *phi) const {
        for (int b = 0; b < n; b++)
            if (t == x[b]) {
                for (int m = 0; m < n; m++) phi[m] = (m == b);
                return;
            }
        double s = 0;
        for (int m = 0; m < n; m++) s += lam[m] / (t - x[m]);
        for (int b = 0; b < n; b++) phi[b] = lam[b] / (t - x[b]) / s;
    }
    // D[a][b] = phi_b'(x_a)
    void diff(double D[][MAXN]) const {
        for (int a = 0; a < n; a++) {
            double diag = 0;
            for (int b = 0; b < n; b++) {
                if (a == b) continue;
                D[a][b] = (lam[b] / lam[a]) / (x[a] - x[b]);
                diag -= D[a][b];
            }
            D[a][a] = diag;
        }
    }
};

// LU with partial pivoting; solves A X = B for k right-hand sides (row-major, in place).
static bool lu_solve(int n, double *A, double *B, int k) {
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int r = c + 1; r < n; r++)
            if (std::fabs(A[r * n + c]) > std::fabs(A[p * n + c])) p = r;
        if (A[p * n + c] == 0.0) return false;
        if (p != c) {
            for (int j = 0; j < n; j++) std::swap(A[c * n + j], A[p * n + j]);
            for (int j = 0; j < k; j++) std::swap(B[c * k + j], B[p * k + j]);
        }
        for (int r = c + 1; r < n; r++) {
            double f = A[r * n + c] / A[c * n + c];
            for (int j = c; j < n; j++) A[r * n + j] -= f * A[c * n + j];
            for (int j = 0; j < k; j++) B[r * k + j] -= f * B[c * k + j];
        }
    }
    for (int c = n - 1; c >= 0; c--)
        for (int j = 0; j < k; j++) {
            double s = B[c * k + j];
            for (int m = c + 1; m < n; m++) s -= A[c * n + m] * B[m * k + j];
            B[c * k + j] = s / A[c * n + c];
        }
    return true;
}

// Time operator of eq. (pde.nc.dg2) in nodal form: K1 = R R^T - (diag(w) D)^T;
// Kw = K1^{-1} diag(w).
static void time_operator(int n, const double *w, const double D[][MAXN], const double *R, double Kw[][MAXN]) {
    double K1[MAXN * MAXN], B[MAXN * MAXN];
    for (int k = 0; k < n; k++)
        for (int l = 0; l < n; l++) {
            K1[k * n + l] = R[k] * R[l] - w[l] * D[l][k];
            B[k * n + l] = (k == l) ? w[l] : 0.0;
        }
    lu_solve(n, K1, B, n);
    for (int s = 0; s < n; s++)
        for (int t = 0; t < n; t++) Kw[s][t] = B[s * n + t];
}

void gl_nodes(int n, double *x01, double *w01) { gl_newton(n, x01, w01); }

void lagrange_values(int n, const double *xi, double t, double *phi) {
    Bary B;
    B.init(n, xi);
    B.eval(t, phi);
}

void build_tables(int N, int Ns, Tables *T) {
    std::memset(T, 0, sizeof(Tables));
    const int n = N + 1;
    gl_newton(n, T->xi, T->w);
    Bary B;
    B.init(n, T->xi);
    B.diff(T->D);
    B.eval(0.0, T->L);
    B.eval(1.0, T->R);
    time_operator(n, T->w, T->D, T->R, T->Kw);
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++) T->Dvol[a][b] = T->w[b] * T->D[b][a] / T->w[a];
    // eq. (subcell.p): P[s][l] = Ns * integral of phi_l over subinterval s
    for (int s = 0; s < Ns; s++) {
        double acc[MAXN] = {0};
        for (int q = 0; q < n; q++) {
            double phi[MAXN];
            B.eval((s + T->xi[q]) / Ns, phi);
            for (int l = 0; l < n; l++) acc[l] += T->w[q] * phi[l];
        }
        for (int l = 0; l < n; l++) T->P[s][l] = acc[l];
    }
    // eq. (subcell.r): least-squares reconstruction R = (P^T P)^{-1} P^T (with equal
    // subcells it conserves the cell mean, eq. (subcell.r.constraint))
    {
        double PtP[MAXN * MAXN], Pt[MAXN * MAXNS];
        for (int i = 0; i < n; i++) {
            for (int j = 0; j < n; j++) {
                double s = 0;
                for (int q = 0; q < Ns; q++) s += T->P[q][i] * T->P[q][j];
                PtP[i * n + j] = s;
            }
            for (int q = 0; q < Ns; q++) Pt[i * Ns + q] = T->P[q][i];
        }
        lu_solve(n, PtP, Pt, Ns);
        for (int i = 0; i < n; i++)
            for (int q = 0; q < Ns; q++) T->Rg[i][q] = Pt[i * Ns + q];
    }
    // degree-2 scheme on the subgrid
    gl_newton(3, T->xi3, T->w3);
    for (int s = 0; s < Ns; s++)
        for (int g = 0; g < 3; g++) {
            double phi[MAXN];
            B.eval((s + T->xi3[g]) / Ns, phi);
            for (int a = 0; a < n; a++) T->Pq[s * 3 + g][a] = T->w3[g] / Ns * phi[a] / T->w[a];
        }
    Bary B3;
    B3.init(3, T->xi3);
    B3.diff(T->D3);
    B3.eval(0.0, T->L3);
    B3.eval(1.0, T->R3);
    time_operator(3, T->w3, T->D3, T->R3, T->Kw3);
    {
        const int h = n / 2;
        for (int a = 0; a < h; a++)
            for (int b = 0; b < h; b++) {
                T->DE[a][b] = 0.5 * (T->D[a][b] + T->D[a][n - 1 - b]);
                T->DO[a][b] = 0.5 * (T->D[a][b] - T->D[a][n - 1 - b]);
            }
        if (n % 2) {
            for (int a = 0; a < h; a++) T->DE[a][h] = T->D[a][h];
            for (int b = 0; b < h; b++) T->DO[h][b] = T->D[h][b];
        }
        for (int a = 0; a <= MAXN / 2; a++)
            for (int b = 0; b <= MAXN / 2; b++) {
                if (a < MAXN / 2) T->fDE[a][b] = (float)T->DE[a][b];
                if (b < MAXN / 2) T->fDO[a][b] = (float)T->DO[a][b];
            }
    }
    for (int a = 0; a < 3; a++) {
        T->fL3[a] = (float)T->L3[a];
        T->fR3[a] = (float)T->R3[a];
        T->fw3[a] = (float)T->w3[a];
        T->fxi3[a] = (float)T->xi3[a];
        for (int b = 0; b < 3; b++) {
            T->fD3[a][b] = (float)T->D3[a][b];
            T->fKw3[a][b] = (float)T->Kw3[a][b];
        }
    }
    for (int a = 0; a < MAXN; a++) {
        T->fL[a] = (float)T->L[a];
        T->fR[a] = (float)T->R[a];
        T->fw[a] = (float)T->w[a];
        for (int b = 0; b < MAXN; b++) {
            T->fD[a][b] = (float)T->D[a][b];
            T->fKw[a][b] = (float)T->Kw[a][b];
            T->fDvol[a][b] = (float)T->Dvol[a][b];
        }
    }
    // WENO3 stencils {j-2..j}, {j-1..j+1}, {j..j+2}: the quadratic c0 + c1 x + c2 x^2 on
    // the central subcell (x in [0,1]) with the three given averages.
    for (int st = 0; st < 3; st++) {
        double A[9], Bm[9];
        for (int m = 0; m < 3; m++) {
            double o = st - 2 + m;
            for (int p = 0; p < 3; p++) A[m * 3 + p] = (std::pow(o + 1.0, p + 1) - std::pow(o, p + 1)) / (p + 1);
            for (int j = 0; j < 3; j++) Bm[m * 3 + j] = (m == j);
        }
        lu_solve(3, A, Bm, 3);
        for (int p = 0; p < 3; p++)
            for (int j = 0; j < 3; j++) {
                T->weno[st][p][j] = Bm[p * 3 + j];
                T->fweno[st][p][j] = (float)Bm[p * 3 + j];
            }
    }
}

}  // namespace adg
