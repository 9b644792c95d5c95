// Local space-time predictor (a point-owner / line-owner LDS design, see below).
#pragma once
#include <type_traits>

#include "adg_physics.h"

namespace adg {

// ------------------------------------------------------------- space-time predictor
// Eq. (pde.nc.dg2) in nodal form (spatial weights divided out, K1^{-1} L = 1):
//   q^{r+1}(a,s) = u(a) - sum_t Kw[s][t] S(a,t),
//   S(a,t) = sum_k (dt/h_k) sum_b D[a_k][b] F_k(q^r(a|b, t))
// Thread mapping: a "point owner" thread holds one spatial node of one cell with its
// whole time pencil (NV x n values) in registers.  It evaluates the fluxes of the pencil
// and stores them in LDS; "line owner" threads do the length-n spatial contractions
// (n loads -> n outputs each, in place); the point owner accumulates S over the d axes
// and applies the time contraction in registers: d + 1 contractions per sweep.
template <int DIM, int N, typename R = double, int TB = Tune<DIM, N, sizeof(R) == 4>::pred_tb>
struct PredShape;

// 1/x: correctly rounded division in FP64; the hardware reciprocal (within 1 ulp) in
// the FP32 working precision of the mixed form.
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// TB: thread budget of a workgroup (cells per block = TB / n^d)
template <int DIM, int N, typename R, int TB>
struct PredShape {
    static constexpr int n = N + 1;
    static constexpr int NV = DIM + 2;
    static constexpr int NN = cpow(n, DIM);
    static constexpr int NST = NN * n;
    static constexpr int NFN = cpow(n, DIM - 1);
    static constexpr int CPB = NN <= TB ? TB / NN : 1;
    static constexpr int ACT = CPB * NN;                           // active point owners
    static constexpr int BS = ((ACT + 63) / 64) * 64;
    static constexpr int VCMAX = 65536 / (CPB * NST * (int)sizeof(R));
    static constexpr int VC = VCMAX < 1 ? 1 : (VCMAX > NV ? NV : VCMAX);  // vars per LDS chunk
};

// Contraction along axis k of every line held in LDS: line[i] <- c * sum_b M[i][b] line[b]
// (c only if SCALE).  One work item handles the same line of LV variables (independent FMA
// chains sharing each operator entry; for long lines LV is 2 (FP32) or 1 (FP64) to bound
// register use).
// EO: M is the derivative matrix on symmetric nodes, applied through its even / odd parts
// E, O (half-size products on x_b +- x_{n-1-b}: n^2/2 + 2n operations instead of n^2).
template <int DIM, int N, int CPB, int VC, int BS, typename R, bool EO = false, bool SCALE = true>
__device__ __forceinline__ void lds_lines(R *X, int k, int nlines_per_var, int lstride_s, const R (*M)[MAXN], R c,
                                          int tid, int nvalid, const R (*E)[MAXN / 2 + 1] = nullptr,
                                          const R (*O)[MAXN / 2] = nullptr) {
    constexpr int n = N + 1, NN = cpow(n, DIM), NST = NN * n;
    constexpr int LV = (n >= 8) ? (sizeof(R) == 8 ? 1 : 2) : VC;
    constexpr int NG = (VC + LV - 1) / LV;   // variable groups per line
    const int st = (k == 0) ? 1 : (k == 1 ? n : n * n);
    const int nitems = CPB * NG * nlines_per_var;
    for (int it = tid; it < nitems; it += BS) {
        // compiler barrier: keeps the operator rows from being hoisted into registers
        __asm__ volatile("" ::: "memory");
        const int lcl = it / (NG * nlines_per_var);
        const int grp = (it / nlines_per_var) % NG;
        const int j = it % nlines_per_var;          // (a_perp, s) flattened, a_perp fastest
        const int s = j / (NN / n), ap = j % (NN / n);
        int base = 0, rem = ap, mul = 1;
#pragma unroll
        for (int jj = 0; jj < DIM; jj++) {
            if (jj == k) { mul *= n; continue; }
            base += (rem % n) * mul;
            rem /= n;
            mul *= n;
        }
        const int v0 = grp * LV;
        R *line0 = &X[(lcl * VC + v0) * NST + lstride_s * s + base];
        R xb[LV][n];
#pragma unroll
        for (int vv = 0; vv < LV; vv++)
#pragma unroll
            for (int b = 0; b < n; b++) xb[vv][b] = (v0 + vv < nvalid) ? line0[vv * NST + b * st] : R(0);
        if constexpr (EO) {
            constexpr int h = n / 2;
            R e[LV][h], o[LV][h];
#pragma unroll
            for (int vv = 0; vv < LV; vv++)
#pragma unroll
                for (int b = 0; b < h; b++) {
                    e[vv][b] = xb[vv][b] + xb[vv][n - 1 - b];
                    o[vv][b] = xb[vv][b] - xb[vv][n - 1 - b];
                }
#pragma unroll
            for (int i = 0; i < h; i++) {
                R pe[LV], po[LV];
#pragma unroll
                for (int vv = 0; vv < LV; vv++) pe[vv] = po[vv] = 0;
#pragma unroll
                for (int b = 0; b < h; b++) {
                    const R me = E[i][b], mo = O[i][b];
#pragma unroll
                    for (int vv = 0; vv < LV; vv++) {
                        pe[vv] += me * e[vv][b];
                        po[vv] += mo * o[vv][b];
                    }
                }
                if constexpr (n % 2) {
                    const R mm = E[i][h];
#pragma unroll
                    for (int vv = 0; vv < LV; vv++) pe[vv] += mm * xb[vv][h];
                }
#pragma unroll
                for (int vv = 0; vv < LV; vv++)
                    if (v0 + vv < nvalid) {
                        const R yi = po[vv] + pe[vv], yr = po[vv] - pe[vv];
                        line0[vv * NST + i * st] = SCALE ? c * yi : yi;
                        line0[vv * NST + (n - 1 - i) * st] = SCALE ? c * yr : yr;
                    }
            }
            if constexpr (n % 2) {
                R acc[LV];
#pragma unroll
                for (int vv = 0; vv < LV; vv++) acc[vv] = 0;
#pragma unroll
                for (int b = 0; b < h; b++) {
                    const R mo = O[h][b];
#pragma unroll
                    for (int vv = 0; vv < LV; vv++) acc[vv] += mo * o[vv][b];
                }
#pragma unroll
                for (int vv = 0; vv < LV; vv++)
                    if (v0 + vv < nvalid) line0[vv * NST + h * st] = SCALE ? c * acc[vv] : acc[vv];
            }
        } else {
#pragma unroll
            for (int i = 0; i < n; i++) {
                R acc[LV];
#pragma unroll
                for (int vv = 0; vv < LV; vv++) acc[vv] = 0;
#pragma unroll
                for (int b = 0; b < n; b++) {
                    const R m = M[i][b];
#pragma unroll
                    for (int vv = 0; vv < LV; vv++) acc[vv] += m * xb[vv][b];
                }
#pragma unroll
                for (int vv = 0; vv < LV; vv++)
                    if (v0 + vv < nvalid) line0[vv * NST + i * st] = SCALE ? c * acc[vv] : acc[vv];
            }
        }
    }
}

// Blocks vb = vb0, vb0 + vbs, ... of CPB cells each, out of ncell cells.
// DEV (FP32 working precision only): the pencils carry the deviation dq = q - c from the cell's
// reference state c (its first nodal value rounded to FP32) and the fluxes are evaluated as
// F(c + dq) - F(c) in the expanded form of dev_flux; the derivative matrix annihilates the
// constant F(c), so the Picard iteration, the volume term and the traces are those of the
// deviations, and FP32 rounding is relative to the deviation instead of the state.
template <int DIM, int N, bool VOL, typename R, bool DEV = false, int TB = Tune<DIM, N, sizeof(R) == 4>::pred_tb>
__device__ void pred_cells(const PredArgs<R> &A, double gamma_d, int64_t ncell, int64_t vb0, int64_t vbs) {
    static_assert(!DEV || sizeof(R) == 4, "the deviation form is an FP32 form");
    using S = PredShape<DIM, N, R, TB>;
    const R gamma = (R)gamma_d;
    constexpr int n = S::n, NV = S::NV, NN = S::NN, NST = S::NST, NFN = S::NFN, CPB = S::CPB, VC = S::VC;
    __shared__ R X[CPB * VC * NST];
    // operators staged in LDS and read as wave-uniform broadcasts inside the loops (kept
    // out of registers: the n x n matrices would otherwise be hoisted into VGPRs)
    __shared__ R Ds[n][MAXN], Kws[n][MAXN], Dvs[n][MAXN];
    // the spatial contractions use the even / odd form where it saves work (n >= 6)
    constexpr bool EO = n >= 6;
    __shared__ R Es[EO ? MAXN / 2 : 1][MAXN / 2 + 1], Os[EO ? MAXN / 2 + 1 : 1][MAXN / 2];

    const int tid = threadIdx.x;
    const int lc = tid / NN, a = tid % NN;
    const double dt = *A.dt;
    for (int i = tid; i < n * n; i += S::BS) {
        const int r = i / n, cc = i % n;
        Ds[r][cc] = A.D[r * MAXN + cc];
        Kws[r][cc] = A.Kw[r * MAXN + cc];
        Dvs[r][cc] = VOL ? A.Dvol[r * MAXN + cc] : R(0);
    }
    if constexpr (EO) {
        for (int i = tid; i < (MAXN / 2) * (MAXN / 2 + 1); i += S::BS) {
            Es[i / (MAXN / 2 + 1)][i % (MAXN / 2 + 1)] = A.DE[i];
            Os[i / (MAXN / 2)][i % (MAXN / 2)] = A.DO[i];
        }
    }
    __syncthreads();
    const R(*D)[MAXN] = Ds;
    const R(*Kw)[MAXN] = Kws;
    const R(*Dvol)[MAXN] = Dvs;
    // persistent over blocks of CPB cells (uniform per block: barriers stay legal)
    for (int64_t vb = vb0; vb * CPB < ncell; vb += vbs) {
    const int64_t c = vb * CPB + lc;
    const bool owner = (tid < S::ACT) && (c < ncell);

    R u0[NV], q[NV][n], Sacc[NV][n];
    DevRef<DIM, R> cref;
    if (owner) {
        if constexpr (DEV) {
            double c64[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) c64[v] = A.in[c * A.in_cstride + v * A.in_vstride];
            cref = make_devref<DIM, R>(c64, gamma_d);
#pragma unroll
            for (int v = 0; v < NV; v++) u0[v] = (R)(A.in[c * A.in_cstride + v * A.in_vstride + a] - (double)cref.q[v]);
        } else {
#pragma unroll
            for (int v = 0; v < NV; v++) u0[v] = (R)A.in[c * A.in_cstride + v * A.in_vstride + a];
        }
    } else {
        // idle lanes carry a valid constant state so that they never produce NaN
#pragma unroll
        for (int v = 0; v < NV; v++) u0[v] = (v == 0 && !DEV) ? R(1) : R(0);
        if constexpr (!DEV) u0[NV - 1] = R(2.5);
        if constexpr (DEV) {
            double c64[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) c64[v] = (v == 0) ? 1.0 : 0.0;
            c64[NV - 1] = 2.5;
            cref = make_devref<DIM, R>(c64, gamma_d);
        }
    }
#pragma unroll
    for (int v = 0; v < NV; v++)
#pragma unroll
        for (int s = 0; s < n; s++) q[v][s] = u0[v];

    // One Picard sweep.  In the first the iterate is u^n at every time node, so every time slice
    // of the fluxes and of their spatial derivatives is the same: only slice 0 is computed and
    // it stands for all of them (equal to the full sweep in exact arithmetic; the compiled code
    // may round differently, by a few units in the last place).
    auto sweep = [&](auto first_c) __attribute__((always_inline)) {
        constexpr bool FIRST = decltype(first_c)::value;
        constexpr int NT = FIRST ? 1 : n;   // time slices computed
        // 1/rho of every node of the pencil, shared by the fluxes of all axes (for long
        // FP64 pencils recomputed per axis instead, to stay within 256 registers)
        constexpr bool CACHE_IRHO = n < 8 || sizeof(R) == 4;
        R irho[CACHE_IRHO ? n : 1], pr[CACHE_IRHO ? n : 1];
        if constexpr (CACHE_IRHO) {
#pragma unroll
            for (int t = 0; t < NT; t++) {
                if constexpr (DEV) {
                    // deviation form: 1/rho of the full state and the pressure's deviation
                    R dq[NV];
#pragma unroll
                    for (int v = 0; v < NV; v++) dq[v] = q[v][t];
                    irho[t] = recip(cref.q[0] + dq[0]);
                    pr[t] = dev_pressure<DIM, R>(cref, dq, irho[t], gamma);
                } else {
                    irho[t] = recip(q[0][t]);
                    R ke = 0;
#pragma unroll
                    for (int j = 0; j < DIM; j++) ke += q[1 + j][t] * q[1 + j][t];
                    pr[t] = (gamma - R(1)) * (q[NV - 1][t] - R(0.5) * ke * irho[t]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < DIM; k++) {
            const R ck = (R)(dt * A.dth[k]);
            for (int v0 = 0; v0 < NV; v0 += VC) {
                // point phase: fluxes of the time pencil straight into LDS
                if (tid < S::ACT) {
#pragma unroll
                    for (int t = 0; t < NT; t++) {
                        R ir;
                        if constexpr (CACHE_IRHO) ir = irho[t];
                        else ir = recip(q[0][t]);
                        const R un = q[1 + k][t] * ir;
                        R prt;
                        if constexpr (CACHE_IRHO) prt = pr[t];
                        else {
                            R ke = 0;
#pragma unroll
                            for (int j = 0; j < DIM; j++) ke += q[1 + j][t] * q[1 + j][t];
                            prt = (gamma - R(1)) * (q[NV - 1][t] - R(0.5) * ke * ir);
                        }
                        R F[NV];
                        if constexpr (DEV) {
                            R dq[NV];
#pragma unroll
                            for (int v = 0; v < NV; v++) dq[v] = q[v][t];
                            dev_flux<DIM, R>(k, cref, dq, ir, prt, F);
                        } else {
                            F[0] = q[1 + k][t];
#pragma unroll
                            for (int j = 0; j < DIM; j++) F[1 + j] = q[1 + j][t] * un + (j == k ? prt : R(0));
                            F[NV - 1] = un * (q[NV - 1][t] + prt);
                        }
#pragma unroll
                        for (int vv = 0; vv < VC; vv++)
                            if (v0 + vv < NV) X[(lc * VC + vv) * NST + a + NN * t] = F[v0 + vv];
                    }
                }
                __syncthreads();
                lds_lines<DIM, N, CPB, VC, S::BS, R, EO, false>(X, k, FIRST ? NN / n : NN, FIRST ? 0 : NN, D, R(1),
                                                                tid, NV - v0 < VC ? NV - v0 : VC, Es, Os);
                __syncthreads();
                // S = sum_k (dt/h_k) D_k F_k, the factor applied while accumulating
                if (tid < S::ACT) {
#pragma unroll
                    for (int vv = 0; vv < VC; vv++)
                        if (v0 + vv < NV)
#pragma unroll
                            for (int t = 0; t < n; t++) {
                                const R xk = X[(lc * VC + vv) * NST + a + NN * (FIRST ? 0 : t)];
                                Sacc[v0 + vv][t] = (k == 0) ? ck * xk : Sacc[v0 + vv][t] + ck * xk;
                            }
                } else if (k == 0) {
#pragma unroll
                    for (int vv = 0; vv < VC; vv++)
                        if (v0 + vv < NV)
#pragma unroll
                            for (int t = 0; t < n; t++) Sacc[v0 + vv][t] = 0;
                }
                __syncthreads();
            }
        }
        // time contraction in registers (Kw row s broadcast from LDS, shared by the variables)
#pragma unroll
        for (int s = 0; s < n; s++) {
            __asm__ volatile("" ::: "memory");
            R acc[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) acc[v] = 0;
#pragma unroll
            for (int t = 0; t < n; t++) {
                const R kst = Kw[s][t];
#pragma unroll
                for (int v = 0; v < NV; v++) acc[v] += kst * Sacc[v][t];
            }
#pragma unroll
            for (int v = 0; v < NV; v++) q[v][s] = u0[v] - acc[v];
        }
    };
    if (A.iters > 0) sweep(std::true_type{});
    for (int r = 1; r < A.iters; r++) sweep(std::false_type{});

    // ---- volume term of eq. (pde.nc.gw2), divided by the diagonal mass:
    //   (dt/h_k) sum_b [w_b D[b][a_k] / w_{a_k}] sum_s w_s F_k(q(a|b, s))
    if constexpr (VOL) {
        R vol[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) vol[v] = 0;
#pragma unroll
        for (int k = 0; k < DIM; k++) {
            const R ck = (R)(dt * A.dth[k]);
            R Fi[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) Fi[v] = 0;
#pragma unroll
            for (int t = 0; t < n; t++) {
                R qt[NV], F[NV];
#pragma unroll
                for (int v = 0; v < NV; v++) qt[v] = q[v][t];
                if constexpr (DEV) {
                    const R ir = recip(cref.q[0] + qt[0]);
                    dev_flux<DIM, R>(k, cref, qt, ir, dev_pressure<DIM, R>(cref, qt, ir, gamma), F);
                } else {
                    euler_flux<DIM, R>(k, qt, F, gamma);
                }
#pragma unroll
                for (int v = 0; v < NV; v++) Fi[v] += A.w[t] * F[v];
            }
            for (int v0 = 0; v0 < NV; v0 += VC) {
                if (tid < S::ACT) {
#pragma unroll
                    for (int vv = 0; vv < VC; vv++)
                        if (v0 + vv < NV) X[(lc * VC + vv) * NST + a] = Fi[v0 + vv];
                }
                __syncthreads();
                lds_lines<DIM, N, CPB, VC, S::BS, R>(X, k, NN / n, 0, Dvol, ck, tid, NV - v0 < VC ? NV - v0 : VC);
                __syncthreads();
                if (tid < S::ACT) {
#pragma unroll
                    for (int vv = 0; vv < VC; vv++)
                        if (v0 + vv < NV) vol[v0 + vv] += X[(lc * VC + vv) * NST + a];
                }
                __syncthreads();
            }
        }
        if (owner) {
            // u^n is read again here rather than held in registers through the sweeps
#pragma unroll
            for (int v = 0; v < NV; v++)
                A.vol_out[(A.cell0 + c) * NN + (int64_t)v * A.in_vstride + a] =
                    A.in[c * A.in_cstride + v * A.in_vstride + a] + (double)vol[v];
        }
    }

    // ---- face traces: q at xi_k = 0 / 1 per tangential node and time node
    for (int v0 = 0; v0 < NV; v0 += VC) {
        if (tid < S::ACT) {
#pragma unroll
            for (int vv = 0; vv < VC; vv++)
                if (v0 + vv < NV)
#pragma unroll
                    for (int s = 0; s < n; s++) X[(lc * VC + vv) * NST + a + NN * s] = q[v0 + vv][s];
        }
        __syncthreads();
        const int nitems = CPB * VC * 2 * DIM * NFN * n;
        for (int it = tid; it < nitems; it += S::BS) {
            const int lcl = it / (VC * 2 * DIM * NFN * n);
            int rem0 = it % (VC * 2 * DIM * NFN * n);
            const int vv = rem0 / (2 * DIM * NFN * n);
            rem0 %= 2 * DIM * NFN * n;
            const int face = rem0 / (NFN * n);
            const int j = rem0 % (NFN * n);   // ap + NFN*s
            const int s = j / NFN, ap = j % NFN;
            const int k = face >> 1, side = face & 1;
            const int64_t cc = vb * CPB + lcl;
            if (cc >= ncell || v0 + vv >= NV) continue;
            int base = 0, rem = ap, mul = 1;
#pragma unroll
            for (int jj = 0; jj < DIM; jj++) {
                if (jj == k) { mul *= n; continue; }
                base += (rem % n) * mul;
                rem /= n;
                mul *= n;
            }
            const R *line = &X[(lcl * VC + vv) * NST + NN * s + base];
            const int st = (k == 0) ? 1 : (k == 1 ? n : n * n);
            const R *Bv = side ? A.Rb : A.Lb;
            R acc = 0;
#pragma unroll
            for (int b = 0; b < n; b++) acc += Bv[b] * line[b * st];
            A.trace[((cc * 2 * DIM + face) * NV + v0 + vv) * (NFN * n) + j] = acc;
        }
        __syncthreads();
    }
    }  // persistent loop
}

template <int DIM, int N, bool VOL, typename R, bool DEV = false>
// the register budget held to Tune's waves per SIMD (FP32: four, FP64: two by default)
__global__ __launch_bounds__((PredShape<DIM, N, R>::BS), (Tune<DIM, N, sizeof(R) == 4>::pred_wps)) void k_predictor(PredArgs<R> A,
                                                                                                   double gamma_d) {
    pred_cells<DIM, N, VOL, R, DEV>(A, gamma_d, A.ncell, blockIdx.x, gridDim.x);
}

}  // namespace adg
