// HIP kernels for gfx950: one ADER-DG step with the a-posteriori subcell limiter.
// (Templates; the (d, N) instantiations are spread over the adg_inst_*.hip files so that they
// compile in parallel, the dispatch and the launch functions are in adg_kernels.hip.)
//
// Data layout in HBM (FP64):
//   u[v][cell][node]           nodal DG state, node = tensor GL index (x fastest)
//   trace[cell][2d][v][nfn*n]  predictor face traces, nfn = n^(d-1) tangential nodes x n time nodes
//   gbar[cell][2d][v][nfn]     time-integrated Rusanov face flux, one copy per adjacent cell
//   pool[slot][v][sub]         subcell data of troubled cells (sparse), slot = worklist index
//
// Parallel mapping: every kernel is element-local or face-local and writes each output
// from exactly one thread (no atomics on data), so results are bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <type_traits>
#pragma once
#include "adg_internal.h"
#include "adg_kernels.h"
#include "adg_device.h"
#include "adg_predictor.h"

namespace adg {

// ------------------------------------------------------------------- large cells
// 3D cells of degree N = 9 carry 19^3 subcells and 10^3 nodes per variable: the candidate's
// subcell averages, the stages of the sum-factorised projection P and gather R and the
// subcell update's sub-face fluxes (0.4-1.4 MB per cell) exceed the 160 KB of LDS of a CU.
// Those arrays live in a slot of global memory per workgroup (reused cell after cell, so it
// stays in the L2 / Infinity Cache) and the kernels loop over their cells with a grid of at
// most BIG_WG workgroups; the nodal state of the cell stays in LDS.
template <int DIM, int N>
struct BigCell {
    static constexpr bool on = DIM == 3 && N >= 9;
    static constexpr int n = N + 1, NV = DIM + 2, NN = cpow(n, DIM), NS = 2 * N + 1, NSUB = cpow(NS, DIM);
    static constexpr int NSF = cpow(NS, DIM - 1), BIGN = NSUB > NN ? NSUB : NN;
    // corrector: subcell averages + the stage-1 intermediate of P
    static constexpr int64_t CORR = (int64_t)NV * NSUB + (int64_t)NV * NS * NS * n;
    // bounds and flux correction: subcell averages + intermediate, both NV x max(NSUB, NN)
    static constexpr int64_t BND = 2ll * NV * BIGN;
    // subcell update: sub-face fluxes (FP64 at most) or the gather's intermediate, then the
    // new subcell averages and the gathered nodal values
    static constexpr int64_t FB = (int64_t)DIM * (NS + 1) * NSF * NV, TM = (int64_t)NV * BIGN;
    static constexpr int64_t SUB = (FB > TM ? FB : TM) + 2ll * NV * BIGN;
    static constexpr int64_t M1 = CORR > BND ? CORR : BND, M2 = M1 > SUB ? M1 : SUB;
    static constexpr int64_t SLOT = on ? ((M2 + 31) / 32) * 32 : 0;   // doubles, 256-byte aligned
    // the slot's regions in the subcell update
    static constexpr int64_t SUB_VN = FB > TM ? FB : TM, SUB_UG = SUB_VN + (int64_t)NV * BIGN;
};

// ------------------------------------------------------------------- face fluxes
// One thread per (face, tangential node, time node): Rusanov flux weighted by the time
// quadrature weight; the time sum is then taken in LDS in fixed order and written into
// the slot of both adjacent cells.
template <int DIM, int N>
struct FaceShape {
    static constexpr int n = N + 1, NFN = cpow(n, DIM - 1), PER = NFN * n;
    static constexpr int FPB = PER >= 256 ? 1 : 256 / PER;   // faces per block
    static constexpr int BS = ((FPB * PER + 63) / 64) * 64;
};

// The Rusanov flux of the deviation form at one face node and time node.  dL / dR: the
// traces' deviations from the reference states cL / cR of the two cells (first nodal values
// of u^n in FP32); G receives G - F(c) of the left cell (of the inside cell at a boundary or
// wall) and dFc the difference F(c_R) - F(c_L) (zero at a boundary or wall).
template <int DIM, int N, typename R, int K>
__device__ __forceinline__ void face_flux_dev(const Prob &P, const Tables *__restrict__ T, const double *__restrict__ u,
                                              int64_t cL, int64_t cR, bool hasL, bool hasR, bool wall, const R *dL,
                                              const R *dR, const double *x, double ts, R *G, R *dFc) {
    constexpr int NV = DIM + 2, NN = cpow(N + 1, DIM);
    constexpr int k = K;
    const R g = (R)P.gamma;
    auto ref = [&](int64_t cc) {
        double c64[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) c64[v] = u[((int64_t)v * P.ncell + cc) * NN];
        return make_devref<DIM, R>(c64, P.gamma);
    };
    auto speed = [&](const DevRef<DIM, R> &c, const R *d) {
        R q[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) q[v] = c.q[v] + d[v];
        return fabs(along<DIM, R>(q, k) / q[0]) + sqrt(g * pressure<DIM, R>(q, g) / q[0]);
    };
    auto dflux = [&](const DevRef<DIM, R> &c, const R *d, R *F) {
        const R ir = R(1) / (c.q[0] + d[0]);
        dev_flux<DIM, R>(k, c, d, ir, dev_pressure<DIM, R>(c, d, ir, g), F);
    };
    R FL[NV], FR[NV];
    if (hasL && hasR) {
        const DevRef<DIM, R> rl = ref(cL), rr = ref(cR);
        double ql[NV], qr[NV], fl[NV], fr[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) {
            ql[v] = (double)rl.q[v];
            qr[v] = (double)rr.q[v];
        }
        euler_flux<DIM, double>(k, ql, fl, P.gamma);
        euler_flux<DIM, double>(k, qr, fr, P.gamma);
        dflux(rl, dL, FL);
        dflux(rr, dR, FR);
        const R s = fmax(speed(rl, dL), speed(rr, dR));
#pragma unroll
        for (int v = 0; v < NV; v++) {
            dFc[v] = (R)(fr[v] - fl[v]);
            const R dq = (R)(qr[v] - ql[v]) + (dR[v] - dL[v]);
            G[v] = R(0.5) * (FL[v] + FR[v] + dFc[v]) - R(0.5) * s * dq;
        }
        return;
    }
    // one side is a cell, the other the ghost of the boundary rule or the mirror of a wall,
    // both taken relative to the cell's reference state (the ghost formed in FP64)
    const bool inL = hasL;
    const DevRef<DIM, R> rc = ref(inL ? cL : cR);
    const R *din = inL ? dL : dR;
    double qi[NV], qo[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) qi[v] = (double)rc.q[v] + (double)din[v];
    if (wall) {
        wall_ghost<DIM, double>(k, qi, qo);
    } else {
        bc_ghost<DIM>(P, k, inL ? 1 : 0, qi, x[0], x[1], x[2], ts, qo);
    }
    R dg[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) dg[v] = (R)(qo[v] - (double)rc.q[v]);
    dflux(rc, din, FL);
    dflux(rc, dg, FR);
    const R s = fmax(speed(rc, din), speed(rc, dg));
    // G(q_in, q_ghost) with the inside cell on the left, or G(q_ghost, q_in) with it on the right
#pragma unroll
    for (int v = 0; v < NV; v++) {
        dFc[v] = 0;
        G[v] = R(0.5) * (FL[v] + FR[v]) - R(0.5) * s * (inL ? dg[v] - din[v] : din[v] - dg[v]);
    }
}

// The faces normal to axis K handled by one workgroup (block blk of that axis); K is a
// compile-time constant so that no per-thread array is indexed dynamically.
// DEV: the traces are deviations from each cell's reference state c (its first nodal value of
// u^n, rounded to FP32); each cell's slot receives G - F(c) of that cell, the Rusanov flux
// assembled from the deviation fluxes and the FP64 difference of the two references' fluxes.
template <int DIM, int N, typename R, int K, bool DEV = false>
__device__ __forceinline__ void face_axis(const Tables *__restrict__ T, const Prob &P, const R *__restrict__ trace,
                                          R *__restrict__ gbar, const double *__restrict__ scal, int64_t blk, R *part,
                                          const uint8_t *__restrict__ mask, const double *__restrict__ u) {
    using FS = FaceShape<DIM, N>;
    constexpr int n = N + 1, NV = DIM + 2, NFN = FS::NFN, PER = FS::PER, FPB = FS::FPB;
    constexpr int k = K;
    const int nk = P.nc[k];
    const int nfk = P.periodic[k] ? nk : nk + 1;           // faces along k per line
    int64_t nlines = 1;
    for (int j = 0; j < DIM; j++)
        if (j != k) nlines *= P.nc[j];
    const int64_t nfaces = nlines * nfk;
    const int lf = threadIdx.x / PER, j = threadIdx.x % PER;
    const int s = j / NFN, ap = j % NFN;
    const int64_t fidx = blk * FPB + lf;
    bool active = lf < FPB && fidx < nfaces;
    int64_t cL = -1, cR = -1;
    bool hasL = false, hasR = false, wall = false;
    int fk = 0, ci[3] = {0, 0, 0};
    if (active) {
        fk = (int)(fidx % nfk);
        int64_t line = fidx / nfk;
        // cell coordinates, selected per axis with compile-time indices (a runtime index
        // would move the arrays to scratch memory)
        hasL = fk > 0 || P.periodic[k];
        hasR = fk < nk;
        const int fl = fk > 0 ? fk - 1 : fk - 1 + nk;
        int cl[3] = {0, 0, 0}, cr[3] = {0, 0, 0};
#pragma unroll
        for (int jj = 0; jj < DIM; jj++) {
            if (jj == k) {
                cl[jj] = fl;
                cr[jj] = fk;
            } else {
                ci[jj] = (int)(line % P.nc[jj]);
                line /= P.nc[jj];
                cl[jj] = cr[jj] = ci[jj];
            }
        }
        cL = hasL ? cell_of(P, cl) : -1;
        cR = hasR ? cell_of(P, cr) : -1;
        if (mask) {
            // masked geometry: a face toward a solid cell is a reflective wall of the fluid
            // side; a face with no fluid side carries no flux
            if (hasL && mask[cL]) { hasL = false; wall = true; }
            if (hasR && mask[cR]) { hasR = false; wall = true; }
            if (!hasL && !hasR) active = false;
        }
    }
    if (active) {
        const double dt = scal[0], t0 = scal[1];
        // node position on the face (for boundary states)
        double x[3] = {0, 0, 0};
        {
            int rem = ap;
#pragma unroll
            for (int jj = 0; jj < DIM; jj++) {
                if (jj == k) {
                    x[jj] = P.lo[jj] + P.h[jj] * fk;
                } else {
                    x[jj] = P.lo[jj] + P.h[jj] * (ci[jj] + T->xi[rem % n]);
                    rem /= n;
                }
            }
        }
        R qL[NV], qR[NV], G[NV];
        if (hasL) {
#pragma unroll
            for (int v = 0; v < NV; v++) qL[v] = trace[((cL * 2 * DIM + 2 * k + 1) * NV + v) * (NFN * n) + ap + NFN * s];
        }
        if (hasR) {
#pragma unroll
            for (int v = 0; v < NV; v++) qR[v] = trace[((cR * 2 * DIM + 2 * k) * NV + v) * (NFN * n) + ap + NFN * s];
        }
        if constexpr (DEV) {
            face_flux_dev<DIM, N, R, K>(P, T, u, cL, cR, hasL, hasR, wall, qL, qR, x, scal[1] + T->xi[s] * scal[0], G,
                                        part + ((lf * PER + j) * 2 + 1) * NV);
        } else if (wall) {
            if (hasL) wall_ghost<DIM, R>(k, qL, qR);
            else wall_ghost<DIM, R>(k, qR, qL);
        } else if (!hasL || !hasR) {
            const double ts = t0 + T->xi[s] * dt;
            double qi[NV], qo[NV];
            if (hasL) {
#pragma unroll
                for (int v = 0; v < NV; v++) qi[v] = (double)qL[v];
                bc_ghost<DIM>(P, k, 1, qi, x[0], x[1], x[2], ts, qo);
#pragma unroll
                for (int v = 0; v < NV; v++) qR[v] = (R)qo[v];
            } else {
#pragma unroll
                for (int v = 0; v < NV; v++) qi[v] = (double)qR[v];
                bc_ghost<DIM>(P, k, 0, qi, x[0], x[1], x[2], ts, qo);
#pragma unroll
                for (int v = 0; v < NV; v++) qL[v] = (R)qo[v];
            }
        }
        if constexpr (!DEV) num_flux<DIM, R>(P, T, k, qL, qR, G);
        const R ws = std::is_same<R, double>::value ? (R)T->w[s] : (R)T->fw[s];
        constexpr int PS = DEV ? 2 : 1;   // DEV: [0] the left cell's G - F(c_L), [1] F(c_R) - F(c_L)
#pragma unroll
        for (int v = 0; v < NV; v++) part[(lf * PER + j) * PS * NV + v] = ws * G[v];
    }
    __syncthreads();
    if (active && s == 0) {
        constexpr int PS = DEV ? 2 : 1;
        R acc[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) acc[v] = 0;
        for (int ss = 0; ss < n; ss++)
#pragma unroll
            for (int v = 0; v < NV; v++) acc[v] += part[(lf * PER + ap + NFN * ss) * PS * NV + v];
        if (hasL) {
#pragma unroll
            for (int v = 0; v < NV; v++) gbar[((cL * 2 * DIM + 2 * k + 1) * NV + v) * NFN + ap] = acc[v];
        }
        if (hasR) {
            if constexpr (DEV) {
                // the right cell's slot: G - F(c_R) = (G - F(c_L)) - (F(c_R) - F(c_L)) times the
                // time weights' sum (zero unless both sides are cells)
                if (hasL) {
                    R wsum = 0;
                    for (int ss = 0; ss < n; ss++) wsum += (R)T->fw[ss];
#pragma unroll
                    for (int v = 0; v < NV; v++) acc[v] -= wsum * part[(lf * PER + ap) * PS * NV + NV + v];
                }
            }
#pragma unroll
            for (int v = 0; v < NV; v++) gbar[((cR * 2 * DIM + 2 * k) * NV + v) * NFN + ap] = acc[v];
        }
    }
}

template <int DIM, int N, typename R, bool DEV = false>
__device__ __forceinline__ void face_block(const Tables *__restrict__ T, const Prob &P, const R *__restrict__ trace,
                                           R *__restrict__ gbar, const double *__restrict__ scal, int64_t kb1,
                                           int64_t kb2, int64_t bid, const uint8_t *__restrict__ mask,
                                           const double *__restrict__ u) {
    // one launch for the faces of every axis: blocks [0, kb1) axis 0, [kb1, kb2) axis 1, then axis 2
    using FS = FaceShape<DIM, N>;
    __shared__ R part[FS::FPB * FS::PER * (DIM + 2) * (DEV ? 2 : 1)];
    const int k = (bid < kb1) ? 0 : ((bid < kb2) ? 1 : 2);
    const int64_t blk = (int64_t)bid - (k == 0 ? 0 : (k == 1 ? kb1 : kb2));
    switch (k) {
    case 0: face_axis<DIM, N, R, 0, DEV>(T, P, trace, gbar, scal, blk, part, mask, u); break;
    case 1: face_axis<DIM, N, R, 1, DEV>(T, P, trace, gbar, scal, blk, part, mask, u); break;
    default: face_axis<DIM, N, R, DIM - 1, DEV>(T, P, trace, gbar, scal, blk, part, mask, u); break;
    }
}
template <int DIM, int N, typename R, bool DEV = false>
__global__ __launch_bounds__((FaceShape<DIM, N>::BS)) void k_face(const Tables *__restrict__ T, Prob P,
                                                                 const R *__restrict__ trace, R *__restrict__ gbar,
                                                                 const double *__restrict__ scal, int64_t kb1,
                                                                 int64_t kb2, const uint8_t *__restrict__ mask,
                                                                 const double *__restrict__ u) {
    face_block<DIM, N, R, DEV>(T, P, trace, gbar, scal, kb1, kb2, blockIdx.x, mask, u);
}

// Block-wide reduction of per-thread (min, max) pairs of NV variables: wave shuffles,
// then one LDS exchange between waves.  The result is valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_minmax(double *lo, double *hi, int tid, int bs, double *scratch) {
#pragma unroll
    for (int v = 0; v < NV; v++) {
        lo[v] = wave_min(lo[v]);
        hi[v] = wave_max(hi[v]);
    }
    const int w = tid >> 6, lane = tid & 63, nw = bs >> 6;
    if (lane == 0)
#pragma unroll
        for (int v = 0; v < NV; v++) {
            scratch[(2 * w) * NV + v] = lo[v];
            scratch[(2 * w + 1) * NV + v] = hi[v];
        }
    __syncthreads();
    if (tid == 0)
        for (int ww = 1; ww < nw; ww++)
#pragma unroll
            for (int v = 0; v < NV; v++) {
                lo[v] = fmin(lo[v], scratch[(2 * ww) * NV + v]);
                hi[v] = fmax(hi[v], scratch[(2 * ww + 1) * NV + v]);
            }
    __syncthreads();
}

// Extended-grid index (one ghost ring) of interior cell c.
__device__ __forceinline__ int64_t ext_index(const Prob &P, int64_t c) {
    int ci[3];
    coords_of(P, c, ci);
    int64_t e = 0;
    for (int j = P.dim - 1; j >= 0; j--) e = e * (P.nc[j] + 2) + (ci[j] + 1);
    return e;
}

__device__ __forceinline__ int64_t ext_count(const Prob &P) {
    int64_t next = 1;
    for (int j = 0; j < P.dim; j++) next *= P.nc[j] + 2;
    return next;
}

// Per-variable min / max of one cell's subcell data held in LDS (v[var*nsub + s]),
// stored as that cell's old-time bounds for the next step (the second bounds buffer:
// the first still holds this step's, read by the detection of other cells).
template <int NV>
__device__ __forceinline__ void store_cell_bounds(const Prob &P, const Bufs &B, int64_t c, const double *v, int nsub,
                                                  int tid, int bs, double *scratch) {
    double lo[NV], hi[NV];
#pragma unroll
    for (int k = 0; k < NV; k++) {
        lo[k] = INFINITY;
        hi[k] = -INFINITY;
    }
    for (int sg = tid; sg < nsub; sg += bs)
#pragma unroll
        for (int k = 0; k < NV; k++) {
            lo[k] = fmin(lo[k], v[k * nsub + sg]);
            hi[k] = fmax(hi[k], v[k * nsub + sg]);
        }
    block_minmax<NV>(lo, hi, tid, bs, scratch);
    if (tid == 0) {
        const int64_t e = ext_index(P, c), next = ext_count(P);
        for (int k = 0; k < NV; k++) {
            B.ext_min[1][(int64_t)k * next + e] = lo[k];
            B.ext_max[1][(int64_t)k * next + e] = hi[k];
        }
    }
}

// --------------------------------------------------- tensor application in LDS
// out[v][...] = sum over axis k of M[i][b] in[...b...], applied axis by axis (sum
// factorisation).  Before stage k the axes < k have size M (output) and the axes >= k size
// NI (input).  One thread owns one line along axis k: it loads the NI inputs of its line
// once and produces the M outputs.  The operator entries are the same for every lane, so
// they are read from the table in global memory through scalar loads, not from LDS.
template <int DIM, int K, int M, int NI, int NVAR, int MSTRIDE>
__device__ __forceinline__ void tensor_stage(const double *__restrict__ Mat, const double *src, double *dst, int tid,
                                             int bs) {
    constexpr int S0 = (0 < K) ? M : NI, S1 = (1 < K) ? M : NI, S2 = (DIM == 3) ? ((2 < K) ? M : NI) : 1;
    constexpr int IS[3] = {1, S0, S0 * S1};                               // input strides
    constexpr int O0 = (0 <= K) ? M : NI, O1 = (1 <= K) ? M : NI;
    constexpr int OS[3] = {1, O0, O0 * O1};                               // output strides
    constexpr int SZB = S0 * S1 * S2;
    constexpr int SZA = SZB / NI * M;
    // the one or two axes other than K, with their (common) sizes
    constexpr int A1 = (K == 0) ? 1 : 0, A2 = (K == 2) ? 1 : 2;
    constexpr int SZ[3] = {S0, S1, S2};
    constexpr int N1 = SZ[A1], N2 = (DIM == 3) ? SZ[A2] : 1;
    constexpr int LINES = NVAR * N1 * N2;
    for (int l = tid; l < LINES; l += bs) {
        const int v = l / (N1 * N2);
        const int r = l - v * (N1 * N2);
        const int j1 = r % N1, j2 = r / N1;
        const double *x = src + v * SZB + j1 * IS[A1] + ((DIM == 3) ? j2 * IS[A2] : 0);
        double *y = dst + v * SZA + j1 * OS[A1] + ((DIM == 3) ? j2 * OS[A2] : 0);
        double xin[NI];
#pragma unroll
        for (int b = 0; b < NI; b++) xin[b] = x[b * IS[K]];
#pragma unroll
        for (int i = 0; i < M; i++) {
            double acc = 0.0;
#pragma unroll
            for (int b = 0; b < NI; b++) acc += Mat[i * MSTRIDE + b] * xin[b];
            y[i * OS[K]] = acc;
        }
    }
    __syncthreads();
}

template <int DIM, int M, int NI, int NVAR, int MSTRIDE>
__device__ __forceinline__ void tensor_apply(const double *__restrict__ Mbase, const double *in, double *out, double *tmp, int tid,
                             int bs) {
    // the buffers alternate so that the last stage lands in `out`
    if constexpr (DIM == 2) {
        tensor_stage<2, 0, M, NI, NVAR, MSTRIDE>(Mbase, in, tmp, tid, bs);
        tensor_stage<2, 1, M, NI, NVAR, MSTRIDE>(Mbase, tmp, out, tid, bs);
    } else {
        tensor_stage<3, 0, M, NI, NVAR, MSTRIDE>(Mbase, in, out, tid, bs);
        tensor_stage<3, 1, M, NI, NVAR, MSTRIDE>(Mbase, out, tmp, tid, bs);
        tensor_stage<3, 2, M, NI, NVAR, MSTRIDE>(Mbase, tmp, out, tid, bs);
    }
}

// ------------------------------------------- corrector + scatter + detection
// Threads per cell (one wave while the cell has at most 128 subcells, else two) and cells
// per workgroup.
template <int DIM, int N, typename R>
struct CorrShape {
    static constexpr int NSUB = cpow(2 * N + 1, DIM);
    static constexpr bool BIG = BigCell<DIM, N>::on;
    static constexpr int CW = BIG ? 256 : (NSUB <= 128 ? 64 : 128);
    static constexpr int CPB = (CW == 64) ? Tune<DIM, N, sizeof(R) == 4>::corr_cpb : 1;
    static constexpr int BS = CW * CPB;
    static constexpr int NW = CW / 64;   // waves per cell
    // waves per SIMD that the LDS of one workgroup allows (its state, subcell and stage
    // arrays); the register budget is held to it so that registers do not limit further
    static constexpr int NN = cpow(N + 1, DIM), NV = DIM + 2;
    static constexpr int TMPN = (DIM == 2) ? (2 * N + 1) * (N + 1) : (2 * N + 1) * (2 * N + 1) * (N + 1);
    // (large cells: the nodal state and the face fluxes in LDS, the rest in the global slot)
    static constexpr int LDSB = BIG ? NV * NN * 8 + 2 * DIM * NV * cpow(N + 1, DIM - 1) * 8 + (2 * NW + 2) * NV * 8 + 2048
                                    : CPB * NV * (NN + NSUB + TMPN) * 8 + CPB * (2 * NW + 2) * NV * 8 + 2048;
    static constexpr int WPS0 = (163840 / LDSB) * (BS / 64) / 4;
    static constexpr int WPS = WPS0 < 1 ? 1 : (WPS0 > 6 ? 6 : WPS0);
};

// Candidate of eq. (pde.nc.gw2) (face terms added to the volume-term candidate), then
// v* = P(u*) (eq. (subcell.p)) and the PAD / relaxed-DMP tests of Sec. 4.3.
template <int DIM, int N, typename R>
__device__ __forceinline__ void corrector_detect_block(const Tables *__restrict__ T, const Prob &P, const Bufs &B,
                                                       int cur, int limiter, int64_t bid) {
    using CS = CorrShape<DIM, N, R>;
    constexpr int CW = CS::CW, CPB = CS::CPB, NW = CS::NW;
    const R *gbar = reinterpret_cast<const R *>(B.gbar);
    constexpr int n = N + 1, NV = DIM + 2, NN = cpow(n, DIM), NFN = cpow(n, DIM - 1);
    constexpr int NS = 2 * N + 1, NSUB = cpow(NS, DIM);
    // intermediate of the sum-factorised P: stage 0 (2D) or stage 1 (3D) output
    constexpr int TMP = (DIM == 2) ? NS * n : NS * NS * n;
    __shared__ double us_[CPB][NV * NN];
    __shared__ double red_[CPB][NW * 2 * NV];
    __shared__ int bad_s[CPB][NW];
    __shared__ float mg_s[CPB][NW];
    __shared__ double bnd[CPB][2][NV];    // m_i, M_i of eq. (dmp) per cell
    const int lc = threadIdx.x / CW, tid = threadIdx.x % CW;
    const int64_t c = (int64_t)bid * CPB + lc;
    const bool live = c < P.ncell;         // every thread stays for the barriers
    // masked geometry: a solid cell keeps its state and is never troubled
    const bool solid = live && B.mask && B.mask[c];
    double *us = us_[lc], *red = red_[lc], *vs, *tmp;
    if constexpr (CS::BIG) {
        vs = B.big + (int64_t)blockIdx.x * BigCell<DIM, N>::SLOT;
        tmp = vs + NV * NSUB;
    } else {
        __shared__ double vs_[CPB][NV * NSUB];
        __shared__ double tmp_[CPB][NV * TMP];
        vs = vs_[lc];
        tmp = tmp_[lc];
    }
    const double dt = B.scal[0];
    double *un = B.u[cur ^ 1];
    const double *usrc = solid ? B.u[cur] : un;
    // debug poison of one variable of one cell's candidate (armed by the host for one step)
    const bool poisoned = live && B.scal[4] != 0.0 && (int64_t)B.scal[5] == c;
    const int pvar = poisoned ? (int)B.scal[6] : -1;
    const double pval = B.scal[7];
    // (dt/h_k)/w_a for every axis and node index: 2 divisions per entry, once per block
    __shared__ double coef[3][n];
    if (threadIdx.x < DIM * n) coef[threadIdx.x / n][threadIdx.x % n] = dt / P.h[threadIdx.x / n] / T->w[threadIdx.x % n];
    if (limiter && live && tid < 2 * NV) {
        // min (mm = 0) / max (mm = 1) of variable v over the 3^d block V_i of the
        // per-cell old-time bounds, held on the extended grid (cell c sits at ci + 1; along a
        // periodic axis a neighbour beyond the edge is the wrapped interior cell)
        const int mm = tid / NV, v = tid % NV;
        int ci[3];
        coords_of(P, c, ci);
        int ne[3] = {1, 1, 1};
        for (int j = 0; j < DIM; j++) ne[j] = P.nc[j] + 2;
        const int64_t next = ext_count(P);
        const double *src = (mm ? B.ext_max[0] : B.ext_min[0]) + (int64_t)v * next;
        double acc = mm ? -INFINITY : INFINITY;
        constexpr int NB = cpow(3, DIM);
#pragma unroll
        for (int o = 0; o < NB; o++) {
            const int off[3] = {o % 3, (o / 3) % 3, o / 9};
            int64_t e = 0;
            for (int j = DIM - 1; j >= 0; j--) {
                int x = ci[j] + off[j];   // extended coordinate
                if (P.periodic[j]) x += (x == 0) ? P.nc[j] : ((x == P.nc[j] + 1) ? -P.nc[j] : 0);
                e = e * ne[j] + x;
            }
            acc = mm ? fmax(acc, src[e]) : fmin(acc, src[e]);
        }
        bnd[lc][mm][v] = acc;
    }
    // every global load of the update issued before any store: the cell's face fluxes
    // into LDS, its volume-term candidate into registers
    constexpr int GSZ = 2 * DIM * NV * NFN, EPT = (NV * NN + CW - 1) / CW;
    __shared__ R gs_[CPB][GSZ];
    R *gs = gs_[lc];
    for (int i = tid; i < GSZ; i += CW) gs[i] = live ? gbar[c * GSZ + i] : R(0);
    double uv[EPT];
#pragma unroll
    for (int e = 0; e < EPT; e++) {
        const int it = tid + e * CW;
        uv[e] = (live && it < NV * NN) ? usrc[((int64_t)(it / NN) * P.ncell + c) * NN + it % NN] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EPT; e++) {
        const int it = tid + e * CW;
        if (it >= NV * NN) break;
        const int v = it / NN, a = it % NN;
        int m[3] = {a % n, (a / n) % n, a / (n * n)};
        double val = uv[e];
#pragma unroll
        for (int k = 0; k < DIM; k++) {
            if (solid) break;
            int ap = 0, mul = 1;
            for (int j = 0; j < DIM; j++) {
                if (j == k) continue;
                ap += m[j] * mul;
                mul *= n;
            }
            const int ak = m[k];
            const R Gm = gs[((2 * k) * NV + v) * NFN + ap];
            const R Gp = gs[((2 * k + 1) * NV + v) * NFN + ap];
            // face increment in the working precision R, added to the FP64 candidate
            const R cf = (R)coef[k][ak];
            val += (double)(cf * ((R)T->L[ak] * Gm - (R)T->R[ak] * Gp));
        }
        if (v == pvar) val = pval;
        if (live) un[((int64_t)v * P.ncell + c) * NN + a] = val;
        us[it] = val;
    }
    if (!limiter) return;
    __syncthreads();
    tensor_apply<DIM, NS, n, NV, MAXN>(&T->P[0][0], us, vs, tmp, tid, CW);
    // detection on the NSUB candidate subcell averages
    double m_[NV], M_[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) {
        m_[v] = live ? bnd[lc][0][v] : 0.0;
        M_[v] = live ? bnd[lc][1][v] : 0.0;
    }
    int bad = 0;
    float mg = INFINITY;
    double sr = fmax(fabs(M_[0]), fabs(m_[0]));
    double se = fmax(fabs(M_[DIM + 1]), fabs(m_[DIM + 1]));
    if (!(sr > 0)) sr = 1.0;
    if (!(se > 0)) se = 1.0;
    // per-variable bounds of eq. (dmp) relaxed by eq. (relax), hoisted out of the subcell loop;
    // the margin (a diagnostic) is normalised with reciprocals
    double lo_[NV], hi_[NV], isc[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) {
        const double delta = fmax(P.delta0, P.eps * (M_[v] - m_[v]));
        lo_[v] = m_[v] - delta;
        hi_[v] = M_[v] + delta;
        double sc = fmax(fabs(M_[v]), fabs(m_[v]));
        if (!(sc > 0)) sc = 1.0;
        isc[v] = 1.0 / sc;
    }
    const double isr = 1.0 / sr, ise = 1.0 / se;
    // the same pass takes the candidate's subcell min / max: the next step's old-time
    // bounds of this cell (overwritten later in the step if the cell is recomputed or
    // corrected)
    double lo[NV], hi[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) {
        lo[v] = INFINITY;
        hi[v] = -INFINITY;
    }
    for (int sg = tid; sg < NSUB; sg += CW) {
        double q[NV];
        bool finite = true;
#pragma unroll
        for (int v = 0; v < NV; v++) {
            q[v] = vs[v * NSUB + sg];
            lo[v] = fmin(lo[v], q[v]);
            hi[v] = fmax(hi[v], q[v]);
            if (!isfinite(q[v])) finite = false;
        }
        if (!finite) {
            bad = 1;
            mg = -INFINITY;
            continue;
        }
        const double p = pressure<DIM>(q, P.gamma);
        if (!(q[0] > 0.0) || !(p > 0.0)) bad = 1;
        double lmg = fmin(q[0] * isr, p * ise);
#pragma unroll
        for (int v = 0; v < NV; v++) {
            if (q[v] < lo_[v] || q[v] > hi_[v]) bad = 1;
            lmg = fmin(lmg, fmin(q[v] - lo_[v], hi_[v] - q[v]) * isc[v]);
        }
        mg = fminf(mg, (float)lmg);
    }
    bad = wave_reduce(bad, [](int a, int b) { return a | b; });
    mg = wave_reduce(mg, [](float a, float b) { return fminf(a, b); });
#pragma unroll
    for (int v = 0; v < NV; v++) {
        lo[v] = wave_min(lo[v]);
        hi[v] = wave_max(hi[v]);
    }
    const int w = tid >> 6;
    if ((tid & 63) == 0) {
        bad_s[lc][w] = bad;
        mg_s[lc][w] = mg;
#pragma unroll
        for (int v = 0; v < NV; v++) {
            red[w * 2 * NV + v] = lo[v];
            red[w * 2 * NV + NV + v] = hi[v];
        }
    }
    __syncthreads();
    if (!live) return;
    if (tid == 0) {
        int bd = 0;
        float m = INFINITY;
#pragma unroll
        for (int ww = 0; ww < NW; ww++) {
            bd |= bad_s[lc][ww];
            m = fminf(m, mg_s[lc][ww]);
        }
        B.beta[1][c] = (uint8_t)((!solid && (bd || B.force[c])) ? 1 : 0);
        B.margin[c] = solid ? INFINITY : m;
    }
    if (tid < 2 * NV) {
        // thread v: min of variable v; thread NV + v: max of variable v
        const int v = tid % NV, mx = tid >= NV;
        double r = red[mx * NV + v];
#pragma unroll
        for (int ww = 1; ww < NW; ww++)
            r = mx ? fmax(r, red[ww * 2 * NV + NV + v]) : fmin(r, red[ww * 2 * NV + v]);
        const int64_t e = ext_index(P, c), next = ext_count(P);
        (mx ? B.ext_max[1] : B.ext_min[1])[(int64_t)v * next + e] = r;
    }
}
template <int DIM, int N, typename R>
__global__ __launch_bounds__((CorrShape<DIM, N, R>::BS), (CorrShape<DIM, N, R>::WPS)) void k_corrector_detect(const Tables *__restrict__ T, Prob P,
                                                                         Bufs B, int cur, int limiter) {
    if constexpr (BigCell<DIM, N>::on) {
        // large cells: one cell per iteration on the workgroup's global slot
        for (int64_t c = blockIdx.x; c < P.ncell; c += gridDim.x) {
            corrector_detect_block<DIM, N, R>(T, P, B, cur, limiter, c);
            __syncthreads();
        }
    } else {
        corrector_detect_block<DIM, N, R>(T, P, B, cur, limiter, blockIdx.x);
    }
}

// --------------------------------------------------------- old-time bounds
// Subcell data v^n of eq. (ader.icbc) for one (possibly ghost) cell: the stored
// ADER-WENO result when the cell was troubled at the previous step, else P(u^n).
// Ghost cells (outside a non-periodic boundary) mirror the interior subcells and apply
// the boundary rule at the ghost subcell centre.  Output: per-variable min / max over
// the cell's subcells, for the extended grid with a one-cell ghost ring.
template <int DIM, int N>
__device__ __forceinline__ void cell_bounds_block(const Tables *__restrict__ T, const Prob &P, const Bufs &B, int cur,
                                                  const int64_t *__restrict__ ring, int64_t bid) {
    constexpr int n = N + 1, NV = DIM + 2, NN = cpow(n, DIM);
    constexpr int NS = 2 * N + 1, NSUB = cpow(NS, DIM);
    constexpr int BIG = NSUB > NN ? NSUB : NN;
    __shared__ double us[NV * NN];
    __shared__ double red[2 * NV * 2];
    double *vs, *tmp;
    if constexpr (BigCell<DIM, N>::on) {
        vs = B.big + (int64_t)blockIdx.x * BigCell<DIM, N>::SLOT;
        tmp = vs + NV * BIG;
    } else {
        __shared__ double vs_[NV * BIG];
        __shared__ double tmp_[NV * BIG];
        vs = vs_;
        tmp = tmp_;
    }
    const int tid = threadIdx.x;
    // all extended cells, or only the ghost ring (interior bounds then come from the
    // kernels of the previous step that produced each cell's new subcell data)
    const int64_t e = ring ? ring[bid] : (int64_t)bid;
    int ei[3] = {0, 0, 0}, ne[3] = {1, 1, 1};
    for (int j = 0; j < DIM; j++) ne[j] = P.nc[j] + 2;
    {
        int64_t r = e;
        for (int j = 0; j < DIM; j++) {
            ei[j] = (int)(r % ne[j]) - 1;
            r /= ne[j];
        }
    }
    // masked geometry: a solid cell holds the mirror image of the fluid across its walls,
    // whose subcells are those of the image cell (reversed along the mirrored axes, which
    // leaves the extrema alone) with the mirrored axes' momenta negated
    int istep[3] = {0, 0, 0};
    if (B.mask && solid_at<DIM>(P, B.mask, ei[0], ei[1], ei[2])) {
        solid_image<DIM>(P, B.mask, ei, istep);
        for (int j = 0; j < DIM; j++) ei[j] += istep[j];
    }
    int src[3] = {0, 0, 0}, mir[3] = {0, 0, 0}, gside[3] = {-1, -1, -1};
    for (int j = 0; j < DIM; j++) {
        src[j] = ei[j];
        if (ei[j] < 0 || ei[j] >= P.nc[j]) {
            const int side = ei[j] >= P.nc[j];
            if (P.periodic[j]) {
                src[j] = (ei[j] + P.nc[j]) % P.nc[j];
            } else {
                src[j] = side ? 2 * P.nc[j] - 1 - ei[j] : -1 - ei[j];
                mir[j] = 1;
                gside[j] = side;
            }
        }
    }
    const int64_t cs = cell_of(P, src);
    const double *uo = B.u[cur];
    const int oslot = B.slot[0][cs];
    // a cell flagged beyond the pool capacity has no stored data: fall back to P(u)
    const bool bo = B.beta[0][cs] && oslot >= 0;
    if (bo) {
        const int slot = oslot;
        for (int it = tid; it < NV * NSUB; it += 128) vs[it] = B.pool[0][(int64_t)slot * NV * NSUB + it];
        __syncthreads();
    } else {
        for (int it = tid; it < NV * NN; it += 128) {
            const int v = it / NN, a = it % NN;
            us[it] = uo[((int64_t)v * P.ncell + cs) * NN + a];
        }
        __syncthreads();
        tensor_apply<DIM, NS, n, NV, MAXN>(&T->P[0][0], us, vs, tmp, tid, 128);
    }
    const double t0 = B.scal[1];
    double lo[NV], hi[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) {
        lo[v] = INFINITY;
        hi[v] = -INFINITY;
    }
    for (int sg = tid; sg < NSUB; sg += 128) {
        int gs[3] = {sg % NS, (sg / NS) % NS, sg / (NS * NS)};
        int ss[3] = {gs[0], gs[1], gs[2]};
        for (int j = 0; j < DIM; j++)
            if (mir[j]) ss[j] = NS - 1 - gs[j];
        int sidx = 0;
        for (int j = DIM - 1; j >= 0; j--) sidx = sidx * NS + ss[j];
        double q[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) q[v] = vs[v * NSUB + sidx];
        double x[3] = {0, 0, 0};
#pragma unroll
        for (int j = 0; j < DIM; j++) x[j] = P.lo[j] + P.h[j] * (ei[j] + (gs[j] + 0.5) / NS);
#pragma unroll
        for (int j = 0; j < DIM; j++) {
            if (gside[j] >= 0) {
                double qo[NV];
                bc_ghost<DIM>(P, j, gside[j], q, x[0], x[1], x[2], t0, qo);
#pragma unroll
                for (int v = 0; v < NV; v++) q[v] = qo[v];
            }
        }
#pragma unroll
        for (int v = 0; v < NV; v++) {
            lo[v] = fmin(lo[v], q[v]);
            hi[v] = fmax(hi[v], q[v]);
        }
    }
    block_minmax<NV>(lo, hi, tid, 128, red);
    if (tid == 0) {
        int64_t next = 1;
        for (int j = 0; j < DIM; j++) next *= ne[j];
#pragma unroll
        for (int j = 0; j < DIM; j++) {
            if (!istep[j]) continue;
            const double l = lo[1 + j];
            lo[1 + j] = -hi[1 + j];
            hi[1 + j] = -l;
        }
        for (int v = 0; v < NV; v++) {
            B.ext_min[0][(int64_t)v * next + e] = lo[v];
            B.ext_max[0][(int64_t)v * next + e] = hi[v];
        }
    }
}
// nblk: extended cells of the launch (large cells: the grid loops over them)
template <int DIM, int N>
__global__ __launch_bounds__(128) void k_cell_bounds(const Tables *__restrict__ T, Prob P, Bufs B, int cur,
                                                     const int64_t *__restrict__ ring, int64_t nblk) {
    if constexpr (BigCell<DIM, N>::on) {
        for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
            cell_bounds_block<DIM, N>(T, P, B, cur, ring, b);
            __syncthreads();
        }
    } else {
        cell_bounds_block<DIM, N>(T, P, B, cur, ring, blockIdx.x);
    }
}

// ------------------------------------------------------------------ compaction
// Troubled cells and unlimited neighbours of troubled cells, compacted in cell order
// with wavefront ballots and a block prefix; two passes (count, with the scan of the
// block counts done by the last block to finish, then scatter).
__device__ __forceinline__ bool corr_flag(const Prob &P, const uint8_t *beta, const uint8_t *mask, int64_t c) {
    if (beta[c] || (mask && mask[c])) return false;
    int ci[3];
    coords_of(P, c, ci);
    for (int k = 0; k < P.dim; k++)
        for (int side = 0; side < 2; side++) {
            int nb[3] = {ci[0], ci[1], ci[2]};
            nb[k] += side ? 1 : -1;
            if (nb[k] < 0 || nb[k] >= P.nc[k]) {
                if (!P.periodic[k]) continue;
                nb[k] = (nb[k] + P.nc[k]) % P.nc[k];
            }
            if (beta[cell_of(P, nb)]) return true;
        }
    return false;
}

constexpr int CBS = 256;   // compaction block size

__device__ __forceinline__ void compact_count_block(const Prob &P, const Bufs &B, int64_t cap, int64_t bid,
                                                    int64_t nblk_) {
    __shared__ int cnt[2][CBS / 64];
    __shared__ int last;
    __shared__ int carry[2];
    const int64_t c = (int64_t)bid * CBS + threadIdx.x;
    const bool t = c < P.ncell && B.beta[1][c];
    const bool f = c < P.ncell && corr_flag(P, B.beta[1], B.mask, c);
    const uint64_t bt = __ballot(t), bf = __ballot(f);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        cnt[0][wv] = __popcll(bt);
        cnt[1][wv] = __popcll(bf);
    }
    __syncthreads();
    const int nblk = (int)nblk_;
    if (threadIdx.x == 0) {
        int s0 = 0, s1 = 0;
        for (int w = 0; w < CBS / 64; w++) { s0 += cnt[0][w]; s1 += cnt[1][w]; }
        B.blk[bid] = s0;
        B.blk[nblk + bid] = s1;
        __threadfence();
        // the block that arrives last (no block waits for another) turns the block
        // counts into exclusive offsets
        last = (atomicAdd(&B.counts[4], 1) == nblk - 1);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    if (threadIdx.x == 0) { carry[0] = 0; carry[1] = 0; }
    __syncthreads();
    for (int base = 0; base < nblk; base += CBS) {
        const int i = base + threadIdx.x;
        int v0 = 0, v1 = 0;
        if (i < nblk) {
            v0 = __atomic_load_n(&B.blk[i], __ATOMIC_RELAXED);
            v1 = __atomic_load_n(&B.blk[nblk + i], __ATOMIC_RELAXED);
        }
        // inclusive scan: within each wave by shuffles, then across the waves' totals
        int x0 = v0, x1 = v1;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y0 = __shfl_up(x0, off), y1 = __shfl_up(x1, off);
            if (lane >= off) { x0 += y0; x1 += y1; }
        }
        if (lane == 63) { cnt[0][wv] = x0; cnt[1][wv] = x1; }
        __syncthreads();
        int p0 = carry[0], p1 = carry[1];
        for (int w = 0; w < wv; w++) { p0 += cnt[0][w]; p1 += cnt[1][w]; }
        if (i < nblk) {
            B.blk[i] = p0 + x0 - v0;
            B.blk[nblk + i] = p1 + x1 - v1;
        }
        __syncthreads();
        if (threadIdx.x == CBS - 1) { carry[0] = p0 + x0; carry[1] = p1 + x1; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        B.counts[0] = carry[0];
        B.counts[1] = carry[1];
        if (carry[0] > cap) B.counts[3] = 1;
        B.counts[4] = 0;   // ticket for the next step
        B.counts[5] = 0;   // MOOD layer: flagged subcells, recomputed cells of this step
        B.counts[6] = 0;
    }
}
static __global__ __launch_bounds__(CBS) void k_compact_count(Prob P, Bufs B, int64_t cap) {
    compact_count_block(P, B, cap, blockIdx.x, gridDim.x);
}

__device__ __forceinline__ void compact_scatter_block(const Prob &P, const Bufs &B, int64_t cap, int64_t bid,
                                                      int64_t nblk) {
    __shared__ int woff[2][CBS / 64];
    const int64_t c = (int64_t)bid * CBS + threadIdx.x;
    const bool t = c < P.ncell && B.beta[1][c];
    const bool f = c < P.ncell && corr_flag(P, B.beta[1], B.mask, c);
    const uint64_t bt = __ballot(t), bf = __ballot(f);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (lane == 0) {
        woff[0][wv] = __popcll(bt);
        woff[1][wv] = __popcll(bf);
    }
    __syncthreads();
    int o0 = B.blk[bid], o1 = B.blk[nblk + bid];
    for (int w = 0; w < wv; w++) { o0 += woff[0][w]; o1 += woff[1][w]; }
    if (c < P.ncell) {
        int slot = -1;
        if (t) {
            const int idx = o0 + __popcll(bt & below);
            if (idx < cap) {
                B.tlist[idx] = (int)c;
                slot = idx;
            }
        }
        B.slot[1][c] = slot;
        if (f) B.clist[o1 + __popcll(bf & below)] = (int)c;
    }
}
static __global__ __launch_bounds__(CBS) void k_compact_scatter(Prob P, Bufs B, int64_t cap) {
    compact_scatter_block(P, B, cap, blockIdx.x, gridDim.x);
}

// ------------------------------------------------------ subcell ADER-WENO3
constexpr int SUB_BS = 256;   // threads per workgroup of the subcell recompute

// Workgroups of the subcell recompute per CU (= waves per SIMD), the register budget held to
// it (Tune's sub_wps: by default three for 2D cells up to N = 5, two for larger cells and in 3D).
template <int DIM, int N, typename R>
struct SubShape {
    static constexpr int WPS = Tune<DIM, N, sizeof(R) == 4>::sub_wps;
};


// Positions of one troubled cell's subcell scheme: the Ns^d own subcells first, then
// for each axis k and side the Ns^(d-1) face-adjacent subcells of the neighbour.
template <int DIM>
__device__ __forceinline__ void position_coords(int pos, int Ns, int *L) {
    const int nsub = (DIM == 2) ? Ns * Ns : Ns * Ns * Ns;
    const int nsf = (DIM == 2) ? Ns : Ns * Ns;
    if (pos < nsub) {
        L[0] = pos % Ns;
        L[1] = (pos / Ns) % Ns;
        L[2] = (DIM == 3) ? pos / (Ns * Ns) : 0;
        return;
    }
    const int r = pos - nsub;
    const int face = r / nsf, sp = r % nsf;
    const int k = face >> 1, side = face & 1;
    int tmp = sp;
    for (int j = 0; j < DIM; j++) {
        if (j == k) {
            L[j] = side ? Ns : -1;
            continue;
        }
        L[j] = tmp % Ns;
        tmp /= Ns;
    }
    if (DIM == 2) L[2] = 0;
}

// S1: halo of subcell data v^n (eq. (ader.icbc)) 3 subcells deep around the cell, into
// halo[v][HN^d].  Troubled cell number w of the worklist.  The 3^d source cells of the halo
// (the cell, its neighbours, or the interior cells a non-periodic ghost mirrors) have their
// DG coefficients staged in LDS first (nbu, 3^d x NV x n^d values; null: read from HBM).
template <int DIM, int N>
__device__ __forceinline__ void sub_halo_cell(const Tables *__restrict__ T, const Prob &P, const Bufs &B, int cur, int w,
                              double *halo, double *nbu) {
    constexpr int n = N + 1, NV = DIM + 2, NN = cpow(n, DIM);
    constexpr int NS = 2 * N + 1, NSUB = cpow(NS, DIM), HN = NS + 6, HSZ = cpow(HN, DIM), NB = cpow(3, DIM);
    const int64_t c = B.tlist[w];
    int ci[3];
    coords_of(P, c, ci);
    const double t0 = B.scal[1];
    // source cell of the cell at global coordinates gci (possibly outside the domain)
    auto source = [&](const int *gci, int *src, int *mir, int *gside) {
        for (int j = 0; j < 3; j++) {
            src[j] = j < DIM ? gci[j] : 0;
            mir[j] = 0;
            gside[j] = -1;
        }
        for (int j = 0; j < DIM; j++) {
            if (gci[j] < 0 || gci[j] >= P.nc[j]) {
                const int side = gci[j] >= P.nc[j];
                if (P.periodic[j]) {
                    src[j] = (gci[j] + P.nc[j]) % P.nc[j];
                } else {
                    src[j] = side ? 2 * P.nc[j] - 1 - gci[j] : -1 - gci[j];
                    mir[j] = 1;
                    gside[j] = side;
                }
            }
        }
    };
    if (nbu) {
        for (int i = threadIdx.x; i < NB * NV * NN; i += blockDim.x) {
            const int o = i / (NV * NN), v = (i / NN) % NV, a = i % NN;
            int gci[3] = {0, 0, 0};
            for (int j = 0, r = o; j < DIM; j++, r /= 3) gci[j] = ci[j] + r % 3 - 1;
            int src[3], mir[3], gside[3];
            source(gci, src, mir, gside);
            nbu[i] = B.u[cur][((int64_t)v * P.ncell + cell_of(P, src)) * NN + a];
        }
        __syncthreads();
    }
    for (int hidx = threadIdx.x; hidx < HSZ; hidx += blockDim.x) {
        int hl[3] = {hidx % HN, (hidx / HN) % HN, hidx / (HN * HN)};
        int off[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, ss[3] = {0, 0, 0};
        for (int j = 0; j < DIM; j++) {
            const int Lj = hl[j] - 3;
            off[j] = Lj < 0 ? -1 : (Lj >= NS ? 1 : 0);
            gs[j] = Lj - off[j] * NS;
        }
        int gci[3] = {0, 0, 0};
        for (int j = 0; j < DIM; j++) gci[j] = ci[j] + off[j];
        // masked geometry: a solid cell holds the mirror image of the fluid across its walls
        // (the image cell's subcells reversed along the mirrored axes, their momenta negated)
        int istep[3] = {0, 0, 0};
        bool staged = nbu != nullptr;
        if (B.mask && solid_at<DIM>(P, B.mask, gci[0], gci[1], gci[2])) {
            solid_image<DIM>(P, B.mask, gci, istep);
#pragma unroll
            for (int j = 0; j < DIM; j++)
                if (istep[j]) {
                    gci[j] += istep[j];
                    gs[j] = NS - 1 - gs[j];
                    staged = false;   // the image cell may lie outside the staged block
                }
        }
        int src[3], mir[3], gside[3];
        source(gci, src, mir, gside);
        for (int j = 0; j < DIM; j++) ss[j] = mir[j] ? NS - 1 - gs[j] : gs[j];
        const int64_t cs = cell_of(P, src);
        int sidx = 0;
        for (int j = DIM - 1; j >= 0; j--) sidx = sidx * NS + ss[j];
        double q[NV];
        const int slot = B.slot[0][cs];
        if (B.beta[0][cs] && slot >= 0) {
#pragma unroll
            for (int v = 0; v < NV; v++) q[v] = B.pool[0][((int64_t)slot * NV + v) * NSUB + sidx];
        } else {
            // P(u^n) at one subcell: plain tensor sum over the nodes
            int o = 0;
            for (int j = DIM - 1; j >= 0; j--) o = o * 3 + (off[j] + 1);
            const double *nb = staged ? nbu : nullptr;
#pragma unroll
            for (int v = 0; v < NV; v++) q[v] = 0.0;
            for (int a = 0; a < NN; a++) {
                int m[3] = {a % n, (a / n) % n, a / (n * n)};
                double wgt = 1.0;
                for (int j = 0; j < DIM; j++) wgt *= T->P[ss[j]][m[j]];
#pragma unroll
                for (int v = 0; v < NV; v++)
                    q[v] += wgt * (nb ? nb[(o * NV + v) * NN + a] : B.u[cur][((int64_t)v * P.ncell + cs) * NN + a]);
            }
        }
        double x[3] = {0, 0, 0};
        for (int j = 0; j < DIM; j++) x[j] = P.lo[j] + P.h[j] * (gci[j] + (gs[j] + 0.5) / NS);
        for (int j = 0; j < DIM; j++) {
            if (gside[j] < 0) continue;
            double qo[NV];
            bc_ghost<DIM>(P, j, gside[j], q, x[0], x[1], x[2], t0, qo);
#pragma unroll
            for (int v = 0; v < NV; v++) q[v] = qo[v];
        }
#pragma unroll
        for (int j = 0; j < DIM; j++)
            if (istep[j]) q[1 + j] = -q[1 + j];
#pragma unroll
        for (int v = 0; v < NV; v++) halo[v * HSZ + hidx] = q[v];
    }
}

// S1 in 3D: the halo region by region.  The halo's 3^3 regions are the parts of the 3x3x3 block
// of cells around the troubled cell that lie within three subcells of it (the cell itself,
// three-subcell slabs of its face neighbours, bars of the edge neighbours, cubes of the corner
// neighbours).  Each region has one source cell (the neighbour, its periodic image, the
// interior cell a boundary ghost mirrors, or the fluid image of a solid cell), whose subcells
// the region needs on a box; P(u^n) (eq. (subcell.p)) is sum-factorised over that box axis by
// axis (x, then y, then z) instead of summed over the n^3 nodes at every halo point.  A source
// cell troubled at the previous step gives its stored subcell data instead.  st: scratch of
// NV (NS n^2 + NS^2 n) doubles for the first two stages.
template <int N>
__device__ __forceinline__ void sub_halo_cell3(const Tables *__restrict__ T, const Prob &P, const Bufs &B, int cur, int w,
                                               double *halo, double *st) {
    constexpr int DIM = 3, n = N + 1, NV = 5, NN = n * n * n;
    constexpr int NS = 2 * N + 1, NSUB = NS * NS * NS, HN = NS + 6, HSZ = HN * HN * HN;
    double *st1 = st, *st2 = st + NV * NS * n * n;
    const int64_t c = B.tlist[w];
    int ci[3];
    coords_of(P, c, ci);
    const double t0 = B.scal[1];
    const double *u = B.u[cur];
    for (int o = 0; o < 27; o++) {
        const int off[3] = {o % 3 - 1, (o / 3) % 3 - 1, o / 9 - 1};
        // the region's box of local subcell coordinates gs: the last three subcells of a
        // neighbour below, all of the cell itself, the first three of a neighbour above
        int glo[3], gn[3], gci[3], istep[3] = {0, 0, 0};
#pragma unroll
        for (int j = 0; j < 3; j++) {
            glo[j] = off[j] < 0 ? NS - 3 : 0;
            gn[j] = off[j] == 0 ? NS : 3;
            gci[j] = ci[j] + off[j];
        }
        // masked geometry: a solid cell holds the mirror image of the fluid across its walls
        // (the image cell's subcells reversed along the mirrored axes, their momenta negated)
        if (B.mask && solid_at<DIM>(P, B.mask, gci[0], gci[1], gci[2])) {
            solid_image<DIM>(P, B.mask, gci, istep);
#pragma unroll
            for (int j = 0; j < 3; j++) gci[j] += istep[j];
        }
        // source cell; a non-periodic boundary mirrors the interior cell (gside: its side)
        int src[3], mir[3], gside[3];
#pragma unroll
        for (int j = 0; j < 3; j++) {
            src[j] = gci[j];
            mir[j] = 0;
            gside[j] = -1;
            if (gci[j] < 0 || gci[j] >= P.nc[j]) {
                const int side = gci[j] >= P.nc[j];
                if (P.periodic[j]) {
                    src[j] = (gci[j] + P.nc[j]) % P.nc[j];
                } else {
                    src[j] = side ? 2 * P.nc[j] - 1 - gci[j] : -1 - gci[j];
                    mir[j] = 1;
                    gside[j] = side;
                }
            }
        }
        // source subcell ss = gs, reversed along an axis where exactly one of the image and the
        // boundary mirror reverses it; the box of ss the region needs starts at sslo
        int flip[3], sslo[3];
#pragma unroll
        for (int j = 0; j < 3; j++) {
            flip[j] = (istep[j] != 0) != (mir[j] != 0);
            sslo[j] = flip[j] ? NS - glo[j] - gn[j] : glo[j];
        }
        const int64_t cs = cell_of(P, src);
        const int slot = B.slot[0][cs];
        const bool pooled = B.beta[0][cs] && slot >= 0;
        if (!pooled) {
            // stage 1 (x): st1[v][i0][a2][a1] = sum_a0 P[sslo0 + i0][a0] u[v][a0, a1, a2]
            const int n1 = NV * gn[0] * n * n;
            for (int it = threadIdx.x; it < n1; it += blockDim.x) {
                const int a12 = it % (n * n), i0 = (it / (n * n)) % gn[0], v = it / (n * n * gn[0]);
                const double *x = u + ((int64_t)v * P.ncell + cs) * NN + a12 * n;
                const double *pr = T->P[sslo[0] + i0];
                double acc = 0.0;
#pragma unroll
                for (int a0 = 0; a0 < n; a0++) acc += pr[a0] * x[a0];
                st1[it] = acc;
            }
            __syncthreads();
            // stage 2 (y): st2[v][i0][i1][a2] = sum_a1 P[sslo1 + i1][a1] st1[v][i0][a2][a1]
            const int n2 = NV * gn[0] * gn[1] * n;
            for (int it = threadIdx.x; it < n2; it += blockDim.x) {
                const int a2 = it % n, i1 = (it / n) % gn[1], vi0 = it / (n * gn[1]);   // vi0 = v * gn0 + i0
                const double *x = st1 + ((int64_t)vi0 * n + a2) * n;     // st1[v][i0][a2][a1], a1 fastest
                const double *pr = T->P[sslo[1] + i1];
                double acc = 0.0;
#pragma unroll
                for (int a1 = 0; a1 < n; a1++) acc += pr[a1] * x[a1];
                st2[it] = acc;
            }
            __syncthreads();
        }
        // stage 3 (z) per halo point of the region, all variables, then the boundary rules
        const int np = gn[0] * gn[1] * gn[2];
        for (int it = threadIdx.x; it < np; it += blockDim.x) {
            const int i[3] = {it % gn[0], (it / gn[0]) % gn[1], it / (gn[0] * gn[1])};
            int ss[3], gsI[3], hl[3];
#pragma unroll
            for (int j = 0; j < 3; j++) {
                ss[j] = sslo[j] + i[j];
                gsI[j] = mir[j] ? NS - 1 - ss[j] : ss[j];                 // local coordinate in the (image) cell
                const int gs0 = istep[j] ? NS - 1 - gsI[j] : gsI[j];      // in the halo's own cell
                hl[j] = gs0 + off[j] * NS + 3;
            }
            double q[NV];
            if (pooled) {
                const int sidx = ss[0] + NS * (ss[1] + NS * ss[2]);
#pragma unroll
                for (int v = 0; v < NV; v++) q[v] = B.pool[0][((int64_t)slot * NV + v) * NSUB + sidx];
            } else {
                const double *pr = T->P[ss[2]];
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    const double *x = st2 + (((int64_t)v * gn[0] + i[0]) * gn[1] + i[1]) * n;
                    double acc = 0.0;
#pragma unroll
                    for (int a2 = 0; a2 < n; a2++) acc += pr[a2] * x[a2];
                    q[v] = acc;
                }
            }
            double x[3];
#pragma unroll
            for (int j = 0; j < 3; j++) x[j] = P.lo[j] + P.h[j] * (gci[j] + (gsI[j] + 0.5) / NS);
#pragma unroll
            for (int j = 0; j < 3; j++) {
                if (gside[j] < 0) continue;
                double qo[NV];
                bc_ghost<DIM>(P, j, gside[j], q, x[0], x[1], x[2], t0, qo);
#pragma unroll
                for (int v = 0; v < NV; v++) q[v] = qo[v];
            }
#pragma unroll
            for (int j = 0; j < 3; j++)
                if (istep[j]) q[1 + j] = -q[1 + j];
            const int hidx = hl[0] + HN * (hl[1] + HN * hl[2]);
#pragma unroll
            for (int v = 0; v < NV; v++) halo[v * HSZ + hidx] = q[v];
        }
        __syncthreads();   // the stage buffers are reused by the next region
    }
}

// One-dimensional WENO3 (degree 2, three stencils, lambda = 1, 1e5, 1, eps 1e-14, r 8):
// five averages at offsets -2..2 -> values at the three GL nodes of the central subcell.
__device__ __forceinline__ void weno3(const Tables *__restrict__ T, const double *a, double *out) {
    double c[3][3], wt[3], sum = 0.0;
    const double lam[3] = {1.0, 1.0e5, 1.0};
#pragma unroll
    for (int st = 0; st < 3; st++) {
#pragma unroll
        for (int p = 0; p < 3; p++) {
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < 3; m++) acc += T->weno[st][p][m] * a[st + m];
            c[st][p] = acc;
        }
        const double sig = c[st][1] * c[st][1] + 2.0 * c[st][1] * c[st][2] + (16.0 / 3.0) * c[st][2] * c[st][2];
        double s2 = sig + 1e-14;
        s2 = s2 * s2;
        s2 = s2 * s2;
        s2 = s2 * s2;   // (sigma + eps)^8
        wt[st] = lam[st] / s2;
        sum += wt[st];
    }
    const double isum = 1.0 / sum;
#pragma unroll
    for (int qn = 0; qn < 3; qn++) {
        const double x = T->xi3[qn];
        double acc = 0.0;
#pragma unroll
        for (int st = 0; st < 3; st++) acc += (wt[st] * isum) * (c[st][0] + c[st][1] * x + c[st][2] * x * x);
        out[qn] = acc;
    }
}

// FP32 variant (mixed form): the same weights, each scaled by (sigma_min + eps)^8, i.e.
// lambda_k ((sigma_min + eps) / (sigma_k + eps))^8 before normalisation, so that they stay in
// FP32 range (the unscaled (sigma + eps)^-8 overflows for eps = 1e-14); reciprocals by the
// hardware reciprocal.
__device__ __forceinline__ void weno3(const Tables *__restrict__ T, const float *a, float *out) {
    float c[3][3], sg[3];
    const float lam[3] = {1.0f, 1.0e5f, 1.0f};
#pragma unroll
    for (int st = 0; st < 3; st++) {
#pragma unroll
        for (int p = 0; p < 3; p++) {
            float acc = 0.0f;
#pragma unroll
            for (int m = 0; m < 3; m++) acc += T->fweno[st][p][m] * a[st + m];
            c[st][p] = acc;
        }
        sg[st] = c[st][1] * c[st][1] + 2.0f * c[st][1] * c[st][2] + (16.0f / 3.0f) * c[st][2] * c[st][2] + 1e-14f;
    }
    const float smin = fminf(sg[0], fminf(sg[1], sg[2]));
    float wt[3], sum = 0.0f;
#pragma unroll
    for (int st = 0; st < 3; st++) {
        float r = smin * __builtin_amdgcn_rcpf(sg[st]);
        r = r * r;
        r = r * r;
        r = r * r;
        wt[st] = lam[st] * r;
        sum += wt[st];
    }
    const float isum = __builtin_amdgcn_rcpf(sum);
#pragma unroll
    for (int qn = 0; qn < 3; qn++) {
        const float x = T->fxi3[qn];
        float acc = 0.0f;
#pragma unroll
        for (int st = 0; st < 3; st++) acc += (wt[st] * isum) * (c[st][0] + c[st][1] * x + c[st][2] * x * x);
        out[qn] = acc;
    }
}

// S2: dimension-by-dimension WENO3 reconstruction at every position -> nodal values at
// the 3^d GL points of the subcell (x sweep on the averages, then y (then z) sweeps on
// the nodal values of the previous sweep).  One work item per (position, variable).
template <int DIM, int N, typename R>
__device__ __forceinline__ void sub_recon_cell(const Tables *__restrict__ T, double *Yscratch, int sidx, const double *halo,
                                               R *stg) {
    constexpr int NV = DIM + 2, NS = 2 * N + 1, HN = NS + 6, HSZ = cpow(HN, DIM);
    constexpr int NPOS = cpow(NS, DIM) + 2 * DIM * cpow(NS, DIM - 1), N3 = cpow(3, DIM);
    if constexpr (DIM == 2) {
        (void)stg;
        for (int item = threadIdx.x; item < NPOS * NV; item += blockDim.x) {
            const int v = item / NPOS, pos = item % NPOS;
            int L[3];
            position_coords<DIM>(pos, NS, L);
            const double *h = halo + v * HSZ;
            R *Y = reinterpret_cast<R *>(Yscratch) + ((int64_t)sidx * NPOS + pos) * NV * N3 + v * N3;
            // x sweep on the five rows of the 5 x 5 stencil, then y sweep per x node
            R w1[5][3];
#pragma unroll
            for (int r = 0; r < 5; r++) {
                R a5[5];
#pragma unroll
                for (int o = 0; o < 5; o++) a5[o] = (R)h[(L[1] + r + 1) * HN + (L[0] + o + 1)];
                weno3(T, a5, w1[r]);
            }
#pragma unroll
            for (int qx = 0; qx < 3; qx++) {
                R a5[5], o3[3];
#pragma unroll
                for (int r = 0; r < 5; r++) a5[r] = w1[r][qx];
                weno3(T, a5, o3);
#pragma unroll
                for (int qy = 0; qy < 3; qy++) Y[qy * 3 + qx] = o3[qy];
            }
        }
    } else {
        // 3D: the sweeps are shared between positions.  x sweep of every halo row at the x
        // coordinates of the positions (-1 .. Ns), then the y sweep per x node at their (x, y)
        // coordinates, both into stg; then per position the z sweep per (y, x) node.  The same
        // WENO3 evaluations on the same values as one position at a time (three times fewer).
        constexpr int NI = NS + 2;
        static_assert((int64_t)NV * NI * HN * HN * 3 + (int64_t)NV * NI * NI * HN * 9 <=
                          (int64_t)NPOS * 2 * DIM * NV * cpow(3, DIM - 1) * 3,
                      "the sweeps' intermediates must fit the slot's trace storage");
        R *vx = stg;                                           // [v][i][kh][jh][qx]
        R *vxy = stg + (int64_t)NV * NI * HN * HN * 3;         // [v][i][j][kh][qy][qx]
        for (int it = threadIdx.x; it < NV * NI * HN * HN; it += blockDim.x) {
            const int jh = it % HN, kh = (it / HN) % HN, i = (it / (HN * HN)) % NI, v = it / (HN * HN * NI);
            const double *h = halo + (int64_t)v * HSZ + (kh * HN + jh) * HN + i;
            R a5[5], o3[3];
#pragma unroll
            for (int o = 0; o < 5; o++) a5[o] = (R)h[o];
            weno3(T, a5, o3);
#pragma unroll
            for (int q = 0; q < 3; q++) vx[(int64_t)it * 3 + q] = o3[q];
        }
        __syncthreads();
        for (int it = threadIdx.x; it < NV * NI * NI * HN * 3; it += blockDim.x) {
            const int qx = it % 3, kh = (it / 3) % HN, j = (it / (3 * HN)) % NI;
            const int i = (it / (3 * HN * NI)) % NI, v = it / (3 * HN * NI * NI);
            const R *src = vx + ((((int64_t)v * NI + i) * HN + kh) * HN + j) * 3 + qx;
            R a5[5], o3[3];
#pragma unroll
            for (int y = 0; y < 5; y++) a5[y] = src[y * 3];
            weno3(T, a5, o3);
            R *dst = vxy + ((((int64_t)v * NI + i) * NI + j) * HN + kh) * 9 + qx;
#pragma unroll
            for (int qy = 0; qy < 3; qy++) dst[qy * 3] = o3[qy];
        }
        __syncthreads();
        for (int it = threadIdx.x; it < NPOS * NV * 9; it += blockDim.x) {
            const int qq = it % 9, item = it / 9;
            const int v = item / NPOS, pos = item % NPOS;
            int L[3];
            position_coords<DIM>(pos, NS, L);
            const R *src = vxy + ((((int64_t)v * NI + (L[0] + 1)) * NI + (L[1] + 1)) * HN + (L[2] + 1)) * 9 + qq;
            R a5[5], o3[3];
#pragma unroll
            for (int z = 0; z < 5; z++) a5[z] = src[z * 9];
            weno3(T, a5, o3);
            R *Y = reinterpret_cast<R *>(Yscratch) + ((int64_t)sidx * NPOS + pos) * NV * N3 + v * N3 + qq;
#pragma unroll
            for (int qz = 0; qz < 3; qz++) Y[qz * 9] = o3[qz];
        }
    }
}

// S4: sub-face Rusanov fluxes, FV update, gather, pool store, boundary fluxes.
// MOOD layer (Sec. 6, Fig. algo2): with flagging set, every subcell of the WENO3 result
// that fails PAD or the relaxed DMP against this cell's bounds (mb) is flagged; REDO
// recomputes with the first-order flux on every sub-face next to a flagged subcell (own
// flags, or the face neighbour's, whose pool slot is in nslot).
template <int DIM, int N, typename R, bool REDO>
__device__ __forceinline__ void sub_update_cell(const Tables *__restrict__ T, const Prob &P, const Bufs &B, int cur,
                                                int w, int sidx, const SubScratch &S, int *nonphys, const double *halo,
                                                int flagging,
                                                const double (*mb)[DIM + 2], const int (*nslot)[2],
                                                unsigned char *fbt) {
    constexpr int n = N + 1, NV = DIM + 2, NN = cpow(n, DIM);
    constexpr int NS = 2 * N + 1, NSUB = cpow(NS, DIM), NSF = cpow(NS, DIM - 1), HN = NS + 6, HSZ = cpow(HN, DIM);
    constexpr int NPOS = NSUB + 2 * DIM * NSF, NF3 = cpow(3, DIM - 1);
    constexpr int TRS = 2 * DIM * NV * NF3 * 3;   // trace size per position
    constexpr int BIG = NSUB > NN ? NSUB : NN;
    constexpr int QF = cpow(3 * NS, DIM - 1);     // tangential quadrature points of one face
    constexpr int NFN = cpow(n, DIM - 1);
    // sub-face fluxes (working precision), later the gather's intermediate stage
    constexpr int FBB = DIM * (NS + 1) * NSF * NV * (int)sizeof(R), TMB = NV * BIG * 8;
    R *Fb;
    double *tmp, *vn, *ug;
    if constexpr (BigCell<DIM, N>::on) {
        // large cells: the workgroup's global slot
        using BC = BigCell<DIM, N>;
        double *slot = S.big + (int64_t)sidx * BC::SLOT;
        Fb = reinterpret_cast<R *>(slot);
        tmp = slot;
        vn = slot + BC::SUB_VN;
        ug = slot + BC::SUB_UG;
    } else {
        // fbt: LDS of FBB > TMB ? FBB : TMB bytes (declared by the caller)
        __shared__ double vn_[NV * BIG];
        __shared__ double ug_[NV * BIG];
        Fb = reinterpret_cast<R *>(fbt);
        tmp = reinterpret_cast<double *>(fbt);
        vn = vn_;
        ug = ug_;
    }
    __shared__ double red[2 * NV * (SUB_BS / 64)];
    __shared__ int badc;
    const int ch = sidx;
    const int64_t c = B.tlist[w];
    int ci[3];
    coords_of(P, c, ci);
    const double dt = B.scal[0], t0 = B.scal[1];
    const R *tr = reinterpret_cast<const R *>(S.strace) + (int64_t)ch * NPOS * TRS;
    const R gam = (R)P.gamma;
    if (threadIdx.x == 0) badc = 0;
    // neighbour existence per face of the cell: bit 2k + side; a face toward a solid cell
    // (masked geometry) has no neighbour and is a reflective wall (the same bit of nbwall)
    int nbex = 0, nbwall = 0;
#pragma unroll
    for (int k = 0; k < DIM; k++)
#pragma unroll
        for (int side = 0; side < 2; side++) {
            const int nb = ci[k] + (side ? 1 : -1);
            if (P.periodic[k] || (nb >= 0 && nb < P.nc[k])) {
                const int g0 = ci[0] + (k == 0 ? (side ? 1 : -1) : 0);
                const int g1 = ci[1] + (k == 1 ? (side ? 1 : -1) : 0);
                const int g2 = ci[2] + (k == 2 ? (side ? 1 : -1) : 0);
                if (B.mask && solid_at<DIM>(P, B.mask, g0, g1, g2)) nbwall |= 1 << (2 * k + side);
                else nbex |= 1 << (2 * k + side);
            }
        }
    // Sub-face fluxes.  A sub-face is handled by NF3 consecutive lanes of one wave, one per
    // tangential quadrature point (64 / NF3 sub-faces per wave); a wave takes a run of
    // sub-faces of one axis, so the body is instantiated per axis (compile-time k: no dynamic
    // indexing of per-thread arrays).  The lanes of a sub-face agree on the positivity
    // fallback by a ballot and the first of them sums the tangential points in order.
    constexpr int SPW = 64 / NF3;
    constexpr int PA = (NS + 1) * NSF, WPA = (PA + SPW - 1) / SPW;   // sub-faces, waves per axis
    const int lane = threadIdx.x & 63, sfl = lane / NF3, ap = lane % NF3;
    for (int wt = threadIdx.x >> 6; wt < DIM * WPA; wt += SUB_BS / 64) {
        const int kk = wt / WPA;
        const int it2r = (wt % WPA) * SPW + sfl;
        const bool valid = sfl < SPW && it2r < PA;
        const int it2 = valid ? it2r : 0;   // idle lanes work on an in-range sub-face, store nothing
        const int it = kk * PA + it2;       // sub-face index: axis-major, then face, then tangential
        auto subface = [&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const int f = it2 / NSF;
            const int sp = it2 % NSF;
            // subcell coordinate along axis j of the sub-face's tangential position (j != k):
            // the first tangential axis takes sp % NS, the second sp / NS
            const int mp0 = sp % NS, mp1 = sp / NS;
            auto tang = [&](int j) -> int { return (j < k ? j : j - 1) == 0 ? mp0 : mp1; };
            // positions left (f-1) and right (f) of the sub-face
            auto pos_of = [&](int Lk) -> int {
                if (Lk >= 0 && Lk < NS) {
                    int idx = 0;
#pragma unroll
                    for (int j = DIM - 1; j >= 0; j--) idx = idx * NS + (j == k ? Lk : tang(j));
                    return idx;
                }
                return NSUB + (2 * k + (Lk >= NS ? 1 : 0)) * NSF + sp;
            };
            const int pL = pos_of(f - 1), pR = pos_of(f);
            int low = 0;
            if constexpr (REDO) {
                // flags of the subcells on both sides: own subcells, or the neighbour's layer
                const int own = B.slot[1][B.tlist[w]];
                auto flag_at = [&](int Lk) -> int {
                    int sl = own, side = -1;
                    if (Lk < 0) { side = 0; Lk += NS; }
                    if (Lk >= NS) { side = 1; Lk -= NS; }
                    if (side >= 0) sl = nslot[k][side];
                    if (sl < 0) return 0;
                    int idx = 0;
#pragma unroll
                    for (int j = DIM - 1; j >= 0; j--) idx = idx * NS + (j == k ? Lk : tang(j));
                    return B.mflag[(int64_t)sl * NSUB + idx];
                };
                low = flag_at(f - 1) | flag_at(f);
            }
            const int bside = (f == 0 && !((nbex >> (2 * k)) & 1)) ? 0 : ((f == NS && !((nbex >> (2 * k + 1)) & 1)) ? 1 : -1);
            // subcell averages of both sides (halo coordinates: local subcell + 3)
            double avL[NV], avR[NV];
            {
                int hL = 0, hR = 0;
#pragma unroll
                for (int j = DIM - 1; j >= 0; j--) {
                    hL = hL * HN + ((j == k ? f - 1 : tang(j)) + 3);
                    hR = hR * HN + ((j == k ? f : tang(j)) + 3);
                }
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    avL[v] = halo[v * HSZ + hL];
                    avR[v] = halo[v * HSZ + hR];
                }
            }
            // this lane's tangential quadrature point: position and weight
            const int ma0 = ap % 3, ma1 = ap / 3;
            double wtan = 1.0;
            double x[3] = {0, 0, 0};
#pragma unroll
            for (int j = 0; j < DIM; j++) {
                if (j == k) {
                    x[j] = P.lo[j] + P.h[j] * (ci[j] + (double)f / NS);
                } else {
                    const bool first = (j < k ? j : j - 1) == 0;
                    const int ma = first ? ma0 : ma1;
                    wtan *= T->w3[ma];
                    x[j] = P.lo[j] + P.h[j] * (ci[j] + ((first ? mp0 : mp1) + T->xi3[ma]) / NS);
                }
            }
            // the time-averaged flux at the point: on the predictor's traces (pass 0) or, the
            // positivity fallback, the first-order Rusanov flux of the two subcell averages
            R Gt[NV];
            auto point_flux = [&](int pass) -> bool {
#pragma unroll
                for (int v = 0; v < NV; v++) Gt[v] = 0;
                for (int s = 0; s < 3; s++) {
                    R qL[NV], qR[NV], G[NV];
                    const double ts = t0 + T->xi3[s] * dt;
                    const R *trL = tr + (int64_t)pL * TRS + (2 * k + 1) * NV * NF3 * 3;
                    const R *trR = tr + (int64_t)pR * TRS + (2 * k + 0) * NV * NF3 * 3;
#pragma unroll
                    for (int v = 0; v < NV; v++) {
                        qL[v] = pass ? (R)avL[v] : trL[v * NF3 * 3 + ap + NF3 * s];
                        qR[v] = pass ? (R)avR[v] : trR[v * NF3 * 3 + ap + NF3 * s];
                    }
                    if (bside >= 0 && ((nbwall >> (2 * k + bside)) & 1)) {
                        // reflective wall of the masked geometry
                        if (bside == 0) wall_ghost<DIM, R>(k, qR, qL);
                        else wall_ghost<DIM, R>(k, qL, qR);
                    } else if (bside >= 0) {
                        // ghost state of the boundary rule, evaluated in FP64
                        double qi[NV], qo[NV];
                        if (bside == 0) {
#pragma unroll
                            for (int v = 0; v < NV; v++) qi[v] = (double)qR[v];
                            bc_ghost<DIM>(P, k, 0, qi, x[0], x[1], x[2], ts, qo);
#pragma unroll
                            for (int v = 0; v < NV; v++) qL[v] = (R)qo[v];
                        } else {
#pragma unroll
                            for (int v = 0; v < NV; v++) qi[v] = (double)qL[v];
                            bc_ghost<DIM>(P, k, 1, qi, x[0], x[1], x[2], ts, qo);
#pragma unroll
                            for (int v = 0; v < NV; v++) qR[v] = (R)qo[v];
                        }
                    }
                    if (!pass && !(physical<DIM, R>(qL, gam) && physical<DIM, R>(qR, gam))) return false;
                    // the scheme's flux on the traces; the first-order fallback uses Rusanov
                    if (pass) rusanov<DIM, R>(k, qL, qR, G, gam);
                    else num_flux<DIM, R>(P, T, k, qL, qR, G);
#pragma unroll
                    for (int v = 0; v < NV; v++) Gt[v] += (R)T->w3[s] * G[v];
                }
                return true;
            };
            // Positivity safeguard: if any predictor trace on either side of the sub-face is
            // not a physical state, the whole sub-face takes the first-order flux.
            const bool ok = low ? false : point_flux(0);
            const uint64_t badm = __ballot(valid && !ok);
            const bool fallback = ((badm >> (sfl * NF3)) & ((1ull << NF3) - 1ull)) != 0ull;
            if (fallback) point_flux(1);
            // a sub-face on the cell's own face keeps its time-averaged flux at each tangential
            // quadrature point for the flux correction of the neighbour
            if (valid && (f == 0 || f == NS)) {
                double *fp = S.fpts + ((int64_t)ch * 2 * DIM + 2 * k + (f == NS ? 1 : 0)) * NV * QF;
                const int q = (mp0 * 3 + ma0) + 3 * NS * (mp1 * 3 + ma1);
#pragma unroll
                for (int v = 0; v < NV; v++) fp[v * QF + q] = (double)Gt[v];
            }
            // the sub-face flux: the tangential points' fluxes times their weights, summed in
            // order by the sub-face's first lane
            R Fbar[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) Fbar[v] = 0;
            const R wl = (R)wtan;
#pragma unroll
            for (int a2 = 0; a2 < NF3; a2++) {
                const int src = min(sfl * NF3 + a2, 63);
                const R w2 = __shfl(wl, src);
#pragma unroll
                for (int v = 0; v < NV; v++) Fbar[v] += w2 * __shfl(Gt[v], src);
            }
            if (valid && ap == 0) {
#pragma unroll
                for (int v = 0; v < NV; v++) Fb[it * NV + v] = Fbar[v];
            }
        };
        if (kk == 0) subface(std::integral_constant<int, 0>{});
        else if (kk == 1) subface(std::integral_constant<int, 1>{});
        else subface(std::integral_constant<int, DIM - 1>{});
    }
    __syncthreads();
    // FV update of the cell's own subcells
    const int slot = B.slot[1][c];
    for (int sg = threadIdx.x; sg < NSUB; sg += SUB_BS) {
        int ms[3] = {sg % NS, (sg / NS) % NS, sg / (NS * NS)};
        int hidx = 0;
        for (int j = DIM - 1; j >= 0; j--) hidx = hidx * HN + (ms[j] + 3);
        double q[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) q[v] = halo[v * HSZ + hidx];
        for (int k = 0; k < DIM; k++) {
            int sp = 0, mul = 1;
            for (int j = 0; j < DIM; j++) {
                if (j == k) continue;
                sp += ms[j] * mul;
                mul *= NS;
            }
            const double ck = dt * NS / P.h[k];
#pragma unroll
            for (int v = 0; v < NV; v++) {
                const double Fp = Fb[((k * (NS + 1) + ms[k] + 1) * NSF + sp) * NV + v];
                const double Fm = Fb[((k * (NS + 1) + ms[k]) * NSF + sp) * NV + v];
                q[v] -= ck * (Fp - Fm);
            }
        }
#pragma unroll
        for (int v = 0; v < NV; v++) {
            vn[v * NSUB + sg] = q[v];
            B.pool[1][((int64_t)slot * NV + v) * NSUB + sg] = q[v];
        }
        const bool pad = isfinite(q[0]) && isfinite(q[NV - 1]) && q[0] > 0.0 && pressure<DIM>(q, P.gamma) > 0.0;
        if (!pad) badc = 1;
        if (flagging) {
            // the criteria of Sec. 4.3 on the WENO3 result: PAD and the relaxed DMP
            bool bad = !pad;
#pragma unroll
            for (int v = 0; v < NV; v++) {
                if (!isfinite(q[v])) bad = true;
                const double delta = fmax(P.delta0, P.eps * (mb[1][v] - mb[0][v]));
                if (q[v] < mb[0][v] - delta || q[v] > mb[1][v] + delta) bad = true;
            }
            B.mflag[(int64_t)slot * NSUB + sg] = (uint8_t)bad;
            if (bad) atomicAdd(&B.counts[5], 1);
        }
    }
    // Flux correction data (Sec. 4.4: the face integral of the unlimited neighbour becomes
    // the sum of the integrals over the sub-faces): for each face, variable and tangential
    // node a of the DG basis, the integral of the subcell flux times phi_a over the face,
    // divided by the face weight w_a, from the per-point fluxes (3 Gauss-Legendre points per
    // sub-face and tangential axis; Pq[s*3+g][a] = (w3_g / Ns) phi_a((s + xi3_g) / Ns) / w_a).
    // For large cells the double sum over the face's (3 Ns)^2 = 3249 points is sum-factorised
    // (first along the first tangential axis for every node a0 and point row q1, then along the
    // second; 8.5x fewer operations), its intermediate in the slot's sub-face flux region, which
    // the FV update has read.  (At N = 3 the 441-point sums cost less than the extra barriers.)
    constexpr int QS = 3 * NS, FCT = 2 * DIM * NV * n * QS;
    if constexpr (BigCell<DIM, N>::on) {
        static_assert(FCT <= BigCell<DIM, N>::SUB_VN, "the stage must fit the sub-face flux region");
        __syncthreads();
        for (int it = threadIdx.x; it < FCT; it += SUB_BS) {
            const int a0 = it % n, q1 = (it / n) % QS, fv = it / (n * QS);   // fv = face * NV + v
            const double *fq = S.fpts + ((int64_t)ch * 2 * DIM * NV + fv) * QF + QS * q1;
            double acc = 0.0;
            for (int q0 = 0; q0 < QS; q0++) acc += T->Pq[q0][a0] * fq[q0];
            tmp[((int64_t)fv * n + a0) * QS + q1] = acc;
        }
        __syncthreads();
        for (int it = threadIdx.x; it < 2 * DIM * NV * NFN; it += SUB_BS) {
            const int fv = it / NFN, a = it % NFN, a0 = a % n, a1 = a / n;
            const double *x = tmp + ((int64_t)fv * n + a0) * QS;
            double acc = 0.0;
            for (int q1 = 0; q1 < QS; q1++) acc += T->Pq[q1][a1] * x[q1];
            B.sflux[(int64_t)slot * 2 * DIM * NV * NFN + it] = acc;
        }
    } else {
        for (int it = threadIdx.x; it < 2 * DIM * NV * NFN; it += SUB_BS) {
            const int face = it / (NV * NFN), v = (it / NFN) % NV, a = it % NFN;
            const int a0 = a % n, a1 = a / n;
            const double *fq = S.fpts + ((int64_t)ch * 2 * DIM + face) * NV * QF + v * QF;
            double acc = 0.0;
            for (int ms1 = 0; ms1 < (DIM == 3 ? NS : 1); ms1++)
                for (int ms0 = 0; ms0 < NS; ms0++)
                    for (int g1 = 0; g1 < (DIM == 3 ? 3 : 1); g1++)
                        for (int g0 = 0; g0 < 3; g0++) {
                            const int q0 = ms0 * 3 + g0, q1 = ms1 * 3 + g1;
                            double wgt = T->Pq[q0][a0];
                            if (DIM == 3) wgt *= T->Pq[q1][a1];
                            acc += wgt * fq[q0 + 3 * NS * q1];
                        }
            B.sflux[(int64_t)slot * 2 * DIM * NV * NFN + it] = acc;
        }
    }
    __syncthreads();
    store_cell_bounds<NV>(P, B, c, vn, NSUB, threadIdx.x, SUB_BS, red);
    // gather: u = R v (eq. (subcell.r)), tensor application
    tensor_apply<DIM, n, NS, NV, MAXNS>(&T->Rg[0][0], vn, ug, tmp, threadIdx.x, SUB_BS);
    for (int it = threadIdx.x; it < NV * NN; it += SUB_BS) {
        const int v = it / NN, a = it % NN;
        B.u[cur ^ 1][((int64_t)v * P.ncell + c) * NN + a] = ug[it];
    }
    if (threadIdx.x == 0 && badc) atomicAdd(nonphys, 1);
    __syncthreads();   // LDS reused by the next troubled cell
}

// S3: degree-2 local space-time predictor (eq. (pde.nc.dg2) on the subgrid, mesh size
// h/Ns, three sweeps) of every position of one troubled cell.  The 3^d spatial nodes of a
// position sit on consecutive lanes of one wave (64 / 3^d positions per wave), each lane
// holding its node's time pencil; a contraction along an axis gathers the three nodes of
// the line by lane permutation, so the waves work without LDS or workgroup barriers.
// Output: the face traces of every position, [pos][2d][v][3^(d-1) tangential x 3 time],
// in the working precision R (FP32 in the mixed form).
template <int DIM, typename R, bool XCH = false>
__device__ void sub_predictor(const Tables *__restrict__ T, const R *__restrict__ Y, R *__restrict__ tr,
                              int npos, int nsub, int nsf, double dt, const double *dth, double gamma_d,
                              R *xch = nullptr) {
    constexpr int NV = DIM + 2, NN = cpow(3, DIM), NF = cpow(3, DIM - 1), PPW = 64 / NN;
    constexpr int TRS = 2 * DIM * NV * NF * 3;
    constexpr int ST[3] = {1, 3, 9};
    constexpr bool F32 = sizeof(R) == 4;
    const R gamma = (R)gamma_d;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int slot = lane / NN, a = lane % NN;
    const int ia[3] = {a % 3, (a / 3) % 3, a / 9};
    // Along each axis a lane needs the values of the two other nodes of its line: it reads
    // them from the lanes of line nodes (ia + 1) % 3 and (ia + 2) % 3 (two lane permutations
    // per value; its own node's value it has).  Dk[k][j]: this lane's derivative-matrix row
    // in that order (own node first); src1/src2: the two source lanes.
    R Dk[DIM][3], ck[DIM];
    int src1[DIM], src2[DIM];
#pragma unroll
    for (int k = 0; k < DIM; k++) {
        ck[k] = (R)(dt * dth[k]);
        const int r = ia[k], n1 = (r + 1) % 3, n2 = (r + 2) % 3;
        Dk[k][0] = F32 ? (R)T->fD3[r][r] : (R)T->D3[r][r];
        Dk[k][1] = F32 ? (R)T->fD3[r][n1] : (R)T->D3[r][n1];
        Dk[k][2] = F32 ? (R)T->fD3[r][n2] : (R)T->D3[r][n2];
        src1[k] = lane + (n1 - r) * ST[k];
        src2[k] = lane + (n2 - r) * ST[k];
    }
    for (int base = wv * PPW; base < npos; base += nw * PPW) {
        const int pos = base + slot;
        const bool valid = slot < PPW && pos < npos;
        R u0[NV], q[NV][3];
        if (valid) {
#pragma unroll
            for (int v = 0; v < NV; v++) u0[v] = (R)Y[((int64_t)pos * NV + v) * NN + a];
        } else {
            // idle lanes carry a valid constant state
#pragma unroll
            for (int v = 0; v < NV; v++) u0[v] = (v == 0) ? R(1) : R(0);
            u0[NV - 1] = R(2.5);
        }
#pragma unroll
        for (int v = 0; v < NV; v++)
#pragma unroll
            for (int s = 0; s < 3; s++) q[v][s] = u0[v];
        // Three Picard sweeps.  The first starts from u^n at every time node, so its fluxes and
        // their derivatives are the same on the three time slices: slice 0 is computed and
        // copied (nt: time slices computed, uniform over the wave).
        for (int r = 0; r < 3; r++) {
            const int nt = r == 0 ? 1 : 3;
            R S[NV][3];
#pragma unroll
            for (int k = 0; k < DIM; k++) {
                R F[NV][3];
#pragma unroll
                for (int t = 0; t < 3; t++) {
                    if (t >= nt) break;
                    const R ir = recip(q[0][t]);
                    const R un = q[1 + k][t] * ir;
                    R ke = 0;
#pragma unroll
                    for (int j = 0; j < DIM; j++) ke += q[1 + j][t] * q[1 + j][t];
                    const R prt = (gamma - R(1)) * (q[NV - 1][t] - R(0.5) * ke * ir);
                    F[0][t] = q[1 + k][t];
#pragma unroll
                    for (int j = 0; j < DIM; j++) F[1 + j][t] = q[1 + j][t] * un + (j == k ? prt : R(0));
                    F[NV - 1][t] = un * (q[NV - 1][t] + prt);
                }
                // sum_b D[a_k][b] F(node b of the line): own node, then (ia + 1) % 3, (ia + 2) % 3
                // all lane permutations of the axis first (independent, in flight together); with an
                // exchange buffer (3D), through the wave's own LDS rows instead: each lane writes its
                // fluxes once and reads those of its two line neighbours
                R g1[NV][3], g2[NV][3], x[NV][3];
                if constexpr (XCH) {
                    R *xw = xch + (int64_t)wv * 64 * NV * 3;
#pragma unroll
                    for (int v = 0; v < NV; v++)
#pragma unroll
                        for (int t = 0; t < 3; t++)
                            if (t < nt) xw[lane * (NV * 3) + v * 3 + t] = F[v][t];
                    // lanes of one wave only: order the writes before the reads at wave scope
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                    for (int v = 0; v < NV; v++)
#pragma unroll
                        for (int t = 0; t < 3; t++)
                            if (t < nt) {
                                // (source lanes taken mod 64 as a lane permutation takes them: the
                                // idle lanes past the last position stay within the wave's rows)
                                g1[v][t] = xw[(src1[k] & 63) * (NV * 3) + v * 3 + t];
                                g2[v][t] = xw[(src2[k] & 63) * (NV * 3) + v * 3 + t];
                            }
                    // the next axis overwrites the rows only after every lane has read them
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                } else {
#pragma unroll
                    for (int t = 0; t < 3; t++) {
                        if (t >= nt) break;
#pragma unroll
                        for (int v = 0; v < NV; v++) {
                            g1[v][t] = __shfl(F[v][t], src1[k]);
                            g2[v][t] = __shfl(F[v][t], src2[k]);
                        }
                    }
                }
#pragma unroll
                for (int t = 0; t < 3; t++) {
                    if (t >= nt) break;
#pragma unroll
                    for (int v = 0; v < NV; v++) {
                        x[v][t] = Dk[k][0] * F[v][t] + Dk[k][1] * g1[v][t] + Dk[k][2] * g2[v][t];
                        S[v][t] = (k == 0) ? ck[k] * x[v][t] : S[v][t] + ck[k] * x[v][t];
                    }
                }
            }
            if (nt == 1) {
#pragma unroll
                for (int v = 0; v < NV; v++) S[v][1] = S[v][2] = S[v][0];
            }
            // time contraction K1^{-1} diag(w)
#pragma unroll
            for (int s = 0; s < 3; s++) {
                R acc[NV];
#pragma unroll
                for (int v = 0; v < NV; v++) acc[v] = 0;
#pragma unroll
                for (int t = 0; t < 3; t++) {
                    const R kst = F32 ? (R)T->fKw3[s][t] : (R)T->Kw3[s][t];
#pragma unroll
                    for (int v = 0; v < NV; v++) acc[v] += kst * S[v][t];
                }
#pragma unroll
                for (int v = 0; v < NV; v++) q[v][s] = u0[v] - acc[v];
            }
        }
        // face traces: the lane at the low end of a line writes the xi_k = 0 trace, the lane
        // at the high end the xi_k = 1 trace (with the exchange buffer, the pencils are written
        // once for the three axes)
        R *xq = xch + (int64_t)wv * 64 * NV * 3;
        if constexpr (XCH) {
#pragma unroll
            for (int v = 0; v < NV; v++)
#pragma unroll
                for (int s = 0; s < 3; s++) xq[lane * (NV * 3) + v * 3 + s] = q[v][s];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
#pragma unroll
        for (int k = 0; k < DIM; k++) {
            // the line's three nodes in this lane's order: own, (ia + 1) % 3, (ia + 2) % 3
            R qb[3][NV][3];
#pragma unroll
            for (int v = 0; v < NV; v++)
#pragma unroll
                for (int s = 0; s < 3; s++) {
                    qb[0][v][s] = q[v][s];
                    if constexpr (XCH) {
                        qb[1][v][s] = xq[(src1[k] & 63) * (NV * 3) + v * 3 + s];
                        qb[2][v][s] = xq[(src2[k] & 63) * (NV * 3) + v * 3 + s];
                    } else {
                        qb[1][v][s] = __shfl(q[v][s], src1[k]);
                        qb[2][v][s] = __shfl(q[v][s], src2[k]);
                    }
                }
            // a neighbour-layer position (pos >= nsub) only needs the trace on its face toward
            // the cell: the + face of the low layer, the - face of the high layer
            const int layer = pos >= nsub ? (pos - nsub) / nsf : -1;
            const bool needed = layer < 0 || ((layer >> 1) == k && (layer & 1) == (ia[k] == 0));
            if (valid && ia[k] != 1 && needed) {
                const int side = ia[k] == 2;
                const int r = ia[k], nb[3] = {r, (r + 1) % 3, (r + 2) % 3};
                R Bv[3];
#pragma unroll
                for (int b = 0; b < 3; b++)
                    Bv[b] = F32 ? (R)(side ? T->fR3[nb[b]] : T->fL3[nb[b]]) : (R)(side ? T->R3[nb[b]] : T->L3[nb[b]]);
                int ap = 0, mul = 1;
#pragma unroll
                for (int j = 0; j < DIM; j++) {
                    if (j == k) continue;
                    ap += ia[j] * mul;
                    mul *= 3;
                }
                R *o = tr + (int64_t)pos * TRS + (2 * k + side) * NV * NF * 3;
#pragma unroll
                for (int v = 0; v < NV; v++)
#pragma unroll
                    for (int s = 0; s < 3; s++) {
                        R acc = 0;
#pragma unroll
                        for (int b = 0; b < 3; b++) acc += Bv[b] * qb[b][v][s];
                        o[v * NF * 3 + ap + NF * s] = acc;
                    }
            }
        }
        if constexpr (XCH) {
            // the next positions' sweep overwrites the rows only after every lane has read them
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// Subcell ADER-WENO3 recompute (operator A of eq. (aderweno)) of every troubled cell:
// one persistent launch over the global troubled worklist.  A workgroup takes a
// troubled cell and runs its halo (eq. (ader.icbc)), WENO3 reconstruction, degree-2
// space-time predictor, sub-face fluxes, FV update and gather, using its own scratch
// slot (blockIdx.x), so the scratch scales with the grid, not with the worklist.
// R: working precision of the WENO3 reconstruction, the degree-2 predictor and the sub-face
// fluxes (FP32 in the mixed form); halo, FV update, gather and pool stay FP64.  flagging: also flag the WENO3
// result for the MOOD layer; REDO: the MOOD layer's recompute (only cells with a flag on or
// next to their sub-faces).
// Troubled cell w of one problem's worklist, on the workgroup's scratch slot sidx.
template <int DIM, int N, typename R, bool REDO>
__device__ __forceinline__ void subcell_cell(const Tables *__restrict__ T, const Prob &P, const Bufs &B, int cur,
                                             int w, int sidx, const SubScratch &S, int *nonphys, int flagging) {
    constexpr int NV = DIM + 2, NS = 2 * N + 1, NSUB = cpow(NS, DIM), NSF = cpow(NS, DIM - 1);
    constexpr int NPOS = NSUB + 2 * DIM * NSF, N3 = cpow(3, DIM);
    constexpr int TRS = 2 * DIM * NV * cpow(3, DIM - 1) * 3;
    const double dt = B.scal[0];
    double dth[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < DIM; k++) dth[k] = (double)NS / P.h[k];
    const R *Ys = reinterpret_cast<const R *>(S.Y) + (int64_t)sidx * NPOS * NV * N3;
    R *trs = reinterpret_cast<R *>(S.strace) + (int64_t)sidx * NPOS * TRS;
    // 2D: the halo and the source cells' coefficients live in LDS; 3D: halo in HBM scratch
    constexpr int HSZ = cpow(NS + 6, DIM), NNS = cpow(N + 1, DIM);
    __shared__ double halo_s[DIM == 2 ? NV * HSZ : 1];
    // 2D: the source cells' coefficients of the halo, later the predictor's line-exchange rows
    constexpr int XROWS = (SUB_BS / 64) * 64 * NV * 3 * (int)sizeof(R) / 8;   // doubles
    __shared__ double nbu_s[DIM == 2 ? (9 * NV * NNS > XROWS ? 9 * NV * NNS : XROWS) : 1];
    __shared__ double mb[2][NV];      // m_i, M_i of eq. (dmp) (MOOD flags)
    __shared__ int nslot[3][2];       // pool slots of troubled face neighbours (MOOD recompute)
    double *halo = (DIM == 2) ? halo_s : S.halo + (int64_t)sidx * NV * HSZ;
    double *nbu = (DIM == 2) ? nbu_s : nullptr;
    // LDS of the update's sub-face fluxes and of the gather's intermediate stage (large cells:
    // their global slot); in 3D the halo's sum-factorisation stages use it first
    constexpr int n = N + 1, NN = cpow(n, DIM), BIGN = NSUB > NN ? NSUB : NN;
    constexpr int FBB = DIM * (NS + 1) * NSF * NV * (int)sizeof(R), TMB = NV * BIGN * 8;
    constexpr int FBT = FBB > TMB ? FBB : TMB;
    __shared__ __align__(16) unsigned char fbt[BigCell<DIM, N>::on ? 16 : FBT];
    static_assert(DIM == 2 || BigCell<DIM, N>::on || (NV * NS * n * n + NV * NS * NS * n) * 8 <= FBT,
                  "the 3D halo's stage buffers must fit the sub-face flux LDS");
    static_assert(!BigCell<DIM, N>::on || NV * NS * n * n + NV * NS * NS * n <= BigCell<DIM, N>::SUB_VN,
                  "the 3D halo's stage buffers must fit the slot's sub-face flux region");
    double *hst = BigCell<DIM, N>::on ? S.big + (int64_t)sidx * BigCell<DIM, N>::SLOT : reinterpret_cast<double *>(fbt);
    {
        const int64_t c = B.tlist[w];
        if (!REDO && flagging) {
            // neighbourhood bounds of the cell, as in the detection
            if (threadIdx.x < 2 * NV) {
                const int mm = threadIdx.x / NV, v = threadIdx.x % NV;
                int ci[3];
                coords_of(P, c, ci);
                int ne[3] = {1, 1, 1};
                for (int j = 0; j < DIM; j++) ne[j] = P.nc[j] + 2;
                const int64_t next = ext_count(P);
                const double *src = (mm ? B.ext_max[0] : B.ext_min[0]) + (int64_t)v * next;
                double acc = mm ? -INFINITY : INFINITY;
                constexpr int NB = cpow(3, DIM);
                for (int o = 0; o < NB; o++) {
                    const int off[3] = {o % 3, (o / 3) % 3, o / 9};
                    int64_t e = 0;
                    for (int j = DIM - 1; j >= 0; j--) {
                        int x = ci[j] + off[j];
                        if (P.periodic[j]) x += (x == 0) ? P.nc[j] : ((x == P.nc[j] + 1) ? -P.nc[j] : 0);
                        e = e * ne[j] + x;
                    }
                    acc = mm ? fmax(acc, src[e]) : fmin(acc, src[e]);
                }
                mb[mm][v] = acc;
            }
        }
        if constexpr (REDO) {
            // neighbour slots, then: does a flagged subcell touch one of this cell's sub-faces?
            if (threadIdx.x < 2 * DIM) {
                const int k = threadIdx.x >> 1, side = threadIdx.x & 1;
                int ci[3];
                coords_of(P, c, ci);
                // the neighbour's coordinate along k, then its cell (selections, no dynamic index)
                const int cik = k == 0 ? ci[0] : (k == 1 ? ci[1] : ci[2]);
                const int nck = P.nc[k];
                int nbk = cik + (side ? 1 : -1);
                int sl = -1;
                if (nbk >= 0 && nbk < nck) sl = 0;
                else if (P.periodic[k]) { nbk = (nbk + nck) % nck; sl = 0; }
                if (sl == 0) {
                    int nb[3];
#pragma unroll
                    for (int j = 0; j < 3; j++) nb[j] = (j == k) ? nbk : ci[j];
                    const int64_t cn = cell_of(P, nb);
                    sl = B.beta[1][cn] ? B.slot[1][cn] : -1;
                }
                nslot[k][side] = sl;
            }
            __syncthreads();
            const int own = B.slot[1][c];
            int any = 0;
            for (int i = threadIdx.x; i < NSUB + 2 * DIM * NSF; i += SUB_BS) {
                if (i < NSUB) {
                    any |= B.mflag[(int64_t)own * NSUB + i];
                } else {
                    const int r = i - NSUB, face = r / NSF, sp = r % NSF;
                    const int k = face >> 1, side = face & 1;
                    const int sl = nslot[k][side];
                    if (sl >= 0) {
                        // the neighbour's subcell layer facing this cell
                        const int mp0 = sp % NS, mp1 = sp / NS;
                        int idx = 0;
#pragma unroll
                        for (int j = DIM - 1; j >= 0; j--)
                            idx = idx * NS + ((j == k) ? (side ? 0 : NS - 1) : ((j < k ? j : j - 1) == 0 ? mp0 : mp1));
                        any |= B.mflag[(int64_t)sl * NSUB + idx];
                    }
                }
            }
            if (!__syncthreads_or(any)) return;
            if (threadIdx.x == 0) atomicAdd(&B.counts[6], 1);
        }
        if constexpr (DIM == 3) sub_halo_cell3<N>(T, P, B, cur, w, halo, hst);
        else sub_halo_cell<DIM, N>(T, P, B, cur, w, halo, nbu);
        __syncthreads();
        sub_recon_cell<DIM, N, R>(T, S.Y, sidx, halo, trs);
        __syncthreads();
        // the line exchange of the predictor through LDS rows (free in this phase): in 2D the halo's
        // staging LDS, in 3D the flux LDS where the rows fit (not for large cells)
        constexpr bool XCH = DIM == 2 || (!BigCell<DIM, N>::on && (SUB_BS / 64) * 64 * NV * 3 * (int)sizeof(R) <= FBT);
        R *xrows = DIM == 2 ? reinterpret_cast<R *>(nbu_s) : reinterpret_cast<R *>(fbt);
        sub_predictor<DIM, R, XCH>(T, Ys, trs, NPOS, NSUB, NSF, dt, dth, P.gamma, xrows);
        __syncthreads();
        sub_update_cell<DIM, N, R, REDO>(T, P, B, cur, w, sidx, S, nonphys, halo, REDO ? 0 : flagging, mb, nslot, fbt);
    }
}

template <int DIM, int N, typename R, bool REDO>
__global__ __launch_bounds__(SUB_BS, (SubShape<DIM, N, R>::WPS)) void k_subcell(const Tables *__restrict__ T, Prob P, Bufs B, int cur, int64_t cap,
                                                 int *nonphys, int flagging) {
    const int count = (int)(B.counts[0] < cap ? B.counts[0] : cap);
    const SubScratch S{B.Y, B.strace, B.halo, B.fpts, B.big};
    for (int w = blockIdx.x; w < count; w += gridDim.x)
        subcell_cell<DIM, N, R, REDO>(T, P, B, cur, w, blockIdx.x, S, nonphys, flagging);
}

// Flux correction of unlimited cells next to troubled cells (Sec. 4.4): the DG face
// flux of each face shared with a troubled cell is replaced by the subcell fluxes of
// that face integrated against the basis (the troubled cell's kernel stores those
// integrals per tangential node).
// DEV: the cell's DG face fluxes are held as G - F(c) (the deviation form); the full flux that
// the subcell flux replaces is that plus F(c) times the time weights' sum, formed in FP64.
template <int DIM, int N, typename R, bool DEV = false>
__device__ __forceinline__ void fluxcorr_cell(const Tables *__restrict__ T, const Prob &P, const Bufs &B, int cur,
                                              int wb) {
    const R *gbar = reinterpret_cast<const R *>(B.gbar);
    constexpr int NS_ = 2 * N + 1, NSUB_ = cpow(NS_, DIM), NN_ = cpow(N + 1, DIM), NV_ = DIM + 2;
    constexpr int TMP_ = (DIM == 2) ? NS_ * (N + 1) : NS_ * NS_ * (N + 1);
    __shared__ double us[NV_ * NN_];
    __shared__ double red[2 * NV_ * 2];
    double *vs, *tmp;
    if constexpr (BigCell<DIM, N>::on) {
        vs = B.big + (int64_t)blockIdx.x * BigCell<DIM, N>::SLOT;
        tmp = vs + NV_ * NSUB_;
    } else {
        __shared__ double vs_[NV_ * NSUB_];
        __shared__ double tmp_[NV_ * TMP_];
        vs = vs_;
        tmp = tmp_;
    }
    constexpr int n = N + 1, NV = DIM + 2, NN = cpow(n, DIM), NFN = cpow(n, DIM - 1);
    constexpr int NS = 2 * N + 1;
    {
    const int64_t c = B.clist[wb];
    int ci[3];
    coords_of(P, c, ci);
    const double dt = B.scal[0];
    int64_t nbc[3][2];
    int nslot[3][2];
    for (int k = 0; k < DIM; k++)
        for (int side = 0; side < 2; side++) {
            int nb[3] = {ci[0], ci[1], ci[2]};
            nb[k] += side ? 1 : -1;
            nbc[k][side] = -1;
            nslot[k][side] = -1;
            if (nb[k] < 0 || nb[k] >= P.nc[k]) {
                if (!P.periodic[k]) continue;
                nb[k] = (nb[k] + P.nc[k]) % P.nc[k];
            }
            const int64_t cn = cell_of(P, nb);
            if (B.beta[1][cn] && B.slot[1][cn] >= 0) {
                nbc[k][side] = cn;
                nslot[k][side] = B.slot[1][cn];
            }
        }
    // DEV: F_k(c) of the cell's reference state for every axis, and the time weights' sum
    __shared__ double fcs[DEV ? 3 * NV : 1];
    double wsum = 0.0;
    if constexpr (DEV) {
        for (int ss = 0; ss < n; ss++) wsum += (double)T->fw[ss];
        if (threadIdx.x < DIM) {
            double c64[NV], cq[NV], F[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) c64[v] = B.u[cur][((int64_t)v * P.ncell + c) * NN];
            const DevRef<DIM, float> r = make_devref<DIM, float>(c64, P.gamma);
#pragma unroll
            for (int v = 0; v < NV; v++) cq[v] = (double)r.q[v];
            euler_flux<DIM, double>((int)threadIdx.x, cq, F, P.gamma);
#pragma unroll
            for (int v = 0; v < NV; v++) fcs[threadIdx.x * NV + v] = F[v];
        }
        __syncthreads();
    }
    for (int it = threadIdx.x; it < NV * NN; it += 128) {
        const int v = it / NN, a = it % NN;
        int m[3] = {a % n, (a / n) % n, a / (n * n)};
        double val = B.u[cur ^ 1][((int64_t)v * P.ncell + c) * NN + a];
#pragma unroll
        for (int k = 0; k < DIM; k++) {
            int ap = 0, mul = 1;
#pragma unroll
            for (int j = 0; j < DIM; j++) {
                if (j == k) continue;
                ap += m[j] * mul;
                mul *= n;
            }
            const int ak = m[k];
            const double ck = dt / P.h[k] / T->w[ak];
            for (int side = 0; side < 2; side++) {
                if (nbc[k][side] < 0) continue;
                const int slot = nslot[k][side];
                const double Fsub = B.sflux[(((int64_t)slot * 2 * DIM + 2 * k + (1 - side)) * NV + v) * NFN + ap];
                double Gdg = (double)gbar[((c * 2 * DIM + 2 * k + side) * NV + v) * NFN + ap];
                if constexpr (DEV) Gdg += wsum * fcs[k * NV + v];
                val += side ? ck * T->R[ak] * (Gdg - Fsub) : ck * T->L[ak] * (Fsub - Gdg);
            }
        }
        B.u[cur ^ 1][((int64_t)v * P.ncell + c) * NN + a] = val;
        us[it] = val;
    }
    __syncthreads();
    // the corrected state's subcell min / max are this cell's next old-time bounds
    tensor_apply<DIM, NS, n, NV, MAXN>(&T->P[0][0], us, vs, tmp, threadIdx.x, 128);
    store_cell_bounds<NV>(P, B, c, vs, NSUB_, threadIdx.x, 128, red);
    __syncthreads();   // LDS reused by the next corrected cell
    }
}

template <int DIM, int N, typename R, bool DEV = false>
__global__ __launch_bounds__(128) void k_fluxcorr(const Tables *__restrict__ T, Prob P, Bufs B, int cur, int count,
                                                  int advance) {
    // the step's last kernel also advances t (no other workgroup reads t here) and ends a
    // one-step debug poison of the candidate
    if (advance && blockIdx.x == 0 && threadIdx.x == 0) {
        B.scal[1] += B.scal[0];
        B.scal[4] = 0.0;
    }
    if (count < 0) count = B.counts[1];   // device-driven
    for (int wb = blockIdx.x; wb < count; wb += gridDim.x) fluxcorr_cell<DIM, N, R, DEV>(T, P, B, cur, wb);
}

// ------------------------------------------------------------------ time step
template <int DIM, int N>
__device__ __forceinline__ void lambda_block(const Prob &P, const double *__restrict__ u, double *part, int64_t bid,
                                             int64_t nblk, const uint8_t *__restrict__ mask) {
    constexpr int n = N + 1, NV = DIM + 2, NN = cpow(n, DIM);
    __shared__ double red[256];
    double lam = 0.0;
    const int64_t total = P.ncell * NN;
    for (int64_t i = (int64_t)bid * 256 + threadIdx.x; i < total; i += (int64_t)nblk * 256) {
        if (mask && mask[i / NN]) continue;   // solid cells take no part in the time step
        double q[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) q[v] = u[(int64_t)v * total + i];
        const double cs = sqrt(P.gamma * pressure<DIM>(q, P.gamma) / q[0]);
#pragma unroll
        for (int k = 0; k < DIM; k++) lam = fmax(lam, fabs(q[1 + k] / q[0]) + cs);
    }
    red[threadIdx.x] = lam;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[bid] = red[0];
}
template <int DIM, int N>
__global__ __launch_bounds__(256) void k_lambda(Prob P, const double *__restrict__ u, double *part,
                                                const uint8_t *__restrict__ mask) {
    lambda_block<DIM, N>(P, u, part, blockIdx.x, gridDim.x, mask);
}

__device__ __forceinline__ void dt_final_block(const double *part, int nparts, double *scal, double factor) {
    __shared__ double red[256];
    double lam = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) lam = fmax(lam, part[i]);
    red[threadIdx.x] = lam;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        scal[2] = red[0];
        scal[0] = factor / red[0];
    }
}
static __global__ void k_dt_final(const double *part, int nparts, double *scal, double factor) {
    dt_final_block(part, nparts, scal, factor);
}

static __global__ void k_set_scalar(double *scal, int idx, double val) { scal[idx] = val; }
// t += dt; a debug poison of the candidate lasts one step
static __global__ void k_advance_time(double *scal) {
    scal[1] += scal[0];
    scal[4] = 0.0;
}

// ------------------------------------------------------------- batched launches
// A workgroup of a batched launch looks up its problem and its block in the tile table
// (built on the host from every problem's own grid for that stage) and runs the
// per-problem block body with that problem's arguments; the result is bitwise the
// per-problem launch's.
template <int DIM, int N>
__global__ __launch_bounds__(256) void kb_lambda(const BatchEntry *__restrict__ E, const BTile *__restrict__ tl) {
    const BTile t = tl[blockIdx.x];
    const BatchEntry &e = E[t.p];
    lambda_block<DIM, N>(e.P, e.B.u[e.cur], e.B.lam_part, t.b, t.n, e.B.mask);
}

static __global__ __launch_bounds__(256) void kb_dt_final(const BatchEntry *__restrict__ E) {
    const BatchEntry &e = E[blockIdx.x];
    dt_final_block(e.B.lam_part, e.lam_nb, e.B.scal, e.factor);
}

template <int DIM, int N>
__global__ __launch_bounds__(128) void kb_cell_bounds(const Tables *__restrict__ T, const BatchEntry *__restrict__ E,
                                                      const BTile *__restrict__ tl) {
    const BTile t = tl[blockIdx.x];
    const BatchEntry &e = E[t.p];
    cell_bounds_block<DIM, N>(T, e.P, e.B, e.cur, e.ring, t.b);
}

template <typename R> __device__ __forceinline__ const PredArgs<R> &pred_args(const BatchEntry &e);
template <> __device__ __forceinline__ const PredArgs<float> &pred_args<float>(const BatchEntry &e) { return e.pf; }
template <> __device__ __forceinline__ const PredArgs<double> &pred_args<double>(const BatchEntry &e) { return e.pd; }

template <int DIM, int N, typename R, bool DEV = false>
__global__ __launch_bounds__((PredShape<DIM, N, R>::BS), (Tune<DIM, N, sizeof(R) == 4>::pred_wps)) void kb_predictor(
    const BatchEntry *__restrict__ E, const BTile *__restrict__ tl) {
    const BTile t = tl[blockIdx.x];
    const BatchEntry &e = E[t.p];
    const PredArgs<R> &A = pred_args<R>(e);
    pred_cells<DIM, N, true, R, DEV>(A, e.P.gamma, A.ncell, t.b, A.ncell);
}

template <int DIM, int N, typename R, bool DEV = false>
__global__ __launch_bounds__((FaceShape<DIM, N>::BS)) void kb_face(const Tables *__restrict__ T,
                                                                  const BatchEntry *__restrict__ E,
                                                                  const BTile *__restrict__ tl) {
    const BTile t = tl[blockIdx.x];
    const BatchEntry &e = E[t.p];
    face_block<DIM, N, R, DEV>(T, e.P, reinterpret_cast<const R *>(e.B.trace), reinterpret_cast<R *>(e.B.gbar),
                               e.B.scal, e.kb1, e.kb2, t.b, e.B.mask, e.B.u[e.cur]);
}

// The problem's Prob and Bufs staged in LDS once per workgroup: the corrector's body reads
// them many times, and from LDS they cost neither vector registers nor memory latency.
template <int BS>
__device__ __forceinline__ void stage_entry(const BatchEntry &e, Prob *sP, Bufs *sB) {
    static_assert(sizeof(Prob) % 4 == 0 && sizeof(Bufs) % 4 == 0, "word copies");
    const int *srcP = reinterpret_cast<const int *>(&e.P), *srcB = reinterpret_cast<const int *>(&e.B);
    int *dP = reinterpret_cast<int *>(sP), *dB = reinterpret_cast<int *>(sB);
    for (int i = threadIdx.x; i < (int)(sizeof(Prob) / 4); i += BS) dP[i] = srcP[i];
    for (int i = threadIdx.x; i < (int)(sizeof(Bufs) / 4); i += BS) dB[i] = srcB[i];
    __syncthreads();
}

template <int DIM, int N, typename R>
__global__ __launch_bounds__((CorrShape<DIM, N, R>::BS), (CorrShape<DIM, N, R>::WPS)) void kb_corrector_detect(const Tables *__restrict__ T,
                                                                          const BatchEntry *__restrict__ E,
                                                                          const BTile *__restrict__ tl) {
    __shared__ Prob sP;
    __shared__ Bufs sB;
    const BTile t = tl[blockIdx.x];
    const BatchEntry &e = E[t.p];
    const int cur = e.cur, limiter = e.limiter;
    stage_entry<CorrShape<DIM, N, R>::BS>(e, &sP, &sB);
    corrector_detect_block<DIM, N, R>(T, sP, sB, cur, limiter, t.b);
}

static __global__ __launch_bounds__(CBS) void kb_compact_count(const BatchEntry *__restrict__ E, const BTile *__restrict__ tl) {
    const BTile t = tl[blockIdx.x];
    const BatchEntry &e = E[t.p];
    compact_count_block(e.P, e.B, e.cap, t.b, t.n);
}

static __global__ __launch_bounds__(CBS) void kb_compact_scatter(const BatchEntry *__restrict__ E,
                                                          const BTile *__restrict__ tl) {
    const BTile t = tl[blockIdx.x];
    const BatchEntry &e = E[t.p];
    compact_scatter_block(e.P, e.B, e.cap, t.b, t.n);
}

// The global worklists of a class: exclusive offsets of every problem's troubled cells
// (its count clamped to its pool) and of its corrected neighbours, np + 1 entries each.
// One workgroup of 1024 threads, chunks of 1024 problems with a carried total.
static __global__ __launch_bounds__(1024) void kb_offsets(const BatchEntry *__restrict__ E, int np, int *off_t, int *off_c) {
    __shared__ int wsum[2][16];
    __shared__ int carry[2];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry[0] = carry[1] = 0;
    __syncthreads();
    for (int base = 0; base < np; base += 1024) {
        const int i = base + threadIdx.x;
        int vt = 0, vc = 0;
        if (i < np) {
            const BatchEntry &e = E[i];
            const int64_t ct = e.B.counts[0];
            vt = (int)(ct < e.cap ? ct : e.cap);
            vc = e.B.counts[1];
        }
        int xt = vt, xc = vc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int yt = __shfl_up(xt, o), yc = __shfl_up(xc, o);
            if (lane >= o) { xt += yt; xc += yc; }
        }
        if (lane == 63) { wsum[0][wv] = xt; wsum[1][wv] = xc; }
        __syncthreads();
        int pt = carry[0], pc = carry[1];
        for (int w = 0; w < wv; w++) { pt += wsum[0][w]; pc += wsum[1][w]; }
        if (i < np) { off_t[i] = pt + xt - vt; off_c[i] = pc + xc - vc; }
        __syncthreads();
        if (threadIdx.x == 1023) { carry[0] = pt + xt; carry[1] = pc + xc; }
        __syncthreads();
    }
    if (threadIdx.x == 0) { off_t[np] = carry[0]; off_c[np] = carry[1]; }
}

// problem p with off[p] <= g < off[p + 1] (off non-decreasing, off[0] = 0)
__device__ __forceinline__ int owner_of(const int *__restrict__ off, int np, int g) {
    int lo = 0, hi = np;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Subcell recompute over one global troubled worklist: the troubled cells of every problem
// of the class, in problem order, shared out over the persistent grid.
template <int DIM, int N, typename R, bool REDO>
__global__ __launch_bounds__(SUB_BS, (SubShape<DIM, N, R>::WPS)) void kb_subcell(const Tables *__restrict__ T, const BatchEntry *__restrict__ E,
                                                        int np, const int *__restrict__ off, SubScratch S, int flagging) {
    const int total = off[np];
    for (int g = blockIdx.x; g < total; g += gridDim.x) {
        const int p = owner_of(off, np, g);
        const BatchEntry &e = E[p];
        subcell_cell<DIM, N, R, REDO>(T, e.P, e.B, e.cur, g - off[p], blockIdx.x, S, e.B.counts + 2, flagging);
    }
}

template <int DIM, int N, typename R, bool DEV = false>
__global__ __launch_bounds__(128) void kb_fluxcorr(const Tables *__restrict__ T, const BatchEntry *__restrict__ E,
                                                   int np, const int *__restrict__ off) {
    const int total = off[np];
    for (int g = blockIdx.x; g < total; g += gridDim.x) {
        const int p = owner_of(off, np, g);
        const BatchEntry &e = E[p];
        fluxcorr_cell<DIM, N, R, DEV>(T, e.P, e.B, e.cur, g - off[p]);
    }
}

// t += dt for every problem of the class; a debug poison lasts one step
static __global__ void kb_advance(const BatchEntry *__restrict__ E, int np) {
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
        double *scal = E[p].B.scal;
        scal[1] += scal[0];
        scal[4] = 0.0;
    }
}

// ------------------------------------------------------------------ launchers
template <int DIM, int N>
struct Launch {
    static constexpr int n = N + 1, NV = DIM + 2, NN = cpow(n, DIM), NS = 2 * N + 1;
    static constexpr int NPOS = cpow(NS, DIM) + 2 * DIM * cpow(NS, DIM - 1);

    template <typename R, bool DEV = false>
    static void predictor_t(const StepCtx &C) {
        using S = PredShape<DIM, N, R>;
        PredArgs<R> A;
        fill_pred_args<R>(C, A);
        const int64_t grid = (C.P.ncell + S::CPB - 1) / S::CPB;
        hipLaunchKernelGGL((k_predictor<DIM, N, true, R, DEV>), dim3((unsigned)grid), dim3(S::BS), 0, C.stream, A,
                           C.P.gamma);
    }
    template <typename R>
    static void fill_pred_args(const StepCtx &C, PredArgs<R> &A) {
        A.in = C.B.u[C.cur];
        A.in_cstride = NN;
        A.in_vstride = (int64_t)C.P.ncell * NN;
        A.trace = reinterpret_cast<R *>(C.B.trace);
        A.vol_out = C.B.u[C.cur ^ 1];
        A.ncell = C.P.ncell;
        A.cell0 = 0;
        A.iters = C.picard_iters;
        for (int k = 0; k < 3; k++) A.dth[k] = k < DIM ? 1.0 / C.P.h[k] : 0.0;
        A.dt = C.B.scal;
        if constexpr (std::is_same<R, double>::value) {
            A.D = &C.tab->D[0][0];
            A.Kw = &C.tab->Kw[0][0];
            A.Lb = C.tab->L;
            A.Rb = C.tab->R;
            A.w = C.tab->w;
            A.Dvol = &C.tab->Dvol[0][0];
            A.DE = &C.tab->DE[0][0];
            A.DO = &C.tab->DO[0][0];
        } else {
            A.D = &C.tab->fD[0][0];
            A.Kw = &C.tab->fKw[0][0];
            A.Lb = C.tab->fL;
            A.Rb = C.tab->fR;
            A.w = C.tab->fw;
            A.Dvol = &C.tab->fDvol[0][0];
            A.DE = &C.tab->fDE[0][0];
            A.DO = &C.tab->fDO[0][0];
        }
        A.dcount = nullptr;
        A.dcap = 0;
        A.dmult = 1;
    }
    static void pred_args(const StepCtx &C, PredArgs<float> *pf, PredArgs<double> *pd) {
        fill_pred_args<float>(C, *pf);
        fill_pred_args<double>(C, *pd);
    }
    static void predictor(const StepCtx &C) {
        if (C.precision == ADG_MIXED_DEV) predictor_t<float, true>(C);
        else if (C.precision == ADG_MIXED) predictor_t<float>(C);
        else predictor_t<double>(C);
    }
    template <typename R, bool DEV = false>
    static void faces_t(const StepCtx &C) {
        using FS = FaceShape<DIM, N>;
        int64_t start[4] = {0, 0, 0, 0};   // first block of each axis
        for (int k = 0; k < DIM; k++) {
            int64_t nlines = 1;
            for (int j = 0; j < DIM; j++)
                if (j != k) nlines *= C.P.nc[j];
            const int nfk = C.P.periodic[k] ? C.P.nc[k] : C.P.nc[k] + 1;
            const int64_t nfaces = nlines * nfk;
            start[k + 1] = start[k] + (nfaces + FS::FPB - 1) / FS::FPB;
        }
        const int64_t kb2 = DIM == 3 ? start[2] : start[DIM];
        hipLaunchKernelGGL((k_face<DIM, N, R, DEV>), dim3((unsigned)start[DIM]), dim3(FS::BS), 0, C.stream, C.tab, C.P,
                           reinterpret_cast<const R *>(C.B.trace), reinterpret_cast<R *>(C.B.gbar), C.B.scal,
                           start[1], kb2, C.B.mask, (const double *)C.B.u[C.cur]);
    }
    static void faces(const StepCtx &C) {
        if (C.precision == ADG_MIXED_DEV) faces_t<float, true>(C);
        else if (C.precision == ADG_MIXED) faces_t<float>(C);
        else faces_t<double>(C);
    }
    static void corrector_detect(const StepCtx &C) {
        using CF = CorrShape<DIM, N, float>;
        using CD = CorrShape<DIM, N, double>;
        // large cells: a grid of at most BIG_WG workgroups (one global slot each) loops over the cells
        auto grid = [&](int64_t cpb) {
            const int64_t nb = (C.P.ncell + cpb - 1) / cpb;
            return (unsigned)(BigCell<DIM, N>::on ? std::min<int64_t>(nb, BIG_WG) : nb);
        };
        if (C.precision != ADG_FP64)
            hipLaunchKernelGGL((k_corrector_detect<DIM, N, float>), dim3(grid(CF::CPB)), dim3(CF::BS), 0, C.stream,
                               C.tab, C.P, C.B, C.cur, C.limiter);
        else
            hipLaunchKernelGGL((k_corrector_detect<DIM, N, double>), dim3(grid(CD::CPB)), dim3(CD::BS), 0, C.stream,
                               C.tab, C.P, C.B, C.cur, C.limiter);
    }
    static void bounds(const StepCtx &C) {
        int64_t next = 1;
        for (int j = 0; j < DIM; j++) next *= C.P.nc[j] + 2;
        const int64_t nblk = C.ring_only ? C.nring : next;
        const int64_t grid = BigCell<DIM, N>::on ? std::min<int64_t>(nblk, BIG_WG) : nblk;
        if (nblk > 0)
            hipLaunchKernelGGL((k_cell_bounds<DIM, N>), dim3((unsigned)grid), dim3(128), 0, C.stream, C.tab, C.P, C.B,
                               C.cur, C.ring_only ? C.B.ring : (const int64_t *)nullptr, nblk);
    }
    template <typename R>
    static void subcell_t(const StepCtx &C, int redo) {
        const dim3 g((unsigned)C.subcell_grid), b(SUB_BS);
        if (redo)
            hipLaunchKernelGGL((k_subcell<DIM, N, R, true>), g, b, 0, C.stream, C.tab, C.P, C.B, C.cur, C.capacity,
                               C.B.counts + 2, 0);
        else
            hipLaunchKernelGGL((k_subcell<DIM, N, R, false>), g, b, 0, C.stream, C.tab, C.P, C.B, C.cur, C.capacity,
                               C.B.counts + 2, C.mood);
    }
    // redo = 0: the subcell scheme (flagging its result when the MOOD layer is on); 1: the
    // MOOD layer's recompute
    static void subcell(const StepCtx &C, int redo) {
        if (C.precision != ADG_FP64) subcell_t<float>(C, redo);
        else subcell_t<double>(C, redo);
    }
    static void fluxcorr(const StepCtx &C, int count, int advance) {
        static_assert(BIG_WG >= 512, "the flux correction's grid must fit the large-cell slots");
        const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(count >= 0 ? count : C.P.ncell, 512));
        if (C.precision == ADG_MIXED_DEV)
            hipLaunchKernelGGL((k_fluxcorr<DIM, N, float, true>), dim3(g), dim3(128), 0, C.stream, C.tab, C.P, C.B,
                               C.cur, count, advance);
        else if (C.precision == ADG_MIXED)
            hipLaunchKernelGGL((k_fluxcorr<DIM, N, float>), dim3(g), dim3(128), 0, C.stream, C.tab, C.P, C.B, C.cur,
                               count, advance);
        else
            hipLaunchKernelGGL((k_fluxcorr<DIM, N, double>), dim3(g), dim3(128), 0, C.stream, C.tab, C.P, C.B, C.cur,
                               count, advance);
    }
    // blocks of one problem's launch of a stage (batch tile tables); kb1/kb2: face kernel axes
    static int64_t blocks(int stage, const Prob &P, int precision, int64_t *kb1, int64_t *kb2) {
        switch (stage) {
        case BSTAGE_PREDICTOR: {
            const int64_t cpb = precision != ADG_FP64 ? PredShape<DIM, N, float>::CPB : PredShape<DIM, N, double>::CPB;
            return (P.ncell + cpb - 1) / cpb;
        }
        case BSTAGE_FACE: {
            using FS = FaceShape<DIM, N>;
            int64_t start[4] = {0, 0, 0, 0};
            for (int k = 0; k < DIM; k++) {
                int64_t nlines = 1;
                for (int j = 0; j < DIM; j++)
                    if (j != k) nlines *= P.nc[j];
                const int nfk = P.periodic[k] ? P.nc[k] : P.nc[k] + 1;
                start[k + 1] = start[k] + (nlines * nfk + FS::FPB - 1) / FS::FPB;
            }
            *kb1 = start[1];
            *kb2 = DIM == 3 ? start[2] : start[DIM];
            return start[DIM];
        }
        case BSTAGE_CORRECTOR: {
            const int64_t cpb = precision != ADG_FP64 ? CorrShape<DIM, N, float>::CPB : CorrShape<DIM, N, double>::CPB;
            return (P.ncell + cpb - 1) / cpb;
        }
        case BSTAGE_COMPACT: return (P.ncell + CBS - 1) / CBS;
        default: return 0;
        }
    }
    template <typename R, bool DEV = false>
    static void batched_t(int stage, const BatchLaunch &L) {
        // large cells are stepped problem by problem (a batch refuses them)
        if constexpr (!BigCell<DIM, N>::on) batched_body<R, DEV>(stage, L);
    }
    template <typename R, bool DEV>
    static void batched_body(int stage, const BatchLaunch &L) {
        const hipStream_t st = L.stream;
        switch (stage) {
        case BSTAGE_DT:
            if (L.n_lambda) hipLaunchKernelGGL((kb_lambda<DIM, N>), dim3(L.n_lambda), dim3(256), 0, st, L.E, L.t_lambda);
            hipLaunchKernelGGL(kb_dt_final, dim3(L.np), dim3(256), 0, st, L.E);
            break;
        case BSTAGE_BOUNDS:
            if (L.n_bounds)
                hipLaunchKernelGGL((kb_cell_bounds<DIM, N>), dim3(L.n_bounds), dim3(128), 0, st, L.T, L.E, L.t_bounds);
            break;
        case BSTAGE_PREDICTOR:
            hipLaunchKernelGGL((kb_predictor<DIM, N, R, DEV>), dim3(L.n_pred), dim3(PredShape<DIM, N, R>::BS), 0, st, L.E,
                               L.t_pred);
            break;
        case BSTAGE_FACE:
            hipLaunchKernelGGL((kb_face<DIM, N, R, DEV>), dim3(L.n_face), dim3(FaceShape<DIM, N>::BS), 0, st, L.T, L.E,
                               L.t_face);
            break;
        case BSTAGE_CORRECTOR:
            hipLaunchKernelGGL((kb_corrector_detect<DIM, N, R>), dim3(L.n_corr), dim3(CorrShape<DIM, N, R>::BS), 0, st,
                               L.T, L.E, L.t_corr);
            break;
        case BSTAGE_COMPACT:
            hipLaunchKernelGGL(kb_compact_count, dim3(L.n_compact), dim3(CBS), 0, st, L.E, L.t_compact);
            hipLaunchKernelGGL(kb_compact_scatter, dim3(L.n_compact), dim3(CBS), 0, st, L.E, L.t_compact);
            hipLaunchKernelGGL(kb_offsets, dim3(1), dim3(1024), 0, st, L.E, L.np, L.off_t, L.off_c);
            break;
        case BSTAGE_SUBCELL:
            hipLaunchKernelGGL((kb_subcell<DIM, N, R, false>), dim3(L.sub_grid), dim3(SUB_BS), 0, st, L.T, L.E, L.np,
                               (const int *)L.off_t, L.S, L.mood);
            if (L.mood)
                hipLaunchKernelGGL((kb_subcell<DIM, N, R, true>), dim3(L.sub_grid), dim3(SUB_BS), 0, st, L.T, L.E, L.np,
                                   (const int *)L.off_t, L.S, 0);
            break;
        case BSTAGE_FLUXCORR:
            hipLaunchKernelGGL((kb_fluxcorr<DIM, N, R, DEV>), dim3(L.fc_grid), dim3(128), 0, st, L.T, L.E, L.np,
                               (const int *)L.off_c);
            break;
        case BSTAGE_ADVANCE:
            hipLaunchKernelGGL(kb_advance, dim3(1), dim3(256), 0, st, L.E, L.np);
            break;
        default: break;
        }
    }
    static void batched(int stage, const BatchLaunch &L) {
        if (L.precision == ADG_MIXED_DEV) batched_t<float, true>(stage, L);
        else if (L.precision == ADG_MIXED) batched_t<float>(stage, L);
        else batched_t<double>(stage, L);
    }
    static void lambda(const StepCtx &C, const double *u, double factor) {
        const int64_t total = C.P.ncell * NN;
        int nb = (int)((total + 255) / 256);
        if (nb > C.lam_blocks) nb = C.lam_blocks;
        hipLaunchKernelGGL((k_lambda<DIM, N>), dim3(nb), dim3(256), 0, C.stream, C.P, u, C.B.lam_part, C.B.mask);
        hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(256), 0, C.stream, C.B.lam_part, nb, C.B.scal, factor);
    }
};

struct Ops {
    void (*predictor)(const StepCtx &);
    void (*faces)(const StepCtx &);
    void (*corrector_detect)(const StepCtx &);
    void (*bounds)(const StepCtx &);
    void (*subcell)(const StepCtx &, int);
    void (*fluxcorr)(const StepCtx &, int, int);
    void (*lambda)(const StepCtx &, const double *, double);
    int64_t (*blocks)(int, const Prob &, int, int64_t *, int64_t *);
    void (*batched)(int, const BatchLaunch &);
    void (*pred_args)(const StepCtx &, PredArgs<float> *, PredArgs<double> *);
    int npos;
    int sub_wgs[2];   // workgroups of the persistent subcell launch that fill the chip (FP64, mixed form)
    int64_t big_slot; // doubles per global scratch slot of large cells (0: the class works in LDS)
};

// the (d, N) instantiations, one group per translation unit (null outside the group)
const Ops *ops_2d_a(int N);   // d = 2, N = 1..3
const Ops *ops_2d_b(int N);   // d = 2, N = 4..5
const Ops *ops_2d_c(int N);   // d = 2, N = 6..7
const Ops *ops_2d_d(int N);   // d = 2, N = 8..9
const Ops *ops_3d(int N);     // d = 3, N = 1..3
const Ops *ops_3d_9(int N);   // d = 3, N = 9 (large cells)

template <int DIM, int N>
static Ops make_ops() {
    using L = Launch<DIM, N>;
    return Ops{L::predictor, L::faces, L::corrector_detect, L::bounds, L::subcell, L::fluxcorr, L::lambda,
               L::blocks, L::batched, L::pred_args, L::NPOS,
               {256 * SubShape<DIM, N, double>::WPS, 256 * SubShape<DIM, N, float>::WPS}, BigCell<DIM, N>::SLOT};
}

}  // namespace adg
