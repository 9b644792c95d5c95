// Device helpers shared by the kernels: numerical fluxes, boundary ghost states and cell
// indexing.
#pragma once
#include <cmath>
#include <type_traits>
#include "adg_internal.h"
#include "adg_physics.h"

namespace adg {

// Rusanov flux; wave speed per quadrature node: max over both sides of |u_n| + c.
template <int DIM, typename R = double>
__device__ __forceinline__ void rusanov(int k, const R *qL, const R *qR, R *G, R g) {
    constexpr int NV = DIM + 2;
    R FL[NV], FR[NV];
    euler_flux<DIM, R>(k, qL, FL, g);
    euler_flux<DIM, R>(k, qR, FR, g);
    const R sL = fabs(along<DIM, R>(qL, k) / qL[0]) + sqrt(g * pressure<DIM, R>(qL, g) / qL[0]);
    const R sR = fabs(along<DIM, R>(qR, k) / qR[0]) + sqrt(g * pressure<DIM, R>(qR, g) / qR[0]);
    const R s = fmax(sL, sR);
#pragma unroll
    for (int v = 0; v < NV; v++) G[v] = R(0.5) * (FL[v] + FR[v]) - R(0.5) * s * (qR[v] - qL[v]);
}

// |A(Q)| dQ for the Euler flux Jacobian along axis k: dQ split into the waves of A at Q
// (acoustic, entropy, shear), each scaled by |u_k - c|, |u_k| or |u_k + c|.
template <int DIM, typename R>
__device__ __forceinline__ void abs_jacobian(int k, const R *Q, const R *dQ, R g, R *out) {
    constexpr int NV = DIM + 2;
    const R rho = Q[0], ir = R(1) / Q[0];
    R u[DIM], du[DIM], q2 = 0, mdq = 0, un = 0, duk = 0;
#pragma unroll
    for (int j = 0; j < DIM; j++) {
        u[j] = Q[1 + j] * ir;
        q2 += u[j] * u[j];
        du[j] = (dQ[1 + j] - u[j] * dQ[0]) * ir;
        mdq += u[j] * dQ[1 + j];
        if (j == k) { un = u[j]; duk = du[j]; }
    }
    const R p = pressure<DIM, R>(Q, g);
    const R c2 = g * p * ir, c = sqrt(c2), H = (Q[NV - 1] + p) * ir;
    const R dp = (g - R(1)) * (dQ[NV - 1] - mdq + R(0.5) * q2 * dQ[0]);
    const R a1 = (dp - rho * c * duk) / (R(2) * c2), a5 = (dp + rho * c * duk) / (R(2) * c2);
    const R a2 = dQ[0] - dp / c2;
    const R l1 = fabs(un - c), l2 = fabs(un), l5 = fabs(un + c);
    out[0] = l1 * a1 + l5 * a5 + l2 * a2;
    R e = l1 * a1 * (H - c * un) + l5 * a5 * (H + c * un) + l2 * a2 * R(0.5) * q2;
#pragma unroll
    for (int j = 0; j < DIM; j++) {
        const bool nk = j != k;
        out[1 + j] = l1 * a1 * (u[j] - (nk ? R(0) : c)) + l5 * a5 * (u[j] + (nk ? R(0) : c)) + l2 * a2 * u[j] +
                     (nk ? l2 * rho * du[j] : R(0));
        if (nk) e += l2 * rho * du[j] * u[j];
    }
    out[NV - 1] = e;
}

// Osher-type flux in the universal form: (F(qL) + F(qR))/2 - 1/2 int_0^1 |A(psi(s))| ds
// (qR - qL) on the straight path psi(s) = qL + s (qR - qL), 3-point Gauss-Legendre (xs, ws).
template <int DIM, typename R>
__device__ __forceinline__ void osher(int k, const R *qL, const R *qR, R *G, R g, const R *xs, const R *ws) {
    constexpr int NV = DIM + 2;
    R FL[NV], FR[NV], dQ[NV], acc[NV];
    euler_flux<DIM, R>(k, qL, FL, g);
    euler_flux<DIM, R>(k, qR, FR, g);
#pragma unroll
    for (int v = 0; v < NV; v++) {
        dQ[v] = qR[v] - qL[v];
        acc[v] = 0;
    }
#pragma unroll
    for (int j = 0; j < 3; j++) {
        R psi[NV], o[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) psi[v] = qL[v] + xs[j] * dQ[v];
        abs_jacobian<DIM, R>(k, psi, dQ, g, o);
#pragma unroll
        for (int v = 0; v < NV; v++) acc[v] += ws[j] * o[v];
    }
#pragma unroll
    for (int v = 0; v < NV; v++) G[v] = R(0.5) * (FL[v] + FR[v]) - R(0.5) * acc[v];
}

// The scheme's numerical flux (Sec. 2.3): Rusanov or Osher-type.
template <int DIM, typename R>
__device__ __forceinline__ void num_flux(const Prob &P, const Tables *T, int k, const R *qL, const R *qR, R *G) {
    if (P.flux == 1) {
        R xs[3], ws[3];
#pragma unroll
        for (int j = 0; j < 3; j++) {
            xs[j] = sizeof(R) == 4 ? (R)T->fxi3[j] : (R)T->xi3[j];
            ws[j] = sizeof(R) == 4 ? (R)T->fw3[j] : (R)T->w3[j];
        }
        osher<DIM, R>(k, qL, qR, G, (R)P.gamma, xs, ws);
    } else {
        rusanov<DIM, R>(k, qL, qR, G, (R)P.gamma);
    }
}

template <int DIM, typename R = double>
__device__ __forceinline__ bool physical(const R *q, R g) {
#pragma unroll
    for (int v = 0; v < DIM + 2; v++)
        if (!isfinite(q[v])) return false;
    return q[0] > R(0) && pressure<DIM, R>(q, g) > R(0);
}

// Ghost state of one boundary side (transmissive / reflective / Dirichlet with split).
// The point's coordinates come as values (x0, x1, x2): a selection among the elements of
// an array would become a dynamic index into it.
template <int DIM>
__device__ __forceinline__ void bc_ghost(const Prob &P, int k, int side, const double *qin, double x0, double x1,
                                         double x2, double t, double *qout) {
    constexpr int NV = DIM + 2;
    const BCDev &b = P.bc[k][side];
    int which = 0;
    if (b.split_axis >= 0) {
        const double xs = b.split_axis == 0 ? x0 : (b.split_axis == 1 ? x1 : x2);
        which = (xs < b.split0 + b.split_speed * t) ? 0 : 1;
    }
    // value selections only: a branch per kind would merge pointers into the kernel
    // argument and into the caller's arrays, which moves both to scratch memory
    const int kind = b.kind[which];
    const bool dir = kind == ADG_DIRICHLET, refl = kind == ADG_REFLECTIVE;
#pragma unroll
    for (int v = 0; v < NV; v++) {
        const double st = which ? b.state[1][v] : b.state[0][v];
        const double in = (refl && v == 1 + k) ? -qin[v] : qin[v];
        qout[v] = dir ? st : in;
    }
}

__device__ __forceinline__ int64_t cell_of(const Prob &P, const int *ci) {
    return ci[0] + (int64_t)P.nc[0] * (ci[1] + (int64_t)P.nc[1] * ci[2]);
}
__device__ __forceinline__ void coords_of(const Prob &P, int64_t c, int *ci) {
    ci[0] = (int)(c % P.nc[0]);
    ci[1] = (int)((c / P.nc[0]) % P.nc[1]);
    ci[2] = (int)(c / ((int64_t)P.nc[0] * P.nc[1]));
}

// ------------------------------------------------------------- wave reductions
// A 32-bit value moved down by S lanes within each row of 16 lanes (DPP row_shr); a lane
// whose source lies outside its row keeps its own value (harmless for min, max and or).
template <int S>
__device__ __forceinline__ int row_shr(int x) {
    return __builtin_amdgcn_update_dpp(x, x, 0x110 + S, 0xf, 0xf, false);
}
template <int S>
__device__ __forceinline__ double row_shr(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = row_shr<S>((int)(b & 0xffffffff)), hi = row_shr<S>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int S>
__device__ __forceinline__ float row_shr(float x) {
    return __int_as_float(row_shr<S>(__float_as_int(x)));
}
__device__ __forceinline__ double lane_value(double x, int lane) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ float lane_value(float x, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
__device__ __forceinline__ int lane_value(int x, int lane) { return __builtin_amdgcn_readlane(x, lane); }

// op over the 64 lanes of a wave (every lane active), the result in every lane: shifts of
// 1, 2, 4 and 8 lanes leave each row's result in its last lane, then the four row results
// are combined from scalar registers.  op is associative, commutative and idempotent.
template <typename T, typename Op>
__device__ __forceinline__ T wave_reduce(T x, Op op) {
    x = op(x, row_shr<1>(x));
    x = op(x, row_shr<2>(x));
    x = op(x, row_shr<4>(x));
    x = op(x, row_shr<8>(x));
    return op(op(lane_value(x, 15), lane_value(x, 31)), op(lane_value(x, 47), lane_value(x, 63)));
}
__device__ __forceinline__ double wave_min(double x) {
    return wave_reduce(x, [](double a, double b) { return fmin(a, b); });
}
__device__ __forceinline__ double wave_max(double x) {
    return wave_reduce(x, [](double a, double b) { return fmax(a, b); });
}

// ------------------------------------------------------------- masked geometry
// 1 if the cell at global coordinates g (possibly outside the domain) is solid: outside a
// periodic axis it wraps, outside another axis it is the interior cell it mirrors.
template <int DIM>
__device__ __forceinline__ bool solid_at(const Prob &P, const uint8_t *mask, int g0, int g1, int g2) {
    int c[3] = {g0, g1, g2};
#pragma unroll
    for (int k = 0; k < DIM; k++) {
        const int nk = P.nc[k];
        int x = c[k];
        if (x < 0 || x >= nk) x = P.periodic[k] ? (x % nk + nk) % nk : (x >= nk ? 2 * nk - 1 - x : -1 - x);
        c[k] = x;
    }
    if (DIM == 2) c[2] = 0;
    return mask[cell_of(P, c)] != 0;
}

// The mirror image a solid cell g holds (the fluid across its walls): step[k] = -1 / +1 if
// its lower / upper face neighbour along k is fluid (the lower one first), 0 if neither; the
// image is the cell g + step with the subcell index reversed and the momentum negated along
// every axis with step[k] != 0 (the point reflection at a convex corner of the obstacle).
template <int DIM>
__device__ __forceinline__ void solid_image(const Prob &P, const uint8_t *mask, const int *g, int *step) {
#pragma unroll
    for (int k = 0; k < 3; k++) step[k] = 0;
#pragma unroll
    for (int k = 0; k < DIM; k++) {
        const int lo0 = g[0] - (k == 0), lo1 = g[1] - (k == 1), lo2 = g[2] - (k == 2);
        const int hi0 = g[0] + (k == 0), hi1 = g[1] + (k == 1), hi2 = g[2] + (k == 2);
        step[k] = !solid_at<DIM>(P, mask, lo0, lo1, lo2) ? -1 : (!solid_at<DIM>(P, mask, hi0, hi1, hi2) ? 1 : 0);
    }
}

// The reflective wall of the masked geometry: the ghost state across a wall normal to k.
template <int DIM, typename R>
__device__ __forceinline__ void wall_ghost(int k, const R *qin, R *qout) {
#pragma unroll
    for (int v = 0; v < DIM + 2; v++) qout[v] = (v == 1 + k) ? -qin[v] : qin[v];
}

}  // namespace adg
