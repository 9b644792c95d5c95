// Euler physics used by every kernel (the space-time predictor included): pressure from the
// ideal-gas equation of state and the Euler flux along one axis (Sec. 5).
#pragma once
#include <cmath>
#include "adg_internal.h"

namespace adg {

// ------------------------------------------------------------------ small helpers
template <int B, int E> struct Pow { static constexpr int v = B * Pow<B, E - 1>::v; };
template <int B> struct Pow<B, 0> { static constexpr int v = 1; };

__host__ __device__ constexpr int cpow(int b, int e) { return e == 0 ? 1 : b * cpow(b, e - 1); }

template <int DIM, typename R = double>
__device__ __forceinline__ R pressure(const R *q, R g) {
    R ke = 0;
#pragma unroll
    for (int j = 0; j < DIM; j++) ke += q[1 + j] * q[1 + j];
    return (g - R(1)) * (q[DIM + 1] - R(0.5) * ke / q[0]);
}

// a[1 + k] for a runtime axis k, by selection: a dynamic index would place the
// register array in scratch memory
template <int DIM, typename R>
__device__ __forceinline__ R along(const R *a, int k) {
    R r = a[1];
#pragma unroll
    for (int j = 1; j < DIM; j++)
        if (k == j) r = a[1 + j];
    return r;
}

// Euler flux along axis k (Sec. 5).
template <int DIM, typename R = double>
__device__ __forceinline__ void euler_flux(int k, const R *q, R *F, R g) {
    const R p = pressure<DIM, R>(q, g);
    const R qk = along<DIM, R>(q, k);
    const R un = qk / q[0];
    F[0] = qk;
#pragma unroll
    for (int j = 0; j < DIM; j++) F[1 + j] = q[1 + j] * un + (j == k ? p : R(0));
    F[DIM + 1] = un * (q[DIM + 1] + p);
}

// ------------------------------------------------- deviation form of the flux
// A cell's constant reference state c (the working precision's rounding of its first nodal
// value) with the velocity and total enthalpy E + p of exactly that state.
template <int DIM, typename R>
struct DevRef {
    R q[DIM + 2];
    R u[DIM];
    R h;
};

template <int DIM, typename R>
__device__ __forceinline__ DevRef<DIM, R> make_devref(const double *c64, double g) {
    DevRef<DIM, R> c;
    double q[DIM + 2];
#pragma unroll
    for (int v = 0; v < DIM + 2; v++) {
        c.q[v] = (R)c64[v];
        q[v] = (double)c.q[v];
    }
#pragma unroll
    for (int j = 0; j < DIM; j++) c.u[j] = (R)(q[1 + j] / q[0]);
    c.h = (R)(q[DIM + 1] + pressure<DIM, double>(q, g));
    return c;
}

// The change of the pressure between c and c + dq, written so that every term has the size
// of dq: delta(m.u) = m_c.du + dm.(u_c + du) with du = (dm - u_c drho) / (rho_c + drho).
// irho = 1 / (rho_c + drho).
template <int DIM, typename R>
__device__ __forceinline__ R dev_pressure(const DevRef<DIM, R> &c, const R *dq, R irho, R g) {
    R dmu = 0;
#pragma unroll
    for (int j = 0; j < DIM; j++) {
        const R du = (dq[1 + j] - c.u[j] * dq[0]) * irho;
        dmu += c.q[1 + j] * du + dq[1 + j] * (c.u[j] + du);
    }
    return (g - R(1)) * (dq[DIM + 1] - R(0.5) * dmu);
}

// F_k(c + dq) - F_k(c) (the Euler flux of Sec. 5 expanded about c, exactly, with every term
// of the size of dq, so that its rounding is relative to the deviation, not to the state);
// dp = dev_pressure(c, dq, irho).
template <int DIM, typename R>
__device__ __forceinline__ void dev_flux(int k, const DevRef<DIM, R> &c, const R *dq, R irho, R dp, R *F) {
    R uk = c.u[0];
#pragma unroll
    for (int j = 1; j < DIM; j++)
        if (k == j) uk = c.u[j];
    const R dmk = along<DIM, R>(dq, k);
    const R duk = (dmk - uk * dq[0]) * irho;
    F[0] = dmk;
#pragma unroll
    for (int j = 0; j < DIM; j++) F[1 + j] = c.q[1 + j] * duk + dq[1 + j] * (uk + duk) + (j == k ? dp : R(0));
    F[DIM + 1] = c.h * duk + (dq[DIM + 1] + dp) * (uk + duk);
}

}  // namespace adg
