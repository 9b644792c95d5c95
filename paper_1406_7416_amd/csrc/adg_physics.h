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

}  // namespace adg
