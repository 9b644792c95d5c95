"""Pins of the oracle's reference-element and subcell operators against closed forms.

Sec. 2.1 (tensor Gauss-Legendre nodal basis), Sec. 2.2 eq. (pde.nc.dg2) time operator,
Sec. 4.2 eqs. (subcell.p), (subcell.r), (subcell.r.constraint), (rid).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O


def test_gauss_legendre_closed_forms():
    xi, w, *_ = O.basis(2)
    assert np.allclose(xi, [0.5 - math.sqrt(3) / 6, 0.5 + math.sqrt(3) / 6], atol=1e-15, rtol=0)
    assert np.allclose(w, [0.5, 0.5], atol=1e-15, rtol=0)
    xi, w, *_ = O.basis(3)
    assert np.allclose(xi, [0.5 - math.sqrt(15) / 10, 0.5, 0.5 + math.sqrt(15) / 10], atol=1e-15, rtol=0)
    assert np.allclose(w, [5 / 18, 8 / 18, 5 / 18], atol=1e-15, rtol=0)


@pytest.mark.parametrize("n", range(1, 11))
def test_gauss_legendre_exactness(n):
    # n-point GL integrates x^k exactly on [0,1] for k <= 2n-1
    xi, w, *_ = O.basis(n)
    for k in range(2 * n):
        assert abs(np.dot(w, xi ** k) - 1.0 / (k + 1)) < 2e-15
    # and not for k = 2n (the rule is not exact beyond its degree)
    assert abs(np.dot(w, xi ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-12


@pytest.mark.parametrize("n", [2, 4, 6, 10])
def test_derivative_and_endpoint_operators(n):
    xi, w, D, L, R, Kw = O.basis(n)
    for p in range(n):
        f = xi ** p
        df = p * xi ** (p - 1) if p else np.zeros(n)
        assert np.abs(D @ f - df).max() < 1e-12 * max(1, p * p)
        assert abs(L @ f - (1.0 if p == 0 else 0.0)) < 1e-13
        assert abs(R @ f - 1.0) < 1e-12


@pytest.mark.parametrize("n", [2, 4, 6, 10])
def test_time_operator(n):
    """Time part of eq. (pde.nc.dg2): K1 = R R^T - (diag(w) D)^T.  K1^{-1} L = 1 (the
    initial-data term reproduces a constant), and K1^{-1} diag(w) maps nodal values of a
    polynomial g of degree <= N-1 to the nodal values of int_0^tau g (the weak time-DG
    solution is exact when that integral lies in the degree-N space)."""
    xi, w, D, L, R, Kw = O.basis(n)
    K1 = np.outer(R, R) - (w[:, None] * D).T
    assert np.abs(np.linalg.solve(K1, L) - 1.0).max() < 1e-13
    assert np.abs(np.linalg.solve(K1, np.diag(w)) - Kw).max() < 1e-12
    for p in range(n - 1):
        assert np.abs(Kw @ xi ** p - xi ** (p + 1) / (p + 1)).max() < 1e-13


@pytest.mark.parametrize("N", [1, 2, 3, 5, 9])
def test_projection_pins(N):
    Ns = 2 * N + 1
    P, R = O.subcell_ops(N, Ns)
    xi, w, *_ = O.basis(N + 1)
    assert np.abs(P.sum(axis=1) - 1).max() < 1e-13            # constants
    for p in range(N + 1):                                      # eq. (subcell.p) on monomials
        s = np.arange(Ns)
        exact = Ns * (((s + 1) / Ns) ** (p + 1) - (s / Ns) ** (p + 1)) / (p + 1)
        assert np.abs(P @ xi ** p - exact).max() < 1e-12
    # eq. (rid): R o P = I
    assert np.abs(R @ P - np.eye(N + 1)).max() < 1e-12
    # eq. (subcell.r.constraint): the reconstructed polynomial keeps the cell mean
    rng = np.random.default_rng(N)
    v = rng.normal(size=Ns)
    assert abs(w @ (R @ v) - v.mean()) < 1e-14
    # constrained least squares solved as a KKT system equals R
    A = P / Ns  # integrals over subcells of each basis function (|S| = 1/Ns)
    c = w       # integral over the cell of each basis function
    kkt = np.zeros((N + 2, N + 2))
    kkt[:N + 1, :N + 1] = 2 * A.T @ A
    kkt[:N + 1, N + 1] = c
    kkt[N + 1, :N + 1] = c
    for j in range(Ns):
        e = np.zeros(Ns)
        e[j] = 1.0
        rhs = np.concatenate([2 * A.T @ (e / Ns), [e.mean()]])
        sol = np.linalg.solve(kkt, rhs)
        assert np.abs(sol[:N + 1] - R[:, j]).max() < 1e-11


def test_weno3_reproduces_quadratics():
    """Each 3-cell stencil reproduces quadratics exactly, hence so does any convex
    combination: averages of a quadratic give its exact point values."""
    xi3, *_ = O.basis(3)
    rng = np.random.default_rng(3)
    for _ in range(10):
        c = rng.normal(size=3)
        F = lambda x: c[0] * x + c[1] * x ** 2 / 2 + c[2] * x ** 3 / 3  # antiderivative
        avg = np.array([F(o + 1) - F(o) for o in range(-2, 3)])
        out = O.weno3(avg)
        exact = c[0] + c[1] * xi3 + c[2] * xi3 ** 2
        assert np.abs(out - exact).max() < 1e-11


def test_weno3_non_oscillatory_on_a_step():
    out = O.weno3([0.0, 0.0, 0.0, 1.0, 1.0])
    assert out.min() > -1e-6 and out.max() < 1 + 1e-6
    out = O.weno3([0.0, 0.0, 1.0, 1.0, 1.0])
    assert out.min() > -1e-6 and out.max() < 1 + 1e-6


# ---------------------------------------------------------------- Osher-type flux
def _euler_flux(d, k, g, Q):
    p = (g - 1) * (Q[d + 1] - 0.5 * sum(Q[1 + j] ** 2 for j in range(d)) / Q[0])
    un = Q[1 + k] / Q[0]
    F = np.zeros(d + 2)
    F[0] = Q[1 + k]
    for j in range(d):
        F[1 + j] = Q[1 + j] * un + (p if j == k else 0)
    F[d + 1] = un * (Q[d + 1] + p)
    return F


def _state(d, g, rho, u, p):
    return np.array([rho] + [rho * x for x in u] + [p / (g - 1) + 0.5 * rho * sum(x * x for x in u)])


def _jac(d, k, g, Q, y, eps=1e-6):
    """A(Q) y by a centred difference of the Euler flux (independent of the eigen-split)."""
    return (_euler_flux(d, k, g, Q + eps * y) - _euler_flux(d, k, g, Q - eps * y)) / (2 * eps)


@pytest.mark.parametrize("d", [2, 3])
def test_osher_flux_consistent(d):
    rng = np.random.default_rng(11)
    for _ in range(5):
        q = _state(d, 1.4, rng.uniform(0.2, 2), rng.uniform(-1, 1, d), rng.uniform(0.2, 2))
        for k in range(d):
            G = O.numerical_flux(d, k, 1.4, 1, q, q)
            assert np.abs(G - _euler_flux(d, k, 1.4, q)).max() < 1e-14 * max(1, np.abs(G).max())


def test_osher_flux_resolves_stationary_contact():
    """Zero normal velocity, equal pressure, different densities: the Osher-type flux gives
    the exact flux (0, p, 0, 0); Rusanov adds dissipation."""
    g, p = 1.4, 0.7
    qL, qR = _state(2, g, 1.0, [0, 0], p), _state(2, g, 0.2, [0, 0], p)
    G = O.numerical_flux(2, 0, g, 1, qL, qR)
    assert np.abs(G - np.array([0, p, 0, 0])).max() < 1e-14
    Gr = O.numerical_flux(2, 0, g, 0, qL, qR)
    assert abs(Gr[0]) > 1e-2


@pytest.mark.parametrize("d", [2, 3])
def test_abs_jacobian_matches_jacobian(d):
    """Supersonic along k: |A| dq = A dq; any state: |A| |A| dq = A A dq (A by finite
    differences of the flux, so a wrong eigenvector or wave strength shows)."""
    g = 1.4
    rng = np.random.default_rng(5)
    for k in range(d):
        u = list(rng.uniform(-0.5, 0.5, d))
        u[k] = 3.0
        Q = _state(d, g, 1.1, u, 0.9)            # c ~ 1.06 < u_k
        dq = rng.normal(size=d + 2)
        a = O.abs_jacobian(d, k, g, Q, dq)
        assert np.abs(a - _jac(d, k, g, Q, dq)).max() < 1e-7 * np.abs(a).max()
        Q2 = _state(d, g, 0.8, list(rng.uniform(-0.4, 0.4, d)), 1.3)   # subsonic
        aa = O.abs_jacobian(d, k, g, Q2, O.abs_jacobian(d, k, g, Q2, dq))
        AA = _jac(d, k, g, Q2, _jac(d, k, g, Q2, dq), eps=1e-5)
        assert np.abs(aa - AA).max() < 1e-6 * np.abs(AA).max()


def test_osher_flux_upwind_when_supersonic():
    """All eigenvalues positive along the path: the flux is F(qL) up to the error of the
    3-point rule on the path integral (small for a small jump)."""
    g = 1.4
    qL = _state(2, g, 1.0, [3.0, 0.2], 1.0)
    qR = _state(2, g, 1.03, [3.05, 0.21], 1.04)
    G = O.numerical_flux(2, 0, g, 1, qL, qR)
    FL = _euler_flux(2, 0, g, qL)
    assert np.abs(G - FL).max() < 1e-7 * np.abs(FL).max()
