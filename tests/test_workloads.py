"""Pins of the generated initial data that is not a plain formula of the paper.

Shock-vortex interaction (Sec. 5): the vortex temperature solves dT/dr = (gamma-1)/(R gamma)
v_phi^2/r with T = T0 outside r = b (checked against adaptive quadrature of the ODE's right
side); the resulting vortex is in radial equilibrium, dp/dr = rho v_phi^2/r (the steady
Euler equations in polar form); the post-shock state satisfies the Rankine-Hugoniot
relations of a stationary normal shock."""
import math

import numpy as np
from scipy.integrate import quad

from paper_1406_7416_amd import workloads as W


def test_vortex_temperature_solves_its_ode():
    c = W.SVI
    g = c["gamma"]
    c0 = math.sqrt(g * c["p0"] / c["rho0"])
    vm = c["Mv"] * c0
    for r in (0.0, 0.02, 0.05, 0.075, 0.09, 0.12, 0.16, 0.175, 0.3):
        if r < c["b"]:
            f = lambda s: W.svi_vphi(s, vm, c["a"], c["b"]) ** 2 / s if s > 0 else 0.0
            I = quad(f, r, c["b"], points=[c["a"]] if r < c["a"] else None, limit=200, epsabs=1e-14)[0]
        else:
            I = 0.0
        T = 1.0 - (g - 1.0) / g * I
        assert abs(float(W.svi_temperature(r, 1.0, vm, c["a"], c["b"], g)) - T) < 1e-12


def test_vortex_radial_equilibrium():
    wl = W.shock_vortex(200, 100, 5)
    c = W.SVI
    g = c["gamma"]
    c0 = math.sqrt(g * c["p0"] / c["rho0"])
    vm = c["Mv"] * c0
    r = np.linspace(0.01, 0.17, 33)
    r = r[np.abs(r - c["a"]) > 1e-3]   # central differences across the kink of v_phi at r = a
    h = 1e-6
    x = [c["xc"] + r, np.full_like(r, c["yc"])]
    xp = [c["xc"] + r + h, np.full_like(r, c["yc"])]
    xm = [c["xc"] + r - h, np.full_like(r, c["yc"])]

    def prim(xx):
        q = wl.ic(xx)
        rho = q[0]
        u, v = q[1] / rho, q[2] / rho
        p = (g - 1.0) * (q[3] - 0.5 * rho * (u * u + v * v))
        return rho, p

    rho, _ = prim(x)
    dpdr = (prim(xp)[1] - prim(xm)[1]) / (2 * h)
    vphi = W.svi_vphi(r, vm, c["a"], c["b"])
    assert np.allclose(dpdr, rho * vphi ** 2 / r, rtol=1e-6, atol=1e-8)


def test_post_shock_state_rankine_hugoniot():
    g, rho0, p0 = 1.4, 1.0, 1.0
    u0 = 1.5 * math.sqrt(g * p0 / rho0)
    rho1, u1, p1 = W.normal_shock_downstream(g, rho0, u0, p0)
    E0 = p0 / (g - 1.0) + 0.5 * rho0 * u0 ** 2
    E1 = p1 / (g - 1.0) + 0.5 * rho1 * u1 ** 2
    assert abs(rho0 * u0 - rho1 * u1) < 1e-13
    assert abs(rho0 * u0 ** 2 + p0 - (rho1 * u1 ** 2 + p1)) < 1e-12
    assert abs(u0 * (E0 + p0) - u1 * (E1 + p1)) < 1e-12
    assert rho1 > rho0 and p1 > p0 and u1 < u0   # a compression shock
