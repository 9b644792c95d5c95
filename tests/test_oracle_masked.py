"""Pins of the oracle's masked geometry (the forward-facing step of Sec. 5 removes a
rectangle from the domain; its faces are reflective walls).

* A solid half-domain equals a reflective domain boundary: the problem on [-1, 1] with the
  cells x < 0 solid advances its fluid cells to round-off like the problem on [0, 1] with a
  reflective wall at x = 0 (limiter on, a shock reflected at the wall): faces, the subcell
  halo, the subcell scheme's wall sub-faces and the neighbourhoods of the detection all see
  the wall as the reflective boundary rule does.
* The mirror image held by solid cells is symmetric: with a solid square in a corner and
  smooth initial data symmetric under the swap of x and y, the solution and the detection
  margins stay symmetric (a rule that took one axis first at the obstacle's corner would
  make the bounds of the cells there differ).
* Mass and energy are conserved with walls inside a periodic box (a reflective wall passes
  no mass and no energy), with the limiter active: every troubled cell sees the same image
  in a solid cell, so neighbouring troubled cells compute the same sub-face fluxes (an image
  that depended on the cell reading it lost 1e-7 of the mass per step).
* Solid cells keep their state; the forward-facing step on a coarse grid stays physical.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1406_7416_amd import workloads as W

GAMMA = 1.4


def _totals(o, mask):
    xi, w, *_ = O.basis(o.n)
    Wc = np.multiply.outer(w, w).ravel()
    vol = np.prod([(o.wl.hi[k] - o.wl.lo[k]) / o.wl.ncell[k] for k in range(o.dim)])
    fluid = mask == 0
    return (o.state()[:, fluid, :] * Wc).sum(axis=(1, 2)) * vol


def _slab_ic(mirrored):
    def ic(x, t=0.0):
        X, Y = x[0], x[1]
        ax = np.abs(X)
        rho = np.where(ax < 0.3, 2.0, 1.0) * (1 + 0.1 * np.sin(2 * np.pi * Y))
        p = np.where(ax < 0.3, 2.0, 1.0) + 0 * Y
        u = (-0.5 * np.sign(X) if mirrored else -0.5 + 0 * X) + 0 * Y
        return W.prim_to_cons(GAMMA, rho, [u, 0.2 + 0 * X + 0 * Y], p)
    return ic


def test_solid_half_domain_equals_reflective_wall():
    N, nx, ny = 3, 8, 4
    per = (W.BC.simple(W.PERIODIC), W.BC.simple(W.PERIODIC))
    wall = W.Workload("wall", 2, N, (nx, ny), (0.0, 0.0), (1.0, 1.0),
                      [(W.BC.simple(W.REFLECTIVE), W.BC.simple(W.TRANSMISSIVE)), per], _slab_ic(False))
    masked = W.Workload("masked", 2, N, (2 * nx, ny), (-1.0, 0.0), (1.0, 1.0),
                        [(W.BC.simple(W.TRANSMISSIVE), W.BC.simple(W.TRANSMISSIVE)), per], _slab_ic(False))
    mask = np.zeros((ny, 2 * nx), np.uint8)
    mask[:, :nx] = 1
    ow, om = O.Oracle(wall), O.Oracle(masked)
    om.set_mask(mask.ravel())
    for o, wl in ((ow, wall), (om, masked)):
        u, v = o.project(wl.ic, N + 1)
        o.set_state(u, v)
    uw0 = om.state().reshape(4, ny, 2 * nx, -1)[:, :, :nx].copy()
    troubled = 0
    for _ in range(6):
        dt = ow.cfl_dt()
        assert abs(om.cfl_dt() - dt) < 1e-15 * dt
        troubled += ow.step(dt)
        om.step(dt)
    assert troubled > 0
    uw = ow.state().reshape(4, ny, nx, -1)
    um = om.state().reshape(4, ny, 2 * nx, -1)
    assert np.abs(um[:, :, nx:] - uw).max() < 1e-11 * np.abs(uw).max()
    assert np.array_equal(om.troubled().reshape(ny, 2 * nx)[:, nx:], ow.troubled().reshape(ny, nx))
    assert not om.troubled().reshape(ny, 2 * nx)[:, :nx].any()
    assert np.array_equal(um[:, :, :nx], uw0)   # solid cells keep their state


def _corner(n=12, N=3):
    def ic(x, t=0.0):
        X, Y = x[0], x[1]
        r2 = (X - 0.6) ** 2 + (Y - 0.6) ** 2
        inside = r2 < 0.15 ** 2
        rho = np.where(inside, 1.0, 0.125) + 0 * X
        p = np.where(inside, 1.0, 0.1) + 0 * X
        z = 0 * X + 0 * Y
        return W.prim_to_cons(GAMMA, rho, [z, z], p)
    wl = W.Workload("corner", 2, N, (n, n), (0.0, 0.0), (1.0, 1.0),
                    [(W.BC.simple(W.TRANSMISSIVE), W.BC.simple(W.TRANSMISSIVE))] * 2, ic)
    mask = np.zeros((n, n), np.uint8)
    mask[: n // 2, : n // 2] = 1
    return wl, mask


def _smooth_corner(n=12, N=3):
    def ic(x, t=0.0):
        X, Y = x[0], x[1]
        r2 = (X - 0.62) ** 2 + (Y - 0.62) ** 2
        rho = 1.0 + 0.02 * np.exp(-r2 / 0.01) + 0 * X
        p = rho ** GAMMA
        z = 0 * X + 0 * Y
        return W.prim_to_cons(GAMMA, rho, [z, z], p)
    # a relaxation wide enough that the detection runs every step without flagging the pulse
    wl = W.Workload("corner", 2, N, (n, n), (0.0, 0.0), (1.0, 1.0),
                    [(W.BC.simple(W.TRANSMISSIVE), W.BC.simple(W.TRANSMISSIVE))] * 2, ic, eps=0.5, delta0=0.05)
    mask = np.zeros((n, n), np.uint8)
    mask[: n // 2, : n // 2] = 1
    return wl, mask


def test_corner_rule_keeps_diagonal_symmetry():
    """A smooth pulse next to the corner of a solid square, symmetric under the swap of x and
    y; the limiter runs its detection every step (and stays idle).  The state, and the
    detection margins (which read the solid cells' mirror images in the neighbourhood
    bounds), stay symmetric: the image rule treats the axes alike."""
    wl, mask = _smooth_corner()
    n, N = wl.ncell[0], wl.N
    o = O.Oracle(wl)
    o.set_mask(mask.ravel())
    u, v = o.project(wl.ic, N + 1)
    o.set_state(u, v)
    for _ in range(10):
        assert o.step(o.cfl_dt()) == 0
    q = o.state().reshape(4, n, n, N + 1, N + 1)       # [v][cy][cx][ay][ax]
    sw = q.transpose(0, 2, 1, 4, 3)[[0, 2, 1, 3]]       # x <-> y, momenta swapped
    assert np.abs(q - sw).max() < 1e-12 * np.abs(q).max()
    m = o.margin().reshape(n, n)
    fl = mask == 0
    assert np.abs(m - m.T)[fl].max() < 1e-9


def test_walls_conserve_mass_and_energy():
    wl, mask = _corner(n=12, N=2)
    wl.bcs = [(W.BC.simple(W.PERIODIC), W.BC.simple(W.PERIODIC))] * 2
    o = O.Oracle(wl)
    m = mask.ravel()
    o.set_mask(m)
    u, v = o.project(wl.ic, wl.N + 1)
    o.set_state(u, v)
    t0 = _totals(o, m)
    flagged = 0
    for _ in range(8):
        flagged += o.step(o.cfl_dt())
        t1 = _totals(o, m)
        assert abs(t1[0] - t0[0]) < 1e-13 * abs(t0[0])
        assert abs(t1[3] - t0[3]) < 1e-13 * abs(t0[3])
    assert flagged > 0


def test_forward_facing_step_coarse_stays_physical():
    wl = W.forward_facing_step(60, 20, 3)
    mask = W.step_mask(wl)
    o = O.Oracle(wl)
    o.set_mask(mask)
    u, v = o.project(wl.ic, 4)
    o.set_state(u, v)
    u0 = o.state()
    flagged = 0
    for _ in range(20):
        flagged += o.step(o.cfl_dt())
    q = o.state()
    assert np.array_equal(q[:, mask == 1], u0[:, mask == 1])
    fl = q[:, mask == 0]
    p = (GAMMA - 1) * (fl[3] - 0.5 * (fl[1] ** 2 + fl[2] ** 2) / fl[0])
    assert np.isfinite(fl).all() and fl[0].min() > 0 and p.min() > 0
    assert flagged > 0
    assert o.nonphysical() == 0
