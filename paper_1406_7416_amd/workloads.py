"""Synthetic workloads: initial conditions, boundary conditions and grid shapes.

This module is the single source of inputs for both the oracle-side tests and the GPU
path.  It holds no arithmetic of the numerical method: it only evaluates initial-data
functions at points that the caller supplies, converts primitive to conserved variables
with the ideal-gas equation of state (Sec. 5 of the paper), and describes grids and
boundaries.  Every random draw is seeded (numpy PCG64).

Workloads follow the experiments of Sec. 5 of Dumbser, Zanotti, Loubere, Diot (2014):
  * explosion_2d / explosion_3d   -- Sec. 5, 3D explosion (and its 2D analogue)
  * vortex                        -- Sec. 5, smooth isentropic vortex
  * double_mach                   -- Sec. 5, double Mach reflection (W&C frame)
  * quadrant_batch                -- Sec. 5, 2D Riemann problems (random quadrant states)
  * shock_tube                    -- Sec. 5, Sod and Lax tubes (Table 1)
  * forward_facing_step           -- Sec. 5, forward-facing step (masked geometry, step_mask)
  * contact_wave                  -- polynomial density advected at constant u, p
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

PERIODIC, TRANSMISSIVE, REFLECTIVE, DIRICHLET = 0, 1, 2, 3


@dataclasses.dataclass
class BC:
    """One side of one axis.  Below the split (coordinate along ``split_axis`` smaller
    than ``split0 + split_speed * t``) the first (kind, state) applies, else the second."""
    kind: Tuple[int, int]
    states: Tuple[Tuple[float, ...], Tuple[float, ...]] = ((0.0,) * 5, (0.0,) * 5)
    split_axis: int = -1
    split0: float = 0.0
    split_speed: float = 0.0

    @staticmethod
    def simple(kind: int, state: Sequence[float] = (0.0,) * 5) -> "BC":
        s = tuple(state) + (0.0,) * (5 - len(state))
        return BC((kind, kind), (s, s))


@dataclasses.dataclass
class Workload:
    name: str
    dim: int
    N: int
    ncell: Tuple[int, ...]
    lo: Tuple[float, ...]
    hi: Tuple[float, ...]
    bcs: List[Tuple[BC, BC]]
    ic: Callable  # ic(x: list of coordinate arrays (broadcastable), t) -> conserved list
    gamma: float = 1.4
    cfl: float = 0.0     # 0 -> stable_cfl(N)
    t_end: float = 0.0
    Ns: int = 0          # 0 -> 2N+1
    eps: float = 1e-3
    delta0: float = 1e-4

    @property
    def nv(self) -> int:
        return self.dim + 2

    def __post_init__(self):
        if not self.cfl:
            self.cfl = stable_cfl(self.N)

    @property
    def num_cells(self) -> int:
        return int(np.prod(self.ncell))

    @property
    def subcells(self) -> int:
        return self.Ns if self.Ns else 2 * self.N + 1

    def st_dof_per_step(self) -> int:
        """Space-time degrees of freedom per step and conserved variable (the paper's
        counting: (N+1)^(d+1) per cell)."""
        return self.num_cells * (self.N + 1) ** (self.dim + 1)


# Courant factors applied to the time step rule of Sec. 2.4, eq. (cfl).  The paper states
# that rule as approximate (the DG stability limit "roughly" follows 1/(2N+1)); with the
# Rusanov flux this ADER-DG step is linearly stable only below a factor that falls with
# N.  These factors were measured stable on smooth periodic problems (unlimited scheme).
STABLE_CFL = {1: 0.9, 2: 0.9, 3: 0.7, 4: 0.6, 5: 0.5, 6: 0.45, 7: 0.4, 8: 0.35, 9: 0.3}


def stable_cfl(N: int) -> float:
    return STABLE_CFL.get(N, 0.3)


def prim_to_cons(gamma: float, rho, vel: Sequence, p) -> list:
    """Ideal-gas EOS of Sec. 5: rho E = p/(gamma-1) + rho |v|^2 / 2."""
    ke = sum(np.asarray(v, dtype=np.float64) ** 2 for v in vel)
    out = [np.asarray(rho, dtype=np.float64)]
    out += [np.asarray(rho, dtype=np.float64) * np.asarray(v, dtype=np.float64) for v in vel]
    out.append(np.asarray(p, dtype=np.float64) / (gamma - 1.0) + 0.5 * np.asarray(rho) * ke)
    return out


def sample_grid(ic: Callable, axes: Sequence[np.ndarray], t: float = 0.0) -> np.ndarray:
    """Evaluate ``ic`` on the tensor grid spanned by the per-axis coordinates ``axes``
    (x fastest in the result).  Returns float64 [nv][...z, y, x] flattened per variable.
    The grid is evaluated in slabs along the slowest axis (``ic`` acts point by point), so
    the temporaries stay small next to the result."""
    d = len(axes)
    axes = [np.asarray(a, dtype=np.float64) for a in axes]
    sizes = [len(a) for a in axes]
    per_slab = int(np.prod(sizes[:-1]))
    slab = max(1, min(sizes[-1], (1 << 22) // max(per_slab, 1)))
    out = None
    for z0 in range(0, sizes[-1], slab):
        z1 = min(sizes[-1], z0 + slab)
        mesh = []
        for k, a in enumerate(axes):
            shape = [1] * d
            shape[d - 1 - k] = len(a) if k < d - 1 else z1 - z0
            mesh.append((a if k < d - 1 else a[z0:z1]).reshape(shape))
        vals = ic(mesh, t)
        full = np.broadcast_shapes(*[np.shape(m) for m in mesh])
        if out is None:
            out = np.empty((len(vals), int(np.prod(sizes))))
        for v, val in enumerate(vals):
            out[v, z0 * per_slab:z1 * per_slab] = np.broadcast_to(np.asarray(val, dtype=np.float64), full).ravel()
    return out


# ----------------------------------------------------------------- explosions
def explosion_ic(dim: int, gamma: float = 1.4, R: float = 0.5):
    """Sec. 5 3D explosion (a multi-dimensional Sod problem): rho=1, p=1 inside r <= R,
    rho=0.125, p=0.1 outside, at rest."""
    def ic(x, t=0.0):
        r2 = sum(xx * xx for xx in x)
        inside = r2 <= R * R
        rho = np.where(inside, 1.0, 0.125)
        p = np.where(inside, 1.0, 0.1)
        zero = np.zeros_like(rho)
        return prim_to_cons(gamma, rho, [zero] * dim, p)
    return ic


def explosion_2d(n: int = 40, N: int = 3) -> Workload:
    return Workload("explosion2d", 2, N, (n, n), (-1.0, -1.0), (1.0, 1.0),
                    [(BC.simple(TRANSMISSIVE), BC.simple(TRANSMISSIVE))] * 2,
                    explosion_ic(2), t_end=0.25)


def explosion_3d(n: int = 128, N: int = 3) -> Workload:
    return Workload("explosion3d", 3, N, (n, n, n), (-1.0,) * 3, (1.0,) * 3,
                    [(BC.simple(TRANSMISSIVE), BC.simple(TRANSMISSIVE))] * 3,
                    explosion_ic(3), t_end=0.25)


# -------------------------------------------------------------------- vortex
def vortex_ic(gamma: float = 1.4, beta: float = 5.0, centre=(5.0, 5.0), period: float = 10.0,
              uinf: float = 1.0, vinf: float = 1.0):
    """Sec. 5 isentropic vortex on a periodic box.  reading: the temperature perturbation
    carries beta^2 (dT = -(gamma-1) beta^2/(8 gamma pi^2) exp(1-r^2)); only then is the
    vortex a steady solution of the Euler equations in the moving frame.  p = rho^gamma.
    At time t the exact solution is the initial one translated by (uinf, vinf) t."""
    def ic(x, t=0.0):
        X, Y = x[0], x[1]
        # distance to the nearest periodic image of the translated centre
        xc = centre[0] + uinf * t
        yc = centre[1] + vinf * t
        dx = (X - xc + 0.5 * period) % period - 0.5 * period
        dy = (Y - yc + 0.5 * period) % period - 0.5 * period
        r2 = dx * dx + dy * dy
        e = np.exp(0.5 * (1.0 - r2))
        du = -dy * beta / (2.0 * math.pi) * e
        dv = dx * beta / (2.0 * math.pi) * e
        dT = -(gamma - 1.0) * beta * beta / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
        T = 1.0 + dT
        rho = T ** (1.0 / (gamma - 1.0))
        p = rho ** gamma
        return prim_to_cons(gamma, rho, [uinf + du, vinf + dv], p)
    return ic


def vortex(n: int = 64, N: int = 9, period: float = 10.0) -> Workload:
    return Workload("vortex", 2, N, (n, n), (0.0, 0.0), (period, period),
                    [(BC.simple(PERIODIC), BC.simple(PERIODIC))] * 2,
                    vortex_ic(period=period, centre=(period / 2, period / 2)), t_end=10.0)


# ------------------------------------------------------------ double Mach
def dmr_states(gamma: float = 1.4):
    """Pre-/post-shock states of the Mach-10 shock (Sec. 5, double Mach reflection).
    reading: the printed factor 1/gamma applies to density and pressure only; in the
    Woodward-Colella scaling (pre-shock rho=1.4, p=1) this gives rho=8, p=116.5 and a
    normal velocity 8.25, here for a shock at 60 degrees to the x axis."""
    pre = (1.4, 0.0, 0.0, 1.0)
    post = (8.0, 8.25 * math.cos(math.pi / 6), -8.25 * math.sin(math.pi / 6), 116.5)
    return pre, post


def _cons_tuple(gamma, prim):
    rho, u, v, p = prim
    return (rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v), 0.0)


def double_mach(nx: int = 400, ny: int = 100, N: int = 5, gamma: float = 1.4, Lx: float = 4.0,
                Ly: float = 1.0) -> Workload:
    """Domain [0, Lx] x [0, Ly]; the top boundary carries the exact moving oblique shock
    at y = Ly (a smaller window of the same problem keeps the paper's mesh size)."""
    pre, post = dmr_states(gamma)
    x0 = 1.0 / 6.0
    cpre, cpost = _cons_tuple(gamma, pre), _cons_tuple(gamma, post)

    def ic(x, t=0.0):
        X, Y = x[0], x[1]
        xs = x0 + (Y + 20.0 * t) / math.sqrt(3.0)
        behind = X < xs
        rho = np.where(behind, post[0], pre[0])
        u = np.where(behind, post[1], pre[1])
        v = np.where(behind, post[2], pre[2])
        p = np.where(behind, post[3], pre[3])
        return prim_to_cons(gamma, rho, [u, v], p)

    left = BC.simple(DIRICHLET, cpost)
    right = BC.simple(TRANSMISSIVE)
    # bottom: post-shock inflow for x < 1/6, reflecting wall after
    bottom = BC((DIRICHLET, REFLECTIVE), (cpost, cpost), split_axis=0, split0=x0, split_speed=0.0)
    # top: exact moving shock, x_s(t) = 1/6 + (Ly + 20 t)/sqrt(3)
    top = BC((DIRICHLET, DIRICHLET), (cpost, cpre), split_axis=0,
             split0=x0 + Ly / math.sqrt(3.0), split_speed=20.0 / math.sqrt(3.0))
    return Workload("double_mach", 2, N, (nx, ny), (0.0, 0.0), (Lx, Ly),
                    [(left, right), (bottom, top)], ic, t_end=0.2)


# --------------------------------------------------- shock-vortex interaction
SVI = dict(gamma=1.4, a=0.075, b=0.175, Ms=1.5, Mv=0.7, p0=1.0, rho0=1.0, xc=0.25, yc=0.5, xs=0.5)


def normal_shock_downstream(gamma: float, rho0: float, u0: float, p0: float):
    """Rankine-Hugoniot state behind a stationary normal shock for the upstream state
    (rho0, u0 > 0, p0) (flow in +x)."""
    M2 = u0 * u0 * rho0 / (gamma * p0)
    rho1 = rho0 * (gamma + 1.0) * M2 / ((gamma - 1.0) * M2 + 2.0)
    p1 = p0 * (1.0 + 2.0 * gamma / (gamma + 1.0) * (M2 - 1.0))
    return rho1, u0 * rho0 / rho1, p1


def svi_vphi(r, vm: float, a: float, b: float):
    """Angular velocity of the vortex (Sec. 5, shock-vortex interaction)."""
    r = np.asarray(r, dtype=np.float64)
    rs = np.maximum(r, 1e-300)
    inner = vm * r / a
    ring = vm * a / (a * a - b * b) * (r - b * b / rs)
    return np.where(r <= a, inner, np.where(r <= b, ring, 0.0))


def svi_temperature(r, T0: float, vm: float, a: float, b: float, gamma: float, R: float = 1.0):
    """T(r) of the vortex: dT/dr = (gamma-1)/(R gamma) v_phi^2 / r with T = T0 for r >= b,
    integrated in closed form (v_phi^2/r is r vm^2/a^2 inside a and A^2 (r - 2 b^2/r + b^4/r^3)
    on the ring, A = vm a/(a^2 - b^2))."""
    r = np.asarray(r, dtype=np.float64)
    K = (gamma - 1.0) / (R * gamma)
    A2 = (vm * a / (a * a - b * b)) ** 2

    def ring_primitive(s):
        return A2 * (0.5 * s * s - 2.0 * b * b * np.log(s) - 0.5 * b ** 4 / (s * s))

    # integral of v^2/s from r to b
    ring_part_a = ring_primitive(b) - ring_primitive(a)
    rr = np.clip(r, a, b)
    I_ring = ring_primitive(b) - ring_primitive(rr)
    I_inner = vm * vm / (2.0 * a * a) * (a * a - np.minimum(r, a) ** 2) + ring_part_a
    I = np.where(r >= b, 0.0, np.where(r >= a, I_ring, I_inner))
    return T0 - K * I


def shock_vortex(nx: int = 200, ny: int = 100, N: int = 5) -> Workload:
    """Sec. 5 shock-vortex interaction on [0,2] x [0,1]: stationary normal shock at x = 0.5
    (upstream rho0 = p0 = 1, Mach Ms = 1.5 in +x; downstream by Rankine-Hugoniot) and a vortex
    of Mach Mv = 0.7 at (0.25, 0.5), superposed on the upstream flow.  Boundaries (not given
    in the paper; reading): the upstream state flows in on the left, transmissive elsewhere.
    The paper's mesh size h = 1/100 is the default grid."""
    c = SVI
    g, rho0, p0 = c["gamma"], c["rho0"], c["p0"]
    c0 = math.sqrt(g * p0 / rho0)
    u0 = c["Ms"] * c0
    vm = c["Mv"] * c0
    T0 = p0 / rho0
    rho1, u1, p1 = normal_shock_downstream(g, rho0, u0, p0)

    def ic(x, t=0.0):
        X, Y = x[0], x[1]
        dx, dy = X - c["xc"], Y - c["yc"]
        r = np.sqrt(dx * dx + dy * dy)
        vphi = svi_vphi(r, vm, c["a"], c["b"])
        rs = np.maximum(r, 1e-300)
        T = svi_temperature(r, T0, vm, c["a"], c["b"], g)
        up = X < c["xs"]
        rho = np.where(up, rho0 * (T / T0) ** (1.0 / (g - 1.0)), rho1)
        p = np.where(up, p0 * (T / T0) ** (g / (g - 1.0)), p1)
        u = np.where(up, u0 - vphi * dy / rs, u1)
        v = np.where(up, vphi * dx / rs, 0.0 * X)
        return prim_to_cons(g, rho, [u, v], p)

    inflow = BC.simple(DIRICHLET, _cons_tuple(g, (rho0, u0, 0.0, p0)))
    out = BC.simple(TRANSMISSIVE)
    return Workload("shock_vortex", 2, N, (nx, ny), (0.0, 0.0), (2.0, 1.0),
                    [(inflow, out), (out, out)], ic, gamma=g, t_end=0.7)


# ------------------------------------------------------- forward-facing step
def forward_facing_step(nx: int = 300, ny: int = 100, N: int = 5, gamma: float = 1.4) -> Workload:
    """Sec. 5 forward-facing step: a Mach-3 wind tunnel, rho = gamma, p = 1, u = 3, v = 0,
    on [0,3] x [0,1] without the step [0.6,3] x [0,0.2] (the cells with centres in it are solid,
    step_mask); inflow of the initial state on the left, outflow (transmissive) on the right,
    reflective walls at the top, the bottom and on the step.  The paper's mesh size h = 1/100
    is the default grid; t_end = 4."""
    state = (gamma, 3.0, 0.0, 1.0)

    def ic(x, t=0.0):
        X, Y = x[0], x[1]
        z = 0.0 * X + 0.0 * Y
        return prim_to_cons(gamma, state[0] + z, [state[1] + z, state[2] + z], state[3] + z)

    wl = Workload("forward_step", 2, N, (nx, ny), (0.0, 0.0), (3.0, 1.0),
                  [(BC.simple(DIRICHLET, _cons_tuple(gamma, state)), BC.simple(TRANSMISSIVE)),
                   (BC.simple(REFLECTIVE), BC.simple(REFLECTIVE))], ic, gamma=gamma, t_end=4.0)
    return wl


def step_mask(wl: Workload, x0: float = 0.6, y1: float = 0.2) -> np.ndarray:
    """Solid cells of the forward-facing step: cell centres in [x0, hi_x] x [lo_y, y1], one byte
    per cell, x fastest."""
    nx, ny = wl.ncell[0], wl.ncell[1]
    xc = wl.lo[0] + (np.arange(nx) + 0.5) * (wl.hi[0] - wl.lo[0]) / nx
    yc = wl.lo[1] + (np.arange(ny) + 0.5) * (wl.hi[1] - wl.lo[1]) / ny
    return ((xc[None, :] > x0) & (yc[:, None] < y1)).astype(np.uint8).ravel()


# ------------------------------------------------------- four-quadrant RPs
def quadrant_ic(states, gamma: float = 1.4):
    """Sec. 5 2D Riemann problem: u1 for x>0,y>0; u2 for x<=0,y>0; u3 for x<=0,y<=0;
    u4 for x>0,y<=0.  states: 4 primitive tuples (rho, u, v, p)."""
    def ic(x, t=0.0):
        X, Y = x[0], x[1]
        q = [np.asarray(s, dtype=np.float64) for s in states]
        sel = [(X > 0) & (Y > 0), (X <= 0) & (Y > 0), (X <= 0) & (Y <= 0), (X > 0) & (Y <= 0)]
        prim = []
        for comp in range(4):
            val = np.zeros(np.broadcast_shapes(np.shape(X), np.shape(Y)))
            for s, m in zip(q, sel):
                val = np.where(m, s[comp], val)
            prim.append(val)
        return prim_to_cons(gamma, prim[0], [prim[1], prim[2]], prim[3])
    return ic


QUADRANT_SEED = 20140627


def quadrant_batch(count: int = 256, seed: int = QUADRANT_SEED,
                   grids=(32, 64, 128, 256), degrees=(3, 4, 5)) -> List[Workload]:
    """Independent four-quadrant Riemann problems on [-0.5, 0.5]^2 with transmissive
    boundaries.  Draw order per problem: grid, N, then quadrants 1..4 x (rho, u, v, p)
    with rho, p ~ U[0.1, 2] and u, v ~ U[-1, 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        g = int(grids[rng.integers(len(grids))])
        N = int(degrees[rng.integers(len(degrees))])
        states = []
        for _ in range(4):
            rho = rng.uniform(0.1, 2.0)
            u = rng.uniform(-1.0, 1.0)
            v = rng.uniform(-1.0, 1.0)
            p = rng.uniform(0.1, 2.0)
            states.append((rho, u, v, p))
        out.append(Workload(f"quadrant{i}", 2, N, (g, g), (-0.5, -0.5), (0.5, 0.5),
                            [(BC.simple(TRANSMISSIVE), BC.simple(TRANSMISSIVE))] * 2,
                            quadrant_ic(states), t_end=0.25))
    return out


# ------------------------------------------------------------ shock tubes
SHOCK_TUBES = {  # Table 1: left (rho, u, p), right (rho, u, p), t_final
    "sod": ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 0.2),
    "lax": ((0.445, 0.698, 3.528), (0.5, 0.0, 0.571), 0.14),
}



def periodic_quadrant(n: int = 24, N: int = 3, index: int = 0) -> Workload:
    """A four-quadrant Riemann problem of quadrant_batch on an n x n periodic grid:
    discontinuities on a periodic domain, where mass, momentum and energy are conserved
    exactly by the scheme."""
    wl = quadrant_batch(max(8, index + 1))[index]
    wl.ncell = (n, n)
    wl.N = N
    wl.cfl = STABLE_CFL[N - 1]
    wl.bcs = [(BC.simple(PERIODIC), BC.simple(PERIODIC))] * 2
    return wl

def shock_tube(name: str = "sod", nx: int = 20, ny: int = 5, N: int = 9, gamma: float = 1.4) -> Workload:
    """Sec. 5 shock tubes on [0,1]x[-0.5,0.5], discontinuity at x = 0.5, Dirichlet in x
    (the constant left/right states), periodic in y."""
    (rl, ul, pl), (rr, ur, pr), tf = SHOCK_TUBES[name]

    def ic(x, t=0.0):
        X, Y = x[0], x[1]
        left = X < 0.5
        rho = np.where(left, rl, rr) + 0.0 * Y
        u = np.where(left, ul, ur) + 0.0 * Y
        p = np.where(left, pl, pr) + 0.0 * Y
        return prim_to_cons(gamma, rho, [u, 0.0 * u], p)

    cl = _cons_tuple(gamma, (rl, ul, 0.0, pl))
    cr = _cons_tuple(gamma, (rr, ur, 0.0, pr))
    return Workload(name, 2, N, (nx, ny), (0.0, -0.5), (1.0, 0.5),
                    [(BC.simple(DIRICHLET, cl), BC.simple(DIRICHLET, cr)),
                     (BC.simple(PERIODIC), BC.simple(PERIODIC))], ic, t_end=tf)


# ------------------------------------------------------------ contact wave
def contact_wave_ic(coef: np.ndarray, vel: Sequence[float], p0: float = 1.0, gamma: float = 1.4):
    """rho(x, t) = poly(x - vel t) with constant velocity and pressure: an exact Euler
    solution (a contact wave).  coef[i, j(, k)] multiplies x^i y^j (z^k)."""
    coef = np.asarray(coef, dtype=np.float64)
    dim = coef.ndim

    def ic(x, t=0.0):
        xs = [x[k] - vel[k] * t for k in range(dim)]
        rho = 0.0
        for idx in zip(*np.nonzero(coef)):
            term = coef[idx]
            for k in range(dim):
                term = term * xs[k] ** idx[k]
            rho = rho + term
        shape = np.broadcast_shapes(*[np.shape(a) for a in xs])
        rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), shape)
        return prim_to_cons(gamma, rho, [np.full(shape, vel[k]) for k in range(dim)], np.full(shape, p0))
    return ic


def random_total_degree_poly(dim: int, N: int, seed: int, base: float = 2.0, amp: float = 0.2) -> np.ndarray:
    """Random polynomial of total degree <= N, positive on [0,1]^dim for the given
    amplitude (constant term ``base``, other coefficients ~ amp * U[-1,1] / (deg!))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    coef = np.zeros((N + 1,) * dim)
    for idx in np.ndindex(*coef.shape):
        deg = sum(idx)
        if deg == 0:
            coef[idx] = base
        elif deg <= N:
            coef[idx] = amp * rng.uniform(-1, 1) / math.factorial(deg)
    return coef


def contact_wave(dim: int = 2, N: int = 3, n: int = 4, vel=(0.7, -0.4, 0.3), seed: int = 7) -> Workload:
    coef = random_total_degree_poly(dim, N, seed)
    return Workload("contact", dim, N, (n,) * dim, (0.0,) * dim, (1.0,) * dim,
                    [(BC.simple(TRANSMISSIVE), BC.simple(TRANSMISSIVE))] * dim,
                    contact_wave_ic(coef, vel[:dim]), t_end=0.0)


def random_mask(ncell: int, fraction: float, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.uniform(size=ncell) < fraction).astype(np.uint8)
