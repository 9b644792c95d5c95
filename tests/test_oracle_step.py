"""Pins of the oracle's full step against what the paper and the mathematics fix.

* polynomial reproduction: a contact wave with a total-degree-N density is an exact
  Euler solution inside the scheme's space; predictor (Sec. 2.2) and unlimited corrector
  (Sec. 2.3) reproduce it to round-off;
* conservation of mass, momentum and energy with any mix of troubled cells (Sec. 4.4:
  flux correction of the unlimited neighbours);
* mirror symmetry of the explosion problems;
* order N+1 on the smooth vortex (Sec. 2.4 end, Sec. 5 Table 2);
* shock tubes against the exact Riemann solution (Sec. 5, Table 1);
* the detection logic on hand-built data (Sec. 4.3, eqs. (positivity), (relax), (dmp)).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1406_7416_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def cell_weights(o):
    xi, w, *_ = O.basis(o.n)
    Wt = w
    for _ in range(o.dim - 1):
        Wt = np.multiply.outer(w, Wt)
    return Wt.ravel()


def totals(o):
    vol = np.prod([(o.wl.hi[k] - o.wl.lo[k]) / o.wl.ncell[k] for k in range(o.dim)])
    return (o.state() * cell_weights(o)).sum(axis=(1, 2)) * vol


def l1_density_error(o, t):
    ue, _ = o.project(lambda x, tt: o.wl.ic(x, t), 0)
    vol = np.prod([(o.wl.hi[k] - o.wl.lo[k]) / o.wl.ncell[k] for k in range(o.dim)])
    return float((np.abs(o.state()[0] - ue[0]) * cell_weights(o)).sum() * vol)


def run_to(o, T):
    t, nsteps, troubled = 0.0, 0, 0
    while t < T - 1e-12:
        dt = min(o.cfl_dt(), T - t)
        troubled += o.step(dt)
        t += dt
        nsteps += 1
    return nsteps, troubled


@pytest.mark.parametrize("dim,N", [(2, 1), (2, 2), (2, 3), (2, 5), (2, 9), (3, 1), (3, 2), (3, 3)])
def test_contact_wave_reproduced_exactly(dim, N):
    wl = W.contact_wave(dim=dim, N=N, n=3 if dim == 2 else 2, seed=dim * 10 + N)
    o = O.Oracle(wl, limiter=False)
    u, _ = o.project(wl.ic, 0)
    o.set_state(u)
    dt = o.cfl_dt()
    o.step(dt)
    ue, _ = o.project(lambda x, t: wl.ic(x, dt), 0)
    assert np.abs(o.state() - ue).max() < 2e-13 * max(1, N * N)


@pytest.mark.parametrize("N", [2, 3, 5])
def test_predictor_exact_on_space_time_polynomial(N):
    """The local space-time predictor of eq. (pde.nc.dg2) equals the exact space-time
    solution at its nodes for a total-degree-N contact wave."""
    wl = W.contact_wave(dim=2, N=N, n=1, seed=N)
    o = O.Oracle(wl, limiter=False)
    u, _ = o.project(wl.ic, 0)
    o.set_state(u)
    dt = 0.3 * o.cfl_dt()
    q = O.predictor(2, N, wl.gamma, [dt, dt], N + 1, np.ascontiguousarray(u[:, 0, :]))
    xi, *_ = O.basis(N + 1)
    for s in range(N + 1):
        ue, _ = o.project(lambda x, t: wl.ic(x, xi[s] * dt), 0)
        assert np.abs(q[:, s, :] - ue[:, 0, :]).max() < 1e-12


def test_picard_converges_in_n_sweeps():
    """reading S1: N+1 Picard sweeps reach the fixed point of eq. (pde.nc.dg2) to
    round-off at the time step used (each sweep gains one order in dt)."""
    N = 9
    wl = W.vortex(8, N)
    o = O.Oracle(wl, limiter=False)
    o.init(m=0, detect=False)
    ucell = np.ascontiguousarray(o.state()[:, 27, :])
    dth = [o.cfl_dt() / 1.25] * 2
    q10 = O.predictor(2, N, 1.4, dth, N + 1, ucell)
    q60 = O.predictor(2, N, 1.4, dth, 60, ucell)
    assert np.abs(q10 - q60).max() < 1e-13


@pytest.mark.parametrize("N", [2, 3])
def test_conservation_with_forced_troubled_cells_2d(N):
    wl = W.vortex(8, N)
    o = O.Oracle(wl)
    o.init()
    m0 = totals(o)
    for i in range(3):
        o.force_troubled(W.random_mask(o.ncell, 0.3, seed=i))
        c = o.step(o.cfl_dt())
        assert c >= 1
        assert np.abs(totals(o) - m0).max() < 1e-13 * np.abs(m0).max()


def _periodic_smooth_3d():
    def ic(x, t=0.0):
        rho = 1 + 0.2 * np.sin(2 * np.pi * x[0]) * np.cos(2 * np.pi * x[1]) + 0 * x[2]
        p = 1 + 0.1 * np.cos(2 * np.pi * x[2]) + 0 * x[0]
        z = 0 * x[0] + 0 * x[1] + 0 * x[2]
        return W.prim_to_cons(1.4, rho, [0.3 + z, 0.2 + z, -0.1 + z], p)
    return W.Workload("smooth3d", 3, 2, (4, 4, 4), (0.0,) * 3, (1.0,) * 3,
                      [(W.BC.simple(W.PERIODIC), W.BC.simple(W.PERIODIC))] * 3, ic)


def test_conservation_with_forced_troubled_cells_3d():
    o = O.Oracle(_periodic_smooth_3d())
    o.init()
    m0 = totals(o)
    o.force_troubled(W.random_mask(o.ncell, 0.4, seed=5))
    for _ in range(2):
        o.step(o.cfl_dt())
        assert np.abs(totals(o) - m0).max() < 1e-13 * np.abs(m0).max()


def test_explosion_2d_mirror_symmetry_and_positivity():
    n, N = 20, 3
    o = O.Oracle(W.explosion_2d(n, N))
    o.init()
    for _ in range(8):
        o.step(o.cfl_dt())
    u = o.state().reshape(4, n, n, N + 1, N + 1)     # v, cy, cx, ay, ax
    rho = u[0].transpose(0, 2, 1, 3).reshape(n * (N + 1), n * (N + 1))
    mx = u[1].transpose(0, 2, 1, 3).reshape(rho.shape)
    assert np.abs(rho - rho[:, ::-1]).max() < 1e-12
    assert np.abs(rho - rho[::-1, :]).max() < 1e-12
    assert np.abs(mx + mx[:, ::-1]).max() < 1e-12      # x-momentum is odd under x -> -x
    b = o.troubled().reshape(n, n)
    assert (b == b[:, ::-1]).all() and (b == b[::-1, :]).all() and b.sum() > 0
    # every accepted state is physical at the nodes and on the subcells
    assert (u[0] > 0).all()
    p = 0.4 * (u[3] - 0.5 * (u[1] ** 2 + u[2] ** 2) / u[0])
    assert (p > 0).all()
    assert o.nonphysical() == 0


def test_explosion_3d_mirror_symmetry():
    n, N = 6, 2
    o = O.Oracle(W.explosion_3d(n, N))
    o.init()
    for _ in range(3):
        o.step(o.cfl_dt())
    u = o.state().reshape(5, n, n, n, N + 1, N + 1, N + 1)  # v cz cy cx az ay ax
    rho = u[0].transpose(0, 3, 1, 4, 2, 5).reshape((n * (N + 1),) * 3)  # z y x
    for ax in range(3):
        assert np.abs(rho - np.flip(rho, axis=ax)).max() < 1e-12
    b = o.troubled().reshape(n, n, n)
    for ax in range(3):
        assert (b == np.flip(b, axis=ax)).all()


def _lagrange_matrix(xi, x):
    M = np.ones((len(x), len(xi)))
    for b in range(len(xi)):
        for m in range(len(xi)):
            if m != b:
                M[:, b] *= (x - xi[m]) / (xi[b] - xi[m])
    return M


def l1_density_error_true(o, t):
    """L1 norm of the density error with the DG polynomial evaluated at (N+3)-point GL
    points of every cell (not at its own nodes, where the error superconverges)."""
    n, g = o.n, o.wl.ncell[0]
    xi, *_ = O.basis(n)
    xq, wq, *_ = O.basis(n + 3)
    M = _lagrange_matrix(xi, xq)
    h = (o.wl.hi[0] - o.wl.lo[0]) / g
    u = o.state()[0].reshape(g, g, n, n)
    uq = np.einsum("qa,rb,yxba->yxrq", M, M, u)
    ax = np.concatenate([o.wl.lo[0] + h * (i + xq) for i in range(g)])
    ex = W.sample_grid(lambda x, tt: o.wl.ic(x, t), [ax, ax])[0].reshape(g, n + 3, g, n + 3).transpose(0, 2, 1, 3)
    return float((np.abs(uq - ex) * wq[None, None, :, None] * wq[None, None, None, :]).sum() * h * h)


def _linear_wave(N, g):
    def ic(x, t=0.0):
        rho = 1 + 0.2 * np.sin(2 * np.pi * (x[0] - t) / 10) * np.cos(2 * np.pi * (x[1] - 0.5 * t) / 10)
        return W.prim_to_cons(1.4, rho, [1.0 + 0 * rho, 0.5 + 0 * rho], 1.0 + 0 * rho)
    return W.Workload("wave", 2, N, (g, g), (0, 0), (10, 10),
                      [(W.BC.simple(W.PERIODIC), W.BC.simple(W.PERIODIC))] * 2, ic)


@pytest.mark.parametrize("case,N,grids,flux", [("vortex", 3, (8, 16), 0), ("vortex", 4, (8, 16), 0),
                                               ("wave", 2, (32, 64), 0), ("vortex", 3, (8, 16), 1)])
def test_order_of_accuracy_unlimited(case, N, grids, flux):
    """Order N+1 for smooth solutions (end of Sec. 2.4; Table 2 of Sec. 5), with the Rusanov
    flux and with the Osher-type flux the paper's vortex runs use (Sec. 5)."""
    errs = []
    for g in grids:
        wl = W.vortex(g, N) if case == "vortex" else _linear_wave(N, g)
        o = O.Oracle(wl, limiter=False, flux=flux)
        o.init(m=0, detect=False)
        run_to(o, 1.0)
        errs.append(l1_density_error_true(o, 1.0))
    order = math.log2(errs[0] / errs[1])
    assert order > N + 1 - 0.25, (errs, order)
    if case == "vortex":
        table2 = json.load(open(os.path.join(GOLDEN, "table2_vortex_orders.json")))["rows"]
        assert order > min(table2[str(N)]["order"]) - 0.5


def test_vortex_limiter_idle_when_resolved():
    """Sec. 5 (smooth vortex): on a fine enough mesh the limiter should not act."""
    for g, N in ((16, 5), (8, 9)):
        o = O.Oracle(W.vortex(g, N))
        assert o.init(m=0) == 0
        troubled = sum(o.step(o.cfl_dt()) for _ in range(20))
        assert troubled == 0


def test_sod_against_exact_riemann_solution():
    wl = W.shock_tube("sod", nx=20, ny=2, N=5)
    o = O.Oracle(wl)
    o.init()
    run_to(o, wl.t_end)
    (rl, ul, pl), (rr, ur, pr), tf = W.SHOCK_TUBES["sod"]
    xi, w, *_ = O.basis(wl.N + 1)
    xs = o.axis_points(0, 0)
    exact, _ = O.exact_riemann((rl, ul, pl), (rr, ur, pr), 1.4, (xs - 0.5) / tf)
    u = o.state().reshape(4, 2, 20, wl.N + 1, wl.N + 1)[0, 0]      # cy=0: cx, ay, ax
    rho_x = (u * w[None, :, None]).sum(axis=1).ravel()             # y-average per x node
    err = np.abs(rho_x - exact[:, 0])
    l1 = float((err.reshape(20, wl.N + 1) * w).sum() / 20)
    assert l1 < 0.02, l1
    assert o.nonphysical() == 0
    # away from the waves' cells the solution matches the exact states closely
    far = (np.abs(xs - 0.5) > 0.45)
    assert err[far].max() < 1e-3


def test_initial_detection_logic():
    """eqs. (positivity), (relax), (dmp) on hand-built data, via the initial detection:
    candidate = P(u0), bounds from the supplied exact subcell averages."""
    wl = W.Workload("const", 2, 2, (5, 5), (0, 0), (1, 1),
                    [(W.BC.simple(W.PERIODIC), W.BC.simple(W.PERIODIC))] * 2,
                    lambda x, t=0.0: W.prim_to_cons(1.4, 1.0 + 0 * x[0] + 0 * x[1],
                                                    [0 * x[0], 0 * x[1]], 1.0 + 0 * x[0]))
    o = O.Oracle(wl)
    u, v = o.project(wl.ic, 3)
    rng = np.random.default_rng(0)
    # round-off noise on a constant state passes thanks to delta0 (reading S5)
    assert o.set_state(u + 1e-12 * rng.normal(size=u.shape), v) == 0
    # an overshoot of 2 delta in one cell fails the DMP of that cell only
    u2 = u.copy()
    u2[0, 12, :] += 2e-4
    assert o.set_state(u2, v) == 1 and o.troubled()[12] == 1
    # an overshoot below delta passes
    u3 = u.copy()
    u3[0, 12, :] += 0.5e-4
    assert o.set_state(u3, v) == 0
    # negative density fails PAD even with bounds widened to contain it
    v4 = v.copy()
    v4[0, 7, :] = -1.0
    u4 = u.copy()
    u4[0, 12, :] = -1e-12
    assert o.set_state(u4, v4) >= 1 and o.troubled()[12] == 1
    # a non-finite candidate is troubled
    u5 = u.copy()
    u5[3, 3, 0] = np.nan
    assert o.set_state(u5, v) == 1 and o.troubled()[3] == 1


def test_exact_riemann_solver_pins():
    """Star state of the textbook solver checked by the Rankine-Hugoniot jump conditions
    across the shock and the Riemann invariants across the rarefaction."""
    g = 1.4
    left, right = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    s = np.linspace(-2, 2, 4001)
    out, (ps, us) = O.exact_riemann(left, right, g, s)
    # rarefaction: isentropic, u + 2c/(g-1) constant
    cl = math.sqrt(g * left[2] / left[0])
    rho_sl = left[0] * (ps / left[2]) ** (1 / g)
    csl = math.sqrt(g * ps / rho_sl)
    assert abs((us + 2 * csl / (g - 1)) - (left[1] + 2 * cl / (g - 1))) < 1e-12
    # shock: mass, momentum, energy fluxes balance in the shock frame
    rr, ur, pr = right
    rho_sr = rr * ((ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1))
    S = (rho_sr * us - rr * ur) / (rho_sr - rr)
    def fl(r, u, p):
        E = p / (g - 1) + 0.5 * r * u * u
        return np.array([r * (u - S), r * u * (u - S) + p, E * (u - S) + p * u])
    assert np.abs(fl(rho_sr, us, ps) - fl(rr, ur, pr)).max() < 1e-12
    # sampled solution: far states and monotone density for Sod
    assert np.allclose(out[0], [1.0, 0.0, 1.0]) and np.allclose(out[-1], [0.125, 0.0, 0.1])
    assert (np.diff(out[:, 0]) <= 1e-12).all()


def test_double_mach_post_shock_state_is_rankine_hugoniot():
    """reading S18: a Mach 10 shock into rho=1.4, p=1 (c=1) at rest: the normal
    Rankine-Hugoniot relations give rho=8, p=116.5, |u|=8.25."""
    g, M = 1.4, 10.0
    pre, post = W.dmr_states(g)
    rho1, p1 = pre[0], pre[3]
    c1 = math.sqrt(g * p1 / rho1)
    rho2 = rho1 * (g + 1) * M ** 2 / ((g - 1) * M ** 2 + 2)
    p2 = p1 * (2 * g * M ** 2 - (g - 1)) / (g + 1)
    u2 = M * c1 * (1 - rho1 / rho2)
    assert abs(post[0] - rho2) < 1e-12 and abs(post[3] - p2) < 1e-12
    assert abs(math.hypot(post[1], post[2]) - u2) < 1e-12


@pytest.mark.parametrize("var,value", [(0, float("nan")), (0, -0.5), (3, 50.0)])
def test_poisoned_candidate_equals_forced_troubled_cell(var, value):
    """Sec. 4.3-4.4: the detection acts on the unlimited candidate only.  A candidate made
    non-finite, non-positive or far outside the relaxed DMP bounds flags its cell, and the
    step then equals, bit for bit, the step with that cell forced troubled: the troubled
    cell's candidate is discarded, and no other cell's candidate or bounds depend on it."""
    wl = W.vortex(8, 9)          # resolved: the limiter stays idle without the poison
    cell = 27
    u0, _ = O.Oracle(wl).project(wl.ic, 0)
    runs = {}
    for mode in ("plain", "poison", "force"):
        o = O.Oracle(wl)
        o.set_state(u0)
        dt = o.cfl_dt()
        if mode == "poison":
            o.poison(cell, var, value)
        if mode == "force":
            m = np.zeros(wl.num_cells, dtype=np.uint8)
            m[cell] = 1
            o.force_troubled(m)
        o.step(dt)
        runs[mode] = (o.state(), o.troubled())
        if mode == "poison":
            # one step only: the next step is unpoisoned and the cell goes back to DG
            o.step(dt)
            assert o.troubled()[cell] == 0
    assert runs["plain"][1].sum() == 0
    assert runs["poison"][1][cell] == 1 and runs["poison"][1].sum() == 1
    assert np.array_equal(runs["poison"][1], runs["force"][1])
    assert np.array_equal(runs["poison"][0], runs["force"][0])
    assert np.isfinite(runs["poison"][0]).all()


def test_mood_layer_conserves_and_is_active():
    """MOOD layer after the subcell WENO3 scheme (Sec. 6, Fig. algo2): with first-order
    fluxes on the sub-faces next to flagged subcells, adjacent troubled cells still agree
    on every shared sub-face, so the step stays conservative to round-off; the layer acts
    (flags, recomputed cells) and every result stays physical."""
    wl = W.periodic_quadrant()
    o = O.Oracle(wl, mood=True)
    o.init()
    m0 = totals(o)
    flagged = 0
    for i in range(4):
        o.step(o.cfl_dt())
        f, r = o.mood_stats()
        flagged += f
        assert r <= o.troubled().sum()
        assert np.abs(totals(o) - m0).max() < 1e-13 * np.abs(m0).max()
    assert flagged > 0 and o.nonphysical() == 0
    u = o.state()
    assert np.isfinite(u).all()


def test_mood_layer_changes_nothing_without_flags():
    """On data whose WENO3 candidates pass the detection the layer flags nothing and the
    step is bit for bit the one without it."""
    wl = W.vortex(8, 9)
    mask = W.random_mask(wl.num_cells, 0.3, seed=5)
    out = []
    for mood in (False, True):
        o = O.Oracle(wl, mood=mood)
        o.init(m=0, detect=False)
        o.force_troubled(mask)
        o.step(o.cfl_dt())
        out.append(o.state())
        if mood:
            assert o.mood_stats() == (0, 0)
    assert np.array_equal(out[0], out[1])


def test_mood_first_order_fluxes_where_flagged():
    """Where the layer acts the result differs from the plain subcell scheme and only in
    troubled cells and their face neighbours (the flux correction)."""
    wl = W.periodic_quadrant()
    states = []
    for mood in (False, True):
        o = O.Oracle(wl, mood=mood)
        o.init()
        o.step(o.cfl_dt())
        states.append((o.state(), o.troubled()))
    (ua, ba), (ub, bb) = states
    assert np.array_equal(ba, bb)
    diff = np.abs(ua - ub).max(axis=(0, 2)) > 0
    assert diff.any()
    nx, ny = wl.ncell
    t = ba.reshape(ny, nx).astype(bool)
    near = t | np.roll(t, 1, 0) | np.roll(t, -1, 0) | np.roll(t, 1, 1) | np.roll(t, -1, 1)
    assert not (diff.reshape(ny, nx) & ~near).any()


def test_osher_scheme_contact_wave_and_conservation():
    """With the Osher-type flux the step still reproduces the contact wave exactly and stays
    conservative with troubled cells on discontinuous periodic data."""
    wl = W.contact_wave(dim=2, N=3, n=3, seed=3)
    o = O.Oracle(wl, limiter=False, flux=1)
    o.init(m=0, detect=False)
    dt = o.cfl_dt()
    o.step(dt)
    ue, _ = o.project(lambda x, t: wl.ic(x, dt), 0)
    assert np.abs(o.state() - ue).max() < 1e-12
    wl = W.periodic_quadrant(16, 3)
    o = O.Oracle(wl, flux=1)
    o.init()
    m0 = totals(o)
    for i in range(3):
        o.force_troubled(W.random_mask(o.ncell, 0.2, seed=i))
        o.step(o.cfl_dt())
        assert np.abs(totals(o) - m0).max() < 1e-13 * np.abs(m0).max()
    assert np.isfinite(o.state()).all()


def test_one_step_depends_on_two_cells_around():
    """Locality of one limited step (Sec. 4: the detection of a cell needs its candidate and
    the old data of its 3^d block; a troubled cell's subcell scheme needs its neighbours'
    old data; an unlimited cell's faces need the troubled status of its face neighbours):
    a box cut out of a larger grid, stepped with its own transmissive sides, agrees exactly
    with the larger grid on every cell at least three cells inside the box.  The 3D
    explosion at full size is checked on the GPU through such boxes."""
    nc, N, wn, origin = 18, 3, 12, (6, 3, 3)
    h = 2.0 / nc
    dt = W.stable_cfl(N) * h / (3 * (2 * N + 1) * math.sqrt(1.4))

    def stepped(wl):
        o = O.Oracle(wl)
        o.set_state(o.project(wl.ic, 0)[0], o.project(wl.ic, 1)[1])
        o.step(dt)
        return o

    full = stepped(W.explosion_3d(nc, N))
    lo = tuple(-1.0 + i * h for i in origin)
    bc = (W.BC.simple(W.TRANSMISSIVE), W.BC.simple(W.TRANSMISSIVE))
    box = stepped(W.Workload("box", 3, N, (wn,) * 3, lo, tuple(x + wn * h for x in lo), [bc] * 3, W.explosion_ic(3)))
    i = np.arange(wn)
    z, y, x = np.meshgrid(i + origin[2], i + origin[1], i + origin[0], indexing="ij")
    cells = (x + nc * (y + nc * z)).ravel()
    for depth, exact in ((0, False), (3, True)):
        ok = (i >= depth) & (i < wn - depth)
        m = (ok[:, None, None] & ok[None, :, None] & ok[None, None, :]).ravel()
        same = np.array_equal(box.state()[:, m], full.state()[:, cells[m]]) and \
            np.array_equal(box.troubled()[m], full.troubled()[cells[m]])
        assert same == exact
    ok = (i >= 3) & (i < wn - 3)
    m = (ok[:, None, None] & ok[None, :, None] & ok[None, None, :]).ravel()
    assert box.troubled()[m].sum() > 0
