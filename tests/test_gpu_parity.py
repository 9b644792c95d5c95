"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle, element by
element, on identical seeded inputs.

Tolerance (FP64 form): both sides evaluate the same formulas in double precision with
different summation orders (sum-factorised tensor contractions vs plain sums), so one
step differs by a few units of round-off of the largest contributing terms.  The bound
used is 1e-12 relative to each variable's largest magnitude per step (1e-10 after
several steps), and the troubled-cell maps must be identical.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1406_7416_amd import workloads as W

pytestmark = pytest.mark.gpu


def gpu_problem(wl, **kw):
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_1406_7416_amd import adg
    return adg.Problem(wl, **kw)


def rel_err(a, b):
    """max over variables of max|a-b| / scale_v, scale_v = max|b_v| floored at 1e-3 of the
    largest magnitude of the state (a variable that is zero up to round-off, such as the
    transverse momentum of a 1D problem, is compared at the state's scale)."""
    floor = 1e-3 * np.abs(b).max()
    errs = []
    for v in range(a.shape[0]):
        scale = max(floor, np.abs(b[v]).max(), 1e-300)
        errs.append(np.abs(a[v] - b[v]).max() / scale)
    return max(errs)


def paired(wl, limiter=True, m=None, detect=True, mask=None):
    o = O.Oracle(wl, limiter=limiter)
    if m is None:
        m = wl.N + 1
    u, v = o.project(wl.ic, m)
    o.set_state(u, v if (detect and limiter) else None)
    g = gpu_problem(wl, limiter=limiter)
    g.set_state(u, v if (detect and limiter) else None)
    if mask is not None:
        o.force_troubled(mask)
        g.force_troubled(mask)
    return o, g


def run_parity(o, g, steps, tol_first=1e-12, tol=1e-10, check_beta=True, tol_init=1e-13):
    assert (g.troubled() == o.troubled()).all()
    assert rel_err(g.state(), o.state()) < tol_init
    for s in range(steps):
        dt = o.cfl_dt()
        dtg = g.cfl_dt(o.wl.cfl)
        # (the time step follows the state's largest wave speed: within the state's bound)
        assert abs(dtg - dt) <= max(1e-13, tol_init) * dt
        o.step(dt)
        g.step(dt)
        e = rel_err(g.state(), o.state())
        if check_beta:
            bo, bg = o.troubled(), g.troubled()
            assert (bo == bg).all(), f"step {s}: beta differs in {np.nonzero(bo != bg)[0][:10]}"
        assert e < (tol_first if s == 0 else tol), f"step {s}: rel err {e}"
    assert abs(g.time - o.time) < 1e-14 * max(1.0, o.time)


@pytest.mark.parametrize("dim,N,n", [(2, 3, 3), (2, 9, 2), (3, 2, 2)])
def test_contact_wave_unlimited(dim, N, n):
    wl = W.contact_wave(dim=dim, N=N, n=n, seed=3)
    o, g = paired(wl, limiter=False, m=0)
    dt = o.cfl_dt()
    o.step(dt)
    g.step(dt)
    assert rel_err(g.state(), o.state()) < 1e-12
    ue, _ = o.project(lambda x, t: wl.ic(x, dt), 0)
    assert np.abs(g.state() - ue).max() < 1e-12 * max(1, N * N)


def test_explosion_2d_ragged():
    """Ragged grid (block sizes do not divide it), initial detection, limiter active."""
    wl = W.explosion_2d(20, 3)
    wl.ncell = (19, 13)
    o, g = paired(wl)
    run_parity(o, g, 6)
    assert o.troubled().sum() > 0


@pytest.mark.parametrize("N,n", [(9, 8), (5, 10)])
def test_vortex(N, n):
    o, g = paired(W.vortex(n, N), m=0)
    run_parity(o, g, 3)


@pytest.mark.parametrize("N", [2, 3, 5])
def test_forced_troubled_subcell_path_and_flux_correction(N):
    """A random forced mask drives the subcell ADER-WENO3 recompute, the flux correction
    of unlimited neighbours and the pool across steps on smooth periodic data."""
    wl = W.vortex(8, N)
    o, g = paired(wl, mask=W.random_mask(wl.num_cells, 0.3, seed=N))
    run_parity(o, g, 3)
    assert o.troubled().sum() > 0
    vo, vg = o.subcells(), g.subcells()
    b = o.troubled().astype(bool)
    assert rel_err(vg[:, b], vo[:, b]) < 1e-10


def test_double_mach_small():
    wl = W.double_mach(40, 10, 3)
    o, g = paired(wl)
    run_parity(o, g, 4)


def test_double_mach_window_paper_mesh():
    """Mach-10 shock at the paper's mesh size h = 1/100 with N = 5 on a window of the
    domain (the positivity safeguard of the subcell scheme acts at the shock foot)."""
    wl = W.double_mach(100, 25, 5, Lx=1.0, Ly=0.25)
    o, g = paired(wl)
    run_parity(o, g, 3)
    assert o.nonphysical() == 0 and g.stats()["nonphysical"] == 0


@pytest.mark.parametrize("i", [0, 3])
def test_quadrant_riemann_problem(i):
    wl = W.quadrant_batch(8)[i]
    wl.ncell = (24, 20)
    o, g = paired(wl)
    run_parity(o, g, 3)


def test_sod_tube():
    wl = W.shock_tube("sod", nx=20, ny=2, N=5)
    o, g = paired(wl)
    run_parity(o, g, 5)


def test_explosion_3d_small():
    o, g = paired(W.explosion_3d(6, 2))
    run_parity(o, g, 2)


def test_forced_troubled_3d():
    def ic(x, t=0.0):
        rho = 1 + 0.2 * np.sin(2 * np.pi * x[0]) * np.cos(2 * np.pi * x[1]) + 0 * x[2]
        p = 1 + 0.1 * np.cos(2 * np.pi * x[2]) + 0 * x[0]
        z = 0 * x[0] + 0 * x[1] + 0 * x[2]
        return W.prim_to_cons(1.4, rho, [0.3 + z, 0.2 + z, -0.1 + z], p)
    wl = W.Workload("smooth3d", 3, 3, (4, 5, 3), (0.0,) * 3, (1.0,) * 3,
                    [(W.BC.simple(W.PERIODIC), W.BC.simple(W.PERIODIC))] * 3, ic)
    o, g = paired(wl, mask=W.random_mask(wl.num_cells, 0.4, seed=9))
    run_parity(o, g, 2)


def test_deterministic_bitwise():
    wl = W.explosion_2d(16, 3)
    outs = []
    for _ in range(2):
        o, g = paired(wl)
        for _ in range(4):
            g.step(0.002)
        outs.append((g.state(), g.troubled()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_step_cfl_matches_explicit_dt():
    wl = W.explosion_2d(12, 3)
    _, g1 = paired(wl)
    _, g2 = paired(wl)
    for _ in range(3):
        dt = g1.cfl_dt(wl.cfl)
        g1.step(dt)
        g2.step_cfl(wl.cfl)
    assert np.array_equal(g1.state(), g2.state())
    assert g1.time == g2.time


def test_vortex_full_size_one_step():
    """The benchmark workload (N=9 vortex on 64x64, periodic [0,10]^2) in the launch
    configuration the benchmark times: one step from identical inputs, all outputs."""
    wl = W.vortex(64, 9)
    o, g = paired(wl, m=0)
    run_parity(o, g, 1)
    assert o.troubled().sum() == 0 and g.troubled().sum() == 0


@pytest.mark.parametrize("var,value", [(0, float("nan")), (0, -0.5), (3, 50.0)])
def test_poisoned_candidate(var, value):
    """adg_debug_poison: a corrupted candidate is caught by the a-posteriori detection and
    recomputed by the subcell scheme, as in the oracle; on the GPU the step equals, bit for
    bit, the step with that cell forced troubled, and the poison lasts one step."""
    wl = W.vortex(8, 9)
    cell = 27
    o, g = paired(wl, m=0)
    dt = o.cfl_dt()
    o.poison(cell, var, value)
    g.poison(cell, var, value)
    o.step(dt)
    g.step(dt)
    bo, bg = o.troubled(), g.troubled()
    assert bg[cell] == 1 and bg.sum() == 1 and np.array_equal(bo, bg)
    assert rel_err(g.state(), o.state()) < 1e-12
    _, gf = paired(wl, m=0)
    mask = np.zeros(wl.num_cells, dtype=np.uint8)
    mask[cell] = 1
    gf.force_troubled(mask)
    gf.step(dt)
    assert np.array_equal(g.state(), gf.state())
    g.step(dt)
    assert g.troubled()[cell] == 0
    # the mixed form catches it the same way
    from paper_1406_7416_amd import adg
    gm = gpu_problem(wl, precision=adg.ADG_MIXED)
    gm.set_state(o.project(wl.ic, 0)[0])
    gm.poison(cell, var, value)
    gm.step(dt)
    assert gm.troubled()[cell] == 1 and np.isfinite(gm.state()).all()


def test_config_explosion_2d_full_size():
    """The 2D explosion at its full size (40 x 40, N = 3), initial detection, 5 steps."""
    o, g = paired(W.explosion_2d(40, 3))
    run_parity(o, g, 5)
    assert o.troubled().sum() > 0


def test_config_double_mach_full_size_one_step():
    """The double Mach reflection at its full size (400 x 100 cells on [0,4] x [0,1], N = 5),
    initial detection against one-point subcell averages (exact for its piecewise-constant
    state away from the shock line), one step."""
    o, g = paired(W.double_mach(400, 100, 5), m=1)
    run_parity(o, g, 1)
    assert o.troubled().sum() > 0


def test_config_explosion_3d_16cubed():
    """3D explosion, 16^3 cells, N = 3 (the 3D workload's degree), initial detection against
    one-point subcell averages."""
    o, g = paired(W.explosion_3d(16, 3), m=1)
    run_parity(o, g, 2)
    assert o.troubled().sum() > 0


def test_shock_vortex_small():
    """Shock-vortex interaction (Sec. 5) on a coarse grid, N = 3: standing shock, vortex
    upstream, inflow on the left."""
    o, g = paired(W.shock_vortex(40, 20, 3), m=4)
    run_parity(o, g, 5)
    assert o.troubled().sum() > 0


def test_config_shock_vortex_full_size():
    """Shock-vortex interaction at the paper's mesh size h = 1/100 (200 x 100 cells on
    [0,2] x [0,1], N = 5), initial detection against 3-point subcell averages (exact for the
    uniform states), two steps."""
    o, g = paired(W.shock_vortex(200, 100, 5), m=3)
    run_parity(o, g, 2)
    assert o.troubled().sum() > 0


def test_pool_overflow_is_reported_and_cleared():
    """More troubled cells than the subcell pool holds: the initial detection refuses at
    once; a step that overflows is reported by the following call (the counts stay on the
    device), and a new state clears the error."""
    from paper_1406_7416_amd import adg
    wl = W.explosion_2d(20, 3)
    o = O.Oracle(wl)
    u, v = o.project(wl.ic, wl.N + 1)
    g = gpu_problem(wl, pool_capacity=2)
    with pytest.raises(adg.AdgError, match="-4"):
        g.set_state(u, v)
    g.set_state(u)                  # no initial detection: the first step flags the ring
    o.set_state(u)
    dt = o.cfl_dt()
    g.step(dt)
    assert g.stats()["troubled"] > 2
    with pytest.raises(adg.AdgError, match="-4"):
        g.step(dt)
    with pytest.raises(adg.AdgError, match="-4"):
        g.step(dt)                  # sticky
    # a constant state flags nothing: the error is gone after the new state
    g.set_state(np.ones_like(u) * np.array([1.0, 0.0, 0.0, 2.5])[:, None, None])
    g.step(dt)
    g.step(dt)
    assert g.stats()["troubled"] == 0
