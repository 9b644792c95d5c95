"""The deviation form of the mixed precision (ADG_MIXED_DEV: the FP32 predictor, traces and
face fluxes carried as deviations from each cell's reference state, the fluxes evaluated as
F(c + dq) - F(c) with every term of the size of dq) against the FP64 oracle, and its accuracy
on the smooth isentropic vortex, where the plain mixed form's FP32 rounding of whole states
sets its error (it grows with refinement there).

Tolerances: per step as the plain mixed form (2e-6 of each variable's scale; troubled maps may
differ only where the oracle's detection margin is below 1e-4).  Whole runs: FP32 rounding is
now relative to the deviation of the state within a cell, which shrinks like h, while the
number of steps to t = 10 grows like 1/h: the accumulated rounding falls like h^(1/2) (measured
to t = 10 on the N = 9 vortex: 3.4e-6, 2.5e-6, 1.8e-6 on 16^2, 32^2, 64^2 against the plain
mixed form's 9.3e-5, 1.4e-4, 2.1e-4, which grow), far above the FP64 form's discretisation
error (4.7e-8 .. 1.3e-9) at this order.  Bounds: relative L1 against the oracle's density at
t = 10 below 1e-7 (measured 3.5e-8; the plain mixed form 9.4e-7), errors against the exact
vortex falling with the mesh and below 1e-5.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1406_7416_amd import workloads as W
from test_gpu_end_to_end_l1 import GOLDEN, l1
from test_gpu_mixed import run_mixed

pytestmark = pytest.mark.gpu


def paired_dev(wl, m=None, detect=True, force=None, mask=None):
    import torch
    assert torch.cuda.is_available()
    from paper_1406_7416_amd import adg
    o = O.Oracle(wl)
    g = adg.Problem(wl, precision=adg.ADG_MIXED_DEV)
    if mask is not None:
        o.set_mask(mask)
        g.set_mask(mask)
    u, v = o.project(wl.ic, wl.N + 1 if m is None else m)
    o.set_state(u, v if detect else None)
    g.set_state(u, v if detect else None)
    if force is not None:
        o.force_troubled(force)
        g.force_troubled(force)
    return o, g


@pytest.mark.parametrize("N,n", [(9, 8), (5, 10), (3, 16)])
def test_dev_vortex(N, n):
    o, g = paired_dev(W.vortex(n, N), m=0)
    worst, _ = run_mixed(o, g, 4)
    assert worst > 0


def test_dev_explosion_with_limiter():
    o, g = paired_dev(W.explosion_2d(24, 3))
    _, done = run_mixed(o, g, 6)
    assert int(o.troubled().sum()) > 0 and done >= 3


def test_dev_forced_troubled_flux_correction_and_conservation():
    """Every third cell forced troubled: the flux correction of the unlimited neighbours
    converts their deviation-form face fluxes back to full fluxes; mass and energy stay
    conserved on the periodic vortex (to the FP32 rounding of the deviation increments)."""
    wl = W.vortex(12, 4)
    force = np.zeros(wl.num_cells, np.uint8)
    force[::3] = 1
    o, g = paired_dev(wl, m=0, detect=False, force=force)
    xi, w, *_ = O.basis(wl.N + 1)
    Wc = np.multiply.outer(w, w).ravel()
    tot0 = (g.state() * Wc).sum(axis=(1, 2))
    run_mixed(o, g, 3)
    tot1 = (g.state() * Wc).sum(axis=(1, 2))
    drift = [abs(tot1[v] - tot0[v]) / abs(tot0[v]) for v in (0, 3)]
    print(f"deviation form, 3 steps with forced troubled cells: relative drift of mass {drift[0]:.1e}, "
          f"energy {drift[1]:.1e}", flush=True)
    # the increments of both cells at a face are rounded in FP32 separately (as in the plain
    # mixed form, where they have the size of the flux, here of its deviation)
    assert max(drift) < 1e-9


def test_dev_double_mach_boundaries():
    """Dirichlet inflow, reflective wall and the moving exact shock on the top: the ghost
    states formed from the full FP64 trace and taken relative to the cell's reference."""
    o, g = paired_dev(W.double_mach(40, 10, 3))
    run_mixed(o, g, 4)


def test_dev_forward_facing_step_walls():
    wl = W.forward_facing_step(60, 20, 3)
    o, g = paired_dev(wl, mask=W.step_mask(wl))
    worst = 0.0
    for s in range(4):
        dt = o.cfl_dt()
        o.step(dt)
        g.step(dt)
        diff = np.nonzero(o.troubled() != g.troubled())[0]
        assert np.all(np.abs(o.margin()[diff]) < 1e-4), f"step {s}"
        if len(diff):
            break
        uo = o.state()
        e = np.abs(g.state() - uo).max() / np.abs(uo).max()
        worst = max(worst, e)
        assert e < 2e-6, f"step {s}: {e}"


def test_dev_explosion_3d():
    o, g = paired_dev(W.explosion_3d(10, 2))
    run_mixed(o, g, 3)


def test_dev_batch_equals_individual_steps():
    from paper_1406_7416_amd import adg
    wls = W.quadrant_batch(4)
    for i, wl in enumerate(wls):
        wl.ncell = (16 + 4 * i, 12 + 2 * i)

    def make(wl):
        p = adg.Problem(wl, precision=adg.ADG_MIXED_DEV, pool_capacity=wl.num_cells)
        u, _ = p.project(wl.ic, 0)
        p.set_state(u)
        return p

    ref = [make(wl) for wl in wls]
    bat = [make(wl) for wl in wls]
    for p in ref:
        for _ in range(4):
            p.step_cfl(0.5)
    b = adg.Batch(bat)
    b.step_cfl(0.5, 4)
    for p1, p2 in zip(ref, bat):
        assert np.array_equal(p1.state(), p2.state())
    b.close()


def test_dev_rejects_osher_flux():
    from paper_1406_7416_amd import adg
    with pytest.raises(adg.AdgError, match="-1"):
        adg.Problem(W.vortex(8, 3), precision=adg.ADG_MIXED_DEV, flux=1)


@pytest.mark.timeout(600)
def test_dev_vortex_to_t10_against_oracle():
    from paper_1406_7416_amd import adg
    ro = np.load(GOLDEN)
    wl = W.vortex(16, 9)
    g = adg.Problem(wl, precision=adg.ADG_MIXED_DEV)
    u0, _ = g.project(wl.ic, 0)
    g.set_state(u0)
    while g.time < 10.0 * (1 - 1e-14):
        g.step(min(g.cfl_dt(), 10.0 - g.time))
    e = l1(g.state()[0] - ro, wl) / l1(ro, wl)
    print(f"vortex 16^2 N=9 to t=10, deviation form: relative L1(rho - rho_oracle) {e:.2e}", flush=True)
    g.close()
    assert e < 1e-7


@pytest.mark.timeout(900)
def test_dev_vortex_convergence_matches_fp64():
    """Against the exact vortex at t = 10 on 16^2, 32^2, 64^2 cells (N = 9): the deviation
    form's L1 error falls with the mesh (the plain mixed form's grows)."""
    from paper_1406_7416_amd import adg
    errs = {}
    for form, prec in (("fp64", adg.ADG_FP64), ("dev", adg.ADG_MIXED_DEV)):
        errs[form] = []
        for n in (16, 32, 64):
            wl = W.vortex(n, 9)
            p = adg.Problem(wl, precision=prec)
            u0, _ = p.project(wl.ic, 0)
            p.set_state(u0)
            while p.time < 10.0 * (1 - 1e-14):
                p.step(min(p.cfl_dt(), 10.0 - p.time))
            ue, _ = p.project(lambda x, t: wl.ic(x, 10.0), 0)
            errs[form].append(l1(p.state()[0] - ue[0], wl))
            p.close()
    print(f"vortex N=9 t=10 L1(rho - rho_exact) on 16/32/64: fp64 {errs['fp64']}, deviation form {errs['dev']}",
          flush=True)
    d = errs["dev"]
    assert d[0] > d[1] > d[2]
    assert max(d) < 1e-5
