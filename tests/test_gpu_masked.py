"""Masked geometry on the GPU (Sec. 5, forward-facing step: a rectangle removed from the
domain, its faces reflective walls) against the FP64 oracle, which carries the same
reading of the walls (pinned on the CPU: a solid half-domain equals a reflective domain
boundary, the corner image keeps the diagonal symmetry, walls conserve mass and energy).

Tolerances as in the unmasked parity tests: FP64 form 1e-12 relative per variable after
the first step and 1e-10 after several, identical troubled maps; the batch path bitwise
equal to the per-problem path.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1406_7416_amd import workloads as W
from test_gpu_parity import rel_err, run_parity
from test_oracle_masked import _corner, _slab_ic

pytestmark = pytest.mark.gpu


def masked_pair(wl, mask, precision="fp64", m=None):
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_1406_7416_amd import adg
    o = O.Oracle(wl)
    o.set_mask(mask)
    u, v = o.project(wl.ic, wl.N + 1 if m is None else m)
    o.set_state(u, v)
    g = adg.Problem(wl, precision=adg.ADG_MIXED if precision == "mixed" else adg.ADG_FP64)
    g.set_mask(mask)
    g.set_state(u, v)
    return o, g


def test_forward_facing_step_against_oracle():
    """The coarse forward-facing step (Mach 3 onto the step; the bow shock forms at its
    face and the limiter acts along it and at the corner)."""
    wl = W.forward_facing_step(60, 20, 3)
    mask = W.step_mask(wl)
    o, g = masked_pair(wl, mask)
    u0 = g.state()
    flagged = 0
    for s in range(8):
        dt = o.cfl_dt()
        assert abs(g.cfl_dt(wl.cfl) - dt) <= 1e-13 * dt
        flagged += o.step(dt)
        g.step(dt)
        assert np.array_equal(g.troubled(), o.troubled()), f"step {s}"
        e = rel_err(g.state(), o.state())
        assert e < (1e-12 if s == 0 else 1e-10), f"step {s}: rel err {e}"
    assert flagged > 0
    assert np.array_equal(g.state()[:, mask == 1], u0[:, mask == 1])   # solid cells keep their state
    assert g.stats()["nonphysical"] == 0


def test_forward_facing_step_mixed_precision():
    """Mixed form (FP32 predictor, fluxes and increments).  Away from the step the flow is
    uniform and its exact increment is zero, so the FP32 rounding of the fluxes (of the
    size of the state times the wave speed) shows against the state's overall scale, not
    against the variable's own (the transverse momentum is zero there): the bound is 2e-6
    of the largest state magnitude per step."""
    wl = W.forward_facing_step(60, 20, 3)
    mask = W.step_mask(wl)
    o, g = masked_pair(wl, mask, precision="mixed")
    worst = 0.0
    for s in range(4):
        dt = o.cfl_dt()
        o.step(dt)
        g.step(dt)
        diff = np.nonzero(o.troubled() != g.troubled())[0]
        assert np.all(np.abs(o.margin()[diff]) < 1e-4), f"step {s}: flags differ away from the margin"
        if len(diff):
            break
        uo = o.state()
        e = np.abs(g.state() - uo).max() / np.abs(uo).max()
        worst = max(worst, e)
        assert e < 2e-6, f"step {s}: {e}"
    assert worst > 0


def test_corner_explosion_against_oracle():
    """A blast next to the convex corner of a solid square: the subcell halo, the sub-face
    walls and the neighbourhood bounds all read the corner image."""
    wl, mask = _corner(n=12, N=3)
    o, g = masked_pair(wl, mask.ravel())
    run_parity(o, g, 6)
    assert int(g.troubled().sum()) > 0


def test_solid_half_domain_equals_reflective_wall_on_gpu():
    """The GPU path alone: the problem on [-1, 1] with the cells x < 0 solid advances its
    fluid cells like the problem on [0, 1] with a reflective wall at x = 0."""
    import torch
    assert torch.cuda.is_available()
    from paper_1406_7416_amd import adg
    N, nx, ny = 3, 8, 4
    per = (W.BC.simple(W.PERIODIC), W.BC.simple(W.PERIODIC))
    wall = W.Workload("wall", 2, N, (nx, ny), (0.0, 0.0), (1.0, 1.0),
                      [(W.BC.simple(W.REFLECTIVE), W.BC.simple(W.TRANSMISSIVE)), per], _slab_ic(False))
    masked = W.Workload("masked", 2, N, (2 * nx, ny), (-1.0, 0.0), (1.0, 1.0),
                        [(W.BC.simple(W.TRANSMISSIVE), W.BC.simple(W.TRANSMISSIVE)), per], _slab_ic(False))
    mask = np.zeros((ny, 2 * nx), np.uint8)
    mask[:, :nx] = 1
    gw, gm = adg.Problem(wall), adg.Problem(masked)
    gm.set_mask(mask.ravel())
    for g, wl in ((gw, wall), (gm, masked)):
        u, v = g.project(wl.ic, N + 1)
        g.set_state(u, v)
    troubled = 0
    for _ in range(6):
        dt = gw.cfl_dt(0.5)
        assert abs(gm.cfl_dt(0.5) - dt) < 1e-15 * dt
        gw.step(dt)
        gm.step(dt)
        troubled += int(gw.troubled().sum())
    assert troubled > 0
    uw = gw.state().reshape(4, ny, nx, -1)
    um = gm.state().reshape(4, ny, 2 * nx, -1)
    assert np.abs(um[:, :, nx:] - uw).max() < 1e-11 * np.abs(uw).max()
    assert np.array_equal(gm.troubled().reshape(ny, 2 * nx)[:, nx:], gw.troubled().reshape(ny, nx))
    assert not gm.troubled().reshape(ny, 2 * nx)[:, :nx].any()


def test_masked_problem_in_a_batch_equals_stepping_alone():
    import torch
    assert torch.cuda.is_available()
    from paper_1406_7416_amd import adg
    wl = W.forward_facing_step(60, 20, 3)
    mask = W.step_mask(wl)
    others = W.quadrant_batch(2)
    for q in others:
        q.ncell = (16, 16)

    def make(w, msk):
        g = adg.Problem(w, pool_capacity=w.num_cells)
        if msk is not None:
            g.set_mask(msk)
        u, _ = g.project(w.ic, 0)
        g.set_state(u)
        return g

    ref = [make(wl, mask)] + [make(q, None) for q in others]
    bat = [make(wl, mask)] + [make(q, None) for q in others]
    for g in ref:
        for _ in range(4):
            g.step_cfl(0.5)
    b = adg.Batch(bat)
    b.step_cfl(0.5, 4)
    for g1, g2 in zip(ref, bat):
        assert np.array_equal(g1.state(), g2.state())
        assert np.array_equal(g1.troubled(), g2.troubled())
    assert int(ref[0].troubled().sum()) > 0
    with pytest.raises(adg.AdgError, match="-6"):
        bat[0].set_mask(None)
    b.close()


def test_mask_errors():
    import torch
    assert torch.cuda.is_available()
    from paper_1406_7416_amd import adg
    wl = W.forward_facing_step(30, 10, 2)
    g = adg.Problem(wl)
    with pytest.raises(adg.AdgError, match="-1"):
        g.set_mask(np.ones(wl.num_cells, np.uint8))
    g.set_mask(np.zeros(wl.num_cells, np.uint8))   # no solid cell: no mask
    g.set_mask(None)


def test_explosion_3d_with_solid_block_against_oracle():
    """3D: the explosion next to a solid box in one corner of the domain (walls normal to
    all three axes; the box's edges and its corner take the image along two and three
    axes)."""
    wl = W.explosion_3d(8, 2)
    m = np.zeros((8, 8, 8), np.uint8)   # [z][y][x]
    m[:3, :3, :3] = 1
    o, g = masked_pair(wl, m.ravel())
    run_parity(o, g, 3)
    assert int(g.troubled().sum()) > 0
