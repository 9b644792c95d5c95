"""Batching: independent problems of different grid size and degree advanced with one
hipGraph launch per batch step give bitwise the same states as the same problems
stepped one by one (the per-problem path is itself checked against the oracle)."""
import numpy as np
import pytest

from paper_1406_7416_amd import workloads as W

pytestmark = pytest.mark.gpu


def make(wl, prec):
    from paper_1406_7416_amd import adg
    g = adg.Problem(wl, precision=prec, pool_capacity=wl.num_cells)
    u, _ = g.project(wl.ic, 0)
    g.set_state(u)
    return g


@pytest.mark.parametrize("prec_name", ["fp64", "mixed"])
def test_batch_equals_individual_steps(prec_name):
    import torch
    assert torch.cuda.is_available()
    from paper_1406_7416_amd import adg
    prec = adg.ADG_MIXED if prec_name == "mixed" else adg.ADG_FP64
    wls = W.quadrant_batch(6)
    for i, wl in enumerate(wls):
        wl.ncell = (16 + 4 * i, 12 + 2 * i)   # uneven grids, small for the test
    wls.append(W.explosion_2d(18, 3))
    ref = [make(wl, prec) for wl in wls]
    bat = [make(wl, prec) for wl in wls]
    steps = 5
    for g, wl in zip(ref, wls):
        for _ in range(steps):
            g.step_cfl(0.5)
    b = adg.Batch(bat)
    b.step_cfl(0.5, 2)
    b.step_cfl(0.5, steps - 2)
    for g1, g2, wl in zip(ref, bat, wls):
        assert np.array_equal(g1.state(), g2.state()), wl.name
        assert np.array_equal(g1.troubled(), g2.troubled()), wl.name
        assert g1.time == g2.time
    assert sum(int(g.troubled().sum()) for g in ref) > 0
    dts = b.dts()
    assert np.all(dts > 0)
    b.close()


def test_batch_reports_pool_overflow_and_locks_its_problems():
    """A problem whose troubled cells exceed its pool makes adg_batch_step_cfl fail with
    ADG_ECAPACITY (the replays themselves copy no counters); while the batch exists its
    problems are not stepped or set on their own."""
    import torch
    assert torch.cuda.is_available()
    from paper_1406_7416_amd import adg
    wls = W.quadrant_batch(3)
    for wl in wls:
        wl.ncell = (16, 16)
    ps = []
    for i, wl in enumerate(wls):
        g = adg.Problem(wl, precision=adg.ADG_FP64, pool_capacity=1 if i == 1 else 256)
        u, _ = g.project(wl.ic, 0)
        g.set_state(u)
        ps.append(g)
    b = adg.Batch(ps)
    with pytest.raises(adg.AdgError, match="-6"):
        ps[0].step_cfl(0.5)
    with pytest.raises(adg.AdgError, match="-6"):
        ps[2].set_state(ps[2].state())
    with pytest.raises(adg.AdgError, match="-6"):
        adg.Batch([ps[0]])
    with pytest.raises(adg.AdgError, match="-4"):
        for _ in range(4):
            b.step_cfl(0.5, 2)
    b.close()
    # after the batch: stepping on their own works again (problem 0 has a large pool)
    ps[0].step_cfl(0.5)
    for g in ps:
        g.close()
