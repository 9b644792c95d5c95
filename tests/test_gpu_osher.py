"""The Osher-type numerical flux option (Sec. 2.3) on the GPU against the oracle: element
faces (smooth vortex) and element faces plus sub-faces (explosion with the limiter), both
precision forms."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1406_7416_amd import workloads as W
from test_gpu_parity import gpu_problem, rel_err, run_parity

pytestmark = pytest.mark.gpu


def paired_osher(wl, m, precision=None):
    from paper_1406_7416_amd import adg
    o = O.Oracle(wl, flux=1)
    u, v = o.project(wl.ic, m)
    o.set_state(u, v)
    g = gpu_problem(wl, flux=1, precision=adg.ADG_FP64 if precision is None else precision)
    g.set_state(u, v)
    return o, g


def test_osher_vortex_parity():
    o, g = paired_osher(W.vortex(10, 5), m=0)
    run_parity(o, g, 3)


def test_osher_explosion_with_limiter_parity():
    o, g = paired_osher(W.explosion_2d(20, 3), m=4)
    run_parity(o, g, 4)
    assert o.troubled().sum() > 0


def test_osher_mixed_form():
    from paper_1406_7416_amd import adg
    o, g = paired_osher(W.vortex(8, 9), m=0, precision=adg.ADG_MIXED)
    for _ in range(3):
        dt = o.cfl_dt()
        o.step(dt)
        g.step(dt)
        assert rel_err(g.state(), o.state()) < 2e-6
    assert np.array_equal(o.troubled(), g.troubled())


@pytest.mark.parametrize("prec_name", ["fp64", "mixed"])
def test_osher_vortex_full_size(prec_name):
    """The benchmark's vortex (N = 9, 64 x 64) with the Osher-type flux in the launch
    configuration the benchmark times, one step, both forms."""
    from paper_1406_7416_amd import adg
    prec = adg.ADG_MIXED if prec_name == "mixed" else adg.ADG_FP64
    o, g = paired_osher(W.vortex(64, 9), m=0, precision=prec)
    dt = o.cfl_dt()
    o.step(dt)
    g.step(dt)
    assert rel_err(g.state(), o.state()) < (2e-6 if prec_name == "mixed" else 1e-12)
    assert np.array_equal(o.troubled(), g.troubled())
