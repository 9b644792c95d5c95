"""Edge cases of the step against the FP64 oracle (FP64 form, the parity bounds of the
other tests: 1e-12 relative in the first step, 1e-10 after, identical troubled maps):
  * every cell troubled (the pool at full capacity, no unlimited cell left for the flux
    correction);
  * the lowest degree, N = 1 (three subcells per axis), in 2D and 3D with the limiter;
  * the highest degree, N = 9 (19 subcells per axis, the largest subcell kernel), on the
    subcell path;
  * a grid one cell thick along a periodic axis (the cell is its own neighbour there) with
    Dirichlet sides, cells 24 times longer than wide.
The same cases run in the mixed form (FP32 subcell reconstruction, degree-2 predictor and
sub-face fluxes at N = 1 and N = 9 included) with that form's bounds: 2e-6 relative per step,
troubled maps differing only where the oracle's detection margin is below 1e-4.
"""
import numpy as np
import pytest

from paper_1406_7416_amd import workloads as W
from test_gpu_mixed import paired_mixed, run_mixed
from test_gpu_parity import paired, run_parity

pytestmark = pytest.mark.gpu


def test_every_cell_troubled():
    wl = W.vortex(8, 3)
    o, g = paired(wl, m=0, mask=np.ones(wl.num_cells, dtype=np.uint8))
    run_parity(o, g, 3)
    assert o.troubled().all() and g.troubled().all()
    assert g.stats()["corrected"] == 0


@pytest.mark.parametrize("dim,n", [(2, 16), (3, 6)])
def test_lowest_degree_with_limiter(dim, n):
    wl = W.explosion_2d(n, 1) if dim == 2 else W.explosion_3d(n, 1)
    o, g = paired(wl)
    run_parity(o, g, 3)
    assert o.troubled().sum() > 0


def test_highest_degree_subcell_path():
    wl = W.vortex(6, 9)
    o, g = paired(wl, m=0, mask=W.random_mask(wl.num_cells, 0.3, seed=9))
    run_parity(o, g, 3)
    assert o.troubled().sum() > 0


def test_one_cell_thick_periodic_axis():
    wl = W.shock_tube("sod", nx=24, ny=1, N=4)
    o, g = paired(wl)
    run_parity(o, g, 3)
    assert o.troubled().sum() > 0


def test_every_cell_troubled_mixed():
    wl = W.vortex(8, 3)
    o, g = paired_mixed(wl, m=0, mask=np.ones(wl.num_cells, dtype=np.uint8))
    worst, steps = run_mixed(o, g, 3)
    assert steps == 3 and worst > 0
    assert o.troubled().all() and g.troubled().all()
    assert g.stats()["corrected"] == 0


@pytest.mark.parametrize("dim,n", [(2, 16), (3, 6)])
def test_lowest_degree_with_limiter_mixed(dim, n):
    wl = W.explosion_2d(n, 1) if dim == 2 else W.explosion_3d(n, 1)
    o, g = paired_mixed(wl)
    run_mixed(o, g, 3)
    assert o.troubled().sum() > 0


def test_highest_degree_subcell_path_mixed():
    wl = W.vortex(6, 9)
    o, g = paired_mixed(wl, m=0, mask=W.random_mask(wl.num_cells, 0.3, seed=9))
    worst, steps = run_mixed(o, g, 3)
    assert steps == 3 and worst > 0
    assert o.troubled().sum() > 0


def test_one_cell_thick_periodic_axis_mixed():
    wl = W.shock_tube("sod", nx=24, ny=1, N=4)
    o, g = paired_mixed(wl)
    run_mixed(o, g, 3)
    assert o.troubled().sum() > 0
