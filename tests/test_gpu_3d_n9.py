"""3D cells of degree N = 9 (the 3D explosion of Sec. 5 at P9, N_s = 19): the kernels of large
cells, whose per-cell arrays (19^3 subcell averages, the stages of the projection and gather,
the subcell update's sub-face fluxes) live in per-workgroup slots of global memory, against
the oracle on small grids.

Tolerances as the other parity tests: the FP64 form 1e-12 of each variable's scale on the
first step (1e-10 after), identical troubled maps; the mixed and deviation forms 2e-6, flags
may differ only where the oracle's detection margin is below 1e-4.  The initial state of a
cell troubled at t = 0 is the reconstruction R of its 19^3 subcell averages (eq.
(subcell.r)), contracted in another order by the host code of the library and by the oracle:
it agrees to 1e-12 (measured 1.2e-13; the least-squares operator at N_s = 19 has larger
entries than at the smaller degrees, whose initial states agree to 1e-13).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1406_7416_amd import workloads as W
from test_gpu_mixed import run_mixed
from test_gpu_parity import paired, rel_err, run_parity

pytestmark = pytest.mark.gpu


def smooth3d(n):
    """Smooth periodic data on the unit cube (every cell unlimited unless forced)."""
    def ic(x, t=0.0):
        rho = 1 + 0.2 * np.sin(2 * np.pi * x[0]) * np.cos(2 * np.pi * x[1]) + 0 * x[2]
        p = 1 + 0.1 * np.cos(2 * np.pi * x[2]) + 0 * x[0]
        z = 0 * x[0] + 0 * x[1] + 0 * x[2]
        return W.prim_to_cons(1.4, rho, [0.3 + z, 0.2 + z, -0.1 + z], p)
    return W.Workload("smooth3d", 3, 9, n, (0.0,) * 3, (1.0,) * 3,
                      [(W.BC.simple(W.PERIODIC), W.BC.simple(W.PERIODIC))] * 3, ic)


def paired_form(wl, precision, m=1, mask=None):
    import torch
    assert torch.cuda.is_available()
    from paper_1406_7416_amd import adg
    o = O.Oracle(wl)
    u, v = o.project(wl.ic, m)
    o.set_state(u, v)
    g = adg.Problem(wl, precision=precision)
    g.set_state(u, v)
    if mask is not None:
        o.force_troubled(mask)
        g.force_troubled(mask)
    return o, g


def test_n9_explosion_3d_fp64():
    """4^3 cells of h = 0.5: the sphere cuts every cell, so every cell starts troubled and
    the subcell scheme (19^3 subcells per cell) carries the first step."""
    print("3D N=9 explosion 4^3, FP64", flush=True)
    o, g = paired(W.explosion_3d(4, 9), m=1)
    assert int(o.troubled().sum()) == 64
    run_parity(o, g, 2, tol_init=1e-12)
    b = o.troubled().astype(bool)
    assert b.sum() > 0
    assert rel_err(g.subcells()[:, b], o.subcells()[:, b]) < 1e-10
    assert g.stats()["nonphysical"] == 0


def test_n9_forced_troubled_flux_correction_fp64():
    """Smooth periodic data, a random third of the cells forced troubled: the subcell
    recompute next to unlimited cells, their flux correction and the pool across steps."""
    print("3D N=9 smooth 3x3x2, forced troubled, FP64", flush=True)
    wl = smooth3d((3, 3, 2))
    o, g = paired(wl, m=0, mask=W.random_mask(wl.num_cells, 0.35, seed=4))
    run_parity(o, g, 2, tol_init=1e-12)
    b = o.troubled().astype(bool)
    assert 0 < b.sum() < wl.num_cells
    assert rel_err(g.subcells()[:, b], o.subcells()[:, b]) < 1e-10


def test_n9_explosion_3d_mixed():
    from paper_1406_7416_amd import adg
    print("3D N=9 explosion 4^3, mixed form", flush=True)
    o, g = paired_form(W.explosion_3d(4, 9), adg.ADG_MIXED)
    worst, done = run_mixed(o, g, 2)
    assert worst > 0 and done >= 1


def test_n9_forced_troubled_deviation_form():
    from paper_1406_7416_amd import adg
    print("3D N=9 smooth 3x3x2, forced troubled, deviation form", flush=True)
    wl = smooth3d((3, 3, 2))
    o, g = paired_form(wl, adg.ADG_MIXED_DEV, m=0, mask=W.random_mask(wl.num_cells, 0.35, seed=4))
    worst, done = run_mixed(o, g, 2)
    assert worst > 0 and done == 2


def test_n9_batch_is_refused():
    """Large cells are stepped problem by problem: a batch refuses them with ADG_EINVAL."""
    from paper_1406_7416_amd import adg
    wl = smooth3d((2, 2, 2))
    p = adg.Problem(wl)
    u, _ = p.project(wl.ic, 0)
    p.set_state(u)
    with pytest.raises(adg.AdgError, match="-1"):
        adg.Batch([p])
    p.close()


def test_n9_mood_layer_fp64():
    """The MOOD layer after the subcell scheme (Sec. 6, Fig. algo2) on large cells: the flags
    of the WENO3 result and the recompute (the REDO pass of the subcell kernel) as the oracle's."""
    from test_gpu_parity import gpu_problem
    print("3D N=9 explosion 4^3, FP64, MOOD layer", flush=True)
    wl = W.explosion_3d(4, 9)
    o = O.Oracle(wl, mood=True)
    u, v = o.project(wl.ic, 1)
    o.set_state(u, v)
    g = gpu_problem(wl, mood=True)
    g.set_state(u, v)
    for s in range(2):
        dt = o.cfl_dt()
        o.step(dt)
        g.step(dt)
        assert np.array_equal(o.troubled(), g.troubled()), f"step {s}"
        assert g.mood_stats() == o.mood_stats(), f"step {s}: {g.mood_stats()} vs {o.mood_stats()}"
        e = rel_err(g.state(), o.state())
        print(f"  step {s}: MOOD flagged / recomputed {o.mood_stats()}, rel err {e:.2e}", flush=True)
        assert e < (1e-12 if s == 0 else 1e-10), f"step {s}: rel err {e}"


def test_n9_solid_block_fp64():
    """Masked geometry on large cells: a solid bar in one corner of the 4^3 explosion grid
    (walls normal to all three axes, images along two axes at its edge): the sum-factorised
    halo's image regions and the sub-face walls as the oracle's."""
    from test_gpu_masked import masked_pair
    print("3D N=9 explosion 4^3 with a solid bar, FP64", flush=True)
    wl = W.explosion_3d(4, 9)
    m = np.zeros((4, 4, 4), np.uint8)   # [z][y][x]
    m[:2, :2, :1] = 1
    o, g = masked_pair(wl, m.ravel(), m=1)
    run_parity(o, g, 2, tol_init=1e-12)
    assert np.array_equal(o.troubled(), g.troubled())
