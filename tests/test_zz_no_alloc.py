"""The time-step entry point that allocates nothing (adg_cfl_dt_static: its reduction
scratch is a static device array of the library) against adg_cfl_dt on the same states:
two calls in a row, the second on a smaller grid, each bit-identical to adg_cfl_dt
(the same kernels and the same reduction shape)."""
import numpy as np
import pytest

from paper_1406_7416_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dt_both(wl, cfl):
    import torch
    from paper_1406_7416_amd import adg
    p = adg.Problem(wl)
    u, v = p.project(wl.ic, wl.N + 1)
    p.set_state(u, v)
    for _ in range(2):               # a state that the step has produced
        p.step_cfl(cfl)
    ref = p.cfl_dt(cfl)
    ut = p.state_tensor()
    dt = torch.full((1,), float("nan"), dtype=torch.float64, device=ut.device)
    hmin = min((wl.hi[k] - wl.lo[k]) / wl.ncell[k] for k in range(wl.dim))
    adg.cfl_dt_static(ut, wl.dim, wl.N, wl.gamma, hmin, cfl, dt)
    torch.cuda.synchronize()
    out = float(dt.item())
    p.close()
    return ref, out


def test_cfl_dt_static_matches_cfl_dt_twice_second_smaller():
    import torch
    assert torch.cuda.is_available()
    # a grid whose reduction needs the full 1024 partial maxima, then a smaller one
    big = W.explosion_2d(160, 3)       # 25,600 cells x 16 nodes: 1600 blocks, clamped to 1024
    small = W.explosion_2d(12, 3)      # 144 cells x 16 nodes: 9 blocks
    r1, o1 = _dt_both(big, 0.7)
    r2, o2 = _dt_both(small, 0.7)
    print(f"dt static/ref: {o1!r}/{r1!r}, {o2!r}/{r2!r}", flush=True)
    assert np.isfinite(o1) and o1 == r1
    assert np.isfinite(o2) and o2 == r2
    assert o1 != o2


def test_cfl_dt_static_3d_and_bad_sizes():
    import torch
    from paper_1406_7416_amd import adg
    wl = W.explosion_3d(10, 2)
    r, o = _dt_both(wl, 0.5)
    assert o == r
    u = torch.ones((5, 8, 27), dtype=torch.float64, device="cuda:0")
    dt = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    with pytest.raises(adg.AdgError):
        adg.cfl_dt_static(u, 3, 7, 1.4, 0.1, 0.5, dt)     # 3D N = 7 is not built
    with pytest.raises(adg.AdgError):
        adg.cfl_dt_static(u, 3, 2, 1.0, 0.1, 0.5, dt)     # gamma must exceed 1
