"""The C ABI library loads and exports every function include/adg.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

from paper_1406_7416_amd import adg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "adg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(adg_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_surface():
    assert declared_functions() == sorted(adg.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(adg.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_create_and_plan_without_gpu():
    """adg_create / adg_workspace_bytes / adg_axis_points / adg_project_samples are
    host-side and work without a device."""
    import numpy as np
    from paper_1406_7416_amd import workloads as W
    L = adg.load()
    wl = W.explosion_2d(8, 3)
    g = adg._grid(wl)
    prm = adg._Params()
    prm.limiter = 1
    h = ctypes.c_void_p()
    assert L.adg_create(ctypes.byref(g), 3, 1.4, ctypes.byref(prm), ctypes.byref(h)) == 0
    assert L.adg_workspace_bytes(h) > 0
    x = np.zeros(8 * 4)
    assert L.adg_axis_points(h, 0, 0, adg._dp(x)) == 0
    assert x[0] > -1 and x[-1] < 1 and np.all(np.diff(x) > 0)
    # bad arguments are reported, not crashed on
    h2 = ctypes.c_void_p()
    assert L.adg_create(ctypes.byref(g), 12, 1.4, ctypes.byref(prm), ctypes.byref(h2)) == -1
    assert b"not built" in L.adg_last_error()
    assert L.adg_step(h, 1e-3) == -6   # no state bound yet
    assert L.adg_debug_poison(h, 0, 0, 1.0) == -6
    L.adg_destroy(h)


def test_library_projection_matches_oracle_projection():
    """Initial-data projection (host code of the library) vs the oracle's own."""
    import numpy as np
    from oracle import oracle as O
    from paper_1406_7416_amd import workloads as W
    L = adg.load()
    for wl in (W.explosion_2d(6, 3), W.vortex(4, 5), W.explosion_3d(3, 2)):
        g = adg._grid(wl)
        prm = adg._Params()
        prm.limiter = 1
        h = ctypes.c_void_p()
        assert L.adg_create(ctypes.byref(g), wl.N, wl.gamma, ctypes.byref(prm), ctypes.byref(h)) == 0
        o = O.Oracle(wl)
        for m in (0, wl.N + 1):
            per = (wl.N + 1) if m == 0 else (2 * wl.N + 1) * m
            axes = []
            for k in range(wl.dim):
                x = np.zeros(wl.ncell[k] * per)
                assert L.adg_axis_points(h, k, m, adg._dp(x)) == 0
                assert np.abs(x - o.axis_points(k, m)).max() < 1e-14
                axes.append(x)
            s = np.ascontiguousarray(W.sample_grid(wl.ic, axes))
            nv, nc = wl.dim + 2, wl.num_cells
            u = np.zeros((nv, nc, (wl.N + 1) ** wl.dim))
            v = np.zeros((nv, nc, (2 * wl.N + 1) ** wl.dim)) if m else None
            assert L.adg_project_samples(h, adg._dp(s), m, adg._dp(u), adg._dp(v) if m else None) == 0
            uo, vo = o.project(wl.ic, m)
            assert np.abs(u - uo).max() < 1e-13 * max(1, np.abs(uo).max())
            if m:
                assert np.abs(v - vo).max() < 1e-13 * max(1, np.abs(vo).max())
        L.adg_destroy(h)


def test_degrees_built_per_dimension_and_large_cell_workspace():
    """3D is built for N = 1..3 and 9 (2D for 1..9); other 3D degrees are refused with the
    reason.  A 3D problem of degree 9 plans the large-cell slots (512 per-workgroup slots of
    the arrays that exceed LDS) on top of its state, traces and pool."""
    from paper_1406_7416_amd import workloads as W
    L = adg.load()

    def create(wl, N, cap=0):
        g = adg._grid(wl)
        prm = adg._Params()
        prm.limiter = 1
        prm.Ns = 2 * N + 1
        prm.pool_capacity = cap
        h = ctypes.c_void_p()
        rc = L.adg_create(ctypes.byref(g), N, 1.4, ctypes.byref(prm), ctypes.byref(h))
        return rc, h

    for N in (1, 2, 3, 9):
        rc, h = create(W.explosion_3d(2, N), N)
        assert rc == 0, N
        L.adg_destroy(h)
    for N in (4, 5, 8):
        rc, _ = create(W.explosion_3d(2, N), N)
        assert rc == -1 and b"not built" in L.adg_last_error(), N
    # 4^3 cells of degree 9, pool for every cell: the state (2 copies), the traces and face
    # fluxes, two pools of 19^3 subcells, the subcell chunk scratch and the large-cell slots
    rc, h = create(W.explosion_3d(4, 9), 9)
    assert rc == 0
    nb = L.adg_workspace_bytes(h)
    L.adg_destroy(h)
    nc, nv, n, ns = 64, 5, 10, 19
    state = 2 * 8 * nv * nc * n ** 3
    pools = 2 * 8 * nc * nv * ns ** 3
    slots = 8 * 512 * 176896
    assert nb > state + pools + slots
    # and the slots are the difference a smaller pool does not remove
    rc, h = create(W.explosion_3d(4, 9), 9, cap=8)
    assert rc == 0
    nb8 = L.adg_workspace_bytes(h)
    L.adg_destroy(h)
    assert nb8 > slots and nb - nb8 >= 2 * 8 * (nc - 8) * nv * ns ** 3
