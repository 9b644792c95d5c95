"""Python binding of the C ABI in include/adg.h (libadg.so, built for gfx950).

Argument marshalling only: every step of the method runs in the library's HIP kernels.
PyTorch supplies the device workspace and the stream.  Importing works without a GPU;
creating a Problem needs the built library and fails loudly if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadg.so")

ADG_PERIODIC, ADG_TRANSMISSIVE, ADG_REFLECTIVE, ADG_DIRICHLET = 0, 1, 2, 3
ADG_FP64, ADG_MIXED, ADG_MIXED_DEV = 0, 1, 2

EXPORTS = [
    "adg_last_error", "adg_create", "adg_destroy", "adg_workspace_bytes", "adg_bind", "adg_axis_points",
    "adg_project_samples", "adg_set_state", "adg_get_state", "adg_cfl_dt", "adg_step", "adg_step_cfl",
    "adg_time", "adg_get_troubled", "adg_get_margin", "adg_get_subcells", "adg_get_stats",
    "adg_profile", "adg_profile_read", "adg_batch_create", "adg_batch_step_cfl", "adg_batch_dt",
    "adg_batch_destroy", "adg_debug_force_troubled", "adg_debug_poison", "adg_get_mood_stats",
    "adg_cfl_dt_static", "adg_state_device_ptr", "adg_batch_workspace_bytes", "adg_batch_bind",
    "adg_batch_profile", "adg_batch_profile_read", "adg_batch_classes", "adg_set_mask",
]

BATCH_STAGES = ["dt", "bounds", "predictor", "faces", "corrector_detect", "compact", "subcell", "fluxcorr",
                "advance"]

KERNEL_GROUPS = ["bounds", "predictor", "faces", "corrector_detect", "compact", "subcell", "fluxcorr", "dt"]


class AdgError(RuntimeError):
    pass


class _BC(C.Structure):
    _fields_ = [("kind", C.c_int * 2), ("split_axis", C.c_int), ("split0", C.c_double),
                ("split_speed", C.c_double), ("state", (C.c_double * 5) * 2)]


class _Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int64 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("bc", (_BC * 2) * 3)]


class _Params(C.Structure):
    _fields_ = [("Ns", C.c_int), ("picard_iters", C.c_int), ("precision", C.c_int), ("limiter", C.c_int),
                ("eps", C.c_double), ("delta0", C.c_double), ("pool_capacity", C.c_int64), ("mood", C.c_int),
                ("flux", C.c_int)]


_lib = None


def load():
    """Loads libadg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise AdgError(f"{LIB_PATH} not built: run __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp, dp, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int64
    L.adg_last_error.restype = C.c_char_p
    L.adg_create.argtypes = [C.POINTER(_Grid), C.c_int, C.c_double, C.POINTER(_Params), C.POINTER(vp)]
    L.adg_destroy.argtypes = [vp]
    L.adg_workspace_bytes.restype = C.c_size_t
    L.adg_workspace_bytes.argtypes = [vp]
    L.adg_bind.argtypes = [vp, vp, C.c_size_t, vp]
    L.adg_axis_points.argtypes = [vp, C.c_int, C.c_int, dp]
    L.adg_project_samples.argtypes = [vp, dp, C.c_int, dp, dp]
    L.adg_set_state.argtypes = [vp, vp, C.c_int, dp]
    L.adg_set_mask.argtypes = [vp, C.POINTER(C.c_uint8)]
    L.adg_get_state.argtypes = [vp, vp, C.c_int]
    L.adg_cfl_dt.argtypes = [vp, C.c_double, dp]
    L.adg_step.argtypes = [vp, C.c_double]
    L.adg_step_cfl.argtypes = [vp, C.c_double]
    L.adg_time.argtypes = [vp, dp]
    L.adg_get_troubled.argtypes = [vp, C.POINTER(C.c_uint8), C.POINTER(i64)]
    L.adg_get_margin.argtypes = [vp, C.POINTER(C.c_float)]
    L.adg_get_subcells.argtypes = [vp, dp]
    L.adg_get_stats.argtypes = [vp, C.POINTER(i64)]
    L.adg_debug_force_troubled.argtypes = [vp, C.POINTER(C.c_uint8)]
    L.adg_debug_poison.argtypes = [vp, C.c_int64, C.c_int, C.c_double]
    L.adg_get_mood_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.adg_profile.argtypes = [vp, C.c_int]
    L.adg_profile_read.argtypes = [vp, dp, C.POINTER(i64), C.c_int]
    L.adg_batch_create.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(vp)]
    L.adg_batch_step_cfl.argtypes = [vp, C.c_double, C.c_int]
    L.adg_batch_dt.argtypes = [vp, dp]
    L.adg_batch_destroy.argtypes = [vp]
    L.adg_batch_workspace_bytes.restype = C.c_size_t
    L.adg_batch_workspace_bytes.argtypes = [vp]
    L.adg_batch_bind.argtypes = [vp, vp, C.c_size_t, vp]
    L.adg_batch_profile.argtypes = [vp, C.c_int]
    L.adg_batch_profile_read.argtypes = [vp, dp, C.POINTER(i64)]
    L.adg_batch_classes.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_int]
    L.adg_state_device_ptr.argtypes = [vp, C.POINTER(vp)]
    L.adg_cfl_dt_static.argtypes = [vp, C.c_int, C.c_int, C.c_int64, C.c_double, C.c_double, C.c_double, vp, vp]
    for name in EXPORTS[1:]:
        if name not in ("adg_workspace_bytes", "adg_batch_workspace_bytes"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


ADG_ENONPHYSICAL = -5
_nonphysical_warnings = 0


def _check(rc: int):
    """Raises on an error code.  ADG_ENONPHYSICAL is a warning (the step was taken; the count
    of non-physical subcell results is in Problem.stats()): it is counted, not raised."""
    global _nonphysical_warnings
    if rc == ADG_ENONPHYSICAL:
        _nonphysical_warnings += 1
        return
    if rc != 0:
        raise AdgError(f"adg error {rc}: {load().adg_last_error().decode()}")


def nonphysical_warnings() -> int:
    """How many calls so far returned the ADG_ENONPHYSICAL warning."""
    return _nonphysical_warnings


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _grid(wl) -> _Grid:
    g = _Grid()
    g.dim = wl.dim
    for k in range(3):
        g.n[k] = wl.ncell[k] if k < wl.dim else 1
        g.lo[k] = wl.lo[k] if k < wl.dim else 0.0
        g.hi[k] = wl.hi[k] if k < wl.dim else 1.0
    for k in range(wl.dim):
        for side in range(2):
            b = wl.bcs[k][side]
            cb = g.bc[k][side]
            cb.kind[0], cb.kind[1] = b.kind
            cb.split_axis, cb.split0, cb.split_speed = b.split_axis, b.split0, b.split_speed
            for w in range(2):
                for v in range(5):
                    cb.state[w][v] = b.states[w][v] if v < len(b.states[w]) else 0.0
    return g


def _axis_points(h, wl, axis: int, m: int, n: int, Ns: int) -> np.ndarray:
    per = n if m == 0 else Ns * m
    out = np.zeros(wl.ncell[axis] * per)
    _check(load().adg_axis_points(h, axis, m, _dp(out)))
    return out


def _project(h, wl, ic, m: int, t: float, Ns: int):
    from .workloads import sample_grid
    d, n = wl.dim, wl.N + 1
    axes = [_axis_points(h, wl, k, m, n, Ns) for k in range(d)]
    samples = np.ascontiguousarray(sample_grid(ic, axes, t))
    u = np.zeros((d + 2, wl.num_cells, n ** d))
    v = np.zeros((d + 2, wl.num_cells, Ns ** d)) if m > 0 else None
    _check(load().adg_project_samples(h, _dp(samples), m, _dp(u), _dp(v) if v is not None else None))
    return u, v


def project(wl, m: int, ic=None, t: float = 0.0):
    """Initial data of workload `wl` without a GPU: nodal values u (m = 0: samples at the
    nodes; m > 0: L2 projection with an m-point rule per subcell) and, for m > 0, the
    rule's subcell averages v, for Problem.set_state."""
    L = load()
    Ns = wl.Ns if wl.Ns else 2 * wl.N + 1
    prm = _Params()
    prm.Ns = Ns
    prm.eps, prm.delta0 = wl.eps, wl.delta0
    g = _grid(wl)
    h = C.c_void_p()
    _check(L.adg_create(C.byref(g), wl.N, wl.gamma, C.byref(prm), C.byref(h)))
    try:
        return _project(h, wl, wl.ic if ic is None else ic, m, t, Ns)
    finally:
        L.adg_destroy(h)


class Problem:
    """One problem on one GPU: owns a torch workspace, drives the C ABI."""

    def __init__(self, wl, precision: int = ADG_FP64, limiter: bool = True, pool_capacity: int = 0,
                 picard_iters: int = 0, device: str = "cuda:0", stream=None, mood: bool = False,
                 flux: int = 0):
        import torch
        L = load()
        self.wl = wl
        self.dim, self.nv, self.n = wl.dim, wl.dim + 2, wl.N + 1
        self.Ns = wl.Ns if wl.Ns else 2 * wl.N + 1
        self.ncell = wl.num_cells
        self.nn = self.n ** self.dim
        self.nsub = self.Ns ** self.dim
        prm = _Params()
        prm.Ns = self.Ns
        prm.picard_iters = picard_iters
        prm.precision = precision
        prm.limiter = 1 if limiter else 0
        prm.eps, prm.delta0 = wl.eps, wl.delta0
        prm.pool_capacity = pool_capacity
        prm.mood = 1 if mood else 0
        prm.flux = flux
        self._grid = _grid(wl)
        h = C.c_void_p()
        _check(L.adg_create(C.byref(self._grid), wl.N, wl.gamma, C.byref(prm), C.byref(h)))
        self.h = h
        self.device = torch.device(device)
        nbytes = L.adg_workspace_bytes(self.h)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(L.adg_bind(self.h, C.c_void_p(aligned), nbytes, C.c_void_p(self.stream.cuda_stream)))
        self.workspace_bytes = nbytes

    def close(self):
        if getattr(self, "h", None):
            load().adg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- initial data
    def axis_points(self, axis: int, m: int) -> np.ndarray:
        return _axis_points(self.h, self.wl, axis, m, self.n, self.Ns)

    def project(self, ic, m: int, t: float = 0.0):
        return _project(self.h, self.wl, ic, m, t, self.Ns)

    def set_mask(self, mask: Optional[np.ndarray]):
        """Masked geometry: one byte per cell (x fastest), nonzero = solid; None removes it.
        Call before set_state."""
        if mask is None:
            _check(load().adg_set_mask(self.h, None))
            return
        m = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
        assert m.size == self.wl.num_cells
        _check(load().adg_set_mask(self.h, m.ctypes.data_as(C.POINTER(C.c_uint8))))

    def set_state(self, u, v_exact: Optional[np.ndarray] = None):
        ve = None if v_exact is None else np.ascontiguousarray(v_exact, dtype=np.float64)
        vptr = _dp(ve) if ve is not None else None
        if hasattr(u, "is_cuda") and u.is_cuda:
            assert u.dtype.is_floating_point and u.is_contiguous()
            _check(load().adg_set_state(self.h, C.c_void_p(u.data_ptr()), 1, vptr))
        else:
            uh = np.ascontiguousarray(u, dtype=np.float64)
            _check(load().adg_set_state(self.h, uh.ctypes.data_as(C.c_void_p), 0, vptr))

    def init(self, m: Optional[int] = None, detect: bool = True):
        if m is None:
            m = self.n
        u, v = self.project(self.wl.ic, m)
        self.set_state(u, v if detect else None)

    # ---- stepping
    def cfl_dt(self, cfl: Optional[float] = None) -> float:
        dt = C.c_double()
        _check(load().adg_cfl_dt(self.h, self.wl.cfl if cfl is None else cfl, C.byref(dt)))
        return dt.value

    def step(self, dt: float):
        _check(load().adg_step(self.h, dt))

    def step_cfl(self, cfl: Optional[float] = None):
        _check(load().adg_step_cfl(self.h, self.wl.cfl if cfl is None else cfl))

    def force_troubled(self, mask: Optional[np.ndarray]):
        if mask is None:
            _check(load().adg_debug_force_troubled(self.h, None))
        else:
            m = np.ascontiguousarray(mask, dtype=np.uint8)
            _check(load().adg_debug_force_troubled(self.h, m.ctypes.data_as(C.POINTER(C.c_uint8))))

    # ---- outputs
    @property
    def time(self) -> float:
        t = C.c_double()
        _check(load().adg_time(self.h, C.byref(t)))
        return t.value

    def state(self) -> np.ndarray:
        u = np.zeros((self.nv, self.ncell, self.nn))
        _check(load().adg_get_state(self.h, u.ctypes.data_as(C.c_void_p), 0))
        return u

    def state_device_ptr(self) -> int:
        """Device address of the current state inside the workspace (valid until the next step)."""
        ptr = C.c_void_p()
        _check(load().adg_state_device_ptr(self.h, C.byref(ptr)))
        return ptr.value

    def state_tensor(self):
        import torch
        u = torch.empty((self.nv, self.ncell, self.nn), dtype=torch.float64, device=self.device)
        _check(load().adg_get_state(self.h, C.c_void_p(u.data_ptr()), 1))
        return u

    def troubled(self) -> np.ndarray:
        b = np.zeros(self.ncell, dtype=np.uint8)
        cnt = C.c_int64()
        _check(load().adg_get_troubled(self.h, b.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(cnt)))
        return b

    def margin(self) -> np.ndarray:
        m = np.zeros(self.ncell, dtype=np.float32)
        _check(load().adg_get_margin(self.h, m.ctypes.data_as(C.POINTER(C.c_float))))
        return m

    def subcells(self) -> np.ndarray:
        v = np.zeros((self.nv, self.ncell, self.nsub))
        _check(load().adg_get_subcells(self.h, _dp(v)))
        return v

    def profile(self, enable, groups=None):
        """Starts (clears) or stops per-kernel-group timing; `groups` names the groups
        to time (default: all of KERNEL_GROUPS)."""
        mask = 0
        if enable:
            names = KERNEL_GROUPS if groups is None else groups
            for g in names:
                mask |= 1 << KERNEL_GROUPS.index(g)
        _check(load().adg_profile(self.h, mask))

    def profile_read(self) -> dict:
        ms = np.zeros(8)
        n = (C.c_int64 * 8)()
        _check(load().adg_profile_read(self.h, _dp(ms), n, 8))
        return {g: (float(ms[i]), int(n[i])) for i, g in enumerate(KERNEL_GROUPS)}

    def poison(self, cell: int, var: int, value: float):
        """Debug hook: variable `var` of cell `cell`'s next candidate is set to `value`."""
        _check(load().adg_debug_poison(self.h, int(cell), int(var), float(value)))

    def mood_stats(self):
        """(flagged subcells, recomputed cells) of the last step's MOOD layer."""
        f, r = C.c_int64(), C.c_int64()
        _check(load().adg_get_mood_stats(self.h, C.byref(f), C.byref(r)))
        return f.value, r.value

    def stats(self) -> dict:
        out = (C.c_int64 * 4)()
        _check(load().adg_get_stats(self.h, out))
        return {"troubled": out[0], "corrected": out[1], "nonphysical": out[2], "steps": out[3]}


def cfl_dt_static(u, dim: int, N: int, gamma: float, hmin: float, cfl: float, dt_out, stream=None):
    """Eq. (cfl) time step of a device state tensor u ([var][cell][node], float64) into the
    one-element device tensor dt_out, through the entry point that allocates nothing (its
    reduction scratch is a static device array of the library).  Enqueued on `stream`
    (default: torch's current stream), no host wait."""
    import torch
    assert u.is_cuda and u.dtype == torch.float64 and u.is_contiguous()
    assert dt_out.is_cuda and dt_out.dtype == torch.float64 and dt_out.numel() >= 1
    ncell = u.shape[1]
    s = stream if stream is not None else torch.cuda.current_stream(u.device)
    _check(load().adg_cfl_dt_static(C.c_void_p(u.data_ptr()), dim, N, ncell, gamma, hmin, cfl,
                                     C.c_void_p(dt_out.data_ptr()), C.c_void_p(s.cuda_stream)))


class Batch:
    """Independent problems advanced together: one launch per stage and (d, N) class, the
    whole step captured in a hipGraph, one graph launch per batch step.  The batch's device
    memory is a torch tensor; it runs on torch's current stream of the problems' device."""

    def __init__(self, problems, stream=None):
        import torch
        L = load()
        self.problems = list(problems)
        arr = (C.c_void_p * len(self.problems))(*[p.h.value for p in self.problems])
        h = C.c_void_p()
        _check(L.adg_batch_create(arr, len(self.problems), C.byref(h)))
        self.h = h
        dev = self.problems[0].device
        nbytes = L.adg_batch_workspace_bytes(self.h)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        _check(L.adg_batch_bind(self.h, C.c_void_p(aligned), nbytes, C.c_void_p(self.stream.cuda_stream)))
        self.workspace_bytes = nbytes

    def profile(self, enable: bool):
        """Starts (clears) or stops the per-stage timing (events inside the graphs)."""
        _check(load().adg_batch_profile(self.h, 1 if enable else 0))

    def classes(self):
        """The (dim, N) classes of the batch, in launch order."""
        L = load()
        nc = L.adg_batch_classes(self.h, None, None, 0)
        if nc < 0:
            _check(nc)
        dims, Ns = (C.c_int * nc)(), (C.c_int * nc)()
        L.adg_batch_classes(self.h, dims, Ns, nc)
        return [(dims[i], Ns[i]) for i in range(nc)]

    def profile_read(self) -> dict:
        """{stage: (total ms, timed steps)} and, under "launches", {(stage, (dim, N)): total ms}."""
        cls = self.classes()
        ns = len(BATCH_STAGES)
        ms = np.zeros(ns * len(cls))
        n = C.c_int64()
        _check(load().adg_batch_profile_read(self.h, _dp(ms), C.byref(n)))
        out = {g: (float(ms[i * len(cls):(i + 1) * len(cls)].sum()), int(n.value)) for i, g in enumerate(BATCH_STAGES)}
        out["launches"] = {(g, cls[c]): float(ms[i * len(cls) + c]) for i, g in enumerate(BATCH_STAGES)
                           for c in range(len(cls))}
        return out

    def step_cfl(self, cfl: float, nsteps: int = 1):
        _check(load().adg_batch_step_cfl(self.h, cfl, nsteps))

    def dts(self) -> np.ndarray:
        out = np.zeros(len(self.problems))
        _check(load().adg_batch_dt(self.h, _dp(out)))
        return out

    def close(self):
        if getattr(self, "h", None):
            load().adg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
