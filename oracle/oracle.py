"""ctypes wrapper of the FP64 CPU oracle (liboracle.so built from adg_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark; the product library never uses it.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")


class _BC(C.Structure):
    _fields_ = [("kind", C.c_int * 2), ("split_axis", C.c_int), ("split0", C.c_double),
                ("split_speed", C.c_double), ("state", (C.c_double * 5) * 2)]


class _Config(C.Structure):
    _fields_ = [("dim", C.c_int), ("N", C.c_int), ("Ns", C.c_int), ("picard_iters", C.c_int),
                ("limiter", C.c_int), ("ncell", C.c_int * 3), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("gamma", C.c_double), ("eps", C.c_double),
                ("delta0", C.c_double), ("bc", (_BC * 2) * 3), ("mood", C.c_int), ("flux", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise RuntimeError(f"{_LIB} missing: run __graft_entry__.build() first")
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.or_create.restype = C.c_void_p
        L.or_create.argtypes = [C.POINTER(_Config)]
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_basis.argtypes = [C.c_int, dp, dp, dp, dp, dp, dp]
        L.or_subcell_ops.argtypes = [C.c_int, C.c_int, dp, dp]
        L.or_axis_points.argtypes = [C.c_void_p, C.c_int, C.c_int, dp]
        L.or_project.argtypes = [C.c_void_p, dp, C.c_int, dp, dp]
        L.or_set_state.restype = C.c_int
        L.or_set_state.argtypes = [C.c_void_p, dp, dp]
        L.or_get_state.argtypes = [C.c_void_p, dp]
        L.or_get_troubled.argtypes = [C.c_void_p, C.POINTER(C.c_uint8)]
        L.or_get_margin.argtypes = [C.c_void_p, dp]
        L.or_get_subcells.argtypes = [C.c_void_p, dp]
        L.or_get_bounds.argtypes = [C.c_void_p, dp, dp]
        L.or_force_troubled.argtypes = [C.c_void_p, C.POINTER(C.c_uint8)]
        L.or_set_mask.argtypes = [C.c_void_p, C.POINTER(C.c_uint8)]
        L.or_poison.argtypes = [C.c_void_p, C.c_long, C.c_int, C.c_double]
        L.or_mood_stats.argtypes = [C.c_void_p, C.POINTER(C.c_long), C.POINTER(C.c_long)]
        L.or_numerical_flux.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, dp, dp, dp]
        L.or_abs_jacobian.argtypes = [C.c_int, C.c_int, C.c_double, dp, dp, dp]
        L.or_time.restype = C.c_double
        L.or_time.argtypes = [C.c_void_p]
        L.or_set_time.argtypes = [C.c_void_p, C.c_double]
        L.or_cfl_dt.restype = C.c_double
        L.or_cfl_dt.argtypes = [C.c_void_p, C.c_double]
        L.or_step.restype = C.c_int
        L.or_step.argtypes = [C.c_void_p, C.c_double]
        L.or_nonphysical.restype = C.c_long
        L.or_nonphysical.argtypes = [C.c_void_p]
        L.or_set_threads.argtypes = [C.c_int]
        L.or_get_threads.restype = C.c_int
        L.or_predictor.argtypes = [C.c_int, C.c_int, C.c_double, dp, C.c_int, dp, dp]
        L.or_weno3.argtypes = [dp, dp]
        L.or_exact_riemann.argtypes = [C.c_double] * 7 + [dp, C.c_int, dp, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def basis(n: int):
    """(xi, w, D, L, R, Kw) of the n-point Gauss-Legendre nodal basis on [0,1]."""
    xi, w, L, R = (np.zeros(n) for _ in range(4))
    D, Kw = np.zeros((n, n)), np.zeros((n, n))
    lib().or_basis(n, _dp(xi), _dp(w), _dp(D), _dp(L), _dp(R), _dp(Kw))
    return xi, w, D, L, R, Kw


def subcell_ops(N: int, Ns: int):
    P, R = np.zeros((Ns, N + 1)), np.zeros((N + 1, Ns))
    lib().or_subcell_ops(N, Ns, _dp(P), _dp(R))
    return P, R


def predictor(dim: int, N: int, gamma: float, dt_over_h, iters: int, u_cell: np.ndarray) -> np.ndarray:
    n = N + 1
    q = np.zeros((dim + 2) * n ** (dim + 1))
    dth = np.ascontiguousarray(np.asarray(dt_over_h, dtype=np.float64))
    u = np.ascontiguousarray(u_cell, dtype=np.float64)
    lib().or_predictor(dim, N, gamma, _dp(dth), iters, _dp(u), _dp(q))
    return q.reshape(dim + 2, n, n ** dim)  # [v][s][a]


def weno3(avg5) -> np.ndarray:
    a = np.ascontiguousarray(avg5, dtype=np.float64)
    out = np.zeros(3)
    lib().or_weno3(_dp(a), _dp(out))
    return out


def exact_riemann(left, right, gamma, s):
    s = np.ascontiguousarray(s, dtype=np.float64)
    out = np.zeros(3 * len(s))
    ps = np.zeros(2)
    lib().or_exact_riemann(*left, *right, gamma, _dp(s), len(s), _dp(out), _dp(ps))
    return out.reshape(-1, 3), ps


def set_threads(n: int):
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return lib().or_get_threads()


def make_config(wl, limiter: bool = True, picard_iters: int = 0, mood: bool = False, flux: int = 0) -> _Config:
    c = _Config()
    c.mood = 1 if mood else 0
    c.flux = flux
    c.dim, c.N = wl.dim, wl.N
    c.Ns = wl.Ns if wl.Ns else 2 * wl.N + 1
    c.picard_iters = picard_iters if picard_iters else wl.N + 1
    c.limiter = 1 if limiter else 0
    for k in range(3):
        c.ncell[k] = wl.ncell[k] if k < wl.dim else 1
        c.lo[k] = wl.lo[k] if k < wl.dim else 0.0
        c.hi[k] = wl.hi[k] if k < wl.dim else 1.0
    c.gamma, c.eps, c.delta0 = wl.gamma, wl.eps, wl.delta0
    for k in range(wl.dim):
        for side in range(2):
            b = wl.bcs[k][side]
            cb = c.bc[k][side]
            cb.kind[0], cb.kind[1] = b.kind
            cb.split_axis, cb.split0, cb.split_speed = b.split_axis, b.split0, b.split_speed
            for w in range(2):
                for v in range(5):
                    cb.state[w][v] = b.states[w][v] if v < len(b.states[w]) else 0.0
    return c


class Oracle:
    """One problem advanced by the CPU oracle."""

    def __init__(self, wl, limiter: bool = True, picard_iters: int = 0, mood: bool = False, flux: int = 0):
        self.wl = wl
        self.cfg = make_config(wl, limiter, picard_iters, mood, flux)
        self.h = lib().or_create(C.byref(self.cfg))
        if not self.h:
            raise ValueError("oracle rejected the configuration")
        self.dim, self.nv, self.n = wl.dim, wl.dim + 2, wl.N + 1
        self.Ns = self.cfg.Ns
        self.ncell = wl.num_cells
        self.nn = self.n ** self.dim
        self.nsub = self.Ns ** self.dim

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_destroy(self.h)
            self.h = None

    # ---- initial data
    def axis_points(self, axis: int, m: int) -> np.ndarray:
        per = self.n if m == 0 else self.Ns * m
        out = np.zeros(self.wl.ncell[axis] * per)
        lib().or_axis_points(self.h, axis, m, _dp(out))
        return out

    def project(self, ic, m: int, t: float = 0.0):
        from paper_1406_7416_amd.workloads import sample_grid
        axes = [self.axis_points(k, m) for k in range(self.dim)]
        samples = np.ascontiguousarray(sample_grid(ic, axes, t))
        u = np.zeros((self.nv, self.ncell, self.nn))
        v = np.zeros((self.nv, self.ncell, self.nsub)) if m > 0 else None
        lib().or_project(self.h, _dp(samples), m, _dp(u), _dp(v) if v is not None else None)
        return u, v

    def set_state(self, u: np.ndarray, v_exact: Optional[np.ndarray] = None) -> int:
        u = np.ascontiguousarray(u, dtype=np.float64)
        ve = None if v_exact is None else np.ascontiguousarray(v_exact, dtype=np.float64)
        return lib().or_set_state(self.h, _dp(u), _dp(ve) if ve is not None else None)

    def init(self, m: Optional[int] = None, detect: bool = True) -> int:
        """Project the workload's initial condition and apply the initial detection."""
        if m is None:
            m = self.n
        u, v = self.project(self.wl.ic, m)
        return self.set_state(u, v if detect else None)

    # ---- stepping
    def cfl_dt(self, cfl: Optional[float] = None) -> float:
        return lib().or_cfl_dt(self.h, self.wl.cfl if cfl is None else cfl)

    def step(self, dt: float) -> int:
        return lib().or_step(self.h, dt)

    def poison(self, cell: int, var: int, value: float):
        """Overwrites variable `var` of cell `cell`'s next candidate with `value` (one step)."""
        if lib().or_poison(self.h, cell, var, value) != 0:
            raise ValueError("poison: cell or variable out of range")

    def mood_stats(self):
        """(flagged subcells, recomputed cells) of the last step's MOOD layer."""
        f, r = C.c_long(), C.c_long()
        lib().or_mood_stats(self.h, C.byref(f), C.byref(r))
        return f.value, r.value

    def set_mask(self, mask: Optional[np.ndarray]):
        """Masked geometry: mask[c] = 1 marks a solid cell (before set_state)."""
        if mask is None:
            lib().or_set_mask(self.h, None)
        else:
            m = np.ascontiguousarray(mask, dtype=np.uint8)
            lib().or_set_mask(self.h, m.ctypes.data_as(C.POINTER(C.c_uint8)))

    def force_troubled(self, mask: Optional[np.ndarray]):
        if mask is None:
            lib().or_force_troubled(self.h, None)
        else:
            m = np.ascontiguousarray(mask, dtype=np.uint8)
            lib().or_force_troubled(self.h, m.ctypes.data_as(C.POINTER(C.c_uint8)))

    @property
    def time(self) -> float:
        return lib().or_time(self.h)

    @time.setter
    def time(self, t: float):
        lib().or_set_time(self.h, t)

    # ---- outputs
    def state(self) -> np.ndarray:
        u = np.zeros((self.nv, self.ncell, self.nn))
        lib().or_get_state(self.h, _dp(u))
        return u

    def troubled(self) -> np.ndarray:
        b = np.zeros(self.ncell, dtype=np.uint8)
        lib().or_get_troubled(self.h, b.ctypes.data_as(C.POINTER(C.c_uint8)))
        return b

    def margin(self) -> np.ndarray:
        m = np.zeros(self.ncell)
        lib().or_get_margin(self.h, _dp(m))
        return m

    def subcells(self) -> np.ndarray:
        v = np.zeros((self.nv, self.ncell, self.nsub))
        lib().or_get_subcells(self.h, _dp(v))
        return v

    def bounds(self):
        lo = np.zeros((self.nv, self.ncell))
        hi = np.zeros((self.nv, self.ncell))
        lib().or_get_bounds(self.h, _dp(lo), _dp(hi))
        return lo, hi

    def nonphysical(self) -> int:
        return lib().or_nonphysical(self.h)


def numerical_flux(d, k, gamma, flux, qL, qR):
    """Numerical flux (0 Rusanov, 1 Osher-type) along axis k between conserved states."""
    dp = C.POINTER(C.c_double)
    qL = np.ascontiguousarray(qL, dtype=np.float64)
    qR = np.ascontiguousarray(qR, dtype=np.float64)
    G = np.zeros(d + 2)
    lib().or_numerical_flux(d, k, gamma, flux, qL.ctypes.data_as(dp), qR.ctypes.data_as(dp), G.ctypes.data_as(dp))
    return G


def abs_jacobian(d, k, gamma, Q, dQ):
    """|A(Q)| dQ for the Euler flux Jacobian along axis k."""
    dp = C.POINTER(C.c_double)
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    dQ = np.ascontiguousarray(dQ, dtype=np.float64)
    out = np.zeros(d + 2)
    lib().or_abs_jacobian(d, k, gamma, Q.ctypes.data_as(dp), dQ.ctypes.data_as(dp), out.ctypes.data_as(dp))
    return out
