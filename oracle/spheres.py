"""Python view of the 3D hard-sphere oracle (sphere_oracle.c) -- TEST
INFRASTRUCTURE ONLY."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import build, lib as _lib2d  # noqa: F401  (one shared library)

_L = None


def lib():
    global _L
    if _L is None:
        L = _lib2d()
        vp, u32p, u64p = C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)
        f32p, f64p, i32p, i64p = (C.POINTER(C.c_float), C.POINTER(C.c_double),
                                  C.POINTER(C.c_int), C.POINTER(C.c_int64))
        L.sphere_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                    C.c_int, C.c_double, C.c_float, C.c_int, C.c_uint32,
                                    C.c_uint32, i32p]
        L.sphere_create.restype = vp
        L.sphere_create_grid.argtypes = [C.c_int, C.c_int, C.c_int, C.c_float, C.c_float,
                                         C.c_float, C.c_int64, C.c_float, C.c_int, C.c_uint32,
                                         C.c_uint32, i32p]
        L.sphere_create_grid.restype = vp
        L.sphere_destroy.argtypes = [vp]
        L.sphere_destroy.restype = None
        L.sphere_info.argtypes = [vp, i32p, f32p, i64p]
        L.sphere_info.restype = None
        L.sphere_trial_displacement.argtypes = [C.c_uint32, C.c_uint32, C.c_float, f32p]
        L.sphere_trial_displacement.restype = None
        L.sphere_subsweep_order.argtypes = [vp, C.c_int, C.c_int]
        L.sphere_subsweep_order.restype = None
        L.sphere_sweep_draws.argtypes = [vp, C.c_uint64, i32p, i32p, f32p]
        L.sphere_sweep_draws.restype = None
        L.sphere_shift.argtypes = [vp, C.c_int, C.c_float]
        L.sphere_shift.restype = C.c_int
        L.sphere_sweep.argtypes = [vp, C.c_int64]
        L.sphere_sweep.restype = C.c_int
        L.sphere_get_state.argtypes = [vp, f32p, u32p, u32p, u64p]
        L.sphere_get_state.restype = None
        L.sphere_set_state.argtypes = [vp, f32p, u32p, u32p, C.c_uint64]
        L.sphere_set_state.restype = C.c_int
        L.sphere_counters.argtypes = [vp, u64p, u64p]
        L.sphere_counters.restype = None
        L.sphere_global_positions.argtypes = [vp, f64p]
        L.sphere_global_positions.restype = None
        L.sphere_pair_histogram.argtypes = [vp, u64p]
        L.sphere_pair_histogram.restype = None
        L.sphere_count_overlaps.argtypes = [vp]
        L.sphere_count_overlaps.restype = C.c_int64
        L.sphere_get_acc.argtypes = [vp, f32p]
        L.sphere_get_acc.restype = None
        L.sphere_set_delta.argtypes = [vp, C.c_float]
        L.sphere_set_delta.restype = None
        L.sphere_get_delta.argtypes = [vp]
        L.sphere_get_delta.restype = C.c_float
        _L = L
    return _L


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def trial_displacement(a: int, b: int, delta: float) -> np.ndarray:
    out = np.zeros(3, np.float32)
    lib().sphere_trial_displacement(a, b, delta, _p(out, C.c_float))
    return out


class SphereOracle:
    """Serial checkerboard chain of hard spheres (see sphere_oracle.c)."""

    def __init__(self, handle):
        self._h = handle
        m = np.zeros(3, np.int32)
        w = np.zeros(3, np.float32)
        N = C.c_int64()
        lib().sphere_info(self._h, _p(m, C.c_int), _p(w, C.c_float), C.byref(N))
        self.m, self.w, self.N = m.tolist(), w.copy(), N.value
        self.C = int(np.prod(m))

    @classmethod
    def lattice(cls, nx, ny, nz, eta, cells=(0, 0, 0), w_max=0.0, delta=0.1, n_moves=4,
                seed=1, replica=0):
        st = C.c_int()
        h = lib().sphere_create(nx, ny, nz, eta, cells[0], cells[1], cells[2], w_max, delta,
                                n_moves, seed, replica, C.byref(st))
        if not h:
            raise ValueError("sphere_create failed: %d" % st.value)
        return cls(h)

    @classmethod
    def grid(cls, m, w, N, delta=0.1, n_moves=4, seed=1, replica=0):
        st = C.c_int()
        h = lib().sphere_create_grid(m[0], m[1], m[2], w[0], w[1], w[2], N, delta, n_moves, seed,
                                     replica, C.byref(st))
        if not h:
            raise ValueError("sphere_create_grid failed: %d" % st.value)
        return cls(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().sphere_destroy(h)
            self._h = None

    @property
    def box(self):
        return tuple(float(self.m[a]) * float(self.w[a]) for a in range(3))

    def sweep(self, n=1):
        st = lib().sphere_sweep(self._h, n)
        if st != 0:
            raise RuntimeError("sphere_sweep: capacity violated (%d)" % st)

    def subsweep(self, Q, mode=0):
        lib().sphere_subsweep_order(self._h, Q, mode)

    def shift(self, f, d):
        st = lib().sphere_shift(self._h, f, np.float32(d))
        if st != 0:
            raise RuntimeError("sphere_shift failed (%d)" % st)

    def draws(self, sweep):
        order = np.zeros(8, np.int32)
        f = C.c_int()
        d = C.c_float()
        lib().sphere_sweep_draws(self._h, sweep, _p(order, C.c_int), C.byref(f), C.byref(d))
        return order.tolist(), f.value, np.float32(d.value)

    def get_state(self):
        xyz = np.zeros((self.N, 3), np.float32)
        start = np.zeros(self.C + 1, np.uint32)
        tags = np.zeros(self.N, np.uint32)
        sw = C.c_uint64()
        lib().sphere_get_state(self._h, _p(xyz, C.c_float), _p(start, C.c_uint32),
                               _p(tags, C.c_uint32), C.byref(sw))
        return xyz, start, tags, sw.value

    def set_state(self, xyz, start, tags=None, sweep=0):
        xyz = np.ascontiguousarray(xyz, np.float32)
        start = np.ascontiguousarray(start, np.uint32)
        tp = None
        if tags is not None:
            tags = np.ascontiguousarray(tags, np.uint32)
            tp = _p(tags, C.c_uint32)
        st = lib().sphere_set_state(self._h, _p(xyz, C.c_float), _p(start, C.c_uint32), tp, sweep)
        if st != 0:
            raise ValueError("sphere_set_state rejected the state (%d)" % st)

    def counters(self):
        t, a = C.c_uint64(), C.c_uint64()
        lib().sphere_counters(self._h, C.byref(t), C.byref(a))
        return t.value, a.value

    def global_positions(self):
        out = np.zeros((self.N, 3), np.float64)
        lib().sphere_global_positions(self._h, _p(out, C.c_double))
        return out

    def pair_histogram(self):
        h = np.zeros(200, np.uint64)
        lib().sphere_pair_histogram(self._h, _p(h, C.c_uint64))
        return h

    def count_overlaps(self):
        return int(lib().sphere_count_overlaps(self._h))

    def acc(self):
        """Displacement accumulators [N, 3] in list order."""
        out = np.zeros((self.N, 3), np.float32)
        lib().sphere_get_acc(self._h, _p(out, C.c_float))
        return out

    @property
    def delta(self):
        return np.float32(lib().sphere_get_delta(self._h))

    def set_delta(self, delta):
        lib().sphere_set_delta(self._h, np.float32(delta))
