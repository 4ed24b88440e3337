"""CPU oracle for the MPMC hard-disk chain -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (``paper_1211_1646_amd``)
never does; it shares no code with it.

Contents
  * ``mpmc_oracle.c``  serial checkerboard chain (Alg. 1, 2, 4 of the paper)
  * ``sphere_oracle.c`` the same chain for hard spheres in 3D (``spheres.py``)
  * ``serial_ref.c``   FP64 single-particle Metropolis (statistical reference)
  * ``estimator.py``   FP64 pressure from the contact value (Sec. 4)
  * ``mlp.py``         FP64 move-size network (forward / backward / Adam)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["mpmc_oracle.c", "serial_ref.c", "sphere_oracle.c"]
HIST_BINS = 200


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc: serial, -O2, no FP contraction."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    if not force and os.path.exists(_LIB_PATH):
        built = os.path.getmtime(_LIB_PATH)
        if all(os.path.getmtime(s) <= built for s in srcs):
            return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB_PATH)
        u32p = C.POINTER(C.c_uint32)
        u64p = C.POINTER(C.c_uint64)
        f32p = C.POINTER(C.c_float)
        f64p = C.POINTER(C.c_double)
        i32p = C.POINTER(C.c_int)
        vp = C.c_void_p
        L.oracle_philox.argtypes = [u32p, u32p, u32p]
        L.oracle_philox.restype = None
        L.oracle_bounded.argtypes = [C.c_uint32, C.c_uint32]
        L.oracle_bounded.restype = C.c_uint32
        L.oracle_trial_displacement.argtypes = [C.c_uint32, C.c_float, f32p, f32p]
        L.oracle_trial_displacement.restype = None
        L.oracle_disk_displacement.argtypes = [C.c_uint32, C.c_float, f32p, f32p]
        L.oracle_disk_displacement.restype = None
        L.oracle_visit_sequence.argtypes = [C.c_int, C.c_int, i32p]
        L.oracle_visit_sequence.restype = None
        L.oracle_geometry.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                      C.c_double, C.c_double, i32p, i32p, f32p, f32p,
                                      i32p, f64p, f64p]
        L.oracle_geometry.restype = C.c_int
        L.oracle_create.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                    C.c_double, C.c_double, C.c_float, C.c_int,
                                    C.c_uint32, C.c_uint32, C.c_int, i32p]
        L.oracle_create.restype = vp
        L.oracle_create_grid.argtypes = [C.c_int, C.c_int, C.c_float, C.c_float, C.c_float,
                                         C.c_int, C.c_uint32, C.c_uint32, C.c_int, i32p]
        L.oracle_create_grid.restype = vp
        L.oracle_destroy.argtypes = [vp]
        L.oracle_destroy.restype = None
        L.oracle_info.argtypes = [vp, i32p, i32p, f32p, f32p, i32p, C.POINTER(C.c_int64)]
        L.oracle_info.restype = None
        L.oracle_min_pair_r2.argtypes = [vp]
        L.oracle_min_pair_r2.restype = C.c_float
        L.oracle_set_threads.argtypes = [vp, C.c_int]
        L.oracle_set_threads.restype = C.c_int
        for name, at in [("oracle_set_delta", [vp, C.c_float]),
                         ("oracle_set_seed", [vp, C.c_uint32]),
                         ("oracle_set_n_moves", [vp, C.c_int]),
                         ("oracle_set_cell_order", [vp, C.c_int]),
                         ("oracle_subsweep", [vp, C.c_int]),
                         ("oracle_shift_cells", [vp, C.c_int, C.c_float]),
                         ("oracle_get_counters", [vp, u64p, u64p]),
                         ("oracle_get_state", [vp, f32p, u32p, u64p]),
                         ("oracle_get_aux", [vp, f32p, u32p]),
                         ("oracle_get_accept_log", [vp, u32p]),
                         ("oracle_reset_acc", [vp]),
                         ("oracle_hist_edges", [f32p])]:
            getattr(L, name).argtypes = at
            getattr(L, name).restype = None
        L.oracle_get_delta.argtypes = [vp]
        L.oracle_get_delta.restype = C.c_float
        L.oracle_get_sweep.argtypes = [vp]
        L.oracle_get_sweep.restype = C.c_uint64
        L.oracle_sweep.argtypes = [vp, C.c_int64]
        L.oracle_sweep.restype = C.c_int
        L.oracle_sweep_draws.argtypes = [vp, C.c_uint64, i32p, i32p, f32p]
        L.oracle_sweep_draws.restype = None
        L.oracle_num_particles.argtypes = [vp]
        L.oracle_num_particles.restype = C.c_int64
        L.oracle_set_state.argtypes = [vp, f32p, u32p, C.c_uint64, u32p]
        L.oracle_set_state.restype = C.c_int
        L.oracle_count_overlaps.argtypes = [vp]
        L.oracle_count_overlaps.restype = C.c_int64
        L.oracle_check_capacity.argtypes = [vp]
        L.oracle_check_capacity.restype = C.c_int
        L.oracle_pair_histogram.argtypes = [vp, u64p]
        L.oracle_pair_histogram.restype = C.c_int
        L.oracle_tuned_delta.argtypes = [C.c_float, C.c_uint64, C.c_uint64, C.c_float, C.c_float]
        L.oracle_tuned_delta.restype = C.c_float
        # serial single-particle reference
        L.serial_create.argtypes = [C.c_int64, f64p, f64p, C.c_double, C.c_double,
                                    C.c_double, C.c_uint64]
        L.serial_create.restype = vp
        L.serial_destroy.argtypes = [vp]
        L.serial_destroy.restype = None
        L.serial_run.argtypes = [vp, C.c_int64]
        L.serial_run.restype = None
        L.serial_counters.argtypes = [vp, u64p, u64p]
        L.serial_counters.restype = None
        L.serial_positions.argtypes = [vp, f64p, f64p]
        L.serial_positions.restype = None
        L.serial_pair_histogram.argtypes = [vp, C.c_int, C.c_double, u64p]
        L.serial_pair_histogram.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


# ---------------------------------------------------------------- primitives
def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().oracle_philox(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def bounded(v: int, k: int) -> int:
    return int(lib().oracle_bounded(v, k))


def trial_displacement(word: int, delta: float):
    dx, dy = C.c_float(), C.c_float()
    lib().oracle_trial_displacement(word, delta, C.byref(dx), C.byref(dy))
    return np.float32(dx.value), np.float32(dy.value)


def disk_displacement(word: int, delta: float):
    dx, dy = C.c_float(), C.c_float()
    lib().oracle_disk_displacement(word, delta, C.byref(dx), C.byref(dy))
    return np.float32(dx.value), np.float32(dy.value)


def visit_sequence(n: int, n_moves: int):
    out = np.zeros(n_moves, np.int32)
    lib().oracle_visit_sequence(n, n_moves, _ptr(out, C.c_int))
    return out.tolist()


def hist_edges() -> np.ndarray:
    e = np.zeros(HIST_BINS + 1, np.float32)
    lib().oracle_hist_edges(_ptr(e, C.c_float))
    return e


def tuned_delta(delta, trials, accepts, wx, wy) -> np.float32:
    return np.float32(lib().oracle_tuned_delta(delta, trials, accepts, wx, wy))


def geometry(nx, ny, phi, cells=(0, 0), w_min=1.0, w_max=0.0):
    mx, my, cap = C.c_int(), C.c_int(), C.c_int()
    wx, wy = C.c_float(), C.c_float()
    Lx, Ly = C.c_double(), C.c_double()
    st = lib().oracle_geometry(nx, ny, phi, cells[0], cells[1], w_min, w_max,
                               C.byref(mx), C.byref(my), C.byref(wx), C.byref(wy),
                               C.byref(cap), C.byref(Lx), C.byref(Ly))
    if st != 0:
        raise ValueError("oracle_geometry failed: %d" % st)
    return dict(mx=mx.value, my=my.value, wx=np.float32(wx.value), wy=np.float32(wy.value),
                cap=cap.value, Lx=Lx.value, Ly=Ly.value)


# ------------------------------------------------------------------- system
class OracleSystem:
    """Serial checkerboard chain on host memory (see mpmc_oracle.c)."""

    FLAG_ACC = 1
    FLAG_TAG = 2
    FLAG_DISK = 8
    FLAG_NO_PARTICLE_SHUFFLE = 16
    FLAG_NO_SET_SHUFFLE = 32

    def __init__(self, handle):
        self._h = handle
        L = lib()
        mx, my, cap = C.c_int(), C.c_int(), C.c_int()
        wx, wy = C.c_float(), C.c_float()
        N = C.c_int64()
        L.oracle_info(self._h, C.byref(mx), C.byref(my), C.byref(wx), C.byref(wy),
                      C.byref(cap), C.byref(N))
        self.mx, self.my, self.cap = mx.value, my.value, cap.value
        self.wx, self.wy = np.float32(wx.value), np.float32(wy.value)
        self.C = self.mx * self.my

    @classmethod
    def lattice(cls, nx, ny, phi, cells=(0, 0), w_min=1.0, w_max=0.0, delta=0.1,
                n_moves=4, seed=1, replica=0, flags=0):
        st = C.c_int()
        h = lib().oracle_create(nx, ny, phi, cells[0], cells[1], w_min, w_max, delta,
                                n_moves, seed, replica, flags, C.byref(st))
        if not h:
            raise ValueError("oracle_create failed: %d" % st.value)
        return cls(h)

    @classmethod
    def grid(cls, mx, my, wx, wy, delta=0.1, n_moves=4, seed=1, replica=0, flags=0):
        st = C.c_int()
        h = lib().oracle_create_grid(mx, my, wx, wy, delta, n_moves, seed, replica, flags,
                                     C.byref(st))
        if not h:
            raise ValueError("oracle_create_grid failed: %d" % st.value)
        return cls(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oracle_destroy(h)
            self._h = None

    # -- dynamics
    def sweep(self, n=1):
        st = lib().oracle_sweep(self._h, n)
        if st != 0:
            raise RuntimeError("oracle_sweep: capacity violated (%d)" % st)

    def subsweep(self, Q):
        lib().oracle_subsweep(self._h, Q)

    def shift(self, f, d):
        lib().oracle_shift_cells(self._h, f, np.float32(d))
        if lib().oracle_check_capacity(self._h) != 0:
            raise RuntimeError("oracle shift: capacity violated")

    def draws(self, sweep=None):
        if sweep is None:
            sweep = self.sweep_index
        order = np.zeros(4, np.int32)
        f = C.c_int()
        d = C.c_float()
        lib().oracle_sweep_draws(self._h, sweep, _ptr(order, C.c_int), C.byref(f), C.byref(d))
        return order.tolist(), f.value, np.float32(d.value)

    # -- parameters
    def set_delta(self, delta):
        lib().oracle_set_delta(self._h, delta)

    @property
    def delta(self):
        return np.float32(lib().oracle_get_delta(self._h))

    def set_seed(self, seed):
        lib().oracle_set_seed(self._h, seed)

    def set_n_moves(self, n):
        lib().oracle_set_n_moves(self._h, n)

    def set_threads(self, n):
        """OpenMP threads over the cells of each sub-sweep (the chain is the
        same for any count); returns the count in effect."""
        return int(lib().oracle_set_threads(self._h, int(n)))

    def set_cell_order(self, mode):
        lib().oracle_set_cell_order(self._h, mode)

    @property
    def sweep_index(self):
        return int(lib().oracle_get_sweep(self._h))

    @property
    def N(self):
        return int(lib().oracle_num_particles(self._h))

    # -- state
    def counters(self):
        t, a = C.c_uint64(), C.c_uint64()
        lib().oracle_get_counters(self._h, C.byref(t), C.byref(a))
        return t.value, a.value

    def get_state(self):
        N = self.N
        xy = np.zeros((N, 2), np.float32)
        start = np.zeros(self.C + 1, np.uint32)
        sw = C.c_uint64()
        lib().oracle_get_state(self._h, _ptr(xy, C.c_float), _ptr(start, C.c_uint32), C.byref(sw))
        return xy, start, sw.value

    def set_state(self, xy, start, sweep=0, tag=None):
        xy = np.ascontiguousarray(xy, np.float32)
        start = np.ascontiguousarray(start, np.uint32)
        tp = None
        if tag is not None:
            tag = np.ascontiguousarray(tag, np.uint32)
            tp = _ptr(tag, C.c_uint32)
        st = lib().oracle_set_state(self._h, _ptr(xy, C.c_float), _ptr(start, C.c_uint32),
                                    sweep, tp)
        if st != 0:
            raise ValueError("oracle_set_state rejected the state (%d)" % st)

    def aux(self):
        N = self.N
        acc = np.zeros((N, 2), np.float32)
        tag = np.zeros(N, np.uint32)
        lib().oracle_get_aux(self._h, _ptr(acc, C.c_float), _ptr(tag, C.c_uint32))
        return acc, tag

    def reset_acc(self):
        lib().oracle_reset_acc(self._h)

    def accept_log(self):
        """Bit s of entry c: trial s (s < 32) of cell c's latest update was
        accepted (row-major cells)."""
        out = np.zeros(self.mx * self.my, np.uint32)
        lib().oracle_get_accept_log(self._h, _ptr(out, C.c_uint32))
        return out

    def min_pair_r2(self):
        """Smallest r^2 over ordered neighbour pairs, in the first disk's
        frame (2.0 when there is none)."""
        return float(lib().oracle_min_pair_r2(self._h))

    def count_overlaps(self):
        return int(lib().oracle_count_overlaps(self._h))

    def pair_histogram(self):
        h = np.zeros(HIST_BINS, np.uint64)
        st = lib().oracle_pair_histogram(self._h, _ptr(h, C.c_uint64))
        if st != 0:
            raise ValueError("oracle_pair_histogram: grid too small for the reach")
        return h

    # -- derived
    def global_positions(self):
        """FP64 global coordinates (cell origin + local), list order."""
        xy, start, _ = self.get_state()
        counts = np.diff(start.astype(np.int64))
        cell = np.repeat(np.arange(self.C), counts)
        cx = cell % self.mx
        cy = cell // self.mx
        gx = cx * np.float64(self.wx) + xy[:, 0].astype(np.float64)
        gy = cy * np.float64(self.wy) + xy[:, 1].astype(np.float64)
        return gx, gy

    @property
    def box(self):
        return self.mx * np.float64(self.wx), self.my * np.float64(self.wy)


class SerialReference:
    """FP64 single-particle Metropolis (serial_ref.c)."""

    def __init__(self, x, y, Lx, Ly, delta, seed=12345):
        x = np.ascontiguousarray(x, np.float64)
        y = np.ascontiguousarray(y, np.float64)
        self.N = len(x)
        self._h = lib().serial_create(self.N, _ptr(x, C.c_double), _ptr(y, C.c_double),
                                      Lx, Ly, delta, seed)
        if not self._h:
            raise ValueError("serial_create failed")
        self.Lx, self.Ly = Lx, Ly

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().serial_destroy(h)
            self._h = None

    def run(self, n_trials):
        lib().serial_run(self._h, n_trials)

    def counters(self):
        t, a = C.c_uint64(), C.c_uint64()
        lib().serial_counters(self._h, C.byref(t), C.byref(a))
        return t.value, a.value

    def positions(self):
        x = np.zeros(self.N)
        y = np.zeros(self.N)
        lib().serial_positions(self._h, _ptr(x, C.c_double), _ptr(y, C.c_double))
        return x, y

    def pair_histogram(self, nbins=HIST_BINS, dr=1e-4):
        h = np.zeros(nbins, np.uint64)
        lib().serial_pair_histogram(self._h, nbins, dr, _ptr(h, C.c_uint64))
        return h
