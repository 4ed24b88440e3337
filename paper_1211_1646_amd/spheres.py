"""Python face of the hard-sphere calls of libmpmc.so (include/mpmc_sphere.h):
the checkerboard chain in three dimensions on one GPU.

The paper states its method for d dimensions (Sec. 2): 8 checkerboard sets,
the 27-cell neighbourhood, 6 shift directions.  Torch provides the device
buffers and a stream; every step runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib as L


@dataclass
class SphereConfig:
    """Parameters of mpmc_sphere_params (sigma = 1)."""
    lattice_nx: int = 0
    lattice_ny: int = 0
    lattice_nz: int = 0
    eta: float = 0.0
    cells_x: int = 0
    cells_y: int = 0
    cells_z: int = 0
    w_max: float = 0.0
    cell_w_x: float = 0.0
    cell_w_y: float = 0.0
    cell_w_z: float = 0.0
    n_particles: int = 0
    delta: float = 0.1
    n_moves: int = 4
    seed: int = 1
    replica: int = 0
    flags: int = 0

    def to_c(self) -> L.SphereParams:
        p = L.SphereParams()
        for name, _ in L.SphereParams._fields_:
            setattr(p, name, getattr(self, name))
        return p


def sphere_geometry(cfg: SphereConfig) -> dict:
    """Derived geometry (host only, no GPU needed)."""
    g = L.SphereGeometry()
    L.check(L.load().mpmc_sphere_geometry_of(C.byref(cfg.to_c()), C.byref(g)))
    return {name: getattr(g, name) for name, _ in L.SphereGeometry._fields_}


def sphere_required_bytes(cfg: SphereConfig) -> dict:
    s = L.SphereBufferSizes()
    L.check(L.load().mpmc_sphere_required_bytes(C.byref(cfg.to_c()), C.byref(s)))
    return {name: getattr(s, name) for name, _ in L.SphereBufferSizes._fields_}


class HardSphereSystem:
    """One system of hard spheres resident on a GPU."""

    def __init__(self, cfg: SphereConfig, device: str = "cuda:0"):
        import torch
        self.cfg = cfg
        self.lib = L.load()
        self.device = torch.device(device)
        sizes = sphere_required_bytes(cfg)
        geo = sphere_geometry(cfg)
        self.geometry = geo
        self.N = int(geo["n_particles"])
        self.m = (geo["cells_x"], geo["cells_y"], geo["cells_z"])
        self.C = int(np.prod(self.m))
        self.w = np.array([geo["w_x"], geo["w_y"], geo["w_z"]], np.float32)

        def buf(n):
            return torch.empty(max(int(n), 256), dtype=torch.uint8, device=self.device)

        self._t = {k: [buf(sizes[k]), buf(sizes[k])] for k in ("pos", "count")}
        self._t["tag"] = [buf(sizes["tag"]), buf(sizes["tag"])] if sizes["tag"] else None
        self._t["acc"] = [buf(sizes["acc"]), buf(sizes["acc"])] if sizes["acc"] else None
        self._work = buf(sizes["work"])
        self._ctl = buf(sizes["ctl"])
        b = L.SphereBuffers()
        for i in range(2):
            b.pos[i] = self._t["pos"][i].data_ptr()
            b.count[i] = self._t["count"][i].data_ptr()
            b.tag[i] = self._t["tag"][i].data_ptr() if self._t["tag"] else None
            b.acc[i] = self._t["acc"][i].data_ptr() if self._t["acc"] else None
        b.work = self._work.data_ptr()
        b.ctl = self._ctl.data_ptr()
        self.stream = torch.cuda.Stream(device=self.device)
        torch.cuda.synchronize(self.device)
        h = C.c_void_p()
        L.check(self.lib.mpmc_sphere_init(C.byref(cfg.to_c()), C.byref(b),
                                          C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self.lib.mpmc_sphere_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ dynamics
    def sweep(self, n: int = 1):
        L.check(self.lib.mpmc_sphere_sweep(self._h, int(n)))

    def subsweep(self, set_index: int):
        L.check(self.lib.mpmc_sphere_subsweep(self._h, int(set_index)))

    def shift(self, f: int = -1, d: float = 0.0):
        L.check(self.lib.mpmc_sphere_shift(self._h, int(f), float(d)))

    def synchronize(self):
        L.check(self.lib.mpmc_sphere_synchronize(self._h))

    def set_launch(self, lanes_per_cell: int):
        """Sub-sweep lanes per active cell (1, 2 or 4); results do not change."""
        L.check(self.lib.mpmc_sphere_set_launch(self._h, int(lanes_per_cell)))

    def set_delta(self, delta: float):
        L.check(self.lib.mpmc_sphere_set_delta(self._h, float(delta)))

    def tune(self, window_sweeps: int, n_windows: int):
        """Plain acceptance tuner: n_windows windows of window_sweeps sweeps,
        delta rescaled towards 30 % acceptance after each (on the device)."""
        L.check(self.lib.mpmc_sphere_tune(self._h, int(window_sweeps), int(n_windows)))

    def delta(self) -> np.float32:
        v = C.c_float()
        L.check(self.lib.mpmc_sphere_get_delta(self._h, C.byref(v)))
        return np.float32(v.value)

    # --------------------------------------------------------------- state
    def get_state(self, with_tags: bool = False):
        """(xyz [N, 3], start [C + 1], sweep) and, with_tags, tags [N]."""
        xyz = np.empty((self.N, 3), np.float32)
        start = np.empty(self.C + 1, np.uint32)
        tags = np.empty(self.N, np.uint32) if with_tags else None
        sw = C.c_uint64()
        L.check(self.lib.mpmc_sphere_get_state(self._h, xyz.ctypes.data, start.ctypes.data,
                                               tags.ctypes.data if with_tags else None,
                                               C.byref(sw)))
        if with_tags:
            return xyz, start, int(sw.value), tags
        return xyz, start, int(sw.value)

    def set_state(self, xyz, start, sweep: int = 0, tags=None):
        xyz = np.ascontiguousarray(xyz, np.float32)
        start = np.ascontiguousarray(start, np.uint32)
        tp = None
        if tags is not None:
            tags = np.ascontiguousarray(tags, np.uint32)
            tp = tags.ctypes.data
        L.check(self.lib.mpmc_sphere_set_state(self._h, xyz.ctypes.data if xyz.size else None,
                                               start.ctypes.data, int(sweep), tp))

    def counters(self):
        t, a = C.c_uint64(), C.c_uint64()
        L.check(self.lib.mpmc_sphere_get_counters(self._h, C.byref(t), C.byref(a)))
        return int(t.value), int(a.value)

    def acc(self):
        """Displacement accumulators [N, 3] in list order (MPMC_FLAG_ACC)."""
        out = np.empty((self.N, 3), np.float32)
        L.check(self.lib.mpmc_sphere_get_acc(self._h, out.ctypes.data))
        return out

    def msd(self) -> float:
        """Mean |acc|^2 over the spheres, reduced on the device in FP64."""
        v = C.c_double()
        L.check(self.lib.mpmc_sphere_msd(self._h, C.byref(v)))
        return v.value

    def reset_acc(self):
        L.check(self.lib.mpmc_sphere_reset_acc(self._h))

    def count_overlaps(self) -> int:
        v = C.c_int64()
        L.check(self.lib.mpmc_sphere_count_overlaps(self._h, C.byref(v)))
        return int(v.value)

    # ------------------------------------------------------------ pressure
    def pair_histogram(self, reset: bool = False):
        L.check(self.lib.mpmc_sphere_pair_histogram(self._h, 1 if reset else 0))

    def pressure(self):
        """(beta P sigma^3, g(sigma+), histogram, number of configurations)."""
        p, g0 = C.c_double(), C.c_double()
        hist = np.zeros(L.HIST_BINS, np.uint64)
        ns = C.c_uint64()
        L.check(self.lib.mpmc_sphere_pressure(self._h, C.byref(p), C.byref(g0),
                                              hist.ctypes.data_as(C.POINTER(C.c_uint64)),
                                              C.byref(ns)))
        return p.value, g0.value, hist, int(ns.value)

    @property
    def density(self) -> float:
        return float(self.geometry["density"])
