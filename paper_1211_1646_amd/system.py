"""Python face of libmpmc.so: a hard-disk system on one GPU.

Torch provides the device buffers (sized by mpmc_required_bytes) and a
dedicated stream; every step of the simulation runs in the library's HIP
kernels.  Method: Anderson et al., arXiv:1211.1646 (Alg. 1, 2, 4; Sec. 4).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib as L


@dataclass
class SystemConfig:
    """Parameters of mpmc_params (sigma = 1)."""
    lattice_nx: int = 0
    lattice_ny: int = 0
    phi: float = 0.0
    cells_x: int = 0
    cells_y: int = 0
    w_min: float = 1.0
    w_max: float = 0.0
    cell_w_x: float = 0.0
    cell_w_y: float = 0.0
    n_particles: int = 0
    delta: float = 0.1
    n_moves: int = 4
    seed: int = 1
    replica: int = 0
    flags: int = 0

    def to_c(self) -> L.Params:
        p = L.Params()
        for name, _ in L.Params._fields_:
            setattr(p, name, getattr(self, name))
        return p


def geometry(cfg: SystemConfig) -> dict:
    """Derived geometry (host only, no GPU needed)."""
    g = L.Geometry()
    L.check(L.load().mpmc_geometry_of(C.byref(cfg.to_c()), C.byref(g)))
    return {name: getattr(g, name) for name, _ in L.Geometry._fields_}


def required_bytes(cfg: SystemConfig) -> dict:
    s = L.BufferSizes()
    L.check(L.load().mpmc_required_bytes(C.byref(cfg.to_c()), C.byref(s)))
    return {name: getattr(s, name) for name, _ in L.BufferSizes._fields_}


def batch_required_bytes(cfgs) -> dict:
    arr = (L.Params * len(cfgs))(*[c.to_c() for c in cfgs])
    s = L.BufferSizes()
    L.check(L.load().mpmc_batch_required_bytes(arr, len(cfgs), C.byref(s)))
    return {name: getattr(s, name) for name, _ in L.BufferSizes._fields_}


class _Buffers:
    """Caller-owned device buffers for one handle (torch tensors)."""

    def __init__(self, sizes: dict, device):
        import torch

        def buf(n):
            return torch.empty(max(int(n), 256), dtype=torch.uint8, device=device)

        self.t = {k: [buf(sizes[k]), buf(sizes[k])] for k in ("pos", "count")}
        self.t["acc"] = [buf(sizes["acc"]), buf(sizes["acc"])] if sizes["acc"] else None
        self.t["tag"] = [buf(sizes["tag"]), buf(sizes["tag"])] if sizes["tag"] else None
        self.work = buf(sizes["work"])
        self.ctl = buf(sizes["ctl"])
        self.alog = buf(sizes["accept_log"]) if sizes["accept_log"] else None
        b = L.Buffers()
        for i in range(2):
            b.pos[i] = self.t["pos"][i].data_ptr()
            b.count[i] = self.t["count"][i].data_ptr()
            b.acc[i] = self.t["acc"][i].data_ptr() if self.t["acc"] else None
            b.tag[i] = self.t["tag"][i].data_ptr() if self.t["tag"] else None
        b.work = self.work.data_ptr()
        b.ctl = self.ctl.data_ptr()
        b.accept_log = self.alog.data_ptr() if self.alog is not None else None
        self.c = b

    def __getitem__(self, k):
        return self.t[k]


class HardDiskSystem:
    """One system of hard disks resident on a GPU."""

    def __init__(self, cfg: SystemConfig, device: str = "cuda:0"):
        import torch
        self.cfg = cfg
        self.lib = L.load()
        self.device = torch.device(device)
        sizes = required_bytes(cfg)
        self.geometry = geometry(cfg)
        self.N = int(self.geometry["n_particles"])
        self.mx, self.my = self.geometry["cells_x"], self.geometry["cells_y"]
        self.C = self.mx * self.my
        self.wx = np.float32(self.geometry["w_x"])
        self.wy = np.float32(self.geometry["w_y"])
        self.cap = self.geometry["capacity"]
        self._bufs = _Buffers(sizes, self.device)
        self.stream = torch.cuda.Stream(device=self.device)
        torch.cuda.synchronize(self.device)
        h = C.c_void_p()
        L.check(self.lib.mpmc_init_system(C.byref(cfg.to_c()), C.byref(self._bufs.c),
                                          C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self.block = 256
        self.lanes = 1

    # ----------------------------------------------------------- lifecycle
    def close(self):
        if getattr(self, "_h", None):
            self.lib.mpmc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ dynamics
    def sweep(self, n: int = 1, seed: int | None = None):
        L.check(self.lib.mpmc_sweep(self._h, int(n), self.cfg.seed if seed is None else int(seed)))
        if seed is not None:
            self.cfg.seed = int(seed)

    def set_fused(self, on: bool = True):
        """Whole sweeps in one tiled launch where supported (the default), or
        four sub-sweep launches and a rebuild; the chain is the same."""
        L.check(self.lib.mpmc_set_sweep_kernel(self._h, 1 if on else 0))

    @property
    def fused(self) -> bool:
        v = C.c_int32()
        L.check(self.lib.mpmc_get_sweep_kernel(self._h, C.byref(v)))
        return bool(v.value)

    @property
    def fused_tile(self):
        """(compiled tile side, chosen interior tx, ty) of the fused sweep,
        zeros when sweeps do not run fused."""
        v = [C.c_int32() for _ in range(3)]
        L.check(self.lib.mpmc_get_fused_tile(self._h, *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def prepare_sweeps(self, n: int):
        """Capture the graphs a following sweep(n) launches (runs nothing)."""
        L.check(self.lib.mpmc_prepare_sweeps(self._h, int(n)))

    def subsweep(self, set_index: int):
        L.check(self.lib.mpmc_subsweep(self._h, int(set_index)))

    def shift_and_rebin(self, f: int = -1, d: float = 0.0):
        L.check(self.lib.mpmc_shift_and_rebin(self._h, int(f), float(np.float32(d))))

    def tune(self, window_sweeps: int, n_windows: int):
        L.check(self.lib.mpmc_tune(self._h, int(window_sweeps), int(n_windows)))

    def control(self, net, window_sweeps: int, n_windows: int):
        """The learned controller over n_windows windows (see MoveSizeNet)."""
        net.stream.synchronize()
        L.check(self.lib.mpmc_control(self._h, C.c_void_p(net.W.data_ptr()), int(window_sweeps),
                                      int(n_windows)))

    def set_launch(self, lanes_per_cell: int = 1, block_size: int = 256):
        L.check(self.lib.mpmc_set_launch(self._h, int(lanes_per_cell), int(block_size)))
        self.lanes = int(lanes_per_cell)
        self.block = int(block_size)

    AUTOTUNE_CANDIDATES = 12   # lanes {1, 2, 4} x workgroup {64, 128, 192, 256}

    def autotune(self, sweeps: int = 32):
        """Pick the fastest sub-sweep launch shape (results are identical for
        every shape); the chain advances by 2 * sweeps per candidate.
        Returns (lanes per cell, workgroup size, microseconds per sweep)."""
        l, b, us = C.c_int32(), C.c_int32(), C.c_double()
        L.check(self.lib.mpmc_autotune(self._h, int(sweeps), C.byref(l), C.byref(b), C.byref(us)))
        self.lanes = int(l.value)
        self.block = int(b.value)
        return self.lanes, self.block, us.value

    def synchronize(self):
        L.check(self.lib.mpmc_synchronize(self._h))

    # ---------------------------------------------------------- parameters
    @property
    def delta(self) -> np.float32:
        d = C.c_float()
        L.check(self.lib.mpmc_get_delta(self._h, C.byref(d)))
        return np.float32(d.value)

    def set_delta(self, delta: float):
        L.check(self.lib.mpmc_set_delta(self._h, float(np.float32(delta))))

    def set_n_moves(self, n_moves: int):
        """Trial moves per active cell and sub-sweep (changes the chain)."""
        L.check(self.lib.mpmc_set_n_moves(self._h, int(n_moves)))

    # --------------------------------------------------------------- state
    def get_state(self):
        xy = np.empty((self.N, 2), np.float32)
        start = np.empty(self.C + 1, np.uint32)
        sw = C.c_uint64()
        L.check(self.lib.mpmc_get_state(self._h, xy.ctypes.data, start.ctypes.data, C.byref(sw)))
        return xy, start, int(sw.value)

    def set_state(self, xy, start, sweep: int = 0, tags=None):
        xy = np.ascontiguousarray(xy, np.float32)
        start = np.ascontiguousarray(start, np.uint32)
        tp = None
        if tags is not None:
            tags = np.ascontiguousarray(tags, np.uint32)
            tp = tags.ctypes.data
        L.check(self.lib.mpmc_set_state(self._h, xy.ctypes.data if xy.size else None,
                                        start.ctypes.data, int(sweep), tp))

    def aux(self):
        acc = np.zeros((self.N, 2), np.float32) if self._bufs["acc"] else None
        tag = np.zeros(self.N, np.uint32) if self._bufs["tag"] else None
        L.check(self.lib.mpmc_get_aux(self._h, acc.ctypes.data if acc is not None else None,
                                      tag.ctypes.data if tag is not None else None))
        return acc, tag

    def reset_acc(self):
        L.check(self.lib.mpmc_reset_acc(self._h))

    def set_acc(self, acc):
        """Load accumulators [N][2] in the current list order (checkpoint resume)."""
        acc = np.ascontiguousarray(acc, np.float32)
        L.check(self.lib.mpmc_set_acc(self._h, acc.ctypes.data))

    def accept_log(self):
        """Per-cell accept bits of each cell's latest update (row-major)."""
        out = np.zeros(self.C, np.uint32)
        L.check(self.lib.mpmc_get_accept_log(self._h, out.ctypes.data))
        return out

    def msd(self) -> float:
        v = C.c_double()
        L.check(self.lib.mpmc_msd(self._h, C.byref(v)))
        return v.value

    def count_overlaps(self) -> int:
        v = C.c_int64()
        L.check(self.lib.mpmc_count_overlaps(self._h, C.byref(v)))
        return int(v.value)

    def counters(self):
        t, a = C.c_uint64(), C.c_uint64()
        L.check(self.lib.mpmc_get_counters(self._h, C.byref(t), C.byref(a)))
        return int(t.value), int(a.value)

    # ------------------------------------------------------------ pressure
    def pair_histogram(self, reset: bool = False):
        L.check(self.lib.mpmc_pair_histogram(self._h, 1 if reset else 0))

    def pressure_from_contact(self):
        """(P*, g(sigma+), histogram, number of configurations)."""
        p, g0 = C.c_double(), C.c_double()
        hist = np.zeros(L.HIST_BINS, np.uint64)
        ns = C.c_uint64()
        L.check(self.lib.mpmc_pressure_from_contact(
            self._h, C.byref(p), C.byref(g0), hist.ctypes.data_as(C.POINTER(C.c_uint64)),
            C.byref(ns)))
        return p.value, g0.value, hist, int(ns.value)

    @property
    def box(self):
        return self.mx * np.float64(self.wx), self.my * np.float64(self.wy)


class HardDiskBatch:
    """Independent hard-disk systems of uneven N and packing fraction sharing
    one handle: every kernel launch advances all of them, and replica r
    evolves exactly as a HardDiskSystem built from cfgs[r] would."""

    def __init__(self, cfgs, device: str = "cuda:0"):
        import torch
        self.cfgs = list(cfgs)
        self.lib = L.load()
        self.device = torch.device(device)
        sizes = batch_required_bytes(self.cfgs)
        self._bufs = _Buffers(sizes, self.device)
        self.stream = torch.cuda.Stream(device=self.device)
        torch.cuda.synchronize(self.device)
        arr = (L.Params * len(self.cfgs))(*[c.to_c() for c in self.cfgs])
        h = C.c_void_p()
        L.check(self.lib.mpmc_batch_init(arr, len(self.cfgs), C.byref(self._bufs.c),
                                         C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self.block = 256
        self.lanes = 1
        self.R = len(self.cfgs)
        self.geometries = []
        for r in range(self.R):
            g = L.Geometry()
            L.check(self.lib.mpmc_replica_geometry(h, r, C.byref(g)))
            self.geometries.append({name: getattr(g, name) for name, _ in L.Geometry._fields_})
        self.N = sum(int(g["n_particles"]) for g in self.geometries)

    def stats(self, with_msd: bool = False):
        """(trials[R], accepts[R], delta[R], msd[R] or None) of every replica."""
        R = self.R
        tr = np.zeros(R, np.uint64)
        ac = np.zeros(R, np.uint64)
        dl = np.zeros(R, np.float32)
        msd = np.zeros(R, np.float64) if with_msd else None
        L.check(self.lib.mpmc_batch_stats(self._h, tr.ctypes.data, ac.ctypes.data, dl.ctypes.data,
                                          msd.ctypes.data if with_msd else None))
        return tr, ac, dl, msd

    def control(self, net, window_sweeps: int, n_windows: int):
        """The learned controller over n_windows windows (see MoveSizeNet)."""
        net.stream.synchronize()   # parameters written on the network's stream
        L.check(self.lib.mpmc_control(self._h, C.c_void_p(net.W.data_ptr()), int(window_sweeps),
                                      int(n_windows)))

    close = HardDiskSystem.close
    prepare_sweeps = HardDiskSystem.prepare_sweeps
    set_fused = HardDiskSystem.set_fused
    fused = HardDiskSystem.fused
    __del__ = HardDiskSystem.__del__
    subsweep = HardDiskSystem.subsweep
    shift_and_rebin = HardDiskSystem.shift_and_rebin
    tune = HardDiskSystem.tune
    set_launch = HardDiskSystem.set_launch
    autotune = HardDiskSystem.autotune
    AUTOTUNE_CANDIDATES = HardDiskSystem.AUTOTUNE_CANDIDATES
    synchronize = HardDiskSystem.synchronize
    set_delta = HardDiskSystem.set_delta
    set_n_moves = HardDiskSystem.set_n_moves

    def set_replica_n_moves(self, r: int, n_moves: int):
        L.check(self.lib.mpmc_replica_set_n_moves(self._h, int(r), int(n_moves)))
    reset_acc = HardDiskSystem.reset_acc
    count_overlaps = HardDiskSystem.count_overlaps
    counters = HardDiskSystem.counters
    pair_histogram = HardDiskSystem.pair_histogram

    def sweep(self, n: int = 1, seed: int | None = None):
        s = self.cfgs[0].seed if seed is None else int(seed)
        L.check(self.lib.mpmc_sweep(self._h, int(n), s))
        if seed is not None:
            for c in self.cfgs:
                c.seed = int(seed)

    def _cells(self, r):
        g = self.geometries[r]
        return g["cells_x"] * g["cells_y"]

    def get_state(self, r: int):
        n = int(self.geometries[r]["n_particles"])
        xy = np.empty((n, 2), np.float32)
        start = np.empty(self._cells(r) + 1, np.uint32)
        sw = C.c_uint64()
        L.check(self.lib.mpmc_replica_get_state(self._h, int(r), xy.ctypes.data if n else None,
                                                start.ctypes.data, C.byref(sw)))
        return xy, start, int(sw.value)

    def set_state(self, r: int, xy, start, sweep: int = 0, tags=None):
        xy = np.ascontiguousarray(xy, np.float32)
        start = np.ascontiguousarray(start, np.uint32)
        tp = None
        if tags is not None:
            tags = np.ascontiguousarray(tags, np.uint32)
            tp = tags.ctypes.data
        L.check(self.lib.mpmc_replica_set_state(self._h, int(r), xy.ctypes.data if xy.size else None,
                                                start.ctypes.data, int(sweep), tp))

    def set_acc(self, r: int, acc):
        acc = np.ascontiguousarray(acc, np.float32)
        L.check(self.lib.mpmc_replica_set_acc(self._h, int(r), acc.ctypes.data))

    def aux(self, r: int):
        n = int(self.geometries[r]["n_particles"])
        acc = np.zeros((n, 2), np.float32) if self._bufs["acc"] else None
        tag = np.zeros(n, np.uint32) if self._bufs["tag"] else None
        L.check(self.lib.mpmc_replica_get_aux(self._h, int(r),
                                              acc.ctypes.data if acc is not None and n else None,
                                              tag.ctypes.data if tag is not None and n else None))
        return acc, tag

    def accept_log(self, r: int):
        out = np.zeros(self._cells(r), np.uint32)
        L.check(self.lib.mpmc_replica_get_accept_log(self._h, int(r), out.ctypes.data))
        return out

    def msd(self, r: int) -> float:
        v = C.c_double()
        L.check(self.lib.mpmc_replica_msd(self._h, int(r), C.byref(v)))
        return v.value

    def replica_counters(self, r: int):
        t, a = C.c_uint64(), C.c_uint64()
        L.check(self.lib.mpmc_replica_get_counters(self._h, int(r), C.byref(t), C.byref(a)))
        return int(t.value), int(a.value)

    def delta(self, r: int) -> np.float32:
        d = C.c_float()
        L.check(self.lib.mpmc_replica_get_delta(self._h, int(r), C.byref(d)))
        return np.float32(d.value)

    def set_replica_delta(self, r: int, delta: float):
        L.check(self.lib.mpmc_replica_set_delta(self._h, int(r), float(np.float32(delta))))

    def pressure_from_contact(self, r: int):
        p, g0 = C.c_double(), C.c_double()
        hist = np.zeros(L.HIST_BINS, np.uint64)
        ns = C.c_uint64()
        L.check(self.lib.mpmc_replica_pressure_from_contact(
            self._h, int(r), C.byref(p), C.byref(g0), hist.ctypes.data_as(C.POINTER(C.c_uint64)),
            C.byref(ns)))
        return p.value, g0.value, hist, int(ns.value)
