"""ctypes declarations of the C ABI in include/mpmc.h and include/mpmc_sphere.h
(argument marshalling only).

Loading fails loudly when libmpmc.so has not been built: there is no
fallback implementation of any step.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpmc.so")

MPMC_OK = 0
MPMC_EINVAL = -1
MPMC_EGEOM = -2
MPMC_EOVERLAP = -3
MPMC_EHIP = -4
MPMC_EDEVICE = -5
MPMC_ESTATE = -6
FLAG_ACC = 1
FLAG_TAG = 2
FLAG_ACCEPT_LOG = 4
FLAG_DISK = 8        # in-circle trial moves (the paper's proposal)
FLAG_NO_PARTICLE_SHUFFLE = 16  # diagnostic: breaks detailed balance (Table 1)
FLAG_NO_SET_SHUFFLE = 32       # diagnostic: sets always a, b, c, d (Table 1)
FLAG_LEAVE = 64                # diagnostic: moves may leave the cell (Sec. 2.4)
FLAG_LEAVE_ONCE = 128          # diagnostic: leaving allowed, each disk moved once per sweep
HIST_BINS = 200
MLP_PARAMS = 1217

STATUS_NAMES = {0: "MPMC_OK", -1: "MPMC_EINVAL", -2: "MPMC_EGEOM", -3: "MPMC_EOVERLAP",
                -4: "MPMC_EHIP", -5: "MPMC_EDEVICE", -6: "MPMC_ESTATE"}


class Params(C.Structure):
    _fields_ = [("lattice_nx", C.c_int32), ("lattice_ny", C.c_int32), ("phi", C.c_double),
                ("cells_x", C.c_int32), ("cells_y", C.c_int32),
                ("w_min", C.c_double), ("w_max", C.c_double),
                ("cell_w_x", C.c_float), ("cell_w_y", C.c_float),
                ("n_particles", C.c_int64), ("delta", C.c_float), ("n_moves", C.c_int32),
                ("seed", C.c_uint32), ("replica", C.c_uint32), ("flags", C.c_uint32)]


class Geometry(C.Structure):
    _fields_ = [("n_particles", C.c_int64), ("cells_x", C.c_int32), ("cells_y", C.c_int32),
                ("w_x", C.c_float), ("w_y", C.c_float), ("capacity", C.c_int32),
                ("box_x", C.c_double), ("box_y", C.c_double), ("density", C.c_double)]


class BufferSizes(C.Structure):
    _fields_ = [("pos", C.c_size_t), ("count", C.c_size_t), ("acc", C.c_size_t),
                ("tag", C.c_size_t), ("work", C.c_size_t), ("ctl", C.c_size_t),
                ("accept_log", C.c_size_t)]


class Buffers(C.Structure):
    _fields_ = [("pos", C.c_void_p * 2), ("count", C.c_void_p * 2), ("acc", C.c_void_p * 2),
                ("tag", C.c_void_p * 2), ("work", C.c_void_p), ("ctl", C.c_void_p),
                ("accept_log", C.c_void_p)]


class SphereParams(C.Structure):
    _fields_ = [("lattice_nx", C.c_int32), ("lattice_ny", C.c_int32), ("lattice_nz", C.c_int32),
                ("eta", C.c_double), ("cells_x", C.c_int32), ("cells_y", C.c_int32),
                ("cells_z", C.c_int32), ("w_max", C.c_double), ("cell_w_x", C.c_float),
                ("cell_w_y", C.c_float), ("cell_w_z", C.c_float), ("n_particles", C.c_int64),
                ("delta", C.c_float), ("n_moves", C.c_int32), ("seed", C.c_uint32),
                ("replica", C.c_uint32), ("flags", C.c_uint32)]


class SphereGeometry(C.Structure):
    _fields_ = [("n_particles", C.c_int64), ("cells_x", C.c_int32), ("cells_y", C.c_int32),
                ("cells_z", C.c_int32), ("w_x", C.c_float), ("w_y", C.c_float),
                ("w_z", C.c_float), ("box_x", C.c_double), ("box_y", C.c_double),
                ("box_z", C.c_double), ("density", C.c_double)]


class SphereBufferSizes(C.Structure):
    _fields_ = [("pos", C.c_size_t), ("count", C.c_size_t), ("tag", C.c_size_t),
                ("acc", C.c_size_t), ("work", C.c_size_t), ("ctl", C.c_size_t)]


class SphereBuffers(C.Structure):
    _fields_ = [("pos", C.c_void_p * 2), ("count", C.c_void_p * 2), ("tag", C.c_void_p * 2),
                ("acc", C.c_void_p * 2), ("work", C.c_void_p), ("ctl", C.c_void_p)]


class MPMCError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


# name -> (restype, argtypes)
_H = C.c_void_p
_SIGNATURES = {
    "mpmc_geometry_of": (C.c_int32, [C.POINTER(Params), C.POINTER(Geometry)]),
    "mpmc_required_bytes": (C.c_int32, [C.POINTER(Params), C.POINTER(BufferSizes)]),
    "mpmc_init_system": (C.c_int32, [C.POINTER(Params), C.POINTER(Buffers), C.c_void_p,
                                     C.POINTER(C.c_void_p)]),
    "mpmc_sweep": (C.c_int32, [_H, C.c_int64, C.c_uint32]),
    "mpmc_prepare_sweeps": (C.c_int32, [_H, C.c_int64]),
    "mpmc_set_sweep_kernel": (C.c_int32, [_H, C.c_int32]),
    "mpmc_get_sweep_kernel": (C.c_int32, [_H, C.POINTER(C.c_int32)]),
    "mpmc_get_fused_tile": (C.c_int32, [_H, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_int32)]),
    "mpmc_set_acc": (C.c_int32, [_H, C.c_void_p]),
    "mpmc_replica_set_acc": (C.c_int32, [_H, C.c_int32, C.c_void_p]),
    "mpmc_subsweep": (C.c_int32, [_H, C.c_int32]),
    "mpmc_shift_and_rebin": (C.c_int32, [_H, C.c_int32, C.c_float]),
    "mpmc_pair_histogram": (C.c_int32, [_H, C.c_int32]),
    "mpmc_pressure_from_contact": (C.c_int32, [_H, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                               C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "mpmc_get_state": (C.c_int32, [_H, C.c_void_p, C.c_void_p, C.POINTER(C.c_uint64)]),
    "mpmc_set_state": (C.c_int32, [_H, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p]),
    "mpmc_get_aux": (C.c_int32, [_H, C.c_void_p, C.c_void_p]),
    "mpmc_reset_acc": (C.c_int32, [_H]),
    "mpmc_msd": (C.c_int32, [_H, C.POINTER(C.c_double)]),
    "mpmc_count_overlaps": (C.c_int32, [_H, C.POINTER(C.c_int64)]),
    "mpmc_get_counters": (C.c_int32, [_H, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "mpmc_set_delta": (C.c_int32, [_H, C.c_float]),
    "mpmc_get_delta": (C.c_int32, [_H, C.POINTER(C.c_float)]),
    "mpmc_tune": (C.c_int32, [_H, C.c_int32, C.c_int32]),
    "mpmc_set_launch": (C.c_int32, [_H, C.c_int32, C.c_int32]),
    "mpmc_autotune": (C.c_int32, [_H, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_double)]),
    "mpmc_synchronize": (C.c_int32, [_H]),
    "mpmc_batch_required_bytes": (C.c_int32, [C.POINTER(Params), C.c_int32, C.POINTER(BufferSizes)]),
    "mpmc_batch_init": (C.c_int32, [C.POINTER(Params), C.c_int32, C.POINTER(Buffers), C.c_void_p,
                                    C.POINTER(C.c_void_p)]),
    "mpmc_num_replicas": (C.c_int32, [_H, C.POINTER(C.c_int32)]),
    "mpmc_replica_geometry": (C.c_int32, [_H, C.c_int32, C.POINTER(Geometry)]),
    "mpmc_replica_pressure_from_contact": (C.c_int32, [_H, C.c_int32, C.POINTER(C.c_double),
                                                       C.POINTER(C.c_double), C.POINTER(C.c_uint64),
                                                       C.POINTER(C.c_uint64)]),
    "mpmc_replica_get_state": (C.c_int32, [_H, C.c_int32, C.c_void_p, C.c_void_p,
                                           C.POINTER(C.c_uint64)]),
    "mpmc_replica_set_state": (C.c_int32, [_H, C.c_int32, C.c_void_p, C.c_void_p, C.c_uint64,
                                           C.c_void_p]),
    "mpmc_replica_get_aux": (C.c_int32, [_H, C.c_int32, C.c_void_p, C.c_void_p]),
    "mpmc_replica_msd": (C.c_int32, [_H, C.c_int32, C.POINTER(C.c_double)]),
    "mpmc_replica_get_counters": (C.c_int32, [_H, C.c_int32, C.POINTER(C.c_uint64),
                                              C.POINTER(C.c_uint64)]),
    "mpmc_replica_set_delta": (C.c_int32, [_H, C.c_int32, C.c_float]),
    "mpmc_replica_get_delta": (C.c_int32, [_H, C.c_int32, C.POINTER(C.c_float)]),
    "mpmc_batch_stats": (C.c_int32, [_H, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mpmc_get_accept_log": (C.c_int32, [_H, C.c_void_p]),
    "mpmc_set_n_moves": (C.c_int32, [_H, C.c_int32]),
    "mpmc_replica_set_n_moves": (C.c_int32, [_H, C.c_int32, C.c_int32]),
    "mpmc_replica_get_accept_log": (C.c_int32, [_H, C.c_int32, C.c_void_p]),
    "mpmc_control": (C.c_int32, [_H, C.c_void_p, C.c_int32, C.c_int32]),
    "mpmc_mlp_work_bytes": (C.c_int32, [C.c_int32, C.POINTER(C.c_size_t)]),
    "mpmc_mlp_forward": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                     C.c_void_p]),
    "mpmc_mlp_backward": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mpmc_mlp_backward_noalloc": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                              C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mpmc_mlp_mse": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p]),
    "mpmc_adam_step": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                   C.c_float, C.c_float, C.c_float, C.c_float, C.c_int32,
                                   C.c_void_p]),
    "mpmc_sphere_geometry_of": (C.c_int32, [C.POINTER(SphereParams), C.POINTER(SphereGeometry)]),
    "mpmc_sphere_required_bytes": (C.c_int32, [C.POINTER(SphereParams),
                                               C.POINTER(SphereBufferSizes)]),
    "mpmc_sphere_init": (C.c_int32, [C.POINTER(SphereParams), C.POINTER(SphereBuffers),
                                     C.c_void_p, C.POINTER(C.c_void_p)]),
    "mpmc_sphere_sweep": (C.c_int32, [_H, C.c_int64]),
    "mpmc_sphere_subsweep": (C.c_int32, [_H, C.c_int32]),
    "mpmc_sphere_shift": (C.c_int32, [_H, C.c_int32, C.c_float]),
    "mpmc_sphere_get_state": (C.c_int32, [_H, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.POINTER(C.c_uint64)]),
    "mpmc_sphere_set_state": (C.c_int32, [_H, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p]),
    "mpmc_sphere_get_counters": (C.c_int32, [_H, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "mpmc_sphere_set_delta": (C.c_int32, [_H, C.c_float]),
    "mpmc_sphere_get_delta": (C.c_int32, [_H, C.POINTER(C.c_float)]),
    "mpmc_sphere_tune": (C.c_int32, [_H, C.c_int32, C.c_int32]),
    "mpmc_sphere_pair_histogram": (C.c_int32, [_H, C.c_int32]),
    "mpmc_sphere_pressure": (C.c_int32, [_H, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                         C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "mpmc_sphere_count_overlaps": (C.c_int32, [_H, C.POINTER(C.c_int64)]),
    "mpmc_sphere_set_launch": (C.c_int32, [_H, C.c_int32]),
    "mpmc_sphere_get_acc": (C.c_int32, [_H, C.c_void_p]),
    "mpmc_sphere_msd": (C.c_int32, [_H, C.POINTER(C.c_double)]),
    "mpmc_sphere_reset_acc": (C.c_int32, [_H]),
    "mpmc_sphere_synchronize": (C.c_int32, [_H]),
    "mpmc_sphere_destroy": (None, [_H]),
    "mpmc_destroy": (None, [_H]),
    "mpmc_last_error": (C.c_char_p, []),
}

_lib = None


def load() -> C.CDLL:
    """Load libmpmc.so from the package directory; raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmpmc.so is not built (%s); run python -m "
                              "paper_1211_1646_amd.build" % LIB_PATH)
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int) -> None:
    if status != MPMC_OK:
        msg = load().mpmc_last_error()
        raise MPMCError(status, msg.decode() if msg else "")
