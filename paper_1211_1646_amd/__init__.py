"""MPMC hard-disk Monte Carlo on MI355X (HIP, gfx950).

Massively parallel Metropolis Monte Carlo of hard disks after Anderson,
Jankowski, Grubb, Engel and Glotzer (arXiv:1211.1646): checkerboard
sub-sweeps with in-cell trial moves (Alg. 1, 2), random cell shift and
rebuild of the cell lists (Alg. 4), pressure from the contact value of g(r)
(Sec. 4), and the same chain for hard spheres in three dimensions (the
method in d = 3, Sec. 2).  The work runs in libmpmc.so (include/mpmc.h,
include/mpmc_sphere.h); this package only marshals arguments.
"""
from ._lib import (FLAG_ACC, FLAG_ACCEPT_LOG, FLAG_DISK, FLAG_LEAVE,  # noqa: F401
                   FLAG_LEAVE_ONCE, FLAG_NO_PARTICLE_SHUFFLE, FLAG_NO_SET_SHUFFLE, FLAG_TAG,
                   HIST_BINS, MPMCError, load)
from .spheres import (HardSphereSystem, SphereConfig, sphere_geometry,  # noqa: F401
                      sphere_required_bytes)
from .system import (HardDiskBatch, HardDiskSystem, SystemConfig, batch_required_bytes,  # noqa: F401
                     geometry, required_bytes)

__all__ = ["HardDiskSystem", "HardDiskBatch", "SystemConfig", "geometry", "required_bytes",
           "batch_required_bytes", "MPMCError", "FLAG_ACC", "FLAG_ACCEPT_LOG", "FLAG_DISK", "FLAG_NO_PARTICLE_SHUFFLE",
           "FLAG_NO_SET_SHUFFLE", "FLAG_LEAVE", "FLAG_LEAVE_ONCE", "FLAG_TAG", "HIST_BINS", "load", "HardSphereSystem", "SphereConfig",
           "sphere_geometry", "sphere_required_bytes"]
