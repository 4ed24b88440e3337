"""The hard-sphere calls of the C-ABI library (include/mpmc_sphere.h): struct
layouts, and host-side geometry, buffer sizes and argument checks against
the 3D oracle.  No GPU calls."""
import ctypes as C
import math
import os
import subprocess

import numpy as np
import pytest

from oracle.spheres import SphereOracle
from paper_1211_1646_amd import _lib as L
from paper_1211_1646_amd.spheres import SphereConfig, sphere_geometry, sphere_required_bytes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_sphere_struct_layouts_match_header(tmp_path):
    structs = {"mpmc_sphere_params": L.SphereParams, "mpmc_sphere_geometry": L.SphereGeometry,
               "mpmc_sphere_buffer_sizes": L.SphereBufferSizes,
               "mpmc_sphere_buffers": L.SphereBuffers}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mpmc_sphere.h"',
             "int main(void){"]
    for cname, cls in structs.items():
        lines.append('printf("%%s %%zu\\n", "%s", sizeof(%s));' % (cname, cname))
        for fname, _ in cls._fields_:
            lines.append('printf("%%s.%%s %%zu\\n", "%s", "%s", offsetof(%s, %s));'
                         % (cname, fname, cname, fname))
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = dict(line.rsplit(" ", 1) for line in
               subprocess.run([str(exe)], capture_output=True, text=True).stdout.split("\n") if line)
    for cname, cls in structs.items():
        assert int(out[cname]) == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(out["%s.%s" % (cname, fname)]) == getattr(cls, fname).offset, (cname, fname)


@pytest.mark.parametrize("n,eta,w_max", [
    ((10, 10, 10), 0.3, 0.0), ((8, 10, 12), 0.45, 0.0), ((12, 12, 12), 0.5, 0.0),
    ((20, 20, 20), 0.1, 0.0), ((16, 16, 16), 0.4, 1.1), ((100, 100, 100), 0.45, 0.0),
    ((6, 6, 6), math.pi / 6, 0.0)])
def test_sphere_geometry_agrees_with_oracle(n, eta, w_max):
    g = sphere_geometry(SphereConfig(lattice_nx=n[0], lattice_ny=n[1], lattice_nz=n[2], eta=eta,
                                     w_max=w_max, delta=0.1))
    o = SphereOracle.lattice(*n, eta, w_max=w_max, delta=0.1)
    assert (g["cells_x"], g["cells_y"], g["cells_z"]) == tuple(o.m)
    assert np.array_equal(np.float32([g["w_x"], g["w_y"], g["w_z"]]), o.w)
    assert g["n_particles"] == n[0] * n[1] * n[2] == o.N
    assert abs(g["density"] * math.pi / 6 - eta) < 1e-6 * eta + 1e-9


def test_sphere_required_bytes():
    cfg = SphereConfig(lattice_nx=10, lattice_ny=10, lattice_nz=10, eta=0.3, flags=L.FLAG_TAG)
    g = sphere_geometry(cfg)
    C_ = g["cells_x"] * g["cells_y"] * g["cells_z"]
    s = sphere_required_bytes(cfg)
    assert s["pos"] >= 16 * 8 * C_ and s["pos"] % 256 == 0
    assert s["count"] >= 4 * C_ and s["tag"] >= 4 * 8 * C_
    assert s["ctl"] > 0 and s["work"] > 0
    s0 = sphere_required_bytes(SphereConfig(lattice_nx=10, lattice_ny=10, lattice_nz=10, eta=0.3))
    assert s0["tag"] == 0 and s0["acc"] == 0
    s1 = sphere_required_bytes(SphereConfig(lattice_nx=10, lattice_ny=10, lattice_nz=10, eta=0.3,
                                            flags=L.FLAG_ACC))
    assert s1["acc"] == s1["pos"] and s1["work"] >= 8 * ((C_ + 255) // 256)


@pytest.mark.parametrize("kw,status", [
    (dict(lattice_nx=10, lattice_ny=10, lattice_nz=10, eta=0.6), L.MPMC_EINVAL),
    (dict(lattice_nx=10, lattice_ny=10, lattice_nz=10, eta=0.3, flags=L.FLAG_DISK), L.MPMC_EINVAL),
    (dict(lattice_nx=10, lattice_ny=10, lattice_nz=10, eta=0.3, delta=0.6), L.MPMC_EINVAL),
    (dict(lattice_nx=10, lattice_ny=10, lattice_nz=10, eta=0.3, n_moves=-1), L.MPMC_EINVAL),
    (dict(lattice_nx=10, lattice_ny=10, lattice_nz=10, eta=0.3, cells_x=13), L.MPMC_EGEOM),
    (dict(lattice_nx=10, lattice_ny=10, lattice_nz=10, eta=0.3, cells_x=6), L.MPMC_EGEOM),
    (dict(cells_x=4, cells_y=4, cells_z=2, cell_w_x=1.1, cell_w_y=1.1, cell_w_z=1.1), L.MPMC_EGEOM),
    (dict(cells_x=4, cells_y=4, cells_z=4, cell_w_x=1.2, cell_w_y=1.1, cell_w_z=1.1), L.MPMC_EGEOM),
    (dict(cells_x=4, cells_y=4, cells_z=4, cell_w_x=0.99, cell_w_y=1.1, cell_w_z=1.1), L.MPMC_EGEOM),
    (dict(cells_x=4, cells_y=4, cells_z=4, cell_w_x=1.1, cell_w_y=1.1, cell_w_z=1.1,
          n_particles=513), L.MPMC_EINVAL)])
def test_sphere_geometry_errors(kw, status):
    kw.setdefault("delta", 0.1)
    with pytest.raises(L.MPMCError) as e:
        sphere_geometry(SphereConfig(**kw))
    assert e.value.status == status
