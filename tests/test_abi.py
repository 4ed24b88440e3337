"""The C-ABI library: it loads, exports every declared symbol, and its host-side
logic (geometry, buffer sizes, argument checks) agrees with the oracle.
No GPU calls."""
import math
import os
import re

import numpy as np
import pytest

import oracle
import paper_1211_1646_amd as pkg
from paper_1211_1646_amd import _lib as L
from paper_1211_1646_amd.system import SystemConfig, geometry, required_bytes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(mpmc_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = _declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L._SIGNATURES), set(names) ^ set(L._SIGNATURES)


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes field sits at the offset the C compiler gives it."""
    import ctypes as C
    import subprocess
    structs = {"mpmc_params": L.Params, "mpmc_geometry": L.Geometry,
               "mpmc_buffer_sizes": L.BufferSizes, "mpmc_buffers": L.Buffers}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mpmc.h"', "int main(void){"]
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


@pytest.mark.parametrize("nx,phi,w_min,w_max", [
    (64, 0.60, 1.0, 0.0), (256, 0.70, 1.0, 0.0), (1024, 0.70, 1.0, math.sqrt(2.0)),
    (1024, 0.716, 1.0, math.sqrt(2.0)), (1024, 0.72, 1.0, math.sqrt(2.0)),
    (1024, 0.70, 1.0, 1.932), (96, 0.65, 1.0, 0.0), (500, 0.73, 1.0, 0.0), (20, 0.45, 1.2, 0.0)])
def test_geometry_agrees_with_oracle(nx, phi, w_min, w_max):
    g = geometry(SystemConfig(lattice_nx=nx, lattice_ny=nx, phi=phi, w_min=w_min, w_max=w_max))
    o = oracle.geometry(nx, nx, phi, w_min=w_min, w_max=w_max)
    assert (g["cells_x"], g["cells_y"], g["capacity"]) == (o["mx"], o["my"], o["cap"])
    assert np.float32(g["w_x"]) == o["wx"] and np.float32(g["w_y"]) == o["wy"]
    assert g["n_particles"] == nx * nx
    assert g["box_x"] == g["cells_x"] * np.float64(o["wx"])
    assert abs(g["density"] * np.pi / 4 - phi) < 1e-6


def test_required_bytes():
    cfg = SystemConfig(lattice_nx=64, lattice_ny=64, phi=0.6, flags=pkg.FLAG_ACC | pkg.FLAG_TAG)
    s = required_bytes(cfg)
    g = geometry(cfg)
    N, C = g["n_particles"], g["cells_x"] * g["cells_y"]
    cap = g["capacity"]
    assert s["pos"] >= 8 * C * cap and s["acc"] >= 8 * C * cap and s["tag"] >= 4 * C * cap
    assert s["count"] >= 4 * C
    assert all(v % 256 == 0 for v in s.values())
    assert required_bytes(SystemConfig(lattice_nx=64, lattice_ny=64, phi=0.6))["acc"] == 0


@pytest.mark.parametrize("kw,status", [
    (dict(lattice_nx=8, lattice_ny=7, phi=0.5), L.MPMC_EINVAL),          # odd rows
    (dict(lattice_nx=8, lattice_ny=8, phi=0.95), L.MPMC_EINVAL),         # phi too large
    (dict(lattice_nx=4, lattice_ny=4, phi=0.7), L.MPMC_EGEOM),           # grid < 4
    (dict(lattice_nx=64, lattice_ny=64, phi=0.6, cells_x=77), L.MPMC_EGEOM),   # odd grid
    (dict(lattice_nx=64, lattice_ny=64, phi=0.6, cells_x=80), L.MPMC_EGEOM),   # w < 1
    (dict(lattice_nx=64, lattice_ny=64, phi=0.6, w_min=2.0), L.MPMC_EGEOM),    # w > 1.932
    (dict(cells_x=6, cells_y=6, cell_w_x=1.2, cell_w_y=0.9, n_particles=4), L.MPMC_EGEOM),
    (dict(cells_x=4, cells_y=4, cell_w_x=1.2, cell_w_y=1.2, n_particles=65), L.MPMC_EGEOM),
])
def test_geometry_errors(kw, status):
    with pytest.raises(L.MPMCError) as e:
        geometry(SystemConfig(**kw))
    assert e.value.status == status
    assert L.load().mpmc_last_error()


def test_package_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        L.load()


def test_library_exports_nothing_but_the_c_abi():
    """The internal C++ launch helpers stay out of the dynamic symbol table."""
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    names = [ln.split()[-1] for ln in out.splitlines() if ln.split()[1:2] == ["T"]]
    assert names and all(n.startswith("mpmc_") for n in names), [n for n in names
                                                                  if not n.startswith("mpmc_")]


def _batch_sizes(cfgs):
    import ctypes as C
    arr = (L.Params * max(len(cfgs), 1))(*[c.to_c() for c in cfgs])
    s = L.BufferSizes()
    st = L.load().mpmc_batch_required_bytes(arr, len(cfgs), C.byref(s))
    return st, s


def test_batch_required_bytes_covers_the_replicas():
    """Padded layout: cells rounded up (with at least one spare) to 256 per
    replica, the largest capacity's slots per cell; one control block per
    replica."""
    from paper_1211_1646_amd import workloads as W
    specs = W.replicas(8, seed=3)
    cfgs = [SystemConfig(lattice_nx=s["nx"], lattice_ny=s["ny"], phi=s["phi"], delta=0.1,
                         replica=r, flags=pkg.FLAG_ACC | pkg.FLAG_TAG | L.FLAG_ACCEPT_LOG)
            for r, s in enumerate(specs)]
    st, s = _batch_sizes(cfgs)
    assert st == L.MPMC_OK
    cells, cap = 0, 0
    for c in cfgs:
        g = geometry(c)
        C_r = g["cells_x"] * g["cells_y"]
        cells += (C_r + 1 + 255) // 256 * 256
        cap = max(cap, g["capacity"])
    # slots: the largest capacity per cell, for every (padded) cell
    assert s.pos >= 8 * cells * cap and s.pos < 8 * cells * cap + 256
    assert s.acc == s.pos and s.tag >= 4 * cells * cap
    assert s.count >= 4 * cells and s.count < 4 * cells + 256
    assert s.accept_log >= 4 * cells
    single = required_bytes(cfgs[0])
    assert single["ctl"] < s.ctl
    # one replica: the batch sizes are the single-system sizes
    st1, s1 = _batch_sizes(cfgs[:1])
    assert st1 == L.MPMC_OK and s1.pos == single["pos"] and s1.ctl == single["ctl"]


def test_batch_argument_errors():
    a = SystemConfig(lattice_nx=16, lattice_ny=16, phi=0.6, delta=0.1)
    b = SystemConfig(lattice_nx=20, lattice_ny=20, phi=0.7, delta=0.1, flags=pkg.FLAG_ACC)
    assert _batch_sizes([])[0] == L.MPMC_EINVAL                      # no replica
    assert _batch_sizes([a, b])[0] == L.MPMC_EINVAL                  # flags differ
    bad = SystemConfig(lattice_nx=16, lattice_ny=15, phi=0.6, delta=0.1)
    assert _batch_sizes([a, bad])[0] == L.MPMC_EINVAL                # odd rows
    wide = SystemConfig(lattice_nx=16, lattice_ny=16, phi=0.6, cells_x=4, cells_y=4, delta=0.1)
    assert _batch_sizes([a, wide])[0] == L.MPMC_EGEOM                # cells too wide
    big_delta = SystemConfig(lattice_nx=16, lattice_ny=16, phi=0.6, delta=0.9)
    assert _batch_sizes([a, big_delta])[0] == L.MPMC_EINVAL          # delta > w/2
    assert L.load().mpmc_last_error()
    # the proposal may differ between replicas; other flags may not
    d = SystemConfig(lattice_nx=20, lattice_ny=20, phi=0.7, delta=0.1, flags=pkg.FLAG_DISK)
    assert _batch_sizes([a, d])[0] == L.MPMC_OK
    ad = SystemConfig(lattice_nx=20, lattice_ny=20, phi=0.7, delta=0.1,
                      flags=pkg.FLAG_DISK | pkg.FLAG_ACC)
    assert _batch_sizes([d, ad])[0] == L.MPMC_EINVAL
    ab = SystemConfig(lattice_nx=20, lattice_ny=20, phi=0.7, delta=0.1,
                      flags=pkg.FLAG_NO_PARTICLE_SHUFFLE | pkg.FLAG_NO_SET_SHUFFLE)
    assert _batch_sizes([a, d, ab])[0] == L.MPMC_OK
    lv = SystemConfig(lattice_nx=16, lattice_ny=16, phi=0.6, delta=0.1,
                      flags=pkg.FLAG_LEAVE | pkg.FLAG_LEAVE_ONCE)
    assert _batch_sizes([a, lv])[0] == L.MPMC_OK                     # chain flags may differ
    unknown = SystemConfig(lattice_nx=16, lattice_ny=16, phi=0.6, delta=0.1, flags=256)
    assert _batch_sizes([unknown])[0] == L.MPMC_EINVAL


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "4"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
