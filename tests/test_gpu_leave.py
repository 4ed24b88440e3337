"""The two cell-leaving pitfalls of Sec. 2.4 (diagnostic flags) on the GPU
against the oracle, bit for bit, through the C ABI: the sub-sweep with the
widened trial window (and n_M = n for leave-once) and the general rebuild
that re-homes disks on both axes.  Needs an MI355X."""
import math
import sys

import numpy as np
import pytest

from oracle import OracleSystem

pytestmark = pytest.mark.gpu
LEAVE, LEAVE_ONCE = 64, 128


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1211_1646_amd as pkg
    pkg.load()
    return pkg


def same(G, O, what):
    gx, gs, gsw = G.get_state()
    ox, os_, osw = O.get_state()
    assert gsw == osw, (what, gsw, osw)
    assert np.array_equal(gs, os_), (what, "cell lists differ")
    assert np.array_equal(gx.view(np.uint32), ox.view(np.uint32)), (what, "positions differ")
    ga, gt = G.aux()
    oa, ot = O.aux()
    assert np.array_equal(gt, ot), (what, "tags differ")
    assert np.array_equal(ga.view(np.uint32), oa.view(np.uint32)), (what, "accumulators differ")
    assert G.counters() == O.counters(), (what, G.counters(), O.counters())


@pytest.mark.parametrize("flag", [LEAVE, LEAVE_ONCE])
@pytest.mark.parametrize("nx,ny,phi,w_max", [(24, 24, 0.70, math.sqrt(2.0)),
                                             (20, 22, 0.72, 1.932), (40, 40, 0.60, 1.8)])
def test_leaving_matches_oracle(gpu, flag, nx, ny, phi, w_max):
    log("  leave flag %d nx=%d phi=%.2f w_max=%.3f" % (flag, nx, phi, w_max))
    kw = dict(phi=phi, w_max=w_max, delta=0.2, n_moves=4, seed=4)
    G = gpu.HardDiskSystem(gpu.SystemConfig(lattice_nx=nx, lattice_ny=ny, flags=3 | 4 | flag, **kw))
    O = OracleSystem.lattice(nx, ny, flags=3 | 4 | flag, **kw)
    assert not G.fused
    for k in range(20):
        G.sweep(1)
        O.sweep(1)
        assert np.array_equal(G.accept_log(), O.accept_log()), k
        assert G.counters() == O.counters(), k
    same(G, O, "20 sweeps")
    G.sweep(33)
    O.sweep(33)
    same(G, O, "53 sweeps")
    assert G.count_overlaps() == 0


def test_leaving_in_a_mixed_batch(gpu):
    """Replicas with and without the pitfalls share one handle; each
    equals its own oracle run."""
    specs = [(16, 16, 0.66, 0), (24, 24, 0.70, LEAVE), (20, 20, 0.72, LEAVE_ONCE | 8)]
    cfgs = [gpu.SystemConfig(lattice_nx=a, lattice_ny=a, phi=ph, w_max=math.sqrt(2.0), delta=0.15,
                             n_moves=4, seed=6, replica=r, flags=3 | fl)
            for r, (a, _, ph, fl) in enumerate(specs)]
    B = gpu.HardDiskBatch(cfgs)
    B.sweep(29)
    for r, (a, _, ph, fl) in enumerate(specs):
        O = OracleSystem.lattice(a, a, ph, w_max=math.sqrt(2.0), delta=0.15, n_moves=4, seed=6,
                                 replica=r, flags=3 | fl)
        O.sweep(29)
        bx, bs, _ = B.get_state(r)
        ox, os_, _ = O.get_state()
        assert np.array_equal(bs, os_) and np.array_equal(bx.view(np.uint32), ox.view(np.uint32)), r
        assert B.replica_counters(r) == O.counters(), r
