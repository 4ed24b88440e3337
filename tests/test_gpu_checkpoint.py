"""Checkpoint and resume with displacement accumulators, through the C ABI:
state + accumulators + tags taken mid-run and loaded into a fresh handle
continue bit for bit as the uninterrupted run (and as the oracle).  Needs
an MI355X."""
import math

import numpy as np
import pytest

from oracle import OracleSystem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1211_1646_amd as pkg
    pkg.load()
    return pkg


def test_resume_with_accumulators(gpu):
    kw = dict(phi=0.70, w_max=math.sqrt(2.0), delta=0.15, n_moves=4, seed=21)
    A = gpu.HardDiskSystem(gpu.SystemConfig(lattice_nx=48, lattice_ny=48, flags=3, **kw))
    A.sweep(37)
    xy, st, sw = A.get_state()
    acc, tags = A.aux()
    t_mid, a_mid = A.counters()
    B = gpu.HardDiskSystem(gpu.SystemConfig(cells_x=A.mx, cells_y=A.my, cell_w_x=float(A.wx),
                                            cell_w_y=float(A.wy), n_particles=A.N, delta=0.15,
                                            n_moves=4, seed=21, flags=3))
    B.set_state(xy, st, sw, tags)
    B.set_acc(acc)
    A.sweep(29)
    B.sweep(29)
    ax, ast, asw = A.get_state()
    bx, bst, bsw = B.get_state()
    assert asw == bsw == 66 and np.array_equal(ast, bst)
    assert np.array_equal(ax.view(np.uint32), bx.view(np.uint32))
    aa, at = A.aux()
    ba, bt = B.aux()
    assert np.array_equal(at, bt)
    assert np.array_equal(aa.view(np.uint32), ba.view(np.uint32))
    ta, aa_ = A.counters()
    tb, ab = B.counters()
    assert (ta - t_mid, aa_ - a_mid) == (tb, ab)
    assert A.msd() == B.msd()
    # and the oracle from the lattice agrees with both
    O = OracleSystem.lattice(48, 48, flags=3, **kw)
    O.sweep(66)
    ox, ost, _ = O.get_state()
    oa, ot = O.aux()
    assert np.array_equal(ox.view(np.uint32), bx.view(np.uint32))
    assert np.array_equal(oa.view(np.uint32), ba.view(np.uint32))


def test_set_acc_needs_the_flag(gpu):
    from paper_1211_1646_amd import _lib as L
    S = gpu.HardDiskSystem(gpu.SystemConfig(lattice_nx=16, lattice_ny=16, phi=0.5, delta=0.1,
                                            n_moves=4, seed=1, flags=0))
    with pytest.raises(L.MPMCError):
        S.set_acc(np.zeros((S.N, 2), np.float32))
