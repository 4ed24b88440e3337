"""The two cell-leaving pitfalls of Sec. 2.4 in the oracle (diagnostic
variants): moves may leave the cell by up to (w - 1)/2 per axis; the
leave-once form moves every disk exactly once per sweep.  Pins: with cells
exactly one diameter wide the leaving window is empty and the chain is the
plain one, bit for bit; the cells of one set stay independent (any visiting
order gives the same state); nothing is lost, every disk is re-homed into
(0, w] by the shift, no pair overlaps; the leave-once form makes exactly N
trial moves per sweep."""
import math

import numpy as np
import pytest

from oracle import OracleSystem

LEAVE, LEAVE_ONCE = 64, 128


def state(O):
    xy, st, sw = O.get_state()
    return xy.view(np.uint32).copy(), st.copy(), sw


@pytest.mark.parametrize("flag", [LEAVE, LEAVE_ONCE])
def test_leaving_invariants(flag):
    O = OracleSystem.lattice(24, 24, 0.70, w_max=math.sqrt(2.0), delta=0.2, n_moves=4, seed=3,
                             flags=2 | flag)
    N = O.N
    wx, wy = np.float32(O.wx), np.float32(O.wy)
    for k in range(60):
        t0, _ = O.counters()
        O.sweep(1)
        t1, _ = O.counters()
        if flag == LEAVE_ONCE:
            assert t1 - t0 == N, k           # every disk moved (tried) exactly once
        xy, st, _ = O.get_state()
        assert st[-1] == N
        assert np.all(xy[:, 0] > 0) and np.all(xy[:, 0] <= wx)
        assert np.all(xy[:, 1] > 0) and np.all(xy[:, 1] <= wy)
        _, tags = O.aux()
        assert np.array_equal(np.sort(tags), np.arange(N, dtype=np.uint32))
        assert O.count_overlaps() == 0, k


@pytest.mark.parametrize("flag", [LEAVE, LEAVE_ONCE])
def test_leaving_cell_order_does_not_matter(flag):
    runs = []
    for mode in (0, 1, 2):
        O = OracleSystem.lattice(20, 22, 0.72, w_max=math.sqrt(2.0), delta=0.2, n_moves=5,
                                 seed=9, flags=flag)
        O.set_cell_order(mode)
        O.sweep(30)
        runs.append(state(O))
    for r in runs[1:]:
        assert np.array_equal(r[0], runs[0][0]) and np.array_equal(r[1], runs[0][1])


def test_leaving_actually_leaves():
    """Some accepted moves end outside the cell before the shift (else the
    variant would be the plain chain in disguise)."""
    O = OracleSystem.lattice(24, 24, 0.60, w_max=math.sqrt(2.0), delta=0.25, n_moves=4, seed=5,
                             flags=LEAVE)
    P = OracleSystem.lattice(24, 24, 0.60, w_max=math.sqrt(2.0), delta=0.25, n_moves=4, seed=5,
                             flags=0)
    O.sweep(5)
    P.sweep(5)
    assert O.counters()[1] > P.counters()[1]     # more accepts: the in-cell rule is relaxed
    assert not np.array_equal(state(O)[0], state(P)[0])


def test_unit_cells_make_leaving_the_plain_chain():
    """w = 1 exactly: the window (w - 1)/2 is empty, so the leaving variant
    makes exactly the plain chain's decisions and positions."""
    P = OracleSystem.lattice(16, 16, 0.55, w_max=0.0, delta=0.15, n_moves=4, seed=2)
    xy, st, sw = P.get_state()
    a = OracleSystem.grid(P.mx, P.my, 1.0, 1.0, delta=0.15, n_moves=4, seed=2, flags=0)
    b = OracleSystem.grid(P.mx, P.my, 1.0, 1.0, delta=0.15, n_moves=4, seed=2, flags=LEAVE)
    # a state on unit cells: the lattice's disks rescaled into unit cells
    # would overlap, so take every fourth disk of each cell's list
    keep_xy, keep_st = [], [0]
    for c in range(P.mx * P.my):
        sel = xy[st[c]:st[c + 1]][:1]
        sel = np.minimum(sel, np.float32(1.0))
        keep_xy.append(sel)
        keep_st.append(keep_st[-1] + len(sel))
    kxy = np.concatenate(keep_xy).astype(np.float32)
    kst = np.array(keep_st, np.uint32)
    a.set_state(kxy, kst)
    b.set_state(kxy, kst)
    if a.count_overlaps():
        pytest.skip("constructed state overlaps")
    a.sweep(40)
    b.sweep(40)
    assert np.array_equal(state(a)[0], state(b)[0])
    assert np.array_equal(state(a)[1], state(b)[1])
    assert a.counters() == b.counters()
