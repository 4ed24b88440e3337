"""Pins for the oracle's primitives: Philox, the integer and displacement maps,
the visit rule, geometry and the tuner arithmetic.  CPU only."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ Philox
@pytest.fixture(scope="module")
def rocrand_pin(tmp_path_factory):
    """rocRAND's Philox4x32-10 engine, built from its header for the host."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND pin")
    exe = str(tmp_path_factory.mktemp("pin") / "rocrand_philox")
    subprocess.run([hipcc, "-O1", os.path.join(HERE, "pins", "rocrand_philox.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def _rocrand_blocks(exe, cases):
    text = "".join("%x %x %x %x %x %x\n" % (tuple(c) + tuple(k)) for c, k in cases)
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    return [[int(w, 16) for w in line.split()] for line in out.strip().splitlines()]


def test_philox_matches_rocrand(rocrand_pin):
    rng = np.random.default_rng(20121107)
    cases = [([0, 0, 0, 0], [0, 0]),
             ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2),
             ([0xFFFFFFFF, 0xFFFFFFFF, 0, 0], [1, 0]),
             ([0xFFFFFFFF, 7, 0, 0x80000000], [1, 0]),      # sweep-global block
             ([123456, 999, 0, 0x40000000], [1, 0]),        # a shuffle block
             ([589763, 0xFFFFFFFF, 1, 0x00000001], [3, 63])]  # sweep >= 2^32
    for _ in range(200):
        cases.append((rng.integers(0, 2 ** 32, 4, dtype=np.uint64).tolist(),
                      rng.integers(0, 2 ** 32, 2, dtype=np.uint64).tolist()))
    ref = _rocrand_blocks(rocrand_pin, cases)
    for (c, k), r in zip(cases, ref):
        assert oracle.philox(c, k).tolist() == r, (c, k)


def test_philox_counter_and_key_sensitivity():
    base = oracle.philox([5, 6, 7, 8], [1, 2])
    for i in range(4):
        c = [5, 6, 7, 8]
        c[i] ^= 1
        assert (oracle.philox(c, [1, 2]) != base).sum() >= 3
    assert (oracle.philox([5, 6, 7, 8], [1, 3]) != base).sum() >= 3


# ------------------------------------------------------ integer / FP maps
def test_bounded_range_and_extremes():
    for k in range(1, 9):
        assert oracle.bounded(0, k) == 0
        assert oracle.bounded(0xFFFFFFFF, k) == k - 1
        # the boundaries of the k equal parts of [0, 2^32)
        for j in range(1, k):
            edge = -(-(j << 32) // k)  # ceil(j 2^32 / k)
            assert oracle.bounded(edge, k) == j
            assert oracle.bounded(edge - 1, k) == j - 1


def test_displacement_map_exhaustive():
    """Every 16-bit half maps to the midpoint (2h+1-65536)/65536 of a
    sub-interval of (-1, 1), exactly, and the proposal is symmetric."""
    for delta in (np.float32(0.1), np.float32(0.16), np.float32(0.7071)):
        h = np.arange(65536, dtype=np.int64)
        exact = (2 * h + 1 - 65536) / 65536.0
        dx = np.empty(65536, np.float32)
        dy = np.empty(65536, np.float32)
        for v in range(0, 65536):
            a, b = oracle.trial_displacement((v << 16) | (65535 - v), delta)
            dx[v], dy[65535 - v] = a, b
        # single rounding of the exact midpoint times delta
        assert np.array_equal(dx, (exact.astype(np.float32) * delta).astype(np.float32))
        assert np.array_equal(dx, dy)
        assert np.array_equal(dx, -dx[::-1])          # symmetric proposal
        assert np.all(np.abs(dx) < delta)
        assert dx.min() == -dx.max()


def _disk_moves(words, delta):
    out = np.empty((len(words), 2), np.float32)
    for i, w in enumerate(words):
        out[i] = oracle.disk_displacement(int(w), delta)
    return out


def test_disk_displacement_angles_exhaustive():
    """In-circle proposal (Alg. 2's inCircle), angle half: for every one of
    the 65536 angle words, the move points along (2h+1) pi / 65536 to within
    FP32 rounding; flipping bit 15 gives exactly the opposite move and adding
    a quarter (bit 14) turns it exactly by 90 degrees, so the proposal is
    symmetric; its length does not depend on the angle beyond rounding."""
    delta = np.float32(0.16)
    ha = np.arange(65536, dtype=np.uint32)
    for hr in (0, 40000, 65535):
        d = _disk_moves((hr << 16) | ha, delta).astype(np.float64)
        r = float(np.float32(np.sqrt(np.float64((2 * hr + 1) / 131072.0)))) * float(delta)
        theta = (2 * ha.astype(np.float64) + 1) * math.pi / 65536
        assert np.abs(d[:, 0] / r - np.cos(theta)).max() < 3e-7
        assert np.abs(d[:, 1] / r - np.sin(theta)).max() < 3e-7
        opp = d[ha ^ 0x8000]
        assert np.array_equal(opp, -d)
        turned = d[(ha + 0x4000) & 0xFFFF]
        assert np.array_equal(turned[:, 0], -d[:, 1]) and np.array_equal(turned[:, 1], d[:, 0])
        assert np.abs(np.hypot(d[:, 0], d[:, 1]) / r - 1).max() < 4e-7


def test_disk_displacement_radii_exhaustive():
    """Radius half: the squared length of the move, over the 65536 radius
    words at a fixed angle, is uniform on (0, delta^2) -- the fraction of
    words with |move| <= t delta is t^2 to within one word -- so the move is
    uniform in area; every move lies strictly inside the disk."""
    for delta in (np.float32(0.16), np.float32(0.7071)):
        hr = np.arange(65536, dtype=np.uint32)
        for ha in (0x1234, 0xBEEF):
            d = _disk_moves((hr << 16) | ha, delta).astype(np.float64)
            rr = np.hypot(d[:, 0], d[:, 1]) / float(delta)
            assert rr.max() < 1.0 and rr.min() > 0.0
            assert np.all(np.diff(rr) >= -1e-6)          # monotone in the word
            for t in np.linspace(0.05, 1.0, 20):
                frac = np.count_nonzero(rr <= t) / 65536.0
                assert abs(frac - t * t) < 2.0 / 65536 + 1e-6, (t, frac)
        # the same four moves at the centre angle of each quadrant
        q = _disk_moves([(65535 << 16) | (0x2000 + 0x4000 * k) for k in range(4)], delta)
        assert np.array_equal(q[2], -q[0]) and np.array_equal(q[3], -q[1])


def test_visit_rule_paper_example():
    """Sec. 2.3 worked example: n_M = 6 moves over n = 4 particles visit list
    slots [0,1,2,3,0,1]; after the shuffle [1,0,3,2] they visit particles
    [1,0,3,2,1,0], the reverse sequence."""
    slots = oracle.visit_sequence(4, 6)
    assert slots == [0, 1, 2, 3, 0, 1]
    shuffled = [1, 0, 3, 2]
    assert [shuffled[s] for s in slots] == [1, 0, 3, 2, 1, 0]
    assert oracle.visit_sequence(1, 4) == [0, 0, 0, 0]
    assert oracle.visit_sequence(3, 4) == [0, 1, 2, 0]


# ----------------------------------------------------------------- geometry
def test_geometry_small_and_large_workloads():
    g = oracle.geometry(64, 64, 0.60)                       # w >= 1 rule
    assert (g["mx"], g["my"], g["cap"]) == (78, 68, 4)
    assert abs(g["wx"] - 1.00876) < 1e-5 and abs(g["wy"] - 1.00209) < 1e-5
    g = oracle.geometry(256, 256, 0.70)
    assert (g["mx"], g["my"]) == (290, 252)
    g = oracle.geometry(1024, 1024, 0.70, w_max=np.sqrt(2.0))   # w < sqrt(2): cap 4
    assert (g["mx"], g["my"], g["cap"]) == (826, 714, 4)
    for phi, cells in [(0.716, (816, 706)), (0.720, (814, 704))]:
        g = oracle.geometry(1024, 1024, phi, w_max=np.sqrt(2.0))
        assert (g["mx"], g["my"]) == cells
    g = oracle.geometry(1024, 1024, 0.70, w_max=1.932)
    assert (g["mx"], g["my"], g["cap"]) == (604, 524, 7)
    # the box: area N pi / (4 phi), aspect 2/sqrt(3) for a square lattice
    assert abs(g["Lx"] * g["Ly"] - 1024 * 1024 * np.pi / (4 * 0.70)) < 1e-6 * g["Lx"] * g["Ly"]
    assert abs(g["Lx"] / g["Ly"] - 2 / np.sqrt(3)) < 1e-12


def test_capacity_thresholds():
    """Fig. 3: a cell narrower than sqrt(2) sigma holds at most four disks;
    the next thresholds are the optimal 6-, 7- and 8-point packings."""
    def cap_for(w):
        S = oracle.OracleSystem.grid(8, 8, np.float32(w), np.float32(w), delta=0.1)
        return S.cap
    assert cap_for(1.0) == 4
    assert cap_for(1.4141) == 4
    assert cap_for(1.4143) == 5
    assert cap_for(1.6640) == 5
    assert cap_for(1.6642) == 6
    assert cap_for(1.8660) == 6
    assert cap_for(1.8661) == 7
    assert cap_for(1.9318) == 7
    with pytest.raises(ValueError):
        cap_for(1.9319)
    with pytest.raises(ValueError):
        oracle.OracleSystem.grid(6, 7, np.float32(1.2), np.float32(1.2))   # odd grid
    with pytest.raises(ValueError):
        oracle.OracleSystem.grid(2, 8, np.float32(1.2), np.float32(1.2))   # too small
    with pytest.raises(ValueError):
        oracle.OracleSystem.grid(8, 8, np.float32(0.99), np.float32(1.2))  # w < sigma


def test_capacity_bound_is_tight_for_five_points():
    """Five centres with mutual distance >= 1 do fit in a square of side
    sqrt(2) (four corners + centre): the threshold is not conservative."""
    w = np.sqrt(2.0)
    pts = np.array([[0, 0], [w, 0], [0, w], [w, w], [w / 2, w / 2]])
    d = np.sqrt(((pts[:, None] - pts[None]) ** 2).sum(-1))
    assert d[np.triu_indices(5, 1)].min() >= 1.0 - 1e-12


# -------------------------------------------------------------------- tuner
def test_tuner_special_cases():
    wx = wy = np.float32(1.2)
    d = np.float32(0.1)
    assert oracle.tuned_delta(d, 1000, 300, wx, wy) == d            # on target
    assert oracle.tuned_delta(d, 1000, 0, wx, wy) == np.float32(0.05)   # floor 0.5
    assert oracle.tuned_delta(d, 1000, 1000, wx, wy) == np.float32(0.2)  # cap 2
    assert oracle.tuned_delta(d, 0, 0, wx, wy) == d                  # empty window
    assert oracle.tuned_delta(np.float32(0.5), 10, 10, wx, wy) == np.float32(0.6)  # w/2
    assert oracle.tuned_delta(np.float32(0.0015), 10, 0, wx, wy) == np.float32(1e-3)
    # proportional in between
    assert abs(float(oracle.tuned_delta(d, 1000, 450, wx, wy)) - 0.15) < 1e-7
