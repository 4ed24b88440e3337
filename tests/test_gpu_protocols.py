"""Whole protocols of the benchmark workloads against the oracle, through
the C ABI: the medium workload's tuner + production run with its pressure
estimate, and the 1M-disk benchmark's own set-up and timed launches.
Needs an MI355X; the oracle runs with OpenMP over the cells of each set
(the same chain as the serial one, pinned on the CPU)."""
import math
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import OracleSystem
from oracle import estimator as E

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1211_1646_amd as pkg
    pkg.load()
    return pkg


def assert_same(G, O, what=""):
    gx, gs, gsw = G.get_state()
    ox, os_, osw = O.get_state()
    assert gsw == osw, (what, gsw, osw)
    assert np.array_equal(gs, os_), (what, "cell lists differ", int(np.argmax(gs != os_)))
    bad = np.nonzero(np.any(gx.view(np.uint32) != ox.view(np.uint32), axis=1))[0]
    assert bad.size == 0, (what, "positions differ", bad[:5])
    assert G.counters() == O.counters(), (what, G.counters(), O.counters())


def oracle_tune(O, window, n):
    for _ in range(n):
        t0, a0 = O.counters()
        O.sweep(window)
        t1, a1 = O.counters()
        O.set_delta(oracle.tuned_delta(O.delta, t1 - t0, a1 - a0, O.wx, O.wy))


@pytest.mark.timeout(1200)
def test_medium_workload_protocol(gpu):
    """65,536 disks (256 x 256 lattice) at phi = 0.70, cells at least one
    diameter wide, delta from 0.1 tuned in 200 windows of 10 sweeps (2,000
    sweeps), then 10,000 production sweeps at the frozen delta.  Tuner:
    delta and counters after every window.  Production: counters every 10
    sweeps, the contact histogram of the configuration every 10 sweeps
    (bit-exact), the whole state every 1,000 sweeps, and P* of the
    accumulated histogram within 1e-9 of the FP64 estimator."""
    kw = dict(phi=0.70, w_max=0.0, delta=0.1, n_moves=4, seed=1)
    G = gpu.HardDiskSystem(gpu.SystemConfig(lattice_nx=256, lattice_ny=256, **kw))
    O = OracleSystem.lattice(256, 256, **kw)
    O.set_threads(threads())
    assert (G.mx, G.my) == (O.mx, O.my) == (290, 252)
    for w in range(200):
        G.tune(10, 1)
        oracle_tune(O, 10, 1)
        assert G.delta == O.delta, (w, G.delta, O.delta)
        assert G.counters() == O.counters(), w
    log("  tuned delta %.6f after 2000 sweeps" % float(G.delta))
    assert_same(G, O, "after the tuner")
    hist = np.zeros(200, np.uint64)
    for k in range(1000):
        G.sweep(10)
        O.sweep(10)
        assert G.counters() == O.counters(), k
        G.pair_histogram(reset=(k == 0))
        hist += O.pair_histogram()
        if (k + 1) % 100 == 0:
            assert_same(G, O, "production %d" % (10 * (k + 1)))
            log("  production sweep %d" % (10 * (k + 1)))
    p, g0, hist_g, ns = G.pressure_from_contact()
    assert ns == 1000 and np.array_equal(hist_g, hist)
    Lx, Ly = O.box
    rho = O.N / (Lx * Ly)
    p_ref, g_ref = E.pressure_from_histogram(hist, 1000, O.N, rho)
    assert abs(p - p_ref) <= 1e-9 * abs(p_ref), (p, p_ref)
    log("  P* = %.6f over 10,000 production sweeps" % p)
    assert G.count_overlaps() == 0


@pytest.mark.timeout(1200)
def test_benchmark_setup_and_timed_launches(gpu):
    """The 1M-disk benchmark's path exactly as bench.py runs it: lattice at
    phi = 0.70 with cells narrower than sqrt(2), delta tuned in 20 windows
    of 10 sweeps, the launch shape fixed, 5 extra warm-up sweeps, then 20
    sweeps as graph launches only (a 16-sweep graph and a 4-sweep graph
    captured beforehand): the whole state equals the oracle's after the
    tuner and after the timed sweeps."""
    kw = dict(phi=0.70, w_max=math.sqrt(2.0), delta=0.1, n_moves=4, seed=1)
    G = gpu.HardDiskSystem(gpu.SystemConfig(lattice_nx=1024, lattice_ny=1024, flags=0, **kw))
    O = OracleSystem.lattice(1024, 1024, **kw)
    O.set_threads(threads())
    G.tune(10, 20)
    oracle_tune(O, 10, 20)
    assert G.delta == O.delta
    log("  tuned delta %.6f" % float(G.delta))
    assert_same(G, O, "after the tuner")
    G.set_launch(1, 192)
    G.sweep(5)
    O.sweep(5)
    G.prepare_sweeps(20)
    G.sweep(20)
    O.sweep(20)
    assert_same(G, O, "after the timed sweeps")
    assert G.count_overlaps() == 0
