"""Parity of the move-size network's HIP kernels (through the C ABI) with the
FP64 oracle, within error bounds derived from the FP32 arithmetic, and of the
in-chain controller step.  Needs an MI355X.

Error model (u = 2^-24, every FP32 operation rounds once, no contraction):
a length-k sum of products carries at most (k + 1) u times the sum of the
absolute terms; tanh is 1-Lipschitz and its FP32 result is within a few
ulp.  The bounds below propagate those through the layers using the
oracle's FP64 activations, then double them."""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import OracleSystem
from oracle import mlp as M

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1211_1646_amd as pkg
    from paper_1211_1646_amd import controller as ctl
    pkg.load()
    return torch, pkg, ctl


def weights(seed, scale=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.uniform(-scale, scale, M.N_PARAMS).astype(np.float32)
    return w


def inputs(seed, n):
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    return rng.uniform(-2.0, 2.0, size=(n, 3)).astype(np.float32)


def forward_bound(w, X):
    """Per-sample bound on |Y_fp32 - Y_exact| and on the hidden errors."""
    P = M.unpack(w.astype(np.float64))
    X = X.astype(np.float64)
    _, (h1, h2) = M.forward(w.astype(np.float64), X)
    a1 = np.abs(X) @ np.abs(P["W1"]).T + np.abs(P["b1"])
    e1 = 5 * U * a1 + 4 * U                                   # 3 terms + bias, tanh
    a2 = np.abs(h1) @ np.abs(P["W2"]).T + np.abs(P["b2"])
    e2 = 34 * U * a2 + e1 @ np.abs(P["W2"]).T + 4 * U
    a3 = np.abs(h2) @ np.abs(P["W3"]).T + np.abs(P["b3"])
    ey = 34 * U * a3[:, 0] + e2 @ np.abs(P["W3"][0])
    return 2 * ey, 2 * e1, 2 * e2


@pytest.mark.parametrize("n", [1, 63, 64, 65, 3001])
def test_forward_matches_oracle(ctx, n):
    torch, pkg, ctl = ctx
    w = weights(n)
    X = inputs(n, n)
    net = ctl.MoveSizeNet(w)
    Xd = torch.from_numpy(X).cuda()
    cache = torch.empty(64 * n, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(net.stream):
        Y = net.forward(Xd, cache)
    net.stream.synchronize()
    y64, (h1, h2) = M.forward(w.astype(np.float64), X.astype(np.float64))
    ey, e1, e2 = forward_bound(w, X)
    err = np.abs(Y.cpu().numpy().astype(np.float64) - y64)
    assert np.all(err <= ey), (float(err.max()), float(ey[np.argmax(err - ey)]))
    c = cache.cpu().numpy().reshape(64, n).T.astype(np.float64)
    assert np.all(np.abs(c[:, :32] - h1) <= e1)
    assert np.all(np.abs(c[:, 32:] - h2) <= e2)


def backward_bound(w, X, h1, h2, dY, rows):
    """Bounds on |dW_fp32 - dW_exact| and |dX_fp32 - dX_exact| for the
    backward pass from the given FP32 inputs.  1 - h^2 is bounded with
    (1 + h^2) because it cancels near saturation."""
    P = M.unpack(w.astype(np.float64))
    X = np.abs(X.astype(np.float64))
    dy = np.abs(dY.astype(np.float64))[:, None]
    W1, W2, W3 = np.abs(P["W1"]), np.abs(P["W2"]), np.abs(P["W3"][0])
    s1, s2 = 1.0 + h1 * h1, 1.0 + h2 * h2
    dz2 = dy * W3 * np.abs(1.0 - h2 * h2)                     # |dz2|
    e_dz2 = 4 * U * dy * W3 * s2
    dh1 = (dz2 @ W2)                                          # |dh1| bound
    e_dh1 = 33 * U * dh1 + e_dz2 @ W2
    dz1 = dh1 * np.abs(1.0 - h1 * h1)
    e_dz1 = e_dh1 + 4 * U * dh1 * s1
    ks = 64 + rows + 2                                        # summation depth
    parts = {
        "W1": e_dz1.T @ X + ks * U * (dz1.T @ X),
        "b1": e_dz1.sum(0) + ks * U * dz1.sum(0),
        "W2": e_dz2.T @ np.abs(h1) + ks * U * (dz2.T @ np.abs(h1)),
        "b2": e_dz2.sum(0) + ks * U * dz2.sum(0),
        "W3": (ks + 1) * U * (dy.T @ np.abs(h2)),
        "b3": ks * U * dy.sum(0),
    }
    eg = M.pack(parts)
    edX = 33 * U * (dz1 @ W1) + e_dz1 @ W1
    return 2 * eg, 2 * edX


@pytest.mark.parametrize("n", [1, 64, 65, 3001])
def test_backward_matches_oracle(ctx, n):
    """dW and dX against FP64 backpropagation from the same FP32 inputs (the
    oracle's activations rounded to FP32 serve as the cache on both sides),
    within the bound of the backward pass's own roundings."""
    torch, pkg, ctl = ctx
    w = weights(10 + n, 0.6)
    X = inputs(10 + n, n)
    dY = np.random.default_rng(n).normal(size=n).astype(np.float32)
    w64, X64 = w.astype(np.float64), X.astype(np.float64)
    _, (h1, h2) = M.forward(w64, X64)
    h1 = h1.astype(np.float32).astype(np.float64)
    h2 = h2.astype(np.float32).astype(np.float64)
    cache_np = np.ascontiguousarray(np.concatenate([h1, h2], axis=1).T.astype(np.float32))
    net = ctl.MoveSizeNet(w)
    Xd = torch.from_numpy(X).cuda()
    dYd = torch.from_numpy(dY).cuda()
    cache = torch.from_numpy(cache_np.reshape(-1)).cuda()
    dX = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(net.stream):
        net.backward(Xd, cache, dYd, dX)
    net.stream.synchronize()
    g = net.g.cpu().numpy().astype(np.float64)
    g64, dX64 = M.backward(w64, X64, (h1, h2), dY.astype(np.float64))
    eg, edX = backward_bound(w, X, h1, h2, dY, (n + 63) // 64)
    bad = np.abs(g - g64) > eg
    assert not bad.any(), (np.nonzero(bad)[0][:5], (np.abs(g - g64) / (eg + 1e-300)).max())
    assert np.all(np.abs(dX.cpu().numpy().astype(np.float64) - dX64) <= edX + 1e-300)


def test_backward_is_reproducible_and_empty_input(ctx):
    torch, pkg, ctl = ctx
    n = 5000
    w = weights(3, 0.8)
    X = torch.from_numpy(inputs(3, n)).cuda()
    dY = torch.from_numpy(np.random.default_rng(3).normal(size=n).astype(np.float32)).cuda()
    net = ctl.MoveSizeNet(w)
    cache = torch.empty(64 * n, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(net.stream):
        net.forward(X, cache)
        g1 = net.backward(X, cache, dY).clone()
        g2 = net.backward(X, cache, dY).clone()
    net.stream.synchronize()
    assert torch.equal(g1, g2)
    # n = 0: the gradient of an empty sum is zero
    e = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(net.stream):
        g0 = net.backward(e, torch.empty(0, device="cuda"), torch.empty(0, device="cuda")).clone()
    net.stream.synchronize()
    assert torch.count_nonzero(g0).item() == 0


def test_mse_matches_oracle(ctx):
    torch, pkg, ctl = ctx
    n = 4097
    rng = np.random.default_rng(5)
    Y = rng.normal(size=n).astype(np.float32)
    T = rng.normal(size=n).astype(np.float32)
    net = ctl.MoveSizeNet()
    with torch.cuda.stream(net.stream):
        dY = net.mse(torch.from_numpy(Y).cuda(), torch.from_numpy(T).cuda())
    net.stream.synchronize()
    loss64, g64 = M.mse_grad(Y.astype(np.float64), T.astype(np.float64))
    # r = Y - T rounds once, r / n once
    assert np.all(np.abs(dY.cpu().numpy() - g64) <= 2 * U * np.abs(g64) + 1e-45)
    # the squares are formed from the rounded r in FP64
    assert abs(net.loss.item() - loss64) <= 4 * U * loss64


def test_adam_matches_oracle(ctx):
    """Five steps with the same gradients on both sides; each FP32 step adds
    at most a few ulp of the step size, plus the rounding of W."""
    torch, pkg, ctl = ctx
    w = weights(21, 0.5)
    rng = np.random.default_rng(21)
    net = ctl.MoveSizeNet(w)
    w64, m64, v64 = w.astype(np.float64), np.zeros(M.N_PARAMS), np.zeros(M.N_PARAMS)
    lr = 1e-2
    for step in range(1, 6):
        g = rng.normal(size=M.N_PARAMS).astype(np.float32)
        net.g.copy_(torch.from_numpy(g))
        torch.cuda.synchronize()
        with torch.cuda.stream(net.stream):
            net.adam(lr=lr)
        net.stream.synchronize()
        w64, m64, v64 = M.adam_step(w64, m64, v64, g.astype(np.float64), step, lr=lr)
        wg = net.W.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(wg - w64) <= step * (64 * U * lr + 2 * U * np.abs(w64))), step


def test_training_on_gpu_lowers_the_loss(ctx):
    """The oracle's smooth-target problem trained by the HIP kernels."""
    torch, pkg, ctl = ctx
    rng = np.random.Generator(np.random.PCG64(11))
    X = rng.uniform(-1, 1, size=(256, 3))
    T = 0.5 * np.sin(1.5 * X[:, 0]) + 0.3 * X[:, 1] * X[:, 2] - 0.2
    net = ctl.MoveSizeNet(M.init_params(0))
    hist = net.train(X.astype(np.float32), T.astype(np.float32), 1500, lr=3e-3, log_every=500)
    assert hist[-1] < hist[0] / 100, hist


def test_controller_step_matches_oracle(ctx):
    """One window of 12 sweeps in a batch, then the in-chain controller: each
    replica's new delta equals the oracle network's answer for that window's
    counts within the forward bound (the chain before the step is bit-exact,
    so the counts are the oracle's)."""
    torch, pkg, ctl = ctx
    specs = [dict(nx=20, ny=20, phi=0.70, w_max=math.sqrt(2.0), delta=0.15),
             dict(nx=32, ny=32, phi=0.60, w_max=0.0, delta=0.10),
             dict(nx=20, ny=20, phi=0.72, w_max=1.932, delta=0.12),
             dict(nx=24, ny=24, phi=0.66, w_max=0.0, delta=0.30)]
    cfgs = [pkg.SystemConfig(lattice_nx=s["nx"], lattice_ny=s["ny"], phi=s["phi"],
                             w_max=s["w_max"], delta=s["delta"], n_moves=4, seed=1, replica=r,
                             flags=0) for r, s in enumerate(specs)]
    B = pkg.HardDiskBatch(cfgs)
    w = (M.init_params(4, scale=1.5)).astype(np.float32)
    net = ctl.MoveSizeNet(w)
    B.control(net, 12, 1)
    _, _, dl, _ = B.stats()
    for r, s in enumerate(specs):
        O = OracleSystem.lattice(s["nx"], s["ny"], s["phi"], w_max=s["w_max"], delta=s["delta"],
                                 n_moves=4, seed=1, replica=r)
        O.sweep(12)
        t, a = O.counters()
        Lx, Ly = O.box
        phi = O.N * math.pi / (4.0 * Lx * Ly)
        x = M.features(phi, O.N / (O.mx * O.my), a / t).astype(np.float32)
        y, _ = M.forward(w.astype(np.float64), x.astype(np.float64)[None, :])
        ey, _, _ = forward_bound(w, x[None, :])
        d64 = M.delta_from_output(y[0], O.wx, O.wy)
        # exp is monotone: |d - d64| <= d64 (e^ey - 1) plus the final rounding;
        # the FP32 inputs x are the same on both sides up to one rounding each
        # of 20 (phi - 0.7) and friends, covered by doubling ey's input term
        tol = d64 * (math.expm1(float(ey[0]) + 64 * U)) + 2 * U * d64
        log("  replica %d: a=%.4f delta gpu %.7g oracle %.7g tol %.2g" % (r, a / t, dl[r], d64, tol))
        assert abs(float(dl[r]) - d64) <= tol, (r, float(dl[r]), d64, tol)


def test_controller_pipeline_small(ctx):
    """Logged windows -> labels -> training on the GPU -> the controller in the
    chain: samples have the expected shape, labels come from the delta grid,
    the loss falls, and the controlled run keeps delta in range and the
    state overlap-free."""
    torch, pkg, ctl = ctx
    phis = [0.62, 0.70]
    deltas = [0.05, 0.10, 0.20]
    base = [pkg.SystemConfig(lattice_nx=24, lattice_ny=24, phi=p, w_max=math.sqrt(2.0), n_moves=4,
                             seed=1) for p in phis]
    samples, secs = ctl.collect_samples(base, deltas, windows=6, window_sweeps=10, skip=2)
    assert len(samples["phi"]) == len(phis) * len(deltas) * 6 and secs > 0
    assert np.all((samples["acceptance"] >= 0) & (samples["acceptance"] <= 1))
    assert np.all(samples["msd_per_sweep"] > 0)
    best = ctl.label_best_delta(samples)
    assert len(best) == 2 and all(min(abs(v - d) for d in deltas) < 1e-6 for v in best.values())
    X, T = ctl.training_set(samples, best)
    net = ctl.MoveSizeNet(ctl.init_params(0))
    hist = net.train(X, T, 300, lr=3e-3, log_every=100)
    assert hist[-1] < hist[0]
    S = pkg.HardDiskSystem(pkg.SystemConfig(lattice_nx=32, lattice_ny=32, phi=0.68,
                                            w_max=math.sqrt(2.0), delta=0.1, n_moves=4, seed=2))
    S.control(net, 10, 5)
    d = float(S.delta)
    assert 1e-3 <= d <= 0.5 * min(float(S.wx), float(S.wy))
    assert S.count_overlaps() == 0


def test_n_moves_autotuner(ctx):
    torch, pkg, ctl = ctx
    S = pkg.HardDiskSystem(pkg.SystemConfig(lattice_nx=64, lattice_ny=64, phi=0.66,
                                            w_max=math.sqrt(2.0), delta=0.12, n_moves=4, seed=3,
                                            flags=pkg.FLAG_ACC))
    best, rates = ctl.autotune_moves(S, (1, 4, 8), window_sweeps=32)
    assert best in (1, 4, 8) and set(rates) == {1, 4, 8}
    assert all(v > 0 for v in rates.values()) and rates[best] == max(rates.values())
    t0, _ = S.counters()
    S.sweep(1)
    t1, _ = S.counters()
    assert t1 > t0 and S.count_overlaps() == 0
