"""Learned move-size controller: the network's training and use, driven
through the C ABI (every arithmetic step runs in libmpmc.so's kernels; torch
only holds device buffers and the stream).

The controller chooses the maximum trial displacement delta between
equilibration windows from a replica's packing fraction, mean cell
occupancy and recent acceptance; production then runs with delta frozen, so
the sampled chain is the paper's (Sec. 3.3 leaves d free).

Training data are logged from the sweeps themselves: a batch of replicas,
each at one (packing fraction, delta) pair, runs windows of K sweeps and
reports acceptance and mean-square displacement per sweep; the label of a
packing fraction is the delta of largest displacement per sweep.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import _lib as L

N_PARAMS = L.MLP_PARAMS
DELTA_SCALE = 0.1


def features(phi, occupancy, acceptance) -> np.ndarray:
    """Network inputs (the same centring the in-chain kernel applies)."""
    phi = np.asarray(phi, np.float64)
    return np.stack([20.0 * (phi - 0.7), np.asarray(occupancy, np.float64) - 1.5,
                     4.0 * (np.asarray(acceptance, np.float64) - 0.3)], axis=-1)


def target_of_delta(delta) -> np.ndarray:
    """Network output that maps to delta (delta = 0.1 exp(y))."""
    return np.log(np.asarray(delta, np.float64) / DELTA_SCALE)


def init_params(seed: int = 0, scale: float = 1.0) -> np.ndarray:
    """Seeded initial weights: uniform in +-scale/sqrt(fan_in), zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for rows, cols in ((32, 3), (32, 32), (1, 32)):
        b = scale / math.sqrt(cols)
        out.append(rng.uniform(-b, b, rows * cols))
        out.append(np.zeros(rows))
    return np.concatenate(out).astype(np.float32)


class MoveSizeNet:
    """Parameters, Adam moments and workspaces resident on the GPU."""

    def __init__(self, params: np.ndarray | None = None, device: str = "cuda:0", stream=None):
        import torch
        self.torch = torch
        self.lib = L.load()
        self.device = torch.device(device)
        p = init_params() if params is None else np.asarray(params, np.float32)
        assert p.shape == (N_PARAMS,)
        self.W = torch.from_numpy(p.copy()).to(self.device)
        self.m = torch.zeros(N_PARAMS, dtype=torch.float32, device=self.device)
        self.v = torch.zeros(N_PARAMS, dtype=torch.float32, device=self.device)
        self.g = torch.zeros(N_PARAMS, dtype=torch.float32, device=self.device)
        self.loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        torch.cuda.synchronize(self.device)
        self.step = 0
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self._work = None
        self._work_n = -1

    @property
    def s(self):
        return C.c_void_p(self.stream.cuda_stream)

    def params(self) -> np.ndarray:
        self.stream.synchronize()
        return self.W.cpu().numpy().copy()

    def work(self, n: int):
        if n > self._work_n:
            b = C.c_size_t()
            L.check(self.lib.mpmc_mlp_work_bytes(int(n), C.byref(b)))
            self._work = self.torch.empty(int(b.value), dtype=self.torch.uint8,
                                          device=self.device)
            self._work_n = n
        return self._work

    def forward(self, X, cache=None):
        """Y for device X [n][3] (float32, contiguous)."""
        n = int(X.shape[0])
        Y = self.torch.empty(n, dtype=self.torch.float32, device=self.device)
        L.check(self.lib.mpmc_mlp_forward(ptr(self.W), ptr(X), n, ptr(Y),
                                          ptr(cache) if cache is not None else None, self.s))
        return Y

    def backward(self, X, cache, dY, dX=None):
        n = int(X.shape[0])
        w = self.work(n)
        L.check(self.lib.mpmc_mlp_backward(ptr(self.W), ptr(X), ptr(cache), ptr(dY), n,
                                           ptr(self.g), ptr(dX) if dX is not None else None,
                                           ptr(w), self.s))
        return self.g

    def mse(self, Y, T):
        n = int(Y.shape[0])
        dY = self.torch.empty(n, dtype=self.torch.float32, device=self.device)
        L.check(self.lib.mpmc_mlp_mse(ptr(Y), ptr(T), n, ptr(dY), ptr(self.loss), ptr(self.work(n)),
                                      self.s))
        return dY

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        L.check(self.lib.mpmc_adam_step(ptr(self.W), ptr(self.m), ptr(self.v), ptr(self.g),
                                        N_PARAMS, float(lr), float(b1), float(b2), float(eps),
                                        self.step, self.s))

    def train(self, X, T, steps: int, lr: float = 3e-3, log_every: int = 0):
        """Full-batch Adam on the squared error; returns the loss history
        (one value per log_every steps, read back from the device)."""
        torch = self.torch
        X = torch.as_tensor(X, dtype=torch.float32).to(self.device).contiguous()
        T = torch.as_tensor(T, dtype=torch.float32).to(self.device).contiguous()
        n = int(X.shape[0])
        cache = torch.empty(64 * n, dtype=torch.float32, device=self.device)
        hist = []
        self.stream.wait_stream(torch.cuda.current_stream(self.device))   # the uploads above
        with torch.cuda.stream(self.stream):
            for k in range(steps):
                Y = self.forward(X, cache)
                dY = self.mse(Y, T)
                self.backward(X, cache, dY)
                self.adam(lr=lr)
                if log_every and (k % log_every == 0 or k == steps - 1):
                    self.stream.synchronize()
                    hist.append(float(self.loss.item()))
        self.stream.synchronize()
        return hist


def ptr(t):
    return C.c_void_p(t.data_ptr())


def collect_samples(cfgs, deltas, windows: int, window_sweeps: int, skip: int = 2,
                    device: str = "cuda:0", block: int = 0):
    """Run one batch with a replica per (config, delta) and log, per window of
    window_sweeps sweeps: packing fraction, mean occupancy, acceptance,
    delta and mean-square displacement per sweep.  The first `skip` windows
    are run but not logged.  Returns a dict of numpy arrays (one row per
    replica and logged window) and the seconds the logged sweeps took."""
    import dataclasses
    import time

    from .system import HardDiskBatch
    reps = []
    for c in cfgs:
        for d in deltas:
            reps.append(dataclasses.replace(c, delta=float(d), flags=int(c.flags) | L.FLAG_ACC,
                                            replica=len(reps)))
    B = HardDiskBatch(reps, device=device)
    if block:
        B.set_launch(1, block)
    R = B.R
    phi = np.empty(R)
    occ = np.empty(R)
    for r, g in enumerate(B.geometries):
        phi[r] = g["n_particles"] * math.pi / (4.0 * g["box_x"] * g["box_y"])
        occ[r] = g["n_particles"] / (g["cells_x"] * g["cells_y"])
    rows = []
    tr0 = np.zeros(R, np.uint64)
    ac0 = np.zeros(R, np.uint64)
    tr = np.zeros(R, np.uint64)
    ac = np.zeros(R, np.uint64)
    dl = np.zeros(R, np.float32)
    msd = np.zeros(R, np.float64)

    def stats(with_msd):
        L.check(B.lib.mpmc_batch_stats(B._h, tr.ctypes.data, ac.ctypes.data, dl.ctypes.data,
                                       msd.ctypes.data if with_msd else None))

    seconds = 0.0
    for w in range(skip + windows):
        stats(False)
        tr0[:] = tr
        ac0[:] = ac
        B.reset_acc()
        t0 = time.perf_counter()
        B.sweep(window_sweeps)
        stats(True)
        dt = time.perf_counter() - t0
        if w < skip:
            continue
        seconds += dt
        dtr = (tr - tr0).astype(np.float64)
        a = np.where(dtr > 0, (ac - ac0).astype(np.float64) / np.maximum(dtr, 1), 0.0)
        rows.append(np.stack([phi, occ, a, dl.astype(np.float64), msd / window_sweeps], axis=1))
    B.close()
    data = np.concatenate(rows, axis=0)
    return {"phi": data[:, 0], "occupancy": data[:, 1], "acceptance": data[:, 2],
            "delta": data[:, 3], "msd_per_sweep": data[:, 4]}, seconds


def label_best_delta(samples) -> dict:
    """delta*(phi) = the delta of largest mean displacement per sweep, per
    packing fraction (phi values are grouped after rounding to 1e-6)."""
    key = np.round(samples["phi"], 6)
    best = {}
    for k in np.unique(key):
        sel = key == k
        ds = samples["delta"][sel]
        ms = samples["msd_per_sweep"][sel]
        means = {d: ms[ds == d].mean() for d in np.unique(ds)}
        best[float(k)] = float(max(means, key=means.get))
    return best


def training_set(samples, best):
    """Inputs (features of every logged window) and targets (the output for
    delta*(phi) of that window's packing fraction)."""
    key = np.round(samples["phi"], 6)
    X = features(samples["phi"], samples["occupancy"], samples["acceptance"]).astype(np.float32)
    T = target_of_delta(np.array([best[float(k)] for k in key])).astype(np.float32)
    return X, T


def train_controller(cfgs, deltas, windows: int = 600, window_sweeps: int = 10, skip: int = 5,
                     steps: int = 3000, lr: float = 3e-3, seed: int = 0, device: str = "cuda:0"):
    """Log samples from one batch, label them, train a fresh network on the
    GPU.  Returns (net, info) with the labels, sample count and losses."""
    samples, secs = collect_samples(cfgs, deltas, windows, window_sweeps, skip=skip, device=device)
    best = label_best_delta(samples)
    X, T = training_set(samples, best)
    net = MoveSizeNet(init_params(seed), device=device)
    hist = net.train(X, T, steps, lr=lr, log_every=max(1, steps // 10))
    info = {"samples": int(len(X)), "labels": best, "loss_first": hist[0], "loss_last": hist[-1],
            "collect_seconds": secs}
    return net, info


def equilibrate_and_measure(sys_, mode: str, net=None, eq_windows: int = 50,
                            window_sweeps: int = 10, prod_sweeps: int = 1000,
                            sample_every: int = 10, blocks: int = 10):
    """Equilibrate with the plain tuner ("plain") or the learned controller
    ("learned"), freeze delta, then run prod_sweeps production sweeps timed
    with HIP events on the system's stream.  Returns the displacement per
    second (mean |acc|^2 over the production window / its sweep seconds) and
    P* with the standard error over `blocks` blocks of contact histograms."""
    import torch
    if mode == "plain":
        sys_.tune(window_sweeps, eq_windows)
    elif mode == "learned":
        sys_.control(net, window_sweeps, eq_windows)
    else:
        raise ValueError(mode)
    sys_.synchronize()
    delta = float(sys_.delta if not callable(sys_.delta) else sys_.delta(0))
    sys_.reset_acc()
    per_block = prod_sweeps // blocks
    chunks = per_block // sample_every
    ev = []
    p_blocks = []
    for b in range(blocks):
        first = True
        for k in range(chunks):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(sys_.stream)
            sys_.sweep(sample_every)
            e1.record(sys_.stream)
            ev.append((e0, e1))
            sys_.pair_histogram(reset=first)
            first = False
        p, _, _, _ = (sys_.pressure_from_contact() if not hasattr(sys_, "R")
                      else sys_.pressure_from_contact(0))
        p_blocks.append(p)
    sys_.synchronize()
    secs = sum(a.elapsed_time(b) for a, b in ev) * 1e-3
    msd = sys_.msd() if not hasattr(sys_, "R") else sys_.msd(0)
    p_blocks = np.array(p_blocks)
    return {"mode": mode, "delta": delta, "sweeps": per_block * blocks, "seconds": secs,
            "msd": msd, "msd_per_s": msd / secs, "msd_per_sweep": msd / (per_block * blocks),
            "P": float(p_blocks.mean()),
            "P_se": float(p_blocks.std(ddof=1) / math.sqrt(len(p_blocks)))}


def autotune_moves(sys_, candidates=(1, 2, 4, 8), window_sweeps: int = 64):
    """Choose n_M (trial moves per active cell and sub-sweep) by mean-square
    displacement per second: each candidate runs window_sweeps sweeps from
    the state the previous one left, timed with HIP events on the system's
    stream.  n_M changes the chain, so this belongs to equilibration, like
    the delta tuners; every candidate's chain is a valid one.  The system
    must keep displacement accumulators.  Returns (best n_M, {n_M: MSD/s})."""
    import torch
    rates = {}
    for n in candidates:
        sys_.set_n_moves(int(n))
        sys_.sweep(16)                      # re-capture the graph
        sys_.reset_acc()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        sys_.synchronize()
        e0.record(sys_.stream)
        sys_.sweep(window_sweeps)
        e1.record(sys_.stream)
        e1.synchronize()
        secs = e0.elapsed_time(e1) * 1e-3
        msd = sys_.msd() if not hasattr(sys_, "R") else sum(
            g["n_particles"] * sys_.msd(r) for r, g in enumerate(sys_.geometries)) / sys_.N
        rates[int(n)] = msd / secs
    best = max(rates, key=rates.get)
    sys_.set_n_moves(best)
    return best, rates
