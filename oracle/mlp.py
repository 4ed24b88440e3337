"""FP64 oracle of the learned move-size controller -- TEST INFRASTRUCTURE ONLY.

The controller is not part of the paper's method: it only chooses the
maximum trial displacement delta (the free parameter d of Sec. 3.3) during
equilibration, and delta is frozen before production, so the chain that is
sampled is the paper's.  This module is the plain definition of what the HIP
kernels compute, written out in FP64 with numpy:

  * the network: 3 -> 32 -> 32 -> 1, tanh on both hidden layers, linear
    output;
  * reverse-mode gradients of a given output gradient dY (backpropagation);
  * Adam (Kingma and Ba, ICLR 2015, Algorithm 1) with bias correction;
  * the controller's features of a replica and the map from network output
    to delta.

Parameters are one flat vector of 1217 values in this order (row-major, rows
are outputs): W1[32][3], b1[32], W2[32][32], b2[32], W3[1][32], b3[1].
"""
from __future__ import annotations

import math

import numpy as np

N_IN, N_H, N_OUT = 3, 32, 1
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)   # 1217

DELTA_SCALE = 0.1     # delta = DELTA_SCALE * exp(y)
DELTA_MIN = 1e-3


def unpack(w):
    """Views of the flat parameter vector as the six arrays."""
    w = np.asarray(w, dtype=np.float64)
    assert w.shape == (N_PARAMS,)
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = w[o:o + n].reshape(shape)
        o += n
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], np.float64).reshape(-1) for name, _ in SHAPES])


def init_params(seed: int = 0, scale: float = 1.0) -> np.ndarray:
    """Seeded initial weights: uniform in +-scale/sqrt(fan_in), zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            bound = scale / math.sqrt(shape[1])
            parts[name] = rng.uniform(-bound, bound, size=shape)
        else:
            parts[name] = np.zeros(shape)
    return pack(parts).astype(np.float32)


def forward(w, X):
    """Y[n] and the cache (h1[n][32], h2[n][32]) of the network on X[n][3]."""
    P = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ P["W1"].T + P["b1"])
    h2 = np.tanh(h1 @ P["W2"].T + P["b2"])
    y = h2 @ P["W3"].T + P["b3"]
    return y[:, 0], (h1, h2)


def backward(w, X, cache, dY):
    """Gradients (dW flat [1217], dX [n][3]) of sum_i dY_i * Y_i."""
    P = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    h1, h2 = cache
    dy = np.asarray(dY, dtype=np.float64)[:, None]          # [n][1]
    g = {"W3": dy.T @ h2, "b3": dy.sum(axis=0)}
    dz2 = (dy @ P["W3"]) * (1.0 - h2 * h2)                    # [n][32]
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ P["W2"]) * (1.0 - h1 * h1)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    dX = dz1 @ P["W1"]
    return pack(g), dX


def mse_grad(Y, T):
    """Loss 1/(2n) sum (Y - T)^2 and its gradient (Y - T)/n."""
    Y = np.asarray(Y, np.float64)
    T = np.asarray(T, np.float64)
    n = len(Y)
    r = Y - T
    return 0.5 * float(r @ r) / n, r / n


def adam_step(w, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (w, m, v)."""
    w = np.asarray(w, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * np.asarray(g, np.float64)
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * np.asarray(g, np.float64) ** 2
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v


def features(phi, mean_occupancy, acceptance):
    """Network inputs of a replica: packing fraction, mean disks per cell and
    the acceptance of the last window, centred and scaled to O(1)."""
    return np.array([20.0 * (phi - 0.7), mean_occupancy - 1.5, 4.0 * (acceptance - 0.3)],
                    dtype=np.float64)


def delta_from_output(y, wx, wy):
    """delta = 0.1 exp(y), clamped to [1e-3, min(w)/2] as the plain tuner is."""
    d = DELTA_SCALE * math.exp(float(y))
    hi = 0.5 * min(float(wx), float(wy))
    return min(max(d, DELTA_MIN), hi)
