"""FP64 reference of the small pruning network -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may import this module.

The network maps the early trajectory of one start vector to the probability
that it ends in one of the top-ranked unique components:
  features f (16): for passes t = 1..8, the kurtosis of the row before the pass
      and log10(max(step, 1e-12)), interleaved (alpha_1, ls_1, alpha_2, ...),
      then standardised with fixed per-feature mean and standard deviation;
  h1 = relu(W1 f + b1)      (64)
  h2 = relu(W2 h1 + b2)     (64)
  z  = w3 . h2 + b3         (logit);  p = sigmoid(z)
Loss: binary cross-entropy on the logit with a positive-class weight w_pos,
averaged over the rows:  l = -(w_pos y log p + (1 - y) log(1 - p)).
Optimiser: Adam (Kingma & Ba) with bias correction.

Parameters are packed in one vector: W1 (64 x 16, row-major), b1 (64),
W2 (64 x 64), b2 (64), w3 (64), b3 (1) -- 5313 values.
"""
from __future__ import annotations

import numpy as np

H = 64
F_IN = 16
SHAPES = [("W1", (H, F_IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)),
          ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = theta[o:o + n].reshape(shp)
        o += n
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init_params(rng: np.random.Generator) -> np.ndarray:
    """He-uniform weights for the ReLU layers, zero biases."""
    parts = {}
    for name, shp in SHAPES:
        if name.startswith("b"):
            parts[name] = np.zeros(shp)
        else:
            fan_in = shp[-1] if len(shp) > 1 else H
            lim = np.sqrt(6.0 / fan_in)
            parts[name] = rng.uniform(-lim, lim, size=shp)
    return pack(parts)


def features(traj: np.ndarray, mean: np.ndarray, std: np.ndarray) -> np.ndarray:
    """traj: R x 8 x 2 (kurtosis before the pass, step of the pass) -> R x 16."""
    traj = np.asarray(traj, dtype=np.float64)
    f = np.empty((traj.shape[0], 16))
    f[:, 0::2] = traj[:, :, 0]
    f[:, 1::2] = np.log10(np.maximum(traj[:, :, 1], 1e-12))
    return (f - mean) / std


def forward(theta, F):
    p = unpack(theta)
    a1 = F @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ p["w3"] + p["b3"][0]
    return z, (F, a1, h1, a2, h2)


def sigmoid(z):
    z = np.asarray(z, dtype=np.float64)
    return np.where(z >= 0, 1.0 / (1.0 + np.exp(-np.abs(z))), np.exp(-np.abs(z)) / (1.0 + np.exp(-np.abs(z))))


def bce(z, y, w_pos):
    """Mean of -(w_pos y log s(z) + (1 - y) log(1 - s(z))), written with the
    stable log-sigmoid: log s(z) = -softplus(-z), log(1 - s(z)) = -softplus(z)."""
    z = np.asarray(z, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    sp_neg = np.logaddexp(0.0, -z)
    sp_pos = np.logaddexp(0.0, z)
    return float(np.mean(w_pos * y * sp_neg + (1.0 - y) * sp_pos))


def loss_and_grad(theta, F, y, w_pos):
    """Mean loss and its gradient with respect to the packed parameters."""
    p = unpack(theta)
    z, (F, a1, h1, a2, h2) = forward(theta, F)
    y = np.asarray(y, dtype=np.float64)
    R = F.shape[0]
    s = sigmoid(z)
    # d/dz of w_pos y softplus(-z) + (1 - y) softplus(z) = (1 - y) s - w_pos y (1 - s)
    dz = ((1.0 - y) * s - w_pos * y * (1.0 - s)) / R
    g = {}
    g["w3"] = h2.T @ dz
    g["b3"] = np.array([dz.sum()])
    dh2 = np.outer(dz, p["w3"]) * (a2 > 0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ p["W2"]) * (a1 > 0)
    g["W1"] = dh1.T @ F
    g["b1"] = dh1.sum(axis=0)
    return bce(z, y, w_pos), pack(g)


def adam_step(theta, m, v, g, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t is the 1-based step count)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
