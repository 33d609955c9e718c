"""FP64 oracle of the learned search-window network: forward, hand-written
backward, asymmetric quantile (pinball) loss and Adam.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network (an addition to the paper's method, which sizes its hit search
from the covariance): 27 standardised inputs (the 6 propagated parameters and
the 21 upper-triangle covariance entries) -> 64 -> GELU -> 64 -> GELU -> 2,
softplus head times a per-output scale: the half-width of the hit window as an
arc at the layer radius (cm) and in z (cm).  Weights and activations that feed
products are BF16, products accumulate in wider precision; this oracle rounds
to BF16 at exactly those points and computes everything else in FP64.

Loss per output: 20 * max(0, d - w) + max(0, w - d), d = |true offset|; its
minimiser is the 20/21 quantile of d (a missed true hit costs twenty times a
unit of extra width).
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

N_IN, N_H, N_OUT = 27, 64, 2
MISS_WEIGHT = 20.0

_SQRT2 = np.sqrt(2.0)
_INV_SQRT2PI = 1.0 / np.sqrt(2.0 * np.pi)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), via FP32, returned as FP64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    finite = (u & 0x7F800000) != 0x7F800000
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = np.where(finite, r, u.astype(np.uint32)).astype(np.uint32).view(np.float32)
    return out.astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / _SQRT2))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / _SQRT2)) + z * _INV_SQRT2PI * np.exp(-0.5 * z * z)


def softplus(o):
    return np.where(o > 30.0, o, np.log1p(np.exp(np.minimum(o, 30.0))))


def sigmoid(o):
    return 1.0 / (1.0 + np.exp(-o))


def init_params(rng, mu, sd, scale):
    """He-style initialisation; weights are kept as BF16 values."""
    p = {
        "W1": bf16(rng.normal(0, np.sqrt(2.0 / N_IN), (N_H, N_IN))),
        "b1": np.zeros(N_H),
        "W2": bf16(rng.normal(0, np.sqrt(2.0 / N_H), (N_H, N_H))),
        "b2": np.zeros(N_H),
        "W3": bf16(rng.normal(0, np.sqrt(1.0 / N_H), (N_OUT, N_H))),
        "b3": np.zeros(N_OUT),
        "mu": np.asarray(mu, dtype=np.float64),
        "sd": np.asarray(sd, dtype=np.float64),
        "scale": np.asarray(scale, dtype=np.float64),
    }
    return p


TRAINABLE = ("W1", "b1", "W2", "b2", "W3", "b3")


def forward(p, x, round_bf16=True):
    r = bf16 if round_bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    xh = r((np.asarray(x, dtype=np.float64) - p["mu"]) / p["sd"])
    z1 = xh @ p["W1"].T + p["b1"]
    h1 = r(gelu(z1))
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = r(gelu(z2))
    o = h2 @ p["W3"].T + p["b3"]
    w = p["scale"] * softplus(o)
    return dict(xh=xh, z1=z1, h1=h1, z2=z2, h2=h2, o=o, w=w)


def loss(w, d):
    return float(np.mean(MISS_WEIGHT * np.maximum(0.0, d - w) + np.maximum(0.0, w - d)))


def backward(p, cache, d):
    """Gradient of loss(forward(x).w, d) (mean over rows and both outputs).
    The BF16 roundings are treated as identity in the derivative."""
    n = d.shape[0]
    w = cache["w"]
    gw = np.where(w > d, 1.0, np.where(w < d, -MISS_WEIGHT, 0.0)) / (n * N_OUT)
    go = gw * p["scale"] * sigmoid(cache["o"])
    g = {}
    g["W3"] = go.T @ cache["h2"]
    g["b3"] = go.sum(axis=0)
    gz2 = (go @ p["W3"]) * gelu_grad(cache["z2"])
    g["W2"] = gz2.T @ cache["h1"]
    g["b2"] = gz2.sum(axis=0)
    gz1 = (gz2 @ p["W2"]) * gelu_grad(cache["z1"])
    g["W1"] = gz1.T @ cache["xh"]
    g["b1"] = gz1.sum(axis=0)
    return g


def adam_step(master, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba) on the FP64 master weights; t counts from 1.
    Returns the BF16 working copy of the weight matrices."""
    work = {}
    for k in TRAINABLE:
        m[k] = beta1 * m[k] + (1 - beta1) * grads[k]
        v[k] = beta2 * v[k] + (1 - beta2) * grads[k] ** 2
        mh = m[k] / (1 - beta1 ** t)
        vh = v[k] / (1 - beta2 ** t)
        master[k] = master[k] - lr * mh / (np.sqrt(vh) + eps)
        work[k] = bf16(master[k]) if k.startswith("W") else master[k].copy()
    return work


def blob(p, kappa=1.0, floor_rphi=0.01, floor_z=0.1, gate_rphi=0.0, gate_z=0.0):
    """Parameter block of the C oracle (kforacle.c: mu sd W1 b1 W2 b2 W3 b3
    scale kappa floor_rphi floor_z gate_rphi gate_z).  Zero gates consult the
    network for every candidate."""
    parts = [p["mu"], p["sd"], p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"], p["W3"].ravel(), p["b3"],
             p["scale"], [kappa, floor_rphi, floor_z, gate_rphi, gate_z]]
    return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in parts])
