"""Oracle of the learned low-fidelity level: a permutation-invariant set network.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).

Not in the paper: an extra control variate whose optimal OF-MLMC coefficient
(Sec. 2.4.3, eq. (alpha-matvec)) absorbs its error.  Architecture (a
deep-sets network):

    phi(x)   = ReLU(W2 ReLU(W1 x + b1) + b2)            per bubble, 4 -> 128 -> 128
    s        = pool_scale * sum_{bubbles of the set} phi  (sum pooling)
    y        = W4 ReLU(W3 s + b3) + b4                   128 -> 128 -> 5
    output   = y * out_std + out_mean                     (physical units)

Inputs per bubble: ((c - centre) / R_cloud, ln(r / r_median) / sigma).
Loss: mean squared error of the standardised outputs over sets and outputs.
Optimiser: Adam (Kingma and Ba 2015).

Precision reading of the hardware path: the operands of the three 128-wide
contractions (W2 and its input, W3 and its input, and the same operands in
the backward products) are rounded to bfloat16 (round to nearest even from
float32) and the sums are accumulated in float32; everything else is float32.
With bf16=True this oracle applies the same roundings at the same points and
computes in float64, so a comparison isolates the accumulation order.
"""
from __future__ import annotations

import numpy as np

D_IN, WIDTH, D_OUT = 4, 128, 5

PARAM_SHAPES = [("W1", (WIDTH, D_IN)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
                ("W3", (WIDTH, WIDTH)), ("b3", (WIDTH,)), ("W4", (D_OUT, WIDTH)), ("b4", (D_OUT,))]


def param_count() -> int:
    return sum(int(np.prod(s)) for _, s in PARAM_SHAPES)


def unflatten(flat: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in PARAM_SHAPES:
        k = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in PARAM_SHAPES])


def bf16(a) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) via float32, returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def f32(a) -> np.ndarray:
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def features(bubbles: np.ndarray, spec: dict) -> np.ndarray:
    """Per-bubble inputs ((c - centre)/R, ln(r/r_median)/sigma)."""
    b = np.asarray(bubbles, dtype=np.float64).reshape(-1, 4)
    cen = np.asarray(spec.get("center", (0.5, 0.5, 0.5)))
    x = np.empty((b.shape[0], 4))
    x[:, :3] = (b[:, :3] - cen) / spec["cloud_radius"]
    x[:, 3] = np.log(b[:, 3] / spec["r_median"]) / spec["r_sigma"]
    if spec["ndim"] < 3:
        x[:, 2] = 0.0
    return x


def forward(p: dict, x: np.ndarray, offsets: np.ndarray, pool_scale: float, bf16_ops: bool = False):
    """Standardised outputs [sets, 5] and the cache of the backward pass."""
    rnd = bf16 if bf16_ops else (lambda a: a)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = rnd(h1) @ rnd(p["W2"]).T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    S = len(offsets) - 1
    s = np.zeros((S, WIDTH))
    for i in range(S):
        s[i] = pool_scale * h2[offsets[i]:offsets[i + 1]].sum(axis=0)
    z3 = rnd(s) @ rnd(p["W3"]).T + p["b3"]
    a3 = np.maximum(z3, 0.0)
    y = a3 @ p["W4"].T + p["b4"]
    cache = dict(x=x, z1=z1, h1=h1, z2=z2, s=s, z3=z3, a3=a3, offsets=offsets, pool_scale=pool_scale,
                 bf16_ops=bf16_ops)
    return y, cache


def loss_and_grads(p: dict, x, offsets, pool_scale, target, bf16_ops=False):
    """MSE of standardised outputs and its gradient with respect to p."""
    rnd = bf16 if bf16_ops else (lambda a: a)
    y, c = forward(p, x, offsets, pool_scale, bf16_ops)
    S = y.shape[0]
    diff = y - target
    loss = float(np.mean(diff * diff))
    dy = 2.0 * diff / (S * D_OUT)
    g = {}
    g["W4"] = dy.T @ c["a3"]
    g["b4"] = dy.sum(axis=0)
    da3 = dy @ p["W4"]
    dz3 = da3 * (c["z3"] > 0)
    g["W3"] = rnd(dz3).T @ rnd(c["s"])
    g["b3"] = dz3.sum(axis=0)
    ds = rnd(dz3) @ rnd(p["W3"])
    dh2 = np.zeros_like(c["z2"])
    for i in range(S):
        dh2[offsets[i]:offsets[i + 1]] = pool_scale * ds[i]
    dz2 = dh2 * (c["z2"] > 0)
    g["W2"] = rnd(dz2).T @ rnd(c["h1"])
    g["b2"] = dz2.sum(axis=0)
    dh1 = rnd(dz2) @ rnd(p["W2"])
    dz1 = dh1 * (c["z1"] > 0)
    g["W1"] = dz1.T @ c["x"]
    g["b1"] = dz1.sum(axis=0)
    return loss, g


def adam_step(p: dict, g: dict, m: dict, v: dict, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected) in place; t counts from 1."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def he_uniform(seed: int) -> dict:
    """He-uniform weights, zero biases (a neutral initialisation for tests)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in PARAM_SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shp[1])
            p[name] = rng.uniform(-lim, lim, size=shp)
        else:
            p[name] = np.zeros(shp)
    return p
