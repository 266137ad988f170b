"""Learned cost model: CPU oracle -- TEST INFRASTRUCTURE ONLY.

The paper balances uneven per-cell chemistry cost across processes
("DLBFoam: Dynamic load balancing"); the GPU library orders its work queue by
a predicted cost instead. This module is the plain reference for that model:
a 4 -> 64 -> 64 -> 1 ReLU multilayer perceptron predicting ln(substeps) from
four cell features, its mean-squared-error gradient, Adam, the octile bin
edges and the stable longest-first bin order. Two arithmetic modes:

* ``fp64``: everything in float64 (the mathematical definition; pinned by
  finite differences and by PyTorch's own Adam).
* ``bf16``: the GPU's rounding points -- every operand of a contraction
  (weights, activations, back-propagated errors) rounded to bfloat16 with
  round-to-nearest-even, products accumulated exactly (float64) and the
  result stored in float32.

Only the test suite and the benchmark's baseline leg use this module.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 4, 64
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("w3", (N_H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)   # 4545


def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even); returns float64 values."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def f32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def unflatten(theta) -> dict:
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def features(phi, dt) -> np.ndarray:
    """The four scheduling features of each cell of phi [N, 2+Ns] = (T, p, Y):
    (T - 1500)/700, ln(p/1e5), (1/Ns) sum_i log10 max(Y_i, 1e-30) / 10 and
    log10(dt/1e-6). They only steer the queue order, never the results."""
    phi = np.asarray(phi, dtype=np.float64)
    ns = phi.shape[1] - 2
    ell = np.log10(np.maximum(phi[:, 2:], 1e-30)).sum(axis=1) / ns
    out = np.empty((phi.shape[0], 4))
    out[:, 0] = (phi[:, 0] - 1500.0) / 700.0
    out[:, 1] = np.log(phi[:, 1] / 1e5)
    out[:, 2] = ell / 10.0
    out[:, 3] = np.log10(dt / 1e-6)
    return out


def standardize_stats(X):
    """Mean and standard deviation per feature (population), with a floor so
    that a constant feature (for example log10(dt) of one workload) maps to 0."""
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd = np.where(sd < 1e-6, 1.0, sd)
    return mu, sd


def forward(p: dict, Xn, mode: str = "fp64"):
    """Prediction for standardized features Xn [B, 4]; returns y [B] and the
    cache used by the backward pass."""
    Xn = np.asarray(Xn, dtype=np.float64)
    if mode == "fp64":
        a1 = Xn @ p["W1"].T + p["b1"]
        h1 = np.maximum(a1, 0.0)
        a2 = h1 @ p["W2"].T + p["b2"]
        h2 = np.maximum(a2, 0.0)
        y = h2 @ p["w3"] + p["b3"][0]
        return y, dict(Xn=Xn, a1=a1, h1=h1, a2=a2, h2=h2)
    if mode != "bf16":
        raise ValueError(mode)
    xb = bf16_round(Xn)
    a1 = f32(xb @ bf16_round(p["W1"]).T + f32(p["b1"]))
    h1 = np.maximum(a1, 0.0)
    h1b = bf16_round(h1)
    a2 = f32(h1b @ bf16_round(p["W2"]).T + f32(p["b2"]))
    h2 = np.maximum(a2, 0.0)
    h2b = bf16_round(h2)
    y = f32(h2b @ bf16_round(p["w3"]) + f32(p["b3"])[0])
    return y, dict(Xn=xb, a1=a1, h1=h1b, a2=a2, h2=h2b)


def loss_and_grad(p: dict, Xn, T, mode: str = "fp64"):
    """L = mean((y - t)^2) and dL/dparams by back propagation."""
    T = np.asarray(T, dtype=np.float64)
    B = T.shape[0]
    y, c = forward(p, Xn, mode)
    r = y - T
    loss = float(np.mean(r * r))
    g = 2.0 * r / B                                   # dL/dy
    if mode == "fp64":
        d3 = g
        gw3 = c["h2"].T @ d3
        gb3 = np.array([d3.sum()])
        d2 = np.outer(d3, p["w3"]) * (c["a2"] > 0)
        gW2 = d2.T @ c["h1"]
        gb2 = d2.sum(axis=0)
        d1 = (d2 @ p["W2"]) * (c["a1"] > 0)
        gW1 = d1.T @ c["Xn"]
        gb1 = d1.sum(axis=0)
    else:
        d3 = f32(g)
        d3b = bf16_round(d3)
        gw3 = f32(c["h2"].T @ d3b)
        gb3 = f32(np.array([d3.sum()]))
        d2 = f32(np.outer(d3b, bf16_round(p["w3"]))) * (c["a2"] > 0)
        d2b = bf16_round(d2)
        gW2 = f32(d2b.T @ c["h1"])
        gb2 = f32(d2.sum(axis=0))
        d1 = f32(d2b @ bf16_round(p["W2"])) * (c["a1"] > 0)
        d1b = bf16_round(d1)
        gW1 = f32(d1b.T @ c["Xn"])
        gb1 = f32(d1.sum(axis=0))
    grads = dict(W1=gW1, b1=gb1, W2=gW2, b2=gb2, w3=gw3, b3=gb3)
    return loss, grads


def adam_step(theta, grad, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba): returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def octile_edges(pred) -> np.ndarray:
    """Seven edges splitting predictions into eight equally populated bins:
    the values at sorted positions floor(k n / 8), k = 1..7."""
    s = np.sort(np.asarray(pred, dtype=np.float64))
    n = s.shape[0]
    return np.array([s[(k * n) // 8] for k in range(1, 8)])


def bin_index(cost, edges) -> np.ndarray:
    """Bin of each cost: the number of edges not above it (0..7)."""
    cost = np.asarray(cost, dtype=np.float64)
    edges = np.asarray(edges, dtype=np.float64)
    return (cost[:, None] >= edges[None, :]).sum(axis=1)


def binned_order(cost, edges) -> np.ndarray:
    """Queue order: bin 7 (highest predicted cost) first, cell index ascending
    within a bin. Any non-finite cost gives the identity order."""
    cost = np.asarray(cost, dtype=np.float64)
    if not np.all(np.isfinite(cost)):
        return np.arange(cost.shape[0])
    b = bin_index(cost, edges)
    out = []
    for k in range(7, -1, -1):
        out.extend(np.nonzero(b == k)[0].tolist())
    return np.array(out, dtype=np.int64)
