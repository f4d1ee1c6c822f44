"""Reference for the learned per-edge drift surrogate: a 16 -> 64 -> 64 -> 1
ReLU network (the learned-heuristic idea of Sec. 5.2, here a stand-in for the
analytic per-edge drift of the precompute step, Alg. 1 step 2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Precision model, which the GPU kernels follow: inputs, the two weight
matrices, the output weights and the first hidden activations are rounded to
bfloat16 (round to nearest, ties to even, from float32); biases, the second
hidden activations, every product sum and the output are exact here (float64)
and float32 accumulations on the GPU.  This module evaluates that model in
float64 on the same bfloat16 values, so the two differ only by float32
accumulation order.

    z1 = X W1 + b1,  h1 = bf16(relu(z1))
    z2 = h1 W2 + b2, h2 = relu(z2)
    y  = h2 w3 + b3
    L  = mean((y - t)^2)
"""
from __future__ import annotations

import numpy as np


def bf16_round(x) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32 values.
    Written from the definition: keep the top 16 bits of the float32 pattern
    after adding half an ulp of bfloat16 (plus the tie-to-even bit)."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    out = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
    nan = np.isnan(a)
    if nan.any():
        out = out.copy()
        out[nan] = np.nan
    return out


def bf16_bits(x) -> np.ndarray:
    """bfloat16 bit patterns (uint16) of float32 values already on the grid."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    return (a.view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def init_params(seed: int, n_in: int = 16, n_h: int = 64):
    """He-normal weights from a seeded numpy generator, zero biases (float32
    masters)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0.0, np.sqrt(2.0 / n_in), (n_in, n_h)).astype(np.float32)
    W2 = rng.normal(0.0, np.sqrt(2.0 / n_h), (n_h, n_h)).astype(np.float32)
    w3 = rng.normal(0.0, np.sqrt(2.0 / n_h), (n_h,)).astype(np.float32)
    return dict(W1=W1, b1=np.zeros(n_h, np.float32), W2=W2, b2=np.zeros(n_h, np.float32),
                w3=w3, b3=np.zeros(1, np.float32))


def forward(p: dict, X: np.ndarray):
    """Returns (y, cache) in float64 on the bfloat16 tensors of the model."""
    Xb = bf16_round(X).astype(np.float64)
    W1 = bf16_round(p["W1"]).astype(np.float64)
    W2 = bf16_round(p["W2"]).astype(np.float64)
    w3 = bf16_round(p["w3"]).astype(np.float64)
    z1 = Xb @ W1 + p["b1"].astype(np.float64)
    h1 = bf16_round(np.maximum(z1, 0.0).astype(np.float32)).astype(np.float64)
    z2 = h1 @ W2 + p["b2"].astype(np.float64)
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + float(p["b3"][0])
    return y, dict(X=Xb, W1=W1, W2=W2, w3=w3, z1=z1, h1=h1, z2=z2, h2=h2)


def loss(y: np.ndarray, t: np.ndarray) -> float:
    d = y - t.astype(np.float64)
    return float(np.mean(d * d))


def backward(p: dict, X: np.ndarray, t: np.ndarray):
    """Gradients of the mean squared error with respect to the float32 master
    parameters, exact (float64) for the model of ``forward``: straight through
    the bfloat16 rounding of the weights, the rounding of h1 treated as the
    identity, ReLU' = [z > 0].  No rounding is applied to the gradients; a
    kernel that rounds the output gradients to bfloat16 before its matrix
    products is compared with this within the rounding's error bound."""
    y, c = forward(p, X)
    n = X.shape[0]
    dy = 2.0 * (y - t.astype(np.float64)) / n
    g = {}
    g["w3"] = c["h2"].T @ dy
    g["b3"] = np.array([dy.sum()])
    dz2 = np.outer(dy, c["w3"]) * (c["z2"] > 0)
    g["W2"] = c["h1"].T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ c["W2"].T) * (c["z1"] > 0)
    g["W1"] = c["X"].T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return y, g


def gradient_abs_terms(p: dict, X: np.ndarray, t: np.ndarray) -> dict:
    """For every parameter, the sum of the absolute values of the terms its
    gradient adds up (the same products as ``backward`` with every factor
    replaced by its magnitude).  A perturbation of relative size u in each
    factor moves a gradient entry by at most about k u times this sum, k the
    number of perturbed factors on its path, so it scales the error bound of
    a reduced-precision evaluation."""
    y, c = forward(p, X)
    n = X.shape[0]
    ady = np.abs(2.0 * (y - t.astype(np.float64)) / n)
    adz2 = np.outer(ady, np.abs(c["w3"])) * (c["z2"] > 0)
    adz1 = (adz2 @ np.abs(c["W2"]).T) * (c["z1"] > 0)
    return dict(w3=np.abs(c["h2"]).T @ ady, b3=np.array([ady.sum()]),
                W2=np.abs(c["h1"]).T @ adz2, b2=adz2.sum(axis=0),
                W1=np.abs(c["X"]).T @ adz1, b1=adz1.sum(axis=0))


def adam_step(p: dict, g: dict, m: dict, v: dict, step: int, lr: float,
              b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma and Ba, 2015) in float64 on copies of the float32
    masters; returns the new masters as float32."""
    out = {}
    for k in p:
        m[k] = b1 * m.get(k, 0.0) + (1 - b1) * g[k]
        v[k] = b2 * v.get(k, 0.0) + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** step)
        vh = v[k] / (1 - b2 ** step)
        out[k] = (p[k].astype(np.float64) - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)
    return out


def finite_difference(p: dict, X: np.ndarray, t: np.ndarray, key: str, idx, h: float = 1e-6):
    """Central difference of the float64 loss with respect to one parameter,
    evaluated on a float64 copy of the model without bfloat16 rounding of that
    parameter (used to pin ``backward`` on a rounding-free variant)."""
    def f(delta):
        q = {k: v.copy() for k, v in p.items()}
        q[key] = q[key].astype(np.float64)
        q[key][idx] += delta
        return loss(_forward_f64(q, X)[0], t)
    return (f(h) - f(-h)) / (2 * h)


def _forward_f64(p: dict, X: np.ndarray):
    """The same network without any bfloat16 rounding (float64 throughout)."""
    z1 = X.astype(np.float64) @ p["W1"].astype(np.float64) + p["b1"].astype(np.float64)
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].astype(np.float64) + p["b2"].astype(np.float64)
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["w3"].astype(np.float64) + float(np.asarray(p["b3"]).reshape(-1)[0])
    return y, None


def backward_f64(p: dict, X: np.ndarray, t: np.ndarray):
    """Gradients of the rounding-free float64 network (for the finite-difference
    pin; structurally identical to ``backward``)."""
    X = X.astype(np.float64)
    W1, W2 = p["W1"].astype(np.float64), p["W2"].astype(np.float64)
    w3 = p["w3"].astype(np.float64)
    z1 = X @ W1 + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + float(np.asarray(p["b3"]).reshape(-1)[0])
    n = X.shape[0]
    dy = 2.0 * (y - t) / n
    dz2 = np.outer(dy, w3) * (z2 > 0)
    dz1 = (dz2 @ W2.T) * (z1 > 0)
    return dict(w3=h2.T @ dy, b3=np.array([dy.sum()]), W2=h1.T @ dz2, b2=dz2.sum(0),
                W1=X.T @ dz1, b1=dz1.sum(0))


def flat(p: dict) -> np.ndarray:
    """The 5313-value float32 parameter block: W1, b1, W2, b2, w3, b3."""
    return np.concatenate([np.asarray(p[k], np.float64).reshape(-1)
                           for k in ("W1", "b1", "W2", "b2", "w3", "b3")]).astype(np.float32)


def unflat(v: np.ndarray) -> dict:
    v = np.asarray(v, np.float32)
    out, o = {}, 0
    for k, shp in (("W1", (16, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
                   ("w3", (64,)), ("b3", (1,))):
        size = int(np.prod(shp))
        out[k] = v[o:o + size].reshape(shp).copy()
        o += size
    return out
