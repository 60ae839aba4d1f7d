"""Reference of the bracket network (TEST INFRASTRUCTURE ONLY).

A 32 -> 64 -> 64 -> 4 perceptron with tanh hidden layers.  Outputs: u (the
normalised isovalue (s - phi_min)/W) and a 3-vector for the interface
normal.  The device network keeps BF16 weights and activations and
accumulates in FP32; this reference runs in FP64 on the same BF16-rounded
weights, inputs and stored activations (round to nearest even), so the two
differ only by accumulation rounding.  `exact=True` switches every rounding
off (used to pin the backward pass against finite differences).

Loss: mean (u - u*)^2 + 0.1 mean |n - n*|^2 over the batch.
Parameters are a dict of float32 arrays W1 [64,32], b1 [64], W2 [64,64],
b2 [64], W3 [4,64], b3 [4].
"""
from __future__ import annotations

import numpy as np

SHAPES = {"W1": (64, 32), "b1": (64,), "W2": (64, 64), "b2": (64,), "W3": (4, 64), "b3": (4,)}
ORDER = ["W1", "b1", "W2", "b2", "W3", "b3"]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES.values())
NORMAL_WEIGHT = 0.1


def bf16(x):
    """Round float32 values to bfloat16 (nearest even), returned as float64."""
    x = np.ascontiguousarray(np.asarray(x, np.float32))
    b = x.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(x)
    if nan.any():
        out[nan] = np.nan
    return out


def init_params(seed: int) -> dict:
    """Xavier-uniform weights, zero biases (float32)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name in ORDER:
        shp = SHAPES[name]
        if name.startswith("W"):
            lim = np.sqrt(6.0 / (shp[0] + shp[1]))
            p[name] = rng.uniform(-lim, lim, shp).astype(np.float32)
        else:
            p[name] = np.zeros(shp, np.float32)
    return p


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], np.float32).ravel() for k in ORDER])


def unflatten(v: np.ndarray) -> dict:
    out, o = {}, 0
    for k in ORDER:
        n = int(np.prod(SHAPES[k]))
        out[k] = np.asarray(v[o:o + n], np.float32).reshape(SHAPES[k])
        o += n
    return out


def forward(p: dict, X, exact: bool = False) -> dict:
    r = (lambda a: np.asarray(a, np.float64)) if exact else bf16
    x = r(X)
    W1, W2, W3 = r(p["W1"]), r(p["W2"]), r(p["W3"])
    b1, b2, b3 = (np.asarray(p[k], np.float64) for k in ("b1", "b2", "b3"))
    z1 = x @ W1.T + b1
    h1 = r(np.tanh(z1).astype(np.float32)) if not exact else np.tanh(z1)
    z2 = h1 @ W2.T + b2
    h2 = r(np.tanh(z2).astype(np.float32)) if not exact else np.tanh(z2)
    y = h2 @ W3.T + b3
    return dict(x=x, h1=h1, h2=h2, y=y, W1=W1, W2=W2, W3=W3)


def loss(y, T) -> float:
    return float(np.mean((y[:, 0] - T[:, 0]) ** 2) + NORMAL_WEIGHT * np.mean(np.sum((y[:, 1:] - T[:, 1:]) ** 2, 1)))


def backward(p: dict, X, T, exact: bool = False) -> tuple[float, dict]:
    """Loss and gradients; the tanh derivative uses the stored activation."""
    f = forward(p, X, exact)
    B = X.shape[0]
    y, h1, h2, x = f["y"], f["h1"], f["h2"], f["x"]
    dy = np.zeros_like(y)
    dy[:, 0] = 2.0 * (y[:, 0] - T[:, 0]) / B
    dy[:, 1:] = 2.0 * NORMAL_WEIGHT * (y[:, 1:] - T[:, 1:]) / B
    g = {}
    g["W3"] = dy.T @ h2
    g["b3"] = dy.sum(0)
    dz2 = (dy @ f["W3"]) * (1.0 - h2 * h2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ f["W2"]) * (1.0 - h1 * h1)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(0)
    return loss(y, T), g


def adam_step(p: dict, g: dict, state: dict, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8) -> None:
    """In-place Adam update of float32 master parameters."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in ORDER:
        m = state.setdefault("m_" + k, np.zeros(SHAPES[k], np.float32))
        v = state.setdefault("v_" + k, np.zeros(SHAPES[k], np.float32))
        gk = np.asarray(g[k], np.float32)
        m[...] = b1 * m + (1 - b1) * gk
        v[...] = b2 * v + (1 - b2) * gk * gk
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = (p[k] - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)
