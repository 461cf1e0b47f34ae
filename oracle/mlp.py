"""FP64 reference of the MLP surrogate for the inverse number-CDF (test
infrastructure only: used by the tests to check the GPU forward/backward).

Network: features (f0, f1) -> 64 -> SiLU -> 64 -> SiLU -> 64 -> SiLU -> 1.
Parameters are one flat vector in the order
    W1[64][2], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[64], b4
(8577 values).  Features of (chi, u): f0 = (log10 chi + 1)/3, f1 = logit(u)/16.
Output: log2 x.  Loss: mean squared error on log2 x.
"""
from __future__ import annotations

import numpy as np

H = 64
SIZES = [("W1", (H, 2)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)),
         ("b3", (H,)), ("W4", (H,)), ("b4", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(flat) -> dict:
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == N_PARAMS
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], np.float64).reshape(-1) for name, _ in SIZES])


def features(chi, u):
    chi = np.asarray(chi, np.float64)
    u = np.asarray(u, np.float64)
    return np.stack([(np.log10(chi) + 1.0) / 3.0, (np.log(u) - np.log1p(-u)) / 16.0], axis=1)


def _silu(z):
    return z / (1.0 + np.exp(-z))


def _dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(flat, f, cache: bool = False):
    p = unpack(flat)
    z1 = f @ p["W1"].T + p["b1"]
    h1 = _silu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = _silu(z2)
    z3 = h2 @ p["W3"].T + p["b3"]
    h3 = _silu(z3)
    y = h3 @ p["W4"] + p["b4"][0]
    if cache:
        return y, (f, z1, h1, z2, h2, z3, h3)
    return y


def backward(flat, f, dy) -> np.ndarray:
    """Gradient of sum(dy * y) with respect to the flat parameters."""
    p = unpack(flat)
    _, (f, z1, h1, z2, h2, z3, h3) = forward(flat, f, cache=True)
    g = {}
    g["W4"] = h3.T @ dy
    g["b4"] = np.array([dy.sum()])
    dz3 = np.outer(dy, p["W4"]) * _dsilu(z3)
    g["W3"] = dz3.T @ h2
    g["b3"] = dz3.sum(0)
    dz2 = (dz3 @ p["W3"]) * _dsilu(z2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * _dsilu(z1)
    g["W1"] = dz1.T @ f
    g["b1"] = dz1.sum(0)
    return pack(g)


def mse_grad(flat, f, y_target, energy_weight: bool = False) -> tuple[float, np.ndarray]:
    """Loss (1/M) sum w (y - t)^2 and its gradient; w = 1, or with energy_weight
    w = x / E[x] with x = 2^t and E[x] = 8/(15 sqrt 3) (the mean of x under the
    photon-number spectrum F(x)/x)."""
    y = forward(flat, f)
    r = y - y_target
    m = y.size
    w = np.exp2(y_target) / (8.0 / (15.0 * np.sqrt(3.0))) if energy_weight else np.ones_like(r)
    return float((w * r * r).sum() / m), backward(flat, f, 2.0 * w * r / m)


def init(seed: int = 0) -> np.ndarray:
    """He-style initialisation (deterministic)."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.normal(0, np.sqrt(2 / 2), (H, 2)), "b1": np.zeros(H),
         "W2": rng.normal(0, np.sqrt(2 / H), (H, H)), "b2": np.zeros(H),
         "W3": rng.normal(0, np.sqrt(2 / H), (H, H)), "b3": np.zeros(H),
         "W4": rng.normal(0, np.sqrt(1 / H), H), "b4": np.zeros(1)}
    return pack(p)


def bf16_round(a) -> np.ndarray:
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.asarray(a, dtype=np.float32)
    bits = a32.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)
