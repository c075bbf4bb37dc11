"""Plain FP64 reference of the learned warm start's network (numpy).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.

The network is not part of the paper: it maps (geometry flag, eta0, Kn, u_w, T2/T1, r_hat) to the
profile (n, u_t1, T, q_r, P_r,t1) at one radial node.  Layers 6 -> 256 -> 256 -> 256 -> 256 -> 5,
SiLU on the hidden layers, linear output, mean-squared error over the five normalised outputs,
Adam (Kingma & Ba, 2015) with bias correction.  Parameters are packed layer by layer as the
weight matrix [fan_out][fan_in] (row-major) followed by the bias [fan_out].

``bf16=True`` reproduces where a BF16 matrix unit rounds: both operands of every matrix product
are rounded to bfloat16 (round to nearest even) and the product is accumulated exactly (FP64).
"""
from __future__ import annotations

import numpy as np

LAYERS = ((6, 256), (256, 256), (256, 256), (256, 256), (256, 5))
N_PARAMS = sum(o * i + o for i, o in LAYERS)


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (8 exponent bits, 7 stored mantissa bits), nearest even, via FP32."""
    x32 = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params: np.ndarray):
    """[(W [out][in], b [out]) per layer] as views of the packed vector."""
    out, o = [], 0
    for fin, fout in LAYERS:
        W = params[o:o + fin * fout].reshape(fout, fin)
        o += fin * fout
        b = params[o:o + fout]
        o += fout
        out.append((W, b))
    assert o == params.size
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def _mm(a, b, use_bf16: bool):
    if use_bf16:
        a, b = bf16(a), bf16(b)
    return a @ b


def forward(params: np.ndarray, X: np.ndarray, use_bf16: bool = False):
    """Returns (Y, cache) with cache = [(input of layer, pre-activation)] per layer."""
    h = np.asarray(X, dtype=np.float64)
    cache = []
    layers = unpack(np.asarray(params, dtype=np.float64))
    for li, (W, b) in enumerate(layers):
        z = _mm(h, W.T, use_bf16) + b
        cache.append((h, z))
        h = silu(z) if li < len(layers) - 1 else z
    return h, cache


def loss_grad(params: np.ndarray, X: np.ndarray, T: np.ndarray, use_bf16: bool = False):
    """Mean-squared error over rows x outputs and its gradient (packed like params)."""
    Y, cache = forward(params, X, use_bf16)
    R = Y.shape[0]
    diff = Y - T
    loss = float((diff * diff).sum() / (R * Y.shape[1]))
    dz = 2.0 * diff / (R * Y.shape[1])
    layers = unpack(np.asarray(params, dtype=np.float64))
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        h, _ = cache[li]
        dW = _mm(dz.T, h, use_bf16)
        db = dz.sum(axis=0)
        grads[li] = (dW, db)
        if li > 0:
            dh = _mm(dz, W, use_bf16)
            dz = dh * dsilu(cache[li - 1][1])
    flat = np.concatenate([np.concatenate([dW.reshape(-1), db]) for dW, db in grads])
    return loss, flat


def adam(params, grad, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (t counts from 1); returns new (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# Input features: the geometry flag as is, the other five inputs mapped affinely to zero mean and
# unit variance under the sweep's distributions (eta0 ~ U(0.01, 0.3), log10 Kn ~ U(-2, 1),
# u_w ~ U(0, 0.5), T2/T1 ~ U(1, 2), r_hat ~ U(0, 1)).
def features(geometry: int, eta0: float, kn: float, uw: float, tratio: float, r_hat: np.ndarray) -> np.ndarray:
    r_hat = np.asarray(r_hat, dtype=np.float64)
    out = np.zeros((r_hat.size, 6))
    out[:, 0] = float(geometry)
    out[:, 1] = (eta0 - 0.155) / (0.29 / np.sqrt(12.0))
    out[:, 2] = (np.log10(kn) + 0.5) / (3.0 / np.sqrt(12.0))
    out[:, 3] = (uw - 0.25) / (0.5 / np.sqrt(12.0))
    out[:, 4] = (tratio - 1.5) / (1.0 / np.sqrt(12.0))
    out[:, 5] = (r_hat - 0.5) / (1.0 / np.sqrt(12.0))
    return out
