"""Per-block network of the learned encoder control -- TEST INFRASTRUCTURE ONLY.

Plain numpy: the forward pass, the loss, its gradient written out layer by
layer, the Adam step and bfloat16 rounding, for checking the library's GPU
kernels.  Network: 16 features -> 64 ReLU -> 64 ReLU -> 37 logits (10
threshold classes, 27 range classes); parameters W1[64][16], b1[64],
W2[64][64], b2[64], W3[37][64], b3[37] in one flat vector.  Loss of a row:
softmax cross-entropy of each head against its label, summed; a batch takes
the mean.

The encoder control is not in the paper (its encoder applies global
thresholds, Sec. 3.2); the network and its training follow the textbook
definitions of a multilayer perceptron, backpropagation and Adam (Kingma and
Ba, 2015).  Pins: the forward pass on hand-set weights, the gradient against
central finite differences, Adam's first step, bfloat16 rounding cases.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT, N_CLS, N_RNG = 16, 64, 37, 10, 27
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(w: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = w[o:o + n].reshape(shape)
        o += n
    return out


def pack(parts: dict) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16_round(x: np.ndarray) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    r = np.where(nan, np.uint64(0x7FC00000), r).astype(np.uint32)
    return r.view(np.float32)


def bf16_bits(x: np.ndarray) -> np.ndarray:
    return (bf16_round(x).view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(h: np.ndarray) -> np.ndarray:
    return (np.asarray(h, dtype=np.uint32) << 16).view(np.float32)


def forward(w: np.ndarray, x: np.ndarray, dtype=np.float64):
    """Logits [n][37] and the activations (h1, h2), in `dtype`."""
    p = {k: v.astype(dtype) for k, v in unpack(np.asarray(w, dtype=np.float64)).items()}
    x = np.asarray(x, dtype=dtype)
    h1 = np.maximum(x @ p["W1"].T + p["b1"], 0)
    h2 = np.maximum(h1 @ p["W2"].T + p["b2"], 0)
    z = h2 @ p["W3"].T + p["b3"]
    return z, h1, h2


def forward_bf16(w: np.ndarray, x: np.ndarray):
    """Logits with the inputs and both hidden layers' outputs rounded to
    bfloat16 (to nearest, ties to even) and every sum in float64."""
    p = {k: v.astype(np.float64) for k, v in unpack(np.asarray(w, dtype=np.float64)).items()}
    r = lambda a: bf16_round(np.asarray(a, dtype=np.float32)).astype(np.float64)
    h1 = r(np.maximum(r(x) @ p["W1"].T + p["b1"], 0))
    h2 = r(np.maximum(h1 @ p["W2"].T + p["b2"], 0))
    return h2 @ p["W3"].T + p["b3"]


def predict(w: np.ndarray, x: np.ndarray, dtype=np.float32):
    """Argmax of each head (first maximum) and the threshold head's top
    softmax probability."""
    z, _, _ = forward(w, x, dtype)
    zt, zr = z[:, :N_CLS], z[:, N_CLS:]
    ct, cr = np.argmax(zt, axis=1), np.argmax(zr, axis=1)
    e = np.exp(zt - zt.max(axis=1, keepdims=True))
    conf = 1.0 / e.sum(axis=1)
    return ct.astype(np.int8), cr.astype(np.int8), conf, z


def _softmax(z):
    e = np.exp(z - z.max(axis=1, keepdims=True))
    return e / e.sum(axis=1, keepdims=True)


def loss(w: np.ndarray, x: np.ndarray, cls: np.ndarray, rng: np.ndarray) -> float:
    z, _, _ = forward(w, x)
    n = x.shape[0]
    l = 0.0
    for head, y in ((z[:, :N_CLS], cls), (z[:, N_CLS:], rng)):
        m = head.max(axis=1)
        lse = m + np.log(np.exp(head - m[:, None]).sum(axis=1))
        l += float(np.sum(lse - head[np.arange(n), y]))
    return l / n


def loss_and_grad(w: np.ndarray, x: np.ndarray, cls: np.ndarray, rng: np.ndarray):
    """Mean loss over the rows and its gradient (float64), by the chain rule
    through each layer."""
    w = np.asarray(w, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    p = unpack(w)
    n = x.shape[0]
    z, h1, h2 = forward(w, x)
    dz = np.zeros_like(z)
    dz[:, :N_CLS] = _softmax(z[:, :N_CLS])
    dz[np.arange(n), cls] -= 1.0
    dz[:, N_CLS:] = _softmax(z[:, N_CLS:])
    dz[np.arange(n), N_CLS + np.asarray(rng)] -= 1.0
    dz /= n
    g = {"W3": dz.T @ h2, "b3": dz.sum(axis=0)}
    dh2 = (dz @ p["W3"]) * (h2 > 0)
    g["W2"], g["b2"] = dh2.T @ h1, dh2.sum(axis=0)
    dh1 = (dh2 @ p["W2"]) * (h1 > 0)
    g["W1"], g["b1"] = dh1.T @ x, dh1.sum(axis=0)
    return loss(w, x, cls, rng), pack(g)


def adam(master, m, v, grad, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One bias-corrected Adam step; returns (master, m, v, bf16 bits)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    master = master - lr * mh / (np.sqrt(vh) + eps)
    return master, m, v, bf16_bits(master.astype(np.float32))
