"""FP64 reference of the surrogate MLP -- TEST INFRASTRUCTURE ONLY.

Network (per bump shape): 6 -> 256 -> 256 -> 256 -> 6, SiLU on the hidden
layers, y = W4 h3 + b4.  Parameter vector layout (134918 values):
    W1[256][6], b1[256], W2[256][256], b2[256], W3[256][256], b3[256],
    W4[6][256], b4[6]
Loss: mean over the batch of the sum of squared output errors.

bf16=True emulates the GPU's arithmetic.  The first layer (K = 6) and the
output layer (N = 6) are wide (x, W1, h3, W4, dL/dy, dL/dz1 not rounded).
The forward 256x256 products use three-term split bfloat16: with
hi = bf16(v), lo = bf16(v - hi) for both operands, A B is taken as
Ah Bh + Ah Bl + Al Bh.  The backward products round their operands to
bfloat16 once: the signals dL/dz3, dL/dz2, the weights W3, W2 and, for the
weight gradients, the layer inputs h1, h2.  Rounding is to nearest even;
biases, pre-activations and accumulations stay wide.
"""
from __future__ import annotations

import numpy as np

SIZES = [(256, 6), (256, 256), (256, 256), (6, 256)]
N_PARAMS = sum(o * i + o for o, i in SIZES)


def split(p):
    """Views W1, b1, ..., W4, b4 into a flat parameter vector."""
    out, k = [], 0
    for o, i in SIZES:
        out.append(p[k:k + o * i].reshape(o, i))
        k += o * i
        out.append(p[k:k + o])
        k += o
    return out


def bf16_round(a):
    """Round float values to bfloat16 precision (nearest even), returned as
    float64."""
    f = np.asarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def split_bf16(a):
    """(hi, lo) with hi = bf16(a), lo = bf16(a - hi)."""
    hi = bf16_round(a)
    return hi, bf16_round(np.asarray(a, np.float64) - hi)


def split_product(A, B):
    """A @ B in three-term split bfloat16: Ah Bh + Ah Bl + Al Bh."""
    Ah, Al = split_bf16(A)
    Bh, Bl = split_bf16(B)
    return Ah @ Bh + Ah @ Bl + Al @ Bh


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(seed):
    """He-style uniform init (fan-in), biases zero."""
    rng = np.random.default_rng(seed)
    p = np.zeros(N_PARAMS)
    parts = split(p)
    for li, (o, i) in enumerate(SIZES):
        lim = np.sqrt(6.0 / i) * (0.5 if li == 3 else 1.0)
        parts[2 * li][:] = rng.uniform(-lim, lim, size=(o, i))
    return p


def forward(p, x, bf16=False):
    """Returns y [n,6] and the cache (inputs of each layer as the backward's
    weight gradients use them, pre-activations)."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    W1, b1, W2, b2, W3, b3, W4, b4 = split(np.asarray(p, np.float64))
    hs, zs = [], []
    h = np.asarray(x, np.float64)
    for li, (W, b) in enumerate(((W1, b1), (W2, b2), (W3, b3))):
        hs.append(h if li == 0 else r(h))
        if li == 0 or not bf16:
            z = h @ W.T + b
        else:
            z = split_product(h, W.T) + b
        zs.append(z)
        h = silu(z)
    hs.append(h)
    y = h @ W4.T + b4
    return y, (hs, zs)


def backward(p, x, dy, bf16=False):
    """Gradient of sum(dy * y) with respect to the flat parameters."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    y, (hs, zs) = forward(p, x, bf16)
    W1, b1, W2, b2, W3, b3, W4, b4 = split(np.asarray(p, np.float64))
    g = np.zeros(N_PARAMS)
    gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4 = split(g)
    d = np.asarray(dy, np.float64)
    gW4[:] = d.T @ hs[3]
    gb4[:] = d.sum(0)
    dh = d @ W4                             # dL/dh3
    for W, gW, gb, li in ((W3, gW3, gb3, 2), (W2, gW2, gb2, 1), (W1, gW1, gb1, 0)):
        dz = dh * dsilu(zs[li])
        gW[:] = (r(dz) if li > 0 else dz).T @ hs[li]
        gb[:] = dz.sum(0)
        if li > 0:
            dh = r(dz) @ r(W)
    return g


def loss_and_grad(p, x, target, bf16=False):
    """MSE loss (mean over samples of the squared error summed over the 6
    outputs) and its gradient with respect to the flat parameters."""
    y, _ = forward(p, x, bf16)
    n = x.shape[0]
    diff = y - target
    loss = float((diff * diff).sum() / n)
    return loss, backward(p, x, 2.0 * diff / n, bf16)
