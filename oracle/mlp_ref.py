"""Plain FP64 numpy reference of the warm-start network, for checking the
GPU forward and backward kernels.  TEST INFRASTRUCTURE ONLY.

Network: h1 = silu(x W1^T + b1), h2 = silu(h1 W2^T + b2), h3 = silu(h2 W3^T
+ b3), y = h3 W4^T + b4, loss = mean((y - t)^2) over all entries;
silu(z) = z / (1 + e^-z).  Gradients by the chain rule written out.

With ``rnd`` (a function rounding an array to the operand precision of a
matrix product, e.g. bf16_round), both operands of every matrix product are
rounded by it before the product is taken exactly in FP64 (the product
formats of a matrix-core implementation: BF16 operands, wide accumulation);
sums, biases and SiLU stay FP64.  rnd=None is the exact network.
"""
import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def bf16_round(x):
    """Nearest bfloat16 (8-bit significand), ties to even, of float32 values
    (inputs are first rounded to float32), returned as float64."""
    b = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _mm(a, b, rnd):
    if rnd is None:
        return a @ b
    return rnd(a) @ rnd(b)


def forward(Ws, bs, X, rnd=None):
    """X: [rows x n_in] -> (Y, cache)."""
    h = X.astype(np.float64)
    zs, hs = [], [h]
    for l in range(3):
        z = _mm(h, Ws[l].T.astype(np.float64), rnd) + bs[l].astype(np.float64)
        zs.append(z)
        h = silu(z)
        hs.append(h)
    y = _mm(h, Ws[3].T.astype(np.float64), rnd) + bs[3].astype(np.float64)
    return y, (zs, hs)


def loss_and_grads(Ws, bs, X, T, rnd=None):
    y, (zs, hs) = forward(Ws, bs, X, rnd)
    n = y.size
    d = y - T
    loss = float((d * d).sum() / n)
    g = 2.0 * d / n                      # dL/dy
    dW, db = [None] * 4, [None] * 4
    dW[3] = _mm(g.T, hs[3], rnd)
    db[3] = g.sum(0)
    dh = _mm(g, Ws[3].astype(np.float64), rnd)
    for l in (2, 1, 0):
        dz = dh * dsilu(zs[l])
        dW[l] = _mm(dz.T, hs[l], rnd)
        db[l] = dz.sum(0)
        dh = _mm(dz, Ws[l].astype(np.float64), rnd)
    return loss, dW, db
