"""Plain FP64 numpy reference of the warm-start network, for checking the
GPU forward and backward kernels.  TEST INFRASTRUCTURE ONLY.

Network: h1 = silu(x W1^T + b1), h2 = silu(h1 W2^T + b2), h3 = silu(h2 W3^T
+ b3), y = h3 W4^T + b4, loss = mean((y - t)^2) over all entries;
silu(z) = z / (1 + e^-z).  Gradients by the chain rule written out.
"""
import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(Ws, bs, X):
    """X: [rows x n_in] -> (Y, cache)."""
    h = X.astype(np.float64)
    zs, hs = [], [h]
    for l in range(3):
        z = h @ Ws[l].T.astype(np.float64) + bs[l].astype(np.float64)
        zs.append(z)
        h = silu(z)
        hs.append(h)
    y = h @ Ws[3].T.astype(np.float64) + bs[3].astype(np.float64)
    return y, (zs, hs)


def loss_and_grads(Ws, bs, X, T):
    y, (zs, hs) = forward(Ws, bs, X)
    n = y.size
    d = y - T
    loss = float((d * d).sum() / n)
    g = 2.0 * d / n                      # dL/dy
    dW, db = [None] * 4, [None] * 4
    dW[3] = g.T @ hs[3]
    db[3] = g.sum(0)
    dh = g @ Ws[3].astype(np.float64)
    for l in (2, 1, 0):
        dz = dh * dsilu(zs[l])
        dW[l] = dz.T @ hs[l]
        db[l] = dz.sum(0)
        dh = dz @ Ws[l].astype(np.float64)
    return loss, dW, db
