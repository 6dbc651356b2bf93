"""The FP64 numpy reference of the warm-start network (used to check the GPU
forward/backward kernels), pinned against central finite differences."""
import numpy as np

import mlp_ref


def _net(rng, dims):
    Ws = [rng.normal(0, 1 / np.sqrt(dims[l]), (dims[l + 1], dims[l])) for l in range(4)]
    bs = [rng.normal(0, 0.1, dims[l + 1]) for l in range(4)]
    return Ws, bs


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    dims = [7, 9, 9, 9, 4]
    Ws, bs = _net(rng, dims)
    X = rng.normal(size=(11, dims[0]))
    T = rng.normal(size=(11, dims[-1]))
    loss, dW, db = mlp_ref.loss_and_grads(Ws, bs, X, T)
    h = 1e-6
    for l in range(4):
        for (i, j) in [(0, 0), (dims[l + 1] - 1, dims[l] - 1), (1, 2)]:
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][i, j] += h
            Wm[l][i, j] -= h
            fd = (mlp_ref.loss_and_grads(Wp, bs, X, T)[0] -
                  mlp_ref.loss_and_grads(Wm, bs, X, T)[0]) / (2 * h)
            assert abs(fd - dW[l][i, j]) <= 1e-7 * max(1.0, abs(fd))
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[l][1] += h
        bm[l][1] -= h
        fd = (mlp_ref.loss_and_grads(Ws, bp, X, T)[0] - mlp_ref.loss_and_grads(Ws, bm, X, T)[0]) / (2 * h)
        assert abs(fd - db[l][1]) <= 1e-7 * max(1.0, abs(fd))


def test_silu_derivative():
    z = np.linspace(-8, 8, 41)
    h = 1e-6
    fd = (mlp_ref.silu(z + h) - mlp_ref.silu(z - h)) / (2 * h)
    assert np.allclose(fd, mlp_ref.dsilu(z), atol=1e-8)
