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


def test_bf16_rounding_matches_torch():
    """The operand rounding equals torch's float32 -> bfloat16 conversion
    (round to nearest, ties to even), including ties and subnormals."""
    import torch
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.uniform(-30, 30, 4000),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 0.0,
                                  1e-40, -3e-39, 3.3e38])]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp_ref.bf16_round(x), want)


def test_rounded_reference_reduces_to_exact_and_rounds_operands():
    """rnd=None is the exact network; with identity rounding the rounded
    path is the same computation; with BF16 rounding the gradients stay
    within the operands' relative precision (2^-8) of the exact ones."""
    rng = np.random.default_rng(1)
    dims = [10, 16, 16, 16, 5]
    Ws, bs = _net(rng, dims)
    X = rng.normal(size=(40, dims[0]))
    T = rng.normal(size=(40, dims[-1]))
    l0, dW0, db0 = mlp_ref.loss_and_grads(Ws, bs, X, T)
    l1, dW1, db1 = mlp_ref.loss_and_grads(Ws, bs, X, T, rnd=lambda a: a)
    assert l0 == l1 and all(np.array_equal(a, b) for a, b in zip(dW0 + db0, dW1 + db1))
    l2, dW2, db2 = mlp_ref.loss_and_grads(Ws, bs, X, T, rnd=mlp_ref.bf16_round)
    assert 0 < abs(l2 - l0) < 2 ** -7 * l0
    for l in range(4):
        e = np.linalg.norm(dW2[l] - dW0[l]) / np.linalg.norm(dW0[l])
        assert 0 < e < 2 ** -6, (l, e)
