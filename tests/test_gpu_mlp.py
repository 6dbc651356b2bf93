"""The warm-start network on the GPU: the BF16 matrix-core product (lane
layout and all transpose forms), forward/backward against the FP64 numpy
reference, training, and the warm-started solve.  GPU only."""
import numpy as np
import pytest
import torch

import mlp_ref
from paper_2407_18304_amd import mgrhd, synth, warmstart
from paper_2407_18304_amd import workloads as W

import gpu_util as U

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even)."""
    b = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("ta,tb", [(False, False), (False, True), (True, False), (True, True)])
@pytest.mark.parametrize("M,N,K", [(16, 16, 32), (100, 70, 45), (257, 130, 194)])
def test_matrix_core_product(ta, tb, M, N, K, fp32):
    """BF16 operands (fp32 False) or FP32 operands, FP32 accumulation, every
    transpose form, ragged tiles: against the exact product of the operands
    as the kernel takes them."""
    rng = np.random.default_rng(M + N + K)
    A = rng.normal(size=(K, M) if ta else (M, K)).astype(np.float32)
    B = rng.normal(size=(N, K) if tb else (K, N)).astype(np.float32)
    Cg = warmstart.gemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), ta, tb, fp32)
    Ar = A.astype(np.float64) if fp32 else bf16_round(A).astype(np.float64)
    Br = B.astype(np.float64) if fp32 else bf16_round(B).astype(np.float64)
    ref = (Ar.T if ta else Ar) @ (Br.T if tb else Br)
    err = np.abs(Cg.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 1e-5, err


def _small_net(ng=4, seed=3):
    n_in, n_out = 2 + 3 * ng, 1 + ng
    net = warmstart.MLP(n_in, n_out, 128, max_rows=4096, seed=seed)
    return net


def test_forward_and_gradients_match_fp64_reference():
    """Forward, loss and every layer's weight and bias gradients against the
    FP64 reference that rounds both operands of every matrix product to BF16
    where the kernels do (staging of each product's tiles), with exact
    products: within 1e-3 per layer (what remains is FP32 accumulation and
    the odd operand rounded the other way after an FP32-level difference)."""
    rng = np.random.default_rng(5)
    net = _small_net()
    p = net.get_params()
    Ws, bs = net.unpack(p.astype(np.float64))
    rows = 512
    X = rng.normal(size=(rows, net.n_in)).astype(np.float32)
    T = rng.normal(size=(rows, net.n_out)).astype(np.float32)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()       # feature-major
    Td = torch.from_numpy(T).cuda()
    Y = net.forward(Xd).cpu().numpy()
    rnd = mlp_ref.bf16_round
    yref, _ = mlp_ref.forward(Ws, bs, X.astype(np.float64), rnd)
    assert np.abs(Y - yref).max() / np.abs(yref).max() < 1e-3
    loss = float(net.gradients(Xd, Td).cpu())
    g = net.get_params(which=1)
    gW, gb = net.unpack(g.astype(np.float64))
    lref, dW, db = mlp_ref.loss_and_grads(Ws, bs, X.astype(np.float64), T.astype(np.float64),
                                          rnd)
    assert abs(loss - lref) < 1e-4 * lref
    errs = []
    for l in range(4):
        eW = np.linalg.norm(gW[l] - dW[l]) / np.linalg.norm(dW[l])
        eb = np.linalg.norm(gb[l] - db[l]) / np.linalg.norm(db[l])
        errs.append((eW, eb))
        assert eW < 1e-3 and eb < 1e-3, (l, eW, eb)
    print("per-layer gradient errors (W, b):", errs)


def test_fp32_products_gradients_match_fp64_reference():
    """The FP32 checking path (FP32 operands in every product): forward,
    loss and per-layer gradients against the exact FP64 network within 1e-6
    (FP32 rounding of stored activations and of the accumulation)."""
    rng = np.random.default_rng(9)
    net = _small_net(seed=4)
    net.set_fp32_products(True)
    p = net.get_params()
    Ws, bs = net.unpack(p.astype(np.float64))
    rows = 384
    X = rng.normal(size=(rows, net.n_in)).astype(np.float32)
    T = rng.normal(size=(rows, net.n_out)).astype(np.float32)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    Td = torch.from_numpy(T).cuda()
    Y = net.forward(Xd).cpu().numpy()
    yref, _ = mlp_ref.forward(Ws, bs, X.astype(np.float64))
    assert np.abs(Y - yref).max() / np.abs(yref).max() < 1e-6
    loss = float(net.gradients(Xd, Td).cpu())
    g = net.get_params(which=1)
    gW, gb = net.unpack(g.astype(np.float64))
    lref, dW, db = mlp_ref.loss_and_grads(Ws, bs, X.astype(np.float64), T.astype(np.float64))
    assert abs(loss - lref) < 1e-6 * lref
    for l in range(4):
        eW = np.linalg.norm(gW[l] - dW[l]) / np.linalg.norm(dW[l])
        eb = np.linalg.norm(gb[l] - db[l]) / np.linalg.norm(db[l])
        assert eW < 1e-6 and eb < 1e-6, (l, eW, eb)
    net.set_fp32_products(False)
    Yb = net.forward(Xd).cpu().numpy()
    assert np.abs(Yb - Y).max() > 1e-6 * np.abs(Y).max()       # back on BF16 operands


def test_training_reduces_loss_on_a_smooth_map():
    rng = np.random.default_rng(7)
    net = _small_net(seed=11)
    n = 16384
    X = rng.normal(size=(n, net.n_in)).astype(np.float32)
    T = np.stack([np.sin(X[:, k % net.n_in]) + 0.3 * X[:, (k + 1) % net.n_in] ** 2
                  for k in range(net.n_out)], 1).astype(np.float32)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    Td = torch.from_numpy(T).cuda()
    first = None
    for step in range(300):
        rows = torch.from_numpy(rng.choice(n, 1024, replace=False)).cuda()
        loss = float(net.train_step(Xd[:, rows].contiguous(), Td[rows].contiguous(), 3e-3).cpu())
        first = first or loss
    final = float(((net.forward(Xd) - Td) ** 2).mean())
    assert final < 0.1 * first, (first, final)


@pytest.mark.parametrize("n", [1000, 4096 + 17])
def test_fused_inference_matches_three_kernel_path(n):
    """mgrhd_mlp_infer (features, layers and guess in one kernel) against the
    three-kernel path (features, matrix-core forward, guess) on a random
    network with the 64-group feature layout: both guess kinds, ragged tile."""
    dw = synth.device_workload("config2", n=n)
    ng = dw.ng
    net = warmstart.MLP(2 + 3 * ng, 1 + ng, 128, max_rows=2048, seed=5)
    rng = np.random.default_rng(1)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    Xr = warmstart.features(dw.state, dw.tables, dw.kappa, dw.consts(),
                            torch.zeros(2 + 3 * ng, device="cuda"),
                            torch.ones(2 + 3 * ng, device="cuda"))
    x_mean, x_std = Xr.mean(1), Xr.std(1).clamp_min(1e-3)
    ws = warmstart.WarmStart(net, x_mean.contiguous(), (1.0 / x_std).contiguous(),
                             t(rng.normal(0, 0.1, 1 + ng)), t(np.full(1 + ng, 0.05)), [])
    for kind in (1, 0):
        a = ws.guess(dw.state, dw.tables, dw.kappa, dw.consts(), kind=kind, fused=True)
        b = ws.guess(dw.state, dw.tables, dw.kappa, dw.consts(), kind=kind, fused=False)
        torch.cuda.synchronize()
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.isfinite(a).all()
        e0 = np.abs(a.reshape(-1, n)[0] - b.reshape(-1, n)[0]) / np.abs(b.reshape(-1, n)[0])
        assert e0.max() < 5e-3, (kind, e0.max())          # BF16 products, FP32 features
        if kind == 0:
            E0 = dw.state["E_g"].cpu().numpy()
            ra, rb = a[1:] + E0, b[1:] + E0                     # the guessed E_g
            assert (np.abs(ra - rb) <= 5e-3 * np.abs(rb) + 1e-300).all()


def test_warm_start_same_result_fewer_iterations():
    """Train on solver-generated pairs of the 64-group workload (training
    seed), then solve fresh cells of the workload itself with and without the
    network's temperature guess (guess kind 1)."""
    dw_train = synth.device_workload("config2", n=1 << 16, seed=W.TRAIN_SEED)
    consts = dw_train.consts()
    Xr, Yr, ok = warmstart.make_training_data(dw_train, consts)
    ws = warmstart.train(Xr, Yr, ok, epochs=8, batch=1024, holdout=4096)
    assert ws.history[-1] < ws.history[0]
    del dw_train, Xr, Yr
    dw = synth.device_workload("config2", n=8192)
    pristine = {k: v.clone() for k, v in dw.state.items()}
    res = {}
    for name in ("plain", "warm"):
        for k in dw.state:
            dw.state[k].copy_(pristine[k])
        guess = ws.guess(dw.state, dw.tables, dw.kappa, consts) if name == "warm" else None
        it = torch.zeros(dw.n, dtype=torch.int32, device="cuda")
        stt = torch.zeros(dw.n, dtype=torch.int32, device="cuda")
        st = dw.state
        mgrhd.source_update(st["E_g"], st["F_g"], st["rho"], st["e_gas"], st["v"],
                            dw.tables["edges"], dw.tables["chi_lo"], alpha_chi=dw.tables["alpha"],
                            kappa_scale=dw.kappa, mean_mode=1, polish=1, guess=guess,
                            guess_kind=1, iters=it, status=stt, **consts)
        torch.cuda.synchronize()
        res[name] = ({k: v.cpu().numpy() for k, v in st.items()}, it.cpu().numpy(),
                     stt.cpu().numpy())
    (gp, ip, sp), (gw, iw, sw) = res["plain"], res["warm"]
    ok = (sp == 0) & ((sw & ~4) == 0)
    assert ok.mean() > 0.98
    host = synth.to_host(dw, np.arange(dw.n))
    host.state = {k: v.cpu().numpy() for k, v in pristine.items()}
    for k, e in U.field_errors(host, gw, gp, ok).items():
        assert e < U.TOL, (k, e)
    print(f"held-out loss {ws.history[0]:.3e} -> {ws.history[-1]:.3e}; Newton steps per cell: "
          f"plain {ip[ok].mean():.3f}, warm {iw[ok].mean():.3f}; fallbacks {((sw & 4) != 0).mean():.4f}")
    assert iw[ok].mean() < ip[ok].mean()


def test_parameters_save_and_load(tmp_path):
    """mgrhd_mlp_save / mgrhd_mlp_load: the parameters come back bit for bit;
    a file of other dimensions is refused."""
    a = warmstart.MLP(26, 9)
    p = a.get_params().copy()
    path = tmp_path / "net.bin"
    a.save_params(path)
    b = warmstart.MLP(26, 9, seed=5)
    assert not np.array_equal(b.get_params(), p)
    b.load_params(path)
    assert np.array_equal(b.get_params(), p)
    c = warmstart.MLP(30, 9)
    with pytest.raises(mgrhd.MgrhdError) as e:
        c.load_params(path)
    assert e.value.code == mgrhd.E_SIZE
    with pytest.raises(mgrhd.MgrhdError) as e:
        b.load_params(tmp_path / "missing.bin")
    assert e.value.code == mgrhd.E_OPTION


def _host_features(dw, x_mean, x_istd):
    """The network's inputs written out on the host in FP64 from the state
    (ln T, ln rho, per group ln(E_g / a T^4), |F_g|/(c E_g) and
    ln(c_hat dt rho kappa chi_0,g) with the PPL-fixed group mean of eq. chiQg
    at alpha_Q = -1, chi_0E,g / chi_0,g- = expm1(alpha L)/(alpha L)),
    normalised with the same statistics.  Returns [2 + 3 N_g, n]."""
    st = {k: v.cpu().numpy() for k, v in dw.state.items()}
    ng, n = st["E_g"].shape
    c = dw.consts()
    rho, v = st["rho"], st["v"]
    T = np.maximum((st["e_gas"] - 0.5 * rho * (v ** 2).sum(0)) / (rho * c["c_v"]), 1e-300)
    aT4 = c["a_rad"] * T ** 4
    kap = dw.kappa.cpu().numpy()
    L = np.log(dw.edges[1:] / dw.edges[:-1])
    aL = dw.alpha_chi * L
    ratio = np.where(aL != 0.0, np.expm1(aL) / np.where(aL != 0.0, aL, 1.0), 1.0)
    lchi = np.log(dw.chi_lo * ratio)
    E = st["E_g"]
    F = np.sqrt((st["F_g"] ** 2).sum(0))
    pos = E > 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        le = np.where(pos, np.clip(np.log(E / aT4), -50.0, 50.0), -50.0)
        fr = np.where(pos, np.minimum(F / (c["c"] * E), 2.0), 0.0)
    lcell = np.log(c["c_hat"] * c["dt"] * rho * kap)
    X = np.concatenate([np.log(T)[None], np.log(rho)[None], le, fr, lcell[None] + lchi[:, None]])
    m = x_mean.cpu().numpy().astype(np.float64)[:, None]
    s = x_istd.cpu().numpy().astype(np.float64)[:, None]
    return (X - m) * s, T, rho, 0.5 * rho * (v ** 2).sum(0)


def test_inference_against_host_reference():
    """The features kernel, the three-kernel path and the fused inference
    against a host reference: features from their definitions in FP64, the
    network by the FP64 reference with BF16 operands (mlp_ref), the Newton
    temperature guess from its output.  The GPU forms features in FP32 and
    SiLU in FP32 before rounding to BF16; a value that lands on the other side
    of a BF16 rounding boundary moves a product by 2^-8 of one term, so the
    network output agrees to ~1e-3 of its scale, the guess (y_std = 0.05)
    to ~1e-4 relative."""
    n = 3000
    dw = synth.device_workload("config2", n=n)
    ng = dw.ng
    net = warmstart.MLP(2 + 3 * ng, 1 + ng, 128, max_rows=4096, seed=7)
    rng = np.random.default_rng(2)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    Xr = warmstart.features(dw.state, dw.tables, dw.kappa, dw.consts(),
                            torch.zeros(2 + 3 * ng, device="cuda"),
                            torch.ones(2 + 3 * ng, device="cuda"))
    x_mean = Xr.mean(1).contiguous()
    x_istd = (1.0 / Xr.std(1).clamp_min(1e-3)).contiguous()
    y_mean, y_std = t(rng.normal(0, 0.1, 1 + ng)), t(np.full(1 + ng, 0.05))
    ws = warmstart.WarmStart(net, x_mean, x_istd, y_mean, y_std, [])
    Xh, T, rho, ke = _host_features(dw, x_mean, x_istd)
    # the features kernel (FP64 math, FP32 output)
    Xg = warmstart.features(dw.state, dw.tables, dw.kappa, dw.consts(), x_mean, x_istd)
    Xg = Xg.cpu().numpy().astype(np.float64)
    assert np.abs(Xg - Xh).max() <= 1e-6 * (1.0 + np.abs(Xh).max()), np.abs(Xg - Xh).max()
    # the network on the host, BF16 operands, FP64 sums
    Ws, bs = net.unpack(net.get_params())
    Ws = [w.astype(np.float64) for w in Ws]
    bs = [b.astype(np.float64) for b in bs]
    Y, _ = mlp_ref.forward(Ws, bs, Xh.T, mlp_ref.bf16_round)
    yT = Y[:, 0] * float(y_std[0]) + float(y_mean[0])
    g_ref = rho * dw.c_v * T * np.exp(np.clip(yT, -5.0, 5.0)) + ke
    for fused in (True, False):
        g = ws.guess(dw.state, dw.tables, dw.kappa, dw.consts(), kind=1, fused=fused)
        torch.cuda.synchronize()
        e = np.abs(g.cpu().numpy() - g_ref) / np.abs(g_ref)
        print(f"fused={fused}: max rel guess error {e.max():.3e}, median {np.median(e):.3e}")
        assert e.max() < 1e-3, (fused, e.max())
        assert np.median(e) < 1e-5, (fused, np.median(e))
