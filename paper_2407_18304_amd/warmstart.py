"""Learned warm start of the source update (binding of the mgrhd_mlp_* C ABI
and the training driver).

The network maps (state, dt) features of a cell to its post-update
(ln T, ln E_g) and supplies the Newton initial guess; the FP64 solver then
converges to the same root as plain Newton (which stays the fallback).
Training data are produced by the solver itself (mgrhd_source_update) on
seeded synthetic states; the network is trained with the library's own
BF16-MFMA forward/backward kernels and FP32 Adam.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import json
import math
import types
import os

import numpy as np
import torch

from . import mgrhd

_ready = False


def _lib():
    global _ready
    L = mgrhd.lib()
    if not _ready:
        vp, i32, i64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_float
        L.mgrhd_mlp_create.restype = C.c_int
        L.mgrhd_mlp_create.argtypes = [i32, i32, i32, i64, C.c_uint64, C.POINTER(vp)]
        L.mgrhd_mlp_num_params.restype = i64
        L.mgrhd_mlp_num_params.argtypes = [vp]
        L.mgrhd_mlp_get_params.restype = C.c_int
        L.mgrhd_mlp_get_params.argtypes = [vp, vp, i32]
        L.mgrhd_mlp_set_params.restype = C.c_int
        L.mgrhd_mlp_set_params.argtypes = [vp, vp]
        L.mgrhd_mlp_forward.restype = C.c_int
        L.mgrhd_mlp_forward.argtypes = [vp, vp, i64, i64, vp, vp]
        L.mgrhd_mlp_gradients.restype = C.c_int
        L.mgrhd_mlp_gradients.argtypes = [vp, vp, i64, i64, vp, vp, vp]
        L.mgrhd_mlp_adam_step.restype = C.c_int
        L.mgrhd_mlp_adam_step.argtypes = [vp, f32, vp]
        L.mgrhd_mlp_train_step.restype = C.c_int
        L.mgrhd_mlp_train_step.argtypes = [vp, vp, i64, i64, vp, f32, vp, vp]
        phys = [vp] * 5 + [i64, vp, C.POINTER(mgrhd.OpacityParams), C.c_double, C.c_double,
                           C.POINTER(mgrhd.Options)]
        L.mgrhd_mlp_features.restype = C.c_int
        L.mgrhd_mlp_features.argtypes = phys + [vp, vp, vp, vp]
        L.mgrhd_mlp_targets.restype = C.c_int
        L.mgrhd_mlp_targets.argtypes = phys + [vp, vp, vp, vp, vp]
        L.mgrhd_mlp_guess.restype = C.c_int
        L.mgrhd_mlp_guess.argtypes = phys + [vp, vp, vp, i32, vp, vp]
        L.mgrhd_mlp_infer.restype = C.c_int
        L.mgrhd_mlp_infer.argtypes = [vp] + phys + [vp, vp, vp, vp, i32, vp, vp]
        L.mgrhd_mlp_gemm.restype = C.c_int
        L.mgrhd_mlp_gemm.argtypes = [vp, i32, i32, vp, i32, i32, vp, i32, i64, i32, i32, i32,
                                     vp]
        L.mgrhd_mlp_set_fp32_products.restype = C.c_int
        L.mgrhd_mlp_set_fp32_products.argtypes = [vp, i32]
        L.mgrhd_mlp_save.restype = C.c_int
        L.mgrhd_mlp_save.argtypes = [vp, C.c_char_p]
        L.mgrhd_mlp_load.restype = C.c_int
        L.mgrhd_mlp_load.argtypes = [vp, C.c_char_p]
        L.mgrhd_mlp_destroy.restype = None
        L.mgrhd_mlp_destroy.argtypes = [vp]
        _ready = True
    return L


def _f32(t, name):
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and
            t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 device tensor")
    return t.data_ptr()


def _check(rc, what):
    if rc != 0:
        raise mgrhd.MgrhdError(rc, what)


def gemm(A, B, trans_a=False, trans_b=False, fp32=False):
    """C = op(A) op(B) on the matrix cores (BF16 inputs, or FP32 inputs with
    fp32=True; FP32 accumulation)."""
    M, K = (A.shape[1], A.shape[0]) if trans_a else A.shape
    K2, N = (B.shape[1], B.shape[0]) if trans_b else B.shape
    assert K == K2
    Cm = torch.empty((M, N), dtype=torch.float32, device=A.device)
    _check(_lib().mgrhd_mlp_gemm(_f32(A, "A"), A.shape[1], int(trans_a), _f32(B, "B"), B.shape[1],
                                 int(trans_b), Cm.data_ptr(), N, M, N, K, int(fp32),
                                 torch.cuda.current_stream().cuda_stream), "mgrhd_mlp_gemm")
    return Cm


class MLP:
    """n_in -> n_hidden x3 (SiLU) -> n_out, FP32 master weights on the device."""

    def __init__(self, n_in, n_out, n_hidden=128, max_rows=1 << 16, seed=20240718):
        L = _lib()
        h = C.c_void_p()
        _check(L.mgrhd_mlp_create(n_in, n_hidden, n_out, max_rows, seed, C.byref(h)),
               "mgrhd_mlp_create")
        self._h = h
        self.n_in, self.n_out, self.n_hidden, self.max_rows = n_in, n_out, n_hidden, max_rows
        self.n_params = L.mgrhd_mlp_num_params(h)
        self._loss = torch.zeros(1, dtype=torch.float32, device="cuda")

    def _stream(self):
        return torch.cuda.current_stream().cuda_stream

    def get_params(self, which=0) -> np.ndarray:
        out = np.zeros(self.n_params, np.float32)
        _check(_lib().mgrhd_mlp_get_params(self._h, out.ctypes.data, which), "mgrhd_mlp_get_params")
        return out

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.n_params
        _check(_lib().mgrhd_mlp_set_params(self._h, p.ctypes.data), "mgrhd_mlp_set_params")

    def unpack(self, flat):
        """(W1..W4, b1..b4) views of a flat parameter vector."""
        dims = [self.n_in, self.n_hidden, self.n_hidden, self.n_hidden, self.n_out]
        Ws, bs, o = [], [], 0
        for l in range(4):
            Ws.append(flat[o:o + dims[l] * dims[l + 1]].reshape(dims[l + 1], dims[l]))
            o += dims[l] * dims[l + 1]
        for l in range(4):
            bs.append(flat[o:o + dims[l + 1]])
            o += dims[l + 1]
        return Ws, bs

    def set_fp32_products(self, on=True):
        """FP32 operands in the forward and backward products (checking path)."""
        _check(_lib().mgrhd_mlp_set_fp32_products(self._h, int(bool(on))),
               "mgrhd_mlp_set_fp32_products")

    def save_params(self, path):
        """The network's parameters and dimensions to a file (mgrhd_mlp_save)."""
        _check(_lib().mgrhd_mlp_save(self._h, os.fsencode(path)), "mgrhd_mlp_save")

    def load_params(self, path):
        """Parameters from a file written by save_params for a network of the
        same dimensions (mgrhd_mlp_load)."""
        _check(_lib().mgrhd_mlp_load(self._h, os.fsencode(path)), "mgrhd_mlp_load")

    def forward(self, X_fm, rows=None):
        """X_fm: feature-major [n_in x ld] float32 device tensor -> [rows x n_out]."""
        ld = X_fm.shape[1]
        rows = ld if rows is None else rows
        Y = torch.empty((rows, self.n_out), dtype=torch.float32, device=X_fm.device)
        _check(_lib().mgrhd_mlp_forward(self._h, _f32(X_fm, "X"), ld, rows, Y.data_ptr(),
                                        self._stream()), "mgrhd_mlp_forward")
        return Y

    def gradients(self, X_fm, Y_t):
        rows = Y_t.shape[0]
        _check(_lib().mgrhd_mlp_gradients(self._h, _f32(X_fm, "X"), X_fm.shape[1], rows,
                                          _f32(Y_t, "Y"), self._loss.data_ptr(), self._stream()),
               "mgrhd_mlp_gradients")
        return self._loss

    def train_step(self, X_fm, Y_t, lr):
        rows = Y_t.shape[0]
        _check(_lib().mgrhd_mlp_train_step(self._h, _f32(X_fm, "X"), X_fm.shape[1], rows,
                                           _f32(Y_t, "Y"), float(lr), self._loss.data_ptr(),
                                           self._stream()), "mgrhd_mlp_train_step")
        return self._loss

    def close(self):
        if getattr(self, "_h", None):
            _lib().mgrhd_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
def _phys(state, tables, kappa, consts, S_g=None):
    ng, n = state["E_g"].shape
    op = mgrhd.OpacityParams(ng, mgrhd.MEAN_PPL_FIXED, tables["chi_lo"].data_ptr(),
                             tables["alpha"].data_ptr(), None,
                             None if kappa is None else kappa.data_ptr())
    o = mgrhd.default_options()
    o.c, o.a_rad, o.c_v = consts["c"], consts["a_rad"], consts.get("c_v", 1.5)
    o.h_over_k = consts.get("h_over_k", 1.0)
    o.S_g = None if S_g is None else S_g.data_ptr()
    return ([state[k].data_ptr() for k in ("E_g", "F_g", "rho", "e_gas", "v")] +
            [n, tables["edges"].data_ptr(), C.byref(op), float(consts["dt"]),
             float(consts["c_hat"]), C.byref(o)]), (op, o)


def features(state, tables, kappa, consts, mean, inv_std):
    ng, n = state["E_g"].shape
    X = torch.empty((2 + 3 * ng, n), dtype=torch.float32, device=state["E_g"].device)
    args, keep = _phys(state, tables, kappa, consts)
    _check(_lib().mgrhd_mlp_features(*args, _f32(mean, "mean"), _f32(inv_std, "inv_std"),
                                     X.data_ptr(), torch.cuda.current_stream().cuda_stream),
           "mgrhd_mlp_features")
    return X


def targets(state_in, state_out, tables, kappa, consts):
    ng, n = state_in["E_g"].shape
    Y = torch.empty((n, 1 + ng), dtype=torch.float32, device=state_in["E_g"].device)
    args, keep = _phys(state_in, tables, kappa, consts)
    _check(_lib().mgrhd_mlp_targets(*args, state_out["E_g"].data_ptr(),
                                    state_out["e_gas"].data_ptr(), state_out["v"].data_ptr(),
                                    Y.data_ptr(), torch.cuda.current_stream().cuda_stream),
           "mgrhd_mlp_targets")
    return Y


def guess_from(state, tables, kappa, consts, Yn, y_mean, y_std, S_g=None, kind=1):
    """kind 1: E_gas alone [n] (use with guess_kind=1); kind 0: [N_g+1, n]."""
    ng, n = state["E_g"].shape
    shape = (n,) if kind == 1 else (ng + 1, n)
    g = torch.empty(shape, dtype=torch.float64, device=state["E_g"].device)
    args, keep = _phys(state, tables, kappa, consts, S_g)
    _check(_lib().mgrhd_mlp_guess(*args, _f32(Yn, "Y"), _f32(y_mean, "y_mean"),
                                  _f32(y_std, "y_std"), int(kind), g.data_ptr(),
                                  torch.cuda.current_stream().cuda_stream), "mgrhd_mlp_guess")
    return g


@dataclasses.dataclass
class WarmStart:
    """A trained network with its normalisation statistics."""
    net: MLP
    x_mean: torch.Tensor
    x_istd: torch.Tensor
    y_mean: torch.Tensor
    y_std: torch.Tensor
    history: list

    def guess(self, state, tables, kappa, consts, S_g=None, kind=1, fused=True, out=None):
        """Newton guess for the cells of `state`: kind 1 E_gas [n], kind 0
        [N_g+1, n].  fused: one kernel (mgrhd_mlp_infer), written into `out`
        when given (nothing is allocated then); else features, forward and
        guess as three steps."""
        if not fused:
            X = features(state, tables, kappa, consts, self.x_mean, self.x_istd)
            Yn = self.net.forward(X)
            return guess_from(state, tables, kappa, consts, Yn, self.y_mean, self.y_std, S_g,
                              kind)
        ng, n = state["E_g"].shape
        shape = (n,) if kind == 1 else (ng + 1, n)
        if out is not None:
            if tuple(out.shape) != shape or out.dtype != torch.float64 or not out.is_contiguous():
                raise ValueError(f"guess buffer must be contiguous float64 {shape}")
            g = out
        else:
            g = torch.empty(shape, dtype=torch.float64, device=state["E_g"].device)
        args, keep = _phys(state, tables, kappa, consts, S_g)
        _check(_lib().mgrhd_mlp_infer(self.net._h, *args, _f32(self.x_mean, "x_mean"),
                                      _f32(self.x_istd, "x_istd"), _f32(self.y_mean, "y_mean"),
                                      _f32(self.y_std, "y_std"), int(kind), g.data_ptr(),
                                      torch.cuda.current_stream().cuda_stream),
               "mgrhd_mlp_infer")
        return g

    def save(self, path):
        np.savez(path, params=self.net.get_params(), x_mean=self.x_mean.cpu().numpy(),
                 x_istd=self.x_istd.cpu().numpy(), y_mean=self.y_mean.cpu().numpy(),
                 y_std=self.y_std.cpu().numpy(), history=np.asarray(self.history, np.float64),
                 dims=np.asarray([self.net.n_in, self.net.n_hidden, self.net.n_out]))

    @staticmethod
    def load(path, max_rows=1 << 16):
        d = np.load(path, allow_pickle=False)
        n_in, n_hidden, n_out = (int(x) for x in d["dims"])
        net = MLP(n_in, n_out, n_hidden, max_rows=max_rows)
        net.set_params(d["params"])
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
        return WarmStart(net, t(d["x_mean"]), t(d["x_istd"]), t(d["y_mean"]), t(d["y_std"]),
                         list(d["history"]))


@dataclasses.dataclass
class PatchWarmStart:
    """Warm starts for batches of patches: one network per group count."""
    nets: dict           # N_g -> WarmStart

    def attach(self, batch):
        """Attach every network to the patches of its group count in a
        mgrhd.Batch built with guess buffers: the batch's run/capture/launch
        then starts with one fused inference launch per group count over all
        of that count's patches (mgrhd_batch_attach_mlp)."""
        for ng, ws in self.nets.items():
            batch.attach_mlp(ng, ws)

    def guesses(self, dps, outs, kind=1):
        """Write the Newton guess of every patch (synth.DevicePatch-like:
        state, tables, kappa, layout.ng, consts()) into its buffer in `outs`
        with one fused inference launch per patch on the current stream;
        allocates nothing, so the launches can be captured in a graph.
        (attach() does the same with one launch per group count.)"""
        for dp, out in zip(dps, outs):
            self.nets[dp.layout.ng].guess(dp.state, dp.tables, dp.kappa, dp.consts(), kind=kind,
                                          out=out)


def _stats(M, axis):
    M64 = M.double()
    mean = M64.mean(axis)
    std = M64.std(axis).clamp_min(1e-6)
    return mean.float().contiguous(), std.float().contiguous()


def make_training_data(dw, consts, mean_mode=mgrhd.MEAN_PPL_FIXED):
    """Solve a device workload with the FP64 solver (plain Newton) and return
    raw (un-normalised) features and targets."""
    st_in = {k: v.clone() for k, v in dw.state.items()}
    n = dw.n
    zeros = torch.zeros(2 + 3 * dw.ng, dtype=torch.float32, device="cuda")
    ones = torch.ones_like(zeros)
    Xraw = features(st_in, dw.tables, dw.kappa, consts, zeros, ones)
    st = dw.state
    status = torch.zeros(n, dtype=torch.int32, device="cuda")
    mgrhd.source_update(st["E_g"], st["F_g"], st["rho"], st["e_gas"], st["v"], dw.tables["edges"],
                        dw.tables["chi_lo"], alpha_chi=dw.tables["alpha"], kappa_scale=dw.kappa,
                        mean_mode=mean_mode, polish=1, status=status, **consts)
    Yraw = targets(st_in, st, dw.tables, dw.kappa, consts)
    torch.cuda.synchronize()
    ok = status == 0
    return Xraw, Yraw, ok


def make_training_data_patches(dps, mean_mode=mgrhd.MEAN_PPL_FIXED):
    """Solver pairs from device patches (synth.DevicePatch) that share one
    group count, each with its own edges, opacity table, dt and c_hat: raw
    features [F x n], targets [n x O] and the converged mask over all their
    cells.  The patches' states are overwritten by the solve."""
    Xs, Ys, oks = [], [], []
    for dp in dps:
        shim = types.SimpleNamespace(state=dp.state, tables=dp.tables, kappa=dp.kappa,
                                     n=dp.layout.n, ng=dp.layout.ng)
        X, Y, ok = make_training_data(shim, dp.consts(), mean_mode)
        Xs.append(X)
        Ys.append(Y)
        oks.append(ok)
    return torch.cat(Xs, 1).contiguous(), torch.cat(Ys, 0).contiguous(), torch.cat(oks)


def train(Xraw, Yraw, ok, *, epochs=8, batch=4096, lr=2e-3, n_hidden=128, seed=20240718,
          holdout=1 << 16, t_weight=8.0, log=None):
    """Train on the rows of (Xraw [F x n], Yraw [n x O]) with ok; returns a
    WarmStart and the held-out loss history.  The temperature output (the
    one the Newton guess uses) is normalised by its spread / t_weight, which
    weights its squared error t_weight^2 times more than the other outputs'."""
    idx = torch.nonzero(ok).flatten()
    g = torch.Generator(device="cpu").manual_seed(seed)
    perm = idx[torch.randperm(idx.numel(), generator=g).to(idx.device)]
    hold, tr = perm[:holdout], perm[holdout:]
    x_mean, x_std = _stats(Xraw[:, tr], 1)
    y_mean, y_std = _stats(Yraw[tr], 0)
    y_std[0] = y_std[0] / t_weight
    x_istd = (1.0 / x_std).contiguous()
    X = ((Xraw - x_mean[:, None]) * x_istd[:, None]).contiguous()
    Y = ((Yraw - y_mean[None, :]) / y_std[None, :]).contiguous()
    # rows per forward chunk: the activations of 2^20 rows take ~3 GB
    net = MLP(X.shape[0], Y.shape[1], n_hidden, max_rows=max(batch, 1 << 20), seed=seed)
    Xh, Yh = X[:, hold].contiguous(), Y[hold].contiguous()
    history = []
    steps_per_epoch = max(1, tr.numel() // batch)
    total = epochs * steps_per_epoch
    step = 0
    for ep in range(epochs):
        order = tr[torch.randperm(tr.numel(), generator=g).to(tr.device)]
        for s in range(steps_per_epoch):
            rows = order[s * batch:(s + 1) * batch]
            xb, yb = X[:, rows].contiguous(), Y[rows].contiguous()
            # cosine learning-rate schedule
            lr_t = 0.5 * lr * (1.0 + math.cos(math.pi * step / total))
            net.train_step(xb, yb, lr_t)
            step += 1
        Yp = net.forward(Xh)
        hl = float(((Yp - Yh) ** 2).mean())
        history.append(hl)
        if log:
            log(f"epoch {ep}: held-out loss {hl:.4e}")
    return WarmStart(net, x_mean, x_istd, y_mean, y_std, history)
