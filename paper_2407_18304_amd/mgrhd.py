"""Python binding of the C ABI in include/mgrhd.h (argument marshalling only).

Every step of the source update runs in the HIP kernels of ``libmgrhd.so``;
this module checks tensor shapes/dtypes/devices, passes device pointers and
the current HIP stream, and raises on a non-zero return.  There is no CPU
fallback: without the built library or a GPU the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmgrhd.so")

MEAN_PC, MEAN_PPL_FIXED, MEAN_PPL_FREE = 0, 1, 2
CLOSURE_M1, CLOSURE_EDDINGTON = 0, 1
E_NULL, E_SIZE, E_MODE, E_TABLE, E_SCALAR, E_OPTION, E_DEVICE = -1, -2, -3, -4, -5, -6, -7
ST_OK, ST_NEWTON_MAXIT, ST_OUTER_MAXIT, ST_FALLBACK, ST_INVALID, ST_NONFINITE, ST_BAD_TABLE = (
    0, 1, 2, 4, 8, 16, 32)
MAX_GROUPS = 256

ERRORS = {-1: "NULL pointer", -2: "size out of range", -3: "unknown mode or closure",
          -4: "powerlaw mode needs alpha_chi or chi_hi", -5: "non-positive scalar",
          -6: "option out of range", -7: "no usable device"}


class MgrhdError(RuntimeError):
    def __init__(self, code: int, what: str = "mgrhd_source_update"):
        msg = ERRORS.get(code, f"HIP error {code}")
        super().__init__(f"{what} failed: {msg} (code {code})")
        self.code = code


class OpacityParams(C.Structure):
    _fields_ = [("n_groups", C.c_int32), ("mean_mode", C.c_int32), ("chi_lo", C.c_void_p),
                ("alpha_chi", C.c_void_p), ("chi_hi", C.c_void_p), ("kappa_scale", C.c_void_p),
                ("t_exp", C.c_double), ("t_ref", C.c_double), ("stim", C.c_int32),
                ("reserved", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("c", C.c_double), ("a_rad", C.c_double), ("h_over_k", C.c_double),
                ("c_v", C.c_double), ("eps_newton", C.c_double), ("eps_outer", C.c_double),
                ("max_newton", C.c_int32), ("max_outer", C.c_int32), ("closure", C.c_int32),
                ("polish", C.c_int32), ("S_g", C.c_void_p), ("guess", C.c_void_p),
                ("iters", C.c_void_p), ("outer", C.c_void_p), ("status", C.c_void_p),
                ("guess_kind", C.c_int32), ("reserved", C.c_int32), ("trace", C.c_void_p),
                ("E_g_out", C.c_void_p), ("F_g_out", C.c_void_p), ("e_gas_out", C.c_void_p),
                ("v_out", C.c_void_p)]


_lib = None

# exported symbols of include/mgrhd.h
SYMBOLS = ["mgrhd_source_update", "mgrhd_default_options", "mgrhd_get_variant",
           "mgrhd_recommend_mean_mode",
           "mgrhd_set_variant", "mgrhd_variant_count", "mgrhd_variant_info",
           "mgrhd_imex_workspace_bytes", "mgrhd_imex_step", "mgrhd_imex_step_noalloc",
           "mgrhd_version",
           "mgrhd_transport1d_stage"]


def lib():
    """Load libmgrhd.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        L.mgrhd_source_update.restype = C.c_int
        L.mgrhd_source_update.argtypes = [C.c_void_p] * 5 + [C.c_int64, C.c_void_p,
                                                              C.POINTER(OpacityParams),
                                                              C.c_double, C.c_double, C.c_void_p,
                                                              C.POINTER(Options)]
        L.mgrhd_default_options.restype = None
        L.mgrhd_default_options.argtypes = [C.POINTER(Options)]
        L.mgrhd_get_variant.restype = C.c_int
        L.mgrhd_get_variant.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                        C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.mgrhd_set_variant.restype = C.c_int
        L.mgrhd_set_variant.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32]
        L.mgrhd_variant_count.restype = C.c_int32
        L.mgrhd_variant_count.argtypes = []
        L.mgrhd_variant_info.restype = C.c_int
        L.mgrhd_variant_info.argtypes = [C.c_int32] + [C.POINTER(C.c_int32)] * 3
        L.mgrhd_imex_workspace_bytes.restype = C.c_size_t
        L.mgrhd_imex_workspace_bytes.argtypes = [C.c_int64, C.c_int32]
        L.mgrhd_imex_step.restype = C.c_int
        L.mgrhd_imex_step.argtypes = (L.mgrhd_source_update.argtypes +
                                      [C.c_void_p, C.c_size_t])
        L.mgrhd_imex_step_noalloc.restype = C.c_int
        L.mgrhd_imex_step_noalloc.argtypes = L.mgrhd_source_update.argtypes
        L.mgrhd_version.restype = C.c_char_p
        L.mgrhd_version.argtypes = []
        _lib = L
    return _lib


def _ptr(t, shape=None, dtype=torch.float64, name="array"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


def default_options() -> Options:
    o = Options()
    lib().mgrhd_default_options(C.byref(o))
    return o


def get_variant(n_groups: int, mean_mode: int = MEAN_PPL_FIXED):
    """(lanes per cell, groups per lane, waves per SIMD) used for n_groups."""
    lpc, gpl, wps = C.c_int32(), C.c_int32(), C.c_int32()
    rc = lib().mgrhd_get_variant(n_groups, mean_mode, C.byref(lpc), C.byref(gpl), C.byref(wps))
    if rc:
        raise MgrhdError(rc, "mgrhd_get_variant")
    return lpc.value, gpl.value, wps.value


def transport1d_stage(out, U1, U0, *, a, b, dx, dt_T, c, c_hat, rho, chi_mid, E_left,
                      E_right, stream=None):
    """out = a U0 + b U1 + dt_T T(U1) for a 1D column (mgrhd_transport1d_stage).
    out, U1, U0: dicts of device tensors E_g [N_g, n], F_g [3, N_g, n],
    e_gas [n], v [3, n]; U0 may be None when a == 0."""
    ng, n = U1["E_g"].shape
    L = lib()
    f = L.mgrhd_transport1d_stage
    f.restype = C.c_int
    f.argtypes = [C.c_void_p] * 12 + [C.c_double, C.c_double, C.c_int64, C.c_int32,
                                      C.c_double, C.c_double, C.c_double, C.c_double,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p]
    shapes = {"E_g": (ng, n), "F_g": (3, ng, n), "e_gas": (n,), "v": (3, n)}
    keys = ("E_g", "F_g", "e_gas", "v")
    po = [_ptr(out[k], shapes[k], name=k) for k in keys]
    p1 = [_ptr(U1[k], shapes[k], name=k) for k in keys]
    p0 = [_ptr(U0[k], shapes[k], name=k) if U0 is not None else None for k in keys]
    if stream is None:
        stream = torch.cuda.current_stream(U1["E_g"].device).cuda_stream
    rc = f(*po, *p1, *p0, float(a), float(b), n, ng, float(dx), float(dt_T), float(c),
           float(c_hat), _ptr(rho, (n,), name="rho"), _ptr(chi_mid, (ng,), name="chi_mid"),
           _ptr(E_left, (ng,), name="E_left"), _ptr(E_right, (ng,), name="E_right"), stream)
    if rc != 0:
        raise MgrhdError(rc, "mgrhd_transport1d_stage")


def imex_workspace_bytes(n_cells: int, n_groups: int) -> int:
    return int(lib().mgrhd_imex_workspace_bytes(n_cells, n_groups))


def variants():
    """Compiled variants: list of (lanes per cell, groups per lane, waves per SIMD)."""
    out = []
    for k in range(lib().mgrhd_variant_count()):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        if lib().mgrhd_variant_info(k, C.byref(a), C.byref(b), C.byref(c)) == 0:
            out.append((a.value, b.value, c.value))
    return out


def recommend_mean_mode(edges) -> int:
    """The paper's choice of mean-opacity method for a group structure
    (mgrhd_recommend_mean_mode): MEAN_PC or MEAN_PPL_FIXED."""
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.float64))
    L = lib()
    L.mgrhd_recommend_mean_mode.restype = C.c_int32
    L.mgrhd_recommend_mean_mode.argtypes = [C.c_int32, C.c_void_p]
    rc = L.mgrhd_recommend_mean_mode(len(e) - 1, e.ctypes.data)
    if rc < 0:
        raise MgrhdError(rc, "mgrhd_recommend_mean_mode")
    return rc


def set_variant(n_groups: int, lanes_per_cell: int, groups_per_lane: int,
                waves_per_simd: int = 0):
    rc = lib().mgrhd_set_variant(n_groups, lanes_per_cell, groups_per_lane, waves_per_simd)
    if rc:
        raise MgrhdError(rc, "mgrhd_set_variant")


def source_update(E_g, F_g, rho, e_gas, v, group_edges, chi_lo, *, dt, c_hat,
                  mean_mode=MEAN_PPL_FIXED, alpha_chi=None, chi_hi=None, kappa_scale=None,
                  c=1.0, a_rad=1.0, h_over_k=1.0, c_v=1.5, eps_newton=1e-11, eps_outer=1e-13,
                  max_newton=100, max_outer=20, closure=CLOSURE_M1, polish=0, S_g=None,
                  guess=None, guess_kind=0, iters=None, outer=None, status=None, stream=None,
                  imex_work=None, imex_noalloc=False, t_exp=0.0, t_ref=1.0, stim=0,
                  trace=None, out=None):
    """Source update of the device state (see include/mgrhd.h): in place, or
    with out=(E_g_out, F_g_out, e_gas_out, v_out) (tensors shaped as the
    inputs) from the given state into those, leaving the inputs unchanged.
    guess_kind 0: guess is [N_g+1, n] (E_gas, R_g); 1: guess is [n] (E_gas).
    imex_work: a device tensor of at least imex_workspace_bytes(n, N_g) bytes
    turns the call into one two-stage IMEX step (mgrhd_imex_step);
    imex_noalloc=True makes it the IMEX step that keeps U^(n+1/2) in the
    library's own array and allocates nothing (mgrhd_imex_step_noalloc).
    t_exp, t_ref, stim: temperature dependence of the opacity,
    (T/t_ref)^t_exp [1 - exp(-h nu / k T)]^stim.
    trace: optional int32 device tensor [max_outer, n] receiving the
    cumulative Newton steps at the end of every inner pass (-1: not run)."""
    ng, n = E_g.shape
    o = default_options()
    o.c, o.a_rad, o.h_over_k, o.c_v = c, a_rad, h_over_k, c_v
    o.eps_newton, o.eps_outer = eps_newton, eps_outer
    o.max_newton, o.max_outer, o.closure, o.polish = max_newton, max_outer, closure, polish
    o.S_g = _ptr(S_g, (ng, n), name="S_g")
    o.guess = _ptr(guess, (ng + 1, n) if guess_kind == 0 else (n,), name="guess")
    o.guess_kind = guess_kind
    o.iters = _ptr(iters, (n,), torch.int32, "iters")
    o.outer = _ptr(outer, (n,), torch.int32, "outer")
    o.status = _ptr(status, (n,), torch.int32, "status")
    o.trace = _ptr(trace, (max_outer, n), torch.int32, "trace")
    if out is not None:
        Eo, Fo, eo, vo = out
        o.E_g_out = _ptr(Eo, (ng, n), name="E_g_out")
        o.F_g_out = _ptr(Fo, (3, ng, n), name="F_g_out")
        o.e_gas_out = _ptr(eo, (n,), name="e_gas_out")
        o.v_out = _ptr(vo, (3, n), name="v_out")
    op = OpacityParams(ng, mean_mode, _ptr(chi_lo, (ng,), name="chi_lo"),
                       _ptr(alpha_chi, (ng,), name="alpha_chi"),
                       _ptr(chi_hi, (ng,), name="chi_hi"),
                       _ptr(kappa_scale, (n,), name="kappa_scale"),
                       float(t_exp), float(t_ref), int(stim), 0)
    if stream is None:
        stream = torch.cuda.current_stream(E_g.device).cuda_stream
    args = (_ptr(E_g, (ng, n), name="E_g"), _ptr(F_g, (3, ng, n), name="F_g"),
            _ptr(rho, (n,), name="rho"), _ptr(e_gas, (n,), name="e_gas"),
            _ptr(v, (3, n), name="v"), n, _ptr(group_edges, (ng + 1,), name="group_edges"),
            C.byref(op), float(dt), float(c_hat), stream, C.byref(o))
    if imex_noalloc:
        if imex_work is not None:
            raise ValueError("imex_noalloc takes no imex_work")
        rc = lib().mgrhd_imex_step_noalloc(*args)
    elif imex_work is None:
        rc = lib().mgrhd_source_update(*args)
    else:
        if not (isinstance(imex_work, torch.Tensor) and imex_work.is_cuda and
                imex_work.is_contiguous()):
            raise TypeError("imex_work must be a contiguous device tensor")
        rc = lib().mgrhd_imex_step(*args, imex_work.data_ptr(),
                                   imex_work.numel() * imex_work.element_size())
    if rc != 0:
        raise MgrhdError(rc)


# --------------------------------------------------------------------------
# Batched patches (include/mgrhd.h, mgrhd_batch_*)
class Patch(C.Structure):
    _fields_ = [("E_g", C.c_void_p), ("F_g", C.c_void_p), ("rho", C.c_void_p),
                ("e_gas", C.c_void_p), ("v", C.c_void_p), ("kappa_scale", C.c_void_p),
                ("S_g", C.c_void_p), ("guess", C.c_void_p), ("iters", C.c_void_p),
                ("outer", C.c_void_p), ("status", C.c_void_p), ("group_edges", C.c_void_p),
                ("chi_lo", C.c_void_p), ("alpha_chi", C.c_void_p), ("chi_hi", C.c_void_p),
                ("n_cells", C.c_int64), ("n_groups", C.c_int32), ("reserved", C.c_int32),
                ("dt", C.c_double), ("c_hat", C.c_double), ("trace", C.c_void_p),
                ("E_g_out", C.c_void_p), ("F_g_out", C.c_void_p), ("e_gas_out", C.c_void_p),
                ("v_out", C.c_void_p)]


SYMBOLS += ["mgrhd_batch_set_item_scope", "mgrhd_batch_get_item_scope", "mgrhd_batch_tune",
            "mgrhd_batch_attach_mlp", "mgrhd_batch_infer"]
SYMBOLS += ["mgrhd_batch_create", "mgrhd_batch_set_tuning", "mgrhd_batch_get_tuning",
            "mgrhd_batch_run", "mgrhd_batch_capture", "mgrhd_batch_launch", "mgrhd_batch_cells",
            "mgrhd_batch_destroy"]


def _batch_lib():
    L = lib()
    if not hasattr(L, "_batch_ready"):
        L.mgrhd_batch_create.restype = C.c_int
        L.mgrhd_batch_create.argtypes = [C.POINTER(Patch), C.c_int32, C.c_int32,
                                         C.POINTER(Options), C.POINTER(C.c_void_p)]
        L.mgrhd_batch_set_tuning.restype = C.c_int
        L.mgrhd_batch_set_tuning.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int64]
        L.mgrhd_batch_get_tuning.restype = C.c_int
        L.mgrhd_batch_get_tuning.argtypes = [C.c_void_p, C.POINTER(C.c_int32),
                                             C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        for f in ("mgrhd_batch_run", "mgrhd_batch_capture", "mgrhd_batch_launch"):
            getattr(L, f).restype = C.c_int
            getattr(L, f).argtypes = [C.c_void_p, C.c_void_p]
        L.mgrhd_batch_attach_mlp.restype = C.c_int
        L.mgrhd_batch_attach_mlp.argtypes = [C.c_void_p, C.c_int32] + [C.c_void_p] * 5
        L.mgrhd_batch_infer.restype = C.c_int
        L.mgrhd_batch_infer.argtypes = [C.c_void_p, C.c_void_p]
        L.mgrhd_batch_cells.restype = C.c_int64
        L.mgrhd_batch_cells.argtypes = [C.c_void_p]
        L.mgrhd_batch_destroy.restype = None
        L.mgrhd_batch_destroy.argtypes = [C.c_void_p]
        L._batch_ready = True
    return L


class Batch:
    """A set of patches solved by one persistent launch (optionally replayed
    from a captured hipGraph).  ``patches``: list of dicts with the device
    tensors of each patch (E_g, F_g, rho, e_gas, v, edges, chi_lo, and
    optionally alpha_chi, chi_hi, kappa_scale, S_g, guess, iters, outer,
    status, trace, and out=(E_g_out, F_g_out, e_gas_out, v_out) to update the
    patch out of place) and its dt, c_hat."""

    def __init__(self, patches, *, mean_mode=MEAN_PPL_FIXED, c=1.0, a_rad=1.0, h_over_k=1.0,
                 c_v=1.5, eps_newton=1e-11, eps_outer=1e-13, max_newton=100, max_outer=20,
                 closure=CLOSURE_M1, polish=0, guess_kind=0):
        L = _batch_lib()
        arr = (Patch * len(patches))()
        self._keep = patches      # the tensors must outlive the batch
        for k, p in enumerate(patches):
            ng, n = p["E_g"].shape
            q = arr[k]
            q.E_g = _ptr(p["E_g"], (ng, n), name="E_g")
            q.F_g = _ptr(p["F_g"], (3, ng, n), name="F_g")
            q.rho = _ptr(p["rho"], (n,), name="rho")
            q.e_gas = _ptr(p["e_gas"], (n,), name="e_gas")
            q.v = _ptr(p["v"], (3, n), name="v")
            q.kappa_scale = _ptr(p.get("kappa_scale"), (n,), name="kappa_scale")
            q.S_g = _ptr(p.get("S_g"), (ng, n), name="S_g")
            q.guess = _ptr(p.get("guess"), (ng + 1, n) if guess_kind == 0 else (n,),
                           name="guess")
            q.iters = _ptr(p.get("iters"), (n,), torch.int32, "iters")
            q.outer = _ptr(p.get("outer"), (n,), torch.int32, "outer")
            q.status = _ptr(p.get("status"), (n,), torch.int32, "status")
            q.trace = _ptr(p.get("trace"), (max_outer, n), torch.int32, "trace")
            q.group_edges = _ptr(p["edges"], (ng + 1,), name="edges")
            q.chi_lo = _ptr(p["chi_lo"], (ng,), name="chi_lo")
            q.alpha_chi = _ptr(p.get("alpha_chi"), (ng,), name="alpha_chi")
            q.chi_hi = _ptr(p.get("chi_hi"), (ng,), name="chi_hi")
            q.n_cells, q.n_groups = n, ng
            q.dt, q.c_hat = float(p["dt"]), float(p["c_hat"])
            if p.get("out") is not None:
                Eo, Fo, eo, vo = p["out"]
                q.E_g_out = _ptr(Eo, (ng, n), name="E_g_out")
                q.F_g_out = _ptr(Fo, (3, ng, n), name="F_g_out")
                q.e_gas_out = _ptr(eo, (n,), name="e_gas_out")
                q.v_out = _ptr(vo, (3, n), name="v_out")
        o = default_options()
        o.c, o.a_rad, o.h_over_k, o.c_v = c, a_rad, h_over_k, c_v
        o.eps_newton, o.eps_outer = eps_newton, eps_outer
        o.max_newton, o.max_outer, o.closure, o.polish = max_newton, max_outer, closure, polish
        o.guess_kind = guess_kind
        h = C.c_void_p()
        rc = L.mgrhd_batch_create(arr, len(patches), mean_mode, C.byref(o), C.byref(h))
        if rc != 0:
            raise MgrhdError(rc, "mgrhd_batch_create")
        self._h = h

    def _stream(self, stream):
        return torch.cuda.current_stream().cuda_stream if stream is None else stream

    def set_item_scope(self, per_workgroup: int):
        L = _batch_lib()
        L.mgrhd_batch_set_item_scope.restype = C.c_int
        L.mgrhd_batch_set_item_scope.argtypes = [C.c_void_p, C.c_int32]
        rc = L.mgrhd_batch_set_item_scope(self._h, int(per_workgroup))
        if rc != 0:
            raise MgrhdError(rc, "mgrhd_batch_set_item_scope")

    def get_item_scope(self) -> int:
        L = _batch_lib()
        L.mgrhd_batch_get_item_scope.restype = C.c_int32
        L.mgrhd_batch_get_item_scope.argtypes = [C.c_void_p]
        return int(L.mgrhd_batch_get_item_scope(self._h))

    def tune(self, stream=None):
        """The library's own autotuner (mgrhd_batch_tune): candidate launch
        shapes timed on copies of a sample of every patch; keeps the fastest."""
        L = _batch_lib()
        L.mgrhd_batch_tune.restype = C.c_int
        L.mgrhd_batch_tune.argtypes = [C.c_void_p, C.c_void_p]
        rc = L.mgrhd_batch_tune(self._h, self._stream(stream))
        if rc != 0:
            raise MgrhdError(rc, "mgrhd_batch_tune")
        torch.cuda.synchronize()

    def set_tuning(self, groups_per_lane, blocks_per_cu, chunk_cells):
        rc = _batch_lib().mgrhd_batch_set_tuning(self._h, groups_per_lane, blocks_per_cu,
                                                 chunk_cells)
        if rc:
            raise MgrhdError(rc, "mgrhd_batch_set_tuning")

    def get_tuning(self):
        g, b, ch = C.c_int32(), C.c_int32(), C.c_int64()
        _batch_lib().mgrhd_batch_get_tuning(self._h, C.byref(g), C.byref(b), C.byref(ch))
        return g.value, b.value, ch.value

    def run(self, stream=None):
        rc = _batch_lib().mgrhd_batch_run(self._h, self._stream(stream))
        if rc:
            raise MgrhdError(rc, "mgrhd_batch_run")

    def capture(self, stream=None):
        rc = _batch_lib().mgrhd_batch_capture(self._h, self._stream(stream))
        if rc:
            raise MgrhdError(rc, "mgrhd_batch_capture")

    def launch(self, stream=None):
        rc = _batch_lib().mgrhd_batch_launch(self._h, self._stream(stream))
        if rc:
            raise MgrhdError(rc, "mgrhd_batch_launch")

    def attach_mlp(self, n_groups, ws):
        """Attach a warm-start network (warmstart.WarmStart) to the patches of
        n_groups groups: every run/capture/launch then starts with one fused
        inference launch per attached group count, writing each patch's
        guess buffer, before the solve (mgrhd_batch_attach_mlp)."""
        L = _batch_lib()
        f = lambda t: t.data_ptr()
        rc = L.mgrhd_batch_attach_mlp(self._h, int(n_groups), ws.net._h, f(ws.x_mean),
                                      f(ws.x_istd), f(ws.y_mean), f(ws.y_std))
        if rc:
            raise MgrhdError(rc, "mgrhd_batch_attach_mlp")
        self._keep_nets = getattr(self, "_keep_nets", []) + [ws]   # outlive the batch's use

    def infer(self, stream=None):
        """Only the attached networks' inference (mgrhd_batch_infer)."""
        rc = _batch_lib().mgrhd_batch_infer(self._h, self._stream(stream))
        if rc:
            raise MgrhdError(rc, "mgrhd_batch_infer")

    @property
    def n_cells(self):
        return _batch_lib().mgrhd_batch_cells(self._h)

    def close(self):
        if getattr(self, "_h", None):
            _batch_lib().mgrhd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
