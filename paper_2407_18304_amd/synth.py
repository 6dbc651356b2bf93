"""Device-side generation of the seeded synthetic workloads of ``workloads``
(``libmgrhd_synth.so``): full-size inputs are drawn in HBM directly, so a
256^3 x 64-group state (35 GB) never passes through host memory.  Cell i of a
device workload equals cell i of ``workloads.make`` up to last-bit differences
of the two math libraries."""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np
import torch

from . import workloads as W

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmgrhd_synth.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        L.mgrhd_synth_state.restype = C.c_int
        L.mgrhd_synth_state.argtypes = (
            [C.c_void_p] * 9 + [C.c_int64, C.c_int64, C.c_uint64, C.c_int32, C.c_int32,
                                C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_double,
                                C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                C.c_double, C.c_double, C.c_double, C.c_void_p])
        _lib = L
    return _lib


@dataclasses.dataclass
class DeviceWorkload:
    """A workload resident in HBM (tensors on the device)."""
    name: str
    n: int
    edges: np.ndarray
    chi_lo: np.ndarray
    alpha_chi: np.ndarray
    dt: float
    c_hat: float
    c: float
    a_rad: float
    state: dict          # device tensors E_g, F_g, rho, e_gas, v
    kappa: torch.Tensor
    T: torch.Tensor
    tables: dict         # device tensors edges, chi_lo, alpha
    c_v: float = 1.5
    h_over_k: float = 1.0
    t_exp: float = 0.0   # temperature dependence of the opacity (see workloads)
    t_ref: float = 1.0
    stim: int = 0

    @property
    def ng(self):
        return len(self.chi_lo)

    def consts(self):
        return dict(dt=self.dt, c_hat=self.c_hat, c=self.c, a_rad=self.a_rad, c_v=self.c_v,
                    h_over_k=self.h_over_k)

    def topacity(self):
        return dict(t_exp=self.t_exp, t_ref=self.t_ref, stim=self.stim)

    def fill(self, cell0: int = 0, stream=None, seed=None):
        """(Re)generate the state in place: cells cell0 .. cell0+n-1, drawn with
        the workload's seed (or ``seed``; the opacity table stays the
        workload's)."""
        sp = W.SPECS[self.name]
        seed = sp["seed"] if seed is None else seed
        gl = torch.from_numpy(np.concatenate([W._GL_X, W._GL_W])).to(self.kappa.device)
        s = self.state
        if stream is None:
            stream = torch.cuda.current_stream(self.kappa.device).cuda_stream
        k_scale = 1.0 / (self.dt * self.c_hat)
        k_p = sp["k_p"]
        rc = lib().mgrhd_synth_state(
            s["E_g"].data_ptr(), s["F_g"].data_ptr(), s["rho"].data_ptr(), s["e_gas"].data_ptr(),
            s["v"].data_ptr(), self.kappa.data_ptr(), self.T.data_ptr(),
            self.tables["edges"].data_ptr(), gl.data_ptr(), self.n, cell0,
            np.uint64(seed).item(), self.ng, len(W._GL_X), sp["t_kind"], sp["t_p"][0],
            sp["t_p"][1], sp["k_kind"], k_p[0], k_p[1], k_scale, W.TRAD_RANGE[0],
            W.TRAD_RANGE[1], sp["vmax"], self.c, self.a_rad, self.c_v, stream)
        if rc != 0:
            raise RuntimeError(f"mgrhd_synth_state failed ({rc})")
        torch.cuda.synchronize()
        del gl


def device_workload(name: str, n: int | None = None, cell0: int = 0, dev="cuda",
                    seed=None) -> DeviceWorkload:
    sp = W.SPECS[name]
    n = n or sp["n"]
    u = W.UNITS[name]
    edges, chi_lo, alpha = W.spec_tables(name)
    ng = len(chi_lo)
    f64 = dict(dtype=torch.float64, device=dev)
    state = {"E_g": torch.empty((ng, n), **f64), "F_g": torch.empty((3, ng, n), **f64),
             "rho": torch.empty(n, **f64), "e_gas": torch.empty(n, **f64),
             "v": torch.empty((3, n), **f64)}
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    dw = DeviceWorkload(name, n, edges, chi_lo, alpha, 1.0 / u["c"], u["c"], u["c"], u["a_rad"],
                        state, torch.empty(n, **f64), torch.empty(n, **f64),
                        {"edges": t(edges), "chi_lo": t(chi_lo), "alpha": t(alpha)},
                        **W.spec_topacity(name))
    dw.fill(cell0, seed=seed)
    return dw


def to_host(dw: DeviceWorkload, idx) -> W.Workload:
    """Copy cells ``idx`` of a device workload back as a host Workload (inputs only)."""
    idx_t = torch.as_tensor(np.asarray(idx), device=dw.kappa.device, dtype=torch.long)
    st = {"E_g": dw.state["E_g"][:, idx_t], "F_g": dw.state["F_g"][:, :, idx_t],
          "rho": dw.state["rho"][idx_t], "e_gas": dw.state["e_gas"][idx_t],
          "v": dw.state["v"][:, idx_t]}
    st = {k: np.ascontiguousarray(v.cpu().numpy()) for k, v in st.items()}
    return W.Workload(dw.name, len(idx), dw.edges, dw.chi_lo, dw.alpha_chi,
                      dw.kappa[idx_t].cpu().numpy(), st, dw.T[idx_t].cpu().numpy(), dt=dw.dt,
                      c_hat=dw.c_hat, c=dw.c, a_rad=dw.a_rad, **dw.topacity())


@dataclasses.dataclass
class DevicePatch:
    layout: "W.PatchLayout"
    state: dict          # device tensors E_g, F_g, rho, e_gas, v
    kappa: torch.Tensor
    T: torch.Tensor
    tables: dict         # device tensors edges, chi_lo, alpha
    dt: float
    c_hat: float
    seed: int = None     # state seed (None: the patch workload's)

    def consts(self):
        u = W.UNITS["patches"]
        return dict(c=u["c"], a_rad=u["a_rad"], h_over_k=1.0, c_v=1.5, dt=self.dt,
                    c_hat=self.c_hat)


def device_patches(layouts, dev="cuda", stream=None, seed=None):
    """Allocate and fill every patch of ``layouts`` in HBM (state as config2,
    units of the patch family); cell numbers are the layouts' global ones.
    seed: the state seed (default: the patch workload's)."""
    u = W.UNITS["patches"]
    dt = 1.0 / u["c"]
    f64 = dict(dtype=torch.float64, device=dev)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    out = []
    for L in layouts:
        n, ng = L.n, L.ng
        st = {"E_g": torch.empty((ng, n), **f64), "F_g": torch.empty((3, ng, n), **f64),
              "rho": torch.empty(n, **f64), "e_gas": torch.empty(n, **f64),
              "v": torch.empty((3, n), **f64)}
        kap, T = torch.empty(n, **f64), torch.empty(n, **f64)
        tabs = {"edges": t(L.edges), "chi_lo": t(L.chi_lo), "alpha": t(L.alpha_chi)}
        out.append(DevicePatch(L, st, kap, T, tabs, dt, u["c"], seed))
    fill_patches(out, stream)
    return out


def fill_patches(dps, stream=None):
    """(Re)generate the state of every device patch in place."""
    if not dps:
        return
    sp = W.SPECS["config2"]
    u = W.UNITS["patches"]
    dev = dps[0].kappa.device
    gl = torch.from_numpy(np.concatenate([W._GL_X, W._GL_W])).to(dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    for dp in dps:
        L, st = dp.layout, dp.state
        rc = lib().mgrhd_synth_state(
            st["E_g"].data_ptr(), st["F_g"].data_ptr(), st["rho"].data_ptr(),
            st["e_gas"].data_ptr(), st["v"].data_ptr(), dp.kappa.data_ptr(), dp.T.data_ptr(),
            dp.tables["edges"].data_ptr(), gl.data_ptr(), L.n, L.cell0,
            np.uint64(W.PATCH_SPEC["seed"] if dp.seed is None else dp.seed).item(), L.ng, len(W._GL_X), sp["t_kind"],
            sp["t_p"][0], sp["t_p"][1], sp["k_kind"], sp["k_p"][0], sp["k_p"][1],
            1.0 / (dp.dt * u["c"]), W.TRAD_RANGE[0], W.TRAD_RANGE[1], sp["vmax"], u["c"],
            u["a_rad"], 1.5, stream)
        if rc != 0:
            raise RuntimeError(f"mgrhd_synth_state failed ({rc})")
    torch.cuda.synchronize()
    del gl


def patch_to_host(dp: DevicePatch, idx=None) -> W.Workload:
    """Copy (cells idx of) a device patch back as a host Workload."""
    n = dp.layout.n
    idx = np.arange(n) if idx is None else np.asarray(idx)
    it = torch.as_tensor(idx, device=dp.kappa.device, dtype=torch.long)
    st = {"E_g": dp.state["E_g"][:, it], "F_g": dp.state["F_g"][:, :, it],
          "rho": dp.state["rho"][it], "e_gas": dp.state["e_gas"][it], "v": dp.state["v"][:, it]}
    st = {k: np.ascontiguousarray(v.cpu().numpy()) for k, v in st.items()}
    u = W.UNITS["patches"]
    return W.Workload(f"patch{dp.layout.index}", len(idx), dp.layout.edges, dp.layout.chi_lo,
                      dp.layout.alpha_chi, dp.kappa[it].cpu().numpy(), st, dp.T[it].cpu().numpy(),
                      dt=dp.dt, c_hat=dp.c_hat, **u)
