"""Helpers for the GPU parity tests: move a workload to the device, run the
HIP path through the C ABI, run the oracle on the same inputs, and compare
field by field."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_2407_18304_amd import mgrhd

FIELDS = ("E_g", "F_g", "e_gas", "v")


def device_tables(w, dev="cuda"):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    return dict(edges=t(w.edges), chi_lo=t(w.chi_lo), alpha=t(w.alpha_chi), kappa=t(w.kappa))


def run_gpu(w, mode, *, polish=1, closure=0, max_outer=10, max_newton=100, eps_newton=1e-11,
            guess=None, S_g=None, use_chi_hi=False, dev="cuda"):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    st = {k: t(w.state[k]) for k in ("E_g", "F_g", "rho", "e_gas", "v")}
    tab = device_tables(w, dev)
    n = w.n
    iters = torch.zeros(n, dtype=torch.int32, device=dev)
    outer = torch.zeros(n, dtype=torch.int32, device=dev)
    status = torch.full((n,), -1, dtype=torch.int32, device=dev)
    chi_hi = t(w.chi_lo * (w.edges[1:] / w.edges[:-1]) ** w.alpha_chi) if use_chi_hi else None
    mgrhd.source_update(st["E_g"], st["F_g"], st["rho"], st["e_gas"], st["v"], tab["edges"],
                        tab["chi_lo"], mean_mode=mode,
                        alpha_chi=None if use_chi_hi else tab["alpha"], chi_hi=chi_hi,
                        kappa_scale=tab["kappa"], dt=w.dt, c_hat=w.c_hat, c=w.c, a_rad=w.a_rad,
                        h_over_k=w.h_over_k, c_v=w.c_v, polish=polish, closure=closure,
                        max_outer=max_outer, max_newton=max_newton, eps_newton=eps_newton,
                        guess=None if guess is None else t(guess),
                        S_g=None if S_g is None else t(S_g), iters=iters, outer=outer,
                        status=status)
    torch.cuda.synchronize()
    out = {k: st[k].cpu().numpy() for k in st}
    return out, iters.cpu().numpy(), outer.cpu().numpy(), status.cpu().numpy()


def run_oracle(w, mode, *, polish=1, closure=0, max_outer=10, max_newton=100, eps_newton=1e-11,
               guess=None, S_g=None):
    return oracle.source_update(w.state, w.edges, w.chi_lo, alpha_chi=w.alpha_chi,
                                kappa_scale=w.kappa, mean_mode=mode, polish=polish,
                                closure=closure, max_outer=max_outer, max_newton=max_newton,
                                eps_newton=eps_newton, guess=guess, S_g=S_g, **w.consts())


def field_errors(w, gpu, ora, mask=None):
    """Per field: max relative error with the floors of the parity metric.
    Energies (E_g, E_gas): |a - b| / max(|b|, 1e-16 E_tot), per cell and group.
    Vectors (F_g per group, v per cell) are compared as vectors:
    max_d |a_d - b_d| / max(|b|_2, floor), with floor 1e-16 of the cell's
    momentum scale |rho v| + sum_g |F_g|/(c c_hat) (in the field's units)."""
    st = w.state
    cc = w.c / w.c_hat
    etot = st["e_gas"] + (1.0 / cc) * st["E_g"].sum(0)
    pscale = np.abs(st["rho"] * st["v"]).sum(0) + np.abs(st["F_g"]).sum((0, 1)) / (w.c * w.c_hat)
    out = {}
    for k in FIELDS:
        a, b = gpu[k], ora[k]
        if k in ("E_g", "e_gas"):
            err = (np.abs(a - b) / np.maximum(np.abs(b), 1e-16 * etot)).reshape(-1, w.n)
        elif k == "F_g":
            nrm = np.sqrt((b * b).sum(0))                        # [N_g, n]
            fl = 1e-16 * pscale * w.c * w.c_hat
            err = np.abs(a - b).max(0) / np.maximum(nrm, fl)
        else:
            nrm = np.sqrt((b * b).sum(0))
            err = (np.abs(a - b).max(0) / np.maximum(nrm, 1e-16 * pscale / st["rho"]))[None]
        if mask is not None:
            err = err[:, mask]
        out[k] = float(err.max()) if err.size else 0.0
    return out
