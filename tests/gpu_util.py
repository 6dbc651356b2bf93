"""Helpers for the GPU parity tests: move a workload to the device, run the
HIP path through the C ABI, run the oracle on the same inputs, and compare
field by field."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_2407_18304_amd import mgrhd

FIELDS = ("E_g", "F_g", "e_gas", "v")

TOL = 1e-10   # relative parity bound on every field
# Cells where the two sides take a different number of Newton steps or outer
# passes (a stop test sitting on its threshold, < 1% of cells) differ by the
# last increment of a converged iteration: bounded by this instead.
TOL_COUNT_FLIP = 1e-8


def device_tables(w, dev="cuda"):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    return dict(edges=t(w.edges), chi_lo=t(w.chi_lo), alpha=t(w.alpha_chi), kappa=t(w.kappa))


def run_gpu(w, mode, *, polish=1, closure=0, max_outer=10, max_newton=100, eps_newton=1e-11,
            guess=None, guess_kind=0, S_g=None, use_chi_hi=False, dev="cuda"):
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
                        guess=None if guess is None else t(guess), guess_kind=guess_kind,
                        S_g=None if S_g is None else t(S_g), iters=iters, outer=outer,
                        status=status, **w.topacity())
    torch.cuda.synchronize()
    out = {k: st[k].cpu().numpy() for k in st}
    return out, iters.cpu().numpy(), outer.cpu().numpy(), status.cpu().numpy()


def run_oracle(w, mode, *, polish=1, closure=0, max_outer=10, max_newton=100, eps_newton=1e-11,
               guess=None, guess_kind=0, S_g=None):
    return oracle.source_update(w.state, w.edges, w.chi_lo, alpha_chi=w.alpha_chi,
                                kappa_scale=w.kappa, mean_mode=mode, polish=polish,
                                closure=closure, max_outer=max_outer, max_newton=max_newton,
                                eps_newton=eps_newton, guess=guess, guess_kind=guess_kind,
                                S_g=S_g, **w.consts(), **w.topacity())


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


def compare(w, gpu, ref, label="", tol=TOL, tol_flip=TOL_COUNT_FLIP):
    """Parity of a GPU result with a reference result (the oracle, or another
    GPU entry point) on the same inputs w.  gpu, ref = (state, iters, outer,
    status).  Cells whose outer iteration does not contract (status bit 2) are
    checked for validity only: their last iterate, and whether they still
    stop inside the pass limit, depend on rounding.  All other cells must
    agree in status; converged cells within tol (same counts) or tol_flip
    (Newton or outer count differs by a threshold flip)."""
    g, gi, go, gs = gpu
    o, oi, oo, os_ = ref
    chaotic = ((gs | os_) & 2) != 0
    both = (gs == os_) | (chaotic & ((gs & ~2) == 0) & ((os_ & ~2) == 0))
    assert both.mean() > 0.99, f"{label}: status agreement {both.mean():.4f}"
    conv = (os_ == 0) & (gs == 0)
    same = conv & (gi == oi) & (go == oo)
    flip = conv & ~same
    err = field_errors(w, g, o, same)
    err_flip = field_errors(w, g, o, flip)
    print(f"{label}: n={w.n} N_g={w.ng} converged {conv.mean():.4f} non-contracting "
          f"{chaotic.mean():.4f} (gpu {((gs & 2) != 0).mean():.4f} ref {((os_ & 2) != 0).mean():.4f})"
          f" same counts {same.mean():.4f} errors {err} count-flip cells {flip.sum()} "
          f"(outer {(conv & (go != oo)).sum()}) {err_flip}")
    for k, e in err.items():
        assert e < tol, (label, k, e)
    for k, e in err_flip.items():
        assert e < tol_flip, (label, k, e)
    # The outer stop test compares the change of the velocity terms with
    # 1e-13 E_tot, a few hundred rounding errors: which pass meets it is
    # decided by rounding in a few percent of the cells, and in up to a tenth
    # of them with one group spanning the whole spectrum (the results of those
    # cells still agree within tol_flip, checked above).
    assert flip.sum() <= max(0.25 * conv.sum(), 1), (label, int(flip.sum()))
    assert np.abs(gi[conv] - oi[conv]).max(initial=0) <= 2
    # non-contracting cells: finite
    for k in FIELDS:
        assert np.isfinite(g[k].reshape(-1, w.n)[:, chaotic]).all(), (label, k)
    # invalid / untouched cells are left exactly as they were
    inv = (os_ & 8) != 0
    for k in FIELDS:
        a, b = g[k].reshape(-1, w.n)[:, inv], w.state[k].reshape(-1, w.n)[:, inv]
        assert np.array_equal(a, b), (label, k)
    return g, gs


def full_size_sampled(name, mode, n_sample, seed):
    """Draw the whole workload ``name`` on the device, solve it in place with
    the benchmark's launch configuration (the autotuner's cached variant for
    this GPU), and compare ``n_sample`` random cells with the oracle run on
    the same (device-drawn) inputs."""
    from paper_2407_18304_amd import autotune, synth
    dw = synth.device_workload(name)
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(dw.n, n_sample, replace=False))
    host = synth.to_host(dw, idx)                        # pristine inputs of the sample
    cache = autotune.apply_cache(mode=mode)
    try:
        n = dw.n
        iters = torch.zeros(n, dtype=torch.int32, device="cuda")
        outer = torch.zeros(n, dtype=torch.int32, device="cuda")
        status = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        s = dw.state
        mgrhd.source_update(s["E_g"], s["F_g"], s["rho"], s["e_gas"], s["v"],
                            dw.tables["edges"], dw.tables["chi_lo"], mean_mode=mode,
                            alpha_chi=dw.tables["alpha"], kappa_scale=dw.kappa, polish=1,
                            iters=iters, outer=outer, status=status, **dw.consts(),
                            **dw.topacity())
        torch.cuda.synchronize()
        assert bool((status >= 0).all())
        it = torch.as_tensor(idx, device="cuda")
        gpu = ({"E_g": s["E_g"][:, it].cpu().numpy(), "F_g": s["F_g"][:, :, it].cpu().numpy(),
                "e_gas": s["e_gas"][it].cpu().numpy(), "v": s["v"][:, it].cpu().numpy()},
               iters[it].cpu().numpy(), outer[it].cpu().numpy(), status[it].cpu().numpy())
    finally:
        for key in cache.get("single", {}):
            mgrhd.set_variant(int(key.split(":")[0]), 0, 0)
        del dw
        torch.cuda.empty_cache()
    compare(host, gpu, run_oracle(host, mode),
            label=f"{name} full size, {n_sample} sampled cells, mode {mode}")
    return idx, host
