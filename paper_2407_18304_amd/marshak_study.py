"""Convergence of the three group-mean opacity methods on the Marshak wave with
chi_0 ~ nu^-2 (He, Wibking & Krumholz 2024, Sec. 4.1.3): PC, PPL with fixed
slopes and PPL with fitted slopes at 4, 8 and 16 log-spaced groups over
[6e10, 6e14] Hz, each against a 128-group PC reference computed the same way,
all on the GPU (paper_2407_18304_amd.column1d).  Reports, at t = 1.36e-7 s,
the error of the gas temperature, the total radiation temperature and the
radiation temperatures of the four frequency bands [6e10, 6e11, 6e12, 6e13,
6e14] Hz (eq. Tgdef on the energy summed over each band):
    L1  = sum_i |T_i - T_ref,i| / sum_i |T_ref,i - T_0|   (of the temperature rise)
    max = max_i |T_i - T_ref,i|  [K]

The paper does not say which opacity a PC group takes for a continuous
opacity; both the value at the lower edge (the library's reading for a
powerlaw table) and the value at the group's log-centre are run, and the
128-group reference takes the centre value (its groups span 7.5% in
frequency).

    python -m paper_2407_18304_amd.marshak_study [--out results.json]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

BANDS = np.array([6e10, 6e11, 6e12, 6e13, 6e14])
MODES = {0: "PC", 1: "PPL-fixed", 2: "PPL-free"}


def run_one(ng, mode, n_cells=None, graph_steps=500, log=None, pc_at="lower"):
    """pc_at: which opacity a PC group takes for this continuous opacity (the
    paper does not say): its value at the lower edge, or at the log-centre."""
    from . import column1d
    from . import workloads as W
    prob = W.marshak(ng, n_cells=n_cells)
    if mode == 0 and pc_at == "centre":
        prob.chi_lo = prob.chi_mid.copy()
    col = column1d.Column1D(prob, mode)
    steps = column1d.steps_to(prob.t_end, prob.dt)
    t0 = time.perf_counter()
    col.run(steps, graph_steps=graph_steps)
    import torch
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    Tg, Tr, _ = col.temperatures()
    st = col.state()
    bands = column1d.band_temperatures(st["E_g"], prob.edges, BANDS, prob.a_rad)
    status = col.status_any.cpu().numpy()
    if log:
        log(f"  N_g={ng:3d} {MODES[mode] + ('' if mode else '/' + pc_at):15s}: {steps} steps in {wall:.1f} s "
            f"({steps / wall:.0f} steps/s), status bits {int(np.bitwise_or.reduce(status))}")
    return {"T_gas": Tg, "T_rad": Tr, "bands": bands, "steps": steps, "wall_s": wall,
            "status_or": int(np.bitwise_or.reduce(status)), "n_cells": prob.n}


def errors(r, ref, T0=300.0):
    out = {}
    pairs = [("T_gas", r["T_gas"], ref["T_gas"]), ("T_rad", r["T_rad"], ref["T_rad"])]
    pairs += [(f"band{k}", r["bands"][k], ref["bands"][k]) for k in range(len(BANDS) - 1)]
    for name, a, b in pairs:
        rise = np.abs(b - T0).sum()
        out[name] = {"L1": float(np.abs(a - b).sum() / rise) if rise > 0 else None,
                     "max_K": float(np.abs(a - b).max())}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="")
    ap.add_argument("--cells", type=int, default=0)
    ap.add_argument("--groups", default="4,8,16")
    ap.add_argument("--ref-groups", type=int, default=128)
    ap.add_argument("--ref-pc", default="centre", choices=("lower", "centre"))
    args = ap.parse_args(argv)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    cells = args.cells or None
    log("reference")
    ref = run_one(args.ref_groups, 0, cells, log=log, pc_at=args.ref_pc)
    res = {"reference": {"n_groups": args.ref_groups, "mode": f"PC ({args.ref_pc})",
                         "steps": ref["steps"],
                         "wall_s": ref["wall_s"], "status_or": ref["status_or"],
                         "T_gas": ref["T_gas"].tolist(), "T_rad": ref["T_rad"].tolist(),
                         "bands": ref["bands"].tolist()},
           "runs": []}
    for ng in (int(x) for x in args.groups.split(",")):
        for mode, pc_at in ((0, "lower"), (0, "centre"), (1, None), (2, None)):
            r = run_one(ng, mode, cells, log=log, pc_at=pc_at)
            e = errors(r, ref)
            name = MODES[mode] + (f" ({pc_at})" if pc_at else "")
            res["runs"].append({"n_groups": ng, "mode": name, "steps": r["steps"],
                                "wall_s": r["wall_s"], "status_or": r["status_or"],
                                "errors": e})
            log(f"    T_gas L1 {e['T_gas']['L1']:.4f}  T_rad L1 {e['T_rad']['L1']:.4f}  bands L1 "
                + " ".join(f"{e[f'band{k}']['L1']:.4f}" if e[f'band{k}']['L1'] is not None
                           else "-" for k in range(4)))
    text = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(json.dumps({"runs": res["runs"]}))


if __name__ == "__main__":
    main()
