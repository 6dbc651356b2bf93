#!/usr/bin/env python3
"""Benchmark of the multigroup source update on one MI355X.

A step is one full source update (inner Newton, energy, flux and momentum
updates, outer passes) of every cell of the workload.  The inputs are drawn
in HBM by the device generator.  The single-table workloads update out of
place (mgrhd_options.E_g_out ...): every step reads the same inputs, left
unchanged, and writes the updated state to separate arrays, as a time step
from U^(n) to U^(n+1) does, so every step solves the same input
distribution with nothing but the update in the timed region.  The batched
patches update in place; their inputs are drawn again in HBM by the device
generator before every step, outside the timed region (HIP events bracket
each graph launch).

Prints one JSON line (see the repository's benchmark contract)."""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "config1": "128^3 cells, 16 groups, FP64 (random powerlaw opacity table)",
    "config4": "2000 AMR-like patches (sides 8-64, 8-64 groups, own tables), one persistent "
               "launch replayed from a hipGraph, FP64",
    "config2": "256^3 cells, 64 groups, FP64 (T over 3 decades, tau 1e-3..1e6)",
    "config0": "16^3 cells, 4 groups, FP64",
    "config5": "128^3 cells, 16 groups, FP64, temperature-dependent opacity of the "
               "pulse test (nu^-3, T^-1/2, stimulated emission) evaluated at every iterate",
    "column": "1D column of 2^21 cells, 16 groups, FP64: two-stage IMEX steps of the "
              "Marshak problem with nu^-2 opacity (explicit M1 transport + implicit source update "
              "per stage), steps replayed from a HIP graph",
}
PEAK_HBM = 8.0e12            # bytes/s
PEAK_FP64 = 78.6e12          # FP64 vector FLOP/s


SOLVER_SOURCES = ("source_update.hip", "source_update_full.hip", "solver_kernel.hpp",
                  "solver_device.hpp", "planck_device.hpp", "planck_poly.inc")


def kernel_source_sha() -> str:
    """Hash of the sources of the single-table solver kernel: a measured HBM
    traffic is reported only for the sources it was measured on."""
    import hashlib
    h = hashlib.sha256()
    for name in SOLVER_SOURCES:
        h.update(name.encode())
        h.update(open(os.path.join(ROOT, "paper_2407_18304_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` on `workload` from the rocprofv3 PMC
    summary in profiles/traffic.json (FETCH_SIZE and WRITE_SIZE, each scaled
    by the same counter on a plain copy of known size), or None when there is
    none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(workload)
    if not rec or rec.get("source_sha") != kernel_source_sha() or rec.get("kernel") != kernel:
        return None
    return rec["traffic_bytes"]


def copy_bandwidth(gib=4, reps=3):
    """Achievable HBM bandwidth of a plain device-to-device copy of `gib` GiB
    (bytes read + written per second, best of `reps`), the practical ceiling
    beside the 8 TB/s peak."""
    import torch
    n = (gib << 30) // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    best = 0.0
    for _ in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, 2.0 * 8 * n / (e0.elapsed_time(e1) * 1e-3))
    del a, b
    torch.cuda.empty_cache()
    return {"GB/s": best / 1e9, "bytes": 2 * 8 * n, "kind": "device-to-device copy"}


def bytes_per_cell(ng: int) -> int:
    """Algorithmic HBM bytes per cell-update: E_g, F_g, E_gas, v read and
    written (8(4 N_g + 4) each way), rho and the opacity scale read (16), and
    the int32 Newton count, outer count and status written (12)."""
    return 2 * 8 * (4 * ng + 4) + 16 + 12


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="config2", choices=list(WORKLOADS))
    ap.add_argument("--no-ng16", action="store_true",
                    help="default workload only: skip the 128^3 x 16-group figures reported "
                         "beside it")
    ap.add_argument("--mode", type=int, default=1, help="0 PC, 1 PPL-fixed, 2 PPL-free")
    ap.add_argument("--closure", type=int, default=0, help="0 M1, 1 Eddington")
    ap.add_argument("--polish", type=int, default=1, help="extra Newton steps after convergence")
    ap.add_argument("--cells", type=int, default=0, help="override the cell count")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample (0 = skip)")
    ap.add_argument("--patches", type=int, default=0, help="config4: override the patch count")
    ap.add_argument("--warm", action="store_true",
                    help="learned warm start: train the network on 2^20 solver pairs of the "
                         "same distribution (training seed, untimed; config4: one network per "
                         "group count), then time network inference + solve per step, and "
                         "plain steps for comparison")
    ap.add_argument("--tune", action="store_true",
                    help="config4: run the batch autotuner before timing")
    ap.add_argument("--train-cells", type=int, default=1 << 20)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--tuning", default="",
                    help="config4: batch tuning G,B,C[,S] (groups per lane, workgroups per CU, "
                         "cells per item, item scope: 0 wave, 1|2 workgroup)")
    ap.add_argument("--variant", default="",
                    help="kernel variant override LPCxG[xW] (lanes per cell, groups per lane, "
                         "waves per SIMD), e.g. 16x4 or 16x4x3")
    ap.add_argument("--replicate-cell", type=int, default=-1,
                    help="analysis: every cell gets the state (and opacity scale) of this "
                         "cell, so the cells of a wave never diverge (single-table workloads)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the source update has "
                                   "no cross-GPU step (each GPU would own its own cells)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    if args.workload == "config4":
        return run_batch(args)
    if args.workload == "column":
        return run_column(args)
    result = run_single(args.workload, args)
    if args.workload == "config2" and not (args.cells or args.warm or args.no_ng16):
        torch.cuda.empty_cache()
        result["n_g16"] = run_single("config1", args, extra=True)
    print(json.dumps(result), flush=True)


def run_single(name, args, extra=False):
    """Time the single-table source update on workload `name`; returns the
    result dict (extra: the figures reported beside the main workload)."""
    import numpy as np
    import torch

    from paper_2407_18304_amd import flops as F
    from paper_2407_18304_amd import mgrhd, synth
    from paper_2407_18304_amd import workloads as W

    dev = torch.device("cuda:0")
    n = (0 if extra else args.cells) or W.SPECS[name]["n"]
    dw = synth.device_workload(name, n=n)
    ng = dw.ng
    if args.replicate_cell >= 0 and not extra:
        c = args.replicate_cell
        for k, t in dw.state.items():
            t.copy_(t[..., c:c + 1].expand_as(t))
        dw.kappa.fill_(float(dw.kappa[c]))
    if args.variant:
        mgrhd.set_variant(ng, *(int(x) for x in args.variant.split("x")))
    else:
        from paper_2407_18304_amd import autotune
        autotune.apply_cache(mode=args.mode)   # the autotuner's choices for this GPU
    st = dw.state     # the inputs: read by every step, never modified
    res = {k: torch.empty_like(st[k]) for k in ("E_g", "F_g", "e_gas", "v")}   # the outputs
    iters = torch.zeros(n, dtype=torch.int32, device=dev)
    outer = torch.zeros(n, dtype=torch.int32, device=dev)
    status = torch.zeros(n, dtype=torch.int32, device=dev)
    tab = dw.tables
    stream = torch.cuda.current_stream(dev)

    ws, winfo = None, None
    if args.warm and not extra:
        ws, winfo = train_warm(name, args)

    exact_guess = None     # E_gas of the plain solution: the best temperature guess

    def solve(warm=False):
        if warm == "exact":
            guess = exact_guess
        else:
            guess = ws.guess(st, tab, dw.kappa, dw.consts()) if warm else None
        mgrhd.source_update(st["E_g"], st["F_g"], st["rho"], st["e_gas"], st["v"], tab["edges"],
                            tab["chi_lo"], alpha_chi=tab["alpha"], kappa_scale=dw.kappa,
                            mean_mode=args.mode, polish=args.polish, closure=args.closure,
                            guess=guess, guess_kind=1,
                            iters=iters, outer=outer, status=status,
                            stream=stream.cuda_stream, **dw.consts(), **dw.topacity(),
                            out=(res["E_g"], res["F_g"], res["e_gas"], res["v"]))

    def timed(warm):
        for _ in range(args.warmup):
            solve(warm)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        t0 = time.perf_counter()
        for k in range(args.steps):
            ev[k][0].record(stream)
            solve(warm)
            ev[k][1].record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return t0, t1, [a.elapsed_time(b) for a, b in ev]

    warm = args.warm and not extra
    if warm:
        _, _, plain_ms = timed(False)
        plain_it = iters.cpu().numpy().copy()
        plain_st = status.cpu().numpy().copy()
        plain_state = {k: res[k].clone() for k in ("E_g", "F_g", "e_gas", "v")}
        # the ceiling of any temperature guess: the solve started from the
        # plain solution's own E_gas (guess kind 1), on the same inputs
        exact_guess = plain_state["e_gas"]
        _, _, exact_ms = timed("exact")
        exact_it = iters.cpu().numpy().copy()
        # the fused inference kernel alone, on pristine inputs, against the
        # matrix-core peak: the products it computes (temperature output only)
        gbuf = torch.empty(n, dtype=torch.float64, device=dev)
        ws.guess(st, tab, dw.kappa, dw.consts(), out=gbuf)
        inf_ms = []
        for _ in range(args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ws.guess(st, tab, dw.kappa, dw.consts(), out=gbuf)
            e1.record(stream)
            stream.synchronize()
            inf_ms.append(e0.elapsed_time(e1))
        del gbuf
        n_in, n_h = 2 + 3 * ng, ws.net.n_hidden
        mlp_flop = 2.0 * (n_in * n_h + 2 * n_h * n_h + n_h * 1) * n
        mlp_bytes = (8 * (4 * ng + 5) + 8) * n     # state read, guess written
        inf_s = float(np.mean(inf_ms)) * 1e-3
        winfo["inference"] = {
            "ms": inf_s * 1e3,
            "roofline": {"bound": "mfma", "achieved": mlp_flop / inf_s / 1e12, "peak": 2500.0,
                         "unit": "TFLOP/s", "frac": mlp_flop / inf_s / 2.5e15,
                         "flop_per_cell": mlp_flop / n, "dtype": "bf16 products, fp32 accumulation"},
            "hbm": {"achieved": mlp_bytes / inf_s / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                    "frac": mlp_bytes / inf_s / PEAK_HBM, "bytes_per_cell": mlp_bytes / n}}
    t0, t1, kern_ms = timed(warm)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n * args.steps / (t1 - t0)

    it = iters.cpu().numpy()
    ou = outer.cpu().numpy()
    stt = status.cpu().numpy()
    kern_s = float(np.mean(kern_ms)) * 1e-3
    bpc = bytes_per_cell(ng)
    achieved_bw = bpc * n / kern_s
    # FP64 work of the last step (every step solves the same inputs)
    u = dw.consts()
    T_fin = (res["e_gas"] - 0.5 * st["rho"] * (res["v"] ** 2).sum(0)) / (st["rho"] * u["c_v"])
    mix = F.edge_mix(W.spec_tables(name)[0], u["h_over_k"], T_fin.clamp(min=1e-300))
    valid = torch.from_numpy(((stt & 8) == 0).astype(np.float64)).to(dev)
    fpc = F.flops_per_cell(ng, args.mode, iters.double(), outer.double(), mix, valid=valid,
                           t_exp=dw.t_exp, stim=dw.stim)
    flop = float(fpc.sum())
    flop1 = float(F.flops_per_cell(ng, args.mode, iters.double(), outer.double(), mix,
                                   u=F.UNIT_DIV_SQRT_1, valid=valid, t_exp=dw.t_exp,
                                   stim=dw.stim).sum())
    achieved_fl = flop / kern_s
    # the binding ceiling is the lower of the two for this workload
    ceil_alu = PEAK_FP64 / (flop / n)
    ceil_hbm = PEAK_HBM / bpc
    lpc_, g_, w_ = mgrhd.get_variant(ng, args.mode)
    td = "true" if (dw.t_exp != 0.0 or dw.stim) else "false"
    full = "true" if lpc_ * g_ == ng else "false"
    kname = f"k_source_update<{g_}, {lpc_}, {args.mode}, {w_}, {td}, {full}>"
    traffic = None if (warm or args.cells or args.mode != 1) else measured_traffic(name, kname)
    # headline pricing: +, -, x = 1, FMA = 2, division and square root = 1,
    # exp/expm1/log by their gfx950 instruction counts; beside it, the same
    # count with divisions and square roots also priced by their instruction
    # sequences
    ceil_alu = PEAK_FP64 / (flop1 / n)
    roof_alu = {"bound": "alu", "achieved": flop1 / kern_s / 1e12, "peak": PEAK_FP64 / 1e12,
                "unit": "TFLOP/s", "frac": flop1 / kern_s / PEAK_FP64, "traffic": traffic,
                "flop_per_cell": flop1 / n, "ceiling_cells_per_s": ceil_alu,
                "pricing": "div and sqrt = 1 FLOP; exp, expm1, log by instruction count",
                "flop_per_cell_div_sqrt_by_instructions": flop / n,
                "frac_div_sqrt_by_instructions": achieved_fl / PEAK_FP64}
    roof_hbm = {"bound": "hbm", "achieved": achieved_bw / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": achieved_bw / PEAK_HBM, "traffic": traffic,
                "bytes_per_cell": bpc, "ceiling_cells_per_s": ceil_hbm}
    roof, other = (roof_alu, roof_hbm) if ceil_alu <= ceil_hbm else (roof_hbm, roof_alu)

    result = {
        "metric": "cell-updates/s of multigroup source solve (N_g=16,64); Newton iters/cell",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded counter-based generator, drawn in HBM)",
        "config": {"workload": WORKLOADS[name] + ", " + ["PC", "PPL-fixed", "PPL-free"][args.mode] +
                   (f", every cell holding cell {args.replicate_cell}'s state"
                    if args.replicate_cell >= 0 and not extra else ""),
                   "cells": n, "n_groups": ng,
                   "mean_mode": ["PC", "PPL-fixed", "PPL-free"][args.mode],
                   "kernel_variant": "x".join(map(str, mgrhd.get_variant(ng, args.mode))),
                   "eps_newton": 1e-11, "polish": args.polish,
                   "closure": ["M1", "Eddington"][args.closure]},
        "newton_iters_per_cell": {"mean": float(it.mean()), "p50": float(np.percentile(it, 50)),
                                  "p99": float(np.percentile(it, 99)), "max": int(it.max())},
        "outer_passes_per_cell": {"mean": float(ou.mean()), "max": int(ou.max())},
        "status_counts": {str(k): int(v) for k, v in enumerate(np.bincount(stt)) if v},
        "kernel_ms": {"mean": float(np.mean(kern_ms)), "min": float(np.min(kern_ms))},
        "roofline": roof,
        "roofline_other": other,
    }
    if not extra:
        result["hbm_copy_ceiling"] = copy_bandwidth()
    if extra:
        return {"workload": result["config"]["workload"], "cells": n, "n_groups": ng,
                "value": value,
                "ms_per_step": ms_per_step, "config": result["config"],
                "newton_iters_per_cell": result["newton_iters_per_cell"],
                "outer_passes_per_cell": result["outer_passes_per_cell"],
                "status_counts": result["status_counts"], "kernel_ms": result["kernel_ms"],
                "roofline": roof, "roofline_other": other}
    if warm:
        ok = (plain_st == 0) & ((stt & ~4) == 0)
        dev_max = 0.0
        for k in ("E_g", "e_gas"):
            d = ((res[k] - plain_state[k]).abs() /
                 plain_state[k].abs().clamp(min=1e-300)).reshape(-1, n)[:, torch.from_numpy(ok).to(dev)]
            dev_max = max(dev_max, float(d.max()) if d.numel() else 0.0)
        winfo.update({
            "ms_per_step_with_network": float(np.mean(kern_ms)),
            "ms_per_step_plain": float(np.mean(plain_ms)),
            "speedup": float(np.mean(plain_ms) / np.mean(kern_ms)),
            "newton_iters_plain": float(plain_it[ok].mean()),
            "newton_iters_warm": float(it[ok].mean()),
            "ceiling": {
                "what": "solve started from the plain solution's own E_gas (the exact "
                        "temperature guess, guess kind 1), no inference",
                "ms_solve": float(np.mean(exact_ms)),
                "newton_iters": float(exact_it[ok].mean()),
                "break_even_inference_ms": float(np.mean(plain_ms) - np.mean(exact_ms))},
            "fallbacks": int(((stt & 4) != 0).sum()),
            "max_rel_diff_vs_plain_E": dev_max,
        })
        result["warm_start"] = winfo
        result["config"]["warm_start"] = "network temperature guess (guess kind 1)"

    if args.cpu_seconds > 0:
        torch.cuda.synchronize()
        result["cpu_baseline"] = cpu_baseline(dw, args.mode, args.cpu_seconds)
    return result


def train_warm(name, args):
    """Train the warm-start network on solver pairs of the workload's
    distribution drawn with the training seed (not timed)."""
    import torch

    from paper_2407_18304_amd import synth, warmstart
    from paper_2407_18304_amd import workloads as W

    t0 = time.perf_counter()
    dw = synth.device_workload(name, n=args.train_cells, seed=W.TRAIN_SEED)
    Xr, Yr, ok = warmstart.make_training_data(dw, dw.consts())
    t1 = time.perf_counter()
    ws = warmstart.train(Xr, Yr, ok, epochs=args.epochs, batch=4096, holdout=1 << 16,
                         log=lambda m: print(m, file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    del dw, Xr, Yr, ok
    torch.cuda.empty_cache()
    return ws, {"train_pairs": args.train_cells, "epochs": args.epochs,
                "heldout_loss_first_last": [ws.history[0], ws.history[-1]],
                "pair_generation_s": t1 - t0, "training_s": t2 - t1}


def run_column(args):
    """Two-stage IMEX steps (transport + source per stage) of a long 1D column
    with the Marshak problem's physics; the transport kernel is also timed on
    its own for its HBM roofline."""
    import numpy as np
    import torch

    from paper_2407_18304_amd import column1d, mgrhd
    from paper_2407_18304_amd import workloads as W
    n = args.cells or (1 << 21)
    ng = 16
    prob = W.marshak(ng, n_cells=n)
    prob.dx = W.MARSHAK["length"] / 500                 # the Marshak cell size, longer column
    prob.dt = W.MARSHAK["cfl"] * prob.dx / prob.c
    col = column1d.Column1D(prob, args.mode)
    col.run(args.warmup * 2 + 1, graph_steps=0)
    torch.cuda.synchronize()
    graph_steps = max(1, args.steps)
    col.run(graph_steps, graph_steps=graph_steps)     # capture (and run) the graph once
    torch.cuda.synchronize()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    s0.record()
    col._graph.replay()
    s1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    steps = graph_steps
    value = n * steps / (t1 - t0)
    # the transport stage alone (stage 2 form: reads U^n and U^(n+1/2))
    U, Ut = col.U, col.Ut
    out = {k: torch.empty_like(v) for k, v in Ut.items()}
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        col._stage(out, Ut, U, 0.5, 0.5, 0.5 * prob.dt)
    e1.record()
    torch.cuda.synchronize()
    t_tr = e0.elapsed_time(e1) * 1e-3 / reps
    bytes_tr = (96 * ng + 104) * n                     # algorithmic bytes of one stage-2 launch
    status = col.status_any.cpu().numpy()
    result = {
        "metric": "cell-updates/s of multigroup source solve (N_g=16,64); Newton iters/cell",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": (t1 - t0) * 1e3 / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (Marshak initial state: uniform 300 K, black-body boundary at 1000 K)",
        "config": {"workload": WORKLOADS["column"], "cells": n, "n_groups": ng,
                   "mean_mode": ["PC", "PPL-fixed", "PPL-free"][args.mode],
                   "kernel_variant": "x".join(map(str, mgrhd.get_variant(ng, args.mode))),
                   "eps_newton": 1e-11, "polish": 1, "closure": "M1"},
        "status_or": int(np.bitwise_or.reduce(status)),
        "transport_stage": {"bound": "hbm", "ms": t_tr * 1e3,
                            "achieved": bytes_tr / t_tr / 1e9, "peak": PEAK_HBM / 1e9,
                            "unit": "GB/s", "frac": bytes_tr / t_tr / PEAK_HBM,
                            "bytes_per_launch": bytes_tr},
    }
    print(json.dumps(result), flush=True)


def run_batch(args):
    """Uneven AMR-like patches in one persistent launch replayed from a
    hipGraph.  The 2000-patch state (~155 GB) leaves no room for a pristine
    copy, so each step's inputs are regenerated in HBM by the device generator
    before the step (untimed); HIP events bracket each graph launch."""
    import numpy as np
    import torch

    from paper_2407_18304_amd import flops as F
    from paper_2407_18304_amd import mgrhd, synth
    from paper_2407_18304_amd import workloads as W

    layouts = W.patch_layouts(n_patches=args.patches or None)
    dps = synth.device_patches(layouts)
    n = sum(L.n for L in layouts)
    u = W.UNITS["patches"]
    pd = []
    for dp in dps:
        m = dp.layout.n
        d = dict(dp.state)
        d.update(edges=dp.tables["edges"], chi_lo=dp.tables["chi_lo"],
                 alpha_chi=dp.tables["alpha"], kappa_scale=dp.kappa, dt=dp.dt, c_hat=dp.c_hat,
                 iters=torch.zeros(m, dtype=torch.int32, device="cuda"),
                 outer=torch.zeros(m, dtype=torch.int32, device="cuda"),
                 status=torch.zeros(m, dtype=torch.int32, device="cuda"))
        pd.append(d)
    b = mgrhd.Batch(pd, mean_mode=args.mode, polish=1, c=u["c"], a_rad=u["a_rad"])
    if args.tuning:
        tv = [int(x) for x in args.tuning.split(",")]
        b.set_tuning(*tv[:3])
        if len(tv) > 3:
            b.set_item_scope(tv[3])
    elif args.tune:
        from paper_2407_18304_amd import autotune
        autotune.tune_batch(b, lambda: synth.fill_patches(dps), reps=1,
                            log=lambda m: print(m, file=sys.stderr, flush=True))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.capture(stream.cuda_stream)
    torch.cuda.synchronize()

    def timed(launch):
        for _ in range(args.warmup):
            synth.fill_patches(dps)
            launch()
            stream.synchronize()
        ms = []
        for _ in range(args.steps):
            synth.fill_patches(dps)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(stream):
                e0.record(stream)
                launch()
                e1.record(stream)
            stream.synchronize()
            ms.append(e0.elapsed_time(e1))
        return ms

    winfo = None
    if args.warm:
        # one network per group count, trained on patches drawn with the
        # training seed (untimed); the timed step is [inference of every
        # patch -> batched solve] replayed from one graph, against the plain
        # batched solve on the same inputs
        from paper_2407_18304_amd import warmstart
        nets, winfo = train_warm_patches(sorted({L.ng for L in layouts}), args)
        plain_ms = timed(lambda: b.launch(stream.cuda_stream))
        k_s = 64
        plain_it = np.concatenate([d["iters"].cpu().numpy() for d in pd])
        plain_st = np.concatenate([d["status"].cpu().numpy() for d in pd])
        sample = [{k: dp.state[k][..., :k_s].clone() for k in ("E_g", "F_g", "e_gas", "v")}
                  for dp in dps]
        guesses = [torch.empty(dp.layout.n, dtype=torch.float64, device="cuda") for dp in dps]
        bw = mgrhd.Batch([dict(d, guess=g) for d, g in zip(pd, guesses)], mean_mode=args.mode,
                         polish=1, c=u["c"], a_rad=u["a_rad"], guess_kind=1)
        bw.set_tuning(*b.get_tuning())
        bw.set_item_scope(b.get_item_scope())
        pws = warmstart.PatchWarmStart(nets)
        pws.attach(bw)                         # one inference launch per group count
        synth.fill_patches(dps)
        with torch.cuda.stream(stream):        # eager once
            bw.run(stream.cuda_stream)
        stream.synchronize()
        with torch.cuda.stream(stream):        # inference + solve in the batch's graph
            bw.capture(stream.cuda_stream)
        # the ceiling of any temperature guess: each patch solved from the
        # plain solution's own E_gas (guess kind 1), no inference
        exact = [d["e_gas"].clone() for d in pd]
        bx = mgrhd.Batch([dict(d, guess=g) for d, g in zip(pd, exact)], mean_mode=args.mode,
                         polish=1, c=u["c"], a_rad=u["a_rad"], guess_kind=1)
        bx.set_tuning(*b.get_tuning())
        bx.set_item_scope(b.get_item_scope())
        with torch.cuda.stream(stream):
            bx.capture(stream.cuda_stream)
        torch.cuda.synchronize()
        exact_ms = timed(lambda: bx.launch(stream.cuda_stream))
        exact_it = np.concatenate([d["iters"].cpu().numpy() for d in pd])
        bx.close()
        del exact
        gi = torch.cuda.CUDAGraph()            # the inference launches alone
        with torch.cuda.graph(gi, stream=stream, capture_error_mode="thread_local"):
            bw.infer(stream.cuda_stream)
        torch.cuda.synchronize()
        infer_ms = timed(gi.replay)
        kern_ms = timed(lambda: bw.launch(stream.cuda_stream))
        dmax = 0.0
        for dp, smp in zip(dps, sample):
            for k in ("E_g", "e_gas"):
                a, r = dp.state[k][..., :k_s], smp[k]
                dmax = max(dmax, float(((a - r).abs() / r.abs().clamp(min=1e-300)).max()))
        warm_it = np.concatenate([d["iters"].cpu().numpy() for d in pd])
        warm_st = np.concatenate([d["status"].cpu().numpy() for d in pd])
        ok = (plain_st == 0) & ((warm_st & ~4) == 0)
        winfo.update({
            "ms_per_step_with_network": float(np.mean(kern_ms)),
            "ms_per_step_plain": float(np.mean(plain_ms)),
            "ms_inference_alone": float(np.mean(infer_ms)),
            "speedup": float(np.mean(plain_ms) / np.mean(kern_ms)),
            "newton_iters_plain": float(plain_it[ok].mean()),
            "newton_iters_warm": float(warm_it[ok].mean()),
            "ceiling": {
                "what": "batched solve started from the plain solution's own E_gas in every "
                        "cell (the exact temperature guess, guess kind 1), no inference",
                "ms_solve": float(np.mean(exact_ms)),
                "newton_iters": float(exact_it[ok].mean()),
                "break_even_inference_ms": float(np.mean(plain_ms) - np.mean(exact_ms))},
            "fallbacks": int(((warm_st & 4) != 0).sum()),
            "max_rel_diff_vs_plain_E_sampled": dmax,
            "sample": f"first {k_s} cells of every patch",
        })
    else:
        kern_ms = timed(lambda: b.launch(stream.cuda_stream))
    kern_s = float(np.mean(kern_ms)) * 1e-3
    # per-cell work of the last step
    flop = flop1 = 0.0
    byts = 0.0
    it_all, ou_all, st_all = [], [], []
    for dp, d in zip(dps, pd):
        L = dp.layout
        st = dp.state
        T_fin = (st["e_gas"] - 0.5 * st["rho"] * (st["v"] ** 2).sum(0)) / (st["rho"] * 1.5)
        mix = F.edge_mix(L.edges, 1.0, T_fin.clamp(min=1e-300))
        valid = ((d["status"] & 8) == 0).double()
        flop += float(F.flops_per_cell(L.ng, args.mode, d["iters"].double(), d["outer"].double(),
                                       mix, valid=valid).sum())
        flop1 += float(F.flops_per_cell(L.ng, args.mode, d["iters"].double(),
                                        d["outer"].double(), mix, u=F.UNIT_DIV_SQRT_1,
                                        valid=valid).sum())
        byts += L.n * bytes_per_cell(L.ng)
        it_all.append(d["iters"].cpu().numpy())
        ou_all.append(d["outer"].cpu().numpy())
        st_all.append(d["status"].cpu().numpy())
    it, ou, stt = (np.concatenate(x) for x in (it_all, ou_all, st_all))
    # the same pricing as the single-table line: division and square root = 1
    # FLOP in the headline, priced by their instruction sequences beside it
    ceil_alu = PEAK_FP64 / (flop1 / n)
    ceil_hbm = PEAK_HBM / (byts / n)
    roof_alu = {"bound": "alu", "achieved": flop1 / kern_s / 1e12, "peak": PEAK_FP64 / 1e12,
                "unit": "TFLOP/s", "frac": flop1 / kern_s / PEAK_FP64, "traffic": None,
                "flop_per_cell": flop1 / n, "ceiling_cells_per_s": ceil_alu,
                "pricing": "div and sqrt = 1 FLOP; exp, expm1, log by instruction count",
                "flop_per_cell_div_sqrt_by_instructions": flop / n,
                "frac_div_sqrt_by_instructions": flop / kern_s / PEAK_FP64}
    roof_hbm = {"bound": "hbm", "achieved": byts / kern_s / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": byts / kern_s / PEAK_HBM, "traffic": None,
                "bytes_per_cell": byts / n, "ceiling_cells_per_s": ceil_hbm}
    roof, other = (roof_alu, roof_hbm) if ceil_alu <= ceil_hbm else (roof_hbm, roof_alu)
    result = {
        "metric": "cell-updates/s of multigroup source solve (N_g=16,64); Newton iters/cell",
        "value": n / kern_s,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": kern_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded counter-based generator, drawn in HBM before each step)",
        "config": {"workload": WORKLOADS["config4"], "cells": n, "patches": len(layouts),
                   "mean_mode": ["PC", "PPL-fixed", "PPL-free"][args.mode],
                   "batch_tuning": list(b.get_tuning()), "item_scope": b.get_item_scope(), "eps_newton": 1e-11, "polish": 1,
                   "closure": "M1", "timing": "HIP events around each graph launch"},
        "newton_iters_per_cell": {"mean": float(it.mean()), "p50": float(np.percentile(it, 50)),
                                  "p99": float(np.percentile(it, 99)), "max": int(it.max())},
        "outer_passes_per_cell": {"mean": float(ou.mean()), "max": int(ou.max())},
        "status_counts": {str(k): int(v) for k, v in enumerate(np.bincount(stt)) if v},
        "kernel_ms": {"mean": float(np.mean(kern_ms)), "min": float(np.min(kern_ms))},
        "roofline": roof,
        "roofline_other": other,
    }
    if winfo is not None:
        result["warm_start"] = winfo
        result["config"]["warm_start"] = ("one network per group count, temperature guess "
                                          "(guess kind 1); one inference launch per group "
                                          "count and the batched solve replayed from the "
                                          "batch's graph")
        result["config"]["timing"] = "HIP events around each graph launch (inference + solve)"
    print(json.dumps(result), flush=True)


def train_warm_patches(ngs, args):
    """One warm-start network per group count, trained on solver pairs of
    patches of that group count drawn with the training seed (their own
    random tables; untimed)."""
    import torch

    from paper_2407_18304_amd import synth, warmstart
    from paper_2407_18304_amd import workloads as W

    # many small patches: 256 tables per group count (16^3 cells each), so
    # that the network sees the spread of tables the evaluation patches have
    side = 16
    nets, info = {}, {"train_pairs_per_group_count": args.train_cells, "epochs": args.epochs,
                      "training_patches_per_group_count": max(1, args.train_cells // side ** 3)}
    for ng in ngs:
        t0 = time.perf_counter()
        layouts = W.patch_layouts(n_patches=max(1, args.train_cells // side ** 3),
                                  seed=W.TRAIN_SEED, sides=(side,), ngs=(ng,))
        dps = synth.device_patches(layouts, seed=W.TRAIN_SEED)
        Xr, Yr, ok = warmstart.make_training_data_patches(dps)
        t1 = time.perf_counter()
        ws = warmstart.train(Xr, Yr, ok, epochs=args.epochs, batch=4096,
                             holdout=min(1 << 16, int(ok.sum()) // 8),
                             log=lambda m: print(f"N_g={ng} {m}", file=sys.stderr, flush=True))
        torch.cuda.synchronize()
        nets[ng] = ws
        info[f"N_g={ng}"] = {"heldout_loss_first_last": [ws.history[0], ws.history[-1]],
                             "pair_generation_s": t1 - t0,
                             "training_s": time.perf_counter() - t1}
        del dps, Xr, Yr, ok
        torch.cuda.empty_cache()
    return nets, info


def cpu_baseline(dw, mode, target_s):
    """The oracle (as it stands) on the host cores, on a bounded random sample
    of the same cells (inputs copied back from HBM)."""
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle
    from paper_2407_18304_amd import synth
    # the host share of the GPU (OMP_NUM_THREADS where it is set), not the machine
    cores = int(os.environ.get("OMP_NUM_THREADS", 0)) or os.cpu_count() or 1
    rng = np.random.default_rng(7)
    m = min(dw.n, 4096)
    idx = np.sort(rng.choice(dw.n, m, replace=False))
    w = synth.to_host(dw, idx)
    t0 = time.perf_counter()
    oracle.source_update(w.state, w.edges, w.chi_lo, alpha_chi=w.alpha_chi, kappa_scale=w.kappa,
                         mean_mode=mode, polish=1, n_threads=cores, **w.consts(),
                         **w.topacity())
    dt = time.perf_counter() - t0
    m2 = int(min(dw.n, max(m, m * target_s / max(dt, 1e-3))))
    if m2 > m:
        idx = np.sort(rng.choice(dw.n, m2, replace=False))
        w = synth.to_host(dw, idx)
        t0 = time.perf_counter()
        oracle.source_update(w.state, w.edges, w.chi_lo, alpha_chi=w.alpha_chi,
                             kappa_scale=w.kappa, mean_mode=mode, polish=1, n_threads=cores,
                             **w.consts(), **w.topacity())
        dt = time.perf_counter() - t0
        m = m2
    return {"value": m / dt, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "value_per_core": m / dt / cores,
            "sample": f"{m} random cells of the same workload, {dt:.1f} s on {cores} threads",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
