"""Autotuner for the source-update kernels.

Single-table kernel: the compiled variants (lanes per cell x groups per lane
x register budget) that cover N_g are timed on a sample of the workload (inputs restored before
every timed launch, HIP events on the launch stream) and the fastest is
installed with mgrhd_set_variant.  Batched launch: groups per lane, resident
workgroups per CU and cells per work item are timed the same way.  Results are
cached per (GPU architecture, N_g, mean mode) in a JSON file.
"""
from __future__ import annotations

import json
import os

import torch

from . import mgrhd

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")


def arch() -> str:
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def load_cache(path=CACHE) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save_cache(cache, path=CACHE):
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def apply_cache(path=CACHE, mode=None) -> dict:
    """Install the cached single-table choices for this GPU (for mean mode
    `mode`, or all); returns them."""
    cache = load_cache(path).get(arch(), {})
    for key, rec in cache.get("single", {}).items():
        ng, m = (int(x) for x in key.split(":"))
        if mode is not None and m != mode:
            continue
        try:
            mgrhd.set_variant(ng, rec["lanes_per_cell"], rec["groups_per_lane"],
                              rec.get("waves_per_simd", 0))
        except mgrhd.MgrhdError:
            pass
    return cache


def _time(fn, restore, reps=3):
    s = torch.cuda.current_stream()
    best = float("inf")
    for _ in range(reps):
        restore()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        fn()
        b.record(s)
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def tune_single(dw, mode=mgrhd.MEAN_PPL_FIXED, reps=3, path=CACHE, log=print):
    """Time every compiled variant covering dw.ng on the device workload dw."""
    pristine = {k: v.clone() for k, v in dw.state.items()}
    st = dw.state

    def restore():
        for k in ("E_g", "F_g", "e_gas", "v"):
            st[k].copy_(pristine[k])

    def run():
        mgrhd.source_update(st["E_g"], st["F_g"], st["rho"], st["e_gas"], st["v"],
                            dw.tables["edges"], dw.tables["chi_lo"], alpha_chi=dw.tables["alpha"],
                            kappa_scale=dw.kappa, mean_mode=mode, polish=1, **dw.consts())

    results = []
    for lpc, g, wps in mgrhd.variants():
        if lpc * g < dw.ng or lpc * g >= 2 * dw.ng:
            continue
        mgrhd.set_variant(dw.ng, lpc, g, wps)
        run()                    # warm up (first launch loads the code object)
        ms = _time(run, restore, reps)
        results.append((ms, lpc, g, wps))
        log(f"  N_g={dw.ng} mode={mode}: {lpc} lanes x {g} groups, {wps} waves/SIMD -> {ms:.3f} ms")
    restore()
    ms, lpc, g, wps = min(results)
    mgrhd.set_variant(dw.ng, lpc, g, wps)
    cache = load_cache(path)
    ent = cache.setdefault(arch(), {}).setdefault("single", {})
    ent[f"{dw.ng}:{mode}"] = {"lanes_per_cell": lpc, "groups_per_lane": g, "waves_per_simd": wps,
                             "ms": ms, "cells": dw.n, "all": [list(r) for r in sorted(results)]}
    save_cache(cache, path)
    return lpc, g, wps, ms


def tune_batch(batch, restore, candidates=None, reps=2, path=CACHE, key="patches", log=print):
    """Time batch tunings (groups per lane, blocks per CU, cells per item,
    item scope)."""
    if candidates is None:
        candidates = [(g, b, ch, 0) for g in (2, 4) for b in (0, 1) for ch in (1024, 4096)]
        candidates += [(2, 0, ch, 1) for ch in (128, 256, 512, 1024)]
        candidates += [(2, 0, ch, 2) for ch in (256, 1024)]
        candidates += [(4, 0, 1024, 2)]
    results = []
    for g, b, ch, sc in candidates:
        try:
            batch.set_tuning(g, b, ch)
            batch.set_item_scope(sc)
        except mgrhd.MgrhdError:
            continue
        batch.run()
        ms = _time(batch.run, restore, reps)
        results.append((ms, g, b, ch, sc))
        log(f"  batch: {g} groups/lane, {b or 'all'} blocks/CU, {ch} cells/item, "
            f"items per {'workgroup (%d waves/SIMD)' % (4 - sc) if sc else 'wave'} -> {ms:.3f} ms")
    restore()
    ms, g, b, ch, sc = min(results)
    batch.set_tuning(g, b, ch)
    batch.set_item_scope(sc)
    cache = load_cache(path)
    cache.setdefault(arch(), {}).setdefault("batch", {})[key] = {
        "groups_per_lane": g, "blocks_per_cu": b, "chunk_cells": ch, "item_scope": sc, "ms": ms,
        "all": [list(r) for r in sorted(results)]}
    save_cache(cache, path)
    return g, b, ch, sc, ms
