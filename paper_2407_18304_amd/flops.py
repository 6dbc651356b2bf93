"""FP64 operation count of the source update, for its ALU roofline.

The source update does no dense contraction: its arithmetic runs on the FP64
vector ALUs (peak 78.6 TFLOP/s on MI355X: 256 CUs x 2.4 GHz x 64 FP64 FMA
lanes per CU per clock x 2).  The count below is the algorithmic work of the
method as the kernels write it, per cell, in FLOP-equivalents:

* +, -, x = 1 and fused multiply-add = 2; comparisons, selects, integer and
  memory work = 0;
* a call of exp, expm1, log, sqrt, a division or the kernels' own e^{-x},
  range-bounded reciprocal and square root (exp_neg, rcp_nr, sqrt_1_4 of
  planck_device.hpp) costs the FLOP-equivalents of
  the FP64 instruction sequence gfx950 code uses for it (FMA = 2, every other
  FP64 arithmetic instruction = 1, compares 0), counted in the assembly of a
  probe kernel built with the library's flags (``python -m
  paper_2407_18304_amd.flops``, which prints the weights below).

Per-unit counts come from the kernel source, operation by operation (the
table in ``UNIT`` names each term).  The number of units per cell follows
from the kernel's own per-cell counters: with ``iters`` Newton steps (polish
steps not included) and ``outer`` passes, a cell takes ``iters + outer + 1``
material evaluations, ``iters + outer`` Newton steps (one polish step per
pass) and ``outer`` flux updates.  Which branch an edge's Planck evaluation
takes depends on x = (h/k) nu / T; the count uses each cell's final
temperature for every evaluation of that cell (the Newton iterates of a cell
differ from it by the step, a small fraction of T).
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
import tempfile
from collections import Counter

import numpy as np

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")

# FLOP-equivalents of one call on gfx950 (measured by measure_weights())
W = {"exp": 29, "expm1": 34, "log": 84, "div": 17, "sqrt": 19, "exp_neg": 34, "rcp_nr": 9,
     "sqrt_1_4": 17}

PC, FIXED, FREE = 0, 1, 2


def unit_costs(w=W):
    """Per-unit FLOP-equivalents of the kernel source (see module doc)."""
    e, m1, lg, dv, sq = w["exp"], w["expm1"], w["log"], w["div"], w["sqrt"]
    en, rc, s14 = w["exp_neg"], w["rcp_nr"], w["sqrt_1_4"]
    # one Planck edge: x = hk/T * nu (1), x^2 and x^3 (2), then by branch
    edge_common = 1 + 2
    poly_P = 14 * 2 + 6              # degree-14 Horner in x^2 and the bracket
    poly_E = 16 * 2 + 6              # degree-16 Horner in x^2 for x/(e^x-1) and the bracket
    edge = {
        "x<=2": edge_common + poly_P + poly_E,
        "2<x<=4": edge_common + poly_P + poly_E,
        # e^{-x}, the 10-term tail as four degree-9 Horner chains in u and their
        # combination, then x^4/(1 - u) (three products, 1 - u, a reciprocal)
        "x>4": edge_common + en + 4 * 9 * 2 + 10 + (4 + rc),
        # the lowest edge at x <= 0.1: both polynomials truncated to degree 3
        "low": edge_common + 2 * (3 * 2 + 6),
    }
    # group data from its two edges (group_planck)
    group = {"both<=4": 1, "straddle": 4, "wien": 3 + dv}
    # per group and evaluation, after the Planck data: B~, Delta(nu B~), dB/dT (8)
    ev_group = {
        PC: 1 + 8 + 3,                                        # chi (1), emit
        FIXED: 1 + 8 + 4 + 4 + 3 + dv + 5,                    # chi, dchib, chi_F num/den, emit
        # E_g of the iterate (1), logs of the two slope fits (B and E), two
        # slope pairs, two group means (two expm1-brackets, a division and a
        # rescaling exp each), chi_F, emit
        FREE: 1 + 8 + 1 + (2 * lg + 3) + 2 * (2 * (2 + dv)) +
              2 * (1 + 1 + 2 * (2 + m1 + dv) + 3 + dv + e) + 3 + 6 + 3 + dv + 5,
    }
    ev_cell = 2 + 3 + dv + 1           # T = (E_gas - ke)/(rho c_v) (2), a T^4, 1/T, hk/T
    # Newton step per group: W (5, with v.F cached per pass), E_g (3), F_R (2),
    # J_g0 (1), a_g b_g (2), four sums (4), update of R_g (4); PPL-free adds
    # chi_B/chi_E and its two products, 1/tau (1 + div) and 1/J_gg (1 + rcp)
    nt_group = {PC: 21, FIXED: 21, FREE: 21 + 2 + dv + (1 + dv) + (1 + rc)}
    # per cell: F_G (3), the two stop tests (3), dx_0 (numerator and
    # denominator 4, a division by a reciprocal and one correction: rc + 5),
    # the positivity check of the step (3), the update of E_gas (2)
    nt_cell = 3 + 3 + 4 + (rc + 5) + 3 + 2
    # flux update per group: E_new (1), M1 closure P.v (F.F: 5, 1/(cE): 1+div,
    # f^2: 2, chi: 2 + sqrt on [1,4] + 2 + reciprocal + 2 + 1, p: 2,
    # q: 4 + F.v (5) + div, P.v: 12), 1/(1+cdt chi_F) (2 + reciprocal), chi_E and
    # (1+a)chi_E (3), three components (3 x 8), the new v.F (5) and the dW term (5)
    closure = 5 + (1 + dv) + 2 + (2 + s14 + 2 + rc + 2 + 1) + 2 + (9 + dv) + 12
    fx_group = 1 + closure + (2 + rc) + 3 + 24 + 10
    # per cell: 1/rho (1), the momentum update (12), dW scale (1), new kinetic
    # energy (7), the next pass's E_gas (2), the outer test (1)
    fx_cell = 1 + 12 + 1 + 7 + 2 + 1
    # cell load: per group E0 (1), sum (1), v.F (5), 1/tau (2 + div) and
    # 1/J_gg (1 + reciprocal) in PC and PPL-fixed; per cell rho kappa (1),
    # 1/(rho c_v) (1 + div), kinetic energy (7), E_tot (2), 1/E_tot (div)
    ld_group = {PC: 7 + (2 + dv) + (1 + rc), FIXED: 7 + (2 + dv) + (1 + rc), FREE: 7}
    ld_cell = 1 + (1 + dv) + 7 + 2 + dv
    # Temperature-dependent opacity, on top of the above.  Per evaluation and
    # cell: (T/T_ref)^beta = exp(beta ln(T/T_ref)).  Per edge with the
    # stimulated-emission factor: x/(x + x/(e^x-1)) below the Wien side, 1 - u
    # beyond.  Per group: chi_0,g- at T (2 products, 3 with the factor); with
    # the factor in PPL, the ratio s_g+/s_g-, the index change ln(ratio)/ln r,
    # r^alpha times the ratio, and in PPL-fixed the mean of eq. chiQg at the
    # new index (a y = aL, an expm1-bracket, a division, the rescaling exp of
    # half the groups, the product).  Per Newton step and group: 1/tau and
    # 1/J_gg (no longer per-cell constants); the cell load skips them.
    td = dict(
        ev_cell_pow=1 + lg + e + 1,
        edge_stim={"nonwien": 1 + dv, "wien": 1},
        ev_group={PC: 2, FIXED: 3, FREE: 2},
        ev_group_stim={PC: 1, FIXED: 1 + dv + lg + dv + 1 + 1 + (1 + m1 + dv) + dv + e / 2,
                       FREE: 1 + dv + lg + dv + 1 + 1},
        nt_group={PC: (1 + dv) + (1 + rc), FIXED: (1 + dv) + (1 + rc), FREE: 0},
        ld_group={PC: -((2 + dv) + (1 + rc)), FIXED: -((2 + dv) + (1 + rc)), FREE: 0},
    )
    return dict(edge=edge, group=group, ev_group=ev_group, ev_cell=ev_cell,
                nt_group=nt_group, nt_cell=nt_cell, fx_group=fx_group, fx_cell=fx_cell,
                ld_group=ld_group, ld_cell=ld_cell, td=td)


UNIT = unit_costs()
# The same count with every division and square root (the kernels' range-bounded
# reciprocal and square root included) as one operation, transcendentals as
# above: the lower figure a convention that prices only exp/expm1/log by their
# instruction sequences gives.
UNIT_DIV_SQRT_1 = unit_costs(dict(W, div=1, sqrt=1, rcp_nr=1, sqrt_1_4=1))


def edge_mix(nu, hk, T):
    """Per cell: numbers of edges with x <= 2, 2 < x <= 4, x > 4 and of groups
    whose edges are both at x <= 4, straddle x = 4, or lie beyond it.
    nu: ascending edges [N_g+1]; T: final temperatures [n] (numpy or torch)."""
    xp = _xp(T)
    ng = len(nu) - 1
    nu_t = xp.asarray(nu) if xp is np else xp.as_tensor(nu, dtype=T.dtype, device=T.device)
    n2 = _searchsorted(xp, nu_t, 2.0 * T / hk)
    n4 = _searchsorted(xp, nu_t, 4.0 * T / hk)
    e_le2 = n2
    e_24 = n4 - n2
    e_gt4 = (ng + 1) - n4
    g_wien = xp.clip(ng - n4, 0, None) if xp is np else (ng - n4).clamp(min=0)
    g_strad = ((n4 >= 1) & (n4 <= ng)) * 1
    g_both = ng - g_wien - g_strad
    low0 = (nu_t[0] * hk / T <= 0.1) * 1     # the lowest edge takes the short path
    return e_le2, e_24, e_gt4, g_both, g_strad, g_wien, low0


def _xp(a):
    return np if isinstance(a, np.ndarray) else sys.modules["torch"]


def _searchsorted(xp, sorted_seq, v):
    if xp is np:
        return np.searchsorted(sorted_seq, v, side="right")
    return xp.searchsorted(sorted_seq, v.contiguous(), right=True)


def flops_per_cell(ng, mode, iters, outer, mix, u=UNIT, valid=None, t_exp=0.0, stim=0):
    """FLOP-equivalents per cell (array).  iters, outer: the kernel's per-cell
    counters; mix: edge_mix(...) of the cell's final temperature; t_exp, stim:
    the opacity's temperature dependence."""
    e_le2, e_24, e_gt4, g_both, g_strad, g_wien, low0 = mix
    E = u["edge"]
    G = u["group"]
    per_eval = (e_le2 * E["x<=2"] + e_24 * E["2<x<=4"] + e_gt4 * E["x>4"] +
                g_both * G["both<=4"] + g_strad * G["straddle"] + g_wien * G["wien"] +
                ng * u["ev_group"][mode] + u["ev_cell"] -
                low0 * (E["x<=2"] - E["low"]))
    tdep = t_exp != 0.0 or stim != 0
    if tdep:
        T = u["td"]
        per_eval = per_eval + ng * T["ev_group"][mode]
        if t_exp != 0.0:
            per_eval = per_eval + T["ev_cell_pow"]
        if stim:
            per_eval = per_eval + ((e_le2 + e_24) * T["edge_stim"]["nonwien"] +
                                   e_gt4 * T["edge_stim"]["wien"] +
                                   ng * T["ev_group_stim"][mode])
    n_eval = iters + outer + 1
    n_newton = iters + outer
    nt_group = u["nt_group"][mode] + (u["td"]["nt_group"][mode] if tdep else 0)
    ld_group = u["ld_group"][mode] + (u["td"]["ld_group"][mode] if tdep else 0)
    f = (n_eval * per_eval + n_newton * (ng * nt_group + u["nt_cell"]) +
         outer * (ng * u["fx_group"] + u["fx_cell"]) + ng * ld_group + u["ld_cell"])
    if valid is not None:
        f = f * valid
    return f


# ---------------------------------------------------------------------------
PROBE = r"""
#include <hip/hip_runtime.h>
#include <cmath>
#include "planck_device.hpp"
#define K(name, expr) extern "C" __global__ void name(const double* __restrict__ a, \
    double* __restrict__ o) { int i = threadIdx.x; double x = a[i]; o[i] = expr; }
K(p_exp, exp(x))
K(p_expm1, expm1(x))
K(p_log, log(x))
K(p_div, a[i + 64] / x)
K(p_sqrt, sqrt(x))
K(p_exp_neg, mgrhd::exp_neg(x))
K(p_rcp_nr, mgrhd::rcp_nr(x))
K(p_sqrt_1_4, mgrhd::sqrt_1_4(x))
"""


def _flop_weight(ins: str) -> int:
    if "_cmp" in ins or "cvt" in ins or "class" in ins:
        return 0
    if ins.startswith(("v_fma_f64", "v_fmac_f64", "v_div_fmas_f64")):
        return 2
    return 1


def measure_weights(hipcc="/opt/rocm/bin/hipcc", arch="gfx950"):
    """Compile the probe with the library's FP64 flags and count the
    FLOP-equivalents of each function's FP64 instructions."""
    with tempfile.TemporaryDirectory() as d:
        src, asm = os.path.join(d, "probe.hip"), os.path.join(d, "probe.s")
        with open(src, "w") as f:
            f.write(PROBE)
        subprocess.run([hipcc, f"--offload-arch={arch}", "-O3", "-Xclang", "-target-feature",
                        "-Xclang", "-packed-fp32-ops", "-I", CSRC, "--cuda-device-only", "-S",
                        "-o", asm, src], check=True, capture_output=True)
        text = open(asm).read()
    out, cur, body = {}, None, []
    for line in text.splitlines():
        m = re.match(r"^p_(\w+):", line)
        if m:
            cur, body = m.group(1), []
            continue
        if cur is None:
            continue
        tok = line.strip().split()
        if tok and tok[0] == "s_endpgm":
            c = Counter(t for t in body if t.startswith("v_") and "f64" in t)
            out[cur] = sum(_flop_weight(k) * v for k, v in c.items())
            cur = None
        elif tok:
            body.append(tok[0])
    return out


if __name__ == "__main__":
    w = measure_weights()
    print("FLOP-equivalents per call:", w)
    u = unit_costs(w)
    for k, v in u.items():
        print(f"  {k}: {v}")
