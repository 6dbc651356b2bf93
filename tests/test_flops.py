"""The FP64 operation model of the ALU roofline: edge-branch census against a
brute-force count, the unit-count bookkeeping, and the per-call weights
against the gfx950 assembly of this library's compiler."""
import os
import shutil

import numpy as np
import pytest

from paper_2407_18304_amd import flops as F


def test_edge_mix_matches_brute_force():
    rng = np.random.default_rng(0)
    nu = np.geomspace(1e-3, 1e3, 17)
    T = 10.0 ** rng.uniform(-4, 4, 5000)
    mix = F.edge_mix(nu, 1.0, T)
    x = nu[None, :] / T[:, None]
    assert np.array_equal(mix[0], (x <= 2).sum(1))
    assert np.array_equal(mix[1], ((x > 2) & (x <= 4)).sum(1))
    assert np.array_equal(mix[2], (x > 4).sum(1))
    lo_w, hi_w = x[:, :-1] > 4, x[:, 1:] > 4
    assert np.array_equal(mix[5], lo_w.sum(1))
    assert np.array_equal(mix[4], (~lo_w & hi_w).sum(1))
    assert np.array_equal(mix[3], (~lo_w & ~hi_w).sum(1))


def test_flops_bookkeeping():
    nu = np.geomspace(1e-3, 1e3, 65)
    T = np.array([1.0, 1.0, 1.0])
    mix = F.edge_mix(nu, 1.0, T)
    it = np.array([2.0, 3.0, 3.0])
    ou = np.array([1.0, 1.0, 2.0])
    f = F.flops_per_cell(64, F.FIXED, it, ou, mix)
    u = F.UNIT
    # one more Newton step adds one evaluation and one Newton step
    ev = (mix[0][0] * u["edge"]["x<=2"] + mix[1][0] * u["edge"]["2<x<=4"] +
          mix[2][0] * u["edge"]["x>4"] + mix[3][0] * u["group"]["both<=4"] +
          mix[4][0] * u["group"]["straddle"] + mix[5][0] * u["group"]["wien"] +
          64 * u["ev_group"][F.FIXED] + u["ev_cell"] -
          mix[6][0] * (u["edge"]["x<=2"] - u["edge"]["low"]))
    assert mix[6][0] == 1                     # x = 1e-3 at T = 1: the short path
    nt = 64 * u["nt_group"][F.FIXED] + u["nt_cell"]
    assert f[1] - f[0] == pytest.approx(ev + nt)
    # one more pass adds an evaluation, a Newton step (its polish) and a flux update
    assert f[2] - f[1] == pytest.approx(ev + nt + 64 * u["fx_group"] + u["fx_cell"])
    # invalid cells count nothing
    assert F.flops_per_cell(64, F.FIXED, it, ou, mix, valid=np.zeros(3)).sum() == 0
    # PPL-free costs more per evaluation than PPL-fixed, which costs more than PC
    assert u["ev_group"][F.FREE] > u["ev_group"][F.FIXED] > u["ev_group"][F.PC]
    # with divisions and square roots as one operation: the Planck edges below
    # the Wien side hold none, so they cost the same; the closure holds two
    # divisions, a reciprocal and a square root, each now 1
    u1 = F.UNIT_DIV_SQRT_1
    assert u1["edge"]["x<=2"] == u["edge"]["x<=2"]
    w = F.W
    assert u["fx_group"] - u1["fx_group"] == (2 * (w["div"] - 1) + 2 * (w["rcp_nr"] - 1) +
                                              (w["sqrt_1_4"] - 1))
    f1 = F.flops_per_cell(64, F.FIXED, it, ou, mix, u=u1)
    assert (f1 < f).all()


@pytest.mark.skipif(not shutil.which("hipcc") and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="needs hipcc")
def test_weights_match_the_compiler():
    assert F.measure_weights() == F.W
