"""The two-stage IMEX step of the source terms (mgrhd_imex_step, eqs. imex1
and imex2 with no transport) on the GPU: the Doppler test of Sec. 4.2.1
reaches the printed equilibrium temperature and the Doppler-shifted group
flux spectrum (eq. Fdiff), and the trajectory matches the oracle stepped with
the same two stages.  GPU only."""
import os

import numpy as np
import pytest
import torch

import mp_ref
import oracle
from paper_2407_18304_amd import mgrhd
from paper_2407_18304_amd import workloads as W

import gpu_util as U

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    vals = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = line.split("=")
            vals[k.strip()] = float(v)
    return vals


def _state(ng, n):
    # T0 = 1, E = F = 0, v = 1e-3 c along x, rho = 1, C_V = 3/2
    v = np.zeros((3, n))
    v[0] = 1e-3
    return {"E_g": np.zeros((ng, n)), "F_g": np.zeros((3, ng, n)), "rho": np.ones(n),
            "e_gas": 1.5 * np.ones(n) + 0.5 * (v * v).sum(0), "v": v}


@pytest.mark.parametrize("ng", [8, 16, 64])
def test_doppler_equilibrium_imex(ng):
    gold = _golden("doppler_equilibrium.txt")
    n = 3
    edges = np.logspace(-3, 2, ng + 1)
    chi = np.full(ng, 1e5)
    dt, steps = 8.0, 125                        # to t = 1000
    kw = dict(mean_mode=0, c_hat=1.0, c=1.0, a_rad=1.0, polish=1, max_outer=30)
    # GPU: one mgrhd_imex_step per step
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()
    st = {k: t(v) for k, v in _state(ng, n).items()}
    e_d, chi_d = t(edges), t(chi)
    work = torch.empty(mgrhd.imex_workspace_bytes(n, ng) // 8, dtype=torch.float64,
                       device="cuda")
    status = torch.zeros(n, dtype=torch.int32, device="cuda")
    for _ in range(steps):
        mgrhd.source_update(st["E_g"], st["F_g"], st["rho"], st["e_gas"], st["v"], e_d, chi_d,
                            dt=dt, status=status, imex_work=work, **kw)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in st.items()}
    assert (status.cpu().numpy() == 0).all()
    T = (g["e_gas"] - 0.5 * g["rho"] * (g["v"] ** 2).sum(0)) / (1.5 * g["rho"])
    assert np.abs(T - gold["T_eq_exact"]).max() < 2e-6
    x = edges / T[0]
    B = np.array([float(mp_ref.group_fraction(x[k], x[k + 1])) * T[0] ** 4 for k in range(ng)])
    nuB = np.array([float(mp_ref.edge_term(xe)) * T[0] ** 4 for xe in x])
    Fdiff = g["v"][0, 0] * (4.0 / 3.0 * B - (nuB[1:] - nuB[:-1]) / 3.0)
    big = B > 1e-6 * B.max()
    assert np.abs(g["F_g"][0, big, 0] / Fdiff[big] - 1).max() < gold["flux_rel_err_max"]
    # the oracle, stepped with the same two stages
    o = _state(ng, n)
    for _ in range(steps):
        half, *_ = oracle.source_update(o, edges, chi, dt=dt, **kw)
        mid = {k: 0.5 * (o[k] + half[k]) for k in ("E_g", "F_g", "e_gas", "v")}
        mid["rho"] = o["rho"]
        o, *_ = oracle.source_update(mid, edges, chi, dt=0.5 * dt, **kw)
    w = W.Workload("doppler", n, edges, chi, np.zeros(ng), np.ones(n), _state(ng, n), T,
                     dt=dt, c_hat=1.0, c=1.0, a_rad=1.0)
    for k, e in U.field_errors(w, g, o).items():
        assert e < 1e-10, (k, e)


def test_imex_workspace_too_small_is_rejected():
    ng, n = 4, 10
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()
    s = {k: t(v) for k, v in _state(ng, n).items()}
    work = torch.empty(8, dtype=torch.float64, device="cuda")
    with pytest.raises(mgrhd.MgrhdError):
        mgrhd.source_update(s["E_g"], s["F_g"], s["rho"], s["e_gas"], s["v"],
                            t(np.logspace(-3, 2, ng + 1)), t(np.ones(ng)), dt=1.0, c_hat=1.0,
                            mean_mode=0, imex_work=work)
