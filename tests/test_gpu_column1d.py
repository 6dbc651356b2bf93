"""The 1D column of the IMEX integrator on the GPU (mgrhd_transport1d_stage
and mgrhd_source_update per stage, paper_2407_18304_amd/column1d.py): the
transport stage against the oracle's transport operator, and whole IMEX steps
of the Marshak problem against the oracle's steps, eager and replayed from a
HIP graph.  GPU only."""
import numpy as np
import pytest
import torch

from paper_2407_18304_amd import column1d, mgrhd
from paper_2407_18304_amd import workloads as W

import transport1d as T

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

C = W.CGS["c"]


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _random_state(rng, ng, n):
    E = rng.uniform(0.1, 2.0, (ng, n))
    F = np.zeros((3, ng, n))
    F[0] = rng.uniform(-1.0, 1.0, (ng, n)) * C * E
    F[1] = rng.uniform(-0.3, 0.3, (ng, n)) * C * E
    return {"E_g": E, "F_g": F, "e_gas": rng.uniform(1.0, 2.0, n), "v": rng.normal(size=(3, n))}


@pytest.mark.parametrize("ng,n", [(1, 1), (4, 37), (16, 500)])
def test_transport_stage_matches_oracle(ng, n):
    rng = np.random.default_rng(ng * 1000 + n)
    U0, U1 = _random_state(rng, ng, n), _random_state(rng, ng, n)
    rho = rng.uniform(0.5, 2.0, n)
    chi_mid = 10.0 ** rng.uniform(-2, 4, ng)
    El, Er = rng.uniform(0.1, 2.0, ng), rng.uniform(0.1, 2.0, ng)
    dx, dtT = 0.04, 0.3 * 0.04 / C
    a, b = 0.5, 0.5
    d0, d1 = {k: _t(v) for k, v in U0.items()}, {k: _t(v) for k, v in U1.items()}
    out = {k: torch.empty_like(v) for k, v in d1.items()}
    mgrhd.transport1d_stage(out, d1, d0, a=a, b=b, dx=dx, dt_T=dtT, c=C, c_hat=C, rho=_t(rho),
                            chi_mid=_t(chi_mid), E_left=_t(El), E_right=_t(Er))
    torch.cuda.synchronize()
    dE, dF = T.transport_rhs(U1["E_g"], U1["F_g"][0], dx, C, C, El, Er,
                             chi_mid[:, None] * rho[None, :])
    refE = a * U0["E_g"] + b * U1["E_g"] + dtT * dE
    refF = a * U0["F_g"] + b * U1["F_g"]
    refF[0] += dtT * dF
    scale = np.abs(U0["E_g"]) + np.abs(U1["E_g"])
    assert np.abs(out["E_g"].cpu().numpy() - refE).max() / scale.max() < 1e-14
    assert np.abs(out["F_g"].cpu().numpy() - refF).max() / (C * scale.max()) < 1e-14
    assert np.allclose(out["e_gas"].cpu().numpy(), a * U0["e_gas"] + b * U1["e_gas"], rtol=1e-15)
    assert np.allclose(out["v"].cpu().numpy(), a * U0["v"] + b * U1["v"], rtol=1e-15, atol=1e-15)
    # the output may alias U0 (read and written by the same thread), not U1
    mgrhd.transport1d_stage(d0, d1, d0, a=a, b=b, dx=dx, dt_T=dtT, c=C, c_hat=C, rho=_t(rho),
                            chi_mid=_t(chi_mid), E_left=_t(El), E_right=_t(Er))
    torch.cuda.synchronize()
    assert torch.equal(d0["E_g"], out["E_g"]) and torch.equal(d0["F_g"], out["F_g"])
    with pytest.raises(mgrhd.MgrhdError):
        mgrhd.transport1d_stage(d1, d1, None, a=0.0, b=1.0, dx=dx, dt_T=dtT, c=C, c_hat=C,
                                rho=_t(rho), chi_mid=_t(chi_mid), E_left=_t(El), E_right=_t(Er))


def _fields_close(g, o, tol):
    for k in ("E_g", "e_gas"):
        err = np.abs(g[k] - o[k]) / np.maximum(np.abs(o[k]), 1e-30)
        assert err.max() < tol, (k, err.max())
    # fluxes: relative, with a floor of 1e-6 of the free-streaming flux c E_g of
    # the cell (ahead of the wave and at the far boundary the flux is the
    # difference of nearly equal energies, where rounding decides its digits)
    fl = 1e-6 * C * np.abs(o["E_g"])[None]
    err = np.abs(g["F_g"] - o["F_g"]) / np.maximum(np.abs(o["F_g"]), fl)
    assert err.max() < tol, ("F_g", err.max())


@pytest.mark.parametrize("ng,mode", [(4, 0), (4, 1), (4, 2), (8, 1)])
def test_marshak_steps_match_oracle(ng, mode):
    """60 IMEX steps of the Marshak problem (the wave enters from the left)."""
    prob = W.marshak(ng, n_cells=120)
    col = column1d.Column1D(prob, mode)
    col.run(60, graph_steps=0)
    g = col.state()
    assert ((col.status_any.cpu().numpy() & ~4) == 0).all()
    U = {k: v.copy() for k, v in prob.state.items()}
    for _ in range(60):
        U, _ = T.imex_step(U, prob, mode)
    assert (np.abs(U["E_g"] - prob.state["E_g"]) > 0).any()          # something happened
    _fields_close(g, U, 1e-10)


def test_graph_replay_equals_eager_steps():
    prob = W.marshak(8, n_cells=64)
    a = column1d.Column1D(prob, 1)
    a.run(45, graph_steps=0)
    b = column1d.Column1D(prob, 1)
    b.run(45, graph_steps=11)                 # 1 eager + 4 replays of 11 steps + 0 eager
    assert a.steps_done == b.steps_done == 45
    sa, sb = a.state(), b.state()
    for k in ("E_g", "F_g", "e_gas", "v"):
        assert np.array_equal(sa[k], sb[k]), k
