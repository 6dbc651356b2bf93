"""Pins of the transport oracle (oracle/transport1d.py): exact translation of a
free-streaming pulse, flux-form conservation, a stationary uniform state, the
diffusion rate c/(3 chi) of the optically thick limit against the closed form
of a spreading Gaussian, and a stationary equilibrium through the whole IMEX
step.  CPU only."""
import numpy as np
import pytest

import transport1d as T
from paper_2407_18304_amd import workloads as W

C = 3.0e10


def test_free_streaming_pulse_translates_exactly():
    """F = cE (f = 1, chi(f) = 1, P = E) at c dt = dx: one explicit step moves
    every E and F exactly one cell downstream (the flux is then the upwind one)."""
    n = 40
    x = np.arange(n)
    E = np.where((x > 10) & (x < 20), 1.0 + 0.1 * x, 0.0)[None, :]
    F = C * E
    dx = 1.0
    dt = dx / C
    dE, dF = T.transport_rhs(E, F, dx, C, C, [0.0], [0.0], np.zeros((1, n)))
    E1, F1 = E + dt * dE, F + dt * dF
    assert np.allclose(E1[0, 1:], E[0, :-1], rtol=1e-14, atol=1e-14)
    assert np.allclose(F1[0, 1:], F[0, :-1], rtol=1e-14, atol=1e-14 * C)


def test_uniform_state_is_stationary_and_flux_form_conserves():
    n, ng = 30, 3
    E = np.full((ng, n), 2.5)
    dE, dF = T.transport_rhs(E, np.zeros((ng, n)), 0.1, C, C, np.full(ng, 2.5),
                             np.full(ng, 2.5), np.full((ng, n), 7.0))
    assert np.abs(dE).max() == 0.0 and np.abs(dF).max() == 0.0
    # any state: the total changes only by the boundary fluxes
    rng = np.random.default_rng(0)
    E = rng.uniform(0.5, 2.0, (ng, n))
    F = rng.uniform(-0.5, 0.5, (ng, n)) * C * E
    chi = rng.uniform(0.1, 10.0, (ng, n))
    El, Er = np.full(ng, 1.0), np.full(ng, 0.7)
    dE, dF = T.transport_rhs(E, F, 0.1, C, C, El, Er, chi)
    # boundary fluxes written out for the two ghost faces
    def face(EL, ER, FL, FR, chiL, chiR):
        PL = T.eddington_factor(EL, FL, C) * EL
        PR = T.eddington_factor(ER, FR, C) * ER
        eps = T.ap_factor(0.1 * 0.5 * (chiL + chiR))
        return 0.5 * (FL + FR) - eps * C * 0.5 * (ER - EL), C * C * 0.5 * (PL + PR) - C * 0.5 * (FR - FL)
    lE, lF = face(El, E[:, 0], 0.0, F[:, 0], chi[:, 0], chi[:, 0])
    rE, rF = face(E[:, -1], Er, F[:, -1], 0.0, chi[:, -1], chi[:, -1])
    assert np.allclose(dE.sum(1) * 0.1, lE - rE, rtol=1e-12)
    assert np.allclose(dF.sum(1) * 0.1, lF - rF, rtol=1e-12)


def test_thick_limit_diffuses_at_c_over_3chi():
    """Optically thick medium (tau = 100 per cell) with the flux relaxed
    implicitly as the source update does with v = 0 (eq. numF1:
    F <- F^(t)/(1 + c dt chi)): a Gaussian's variance grows as 2 D t with
    D = c/(3 chi), to the 1.5/tau of the residual dissipation and the time
    discretisation."""
    n, dx, chi = 240, 1.0, 100.0
    x = (np.arange(n) - n / 2 + 0.5) * dx
    s0 = 12.0
    E = np.exp(-x ** 2 / (2 * s0 ** 2))[None, :]
    F = np.zeros_like(E)
    dt = 0.5 * dx / C
    D = C / (3 * chi)
    steps = 6000
    chic = np.full((1, n), chi)
    for _ in range(steps):
        dE, dF = T.transport_rhs(E, F, dx, C, C, [0.0], [0.0], chic)
        E = E + dt * dE
        F = (F + dt * dF) / (1.0 + C * dt * chi)
    t = steps * dt
    var = (E[0] * x ** 2).sum() / E[0].sum()
    assert abs(E.sum() - np.exp(-x ** 2 / (2 * s0 ** 2)).sum()) < 1e-9 * E.sum()
    assert abs((var - s0 ** 2) / (2 * D * t) - 1.0) < 0.05


def test_equilibrium_is_stationary_through_the_imex_step(ora):
    """Uniform T = 300 K with E_g = B_g(T) and both boundaries at 300 K: one
    full step (transport, source solves of both stages) leaves it unchanged."""
    prob = W.marshak(4, n_cells=12)
    T0 = 300.0
    Eb = np.array([ora.group_planck(prob.h_over_k * prob.edges[g] / T0,
                                    prob.h_over_k * prob.edges[g + 1] / T0) for g in range(4)])
    Eb = prob.a_rad * T0 ** 4 * Eb[:, 0] * np.exp(-Eb[:, 3])       # the oracle's B~_g(T0)
    prob.state["E_g"] = np.repeat(Eb[:, None], prob.n, axis=1)
    prob.E_left = prob.E_right = Eb
    U1, (s1, s2) = T.imex_step(prob.state, prob, 1)
    assert (s1 == 0).all() and (s2 == 0).all()
    for k in ("E_g", "e_gas"):
        assert np.allclose(U1[k], prob.state[k], rtol=1e-12, atol=0), k
    assert np.abs(U1["F_g"]).max() < 1e-12 * C * prob.state["E_g"].max()
