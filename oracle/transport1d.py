"""Plain numpy oracle of the 1D explicit M1 radiation transport and of one
two-stage IMEX step with the source update (He, Wibking & Krumholz 2024,
Sec. 2.3: eqs. dysf, ysf, imex1, imex2).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  It shares no code with the GPU library.

Transport operator T(U) of eq. ysf in 1D, per group, on the x-components:
    dE_g/dt = -(c_hat/c) dF_g/dx,    dF_g/dt = -c_hat c dP_g/dx,
    P_g = chi(f) E_g (the M1 Eddington factor of Levermore 1984 along x,
    f = |F_g|/(c E_g) clipped to 1).
READING (the paper defers the transport scheme to its grey predecessor):
finite volumes with the local Lax-Friedrichs (HLL with wave speeds -+c_hat)
flux at each face,
    Phi_E = (c_hat/c) (F_L + F_R)/2 - eps c_hat (E_R - E_L)/2,
    Phi_F = c_hat c (P_L + P_R)/2 - c_hat (F_R - F_L)/2,
where the dissipation of the energy flux is scaled by eps = min(1, 1/tau)^2,
tau = dx (chi_L + chi_R)/2 the optical depth of a cell at the face, so that
in optically thick cells the energy moves by the flux that the implicit
source has relaxed towards its diffusion value and not by numerical
diffusion.  Boundary ghost cells hold given energy densities and zero flux.
The y and z flux components carry no transport (they stay as set).

IMEX step (eqs. imex1, imex2 with S from the source update): stage 1
transports U^n and solves the source terms with theta dt = dt; stage 2 starts
from (U^n + U^(n+1/2))/2 + (dt/2) T(U^(n+1/2)) (eq. imex2 with
dt S(U^(n+1/2)) = U^(n+1/2) - U^n - dt T(U^n) from eq. imex1) and solves with
theta dt = dt/2.
"""
from __future__ import annotations

import numpy as np

import oracle as O


def eddington_factor(E, F, c):
    """Levermore's M1 factor chi(f) along x, f = |F|/(cE) clipped to 1; 1/3
    where E <= 0."""
    E = np.asarray(E, float)
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.where(E > 0.0, np.abs(F) / (c * np.where(E > 0.0, E, 1.0)), 0.0)
    f = np.minimum(f, 1.0)
    return (3.0 + 4.0 * f * f) / (5.0 + 2.0 * np.sqrt(4.0 - 3.0 * f * f))


def ap_factor(tau):
    """Scale of the energy-flux dissipation at a face of optical depth tau."""
    tau = np.asarray(tau, float)
    return np.where(tau > 1.0, 1.0 / np.maximum(tau, 1.0) ** 2, 1.0)


def transport_rhs(E, Fx, dx, c, c_hat, E_left, E_right, chi_cell):
    """T(U) for the energies and x-fluxes: (dE/dt, dFx/dt), each [N_g, n].
    chi_cell: [N_g, n] opacity of each cell (for the dissipation scale)."""
    ng, n = E.shape
    Eg = np.concatenate([np.asarray(E_left, float)[:, None], E, np.asarray(E_right, float)[:, None]],
                        axis=1)
    Fg = np.concatenate([np.zeros((ng, 1)), Fx, np.zeros((ng, 1))], axis=1)
    chig = np.concatenate([chi_cell[:, :1], chi_cell, chi_cell[:, -1:]], axis=1)
    Pg = eddington_factor(Eg, Fg, c) * Eg
    EL, ER = Eg[:, :-1], Eg[:, 1:]
    FL, FR = Fg[:, :-1], Fg[:, 1:]
    PL, PR = Pg[:, :-1], Pg[:, 1:]
    tau = dx * 0.5 * (chig[:, :-1] + chig[:, 1:])
    eps = ap_factor(tau)
    phiE = (c_hat / c) * 0.5 * (FL + FR) - eps * c_hat * 0.5 * (ER - EL)
    phiF = c_hat * c * 0.5 * (PL + PR) - c_hat * 0.5 * (FR - FL)
    return -(phiE[:, 1:] - phiE[:, :-1]) / dx, -(phiF[:, 1:] - phiF[:, :-1]) / dx


def _explicit(a, U0, b, U1, dtT, prob, c_hat, chi_cell):
    """a U0 + b U1 + dtT T(U1) for the radiation; a U0 + b U1 for the gas."""
    out = {}
    for k in ("E_g", "F_g", "e_gas", "v"):
        out[k] = b * U1[k] + (a * U0[k] if a != 0.0 else 0.0)
    out["rho"] = U1["rho"]
    dE, dF = transport_rhs(U1["E_g"], U1["F_g"][0], prob.dx, prob.c, c_hat, prob.E_left,
                           prob.E_right, chi_cell)
    out["E_g"] = out["E_g"] + dtT * dE
    out["F_g"] = np.array(out["F_g"], copy=True)
    out["F_g"][0] = out["F_g"][0] + dtT * dF
    return out


def imex_step(U, prob, mode, c_hat=None, polish=1, n_threads=0, **src):
    """One step of eqs. imex1/imex2 for the 1D problem ``prob`` (see
    workloads.marshak) in mean mode ``mode``.  Returns (U^(n+1), status of
    the two source solves)."""
    c_hat = prob.c if c_hat is None else c_hat
    chi_cell = prob.chi_mid[:, None] * U["rho"][None, :]
    kw = dict(alpha_chi=prob.alpha_chi, mean_mode=mode, c_hat=c_hat, polish=polish,
              n_threads=n_threads, **prob.consts(), **src)
    Ut = _explicit(0.0, U, 1.0, U, prob.dt, prob, c_hat, chi_cell)
    Uh, _, _, s1 = O.source_update(Ut, prob.edges, prob.chi_lo, dt=prob.dt, **kw)
    Ut2 = _explicit(0.5, U, 0.5, Uh, 0.5 * prob.dt, prob, c_hat, chi_cell)
    Un, _, _, s2 = O.source_update(Ut2, prob.edges, prob.chi_lo, dt=0.5 * prob.dt, **kw)
    return Un, (s1, s2)
