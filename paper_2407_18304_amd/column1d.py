"""A 1D column of cells advanced by the two-stage IMEX integrator of the
radiation subsystem (He, Wibking & Krumholz 2024, Sec. 2.3, eqs. imex1 and
imex2), entirely on the GPU: the explicit M1 transport stage
(mgrhd_transport1d_stage) and the implicit source update
(mgrhd_source_update) per stage, state resident in HBM, many steps captured
in one HIP graph and replayed.

    stage 1:  U^t  = U^n + dt T(U^n);                      source update, theta dt = dt
    stage 2:  U^t2 = (U^n + U^(n+1/2))/2 + (dt/2) T(U^(n+1/2)); source update, theta dt = dt/2

(eq. imex2 with dt S(U^(n+1/2)) = U^(n+1/2) - U^n - dt T(U^n) from eq. imex1).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import mgrhd

KEYS = ("E_g", "F_g", "e_gas", "v")


class Column1D:
    """prob: a workloads.Marshak-like description (host arrays); mode: mean
    mode of the source update."""

    def __init__(self, prob, mode, *, polish=1, c_hat=None, dev="cuda", **source_kw):
        self.prob, self.mode, self.polish = prob, mode, polish
        self.c_hat = prob.c if c_hat is None else c_hat
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
        self.U = {k: t(prob.state[k]) for k in ("E_g", "F_g", "rho", "e_gas", "v")}
        self.Ut = {k: torch.empty_like(v) for k, v in self.U.items() if k != "rho"}
        self.tab = {"edges": t(prob.edges), "chi_lo": t(prob.chi_lo),
                    "alpha": t(prob.alpha_chi), "chi_mid": t(prob.chi_mid),
                    "El": t(prob.E_left), "Er": t(prob.E_right)}
        n = prob.n
        self.status = torch.zeros(n, dtype=torch.int32, device=dev)
        self.status_any = torch.zeros(n, dtype=torch.int32, device=dev)
        self.steps_done = 0
        self.source_kw = source_kw
        self._graph, self._graph_steps = None, 0

    # ------------------------------------------------------------------
    def _source(self, U, theta_dt):
        p = self.prob
        mgrhd.source_update(U["E_g"], U["F_g"], self.U["rho"], U["e_gas"], U["v"],
                            self.tab["edges"], self.tab["chi_lo"], mean_mode=self.mode,
                            alpha_chi=self.tab["alpha"], dt=theta_dt, c_hat=self.c_hat,
                            polish=self.polish, status=self.status, **p.consts(),
                            **self.source_kw)
        torch.bitwise_or(self.status_any, self.status, out=self.status_any)

    def _stage(self, out, U1, U0, a, b, dt_T):
        p = self.prob
        mgrhd.transport1d_stage(out, U1, U0, a=a, b=b, dx=p.dx, dt_T=dt_T, c=p.c,
                                c_hat=self.c_hat, rho=self.U["rho"], chi_mid=self.tab["chi_mid"],
                                E_left=self.tab["El"], E_right=self.tab["Er"])

    def step(self):
        """One IMEX step (eager, on the current stream)."""
        dt = self.prob.dt
        U, Ut = self.U, self.Ut
        self._stage(Ut, U, None, 0.0, 1.0, dt)          # U^t = U^n + dt T(U^n)
        self._source(Ut, dt)                            # -> U^(n+1/2) in Ut
        self._stage(U, Ut, U, 0.5, 0.5, 0.5 * dt)       # U <- (U^n + U^(n+1/2))/2 + dt/2 T
        self._source(U, 0.5 * dt)                       # -> U^(n+1) in U
        self.steps_done += 1

    def run(self, steps, graph_steps=500):
        """Advance ``steps`` steps: whole chunks of ``graph_steps`` replayed
        from one captured HIP graph, the rest eagerly."""
        if steps <= 0:
            return
        if self.steps_done == 0:
            self.step()                                  # warm the library's caches
            steps -= 1
        if graph_steps > 1 and steps >= graph_steps:
            if self._graph is None or self._graph_steps != graph_steps:
                s = torch.cuda.Stream()
                s.wait_stream(torch.cuda.current_stream())
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=s):
                    for _ in range(graph_steps):
                        self.step()
                self.steps_done -= graph_steps           # capture does not execute
                self._graph, self._graph_steps = g, graph_steps
            while steps >= graph_steps:
                self._graph.replay()
                self.steps_done += graph_steps
                steps -= graph_steps
        for _ in range(steps):
            self.step()

    # ------------------------------------------------------------------
    def state(self):
        return {k: self.U[k].cpu().numpy() for k in ("E_g", "F_g", "rho", "e_gas", "v")}

    def temperatures(self):
        """(T_gas [n], T_rad [n], T_rad,g [N_g, n]) with E = a T^4 (eq. Tgdef)."""
        st = self.state()
        p = self.prob
        T = (st["e_gas"] - 0.5 * st["rho"] * (st["v"] ** 2).sum(0)) / (st["rho"] * p.c_v)
        E = st["E_g"]
        return T, (E.sum(0) / p.a_rad) ** 0.25, (np.maximum(E, 0.0) / p.a_rad) ** 0.25


def band_temperatures(E_g, edges, bands, a_rad):
    """Radiation temperature of the energy summed over each band (band edges
    must be group edges): [len(bands)-1, n]."""
    out = []
    for lo, hi in zip(bands[:-1], bands[1:]):
        sel = (edges[:-1] >= lo * (1 - 1e-9)) & (edges[1:] <= hi * (1 + 1e-9))
        out.append((np.maximum(E_g[sel].sum(0), 0.0) / a_rad) ** 0.25)
    return np.array(out)


def steps_to(t_end, dt):
    return int(math.ceil(t_end / dt - 1e-9))
