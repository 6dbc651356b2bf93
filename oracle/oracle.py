"""ctypes binding of the plain FP64 CPU oracle (``liboracle_mgrhd.so``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product library never loads it.

The oracle follows He, Wibking & Krumholz (2024), Sec. 2.2 (group-mean
opacities, eqs. chiQg and chiDiff), Sec. 3 (Newton system eqs. FGFR, Rnew,
linear, matrix; energy, flux eq. numF1 and momentum updates) and Appendix A
(slope reconstruction, eqs. sg and minmod).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle_mgrhd.so")
SOURCES = ["planck.c", "opacity.c", "solve.c"]

MEAN_PC, MEAN_PPL_FIXED, MEAN_PPL_FREE = 0, 1, 2
CLOSURE_M1, CLOSURE_EDDINGTON = 0, 1
ST_OK, ST_NEWTON_MAXIT, ST_OUTER_MAXIT, ST_FALLBACK, ST_INVALID, ST_NONFINITE = (
    0, 1, 2, 4, 8, 16)


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc: -O2, strict IEEE (no fast-math)."""
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    cmd = ["gcc", "-O2", "-std=c11", "-D_POSIX_C_SOURCE=200809L", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra", "-o", LIB + ".tmp",
           *srcs, "-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class OraOpacity(C.Structure):
    _fields_ = [("n_groups", C.c_int32), ("mean_mode", C.c_int32),
                ("chi_lo", C.POINTER(C.c_double)), ("alpha_chi", C.POINTER(C.c_double)),
                ("chi_hi", C.POINTER(C.c_double)), ("kappa_scale", C.POINTER(C.c_double)),
                ("t_exp", C.c_double), ("t_ref", C.c_double), ("stim", C.c_int32),
                ("reserved", C.c_int32)]


class OraOptions(C.Structure):
    _fields_ = [("c", C.c_double), ("a_rad", C.c_double), ("h_over_k", C.c_double),
                ("c_v", C.c_double), ("eps_newton", C.c_double), ("eps_outer", C.c_double),
                ("max_newton", C.c_int32), ("max_outer", C.c_int32),
                ("closure", C.c_int32), ("polish", C.c_int32),
                ("S_g", C.POINTER(C.c_double)), ("guess", C.POINTER(C.c_double)),
                ("iters", C.POINTER(C.c_int32)), ("outer", C.POINTER(C.c_int32)),
                ("status", C.POINTER(C.c_int32)), ("guess_kind", C.c_int32),
                ("reserved", C.c_int32), ("trace", C.POINTER(C.c_int32)),
                ("force", C.POINTER(C.c_int32))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        L.ora_planck_P.restype = C.c_double
        L.ora_planck_P.argtypes = [C.c_double]
        L.ora_planck_Q.restype = C.c_double
        L.ora_planck_Q.argtypes = [C.c_double]
        L.ora_planck_Qs.restype = C.c_double
        L.ora_planck_Qs.argtypes = [C.c_double]
        L.ora_group_planck.restype = None
        L.ora_group_planck.argtypes = [C.c_double, C.c_double, dp]
        L.ora_mean_ratio.restype = C.c_double
        L.ora_mean_ratio.argtypes = [C.c_double, C.c_double, C.c_double]
        L.ora_slopes.restype = None
        L.ora_slopes.argtypes = [C.c_int32, dp, dp, dp]
        L.ora_arrowhead_solve.restype = None
        L.ora_arrowhead_solve.argtypes = [C.c_int32, C.c_double, dp, dp, C.c_double, dp, dp]
        L.ora_default_options.restype = None
        L.ora_default_options.argtypes = [C.POINTER(OraOptions)]
        for name in ("ora_source_update", "mgrhd_oracle_source_update"):
            f = getattr(L, name)
            f.restype = C.c_int
            f.argtypes = [dp, dp, dp, dp, dp, C.c_int64, dp, C.POINTER(OraOpacity), C.c_double,
                          C.c_double, C.POINTER(OraOptions), C.c_int32]
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return C.POINTER(C.c_double)()
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    if a is None:
        return C.POINTER(C.c_int32)()
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def planck_P(x: float) -> float:
    return lib().ora_planck_P(float(x))


def planck_Q(x: float) -> float:
    return lib().ora_planck_Q(float(x))


def planck_Qs(x: float) -> float:
    return lib().ora_planck_Qs(float(x))


def group_planck(x_lo: float, x_hi: float):
    """(b, e_lo, e_hi, sigma): scaled group integral and edge terms."""
    out = np.zeros(4)
    lib().ora_group_planck(float(x_lo), float(x_hi), _dp(out))
    return tuple(out)


def mean_ratio(alpha_chi: float, alpha_q: float, L: float) -> float:
    return lib().ora_mean_ratio(float(alpha_chi), float(alpha_q), float(L))


def slopes(nu, logqbar):
    nu = np.ascontiguousarray(nu, dtype=np.float64)
    lq = np.ascontiguousarray(logqbar, dtype=np.float64)
    out = np.zeros(len(lq))
    lib().ora_slopes(len(lq), _dp(nu), _dp(lq), _dp(out))
    return out


def arrowhead_solve(c_over_chat, Jg0, Jgg, FG, FR):
    Jg0 = np.ascontiguousarray(Jg0, dtype=np.float64)
    Jgg = np.ascontiguousarray(Jgg, dtype=np.float64)
    FR = np.ascontiguousarray(FR, dtype=np.float64)
    dx = np.zeros(len(FR) + 1)
    lib().ora_arrowhead_solve(len(FR), float(c_over_chat), _dp(Jg0), _dp(Jgg), float(FG),
                              _dp(FR), _dp(dx))
    return dx


def source_update(state: dict, edges, chi_lo, *, mean_mode=MEAN_PPL_FIXED, alpha_chi=None,
                  chi_hi=None, kappa_scale=None, dt=1.0, c_hat=1.0, c=1.0, a_rad=1.0,
                  h_over_k=1.0, c_v=1.5, eps_newton=1e-11, eps_outer=1e-13,
                  max_newton=100, max_outer=20, closure=CLOSURE_M1, polish=0, S_g=None,
                  guess=None, guess_kind=0, t_exp=0.0, t_ref=1.0, stim=0, n_threads=0,
                  trace=None, force=None):
    """Run the oracle on a copy of ``state`` (dict of E_g [N_g,n], F_g [3,N_g,n],
    rho [n], e_gas [n], v [3,n]).  Returns (new_state, iters, outer, status).
    t_exp, t_ref, stim: temperature dependence of the opacity,
    chi_0 x (T/t_ref)^t_exp [1 - exp(-h nu / k T)]^stim.
    trace: an int32 array [max_outer, n] that receives the cumulative Newton
    steps at the end of every inner pass (-1 for passes not run); force: a
    schedule in the same layout to replay (see ora_options.force)."""
    E = np.array(state["E_g"], dtype=np.float64, order="C", copy=True)
    F = np.array(state["F_g"], dtype=np.float64, order="C", copy=True)
    rho = np.ascontiguousarray(state["rho"], dtype=np.float64)
    eg = np.array(state["e_gas"], dtype=np.float64, order="C", copy=True)
    v = np.array(state["v"], dtype=np.float64, order="C", copy=True)
    ng, n = E.shape
    assert F.shape == (3, ng, n) and v.shape == (3, n) and rho.shape == (n,)
    edges = np.ascontiguousarray(edges, dtype=np.float64)
    chi_lo = np.ascontiguousarray(chi_lo, dtype=np.float64)
    alpha_chi = None if alpha_chi is None else np.ascontiguousarray(alpha_chi, np.float64)
    chi_hi = None if chi_hi is None else np.ascontiguousarray(chi_hi, np.float64)
    kappa_scale = None if kappa_scale is None else np.ascontiguousarray(kappa_scale, np.float64)
    S_g = None if S_g is None else np.ascontiguousarray(S_g, np.float64)
    guess = None if guess is None else np.ascontiguousarray(guess, np.float64)
    if guess is not None and guess_kind == 1 and guess.ndim == 1:
        guess = guess[None, :]                    # temperature-only: row 0 alone
    iters = np.zeros(n, np.int32)
    outer = np.zeros(n, np.int32)
    status = np.zeros(n, np.int32)
    op = OraOpacity(ng, mean_mode, _dp(chi_lo), _dp(alpha_chi), _dp(chi_hi), _dp(kappa_scale),
                    float(t_exp), float(t_ref), int(stim), 0)
    opt = OraOptions()
    lib().ora_default_options(C.byref(opt))
    opt.c, opt.a_rad, opt.h_over_k, opt.c_v = c, a_rad, h_over_k, c_v
    opt.eps_newton, opt.eps_outer = eps_newton, eps_outer
    opt.max_newton, opt.max_outer, opt.closure, opt.polish = max_newton, max_outer, closure, polish
    opt.S_g, opt.guess = _dp(S_g), _dp(guess)
    opt.guess_kind = guess_kind
    opt.iters, opt.outer, opt.status = _ip(iters), _ip(outer), _ip(status)
    if trace is not None:
        assert trace.dtype == np.int32 and trace.shape == (max_outer, n) and trace.flags.c_contiguous
    if force is not None:
        force = np.ascontiguousarray(force, dtype=np.int32)
        assert force.shape == (max_outer, n)
    opt.trace, opt.force = _ip(trace), _ip(force)
    rc = lib().ora_source_update(_dp(E), _dp(F), _dp(rho), _dp(eg), _dp(v), n, _dp(edges),
                                 C.byref(op), float(dt), float(c_hat), C.byref(opt),
                                 int(n_threads))
    if rc != 0:
        raise ValueError(f"oracle rejected the arguments (code {rc})")
    return ({"E_g": E, "F_g": F, "rho": rho, "e_gas": eg, "v": v}, iters, outer, status)
