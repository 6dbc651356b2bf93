"""The device-side Planck and group-mean routines, compiled for the host with
hipcc, pinned against mpmath (polylogarithms, Bernoulli numbers, quadrature).
CPU only: this checks the formulas and constants of the kernels' math; the
GPU parity tests check the device build."""
import ctypes as C
import os
import shutil
import subprocess

import mpmath as mp
import numpy as np
import pytest

import mp_ref

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hostbuild", "device_math_host.hip")


@pytest.fixture(scope="module")
def dm(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("dm") / "libdm.so")
    subprocess.run([hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
                    "-o", out, SRC], check=True, capture_output=True)
    L = C.CDLL(out)
    dp = C.POINTER(C.c_double)
    L.dm_edge.argtypes = [C.c_double, dp]
    L.dm_edge_low.argtypes = [C.c_double, dp]
    L.dm_group.argtypes = [C.c_double, C.c_double, dp]
    L.dm_mean_ratio.restype = C.c_double
    L.dm_mean_ratio.argtypes = [C.c_double, C.c_double, C.c_double]
    L.dm_exp_neg.restype = C.c_double
    L.dm_exp_neg.argtypes = [C.c_double]
    return L


def _call(fn, *args, n=5):
    out = np.zeros(n)
    fn(*args, out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


@pytest.mark.parametrize("x", [0.0, 1e-4, 0.3, 1.0, 1.9, 2.0, 2.01, 3.5, 3.99, 4.0, 4.01, 8.0,
                               30.0, 300.0, 5000.0])
def test_edge_values(dm, x):
    val, eps, u, wien = _call(dm.dm_edge, x, n=4)
    if x <= 4.0:
        assert wien == 0.0
        p = 1 - mp_ref.Q_polylog(x) if x > 0 else 0
        assert abs(val - p) <= 2e-15 * p + 1e-300
        # x/(e^x - 1) = (1 - x/2) + x^2 Ep(x^2) cancels near x = 4 (0.075 out
        # of terms of size 1): a few units of 1e-15 there
        assert abs(eps - mp_ref.edge_term(x)) <= 5e-15 * mp_ref.edge_term(x) + 1e-300
    else:
        qs = mp_ref.Q_polylog(x) * mp.exp(x)
        assert abs(val - qs) <= 2e-15 * qs
        es = mp_ref.edge_term(x) * mp.exp(x)
        assert abs(eps - es) <= 2e-15 * es


@pytest.mark.parametrize("xl,xh", [(1e-3, 0.03), (0.5, 1.5), (1.5, 2.5), (1.9, 2.1), (2.5, 6.0),
                                   (3.9, 4.1), (40.0, 60.0), (0.0, float("inf")),
                                   (3.0, float("inf")), (710.0, 720.0), (3.0e4, 3.1e4)])
def test_group_values(dm, xl, xh):
    b, elo, ehi, sig, scale = _call(dm.dm_group, xl, xh)
    if xl > 700:       # scaled: compare b e^{x_lo} with 40-digit polylogs
        ref = (mp_ref.Q_polylog(xl) - mp_ref.Q_polylog(xh)) * mp.exp(xl)
        assert sig == xl and abs(b - ref) <= 1e-14 * ref
        return
    ref = mp_ref.group_fraction(xl, xh)
    assert abs(b * scale - ref) <= 1e-13 * ref
    assert abs(elo * scale - mp_ref.edge_term(xl)) <= 2e-15 * mp_ref.edge_term(xl) + 1e-300
    assert abs(ehi * scale - mp_ref.edge_term(xh)) <= 2e-15 * mp_ref.edge_term(xh) + 1e-300


@pytest.mark.parametrize("ac,aq,L", [(-2.0, -1.0, 3.45), (1.7, -1.0, 0.86), (-3.2, 0.4, 0.216),
                                     (0.0, 0.7, 1.0), (2.0, -3.0, 1.0), (-2.0, 4000.0, 0.216)])
def test_mean_ratio(dm, ac, aq, L):
    num = mp.quad(lambda u: mp.exp((ac + aq + 1) * u), [0, L])
    den = mp.quad(lambda u: mp.exp((aq + 1) * u), [0, L])
    ref = num / den
    assert abs(dm.dm_mean_ratio(ac, aq, L) - ref) <= 1e-13 * ref


@pytest.mark.parametrize("x", [0.0, 1e-8, 1e-3, 0.01, 0.033, 0.0999, 0.1, 0.2, 3.0, 9.0])
def test_low_edge_matches_full_edge(dm, x):
    """The lowest-edge shortcut (truncated polynomials below x = 0.1, the full
    evaluation above) agrees with mpmath like the full edge."""
    val, eps, u, wien = _call(dm.dm_edge_low, x, n=4)
    full = _call(dm.dm_edge, x, n=4)
    if x > 0.1:
        assert (val, eps, u, wien) == tuple(full)
        return
    assert wien == 0.0 and u == 1.0
    p = 1 - mp_ref.Q_polylog(x) if x > 0 else 0
    assert abs(val - p) <= 1e-15 * p + 1e-300
    assert abs(eps - mp_ref.edge_term(x)) <= 1e-15 * mp_ref.edge_term(x) + 1e-300


def test_exp_neg(dm):
    """The kernels' own e^{-x} (Cody-Waite reduction and a degree-13 Taylor
    polynomial): within 2 units in the last place of mpmath's value over the
    normal range, within one subnormal step below it, 0 beyond x = 746, and
    NaN passed through."""
    rng = np.random.default_rng(5)
    xs = np.concatenate([[0.0, 1e-300, 1e-17, 0.5 * np.log(2), np.log(2), 4.0, 4.0000001,
                          700.0, 708.39, 708.4, 744.4, 745.1, 745.13],
                         rng.uniform(0, 1, 200), rng.uniform(4, 60, 400),
                         10.0 ** rng.uniform(-10, np.log10(745.0), 400)])
    ulp_rel = 2.0 ** -52
    for x in xs:
        got = dm.dm_exp_neg(float(x))
        ref = mp.exp(-mp.mpf(float(x)))
        if ref >= mp.mpf(2.0) ** -1022:
            assert abs(got - ref) <= 2 * ulp_rel * ref, x
        else:
            assert abs(got - ref) <= mp.mpf(2.0) ** -1074, x
    for x in (746.0, 800.0, 1e5, 1e300, float("inf")):
        assert dm.dm_exp_neg(x) == 0.0
    assert np.isnan(dm.dm_exp_neg(float("nan")))
