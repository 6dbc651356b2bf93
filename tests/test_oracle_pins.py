"""Pins of the FP64 CPU oracle against things other than itself: polylog and
quadrature values in mpmath, dense linear algebra, closed forms, invariants of
the method, brute-force roots of the defining equations and the paper's own
printed numbers.  CPU only."""
import math

import mpmath as mp
import numpy as np
import pytest

import mp_ref

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# --------------------------------------------------------------------------
# Planck fractions (Sec. 2.1 normalisation)
@pytest.mark.parametrize("x", [1e-6, 1e-3, 0.05, 0.3, 0.7, 0.999, 1.0, 1.001, 1.5, 2.7,
                               5.0, 11.0, 40.0, 150.0, 600.0, 700.0])
def test_planck_fraction_vs_polylog(ora, x):
    q = mp_ref.Q_polylog(x)
    p = 1 - q
    assert abs(ora.planck_Q(x) - q) <= 1e-15 * q
    assert abs(ora.planck_P(x) - p) <= 1e-14 * p
    assert abs(ora.planck_Qs(x) - q * mp.exp(x)) <= 1e-15 * q * mp.exp(x)


@pytest.mark.parametrize("x", [720.0, 5000.0, 3.2e4])
def test_planck_scaled_tail_vs_polylog(ora, x):
    """e^x Q(x) stays exact where e^{-x} itself is subnormal or zero."""
    qs = mp_ref.Q_polylog(x) * mp.exp(x)
    assert abs(ora.planck_Qs(x) - qs) <= 1e-15 * qs


def test_planck_limits(ora):
    assert ora.planck_P(0.0) == 0.0 and ora.planck_Q(0.0) == 1.0
    assert ora.planck_P(float("inf")) == 1.0 and ora.planck_Q(float("inf")) == 0.0
    # the fraction of the Planck spectrum below x = 1e-3 is (15/pi^4) x^3/3 + ...
    assert abs(ora.planck_P(1e-3) / (15 / math.pi ** 4 * 1e-9 / 3) - 1) < 1e-3
    x = 1e-3
    assert abs(ora.planck_P(x) / (15 / math.pi ** 4 * (x ** 3 / 3 - x ** 4 / 8 + x ** 5 / 60)) - 1) < 1e-12


@pytest.mark.parametrize("xl,xh", [(1e-5, 2e-5), (0.01, 0.5), (0.3, 2.0), (0.95, 1.05),
                                   (2.0, 4.0), (30.0, 45.0), (1e-3, float("inf")),
                                   (0.0, 0.02), (0.0, float("inf"))])
def test_group_planck_vs_quadrature(ora, xl, xh):
    b, elo, ehi, sig = ora.group_planck(xl, xh)
    ref = mp_ref.group_fraction(xl, xh)
    assert abs(b * math.exp(-sig) - ref) <= 1e-13 * ref  # narrow groups at x ~ 1 cancel
    assert abs(elo * math.exp(-sig) - mp_ref.edge_term(xl)) <= 2e-15 * (mp_ref.edge_term(xl) + 1e-300)
    assert abs(ehi * math.exp(-sig) - mp_ref.edge_term(xh)) <= 2e-15 * (mp_ref.edge_term(xh) + 1e-300)


@pytest.mark.parametrize("xl,xh", [(800.0, 900.0), (3.0e4, 3.3e4), (700.0, float("inf"))])
def test_group_planck_wien_tail_does_not_underflow(ora, xl, xh):
    """In the Wien tail the group quantities come back scaled by e^{x_lo}."""
    b, elo, ehi, sig = ora.group_planck(xl, xh)
    assert sig == xl
    qh = 0 if xh == float("inf") else mp_ref.Q_polylog(xh)
    ref = (mp_ref.Q_polylog(xl) - qh) * mp.exp(xl)     # 40-digit difference
    assert abs(b - ref) <= 1e-14 * ref
    assert abs(elo - mp_ref.edge_term(xl) * mp.exp(xl)) <= 1e-14 * elo


def test_dBdT_identity(ora):
    """dB~_g/dT = (4 B~_g - Delta_g(nu B~_nu))/T (used in the Jacobian, eq. linear)."""
    nl, nh = 0.7, 2.3
    f = lambda T: T ** 4 * mp_ref.group_fraction(nl / T, nh / T)
    for T in [0.3, 1.0, 4.0]:
        b, elo, ehi, sig = ora.group_planck(nl / T, nh / T)
        ident = (4 * b - (ehi - elo)) * math.exp(-sig) * T ** 3
        assert abs(ident - mp.diff(f, T)) < 1e-13 * abs(ident)


# --------------------------------------------------------------------------
# eq. chiQg
@pytest.mark.parametrize("ac,aq,L", [(-2.0, -1.0, 3.45), (1.7, -1.0, 0.86), (-3.2, 0.4, 0.216),
                                     (0.5, -1.5, 2.0), (2.0, -3.0, 1.0), (1.0, -2.0, 0.8)])
def test_mean_ratio_vs_quadrature(ora, ac, aq, L):
    ref = mp_ref.mean_quad(1, ac, aq, 1, mp.exp(L))
    assert abs(ora.mean_ratio(ac, aq, L) - ref) <= 1e-14 * ref


def test_mean_ratio_special_cases(ora):
    # alpha_chi = 0 is the PC case exactly
    for aq, L in [(-1.0, 1.0), (0.3, 2.0), (-40.0, 0.2)]:
        assert ora.mean_ratio(0.0, aq, L) == 1.0
    # alpha_Q = -1: [ln r]^-1 (r^a - 1)/a
    L, a = 1.3, 0.7
    assert abs(ora.mean_ratio(a, -1.0, L) - math.expm1(a * L) / a / L) < 1e-15
    # alpha_chi + alpha_Q = -1: numerator ln r
    aq = -2.5
    ac = -1.0 - aq
    ref = L / (math.expm1((aq + 1) * L) / (aq + 1))
    assert abs(ora.mean_ratio(ac, aq, L) - ref) < 1e-14 * ref
    # huge slopes (Wien tails of PPL-free) do not overflow and match quadrature
    # in log space
    for aq in [-3000.0, 4000.0]:
        ac, L = -2.0, 0.216
        r = ora.mean_ratio(ac, aq, L)
        assert np.isfinite(r)
        num = mp.quad(lambda u: mp.exp((ac + aq + 1) * u), [0, L])
        den = mp.quad(lambda u: mp.exp((aq + 1) * u), [0, L])
        assert abs(r - num / den) < 1e-12 * r


# --------------------------------------------------------------------------
# Appendix A slopes
def _logqbar(edges, Q):
    edges = np.asarray(edges)
    with np.errstate(divide="ignore"):
        return np.log(np.maximum(np.asarray(Q, float), 0.0)) - np.log(edges[1:] - edges[:-1])


def test_slopes_exact_for_powerlaw(ora):
    """A pure powerlaw nu^beta on log-spaced groups has interior slopes = beta."""
    edges = np.logspace(-2, 2, 9)
    for beta in [-2.3, 0.0, 1.7, -1.0]:
        Q = (edges[1:] ** (beta + 1) - edges[:-1] ** (beta + 1)) / (beta + 1) if beta != -1 \
            else np.log(edges[1:] / edges[:-1])
        al = ora.slopes(edges, _logqbar(edges, Q))
        assert al[0] == -1.0 and al[-1] == -1.0     # eq. minmod end groups
        assert np.allclose(al[1:-1], beta, rtol=0, atol=1e-12)
        # invariant to scaling Q
        assert np.allclose(ora.slopes(edges, _logqbar(edges, 37.0 * Q)), al, atol=1e-12)


def test_slopes_minmod_cases(ora):
    edges = np.array([1.0, 2.0, 4.0, 8.0, 16.0])
    d = math.log(2.0)
    # specific values Qbar chosen so that the edge slopes are known
    def run(lq):
        return ora.slopes(edges, np.array(lq))
    # slopes +1 then +3 -> minmod +1; -2 then -0.5 -> -0.5; +1 then -1 -> 0
    al = run([0.0, d, 4 * d, 2 * d])     # s = 1, 3, -2
    assert al[1] == pytest.approx(1.0, abs=1e-14) and al[2] == 0.0
    al = run([0.0, -2 * d, -2.5 * d, 0.0])  # s = -2, -0.5, 2.5
    assert al[1] == pytest.approx(-0.5, abs=1e-14) and al[2] == 0.0
    assert list(ora.slopes(edges[:3], np.array([0.0, 5.0]))) == [-1.0, -1.0]


def test_slopes_empty_group_is_a_limit(ora):
    """An empty group acts as Qbar -> 0+: the neighbour keeps its other slope."""
    edges = np.logspace(0, 4, 5)
    lq = np.array([1.0, 0.5, 0.2, -np.inf])
    al = ora.slopes(edges, lq)
    s_left = (0.2 - 0.5) / math.log(10)
    assert al[2] == pytest.approx(s_left, abs=1e-14)
    lq_small = np.array([1.0, 0.5, 0.2, -700.0])
    assert ora.slopes(edges, lq_small)[2] == pytest.approx(s_left, abs=1e-14)
    # two empty neighbours: undefined -> -1
    al = ora.slopes(edges, np.array([1.0, -np.inf, -np.inf, 0.0]))
    assert al[1] == -1.0 and al[2] == -1.0


# --------------------------------------------------------------------------
# eq. matrix
@pytest.mark.parametrize("ng", [1, 2, 5, 8])
def test_arrowhead_vs_dense_lu(ora, ng):
    rng = np.random.default_rng(ng)
    for cc in [1.0, 3.7]:
        Jg0 = rng.uniform(0, 5, ng)
        Jgg = -1.0 - 10.0 ** rng.uniform(-3, 3, ng)
        FG = rng.normal()
        FR = rng.normal(size=ng)
        J = np.zeros((ng + 1, ng + 1))
        J[0, 0] = 1.0
        J[0, 1:] = cc
        J[1:, 0] = Jg0
        J[np.arange(1, ng + 1), np.arange(1, ng + 1)] = Jgg
        ref = np.linalg.solve(J, -np.concatenate([[FG], FR]))
        dx = ora.arrowhead_solve(cc, Jg0, Jgg, FG, FR)
        assert np.allclose(dx, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
