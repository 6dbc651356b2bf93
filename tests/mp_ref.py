"""Independent arbitrary-precision statements of the paper's equations, used
only to pin the oracle.  Everything here is computed by quadrature or closed
form in mpmath, never by the series or closed forms the oracle uses.

Equations (He, Wibking & Krumholz 2024):
  group Planck energy     B~_g = a T^4 (15/pi^4) int_{x-}^{x+} t^3/(e^t-1) dt
  edge term               nu B~_nu = a T^4 (15/pi^4) x^4/(e^x-1)
  mean opacity eq. chiQ   chi_Q = int chi0(nu) Q_nu dnu / int Q_nu dnu,
                          with chi0 = chi_- (nu/nu_-)^a_chi, Q_nu ~ nu^a_Q
  flux mean eq. chiDiff
  slopes App. A eqs. sg, minmod
  residuals eq. eupdate with eq. G0_3 (via eq. Rnew), eq. numF1
"""
import mpmath as mp

mp.mp.dps = 40
C15 = 15 / mp.pi ** 4


def planck_integrand(t):
    if t == 0:
        return mp.mpf(0)
    return t ** 3 / mp.expm1(t)


def Q_polylog(x):
    """Q(x) = (15/pi^4) int_x^inf t^3/(e^t-1) dt = polylog form (Li_1 = -log1p(-e))."""
    x = mp.mpf(x)
    e = mp.exp(-x)
    return C15 * (x ** 3 * (-mp.log1p(-e)) + 3 * x ** 2 * mp.polylog(2, e) +
                  6 * x * mp.polylog(3, e) + 6 * mp.polylog(4, e))


def group_fraction(x_lo, x_hi):
    """(15/pi^4) int_{x_lo}^{x_hi} t^3/(e^t-1) dt by quadrature."""
    x_lo, x_hi = mp.mpf(x_lo), (mp.inf if x_hi == float("inf") else mp.mpf(x_hi))
    pts = [x_lo] + [p for p in (1, 3, 10, 30) if x_lo < p < x_hi] + [x_hi]
    return C15 * mp.quad(planck_integrand, pts)


def edge_term(x):
    x = mp.mpf(x)
    if x == 0 or mp.isinf(x):
        return mp.mpf(0)
    return C15 * x ** 4 / mp.expm1(x)


def mean_quad(chi_lo, a_chi, a_q, nu_lo, nu_hi):
    """eq. chiQ by quadrature of the powerlaw ansatz (Sec. 2.2.2)."""
    nu_lo, nu_hi = mp.mpf(nu_lo), mp.mpf(nu_hi)
    q = lambda nu: (nu / nu_lo) ** a_q
    chi = lambda nu: chi_lo * (nu / nu_lo) ** a_chi
    return mp.quad(lambda nu: chi(nu) * q(nu), [nu_lo, nu_hi]) / mp.quad(q, [nu_lo, nu_hi])


def minmod(a, b):
    if a > 0 and b > 0:
        return min(a, b)
    if a < 0 and b < 0:
        return max(a, b)
    return mp.mpf(0)


def slopes_app_a(edges, Q):
    """App. A: alpha_g from group integrals Q_g (all > 0 here)."""
    ng = len(Q)
    al = [mp.mpf(-1)] * ng
    qbar = [mp.mpf(Q[g]) / (mp.mpf(edges[g + 1]) - mp.mpf(edges[g])) for g in range(ng)]
    nubar = [mp.sqrt(mp.mpf(edges[g + 1]) * mp.mpf(edges[g])) for g in range(ng)]
    s = [mp.log(qbar[g + 1] / qbar[g]) / mp.log(nubar[g + 1] / nubar[g]) for g in range(ng - 1)]
    for g in range(1, ng - 1):
        al[g] = minmod(s[g - 1], s[g])
    return al


class Material:
    """Group data at temperature T for one cell (mode 0 PC, 1 PPL-fixed, 2 PPL-free)."""

    def __init__(self, T, edges, chi_lo_cell, a_chi, mode, a_rad, hk=1, E=None):
        T = mp.mpf(T)
        ng = len(chi_lo_cell)
        aT4 = a_rad * T ** 4
        x = [hk * mp.mpf(e) / T for e in edges]
        self.B = [aT4 * group_fraction(x[g], x[g + 1]) for g in range(ng)]
        self.nuB = [aT4 * edge_term(xe) for xe in x]
        self.dB = [(4 * self.B[g] - (self.nuB[g + 1] - self.nuB[g])) / T for g in range(ng)]
        if mode == 0:
            a_chi = [0] * ng
            self.chiB = self.chiE = self.chiF = [mp.mpf(c) for c in chi_lo_cell]
            self.DchiB = [chi_lo_cell[g] * (self.nuB[g + 1] - self.nuB[g]) for g in range(ng)]
            self.a_chi = a_chi
            return
        if mode == 1:
            aB = aE = [-1] * ng
        else:
            aB = slopes_app_a(edges, self.B)
            aE = slopes_app_a(edges, E)
        self.a_chi = a_chi
        self.chiB = [mean_quad(chi_lo_cell[g], a_chi[g], aB[g], edges[g], edges[g + 1])
                     for g in range(ng)]
        self.chiE = [mean_quad(chi_lo_cell[g], a_chi[g], aE[g], edges[g], edges[g + 1])
                     for g in range(ng)]
        self.DchiB, self.chiF = [], []
        for g in range(ng):
            r = mp.mpf(edges[g + 1]) / mp.mpf(edges[g])
            dchib = chi_lo_cell[g] * (r ** a_chi[g] * self.nuB[g + 1] - self.nuB[g])
            self.DchiB.append(dchib)
            num = (self.chiB[g] + self.chiE[g] / 3) * self.B[g] + \
                (a_chi[g] * self.chiE[g] * self.B[g] - dchib) / 3
            den = mp.mpf(4) / 3 * self.B[g] - (self.nuB[g + 1] - self.nuB[g]) / 3
            self.chiF.append(num / den)


def m1_pressure_dot_v(E, F, v, c):
    """Levermore (1984) closure, P . v."""
    fm = mp.sqrt(sum(f * f for f in F))
    if fm == 0:
        return [E * vi / 3 for vi in v]
    f = min(fm / (c * E), mp.mpf(1))
    chi = (3 + 4 * f * f) / (5 + 2 * mp.sqrt(4 - 3 * f * f))
    n = [fi / fm for fi in F]
    nv = sum(ni * vi for ni, vi in zip(n, v))
    return [E * ((1 - chi) / 2 * v[d] + (3 * chi - 1) / 2 * n[d] * nv) for d in range(3)]
