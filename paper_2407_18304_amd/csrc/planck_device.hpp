// planck_device.hpp -- device-side group Planck integrals and group-mean
// opacities for the source-update kernels (gfx950, FP64).
//
// Normalisation: B~_g = 4 pi B_g / c = a_R T^4 (15/pi^4) int_{x_g-}^{x_g+}
// t^3/(e^t - 1) dt with x = (h/k) nu / T, and the edge term of
// Delta_g(nu B_nu) (eq. G_model1b) is nu B~_nu = a_R T^4 (15/pi^4) x^4/(e^x - 1).
//
// Edges with x <= kXSplit use the Taylor series of t/(e^t - 1) (Bernoulli
// numbers), integrated term by term for the cumulative fraction; the same
// series gives x/(e^x - 1) for the edge term, so no transcendental is needed
// there.  Edges with x > kXSplit use the geometric series
//   e^x int_x^inf t^3/(e^t-1) dt = sum_k e^{-(k-1)x} (x^3/k + 3x^2/k^2 + 6x/k^3 + 6/k^4).
// A group whose lower edge is in the Wien range is returned scaled by
// e^{x_lo}, so that nothing underflows for x up to ~1e300.
#pragma once
#include <hip/hip_runtime.h>

namespace mgrhd {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kC15 = 15.0 / (kPi * kPi * kPi * kPi);
constexpr double kXSplit = 2.0;
constexpr int kBernTerms = 19;   // |B_2m x^2m/(2m)!| < 3e-18 at x = 2 for m = 19
constexpr int kTailTerms = 20;   // e^{-2 k} < 1.4e-17 for k >= 19

// B_2m / (2m)!, m = 1..19 (Bernoulli numbers as exact rationals over (2m)!)
__host__ __device__ constexpr double bern_over_fact(int m) {
  switch (m) {
    case 1: return (1.0 / 6.0) / 2.0;
    case 2: return (-1.0 / 30.0) / 24.0;
    case 3: return (1.0 / 42.0) / 720.0;
    case 4: return (-1.0 / 30.0) / 40320.0;
    case 5: return (5.0 / 66.0) / 3628800.0;
    case 6: return (-691.0 / 2730.0) / 479001600.0;
    case 7: return (7.0 / 6.0) / 87178291200.0;
    case 8: return (-3617.0 / 510.0) / 20922789888000.0;
    case 9: return (43867.0 / 798.0) / 6402373705728000.0;
    case 10: return (-174611.0 / 330.0) / 2432902008176640000.0;
    case 11: return (854513.0 / 138.0) / 1124000727777607680000.0;
    case 12: return (-236364091.0 / 2730.0) / 620448401733239439360000.0;
    case 13: return (8553103.0 / 6.0) / 403291461126605635584000000.0;
    case 14: return (-23749461029.0 / 870.0) / 304888344611713860501504000000.0;
    case 15: return (8615841276005.0 / 14322.0) / 265252859812191058636308480000000.0;
    case 16: return (-7709321041217.0 / 510.0) / 263130836933693530167218012160000000.0;
    case 17: return (2577687858367.0 / 6.0) / 295232799039604140847618609643520000000.0;
    case 18:
      return (-26315271553053477373.0 / 1919190.0) / 371993326789901217467999448150835200000000.0;
    case 19:
      return (2929993913841559.0 / 6.0) / 523022617466601111760007224100074291200000000.0;
    default: return 0.0;
  }
}

// +inf test usable on host and device
__host__ __device__ __forceinline__ bool is_pinf(double x) { return x > 1.7976931348623157e308; }

// Per-edge data at temperature T.
struct Edge {
  double x;     // (h/k) nu / T
  double u;     // e^{-x}            (Wien range only)
  double val;   // P(x), or e^x Q(x) in the Wien range
  double eps;   // (15/pi^4) x^4/(e^x - 1), times e^x in the Wien range
  bool wien;    // x > kXSplit
  bool inf;     // x = +inf
};

__host__ __device__ __forceinline__ Edge planck_edge(double x) {
  Edge e;
  e.x = x;
  e.inf = is_pinf(x);
  e.wien = x > kXSplit;
  if (!e.wien) {
    // x^3 (1/3 - x/8 + sum b_m x^2m/(2m+3)) and x^3 (1 - x/2 + sum b_m x^2m)
    const double y = x * x;
    double sp = 0.0, se = 0.0;
#pragma unroll
    for (int m = kBernTerms; m >= 1; --m) {
      sp = fma(sp, y, bern_over_fact(m) / (2.0 * m + 3.0));
      se = fma(se, y, bern_over_fact(m));
    }
    const double x3 = x * x * x;
    e.val = kC15 * x3 * ((1.0 / 3.0 - 0.125 * x) + sp * y);
    e.eps = kC15 * x3 * ((1.0 - 0.5 * x) + se * y);
    e.u = 1.0;
  } else if (e.inf) {
    e.u = 0.0;
    e.val = 0.0;
    e.eps = 0.0;
  } else {
    const double u = exp(-x);
    const double x1 = 6.0 * x, x2 = 3.0 * x * x, x3 = x * x * x;
    double acc = ((x3 + x2) + x1) + 6.0;
    double t = 1.0;
#pragma unroll
    for (int k = 2; k <= kTailTerms; ++k) {
      t *= u;
      if (t < 1e-17) break;
      const double rk = 1.0 / k;
      acc = fma(t, fma(x3, rk, fma(x2, rk * rk, fma(x1, rk * rk * rk, 6.0 * rk * rk * rk * rk))),
                acc);
    }
    e.u = u;
    e.val = kC15 * acc;
    e.eps = kC15 * x3 * x / (1.0 - u);
  }
  return e;
}

// Group data from its two edges:
//   b      group fraction, times e^{sigma}
//   elo    edge term at nu_g-, times e^{sigma}
//   ehi    edge term at nu_g+, times e^{sigma}
//   sigma  0, or x_lo when the lower edge is in the Wien range
//   scale  e^{-sigma}
struct GroupPlanck {
  double b, elo, ehi, sigma, scale;
};

__host__ __device__ __forceinline__ GroupPlanck group_planck(const Edge& lo, const Edge& hi) {
  GroupPlanck p;
  if (lo.wien) {
    const double d = hi.inf ? 0.0 : exp(lo.x - hi.x);
    p.b = lo.val - d * hi.val;
    p.elo = lo.eps;
    p.ehi = d * hi.eps;
    p.sigma = lo.x;
    p.scale = lo.u;
  } else {
    p.elo = lo.eps;
    if (!hi.wien) {
      p.b = hi.val - lo.val;
      p.ehi = hi.eps;
    } else {
      p.b = (1.0 - hi.u * hi.val) - lo.val;
      p.ehi = hi.u * hi.eps;
    }
    p.sigma = 0.0;
    p.scale = 1.0;
  }
  return p;
}

// (e^{aL} - 1)/a (L when a = 0) times e^{-m}, m = max(aL, 0): the bracket of
// eq. chiQg without overflow.
__host__ __device__ __forceinline__ double phi_scaled(double a, double L, double& m) {
  if (a == 0.0) {
    m = 0.0;
    return L;
  }
  const double y = a * L;
  if (y > 0.0) {
    m = y;
    return -expm1(-y) / a;
  }
  m = 0.0;
  return expm1(y) / a;
}

// chi_0Q,g / chi_0,g- of eq. chiQg for opacity index ac and spectral index aq
__host__ __device__ __forceinline__ double mean_ratio(double ac, double aq, double L) {
  double m1, m2;
  const double num = phi_scaled(ac + aq + 1.0, L, m1);
  const double den = phi_scaled(aq + 1.0, L, m2);
  const double r = num / den;
  return (m1 == m2) ? r : r * exp(m1 - m2);
}

__host__ __device__ __forceinline__ double minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return fmin(a, b);
  if (a < 0.0 && b < 0.0) return fmax(a, b);
  return 0.0;
}

}  // namespace mgrhd
