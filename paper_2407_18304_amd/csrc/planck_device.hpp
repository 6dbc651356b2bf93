// planck_device.hpp -- device-side group Planck integrals and group-mean
// opacities for the source-update kernels (gfx950, FP64).
//
// Normalisation: B~_g = 4 pi B_g / c = a_R T^4 (15/pi^4) int_{x_g-}^{x_g+}
// t^3/(e^t - 1) dt with x = (h/k) nu / T, and the edge term of
// Delta_g(nu B_nu) (eq. G_model1b) is nu B~_nu = a_R T^4 (15/pi^4) x^4/(e^x - 1).
//
// Per edge x:
//   x <= 4  cumulative fraction P(x) = (15/pi^4) x^3 (1/3 - x/8 + y Ap(y)),
//           y = x^2, Ap a near-minimax polynomial (planck_poly.inc);
//   x >  4  e^x Q(x) = (15/pi^4) sum_{k=1..10} e^{-(k-1)x} (x^3/k + 3x^2/k^2
//           + 6x/k^3 + 6/k^4), the geometric series of 1/(e^t - 1), whose
//           11th term is below 2e-18 of the first for x > 4;
//   x <= 4  x/(e^x - 1) = 1 - x/2 + y Ep(y) (no exponential: an edge below the
//           Wien side costs two polynomials, the same instructions in every lane);
//   x >  4  x/(e^x - 1) from u = e^{-x}.
// A group whose lower edge is beyond x = 4 (the Wien side) is returned scaled
// by e^{x_lo}, so that nothing underflows for x up to ~1e300.
#pragma once
#include <hip/hip_runtime.h>

namespace mgrhd {

#include "planck_poly.inc"

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kC15 = 15.0 / (kPi * kPi * kPi * kPi);
constexpr int kTailTerms = 10;

// 1/k^j, the coefficient of u^{k-1} in S_j(u) of the Wien tail
__host__ __device__ constexpr double tail_coef(int k, int j) {
  double r = 1.0;
  for (int i = 0; i < j; ++i) r /= k;
  return r;
}

// fma(a, b, c) for a compile-time constant c.  On the device c is handed to
// v_fma_f64 as a scalar-register pair, built by two scalar moves that issue
// beside the vector stream; left to itself the compiler builds every
// polynomial coefficient with two vector moves, which cost as much issue time
// as the FMA they feed.
__host__ __device__ __forceinline__ double fma_c(double a, double b, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
#else
  return fma(a, b, c);
#endif
}

// 1/d for |d| in [2^-1000, 2^1000] (the callers' denominators are bounded
// away from 0 and overflow): the hardware estimate refined by two
// Newton-Raphson steps, within an ulp, without the scaling and fix-up steps
// of a general division.  The host build divides.
__host__ __device__ __forceinline__ double rcp_nr(double d) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(e, r, r);
  e = fma(-d, r, 1.0);
  return fma(e, r, r);
#else
  return 1.0 / d;
#endif
}

// sqrt(a) for a in [1, 4]: the hardware reciprocal square root refined by a
// Goldschmidt step and two Newton corrections, without range scaling.  The
// host build calls sqrt.
__host__ __device__ __forceinline__ double sqrt_1_4(double a) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double y = __builtin_amdgcn_rsq(a);
  double g = a * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double d = fma(-g, g, a);
  g = fma(d, h, g);
  d = fma(-g, g, a);
  return fma(d, h, g);
#else
  return sqrt(a);
#endif
}

// e^{-x} for x >= 0 (NaN passes through): Cody-Waite reduction
// x = n ln2 + r, |r| <= ln2/2, with ln2 split in a head and a tail so that r
// is exact to the last bits, then e^{-r} by its Taylor series to degree 13
// (remainder below 5e-18 relative) and the scale 2^{-n}.  Results below the
// normal range are rounded to subnormals by the scaling; x > 746 gives 0.
constexpr double kInvLn2 = 1.4426950408889634074;
constexpr double kLn2Hi = 0.69314718055994528623;      // ln 2 rounded to double
constexpr double kLn2Lo = 2.3190468138462996154e-17;   // ln 2 - kLn2Hi
constexpr int kExpDeg = 13;

__host__ __device__ constexpr double inv_factorial(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= i;
  return 1.0 / f;
}

__host__ __device__ __forceinline__ double exp_neg(double x) {
  const double xc = x > 746.0 ? 746.0 : x;
  const double n = rint(xc * kInvLn2);
  const double mr = fma(n, kLn2Lo, fma(n, kLn2Hi, -xc));   // -r
  double p = inv_factorial(kExpDeg);
#pragma unroll
  for (int k = kExpDeg - 1; k >= 0; --k) p = fma_c(p, mr, inv_factorial(k));
  return ldexp(p, -static_cast<int>(fmax(n, 0.0)));   // a NaN n converts as 0
}

// +inf test usable on host and device
__host__ __device__ __forceinline__ bool is_pinf(double x) { return x > 1.7976931348623157e308; }

// Per-edge data at temperature T.
struct Edge {
  double x;     // (h/k) nu / T
  double u;     // e^{-x} on the Wien side, else 1
  double val;   // P(x), or e^x Q(x) on the Wien side
  double eps;   // (15/pi^4) x^4/(e^x - 1), times e^x on the Wien side
  double eb;    // x/(e^x - 1) below the Wien side (1 at x = 0)
  bool wien;    // x > kPlanckSplit
  bool inf;     // x = +inf
};

// 1 - e^{-x} of an edge (the stimulated-emission factor of an opacity): below
// the Wien side x/(x + x/(e^x - 1)), with no exponential; beyond it 1 - u.
// Needs x > 0 below the Wien side.
__host__ __device__ __forceinline__ double stim_factor(const Edge& e) {
  return e.wien ? 1.0 - e.u : e.x / (e.x + e.eb);
}

__host__ __device__ __forceinline__ Edge planck_edge(double x) {
  Edge e;
  e.x = x;
  e.inf = is_pinf(x);
  e.wien = x > kPlanckSplit;
  static_assert(kEdgeSplit == kPlanckSplit, "one polynomial branch below the Wien side");
  double u = 1.0;
  if (e.wien) u = exp_neg(x);
  e.u = u;
  const double y = x * x;
  const double x3 = y * x;
  if (!e.wien) {
    double ap = planck_ap(kApDeg);
#pragma unroll
    for (int k = kApDeg - 1; k >= 0; --k) ap = fma_c(ap, y, planck_ap(k));
    e.val = kC15 * x3 * ((1.0 / 3.0 - 0.125 * x) + ap * y);
    double ep = planck_ep(kEpDeg);
#pragma unroll
    for (int k = kEpDeg - 1; k >= 0; --k) ep = fma_c(ep, y, planck_ep(k));
    e.eb = (1.0 - 0.5 * x) + ep * y;
    e.eps = kC15 * x3 * e.eb;
  } else if (e.inf) {
    e.val = 0.0;
    e.eps = 0.0;
    e.eb = 0.0;
  } else {
    e.eb = 0.0;
    // sum_k u^{k-1} (x^3/k + 3x^2/k^2 + 6x/k^3 + 6/k^4) as
    // x^3 S1(u) + 3x^2 S2(u) + 6x S3(u) + 6 S4(u), S_j(u) = sum_k u^{k-1}/k^j:
    // four Horner chains in u with constant coefficients 1/k^j
    double s1 = tail_coef(kTailTerms, 1), s2 = tail_coef(kTailTerms, 2);
    double s3 = tail_coef(kTailTerms, 3), s4 = tail_coef(kTailTerms, 4);
#pragma unroll
    for (int k = kTailTerms - 1; k >= 1; --k) {
      s1 = fma_c(s1, u, tail_coef(k, 1));
      s2 = fma_c(s2, u, tail_coef(k, 2));
      s3 = fma_c(s3, u, tail_coef(k, 3));
      s4 = fma_c(s4, u, tail_coef(k, 4));
    }
    e.val = kC15 * fma(x3, s1, fma(3.0 * y, s2, fma(6.0 * x, s3, 6.0 * s4)));
    e.eps = kC15 * x3 * x * rcp_nr(1.0 - u);   // 1 - u in [0.98, 1)
  }
  return e;
}

// The same edge data for small x (the lowest edge of a group structure):
// for x <= kLowEdge the polynomials truncated to degree kLowDeg in y = x^2
// reach the accuracy of the full ones (relative error below 2e-16), at a
// quarter of the work.  Falls back to planck_edge above kLowEdge.
constexpr double kLowEdge = 0.1;
constexpr int kLowDeg = 3;

__host__ __device__ __forceinline__ Edge planck_edge_low(double x) {
  if (!(x <= kLowEdge)) return planck_edge(x);
  Edge e;
  e.x = x;
  e.inf = false;
  e.wien = false;
  e.u = 1.0;
  const double y = x * x;
  const double x3 = y * x;
  double ap = planck_ap(kLowDeg), ep = planck_ep(kLowDeg);
#pragma unroll
  for (int k = kLowDeg - 1; k >= 0; --k) {
    ap = fma_c(ap, y, planck_ap(k));
    ep = fma_c(ep, y, planck_ep(k));
  }
  e.val = kC15 * x3 * ((1.0 / 3.0 - 0.125 * x) + ap * y);
  e.eb = (1.0 - 0.5 * x) + ep * y;
  e.eps = kC15 * x3 * e.eb;
  return e;
}

// Group data from its two edges:
//   b      group fraction, times e^{sigma}
//   elo    edge term at nu_g-, times e^{sigma}
//   ehi    edge term at nu_g+, times e^{sigma}
//   sigma  0, or x_lo when the lower edge is on the Wien side
//   scale  e^{-sigma}
struct GroupPlanck {
  double b, elo, ehi, sigma, scale;
};

__host__ __device__ __forceinline__ GroupPlanck group_planck(const Edge& lo, const Edge& hi) {
  GroupPlanck p;
  if (lo.wien) {
    // e^{-(x_hi - x_lo)}: the ratio of the edges' exponentials while e^{-x_lo}
    // is a normal number, else one more exponential
    double d;
    if (hi.inf)
      d = 0.0;
    else if (lo.x < 700.0)
      d = hi.u / lo.u;
    else
      d = exp_neg(hi.x - lo.x);
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
