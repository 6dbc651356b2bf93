/*
 * planck.c -- oracle: group-integrated Planck quantities.  Test infrastructure
 * only (see mgrhd_oracle.h).
 *
 * Normalisation (reading of Sec. 2.1 and of the Doppler test's units): the
 * group Planck energy is B~_g = 4 pi B_g / c = a_R T^4 [P(x_g+) - P(x_g-)],
 * where P(x) = (15/pi^4) int_0^x t^3/(e^t - 1) dt, x = (h/k) nu / T, so that
 * the groups sum to a_R T^4 over all frequencies.  The edge quantity in
 * Delta_g(nu B_nu) (eq. G_model1b) is nu B~_nu = a_R T^4 (15/pi^4) x^4/(e^x-1).
 *
 * Two textbook series, each used where it converges fast:
 *   x <= 1 : t/(e^t-1) = sum_n B_n t^n / n!, integrated term by term,
 *            int_0^x t^3/(e^t-1) dt = sum_n B_n x^(n+3) / (n! (n+3));
 *   x >  1 : 1/(e^t-1) = sum_k e^{-kt}, integrated term by term,
 *            int_x^inf t^3/(e^t-1) dt = sum_k e^{-kx} (x^3/k + 3x^2/k^2 + 6x/k^3 + 6/k^4).
 * Parity: pinned against mpmath polylogarithms at 40 digits (tests).
 */
#include <math.h>
#include "mgrhd_oracle.h"

#define ORA_PI 3.14159265358979323846264338327950288
#define X_SPLIT 1.0

static double c15(void) { return 15.0 / (ORA_PI * ORA_PI * ORA_PI * ORA_PI); }

/* Bernoulli numbers B_2m, m = 1..15, as exact rationals (textbook values). */
static const double bern_num[16] = {0, 1.0, -1.0, 1.0, -1.0, 5.0, -691.0, 7.0,
                                    -3617.0, 43867.0, -174611.0, 854513.0,
                                    -236364091.0, 8553103.0, -23749461029.0,
                                    8615841276005.0};
static const double bern_den[16] = {1, 6.0, 30.0, 42.0, 30.0, 66.0, 2730.0, 6.0,
                                    510.0, 798.0, 330.0, 138.0, 2730.0, 6.0, 870.0,
                                    14322.0};

/* int_0^x t^3/(e^t-1) dt by the Bernoulli series, for 0 <= x <= 1 */
static double lower_integral(double x) {
  if (x == 0.0) return 0.0;
  double x3 = x * x * x;
  double sum = x3 / 3.0 - x3 * x / 8.0;   /* n = 0 and n = 1 (B_1 = -1/2) */
  double fact = 1.0;                      /* (2m)! */
  double xp = x3;                         /* x^(2m+3) */
  for (int m = 1; m <= 15; ++m) {
    fact *= (double)(2 * m - 1) * (double)(2 * m);
    xp *= x * x;
    double term = (bern_num[m] / bern_den[m]) / fact * xp / (double)(2 * m + 3);
    sum += term;
    if (fabs(term) < 1e-19 * fabs(sum)) break;
  }
  return sum;
}

/* e^{x} int_x^inf t^3/(e^t-1) dt by the geometric series, for x > 1 (finite) */
static double upper_integral_scaled(double x) {
  double sum = 0.0;
  for (int k = 1; k <= 400; ++k) {
    double kd = (double)k;
    double poly = x * x * x / kd + 3.0 * x * x / (kd * kd) + 6.0 * x / (kd * kd * kd) +
                  6.0 / (kd * kd * kd * kd);
    double term = exp(-(kd - 1.0) * x) * poly;
    sum += term;
    if (term < 1e-20 * sum) break;
  }
  return sum;
}

double ora_planck_P(double x) {
  if (!(x > 0.0)) return 0.0;
  if (isinf(x)) return 1.0;
  if (x <= X_SPLIT) return c15() * lower_integral(x);
  return 1.0 - ora_planck_Q(x);
}

double ora_planck_Q(double x) {
  if (!(x > 0.0)) return 1.0;
  if (isinf(x)) return 0.0;
  if (x <= X_SPLIT) return 1.0 - c15() * lower_integral(x);
  return c15() * exp(-x) * upper_integral_scaled(x);
}

double ora_planck_Qs(double x) {
  if (x <= X_SPLIT) return exp(x) * ora_planck_Q(x);
  return c15() * upper_integral_scaled(x);
}

/* nu B~_nu / (a T^4) at an edge, times e^{sigma}: (15/pi^4) x^4 e^{sigma}/(e^x - 1) */
static double edge_term(double x, double sigma) {
  if (x == 0.0 || isinf(x)) return 0.0;
  if (x <= X_SPLIT) return c15() * x * x * x * x * exp(sigma) / expm1(x);
  return c15() * exp(4.0 * log(x) - (x - sigma)) / (-expm1(-x));
}

void ora_group_planck(double xl, double xh, double out[4]) {
  double b, sigma;
  if (xl > X_SPLIT) {
    /* Wien side: scale by e^{x_lo} so that nothing underflows */
    sigma = xl;
    b = ora_planck_Qs(xl) - (isinf(xh) ? 0.0 : exp(-(xh - xl)) * ora_planck_Qs(xh));
  } else {
    sigma = 0.0;
    if (xh <= X_SPLIT)
      b = ora_planck_P(xh) - ora_planck_P(xl);
    else
      b = (1.0 - ora_planck_Q(xh)) - ora_planck_P(xl);
  }
  out[0] = b;
  out[1] = edge_term(xl, sigma);
  out[2] = edge_term(xh, sigma);
  out[3] = sigma;
}
