/*
 * opacity.c -- oracle: group-mean opacities (eq. chiQg), the Appendix A slope
 * reconstruction, and the arrowhead elimination of eq. matrix.  Test
 * infrastructure only (see mgrhd_oracle.h).
 */
#include <math.h>
#include "mgrhd_oracle.h"

/* phi(a, L) = (e^{aL} - 1)/a, which is the bracket of eq. chiQg with
 * r^a = e^{aL}; it is L when a = 0 (the ln r special case of Sec. 2.2.2).
 * Returned as phi * e^{-m} with m = max(aL, 0) so that it never overflows. */
static double phi_scaled(double a, double L, double* m) {
  if (a == 0.0) {
    *m = 0.0;
    return L;
  }
  double y = a * L;
  if (y > 0.0) {
    *m = y;
    return -expm1(-y) / a;
  }
  *m = 0.0;
  return expm1(y) / a;
}

/* eq. chiQg divided by chi_{0,g-}:
 *   [ (r^{aQ+1} - 1)/(aQ+1) ]^{-1} [ (r^{achi+aQ+1} - 1)/(achi+aQ+1) ] */
double ora_mean_ratio(double alpha_chi, double alpha_Q, double L) {
  double m_num, m_den;
  double num = phi_scaled(alpha_chi + alpha_Q + 1.0, L, &m_num);
  double den = phi_scaled(alpha_Q + 1.0, L, &m_den);
  return num / den * exp(m_num - m_den);
}

static double minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

/* Appendix A, eqs. sg and minmod.  logqbar[g] = ln(Q_g / (nu_g+ - nu_g-)).
 * READING: an empty group (Q_g <= 0) enters as the limit Q_g -> 0+, i.e.
 * logqbar = -inf, so that the edge slope next to it is -inf or +inf and
 * minmod keeps the slope on the other side (or 0); the slope stays continuous
 * as Q_g crosses zero.  Only a slope between two empty groups is undefined;
 * it leaves the groups next to it at -1, as are the two end groups. */
void ora_slopes(int32_t ng, const double* nu, const double* logqbar, double* alpha) {
  for (int32_t g = 0; g < ng; ++g) alpha[g] = -1.0;
  if (ng <= 2) return;
  for (int32_t g = 1; g < ng - 1; ++g) {
    double lc_m = 0.5 * (log(nu[g - 1]) + log(nu[g]));     /* ln nubar_{g-1} */
    double lc_0 = 0.5 * (log(nu[g]) + log(nu[g + 1]));     /* ln nubar_g     */
    double lc_p = 0.5 * (log(nu[g + 1]) + log(nu[g + 2])); /* ln nubar_{g+1} */
    double s_left = (logqbar[g] - logqbar[g - 1]) / (lc_0 - lc_m);
    double s_right = (logqbar[g + 1] - logqbar[g]) / (lc_p - lc_0);
    if (isnan(s_left) || isnan(s_right)) continue;
    double a = minmod(s_left, s_right);
    if (isfinite(a)) alpha[g] = a;
  }
}

/* eq. matrix: row 0 is (1, c/c_hat, ..., c/c_hat), row g is (Jg0, 0.., Jgg, ..0).
 * Eliminating the first row with rows 1..N_g gives dx_0; each dx_g follows by
 * back-substitution (Sec. 3). */
void ora_arrowhead_solve(int32_t ng, double c_over_chat, const double* Jg0,
                         const double* Jgg, double FG, const double* FR, double* dx) {
  double num = -FG, den = 1.0;
  for (int32_t g = 0; g < ng; ++g) {
    num += c_over_chat * FR[g] / Jgg[g];
    den -= c_over_chat * Jg0[g] / Jgg[g];
  }
  dx[0] = num / den;
  for (int32_t g = 0; g < ng; ++g) dx[g + 1] = (-FR[g] - Jg0[g] * dx[0]) / Jgg[g];
}
