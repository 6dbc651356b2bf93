/* Runs the oracle's entry points on small synthetic cells so that a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer can check them:
 * every mean mode and closure, sources, both warm-start kinds and a failing
 * guess, temperature-dependent opacities, a recorded and a replayed
 * schedule, invalid cells, argument errors and the building blocks.  Exits
 * non-zero when a call returns an unexpected code. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mgrhd_oracle.h"

static unsigned long long s = 88172645463325252ull;
static double urand(void) {
  s ^= s << 13;
  s ^= s >> 7;
  s ^= s << 17;
  return (double)(s >> 11) * 0x1p-53;
}

#define NG 7
#define N 40

int main(void) {
  double edges[NG + 1], chi[NG], ach[NG], chh[NG];
  for (int g = 0; g <= NG; ++g) edges[g] = pow(10.0, -2.0 + 4.0 * g / NG);
  for (int g = 0; g < NG; ++g) {
    chi[g] = pow(10.0, 2.0 * urand() - 1.0);
    ach[g] = -3.0 + 4.0 * urand();
    chh[g] = chi[g] * pow(edges[g + 1] / edges[g], ach[g]);
  }
  double E[NG * N], F[3 * NG * N], rho[N], eg[N], v[3 * N], kap[N], S[NG * N];
  double guess[(NG + 1) * N];
  int32_t it[N], ou[N], st[N], tr[20 * N], tr2[20 * N];
  int bad = 0;
  for (int mode = 0; mode < 3; ++mode)
    for (int clo = 0; clo < 2; ++clo)
      for (int variant = 0; variant < 6; ++variant) {
        for (int i = 0; i < N; ++i) {
          double T = 0.3 + 2.0 * urand();
          rho[i] = 0.5 + urand();
          kap[i] = pow(10.0, 3.0 * urand() - 1.0);
          for (int d = 0; d < 3; ++d) v[d * N + i] = 1e-3 * (2.0 * urand() - 1.0);
          double ke = 0.5 * rho[i] * (v[i] * v[i] + v[N + i] * v[N + i] + v[2 * N + i] * v[2 * N + i]);
          eg[i] = rho[i] * 1.5 * T + ke;
          for (int g = 0; g < NG; ++g) {
            E[g * N + i] = 0.1 * urand() * T * T * T * T;
            S[g * N + i] = 0.01 * urand() * E[g * N + i];
            for (int d = 0; d < 3; ++d)
              F[(d * NG + g) * N + i] = 0.3 * E[g * N + i] * (2.0 * urand() - 1.0);
          }
          guess[i] = variant == 4 ? -1.0 : eg[i] * (1.0 + 1e-3 * urand());
          for (int g = 0; g < NG; ++g) guess[(g + 1) * N + i] = 1e-3 * E[g * N + i];
        }
        if (variant == 5) eg[3] = -1.0; /* an invalid cell */
        ora_opacity op = {NG, mode, chi, ach, NULL, kap, 0.0, 1.0, 0, 0};
        if (variant == 2) {
          op.alpha_chi = NULL;
          op.chi_hi = chh;
          op.t_exp = -0.5;
          op.stim = 1;
        }
        ora_options o;
        ora_default_options(&o);
        o.c = 100.0;
        o.closure = clo;
        o.polish = variant & 1;
        o.iters = it;
        o.outer = ou;
        o.status = st;
        o.trace = tr;
        if (variant == 1) o.S_g = S;
        if (variant >= 3) {
          o.guess = guess;
          o.guess_kind = variant == 3 ? 0 : 1;
        }
        double E2[NG * N], F2[3 * NG * N], eg2[N], v2[3 * N];
        memcpy(E2, E, sizeof E);
        memcpy(F2, F, sizeof F);
        memcpy(eg2, eg, sizeof eg);
        memcpy(v2, v, sizeof v);
        int rc = ora_source_update(E, F, rho, eg, v, N, edges, &op, 0.01, 100.0, &o, 2);
        if (rc != 0) bad |= 1;
        /* replay the recorded schedule on the original inputs */
        o.trace = tr2;
        o.force = tr;
        rc = ora_source_update(E2, F2, rho, eg2, v2, N, edges, &op, 0.01, 100.0, &o, 1);
        if (rc != 0) bad |= 2;
        if (variant != 4 && memcmp(E, E2, sizeof E) != 0) bad |= 4;
      }
  /* argument errors */
  ora_opacity op = {NG, 1, chi, ach, NULL, NULL, 0.0, 1.0, 0, 0};
  if (ora_source_update(E, F, rho, eg, v, N, edges, &op, -1.0, 1.0, NULL, 1) != -5) bad |= 8;
  op.mean_mode = 5;
  if (ora_source_update(E, F, rho, eg, v, N, edges, &op, 1.0, 1.0, NULL, 1) != -6) bad |= 16;
  if (ora_source_update(NULL, F, rho, eg, v, N, edges, &op, 1.0, 1.0, NULL, 1) != -1) bad |= 32;
  /* building blocks */
  double out[4], lq[NG], al[NG], dx[NG + 1], jg0[NG], jgg[NG], fr[NG];
  for (double x = 0.0; x < 800.0; x = x * 1.7 + 0.01) {
    (void)ora_planck_P(x);
    (void)ora_planck_Qs(x);
    ora_group_planck(x, x * 1.3 + 0.1, out);
  }
  ora_group_planck(0.0, INFINITY, out);
  for (int g = 0; g < NG; ++g) {
    lq[g] = g == 3 ? -INFINITY : log(urand() + 0.1);
    jg0[g] = urand();
    jgg[g] = -1.0 - urand();
    fr[g] = urand() - 0.5;
  }
  ora_slopes(NG, edges, lq, al);
  ora_arrowhead_solve(NG, 1.0, jg0, jgg, 0.3, fr, dx);
  (void)ora_mean_ratio(-1.0, 0.0, 2.0);
  (void)ora_mean_ratio(2.5, -3.5, 0.4);
  printf("oracle driver: %s (code %d)\n", bad ? "FAILED" : "ok", bad);
  return bad;
}
