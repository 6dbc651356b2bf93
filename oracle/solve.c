/*
 * solve.c -- oracle: the per-cell implicit matter-radiation source update of
 * Sec. 3 (eqs. egupdate-fupdate), taken step by step in the paper's order:
 *
 *   inner stage  Newton-Raphson on x = (E_gas, R_1..R_Ng) for eqs. FGFR/Rnew,
 *                Jacobian of eq. linear, elimination of eq. matrix, stop rule
 *                with E_tot and eps (Sec. 3);
 *   energy       E_g <- E_g^(t) + R_g + S_g, E_gas <- E_gas^(t) - (c/c_hat) sum R_g;
 *   outer stage  flux update eq. numF1 with the outdated velocity, momentum
 *                update, and repetition until the velocity/flux terms of R_g
 *                stop changing.
 *
 * Mean opacities follow Sec. 2.2 (PC, PPL with fixed slopes, PPL with the
 * Appendix A slopes) and eq. chiDiff for the flux mean.  Readings taken where
 * the paper is silent are marked READING.  Test infrastructure only.
 *
 * Parity unpinned: which root the PPL-free iteration reaches where the
 * minmod slopes kink and several fixed points exist (the slopes lag the
 * iterate); the tests pin that the output is a root of the implicit system,
 * not which one a warm start reaches.
 */
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include "mgrhd_oracle.h"

void ora_default_options(ora_options* o) {
  memset(o, 0, sizeof(*o));
  o->c = 1.0;
  o->a_rad = 1.0;
  o->h_over_k = 1.0;
  o->c_v = 1.5;
  o->eps_newton = 1e-11; /* Sec. 3 */
  o->eps_outer = 1e-13;  /* Sec. 3 */
  o->max_newton = 100;   /* READING: the paper gives no cap */
  o->max_outer = 20;     /* READING: the paper gives no cap; dynamic diffusion
                          * (tau v/c >> 1) needs more than a handful */
  o->closure = ORA_CLOSURE_M1;
  o->polish = 0;
}

typedef struct {
  int64_t n;
  int32_t ng, mode, closure, max_newton, max_outer, polish;
  const double* nu;
  double* lnr;   /* [ng] ln(nu_g+ / nu_g-) */
  double* achi;  /* [ng] alpha_chi (0 in PC) */
  double* lndnu; /* [ng] ln(nu_g+ - nu_g-) */
  const double* chilo;
  const double* kappa;
  double t_exp, t_ref; /* temperature dependence of the opacity (0: none) */
  int32_t stim;        /* 1: stimulated-emission factor 1 - e^{-x}         */
  double dt, chat, c, a, hk, cv, eps, eps_out;
  double *E_g, *F_g, *e_gas, *v;
  const double *rho, *S, *guess;
  int32_t guess_kind;
  int32_t *iters, *outer, *status, *trace;
  const int32_t* force;
} problem;

typedef struct {
  double *Bt, *Dnu, *dBdT, *b, *elo, *ehi, *sig, *chil;
  double *chiB, *chiE, *chiF, *DchiB, *alB, *alE, *logq, *ac;
  double *E0, *S, *R, *FR, *Jg0, *Jgg, *dx, *vF, *Ecur, *F0, *Fk, *Fn;
} work;

/* ---------------------------------------------------------------------- */
/* Planck data, slopes and group-mean opacities at temperature T (Sec. 2.2). */
static void material(const problem* p, work* w, double T, double rho_kappa,
                     const double* Ecur) {
  const int32_t ng = p->ng;
  const double aT4 = p->a * T * T * T * T;
  for (int32_t g = 0; g < ng; ++g) {
    double out[4];
    ora_group_planck(p->hk * p->nu[g] / T, p->hk * p->nu[g + 1] / T, out);
    double scale = exp(-out[3]);
    w->b[g] = out[0];
    w->elo[g] = out[1];
    w->ehi[g] = out[2];
    w->sig[g] = out[3];
    w->Bt[g] = aT4 * out[0] * scale;                /* B~_g = 4 pi B_g / c */
    w->Dnu[g] = aT4 * (out[2] - out[1]) * scale;    /* Delta_g(nu B~_nu)  */
    w->dBdT[g] = (4.0 * w->Bt[g] - w->Dnu[g]) / T;  /* d B~_g / dT        */
    /* chi_{0,g-} at this temperature and the opacity index of the group */
    double f = 1.0, ac = p->achi[g];
    if (p->t_exp != 0.0) f = pow(T / p->t_ref, p->t_exp);
    if (p->stim) {
      double s_lo = -expm1(-p->hk * p->nu[g] / T);      /* 1 - e^{-x} at nu_g- */
      double s_hi = -expm1(-p->hk * p->nu[g + 1] / T);  /* and at nu_g+       */
      f *= s_lo;
      if (p->mode != ORA_MEAN_PC) ac += log(s_hi / s_lo) / p->lnr[g];
    }
    w->chil[g] = rho_kappa * p->chilo[g] * f;
    w->ac[g] = ac;
  }
  if (p->mode == ORA_MEAN_PC) {
    /* eq. m1e1: one constant per group; all means equal it, eq. G_model1b */
    for (int32_t g = 0; g < ng; ++g) {
      w->chiB[g] = w->chiE[g] = w->chiF[g] = w->chil[g];
      w->DchiB[g] = w->chil[g] * w->Dnu[g];
    }
    return;
  }
  if (p->mode == ORA_MEAN_PPL_FIXED) {
    for (int32_t g = 0; g < ng; ++g) w->alB[g] = w->alE[g] = -1.0; /* eq. equality */
  } else {
    /* Appendix A: slopes of B_nu from the group Planck integrals, of E_nu from
     * the current radiation energies (READING: lagged within the iteration). */
    for (int32_t g = 0; g < ng; ++g)
      w->logq[g] = w->b[g] > 0.0 ? log(w->b[g]) - w->sig[g] - p->lndnu[g] : -INFINITY;
    ora_slopes(ng, p->nu, w->logq, w->alB);
    for (int32_t g = 0; g < ng; ++g)
      w->logq[g] = Ecur[g] > 0.0 ? log(Ecur[g]) - p->lndnu[g] : -INFINITY;
    ora_slopes(ng, p->nu, w->logq, w->alE);
  }
  for (int32_t g = 0; g < ng; ++g) {
    double ac = w->ac[g], L = p->lnr[g], chl = w->chil[g];
    w->chiB[g] = chl * ora_mean_ratio(ac, w->alB[g], L); /* eq. chiQg, Q = B */
    w->chiE[g] = chl * ora_mean_ratio(ac, w->alE[g], L); /* eq. chiQg, Q = E */
    /* Delta_g(nu chi_0 B~_nu), group g's own powerlaw at both of its edges */
    double rac = exp(ac * L);
    double dchib_s = chl * (rac * w->ehi[g] - w->elo[g]);
    w->DchiB[g] = aT4 * dchib_s * exp(-w->sig[g]);
    /* eq. chiDiff in the scaled variables (the common factor cancels) */
    double num = (w->chiB[g] + w->chiE[g] / 3.0) * w->b[g] +
                 (ac * w->chiE[g] * w->b[g] - dchib_s) / 3.0;
    double den = (4.0 * w->b[g] - (w->ehi[g] - w->elo[g])) / 3.0;
    double chif = num / den;
    w->chiF[g] = (den > 0.0 && isfinite(chif)) ? chif : w->chiE[g];
  }
}

/* P_g . v for the group closure (Sec. 2.1: M1 per group; or Eddington). */
static void pressure_dot_v(int closure, double c, double E, const double F[3],
                           const double v[3], double Pv[3]) {
  if (!(E > 0.0)) {
    Pv[0] = Pv[1] = Pv[2] = 0.0;
    return;
  }
  double fmag = sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]);
  if (closure == ORA_CLOSURE_EDDINGTON || fmag == 0.0) {
    for (int d = 0; d < 3; ++d) Pv[d] = E * v[d] / 3.0;
    return;
  }
  double f = fmag / (c * E);
  if (f > 1.0) f = 1.0;
  /* Levermore (1984) Eddington factor of the M1 closure */
  double chi = (3.0 + 4.0 * f * f) / (5.0 + 2.0 * sqrt(4.0 - 3.0 * f * f));
  double n[3] = {F[0] / fmag, F[1] / fmag, F[2] / fmag};
  double nv = n[0] * v[0] + n[1] * v[1] + n[2] * v[2];
  for (int d = 0; d < 3; ++d)
    Pv[d] = E * (0.5 * (1.0 - chi) * v[d] + 0.5 * (3.0 * chi - 1.0) * n[d] * nv);
}

/* One inner stage.  Returns 0 converged, 1 hit max_newton, 2 T <= 0.
 * target >= 0: the iteration counts as converged when the cumulative step
 * count reaches target (a replayed schedule) instead of at the stop test. */
static int newton(const problem* p, work* w, double rho, double rho_kappa,
                  double egas0, double etot, const double v[3], double* egv,
                  int32_t* steps, int elim, int32_t target) {
  const int32_t ng = p->ng;
  const double cc = p->c / p->chat;
  const double ke = 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  int32_t polish_left = -1;
  for (;;) {
    double T = (*egv - ke) / (rho * p->cv);
    if (!(T > 0.0) || !isfinite(T)) return 2;
    for (int32_t g = 0; g < ng; ++g) w->Ecur[g] = w->E0[g] + w->R[g] + w->S[g];
    material(p, w, T, rho_kappa, w->Ecur);
    if (elim) {
      /* temperature-only start: at this T, eq. Rnew inverted for E_g and
       * F_R,g = 0 (eq. FGFR) are linear in R_g alone; take that R_g */
      for (int32_t g = 0; g < ng; ++g) {
        double tauE = p->chat * p->dt * w->chiE[g];
        double W = p->chat * p->dt * (1.0 + w->ac[g]) * w->chiF[g] * w->vF[g] /
                   (p->c * p->c);
        w->R[g] = (w->chiB[g] / w->chiE[g] * w->Bt[g] + W / tauE - w->E0[g] - w->S[g]) /
                  (1.0 + 1.0 / tauE);
      }
      elim = 0;
    }

    /* residuals of eq. FGFR with R_g from eq. Rnew inverted for E_g */
    double sumR = 0.0, sumabs = 0.0;
    for (int32_t g = 0; g < ng; ++g) sumR += w->R[g];
    double FG = *egv - egas0 + cc * sumR;
    for (int32_t g = 0; g < ng; ++g) {
      double tauE = p->chat * p->dt * w->chiE[g];
      double W = p->chat * p->dt * (1.0 + w->ac[g]) * w->chiF[g] * w->vF[g] /
                 (p->c * p->c);
      double Eg = w->chiB[g] / w->chiE[g] * w->Bt[g] + (W - w->R[g]) / tauE;
      w->FR[g] = Eg - w->E0[g] - w->R[g] - w->S[g];
      sumabs += fabs(w->FR[g]);
    }
    int conv = fabs(FG) / etot < p->eps && cc * sumabs / etot < p->eps;
    /* a replayed pass ends at its step count, or at the cap as the run did */
    if (target >= 0) conv = *steps >= target && (conv || *steps < p->max_newton);
    if (polish_left < 0 && conv) polish_left = p->polish;
    if (polish_left == 0) return 0;
    if (polish_left < 0 && *steps >= p->max_newton) return 1;

    /* Jacobian of eq. linear (d(chiB/chiE)/dT dropped, as in the paper) */
    for (int32_t g = 0; g < ng; ++g) {
      w->Jg0[g] = w->chiB[g] / w->chiE[g] * w->dBdT[g] / (rho * p->cv);
      w->Jgg[g] = -1.0 / (p->chat * p->dt * w->chiE[g]) - 1.0;
    }
    ora_arrowhead_solve(ng, cc, w->Jg0, w->Jgg, FG, w->FR, w->dx);

    /* READING: halve the step while it would make T <= 0 */
    double lam = 1.0;
    for (int h = 0; h < 30 && !(*egv + lam * w->dx[0] - ke > 0.0); ++h) lam *= 0.5;
    if (!(*egv + lam * w->dx[0] - ke > 0.0)) return 2;
    *egv += lam * w->dx[0];
    for (int32_t g = 0; g < ng; ++g) w->R[g] += lam * w->dx[g + 1];

    if (polish_left > 0)
      --polish_left;
    else
      ++*steps;
    if (polish_left == 0) return 0;
  }
}

static void solve_cell(const problem* p, work* w, int64_t i) {
  const int64_t n = p->n;
  const int32_t ng = p->ng;
  const double cc = p->c / p->chat;
  int32_t st = ORA_ST_OK, steps = 0, passes = 0;

  double rho = p->rho[i];
  double egas0 = p->e_gas[i];
  double v0[3] = {p->v[i], p->v[n + i], p->v[2 * n + i]};
  double kap = p->kappa ? p->kappa[i] : 1.0;
  int ok = rho > 0.0 && isfinite(rho) && kap > 0.0 && isfinite(kap) && isfinite(egas0) &&
           isfinite(v0[0]) && isfinite(v0[1]) && isfinite(v0[2]);
  double sumE0 = 0.0, sumS = 0.0;
  for (int32_t g = 0; g < ng && ok; ++g) {
    w->E0[g] = p->E_g[(int64_t)g * n + i];
    w->S[g] = p->S ? p->S[(int64_t)g * n + i] : 0.0;
    for (int d = 0; d < 3; ++d) {
      w->F0[3 * g + d] = p->F_g[((int64_t)d * ng + g) * n + i];
      ok = ok && isfinite(w->F0[3 * g + d]);
    }
    ok = ok && w->E0[g] >= 0.0 && isfinite(w->E0[g]) && isfinite(w->S[g]);
    sumE0 += w->E0[g];
    sumS += w->S[g];
  }
  double ke0 = 0.5 * rho * (v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2]);
  double etot = egas0 + (p->chat / p->c) * (sumE0 + sumS); /* Sec. 3 */
  ok = ok && (egas0 - ke0) > 0.0 && etot > 0.0;
  if (!ok) {
    st = ORA_ST_INVALID;
    goto done;
  }
  const double rho_kappa = rho * kap;

  double egv;
  int warm = p->guess != NULL;
  if (warm) {
    egv = p->guess[i];
    for (int32_t g = 0; g < ng; ++g)
      w->R[g] = p->guess_kind == 1 ? 0.0 : p->guess[(int64_t)(g + 1) * n + i];
  } else {
    egv = egas0; /* READING: plain Newton starts from the old state */
    for (int32_t g = 0; g < ng; ++g) w->R[g] = 0.0;
  }
  double v[3] = {v0[0], v0[1], v0[2]};
  memcpy(w->Fk, w->F0, sizeof(double) * 3 * (size_t)ng);
  double egas_new = egas0;

  if (p->trace)
    for (int32_t k = 0; k < p->max_outer; ++k) p->trace[(int64_t)k * n + i] = -1;
  for (int32_t k = 0;; ++k) {
    ++passes;
    const int32_t target = p->force ? p->force[(int64_t)k * n + i] : -1;
    for (int32_t g = 0; g < ng; ++g)
      w->vF[g] = v[0] * w->Fk[3 * g] + v[1] * w->Fk[3 * g + 1] + v[2] * w->Fk[3 * g + 2];
    int rc = newton(p, w, rho, rho_kappa, egas0, etot, v, &egv, &steps,
                    k == 0 && warm && p->guess_kind == 1, target);
    if (k == 0 && warm && rc != 0) {
      st |= ORA_ST_FALLBACK;
      egv = egas0;
      for (int32_t g = 0; g < ng; ++g) w->R[g] = 0.0;
      rc = newton(p, w, rho, rho_kappa, egas0, etot, v, &egv, &steps, 0, target);
    }
    if (rc == 1) st |= ORA_ST_NEWTON_MAXIT;
    if (rc == 2) {
      st |= ORA_ST_INVALID;
      goto done;
    }
    /* conservative energy update (Sec. 3) */
    double sumR = 0.0;
    for (int32_t g = 0; g < ng; ++g) {
      w->Ecur[g] = w->E0[g] + w->R[g] + w->S[g];
      sumR += w->R[g];
    }
    egas_new = egas0 - cc * sumR;

    /* outer stage: material state at the updated energies, outdated velocity */
    double ke = 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double T = (egas_new - ke) / (rho * p->cv);
    if (!(T > 0.0) || !isfinite(T)) {
      st |= ORA_ST_INVALID;
      goto done;
    }
    if (p->trace) p->trace[(int64_t)k * n + i] = steps;
    material(p, w, T, rho_kappa, w->Ecur);
    double mom[3] = {rho * v0[0], rho * v0[1], rho * v0[2]};
    for (int32_t g = 0; g < ng; ++g) {
      double Pv[3];
      pressure_dot_v(p->closure, p->c, w->Ecur[g], &w->Fk[3 * g], v, Pv);
      double emit = w->chiB[g] * w->Bt[g] - w->DchiB[g] / 3.0;
      double den = 1.0 + p->chat * p->dt * w->chiF[g];
      for (int d = 0; d < 3; ++d) {
        /* eq. numF1 */
        double Fn = (w->F0[3 * g + d] +
                     p->chat * p->dt * (v[d] * emit + (1.0 + w->ac[g]) * w->chiE[g] * Pv[d])) /
                    den;
        w->Fn[3 * g + d] = Fn;
        mom[d] -= (Fn - w->F0[3 * g + d]) / (p->c * p->chat); /* momentum update */
      }
    }
    double vn[3] = {mom[0] / rho, mom[1] / rho, mom[2] / rho};
    /* change of the velocity/flux terms of eq. Rnew from this pass to the
     * next, and their size (READING: measured against E_tot only) */
    double dW = 0.0, sW = 0.0;
    for (int32_t g = 0; g < ng; ++g) {
      double vf_new = vn[0] * w->Fn[3 * g] + vn[1] * w->Fn[3 * g + 1] + vn[2] * w->Fn[3 * g + 2];
      double vf_old = v[0] * w->Fk[3 * g] + v[1] * w->Fk[3 * g + 1] + v[2] * w->Fk[3 * g + 2];
      double kW = fabs(p->chat * p->dt * (1.0 + w->ac[g]) * w->chiF[g]) / (p->c * p->c);
      dW += kW * fabs(vf_new - vf_old);
      sW += kW * fabs(vf_new);
    }
    /* READING: the next inner pass starts from the temperature of this
     * outer stage, i.e. from the conservatively updated E_gas carrying the
     * change of the kinetic energy, and from this pass's R_g */
    double ke_new = 0.5 * rho * (vn[0] * vn[0] + vn[1] * vn[1] + vn[2] * vn[2]);
    egv = egas_new + (ke_new - ke);
    v[0] = vn[0];
    v[1] = vn[1];
    v[2] = vn[2];
    memcpy(w->Fk, w->Fn, sizeof(double) * 3 * (size_t)ng);
    /* READING: where the velocity terms are large against E_tot (tau v/c >> 1)
     * their change cannot be resolved below their own rounding; the test then
     * accepts a change within 2^-46 (64 roundings) of their size */
    int done_outer = dW < p->eps_out * etot + 0x1p-46 * sW;
    if (!done_outer && k + 1 >= p->max_outer) st |= ORA_ST_OUTER_MAXIT;
    if (p->force) {
      if (k + 1 >= p->max_outer || p->force[(int64_t)(k + 1) * n + i] < 0) break;
    } else if (done_outer || k + 1 >= p->max_outer) {
      break;
    }
  }

  /* store, unless something is not finite */
  {
    int finite = isfinite(egas_new) && isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]);
    for (int32_t g = 0; g < ng; ++g) {
      finite = finite && isfinite(w->Ecur[g]);
      for (int d = 0; d < 3; ++d) finite = finite && isfinite(w->Fk[3 * g + d]);
    }
    if (!finite) {
      st |= ORA_ST_NONFINITE;
      goto done;
    }
    p->e_gas[i] = egas_new;
    for (int d = 0; d < 3; ++d) p->v[(int64_t)d * n + i] = v[d];
    for (int32_t g = 0; g < ng; ++g) {
      p->E_g[(int64_t)g * n + i] = w->Ecur[g];
      for (int d = 0; d < 3; ++d) p->F_g[((int64_t)d * ng + g) * n + i] = w->Fk[3 * g + d];
    }
  }
done:
  if (p->iters) p->iters[i] = steps;
  if (p->outer) p->outer[i] = passes;
  if (p->status) p->status[i] = st;
}

/* ---------------------------------------------------------------------- */
typedef struct {
  const problem* p;
  int64_t lo, hi;
} chunk;

static void* worker(void* arg) {
  chunk* ch = (chunk*)arg;
  const int32_t ng = ch->p->ng;
  /* 24 arrays of N_g doubles, one of N_g + 1 and three of 3 N_g */
  double* mem = (double*)malloc(sizeof(double) * ((size_t)ng * 34 + 1));
  if (!mem) return (void*)1;
  work w;
  double* q = mem;
  double** slots[] = {&w.Bt,  &w.Dnu,  &w.dBdT, &w.b,   &w.elo, &w.ehi, &w.sig,
                      &w.chil, &w.chiB, &w.chiE, &w.chiF, &w.DchiB, &w.alB, &w.alE,
                      &w.logq, &w.E0,  &w.S,    &w.R,   &w.FR,  &w.Jg0, &w.Jgg,
                      &w.vF,  &w.Ecur, &w.ac};
  for (size_t s = 0; s < sizeof(slots) / sizeof(slots[0]); ++s) {
    *slots[s] = q;
    q += ng;
  }
  w.dx = q;
  q += ng + 1;
  w.F0 = q;
  q += 3 * ng;
  w.Fk = q;
  q += 3 * ng;
  w.Fn = q;
  for (int64_t i = ch->lo; i < ch->hi; ++i) solve_cell(ch->p, &w, i);
  free(mem);
  return NULL;
}

int ora_source_update(double* E_g, double* F_g, const double* rho, double* e_gas,
                      double* v, int64_t n, const double* edges, const ora_opacity* op,
                      double dt, double c_hat, const ora_options* opt_in,
                      int32_t n_threads) {
  ora_options defaults;
  ora_default_options(&defaults);
  const ora_options* opt = opt_in ? opt_in : &defaults;
  if (n < 0) return -2;
  if (n == 0) return 0;
  if (!E_g || !F_g || !rho || !e_gas || !v || !edges || !op || !op->chi_lo) return -1;
  const int32_t ng = op->n_groups;
  if (ng < 1 || ng > 4096) return -2;
  if (op->mean_mode < 0 || op->mean_mode > 2) return -6;
  for (int32_t g = 0; g <= ng; ++g)
    if (!(edges[g] >= 0.0) || (g > 0 && !(edges[g] > edges[g - 1]))) return -3;
  if (op->mean_mode != ORA_MEAN_PC && (!(edges[0] > 0.0) || isinf(edges[ng]))) return -3;
  for (int32_t g = 0; g < ng; ++g) {
    if (!(op->chi_lo[g] > 0.0) || !isfinite(op->chi_lo[g])) return -4;
    if (op->mean_mode != ORA_MEAN_PC) {
      if (op->alpha_chi) {
        if (!isfinite(op->alpha_chi[g])) return -4;
      } else if (op->chi_hi) {
        if (!(op->chi_hi[g] > 0.0) || !isfinite(op->chi_hi[g])) return -4;
      } else {
        return -4;
      }
    }
  }
  if (!isfinite(op->t_exp) || (op->t_exp != 0.0 && (!(op->t_ref > 0.0) || !isfinite(op->t_ref))))
    return -4;
  if (op->stim < 0 || op->stim > 1 || (op->stim && !(edges[0] > 0.0))) return -4;
  if (!(dt > 0.0) || !(c_hat > 0.0) || !isfinite(dt) || !isfinite(c_hat)) return -5;
  if (!(opt->c > 0.0) || !(opt->a_rad > 0.0) || !(opt->h_over_k > 0.0) || !(opt->c_v > 0.0))
    return -5;
  if (!(opt->eps_newton > 0.0) || !(opt->eps_outer > 0.0) || opt->max_newton < 1 ||
      opt->max_outer < 1 || opt->polish < 0 || opt->closure < 0 || opt->closure > 1 ||
      opt->guess_kind < 0 || opt->guess_kind > 1)
    return -6;

  problem p;
  memset(&p, 0, sizeof(p));
  p.n = n;
  p.ng = ng;
  p.mode = op->mean_mode;
  p.closure = opt->closure;
  p.max_newton = opt->max_newton;
  p.max_outer = opt->max_outer;
  p.polish = opt->polish;
  p.nu = edges;
  p.chilo = op->chi_lo;
  p.kappa = op->kappa_scale;
  p.t_exp = op->t_exp;
  p.t_ref = op->t_ref;
  p.stim = op->stim;
  p.dt = dt;
  p.chat = c_hat;
  p.c = opt->c;
  p.a = opt->a_rad;
  p.hk = opt->h_over_k;
  p.cv = opt->c_v;
  p.eps = opt->eps_newton;
  p.eps_out = opt->eps_outer;
  p.E_g = E_g;
  p.F_g = F_g;
  p.e_gas = e_gas;
  p.v = v;
  p.rho = rho;
  p.S = opt->S_g;
  p.guess = opt->guess;
  p.guess_kind = opt->guess_kind;
  p.iters = opt->iters;
  p.outer = opt->outer;
  p.status = opt->status;
  p.trace = opt->trace;
  p.force = opt->force;
  double* tab = (double*)malloc(sizeof(double) * 3 * (size_t)ng);
  if (!tab) return -7;
  p.lnr = tab;
  p.achi = tab + ng;
  p.lndnu = tab + 2 * ng;
  for (int32_t g = 0; g < ng; ++g) {
    p.lnr[g] = log(edges[g + 1] / edges[g]);
    p.lndnu[g] = log(edges[g + 1] - edges[g]);
    if (op->mean_mode == ORA_MEAN_PC)
      p.achi[g] = 0.0;
    else if (op->alpha_chi)
      p.achi[g] = op->alpha_chi[g];
    else /* tabulated opacity: index from the edge values (Sec. 2.2.2) */
      p.achi[g] = log(op->chi_hi[g] / op->chi_lo[g]) / p.lnr[g];
  }

  int32_t nt = n_threads > 0 ? n_threads : (int32_t)sysconf(_SC_NPROCESSORS_ONLN);
  if (nt < 1) nt = 1;
  if ((int64_t)nt > n) nt = (int32_t)n;
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nt);
  chunk* ch = (chunk*)malloc(sizeof(chunk) * (size_t)nt);
  int rc = 0;
  if (!th || !ch) {
    rc = -7;
  } else {
    for (int32_t t = 0; t < nt; ++t) {
      ch[t].p = &p;
      ch[t].lo = n * t / nt;
      ch[t].hi = n * (t + 1) / nt;
    }
    int32_t started = 0;
    for (; started < nt; ++started)
      if (pthread_create(&th[started], NULL, worker, &ch[started]) != 0) break;
    if (started < nt) /* run what could not be threaded on this thread */
      for (int32_t t = started; t < nt; ++t) worker(&ch[t]);
    for (int32_t t = 0; t < started; ++t) {
      void* ret = NULL;
      pthread_join(th[t], &ret);
      if (ret) rc = -7;
    }
  }
  free(th);
  free(ch);
  free(tab);
  return rc;
}

int mgrhd_oracle_source_update(double* E_g, double* F_g, const double* rho, double* e_gas,
                               double* v, int64_t n, const double* group_edges,
                               const ora_opacity* op, double dt, double c_hat,
                               const ora_options* opt, int32_t n_threads) {
  return ora_source_update(E_g, F_g, rho, e_gas, v, n, group_edges, op, dt, c_hat, opt,
                           n_threads);
}
