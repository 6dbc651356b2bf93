/*
 * mgrhd_oracle.h -- plain FP64 CPU oracle of the mixed-frame multigroup
 * matter-radiation source update (He, Wibking & Krumholz 2024, Sec. 2.2 and 3).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * source, header, table or helper with the GPU library.
 *
 * Units: every physical constant is an argument (c, c_hat, a_R, h/k, c_v).
 * Frequencies are in the units of group_edges; x = (h/k) nu / T.
 *
 * Layout (host memory, structure of arrays, cell index fastest):
 *   E_g[g*n + i], F_g[(d*N_g + g)*n + i], v[d*n + i], rho[i], e_gas[i].
 *
 * Parity status of each function is stated beside it; every function below is
 * pinned by a CPU test against mpmath quadrature / polylogarithms, dense
 * linear algebra, closed forms or brute-force root finding.
 */
#ifndef MGRHD_ORACLE_H
#define MGRHD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* group-mean opacity model (Sec. 2.2.1, 2.2.2 and Appendix A) */
enum { ORA_MEAN_PC = 0, ORA_MEAN_PPL_FIXED = 1, ORA_MEAN_PPL_FREE = 2 };
/* closure for the group pressure tensor (Sec. 2.1: M1 by default; Eddington) */
enum { ORA_CLOSURE_M1 = 0, ORA_CLOSURE_EDDINGTON = 1 };

/* per-cell status bits */
enum {
  ORA_ST_OK = 0,
  ORA_ST_NEWTON_MAXIT = 1, /* the cell's Newton steps (all passes) hit max_newton */
  ORA_ST_OUTER_MAXIT = 2,  /* the outer flux/momentum loop hit max_outer     */
  ORA_ST_FALLBACK = 4,     /* warm start failed; plain Newton restarted       */
  ORA_ST_INVALID = 8,      /* invalid input or T <= 0; cell left unchanged    */
  ORA_ST_NONFINITE = 16    /* non-finite result; cell left unchanged          */
};

typedef struct {
  int32_t n_groups;          /* N_g >= 1                                        */
  int32_t mean_mode;         /* ORA_MEAN_*                                      */
  const double* chi_lo;      /* [N_g] opacity at each group's lower edge, per
                                unit (rho * kappa_scale)                        */
  const double* alpha_chi;   /* [N_g] powerlaw index, or NULL                   */
  const double* chi_hi;      /* [N_g] opacity at the upper edge (tabulated case,
                                index derived as a log ratio), or NULL          */
  const double* kappa_scale; /* [n] per-cell multiplier, or NULL (=1)           */
  /* Temperature dependence (Sec. 4.1.2 simulation (c); eq. pulsek):
   *   chi_0(nu, T) = rho kappa_scale chi^(nu) (T / t_ref)^t_exp [1 - e^{-x}]^stim,
   * x = (h/k) nu / T, chi^ the table above.  Every Newton iterate evaluates the
   * opacities at its own temperature; the Jacobian drops their T-derivatives,
   * as the paper does for chi_0B/chi_0E (Sec. 3).  READING: in the PPL modes
   * the group's powerlaw passes through the T-dependent values at its two
   * edges (the tabulated-opacity rule of Sec. 2.2.2); PC takes the value at
   * the lower edge, as for a T-independent table.  t_exp = 0 and stim = 0:
   * no temperature dependence. */
  double t_exp;
  double t_ref;              /* > 0 when t_exp != 0                             */
  int32_t stim;              /* 0 or 1; 1 needs group_edges[0] > 0              */
  int32_t reserved;
} ora_opacity;

typedef struct {
  double c, a_rad, h_over_k, c_v; /* c_v per unit mass; C_v = rho c_v        */
  double eps_newton;              /* inner tolerance (paper: 1e-11)           */
  double eps_outer;               /* outer tolerance (paper: 1e-13)           */
  int32_t max_newton, max_outer;
  int32_t closure;                /* ORA_CLOSURE_*                            */
  int32_t polish;                 /* extra Newton steps after convergence     */
  const double* S_g;              /* [N_g][n] optional source, or NULL        */
  const double* guess;            /* [N_g+1][n] warm start (E_gas, R_g) or NULL */
  int32_t* iters;                 /* [n] out: Newton steps (all outer passes) */
  int32_t* outer;                 /* [n] out: outer passes, or NULL           */
  int32_t* status;                /* [n] out: ORA_ST_* bits, or NULL          */
  int32_t guess_kind;             /* 0: guess holds (E_gas, R_g); 1: only row 0
                                     (E_gas) is read and each R_g solves its own
                                     group balance at that temperature        */
  int32_t reserved;
  /* [max_outer][n] out, or NULL: trace[k*n + i] = Newton steps of cell i
   * counted up to the end of inner pass k (cumulative, as iters), written
   * when pass k reaches its outer stage; -1 for every pass that did not. */
  int32_t* trace;
  /* [max_outer][n] in, or NULL: a schedule in the layout of trace.  Pass k of
   * cell i then stops its Newton iteration when the cumulative step count
   * reaches force[k*n + i] (instead of at the stop test; polish steps follow
   * as usual), and the outer loop stops after pass k when force[(k+1)*n + i]
   * is negative or k + 1 = max_outer (instead of at the outer test).  This
   * replays the iteration counts of another implementation, so that two
   * implementations can be compared value by value where a stop test sits on
   * its threshold.  Status bits are still those of the stop tests. */
  const int32_t* force;
} ora_options;

/* Fill *o with the paper's defaults: eps 1e-11 / 1e-13, M1 closure,
 * max_newton 100, max_outer 20, polish 0, unit constants, c_v = 3/2. */
void ora_default_options(ora_options* o);

/* The full source update for n cells, in place, on host arrays.
 * dt is theta*Delta t of the IMEX stage, c_hat the reduced speed of light.
 * n_threads <= 0 uses all online CPUs.  Returns 0, or a negative code for an
 * invalid argument (nothing is modified then). */
int ora_source_update(double* E_g, double* F_g, const double* rho, double* e_gas,
                      double* v, int64_t n, const double* group_edges,
                      const ora_opacity* op, double dt, double c_hat,
                      const ora_options* opt, int32_t n_threads);

/* The same entry point under the name the GPU library's callers look for
 * beside mgrhd_source_update (host arrays, no stream, a thread count). */
int mgrhd_oracle_source_update(double* E_g, double* F_g, const double* rho, double* e_gas,
                               double* v, int64_t n, const double* group_edges,
                               const ora_opacity* op, double dt, double c_hat,
                               const ora_options* opt, int32_t n_threads);

/* ---- building blocks, exported so that tests can pin each one ---------- */

/* Planck fraction P(x) = (15/pi^4) int_0^x t^3/(e^t-1) dt and its complement
 * Q(x) = 1 - P(x); x may be 0 or +inf. */
double ora_planck_P(double x);
double ora_planck_Q(double x);
/* e^x Q(x), finite for every x > 0 */
double ora_planck_Qs(double x);

/* Group Planck data at temperature T for edges nu_lo < nu_hi, per a_R T^4:
 * out[0] = b     (B~_g / (a T^4)) * e^{sigma}
 * out[1] = e_lo  (nu B~_nu / (a T^4)) at nu_lo, times e^{sigma}
 * out[2] = e_hi  same at nu_hi
 * out[3] = sigma (0, or x_lo when the group lies in the Wien tail)
 * Unscaled: B~_g = a T^4 b e^{-sigma}, Delta_g(nu B~) = a T^4 (e_hi-e_lo) e^{-sigma}. */
void ora_group_planck(double x_lo, double x_hi, double out[4]);

/* chi_{0Q,g} / chi_{0,g-} for powerlaw indices alpha_chi and alpha_Q on a group
 * of log width L = ln(nu_+/nu_-) (eq. chiQg). */
double ora_mean_ratio(double alpha_chi, double alpha_Q, double L);

/* Appendix A slope reconstruction: given group integrals Q[N_g] (<=0 allowed),
 * edges nu[N_g+1], return alpha[N_g].  Q given as log of the specific value
 * when logq != NULL (entries may be -inf for empty groups). */
void ora_slopes(int32_t ng, const double* nu, const double* logqbar, double* alpha);

/* Solve the arrowhead Newton system of eq. matrix by elimination:
 * J00 = 1, J0g = c/c_hat, Jg0[g], Jgg[g]; rhs (-F_G, -F_R).  Returns dx[N_g+1]. */
void ora_arrowhead_solve(int32_t ng, double c_over_chat, const double* Jg0,
                         const double* Jgg, double FG, const double* FR, double* dx);

#ifdef __cplusplus
}
#endif
#endif
