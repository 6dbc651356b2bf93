/*
 * mgrhd.h -- C ABI of the MI355X (gfx950) implementation of the per-cell
 * implicit matter-radiation source update of mixed-frame multigroup
 * radiation hydrodynamics (He, Wibking & Krumholz 2024, arXiv:2407.18304).
 *
 * What one call computes, per cell (Sec. 3, eqs. egupdate-fupdate):
 *   inner stage  Newton-Raphson on x = (E_gas, R_1..R_Ng) for eqs. FGFR and
 *                Rnew, with the arrowhead Jacobian of eqs. linear/matrix
 *                eliminated in O(N_g), stopped by the E_tot-relative test
 *                with eps (default 1e-11);
 *   energy       E_g <- E_g + R_g + S_g, E_gas <- E_gas - (c/c_hat) sum_g R_g;
 *   outer stage  flux update eq. numF1 with the outdated velocity, momentum
 *                update, repeated until the velocity/flux terms of eq. Rnew
 *                change by less than eps_outer E_tot (default 1e-13) plus
 *                2^-46 of their own size (the change cannot be resolved
 *                below the rounding of the terms where they are large
 *                against E_tot, tau v/c >> 1), at most max_outer times.
 * Group-mean opacities: piecewise constant (eq. m1e1), piecewise powerlaw
 * with fixed slopes alpha_Q = -1 (eq. equality) or with the slope fit of
 * Appendix A (eqs. sg, minmod); eq. chiQg for chi_0B and chi_0E, eq. chiDiff
 * for chi_0F, Doppler factors (1 + alpha_chi) of eqs. G0_3 and G1_3.
 *
 * Units: every constant is an argument.  B~_g = 4 pi B_g / c is normalised
 * as a_R T^4 times the Planck fraction of the group, x = (h/k) nu / T.
 *
 * Memory: all arrays are DEVICE pointers owned by the caller, FP64, structure
 * of arrays with the cell index fastest:
 *   E_g[g*n + i], F_g[(d*N_g + g)*n + i], v[d*n + i], rho[i], e_gas[i].
 * The state is updated in place, or written to separate output arrays of the
 * same layout (mgrhd_options.E_g_out ... v_out) while the inputs are only
 * read.  Nothing is allocated by mgrhd_source_update.
 * Calls are asynchronous on `stream`; results and per-cell status are valid
 * after the caller synchronises the stream.
 *
 * Errors: a negative return is an argument error found on the host (nothing
 * was enqueued); a positive return is a HIP runtime error from the launch.
 * Errors that can only be seen on the device (a non-ascending edge table, a
 * non-positive opacity entry) are reported per cell as MGRHD_ST_BAD_TABLE and
 * leave the state untouched.
 */
#ifndef MGRHD_H
#define MGRHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* mgrhd_stream_t; /* a hipStream_t */

/* group-mean opacity model */
enum {
  MGRHD_MEAN_PC = 0,        /* piecewise constant, Sec. 2.2.1                */
  MGRHD_MEAN_PPL_FIXED = 1, /* powerlaw, alpha_B = alpha_E = -1, Sec. 2.2.2  */
  MGRHD_MEAN_PPL_FREE = 2   /* powerlaw, slopes by Appendix A                 */
};
/* closure for the group pressure tensor in the flux update (Sec. 2.1) */
enum { MGRHD_CLOSURE_M1 = 0, MGRHD_CLOSURE_EDDINGTON = 1 };

/* per-cell status bits (int32 array, optional) */
enum {
  MGRHD_ST_OK = 0,
  MGRHD_ST_NEWTON_MAXIT = 1, /* the cell's Newton steps (all passes) reached
                                max_newton                                       */
  MGRHD_ST_OUTER_MAXIT = 2,  /* the outer flux/momentum loop reached max_outer   */
  MGRHD_ST_FALLBACK = 4,     /* the warm start failed; plain Newton was rerun     */
  MGRHD_ST_INVALID = 8,      /* invalid cell input or T <= 0: cell untouched      */
  MGRHD_ST_NONFINITE = 16,   /* non-finite result: cell untouched                 */
  MGRHD_ST_BAD_TABLE = 32    /* edge/opacity table rejected on the device         */
};

/* host-side argument errors (negative returns) */
enum {
  MGRHD_E_NULL = -1,     /* a required pointer is NULL                          */
  MGRHD_E_SIZE = -2,     /* n_cells < 0 or n_groups outside [1, MGRHD_MAX_GROUPS] */
  MGRHD_E_MODE = -3,     /* unknown mean_mode or closure                         */
  MGRHD_E_TABLE = -4,    /* powerlaw mode without alpha_chi or chi_hi            */
  MGRHD_E_SCALAR = -5,   /* dt, c_hat or a physical constant not positive/finite */
  MGRHD_E_OPTION = -6,   /* eps, max_newton, max_outer or polish out of range    */
  MGRHD_E_DEVICE = -7    /* no usable device / kernel image                      */
};

#define MGRHD_MAX_GROUPS 256

/* Opacity description.  chi_0(nu) in group g is
 *   rho * kappa_scale[i] * chi_lo[g] * (nu / nu_g-)^alpha_chi[g]
 *       * (T / t_ref)^t_exp * [1 - exp(-(h/k) nu / T)]^stim
 * (Sec. 2.2.2; the temperature factors as in Sec. 4.1.2 simulation (c),
 * t_exp = 3/2, and eq. pulsek, t_exp = -1/2 with stim = 1).  chi_lo,
 * alpha_chi, chi_hi are DEVICE arrays of N_g entries; when alpha_chi is NULL
 * the index is ln(chi_hi/chi_lo)/ln(nu_g+/nu_g-) (tabulated opacity).  PC
 * ignores both and uses chi_lo as the group value.  kappa_scale is a DEVICE
 * array of n_cells entries or NULL (= 1).
 * Temperature dependence (t_exp != 0 or stim = 1): the opacities are
 * evaluated at every Newton iterate's temperature and the Jacobian leaves
 * out their T-derivatives (Sec. 3).  In the PPL modes the group's powerlaw
 * passes through the T-dependent values at its two edges; PC takes the value
 * at the lower edge.  t_exp must be finite, t_ref > 0 when t_exp != 0
 * (MGRHD_E_TABLE otherwise), stim 0 or 1; with stim = 1 group_edges[0] must
 * be > 0 (cells report MGRHD_ST_BAD_TABLE otherwise).  Zero-initialised
 * fields give a T-independent opacity.  The batched entry points take
 * T-independent tables only. */
typedef struct {
  int32_t n_groups;
  int32_t mean_mode;
  const double* chi_lo;
  const double* alpha_chi;
  const double* chi_hi;
  const double* kappa_scale;
  double t_exp;
  double t_ref;
  int32_t stim;
  int32_t reserved;
} mgrhd_opacity_params;

/* Options; mgrhd_default_options() fills the paper's values. */
typedef struct {
  double c, a_rad, h_over_k, c_v; /* c_v per unit mass (C_v = rho c_v)            */
  double eps_newton;              /* inner stop tolerance, default 1e-11 (Sec. 3)  */
  double eps_outer;               /* outer stop tolerance, default 1e-13 (Sec. 3)  */
  int32_t max_newton;             /* cap on a cell's Newton steps summed over its
                                     outer passes; default 100                    */
  int32_t max_outer;              /* default 20                                    */
  int32_t closure;                /* MGRHD_CLOSURE_*                               */
  int32_t polish;                 /* extra Newton steps after convergence, 0..4    */
  const double* S_g;              /* [N_g][n] optional source term (eq. FGFR), or NULL */
  const double* guess;            /* [N_g+1][n] warm start (E_gas, R_g), or NULL   */
  int32_t* iters;                 /* [n] out: Newton steps summed over passes, or NULL */
  int32_t* outer;                 /* [n] out: outer passes, or NULL                */
  int32_t* status;                /* [n] out: MGRHD_ST_* bits, or NULL             */
  int32_t guess_kind;             /* 0: guess holds (E_gas, R_g) for every cell;
                                     1: only row 0 (E_gas, [n]) is read, and each
                                     R_g is taken from its own group balance at
                                     that temperature (eq. Rnew inverted for E_g
                                     with F_R,g = 0, eq. FGFR), so the first Newton
                                     step corrects the temperature alone       */
  int32_t reserved;
  int32_t* trace;                 /* [max_outer][n] out, or NULL: trace[k*n + i] =
                                     Newton steps of cell i counted up to the end
                                     of inner pass k (cumulative, as iters),
                                     written when pass k reaches its outer stage;
                                     -1 for every pass that did not.  A record of
                                     where the stop tests ended each pass (a
                                     checker can replay it)                      */
  /* Out-of-place update (mgrhd_source_update and the IMEX steps): with all
   * four set, the updated E_g, F_g, e_gas, v are written here (same layouts)
   * and the input arrays are only read; a cell left untouched (invalid
   * input, a table error, non-finite results) gets its input values copied.
   * All four NULL: the update is in place.  An output must be its input
   * array or not overlap any argument.  The batch takes them per patch
   * (mgrhd_patch) and returns MGRHD_E_OPTION when any is set here. */
  double* E_g_out;                /* [N_g][n]    */
  double* F_g_out;                /* [3][N_g][n] */
  double* e_gas_out;              /* [n]         */
  double* v_out;                  /* [3][n]      */
} mgrhd_options;

/* Fill *opt with the defaults: c = a_rad = h_over_k = 1, c_v = 3/2,
 * eps_newton = 1e-11, eps_outer = 1e-13, max_newton = 100, max_outer = 20,
 * M1 closure, polish = 0, all optional arrays NULL. */
void mgrhd_default_options(mgrhd_options* opt);

/* The source update of n_cells cells, in place (see the top of this file),
 * or from the given arrays into opt's *_out arrays (out of place).
 *   E_g          [N_g][n]    in/out  group radiation energy densities
 *   F_g          [3][N_g][n] in/out  group radiation fluxes
 *   rho          [n]         in      gas density
 *   e_gas        [n]         in/out  gas total energy density E_gas
 *   v            [3][n]      in/out  gas velocity
 *   group_edges  [N_g+1]     in      DEVICE array, strictly ascending; > 0 and
 *                                    finite in the powerlaw modes, 0 / +inf
 *                                    allowed in PC
 *   opacity      host struct describing device tables
 *   dt           theta * Delta t of the IMEX stage (eqs. egupdate-fupdate)
 *   c_hat        reduced speed of light
 *   stream       HIP stream (NULL = default stream)
 *   opt          NULL for defaults
 * Returns 0 when enqueued, MGRHD_E_* < 0 on a host-side argument error, or a
 * positive hipError_t. */
int mgrhd_source_update(double* E_g, double* F_g, const double* rho, double* e_gas, double* v,
                        int64_t n_cells, const double* group_edges,
                        const mgrhd_opacity_params* opacity, double dt, double c_hat,
                        mgrhd_stream_t stream, const mgrhd_options* opt);

/* Kernel variant used for a given group count: lanes per cell, groups per
 * lane and the register budget, given as the minimum resident waves per SIMD
 * it is compiled for (more waves: fewer registers per lane).
 * mgrhd_set_variant overrides the built-in choice for n_groups (0, 0, 0
 * restores it; waves_per_simd = 0 takes the default budget of the pair);
 * variants that are not compiled, or whose lanes x groups < n_groups, return
 * MGRHD_E_OPTION.  Any pointer of mgrhd_get_variant may be NULL. */
int mgrhd_get_variant(int32_t n_groups, int32_t mean_mode, int32_t* lanes_per_cell,
                      int32_t* groups_per_lane, int32_t* waves_per_simd);
int mgrhd_set_variant(int32_t n_groups, int32_t lanes_per_cell, int32_t groups_per_lane,
                      int32_t waves_per_simd);
/* The mean-opacity method the paper recommends for a group structure
 * (Sec. 4.1.3, after its Marshak-wave convergence study): PC when every
 * group is narrower in ln nu than a tenth of the whole range ln(nu_max/nu_min),
 * PPL with fixed slopes otherwise (which is also the choice for N_g <= 10
 * log-uniform groups).  A grid that reaches 0 or +inf gets PC, the only
 * method defined there.  edges: HOST array of n_groups + 1 ascending values.
 * Returns MGRHD_MEAN_PC or MGRHD_MEAN_PPL_FIXED, or MGRHD_E_NULL / _SIZE /
 * _TABLE (edges not ascending or negative). */
int32_t mgrhd_recommend_mean_mode(int32_t n_groups, const double* edges);

/* The compiled variants, k = 0 .. mgrhd_variant_count() - 1 (for autotuners). */
int32_t mgrhd_variant_count(void);
int mgrhd_variant_info(int32_t k, int32_t* lanes_per_cell, int32_t* groups_per_lane,
                       int32_t* waves_per_simd);

/* ---- Two-stage IMEX step of the source terms (Sec. 2.3, eqs. imex1, imex2) ----
 * With no transport term, one step of the paper's IMEX integrator is
 *   U^(n+1/2) = U^(n) + dt S(U^(n+1/2))            (source update, theta dt = dt)
 *   U^(n+1)   = (U^(n) + U^(n+1/2))/2 + (dt/2) S(U^(n+1))   (theta dt = dt/2).
 * mgrhd_imex_step performs both stages on the state of mgrhd_source_update
 * (same arguments and layout), in place, or with opt's *_out arrays set from
 * U^(n) into those (U^(n) only read).  The first stage writes U^(n+1/2)
 * into the caller's DEVICE workspace `work` of at least
 * mgrhd_imex_workspace_bytes() bytes (8 n (4 N_g + 4)), so that U^(n) is
 * never copied; the midpoint is formed where U^(n+1) goes and the second
 * stage updates it there; nothing is allocated.  opt->iters/outer/status
 * report the second stage.  Returns as mgrhd_source_update; MGRHD_E_SIZE if
 * the workspace is too small. */
size_t mgrhd_imex_workspace_bytes(int64_t n_cells, int32_t n_groups);
int mgrhd_imex_step(double* E_g, double* F_g, const double* rho, double* e_gas, double* v,
                    int64_t n_cells, const double* group_edges,
                    const mgrhd_opacity_params* opacity, double dt, double c_hat,
                    mgrhd_stream_t stream, const mgrhd_options* opt, void* work,
                    size_t work_bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the IMEX
 * step of mgrhd_imex_step with no workspace argument.  U^(n+1/2) is kept in
 * an array owned by the library, MGRHD_IMEX_SCRATCH_DOUBLES doubles (32 MiB) per
 * GPU, held from the first call on that GPU until the process ends; the call
 * allocates nothing.  Limit: mgrhd_imex_workspace_bytes(n_cells, n_groups)
 * <= 32 MiB (at most 61 680 cells at 16 groups, 16 131 at 64), else
 * MGRHD_E_SIZE with nothing enqueued.  Every call on one GPU shares that
 * array: calls that overlap on one GPU (other streams or threads) race and
 * must be serialised by the caller.  Returns as mgrhd_imex_step, or a HIP
 * error if the array's address cannot be obtained. */
#define MGRHD_IMEX_SCRATCH_DOUBLES (4 * 1024 * 1024)
int mgrhd_imex_step_noalloc(double* E_g, double* F_g, const double* rho, double* e_gas,
                            double* v, int64_t n_cells, const double* group_edges,
                            const mgrhd_opacity_params* opacity, double dt, double c_hat,
                            mgrhd_stream_t stream, const mgrhd_options* opt);

/* ---- Explicit stage of the IMEX integrator for a 1D column (Sec. 2.3) ----
 * One launch writes, for every cell i of a 1D column and every group g,
 *   out = a U0 + b U1 + dt_T T(U1)   (E_g, F_g)
 *   out = a U0 + b U1                (e_gas, v)
 * where T is the M1 transport of eq. ysf along x: dE_g/dt = -(c_hat/c) dF_g/dx,
 * dF_g/dt = -c_hat c dP_g/dx, P_g = chi(f) E_g with Levermore's M1 factor,
 * f = |F_g|/(c E_g) clipped to 1, in finite volumes with the local
 * Lax-Friedrichs flux (wave speeds -+c_hat) at each face; the energy flux's
 * dissipation is scaled by min(1, 1/tau)^2, tau = dx (chi_L + chi_R)/2 with
 * chi_i = rho[i] chi_mid[g].  Ghost cells: E_left[g], E_right[g], zero flux.
 * Only the x-components of F_g move; y and z are combined as the gas is.
 * Stage 1 of eqs. imex1/imex2 is (a, b, dt_T) = (0, 1, dt) with U1 = U^n;
 * stage 2 is (1/2, 1/2, dt/2) with U0 = U^n, U1 = U^(n+1/2); each is followed
 * by mgrhd_source_update with theta dt = dt_T * (stage 1: 1, stage 2: 1).
 * Layout as mgrhd_source_update (SoA, cell index fastest); all arrays are
 * DEVICE arrays: E [N_g][n], F [3][N_g][n], e_gas [n], v [3][n], rho [n],
 * chi_mid, E_left, E_right [N_g].  U0 may be NULL when a = 0.  The outputs
 * may alias U0 but not U1 (the stencil reads U1's neighbours;
 * MGRHD_E_OPTION if E_out == E1 or F_out == F1).  Returns 0, MGRHD_E_NULL,
 * MGRHD_E_SIZE, MGRHD_E_SCALAR (dx, c, c_hat not positive, dt_T < 0), or a
 * HIP error from the launch. */
int mgrhd_transport1d_stage(double* E_out, double* F_out, double* e_gas_out, double* v_out,
                            const double* E1, const double* F1, const double* e_gas1,
                            const double* v1, const double* E0, const double* F0,
                            const double* e_gas0, const double* v0, double a, double b,
                            int64_t n_cells, int32_t n_groups, double dx, double dt_T, double c,
                            double c_hat, const double* rho, const double* chi_mid,
                            const double* E_left, const double* E_right,
                            mgrhd_stream_t stream);

/* ---- Batched AMR-like patches: one persistent launch over many patches ----
 * Each patch holds its own SoA block (same layout as mgrhd_source_update,
 * with its own n_cells), its own group count (1..128), edges and opacity
 * table; dt and c_hat are per patch, the options per batch.  All pointers are
 * DEVICE pointers owned by the caller and must stay valid while the batch is
 * used.  The patches are cut into work items of at most `chunk_cells` cells,
 * ordered by decreasing group count; waves take items from a global counter
 * (cleared by a tiny kernel before the solver kernel, so the pair can be
 * captured in a hipGraph) and run the per-cell solver of mgrhd_source_update
 * with lanes per cell = next power of two >= N_g / groups_per_lane.
 * A batch owns a small device work list and counter (allocated by
 * mgrhd_batch_create, freed by mgrhd_batch_destroy; the work list is rebuilt
 * by mgrhd_batch_set_tuning when the cells per item change, which must not
 * overlap a run of the batch); mgrhd_batch_run, _capture and _launch
 * allocate nothing.  Runs of one batch on several streams at once race on
 * that counter. */
typedef struct {
  double* E_g;                /* [N_g][n] in/out */
  double* F_g;                /* [3][N_g][n] in/out */
  const double* rho;          /* [n] */
  double* e_gas;              /* [n] in/out */
  double* v;                  /* [3][n] in/out */
  const double* kappa_scale;  /* [n] or NULL */
  const double* S_g;          /* [N_g][n] or NULL */
  const double* guess;        /* [N_g+1][n] warm start or NULL */
  int32_t* iters;             /* [n] or NULL */
  int32_t* outer;             /* [n] or NULL */
  int32_t* status;            /* [n] or NULL */
  const double* group_edges;  /* [N_g+1] */
  const double* chi_lo;       /* [N_g] */
  const double* alpha_chi;    /* [N_g] or NULL */
  const double* chi_hi;       /* [N_g] or NULL */
  int64_t n_cells;
  int32_t n_groups;
  int32_t reserved;
  double dt;
  double c_hat;
  int32_t* trace;             /* [max_outer][n] out or NULL (as mgrhd_options.trace) */
  /* out of place, as mgrhd_options.E_g_out ... v_out: all four set, or all
   * four NULL (the patch is updated in place) */
  double* E_g_out;            /* [N_g][n] or NULL */
  double* F_g_out;            /* [3][N_g][n] or NULL */
  double* e_gas_out;          /* [n] or NULL */
  double* v_out;              /* [3][n] or NULL */
} mgrhd_patch;

typedef struct mgrhd_batch mgrhd_batch;

/* Validate the descriptors (host array of n_patches) and build the batch.
 * Returns 0 or MGRHD_E_*; *out is NULL on error. */
int mgrhd_batch_create(const mgrhd_patch* patches, int32_t n_patches, int32_t mean_mode,
                       const mgrhd_options* opt, mgrhd_batch** out);
/* Tuning knobs (see the autotuner): groups per lane (2 or 4), resident
 * workgroups per CU (0 = as many as fit), cells per work item.  Defaults:
 * 2, 0, 256 (with work items taken per workgroup, item scope 1).  A new
 * cells-per-item value rebuilds the device work list here (MGRHD_E_DEVICE if
 * that fails; the batch then refuses to run until a rebuild succeeds).  The
 * per-cell state machine is compiled for every lane count per cell (a wave
 * dispatches on its item's patch). */
int mgrhd_batch_set_tuning(mgrhd_batch* b, int32_t groups_per_lane, int32_t blocks_per_cu,
                           int64_t chunk_cells);
int mgrhd_batch_get_tuning(const mgrhd_batch* b, int32_t* groups_per_lane,
                           int32_t* blocks_per_cu, int64_t* chunk_cells);
/* Who takes a work item: 0 = one wave (each wave stages its patch's tables
 * in its own LDS slot); 1 or 2 = one workgroup (its four waves share the
 * item's cells through an LDS counter and one table slot, which leaves LDS
 * for three workgroups per CU; waves that run out of cells wait for the
 * item's last cells), compiled for 3 (scope 1, at 2 groups per lane) or 2
 * waves per SIMD (scope 2).  Default 1.  Changing it drops a captured graph.
 * get returns the scope or MGRHD_E_NULL. */
int mgrhd_batch_set_item_scope(mgrhd_batch* b, int32_t per_workgroup);
int32_t mgrhd_batch_get_item_scope(const mgrhd_batch* b);
/* Autotuner of the batch's launch shape: times a fixed list of candidate
 * tunings (groups per lane 2 or 4, items per wave or per workgroup, 256 or
 * 1024 cells per item) on copies of the first min(n, 1024) cells of every
 * patch, restored before each run, with HIP events on `stream`, and keeps the
 * fastest (as mgrhd_batch_set_tuning and mgrhd_batch_set_item_scope would).
 * The patches' own arrays are only read.  The copies and the sample's work
 * list are allocated for the call and freed before it returns (device memory
 * of about twice the sampled state); synchronous; drops a captured graph if
 * the tuning changes.  Returns 0 or MGRHD_E_*. */
int mgrhd_batch_tune(mgrhd_batch* b, mgrhd_stream_t stream);
/* Enqueue the counter reset and the persistent solver on `stream`. */
int mgrhd_batch_run(mgrhd_batch* b, mgrhd_stream_t stream);
/* Capture mgrhd_batch_run into a hipGraph kept by the batch; launch replays
 * it (capturing on first use). */
int mgrhd_batch_capture(mgrhd_batch* b, mgrhd_stream_t stream);
int mgrhd_batch_launch(mgrhd_batch* b, mgrhd_stream_t stream);
/* Total cells of the batch. */
int64_t mgrhd_batch_cells(const mgrhd_batch* b);
void mgrhd_batch_destroy(mgrhd_batch* b);

/* ---- Learned warm start --------------------------------------------------
 * A multilayer perceptron n_in -> n_hidden -> n_hidden -> n_hidden -> n_out
 * with SiLU activations, trained on (state, dt) -> (post-update T_gas, E_g)
 * pairs produced by mgrhd_source_update, whose prediction becomes the
 * Newton initial guess (opt->guess); plain Newton remains the fallback and
 * the result is the solver's whatever the guess.  Every product runs on the
 * matrix cores as BF16 x BF16 -> FP32; parameters, gradients and Adam moments
 * are FP32.  Matrices: features feature-major X[f * ld_x + row], outputs
 * and targets row-major Y[row * n_out + o].  All data pointers are DEVICE
 * pointers except the host buffers of get/set_params.
 * Features (n_in = 2 + 3 N_g): ln T, ln rho, ln(E_g/a T^4), |F_g|/(c E_g),
 * ln(c_hat dt chi_0E,g); outputs (n_out = 1 + N_g): ln(T_new/T),
 * ln(E_g,new/a T^4).  The handle owns its device buffers (allocated once in
 * create for up to max_rows rows per call).  n_hidden and n_out are at most
 * 256 (MGRHD_E_SIZE otherwise).  Weight gradients are summed over row blocks
 * with atomic adds, so gradients (and training) agree between runs to
 * rounding, not bit for bit. */
typedef struct mgrhd_mlp mgrhd_mlp;
int mgrhd_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, int64_t max_rows,
                     uint64_t seed, mgrhd_mlp** out);
int64_t mgrhd_mlp_num_params(const mgrhd_mlp* m);
/* which = 0: parameters, 1: last gradients; layout: W1..W4 (out x in,
 * row-major) then b1..b4 */
int mgrhd_mlp_get_params(const mgrhd_mlp* m, float* host, int32_t which);
int mgrhd_mlp_set_params(mgrhd_mlp* m, const float* host);
/* Save / load the network's parameters (FP32, the order of
 * mgrhd_mlp_get_params) with its dimensions, in a small binary file: an
 * 8-byte tag "MGRHDMLP", int32 version 1, int32 n_in, n_hidden, n_out, int64
 * n_params, then the parameters, in host byte order.  load accepts only a
 * file of this network's dimensions (MGRHD_E_SIZE otherwise); an unreadable
 * or unwritable file is MGRHD_E_OPTION.  The input/output normalisation
 * statistics belong to the caller.  Synchronous. */
int mgrhd_mlp_save(const mgrhd_mlp* m, const char* path);
int mgrhd_mlp_load(mgrhd_mlp* m, const char* path);
int mgrhd_mlp_forward(mgrhd_mlp* m, const float* X_fm, int64_t ld_x, int64_t rows, float* Y,
                      mgrhd_stream_t stream);
/* gradients of mean((Y - Y_target)^2) into the handle; loss_out (device, may
 * be NULL) receives the loss */
int mgrhd_mlp_gradients(mgrhd_mlp* m, const float* X_fm, int64_t ld_x, int64_t rows,
                        const float* Y_target, float* loss_out, mgrhd_stream_t stream);
int mgrhd_mlp_adam_step(mgrhd_mlp* m, float lr, mgrhd_stream_t stream);
int mgrhd_mlp_train_step(mgrhd_mlp* m, const float* X_fm, int64_t ld_x, int64_t rows,
                         const float* Y_target, float lr, float* loss_out, mgrhd_stream_t stream);
/* features X_fm[(2 + 3 N_g) x n] of a state, z-scored with (mean, inv_std) */
int mgrhd_mlp_features(const double* E_g, const double* F_g, const double* rho, const double* e_gas,
                       const double* v, int64_t n, const double* group_edges,
                       const mgrhd_opacity_params* opacity, double dt, double c_hat,
                       const mgrhd_options* opt, const float* mean, const float* inv_std,
                       float* X_fm, mgrhd_stream_t stream);
/* training targets Y[n x (1 + N_g)] from the state before and after an update */
int mgrhd_mlp_targets(const double* E_g, const double* F_g, const double* rho, const double* e_gas,
                      const double* v, int64_t n, const double* group_edges,
                      const mgrhd_opacity_params* opacity, double dt, double c_hat,
                      const mgrhd_options* opt, const double* E_new, const double* e_gas_new,
                      const double* v_new, float* Y, mgrhd_stream_t stream);
/* Newton guess from a normalised prediction Y_norm [n x (1+N_g)] (row-major)
 * de-normalised with y_mean, y_std [1+N_g]: guess_kind 0 writes
 * [(N_g+1) x n] (E_gas, R_g); guess_kind 1 writes E_gas alone, [n], for
 * mgrhd_options.guess_kind = 1. */
int mgrhd_mlp_guess(const double* E_g, const double* F_g, const double* rho, const double* e_gas,
                    const double* v, int64_t n, const double* group_edges,
                    const mgrhd_opacity_params* opacity, double dt, double c_hat,
                    const mgrhd_options* opt, const float* Y_norm, const float* y_mean,
                    const float* y_std, int32_t guess_kind, double* guess,
                    mgrhd_stream_t stream);
/* Fused inference: features, the three hidden layers, the output layer and
 * the Newton guess in one kernel, activations kept in LDS (BF16 matrix-core
 * products, FP32 accumulation; features formed in FP32).  Requires
 * n_hidden = 128, n_in = 2 + 3 N_g, n_out = 1 + N_g and N_g <= 138.  x_mean,
 * x_istd [n_in], y_mean, y_std [n_out]: the training normalisation (DEVICE).
 * guess_kind 1 computes the temperature output only and writes E_gas [n];
 * guess_kind 0 writes [(N_g+1) x n] (E_gas, R_g).  State arguments as
 * mgrhd_source_update.  Returns MGRHD_E_SIZE if the network does not fit. */
int mgrhd_mlp_infer(mgrhd_mlp* m, const double* E_g, const double* F_g, const double* rho,
                    const double* e_gas, const double* v, int64_t n_cells,
                    const double* group_edges, const mgrhd_opacity_params* opacity, double dt,
                    double c_hat, const mgrhd_options* opt, const float* x_mean,
                    const float* x_istd, const float* y_mean, const float* y_std,
                    int32_t guess_kind, double* guess, mgrhd_stream_t stream);
/* Warm start inside a batch (a13 with a14): attach a network to the batch's
 * patches of n_groups groups.  Every later mgrhd_batch_run / capture /
 * launch first runs, for each attached group count, one fused inference
 * launch over all of that count's work items, writing each patch's guess
 * into its own guess buffer (mgrhd_patch.guess, the layout of the batch's
 * guess_kind), and then the batched solve, which reads it; the inference
 * allocates nothing, so both sit in one captured graph.  The network and
 * statistics (device arrays as for mgrhd_mlp_infer) must outlive the batch's
 * use of them.  Re-attaching a count replaces its network; a captured graph
 * is dropped.  MGRHD_E_NULL (a NULL argument, or a patch of that count
 * without a guess buffer), MGRHD_E_SIZE (no patch of that count, or network
 * dimensions other than 2 + 3 N_g inputs, 1 + N_g outputs, width 128). */
int mgrhd_batch_attach_mlp(mgrhd_batch* b, int32_t n_groups, mgrhd_mlp* m,
                           const float* x_mean, const float* x_istd, const float* y_mean,
                           const float* y_std);
/* Enqueue only the attached networks' inference launches (their guesses into
 * the patches' guess buffers), without the solve. */
int mgrhd_batch_infer(mgrhd_batch* b, mgrhd_stream_t stream);
/* C = op(A) op(B) with the network's matrix-core kernel (FP32 in and out):
 * BF16 operands (fp32 = 0, v_mfma_f32_16x16x32_bf16) or FP32 operands
 * (fp32 = 1, v_mfma_f32_16x16x4_f32); FP32 accumulation either way. */
int mgrhd_mlp_gemm(const float* A, int32_t lda, int32_t trans_a, const float* B, int32_t ldb,
                   int32_t trans_b, float* C, int32_t ldc, int64_t M, int32_t N, int32_t K,
                   int32_t fp32, mgrhd_stream_t stream);
/* Checking path of the training kernels: on = 1 keeps the operands of every
 * forward and backward product of the handle in FP32 (the FP32 matrix-core
 * form) instead of rounding them to BF16, so that gradients can be compared
 * with an FP64 reference at FP32 accuracy; 0 (the default) restores BF16.
 * The fused inference (mgrhd_mlp_infer) always uses BF16.  MGRHD_E_NULL,
 * MGRHD_E_OPTION for other values. */
int mgrhd_mlp_set_fp32_products(mgrhd_mlp* m, int32_t on);
void mgrhd_mlp_destroy(mgrhd_mlp* m);

/* Library version string. */
const char* mgrhd_version(void);

#ifdef __cplusplus
}
#endif
#endif
