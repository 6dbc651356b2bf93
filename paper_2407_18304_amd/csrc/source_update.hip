// source_update.hip -- gfx950 kernels and C ABI of the multigroup
// matter-radiation source update (He, Wibking & Krumholz 2024, Sec. 3).
//
// Work decomposition.  LPC consecutive lanes of a wavefront own one cell (a
// "cell group"); its N_g groups are dealt to the lanes in turn, slot k of lane
// j holding group k*LPC + j (G slots per lane), so that at each slot a wave
// evaluates Planck edges in a narrow band of x and mostly takes one branch.
// Registers hold the Newton unknowns R_g, E_g^(t)+S_g and v.F_g of the
// current outer pass; the fluxes F_g of the pass, the per-cell constants
// 1/tau_g, 1/J_gg and the old-time F_g^(t), v^(t) sit in per-lane LDS slots.
// Group sums (sum R_g, sum |F_R,g|, the two sums of the arrowhead
// elimination, the momentum change, the outer test) are butterflies inside
// the LPC lanes (DPP where the distance fits a row), so every lane of a cell
// holds bit-identical scalars and takes the same branches.
//
// Persistent state machine.  Each workgroup owns a contiguous range of cells,
// which its waves take through a counter in LDS.  One
// trip of the main loop performs exactly one material evaluation (G Planck
// edges, one edge handed over from a neighbour lane, and G group means per
// lane) for every active cell group, followed by
// the consumer of the cell's phase: a Newton step, or the flux/momentum
// update of the outer stage.  The flux-stage evaluation is also the first
// evaluation of the next inner pass (the pass restarts at the same
// temperature).  A cell group whose cell has finished takes the next cell of
// the workgroup's range at the top of the next trip, so cells that converge
// early free their lanes instead of idling until the slowest cell of the wave
// is done.
//
// Kernel tables.  Each variant is compiled four times: for a T-independent or
// T-dependent opacity, and for any N_g or N_g = LPC * G (every slot holds a
// group, so the per-slot group checks compile away); the launcher picks the
// N_g = LPC * G kernel whenever the group count fills the variant exactly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "../../include/mgrhd.h"

#include "solver_kernel.hpp"

namespace mgrhd {

// ---------------------------------------------------------------------------
// Variant table
struct Variant {
  int lpc, g, wpe;  // lanes per cell, groups per lane, minimum waves per SIMD
  // [temperature-dependent opacity][N_g = lpc * g][mean mode]
  KernelFn fn[2][2][3];
  int blocks_per_cu[2][2][3];
};

#define MGRHD_VARIANT(G_, LPC_, WPE_) \
  {LPC_, G_, WPE_, {{MGRHD_VARIANT_MODES(G_, LPC_, WPE_, false, false), {}}, {}}, {}},
static Variant kVariants[] = {MGRHD_FOR_EACH_VARIANT(MGRHD_VARIANT)};
#undef MGRHD_VARIANT
constexpr int kNumVariants = (int)(sizeof(kVariants) / sizeof(kVariants[0]));

// the other kernels come from their own translation units
static void link_kernels() {
  static std::once_flag once;
  std::call_once(once, [] {
    for (int k = 0; k < kNumVariants; ++k)
      for (int m = 0; m < 3; ++m) {
        kVariants[k].fn[1][0][m] = tdep_kernel(k, m);
        kVariants[k].fn[0][1][m] = full_kernel(k, m);
        kVariants[k].fn[1][1][m] = tdep_full_kernel(k, m);
      }
  });
}

// user overrides per group count (0 = built-in choice)
static int g_override_lpc[MGRHD_MAX_GROUPS + 1];
static int g_override_g[MGRHD_MAX_GROUPS + 1];
static int g_override_wpe[MGRHD_MAX_GROUPS + 1];
static std::mutex g_mutex;

// wpe = 0: the default register budget of (lpc, g)
static Variant* find_variant(int lpc, int g, int wpe) {
  for (Variant& v : kVariants)
    if (v.lpc == lpc && v.g == g && (wpe == 0 || v.wpe == wpe)) return &v;
  return nullptr;
}

static Variant* choose_variant(int ng) {
  if (g_override_lpc[ng]) {
    Variant* v = find_variant(g_override_lpc[ng], g_override_g[ng], g_override_wpe[ng]);
    if (v && v->lpc * v->g >= ng) return v;
  }
  // default: 2 groups per lane at 3 waves per SIMD and enough lanes to cover
  // N_g (the fastest on gfx950 at 16 and 64 groups); 4 groups per lane where
  // no 2-group variant covers N_g
  int lpc = 1;
  while (lpc * 2 < ng) lpc <<= 1;
  if (Variant* v = find_variant(lpc, 2, 0)) return v;
  lpc = 1;
  while (lpc * 4 < ng) lpc <<= 1;
  return find_variant(lpc, 4, 0);
}

// resident workgroups per CU of a variant (queried once)
static int resident_blocks(Variant* v, int td, int full, int mode) {
  std::lock_guard<std::mutex> lk(g_mutex);
  int& nb = v->blocks_per_cu[td][full][mode];
  if (nb == 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, v->fn[td][full][mode], kBlock, 0) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
  }
  return nb;
}

static int num_cus() {
  static int cus = 0;
  std::lock_guard<std::mutex> lk(g_mutex);
  if (cus == 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      cus = prop.multiProcessorCount;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

}  // namespace mgrhd

using namespace mgrhd;

extern "C" {

const char* mgrhd_version(void) { return "mgrhd 0.2 (gfx950, fp64, persistent)"; }

void mgrhd_default_options(mgrhd_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->c = 1.0;
  o->a_rad = 1.0;
  o->h_over_k = 1.0;
  o->c_v = 1.5;
  o->eps_newton = 1e-11;
  o->eps_outer = 1e-13;
  o->max_newton = 100;
  o->max_outer = 20;
  o->closure = MGRHD_CLOSURE_M1;
  o->polish = 0;
}

int mgrhd_get_variant(int32_t n_groups, int32_t mean_mode, int32_t* lpc, int32_t* gpl,
                      int32_t* waves_per_simd) {
  (void)mean_mode;
  if (n_groups < 1 || n_groups > MGRHD_MAX_GROUPS) return MGRHD_E_SIZE;
  const Variant* v = choose_variant(n_groups);
  if (!v) return MGRHD_E_OPTION;
  if (lpc) *lpc = v->lpc;
  if (gpl) *gpl = v->g;
  if (waves_per_simd) *waves_per_simd = v->wpe;
  return 0;
}

int32_t mgrhd_variant_count(void) { return kNumVariants; }

int32_t mgrhd_recommend_mean_mode(int32_t n_groups, const double* edges) {
  if (!edges) return MGRHD_E_NULL;
  if (n_groups < 1 || n_groups > MGRHD_MAX_GROUPS) return MGRHD_E_SIZE;
  for (int32_t g = 0; g < n_groups; ++g)
    if (!(edges[g] >= 0.0) || !(edges[g + 1] > edges[g])) return MGRHD_E_TABLE;
  // a grid reaching 0 or infinity has no finite log width: only PC is defined
  if (!(edges[0] > 0.0) || !std::isfinite(edges[n_groups])) return MGRHD_MEAN_PC;
  const double W = std::log(edges[n_groups] / edges[0]);
  double widest = 0.0;
  for (int32_t g = 0; g < n_groups; ++g)
    widest = std::max(widest, std::log(edges[g + 1] / edges[g]));
  return widest < 0.1 * W ? MGRHD_MEAN_PC : MGRHD_MEAN_PPL_FIXED;
}

int mgrhd_variant_info(int32_t k, int32_t* lpc, int32_t* gpl, int32_t* waves_per_simd) {
  if (k < 0 || k >= mgrhd_variant_count()) return MGRHD_E_OPTION;
  if (lpc) *lpc = kVariants[k].lpc;
  if (gpl) *gpl = kVariants[k].g;
  if (waves_per_simd) *waves_per_simd = kVariants[k].wpe;
  return 0;
}

int mgrhd_set_variant(int32_t n_groups, int32_t lpc, int32_t gpl, int32_t waves_per_simd) {
  if (n_groups < 1 || n_groups > MGRHD_MAX_GROUPS) return MGRHD_E_SIZE;
  if (lpc == 0 && gpl == 0) {
    g_override_lpc[n_groups] = g_override_g[n_groups] = g_override_wpe[n_groups] = 0;
    return 0;
  }
  const Variant* v = find_variant(lpc, gpl, waves_per_simd);
  if (!v || v->lpc * v->g < n_groups) return MGRHD_E_OPTION;
  g_override_lpc[n_groups] = lpc;
  g_override_g[n_groups] = gpl;
  g_override_wpe[n_groups] = v->wpe;
  return 0;
}

int mgrhd_source_update(double* E_g, double* F_g, const double* rho, double* e_gas, double* v,
                        int64_t n_cells, const double* group_edges,
                        const mgrhd_opacity_params* op, double dt, double c_hat,
                        mgrhd_stream_t stream, const mgrhd_options* opt_in) {
  mgrhd_options defaults;
  mgrhd_default_options(&defaults);
  const mgrhd_options* opt = opt_in ? opt_in : &defaults;
  if (!op) return MGRHD_E_NULL;
  if (n_cells < 0) return MGRHD_E_SIZE;
  const int ng = op->n_groups;
  if (ng < 1 || ng > MGRHD_MAX_GROUPS) return MGRHD_E_SIZE;
  if (op->mean_mode < 0 || op->mean_mode > 2) return MGRHD_E_MODE;
  if (opt->closure < 0 || opt->closure > 1) return MGRHD_E_MODE;
  const int n_out = !!opt->E_g_out + !!opt->F_g_out + !!opt->e_gas_out + !!opt->v_out;
  if (n_out != 0 && n_out != 4) return MGRHD_E_NULL;  // out of place needs all four
  if (n_cells == 0) return 0;
  if (!E_g || !F_g || !rho || !e_gas || !v || !group_edges || !op->chi_lo) return MGRHD_E_NULL;
  if (op->mean_mode != MGRHD_MEAN_PC && !op->alpha_chi && !op->chi_hi) return MGRHD_E_TABLE;
  auto pos = [](double x) { return x > 0.0 && std::isfinite(x); };
  if (!pos(dt) || !pos(c_hat) || !pos(opt->c) || !pos(opt->a_rad) || !pos(opt->h_over_k) ||
      !pos(opt->c_v))
    return MGRHD_E_SCALAR;
  if (!pos(opt->eps_newton) || !pos(opt->eps_outer) || opt->max_newton < 1 ||
      opt->max_outer < 1 || opt->polish < 0 || opt->polish > 4 || opt->guess_kind < 0 ||
      opt->guess_kind > 1)
    return MGRHD_E_OPTION;
  if (!std::isfinite(op->t_exp) || (op->t_exp != 0.0 && !pos(op->t_ref)) || op->stim < 0 ||
      op->stim > 1)
    return MGRHD_E_TABLE;
  const int td = (op->t_exp != 0.0 || op->stim != 0) ? 1 : 0;

  Variant* var = choose_variant(ng);
  if (!var) return MGRHD_E_OPTION;
  link_kernels();

  KArgs a;
  std::memset(&a, 0, sizeof(a));
  a.E = E_g;
  a.F = F_g;
  a.rho = rho;
  a.egas = e_gas;
  a.v = v;
  if (n_out == 4) {
    a.Eo = opt->E_g_out;
    a.Fo = opt->F_g_out;
    a.egaso = opt->e_gas_out;
    a.vo = opt->v_out;
  }
  a.kappa = op->kappa_scale;
  a.S = opt->S_g;
  a.guess = opt->guess;
  a.guess_kind = opt->guess_kind;
  a.iters = opt->iters;
  a.outer = opt->outer;
  a.status = opt->status;
  a.trace = opt->trace;
  a.edges = group_edges;
  a.chi_lo = op->chi_lo;
  a.alpha = op->alpha_chi;
  a.chi_hi = op->chi_hi;
  a.n = n_cells;
  a.ng = ng;
  a.closure = opt->closure;
  a.dt = dt;
  a.chat = c_hat;
  a.c = opt->c;
  a.a = opt->a_rad;
  a.hk = opt->h_over_k;
  a.cv = opt->c_v;
  a.eps = opt->eps_newton;
  a.eps_out = opt->eps_outer;
  a.max_newton = opt->max_newton;
  a.max_outer = opt->max_outer;
  a.polish = opt->polish;
  a.t_exp = op->t_exp;
  a.itref = op->t_exp != 0.0 ? 1.0 / op->t_ref : 1.0;
  a.stim = op->stim;
  set_derived(a);

  // persistent grid: one resident wave of workgroups, never more workgroups
  // than there are cell groups to fill them
  const int64_t needed = (n_cells * var->lpc + kBlock - 1) / kBlock;
  const int full = var->lpc * var->g == ng ? 1 : 0;  // every slot holds a group
  const int64_t resident =
      (int64_t)num_cus() * resident_blocks(var, td, full, op->mean_mode);
  const int64_t blocks = needed < resident ? needed : resident;
  hipLaunchKernelGGL(var->fn[td][full][op->mean_mode], dim3((unsigned)blocks), dim3(kBlock), 0,
                     (hipStream_t)stream, a);
  const hipError_t err = hipGetLastError();
  return err == hipSuccess ? 0 : (int)err;
}

}  // extern "C"
