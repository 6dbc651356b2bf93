// solver_device.hpp -- device side of the multigroup source update shared by
// the single-table kernel (source_update.hip) and the batched patch kernel
// (batch.hip): group tables in LDS, material evaluation, the Newton and
// outer-stage consumers, and the per-cell state machine.
//
// A "cell group" of LPC consecutive lanes owns one cell; its groups are dealt
// to the lanes in turn, slot k of lane j holding group k*LPC + j (see gidx).
// The lane count per cell is a template
// parameter in the single-table kernel and a run-time value (uniform over the
// wave) in the batched kernel: LPC = 0 in the templates below means "read
// lpc at run time".
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/mgrhd.h"
#include "planck_device.hpp"

namespace mgrhd {

struct KArgs {
  double* E;  // inputs (in place: also the outputs)
  double* F;
  const double* rho;
  double* egas;
  double* v;
  double* Eo;  // outputs: the inputs for an update in place
  double* Fo;
  double* egaso;
  double* vo;
  const double* kappa;
  const double* S;
  const double* guess;
  int32_t* iters;
  int32_t* outer;
  int32_t* status;
  int32_t* trace;  // [max_outer][n] cumulative Newton steps per inner pass, or NULL
  const double* edges;
  const double* chi_lo;
  const double* alpha;
  const double* chi_hi;
  int64_t n;
  int32_t ng;
  int32_t closure;
  double dt, chat, c, a, hk, cv, eps, eps_out;
  int32_t max_newton, max_outer, polish, guess_kind;
  // derived on the host (set_derived): c/c_hat, c_hat/c, c_hat dt, 1/c^2,
  // 1/(c c_hat), c_hat dt / c^2
  double cc, icc, cdt, ic2, iccc, cdt_ic2;
  // temperature dependence of the opacity: (T/T_ref)^t_exp [1 - e^{-x}]^stim
  double t_exp, itref;  // itref = 1/T_ref
  int32_t stim, pad;
};

// Fill the derived constants of a (host side); outputs left NULL are the
// inputs (an update in place).
inline void set_derived(KArgs& a) {
  if (!a.Eo) {
    a.Eo = a.E;
    a.Fo = a.F;
    a.egaso = a.egas;
    a.vo = a.v;
  }
  a.cc = a.c / a.chat;
  a.icc = a.chat / a.c;
  a.cdt = a.chat * a.dt;
  a.ic2 = 1.0 / (a.c * a.c);
  a.iccc = 1.0 / (a.c * a.chat);
  a.cdt_ic2 = a.cdt * a.ic2;
}

// The argument block of a launch where the device can read it with scalar
// loads: the kernel-argument segment (single-table kernel) or the batch's
// device array of patch arguments (never a copy in private memory).  The
// arrays a cell needs once, at its load or its store, are read through it
// (state_ptrs, arg_at_use).
typedef const KArgs __attribute__((address_space(4)))* KArgsRef;

// The state arrays of a launch, read from its argument block where a finished
// cell needs them: the block's address passes through an empty asm, so the
// scalar loads stay at the use (once per finished cell) instead of being
// hoisted out of the persistent loop, where the eight pointers would hold
// sixteen scalar registers for the whole kernel (which spilled 74 of them).
struct StatePtrs {
  const double *E, *F, *egas, *v;  // inputs
  double *Eo, *Fo, *egaso, *vo;     // outputs (the inputs for an update in place)
};
__device__ __forceinline__ StatePtrs state_ptrs(KArgsRef ap) {
  asm volatile("" : "+s"(ap));
  return StatePtrs{ap->E, ap->F, ap->egas, ap->v, ap->Eo, ap->Fo, ap->egaso, ap->vo};
}

// One field of the argument block, read where it is used (as state_ptrs).
// The batched kernels read the constants of a Newton step or an outer stage
// this way too (LaneStore::cst): a patch's arguments live in device memory,
// and held across the loop they spilled hundreds of scalar registers (the
// batched launch over 2000 patches: 631 -> 542 ms); in the single-table
// kernel the scalar loads' waits cost more than its few spills (1%).
template <class T>
__device__ __forceinline__ T arg_at_use(KArgsRef ap, T KArgs::*m) {
  asm volatile("" : "+s"(ap));
  return ap->*m;
}

// Out of place: the input state of cell i copied to the outputs, for a cell
// the update leaves untouched (lane j of the cell's lpc lanes copies rows
// j, j + lpc, ...).  Each array is copied unless its output is the input
// itself (an update may be in place for some arrays and not for others).
__device__ __forceinline__ void copy_through(const KArgs& a, const StatePtrs& p, int64_t i,
                                             int j, int lpc) {
  const int64_t n = a.n;
  const int ng = a.ng;
  for (int r = j; r < 4 * ng + 4; r += lpc) {
    if (r < ng) {
      if (p.Eo != p.E) p.Eo[(int64_t)r * n + i] = p.E[(int64_t)r * n + i];
    } else if (r < 4 * ng) {
      const int64_t q = (int64_t)(r - ng) * n + i;
      if (p.Fo != p.F) p.Fo[q] = p.F[q];
    } else if (r == 4 * ng) {
      if (p.egaso != p.egas) p.egaso[i] = p.egas[i];
    } else {
      const int64_t q = (int64_t)(r - 4 * ng - 1) * n + i;
      if (p.vo != p.v) p.vo[q] = p.v[q];
    }
  }
}

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr double kThird = 1.0 / 3.0;

// LDS copy of the group tables with per-group constants (NGM = G * LPC).
template <int NGM>
struct Tables {
  double nu[NGM + 1];
  double lnr[NGM];    // ln(nu_g+ / nu_g-)
  double achi[NGM];   // opacity powerlaw index (0 in PC)
  double chit[NGM];   // chi_lo table entry (per unit rho * kappa)
  double mfix[NGM];   // PPL-fixed mean ratio chi_0B/chi_0,g- = chi_0E/chi_0,g-
  double chk[NGM];    // PC / PPL-fixed group mean per unit rho * kappa (chit, or chit * mfix)
  double rac[NGM];    // r_g^alpha_chi
  double lndnu[NGM];  // ln(nu_g+ - nu_g-)
  double lnc[NGM];    // (ln nu_g- + ln nu_g+)/2
  int bad;
};

// Lane exchange inside a row of 16 lanes through the DPP crossbar (no LDS
// round trip).  All lanes of one cell group are active together, so the
// source lane is always active, and the destination needs no prior value
// (bound_ctrl: a lane with no source would read 0).
template <int CTRL>
__device__ __forceinline__ double dpp_swap(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Exchange of a value between the 16-lane rows r and r^1 (M = 16) or r^2
// (M = 32) of the wave, same column, by the gfx950 row swaps: with both
// operands holding v, v_permlane16_swap leaves one of the two results holding
// the lane's own value and the other its partner's (the even rows of the
// first operand are swapped with the odd rows of the second; v_permlane32_swap
// likewise for rows 0-1 and 2-3), so their sum is the pair's sum in every lane.
template <int M>
__device__ __forceinline__ double row_swap_sum(double v) {
  const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
  if (M == 16) {
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
  }
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}

// One butterfly level of the group sum: partner lane at distance m.  Levels
// 1 and 2 pair lanes i and i^m (quad permutations); levels 4 and 8 pair lane
// i with the mirror image of i in its 8- or 16-lane block, which holds the
// same partial sum as lane i^m after the lower levels, so every lane adds the
// same two partial sums as the xor butterfly.  Levels 16 and 32 swap whole
// rows (no LDS round trip).
template <int M>
__device__ __forceinline__ double butterfly(double v) {
  if (M == 1) return v + dpp_swap<0xB1>(v);   // quad_perm [1,0,3,2]
  if (M == 2) return v + dpp_swap<0x4E>(v);   // quad_perm [2,3,0,1]
  if (M == 4) return v + dpp_swap<0x141>(v);  // row_half_mirror
  if (M == 8) return v + dpp_swap<0x140>(v);  // row_mirror
  return row_swap_sum<M>(v);
}

// Sum over the lanes of one cell group (bit-identical in every lane).  LPC = 0:
// the group size lpc is a run-time value, uniform over the wave.
template <int LPC>
__device__ __forceinline__ double cell_sum(double v, int lpc) {
  const int n = LPC > 0 ? LPC : lpc;
  if (n >= 2) v = butterfly<1>(v);
  if (n >= 4) v = butterfly<2>(v);
  if (n >= 8) v = butterfly<4>(v);
  if (n >= 16) v = butterfly<8>(v);
  if (n >= 32) v = butterfly<16>(v);
  if (n >= 64) v = butterfly<32>(v);
  return v;
}

// Group held by slot k of lane j.  Dealing the groups to the lanes in turn
// puts adjacent groups on adjacent lanes at every slot, so at one slot the
// cells of a wave evaluate their Planck edges in a narrow band of
// x = h nu / kT and mostly take the same branch (all below the Wien side at
// the first slots, all on it at the last ones).
template <int LPC>
__device__ __forceinline__ int gidx(int j, int k, int lpc) {
  return k * (LPC > 0 ? LPC : lpc) + j;
}

// Value held by lane (j - 1) mod lpc, resp. (j + 1) mod lpc, of this lane's
// cell group.  Every lane of the group must execute it (all are active
// together).  DPP quad permutations and row rotations where they fit the
// group, the LDS crossbar otherwise (DPP rotations fixed up at the group's
// ends measured slower: more scalar registers for the lane masks).
template <int LPC>
__device__ __forceinline__ double from_left(double v, int lpc) {
  const int n = LPC > 0 ? LPC : lpc;
  if (n == 1) return v;
  if (n == 2) return dpp_swap<0xB1>(v);   // quad_perm [1,0,3,2]
  if (n == 4) return dpp_swap<0x93>(v);   // quad_perm [3,0,1,2]
  if (n == 16) return dpp_swap<0x121>(v); // row_ror:1
  const int lane = __lane_id();
  const int base = lane & ~(n - 1);
  return __shfl(v, base + ((lane - base + n - 1) & (n - 1)), kWave);
}
template <int LPC>
__device__ __forceinline__ double from_right(double v, int lpc) {
  const int n = LPC > 0 ? LPC : lpc;
  if (n == 1) return v;
  if (n == 2) return dpp_swap<0xB1>(v);   // quad_perm [1,0,3,2]
  if (n == 4) return dpp_swap<0x39>(v);   // quad_perm [1,2,3,0]
  if (n == 16) return dpp_swap<0x12F>(v); // row_ror:15
  const int lane = __lane_id();
  const int base = lane & ~(n - 1);
  return __shfl(v, base + ((lane - base + 1) & (n - 1)), kWave);
}

// Table entries of group g (edges already staged in t.nu); false if the
// group's table is unusable.
template <int NGM, int MODE>
__device__ __forceinline__ bool table_group(const KArgs& a, Tables<NGM>& t, int g) {
  const double lo = t.nu[g], hi = t.nu[g + 1];
  const double chl = a.chi_lo[g];
  bool ok = hi > lo && chl > 0.0 && !is_pinf(chl);
  double L = 0.0, ac = 0.0, mf = 1.0, rac = 1.0, ldn = 0.0, lc = 0.0;
  if (MODE != MGRHD_MEAN_PC) {
    L = log(hi / lo);
    if (a.alpha) {
      ac = a.alpha[g];
    } else {
      const double chh = a.chi_hi[g];
      ok = ok && chh > 0.0 && !is_pinf(chh);
      ac = log(chh / chl) / L;  // tabulated opacity: index from the edge values
    }
    ok = ok && isfinite(ac);
    mf = mean_ratio(ac, -1.0, L);
    rac = exp(ac * L);
    ldn = log(hi - lo);
    lc = 0.5 * (log(lo) + log(hi));
  }
  t.lnr[g] = L;
  t.achi[g] = ac;
  t.chit[g] = chl;
  t.mfix[g] = mf;
  t.chk[g] = (MODE == MGRHD_MEAN_PC) ? chl : chl * mf;
  t.rac[g] = rac;
  t.lndnu[g] = ldn;
  t.lnc[g] = lc;
  return ok;
}

// Edge g of the table; false if unusable.
template <int NGM, int MODE>
__device__ __forceinline__ bool table_edge(const KArgs& a, Tables<NGM>& t, int g) {
  const double nu = a.edges[g];
  t.nu[g] = nu;
  bool ok = nu >= 0.0;
  if (MODE != MGRHD_MEAN_PC) ok = ok && nu > 0.0 && !is_pinf(nu);
  if (a.stim && g == 0) ok = ok && nu > 0.0;  // 1 - e^{-x} vanishes at x = 0
  return ok;
}

// Stage the tables in LDS (whole workgroup).
template <int NGM, int MODE>
__device__ __forceinline__ bool stage_tables(const KArgs& a, Tables<NGM>& t) {
  if (threadIdx.x == 0) t.bad = 0;
  __syncthreads();
  for (int g = threadIdx.x; g <= a.ng; g += blockDim.x)
    if (!table_edge<NGM, MODE>(a, t, g)) atomicOr(&t.bad, 1);
  __syncthreads();
  for (int g = threadIdx.x; g < a.ng; g += blockDim.x)
    if (!table_group<NGM, MODE>(a, t, g)) atomicOr(&t.bad, 1);
  __syncthreads();
  return t.bad == 0;
}

// Per-lane values held in LDS instead of registers: the fluxes F_k of the
// lane's groups during the outer iteration (3G), in PC and PPL-fixed the
// per-cell constants 1/tau_g = 1/(c_hat dt chi_0E,g) and 1/J_gg of eq. matrix
// (2G), and with KEEP0 the old-time fluxes F^(t) (3G) that every outer stage
// needs (without KEEP0 they are re-read from HBM).  Slot s of thread t lives
// at lds[s * kBlock + t]: the 64 lanes of a wave touch 64 consecutive words,
// free of bank conflicts.  Per-cell values (with KEEP0 the old-time velocity
// v^(t)) live once per cell, not once per lane: field f of cell slot c at
// cells[f * CPB + c], CPB the most cells a workgroup holds at once (kBlock /
// lanes per cell, or kBlock where the lane count varies between waves); all
// lanes of a cell read the same word (an LDS broadcast).
template <int G, bool KEEP0, int CPB = kBlock, bool CONST_AT_USE = false>
struct LaneStore {
  static constexpr bool kKeep0 = KEEP0;
  static constexpr int kSlots = 5 * G + (KEEP0 ? 3 * G : 0);
  static constexpr int kCPB = CPB;
  static constexpr int kCellWords = (KEEP0 ? 3 : 1) * CPB;  // (one unused word-row without)
  double* base;   // &lds[threadIdx.x]
  double* cells;  // the cell area; at_cell() points it at one cell's slot
  KArgsRef args;  // the launch's argument block (state_ptrs)
  __device__ __forceinline__ LaneStore at_cell(int c) const {
    return LaneStore{base, cells + c, args};
  }
  __device__ __forceinline__ LaneStore with_args(KArgsRef ap) const {
    return LaneStore{base, cells, ap};
  }
  // a field of the launch's arguments, read where it is used (arg_at_use)
  template <class T>
  __device__ __forceinline__ T arg(T KArgs::*m) const {
    return arg_at_use(args, m);
  }
  // a constant of the launch (c/c_hat, the tolerances, ...): read where it is
  // used with CONST_AT_USE (the batched kernels), else from a as the
  // compiler likes (the single-table kernel, where it stays in registers)
  template <class T>
  __device__ __forceinline__ T cst(const KArgs& a, T KArgs::*m) const {
    if constexpr (CONST_AT_USE)
      return arg_at_use(args, m);
    else
      return a.*m;
  }
  __device__ __forceinline__ double& F(int d, int k) const { return base[(d * G + k) * kBlock]; }
  __device__ __forceinline__ double& itau(int k) const { return base[(3 * G + k) * kBlock]; }
  __device__ __forceinline__ double& iJgg(int k) const { return base[(4 * G + k) * kBlock]; }
  __device__ __forceinline__ double& F0(int d, int k) const {
    return base[(5 * G + d * G + k) * kBlock];
  }
  __device__ __forceinline__ double& v0(int d) const { return cells[d * CPB]; }
};

// Material data of this lane's groups at one temperature.
template <int G>
struct Cache {
  double Bt[G];    // B~_g
  double dBdT[G];  // dB~_g/dT
  double chiF[G];  // flux mean (eq. chiDiff)
  double emit[G];  // chi_0B B~_g - Delta_g(nu chi_0 B~)/3  (flux source, eq. numF1)
  double chiB[G];  // PPL-free only (otherwise the per-cell constants)
  double chiE[G];  // PPL-free, and every mode with a T-dependent opacity
  double ac[G];    // opacity index at this temperature (T-dependent opacity only)
};

// Appendix A slopes of the lane's groups from ln Qbar (lq, per slot).  The
// neighbours of group g = k lpc + j are on lanes j -+ 1 at the same slot, or
// on the last (first) lane at the previous (next) slot.
template <int G, int LPC, int NGM>
__device__ __forceinline__ void slopes_free(const Tables<NGM>& t, int ng, int j, int lpc,
                                            const double* lq, double* alpha) {
  const int n = LPC > 0 ? LPC : lpc;
#pragma unroll
  for (int k = 0; k < G; ++k) {
    const double lm = from_left<LPC>((j == n - 1) ? (k > 0 ? lq[k - 1] : -INFINITY) : lq[k], lpc);
    const double lp = from_right<LPC>((j == 0) ? (k < G - 1 ? lq[k + 1] : -INFINITY) : lq[k], lpc);
    const int g = gidx<LPC>(j, k, lpc);
    alpha[k] = -1.0;
    if (g <= 0 || g >= ng - 1) continue;
    const double sl = (lq[k] - lm) / (t.lnc[g] - t.lnc[g - 1]);
    const double sr = (lp - lq[k]) / (t.lnc[g + 1] - t.lnc[g]);
    if (isnan(sl) || isnan(sr)) continue;
    const double m = minmod(sl, sr);
    if (isfinite(m)) alpha[k] = m;
  }
}

// Low edge of slot k's group: the high edge of lane j - 1 at this slot, or,
// on lane 0, the high edge of the last lane at the previous slot (kept in
// `prev`; edge 0 before slot 0).  The wien/inf flags follow from x.
template <int LPC>
__device__ __forceinline__ Edge low_edge(const Edge& hi, const Edge& prev, double x_lo, int j,
                                         int lpc) {
  const int n = LPC > 0 ? LPC : lpc;
  const bool last = j == n - 1;
  Edge lo;
  lo.x = x_lo;  // the same product the neighbour formed for its upper edge
  lo.u = from_left<LPC>(last ? prev.u : hi.u, lpc);
  lo.val = from_left<LPC>(last ? prev.val : hi.val, lpc);
  lo.eps = from_left<LPC>(last ? prev.eps : hi.eps, lpc);
  lo.wien = lo.x > kPlanckSplit;
  lo.inf = is_pinf(lo.x);
  return lo;
}

// Temperature dependence of the opacity at one evaluation: fT = (T/T_ref)^beta
// and whether the stimulated-emission factor 1 - e^{-x} applies.
struct OpacityT {
  double fT;
  bool stim;
};

// One material evaluation: Planck data, slopes (PPL-free), group means.
// Without temperature dependence (TD false) chi_0E = chi_0B = rho kappa chk_g
// is fixed per cell in PC and PPL-fixed.  With it (TD), the opacity at the
// group's lower edge is rho kappa chit_g fT [1 - e^{-x_g-}], and in the PPL
// modes the group's index passes through the T-dependent values at both
// edges, alpha_g + ln(s_g+/s_g-)/ln r_g, which makes r^alpha follow as
// r^alpha_g s_g+/s_g-; the means of eq. chiQg are then taken at that index.
template <int G, int LPC, int MODE, int NGM, bool TD = false>
__device__ __forceinline__ void evaluate(const Tables<NGM>& t, int ng, int j, int lpc, double T,
                                         double aT4, double hk, double rho_kappa,
                                         const double* Ecur, Cache<G>& c,
                                         OpacityT ot = OpacityT{1.0, false}) {
  const int n = LPC > 0 ? LPC : lpc;
  const double invT = 1.0 / T;
  const double hkT = hk * invT;
  Edge prev;
  prev.x = prev.u = prev.val = prev.eps = prev.eb = 0.0;
  if (j == n - 1) prev = planck_edge_low(hkT * t.nu[0]);  // edge 0, handed to lane 0
  // stimulated-emission factor of the previous slot's high edge (edge 0 first)
  double prev_s = 1.0;
  if (TD && ot.stim && j == n - 1) prev_s = stim_factor(prev);
  const bool last = j == n - 1;
  if (MODE != MGRHD_MEAN_PPL_FREE) {
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int g = gidx<LPC>(j, k, lpc);
      const Edge hi = planck_edge(hkT * t.nu[min(g + 1, ng)]);
      const Edge lo = low_edge<LPC>(hi, prev, hkT * t.nu[min(g, ng)], j, lpc);
      prev = hi;
      double s_lo = 1.0, s_hi = 1.0;
      if (TD && ot.stim) {
        s_hi = stim_factor(hi);
        s_lo = from_left<LPC>(last ? prev_s : s_hi, lpc);
        prev_s = s_hi;
      }
      if (g >= ng) continue;
      const GroupPlanck p = group_planck(lo, hi);
      const double Bt = aT4 * p.b * p.scale;
      const double Dnu = aT4 * (p.ehi - p.elo) * p.scale;
      c.Bt[k] = Bt;
      c.dBdT[k] = (4.0 * Bt - Dnu) * invT;
      if (!TD) {
        const double ch = rho_kappa * t.chk[g];
        if (MODE == MGRHD_MEAN_PC) {
          c.chiF[k] = ch;
          c.emit[k] = ch * (Bt - Dnu * kThird);
        } else {
          const double ac = t.achi[g];
          const double dchib = rho_kappa * t.chit[g] * (t.rac[g] * p.ehi - p.elo);
          // eq. chiDiff with numerator and denominator both multiplied by 3
          const double num = (4.0 + ac) * ch * p.b - dchib;
          const double den = 4.0 * p.b - (p.ehi - p.elo);
          const double f = num / den;
          c.chiF[k] = (den > 0.0 && isfinite(f)) ? f : ch;
          c.emit[k] = ch * Bt - aT4 * dchib * p.scale * kThird;
        }
      } else {
        const double chl = rho_kappa * t.chit[g] * ot.fT * s_lo;  // chi_0,g- at T
        if (MODE == MGRHD_MEAN_PC) {
          c.chiE[k] = chl;
          c.ac[k] = 0.0;
          c.chiF[k] = chl;
          c.emit[k] = chl * (Bt - Dnu * kThird);
        } else {
          double ac = t.achi[g], rac = t.rac[g], mr = t.mfix[g];
          if (ot.stim) {
            const double q = s_hi / s_lo;
            ac += log(q) / t.lnr[g];
            rac *= q;
            mr = mean_ratio(ac, -1.0, t.lnr[g]);  // eq. chiQg, alpha_Q = -1
          }
          const double ch = chl * mr;
          const double dchib = chl * (rac * p.ehi - p.elo);
          const double num = (4.0 + ac) * ch * p.b - dchib;
          const double den = 4.0 * p.b - (p.ehi - p.elo);
          const double f = num / den;
          c.chiE[k] = ch;
          c.ac[k] = ac;
          c.chiF[k] = (den > 0.0 && isfinite(f)) ? f : ch;
          c.emit[k] = ch * Bt - aT4 * dchib * p.scale * kThird;
        }
      }
    }
  } else {
    double b[G], elo[G], ehi[G], sig[G], scale[G], lqB[G], lqE[G], aB[G], aE[G];
    double slo[G], sq[G];  // with TD: 1 - e^{-x} at the lower edge, and s_g+/s_g-
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int g = gidx<LPC>(j, k, lpc);
      const Edge hi = planck_edge(hkT * t.nu[min(g + 1, ng)]);
      const Edge lo = low_edge<LPC>(hi, prev, hkT * t.nu[min(g, ng)], j, lpc);
      prev = hi;
      slo[k] = sq[k] = 1.0;
      if (TD && ot.stim) {
        const double s_hi = stim_factor(hi);
        slo[k] = from_left<LPC>(last ? prev_s : s_hi, lpc);
        prev_s = s_hi;
        sq[k] = s_hi / slo[k];
      }
      lqB[k] = -INFINITY;
      lqE[k] = -INFINITY;
      b[k] = elo[k] = ehi[k] = sig[k] = 0.0;
      scale[k] = 1.0;
      if (g >= ng) continue;
      const GroupPlanck p = group_planck(lo, hi);
      b[k] = p.b;
      elo[k] = p.elo;
      ehi[k] = p.ehi;
      sig[k] = p.sigma;
      scale[k] = p.scale;
      if (p.b > 0.0) lqB[k] = log(p.b) - p.sigma - t.lndnu[g];
      if (Ecur[k] > 0.0) lqE[k] = log(Ecur[k]) - t.lndnu[g];
    }
    slopes_free<G, LPC, NGM>(t, ng, j, lpc, lqB, aB);
    slopes_free<G, LPC, NGM>(t, ng, j, lpc, lqE, aE);
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int g = gidx<LPC>(j, k, lpc);
      if (g >= ng) continue;
      double ac = t.achi[g], rac = t.rac[g], chl = rho_kappa * t.chit[g];
      const double L = t.lnr[g];
      if (TD) {
        chl *= ot.fT * slo[k];
        if (ot.stim) {
          ac += log(sq[k]) / L;
          rac *= sq[k];
        }
        c.ac[k] = ac;
      }
      const double Bt = aT4 * b[k] * scale[k];
      const double Dnu = aT4 * (ehi[k] - elo[k]) * scale[k];
      c.Bt[k] = Bt;
      c.dBdT[k] = (4.0 * Bt - Dnu) * invT;
      const double chB = chl * mean_ratio(ac, aB[k], L);
      const double chE = chl * mean_ratio(ac, aE[k], L);
      c.chiB[k] = chB;
      c.chiE[k] = chE;
      const double dchib = chl * (rac * ehi[k] - elo[k]);
      const double num = (3.0 * chB + (1.0 + ac) * chE) * b[k] - dchib;  // both times 3
      const double den = 4.0 * b[k] - (ehi[k] - elo[k]);
      const double f = num / den;
      c.chiF[k] = (den > 0.0 && isfinite(f)) ? f : chE;
      c.emit[k] = chB * Bt - aT4 * dchib * scale[k] * kThird;
    }
  }
}

// P_g . v of the group closure (Sec. 2.1: M1 per group, or Eddington).  M1:
// P = E [(1 - chi)/2 I + (3 chi - 1)/2 n n] with n = F/|F| and the Levermore
// Eddington factor chi(f), f = min(|F|/(cE), 1); n (n . v) = F (F . v)/|F|^2,
// and chi needs only f^2, so one square root serves.
__device__ __forceinline__ void pressure_dot_v(int closure, double c, double E, double F0,
                                               double F1, double F2, const double* v,
                                               double* Pv) {
  if (!(E > 0.0)) {
    Pv[0] = Pv[1] = Pv[2] = 0.0;
    return;
  }
  const double FF = F0 * F0 + F1 * F1 + F2 * F2;
  if (closure == MGRHD_CLOSURE_EDDINGTON || FF == 0.0) {
    const double e3 = E * kThird;
    Pv[0] = e3 * v[0];
    Pv[1] = e3 * v[1];
    Pv[2] = e3 * v[2];
    return;
  }
  const double icE = 1.0 / (c * E);
  double f2 = FF * icE * icE;
  f2 = f2 > 1.0 ? 1.0 : f2;
  // 4 - 3 f^2 in [1, 4] and 5 + 2 sqrt(.) in [7, 9]: no range handling needed
  const double chi = (3.0 + 4.0 * f2) * rcp_nr(5.0 + 2.0 * sqrt_1_4(4.0 - 3.0 * f2));
  const double p = 0.5 * (1.0 - chi);
  const double q = 0.5 * (3.0 * chi - 1.0) * (F0 * v[0] + F1 * v[1] + F2 * v[2]) / FF;
  Pv[0] = E * (p * v[0] + q * F0);
  Pv[1] = E * (p * v[1] + q * F1);
  Pv[2] = E * (p * v[2] + q * F2);
}

enum Phase : int { P_EMPTY = 0, P_NEWTON = 1, P_FLUX = 2, P_IDLE = 3 };

// Per-cell-group registers.
template <int G>
struct CellState {
  int64_t i;
  int lpc;  // lanes per cell (run-time copy of the template value)
  int phase, st, steps, passes, k_out, polish_left;
  bool warm, fell_back, elim;
  double rho, rho_kappa, egas0, etot, ke;
  double egv;  // the E_gas iterate; in the outer stage the updated E_gas of the pass
  double ircv;  // 1/(rho c_v)
  double v[3];
  double R[G], E0[G];  // F_g^(t) and v^(t) stay in global memory, F_k in LDS
  double vF[G];        // v_k . F_g,k of the current outer pass
};

// N_g as the state machine sees it.  FULL: every slot of every lane holds a
// group (N_g = LPC * G), so the count is a compile-time constant and the
// per-slot checks g >= N_g compile away (fewer registers, branches and
// execution-mask changes).
template <int G, int LPC, bool FULL>
__device__ __forceinline__ int group_count(const KArgs& a) {
  static_assert(!FULL || LPC > 0, "FULL needs a compile-time lane count");
  return FULL ? LPC * G : a.ng;
}

template <int G, int LPC, int MODE, int NGM, bool TD = false, bool FULL = false,
          class LS>
__device__ __forceinline__ void load_cell(const KArgs& a, const Tables<NGM>& t, int j, int64_t i,
                                          CellState<G>& s, const LS& ls) {
  // 1/tau_g and 1/J_gg are constants of the cell unless the means depend on T
  constexpr bool kFixedTau = MODE != MGRHD_MEAN_PPL_FREE && !TD;
  const int64_t n = ls.arg(&KArgs::n);
  const int ng = group_count<G, LPC, FULL>(a);
  s.i = i;
  s.st = MGRHD_ST_OK;
  s.steps = 0;
  s.passes = 1;
  s.k_out = 0;
  s.polish_left = -1;
  s.fell_back = false;
  const StatePtrs sp = state_ptrs(ls.args);
  s.rho = ls.arg(&KArgs::rho)[i];
  s.egas0 = sp.egas[i];
#pragma unroll
  for (int d = 0; d < 3; ++d) s.v[d] = sp.v[(int64_t)d * n + i];
  const double* kappa = ls.arg(&KArgs::kappa);
  const double* S = ls.arg(&KArgs::S);
  const double kap = kappa ? kappa[i] : 1.0;
  bool ok = s.rho > 0.0 && isfinite(s.rho) && kap > 0.0 && isfinite(kap) && isfinite(s.egas0) &&
            isfinite(s.v[0]) && isfinite(s.v[1]) && isfinite(s.v[2]);
  s.rho_kappa = s.rho * kap;
  s.ircv = 1.0 / (s.rho * ls.cst(a, &KArgs::cv));
  if (LS::kKeep0 && j == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) ls.v0(d) = s.v[d];
  }
  const double cdt = ls.cst(a, &KArgs::cdt);
  double sumE = 0.0;
#pragma unroll
  for (int k = 0; k < G; ++k) {
    const int g = gidx<LPC>(j, k, s.lpc);
    s.R[k] = 0.0;
    s.E0[k] = 0.0;
    s.vF[k] = 0.0;
    double f[3] = {0.0, 0.0, 0.0};
    double it = 0.0, ij = -1.0;
    if (g < ng) {
      const double e = sp.E[(int64_t)g * n + i];
      const double sg = S ? S[(int64_t)g * n + i] : 0.0;
      ok = ok && e >= 0.0 && isfinite(e) && isfinite(sg);
      s.E0[k] = e + sg;
      sumE += e + sg;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        f[d] = sp.F[((int64_t)d * ng + g) * n + i];
        ok = ok && isfinite(f[d]);
      }
      s.vF[k] = s.v[0] * f[0] + s.v[1] * f[1] + s.v[2] * f[2];
      if (kFixedTau) {
        it = 1.0 / (cdt * s.rho_kappa * t.chk[g]);
        ij = rcp_nr(-it - 1.0);  // |-it - 1| >= 1
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      ls.F(d, k) = f[d];
      if (LS::kKeep0) ls.F0(d, k) = f[d];
    }
    if (kFixedTau) {
      ls.itau(k) = it;
      ls.iJgg(k) = ij;
    }
  }
  sumE = cell_sum<LPC>(sumE, s.lpc);
  const double bad = cell_sum<LPC>(ok ? 0.0 : 1.0, s.lpc);
  s.ke = 0.5 * s.rho * (s.v[0] * s.v[0] + s.v[1] * s.v[1] + s.v[2] * s.v[2]);
  s.etot = s.egas0 + ls.cst(a, &KArgs::icc) * sumE;  // E_tot of Sec. 3
  ok = bad == 0.0 && (s.egas0 - s.ke) > 0.0 && s.etot > 0.0;
  const double* guess = ls.arg(&KArgs::guess);
  s.warm = guess != nullptr;
  s.elim = false;
  s.egv = s.egas0;
  if (ok && s.warm) {
    s.egv = guess[i];
    if (ls.cst(a, &KArgs::guess_kind) == 1) {
      s.elim = true;  // R_g from the group balances at the first evaluation
    } else {
#pragma unroll
      for (int k = 0; k < G; ++k) {
        const int g = gidx<LPC>(j, k, s.lpc);
        if (g < ng) s.R[k] = guess[(int64_t)(g + 1) * n + i];
      }
    }
  }
  if (ok) {
    s.phase = P_NEWTON;
  } else {
    s.st = MGRHD_ST_INVALID;
    s.phase = P_EMPTY;
  }
}

template <int G, int LPC, bool FULL = false, class LS>
__device__ __forceinline__ void finish_cell(const KArgs& a, int j, CellState<G>& s,
                                            const LS& ls, bool store, double egas_new = 0.0) {
  const int64_t n = ls.arg(&KArgs::n), i = s.i;
  const int ng = group_count<G, LPC, FULL>(a);
  if (store) {
    double bad = (isfinite(egas_new) && isfinite(s.v[0]) && isfinite(s.v[1]) && isfinite(s.v[2]))
                     ? 0.0 : 1.0;
#pragma unroll
    for (int k = 0; k < G; ++k) {
      if (gidx<LPC>(j, k, s.lpc) >= ng) continue;
      if (!isfinite(s.E0[k] + s.R[k])) bad = 1.0;
#pragma unroll
      for (int d = 0; d < 3; ++d)
        if (!isfinite(ls.F(d, k))) bad = 1.0;
    }
    bad = cell_sum<LPC>(bad, s.lpc);
    const StatePtrs p = state_ptrs(ls.args);
    if (bad != 0.0) {
      s.st |= MGRHD_ST_NONFINITE;
      copy_through(a, p, i, j, s.lpc);
    } else {
#pragma unroll
      for (int k = 0; k < G; ++k) {
        const int g = gidx<LPC>(j, k, s.lpc);
        if (g >= ng) continue;
        p.Eo[(int64_t)g * n + i] = s.E0[k] + s.R[k];
#pragma unroll
        for (int d = 0; d < 3; ++d) p.Fo[((int64_t)d * ng + g) * n + i] = ls.F(d, k);
      }
      if (j == 0) {
        p.egaso[i] = egas_new;
        p.vo[i] = s.v[0];
        p.vo[n + i] = s.v[1];
        p.vo[2 * n + i] = s.v[2];
      }
    }
  } else {
    copy_through(a, state_ptrs(ls.args), i, j, s.lpc);
  }
  if (j == 0) {
    int32_t* const status = ls.arg(&KArgs::status);
    int32_t* const iters = ls.arg(&KArgs::iters);
    int32_t* const outer = ls.arg(&KArgs::outer);
    int32_t* const trace = ls.arg(&KArgs::trace);
    if (status) status[i] = s.st;
    if (iters) iters[i] = s.steps;
    if (outer) outer[i] = s.passes;
    if (trace)  // passes whose outer stage did not run (the last one's did if stored)
      for (int k = store ? s.k_out + 1 : s.k_out; k < ls.cst(a, &KArgs::max_outer); ++k)
        trace[(int64_t)k * n + i] = -1;
  }
  s.phase = P_EMPTY;
}

// End of an inner pass with result rc (0 converged, 1 max_newton, 2 T <= 0).
template <int G, int LPC, bool FULL = false, class LS>
__device__ __forceinline__ void newton_done(const KArgs& a, int j, CellState<G>& s,
                                            const LS& ls, int rc) {
  if (s.k_out == 0 && s.warm && rc != 0 && !s.fell_back) {
    // warm start failed: plain Newton from the old state (status bit 4)
    s.st |= MGRHD_ST_FALLBACK;
    s.fell_back = true;
    s.elim = false;
    s.egv = s.egas0;
#pragma unroll
    for (int k = 0; k < G; ++k) s.R[k] = 0.0;
    s.polish_left = -1;
    return;  // stays in P_NEWTON
  }
  if (rc == 1) s.st |= MGRHD_ST_NEWTON_MAXIT;
  if (rc == 2) {
    s.st |= MGRHD_ST_INVALID;
    finish_cell<G, LPC, FULL>(a, j, s, ls, false);
    return;
  }
  // conservative energy update (Sec. 3)
  double sumR = 0.0;
#pragma unroll
  for (int k = 0; k < G; ++k) sumR += s.R[k];
  sumR = cell_sum<LPC>(sumR, s.lpc);
  s.egv = s.egas0 - ls.cst(a, &KArgs::cc) * sumR;  // E_gas^(t+1) of this pass
  s.phase = P_FLUX;
}

// Temperature-only start: at the cached material state, eq. Rnew inverted for
// E_g and F_R,g = 0 (eq. FGFR) are linear in R_g alone; take that R_g.
template <int G, int LPC, int MODE, int NGM, bool TD = false, bool FULL = false,
          class LS>
__device__ __forceinline__ void group_balance(const KArgs& a, const Tables<NGM>& t, int j,
                                              CellState<G>& s, const LS& ls,
                                              const Cache<G>& c) {
  const int ng = group_count<G, LPC, FULL>(a);
  const double cdt = ls.cst(a, &KArgs::cdt);
  const double ic2 = ls.cst(a, &KArgs::ic2);
#pragma unroll
  for (int k = 0; k < G; ++k) {
    const int g = gidx<LPC>(j, k, s.lpc);
    if (g >= ng) continue;
    double ratio = 1.0, itau;
    if (MODE == MGRHD_MEAN_PPL_FREE || TD) {
      if (MODE == MGRHD_MEAN_PPL_FREE) ratio = c.chiB[k] / c.chiE[k];
      itau = 1.0 / (cdt * c.chiE[k]);
    } else {
      itau = ls.itau(k);
    }
    const double ac = TD ? c.ac[k] : t.achi[g];
    const double W = cdt * (1.0 + ac) * c.chiF[k] * s.vF[k] * ic2;
    s.R[k] = (ratio * c.Bt[k] + W * itau - s.E0[k]) / (1.0 + itau);
  }
  s.elim = false;
}

// Newton consumer: residual of eq. FGFR at the cached material state, the
// elimination of eq. matrix, and the step.
template <int G, int LPC, int MODE, int NGM, bool TD = false, bool FULL = false,
          class LS>
__device__ __forceinline__ void newton_step(const KArgs& a, const Tables<NGM>& t, int j,
                                            CellState<G>& s, const LS& ls,
                                            const Cache<G>& c) {
  const int ng = group_count<G, LPC, FULL>(a);
  const double cc = ls.cst(a, &KArgs::cc);
  const double cdt = ls.cst(a, &KArgs::cdt);
  const double ic2 = ls.cst(a, &KArgs::ic2);
  const double ircv = s.ircv;
  double sumR = 0.0, sumAbs = 0.0, sumA = 0.0, sumB = 0.0;
  double ag[G], bg[G];
#pragma unroll
  for (int k = 0; k < G; ++k) {
    ag[k] = 0.0;
    bg[k] = 0.0;
    const int g = gidx<LPC>(j, k, s.lpc);
    if (g >= ng) continue;
    double ratio = 1.0, itau, iJgg;
    if (MODE == MGRHD_MEAN_PPL_FREE || TD) {
      if (MODE == MGRHD_MEAN_PPL_FREE) ratio = c.chiB[k] / c.chiE[k];
      itau = 1.0 / (cdt * c.chiE[k]);
      iJgg = rcp_nr(-itau - 1.0);  // |-itau - 1| >= 1
    } else {
      itau = ls.itau(k);
      iJgg = ls.iJgg(k);
    }
    const double ac = TD ? c.ac[k] : t.achi[g];
    const double W = cdt * (1.0 + ac) * c.chiF[k] * s.vF[k] * ic2;  // eq. Rnew
    const double Eg = ratio * c.Bt[k] + (W - s.R[k]) * itau;  // eq. Rnew solved for E_g
    const double FR = Eg - s.E0[k] - s.R[k];
    const double Jg0 = ratio * c.dBdT[k] * ircv;               // eq. linear
    ag[k] = FR * iJgg;
    bg[k] = Jg0 * iJgg;
    sumR += s.R[k];
    sumAbs += fabs(FR);
    sumA += ag[k];
    sumB += bg[k];
  }
  sumR = cell_sum<LPC>(sumR, s.lpc);
  sumAbs = cell_sum<LPC>(sumAbs, s.lpc);
  sumA = cell_sum<LPC>(sumA, s.lpc);
  sumB = cell_sum<LPC>(sumB, s.lpc);
  const double FG = s.egv - s.egas0 + cc * sumR;
  // the stop test of Sec. 3, |F_G| / E_tot < eps and (c/c_hat) sum |F_R,g| / E_tot < eps
  const double tol = ls.cst(a, &KArgs::eps) * s.etot;
  const bool conv = fabs(FG) < tol && cc * sumAbs < tol;
  if (s.polish_left < 0 && conv) s.polish_left = ls.cst(a, &KArgs::polish);
  if (s.polish_left == 0) {
    newton_done<G, LPC, FULL>(a, j, s, ls, 0);
    return;
  }
  if (s.polish_left < 0 && s.steps >= ls.cst(a, &KArgs::max_newton)) {
    newton_done<G, LPC, FULL>(a, j, s, ls, 1);
    return;
  }
  // eq. matrix eliminated: dx0, then dx_g = -a_g - b_g dx0
  // the denominator is >= 1 (J_gg < 0, J_g0 >= 0): no scaling needed
  const double den0 = 1.0 - cc * sumB;
  const double num0 = -FG + cc * sumA;
  const double ir0 = rcp_nr(den0);
  const double q0 = num0 * ir0;
  const double dx0 = fma(fma(-den0, q0, num0), ir0, q0);
  double lam = 1.0;
  for (int h = 0; h < 30 && !(s.egv + lam * dx0 - s.ke > 0.0); ++h) lam *= 0.5;
  if (!(s.egv + lam * dx0 - s.ke > 0.0)) {
    newton_done<G, LPC, FULL>(a, j, s, ls, 2);
    return;
  }
  s.egv += lam * dx0;
#pragma unroll
  for (int k = 0; k < G; ++k) s.R[k] += lam * (-ag[k] - bg[k] * dx0);
  if (s.polish_left > 0)
    --s.polish_left;
  else
    ++s.steps;
  if (s.polish_left == 0) newton_done<G, LPC, FULL>(a, j, s, ls, 0);
}

// Outer-stage consumer: flux update eq. numF1 with the outdated velocity,
// momentum update, outer test.  Returns true when the next inner pass starts
// (at the same temperature, so the caller reuses this evaluation).
template <int G, int LPC, int MODE, int NGM, bool TD = false, bool FULL = false,
          class LS>
__device__ __forceinline__ bool flux_step(const KArgs& a, const Tables<NGM>& t, int j,
                                          CellState<G>& s, const LS& ls,
                                          const Cache<G>& c) {
  const int ng = group_count<G, LPC, FULL>(a);
  const int64_t n = ls.arg(&KArgs::n), i = s.i;
  const double cdt = ls.cst(a, &KArgs::cdt);
  if (j == 0) {
    int32_t* const trace = ls.arg(&KArgs::trace);
    if (trace) trace[(int64_t)s.k_out * n + i] = s.steps;
  }
  double dmom[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < G; ++k) {
    const int g = gidx<LPC>(j, k, s.lpc);
    if (g >= ng) continue;
    const double Enew = s.E0[k] + s.R[k];
    const double chE =
        (MODE == MGRHD_MEAN_PPL_FREE || TD) ? c.chiE[k] : s.rho_kappa * t.chk[g];
    const double ac = TD ? c.ac[k] : t.achi[g];
    double Pv[3];
    pressure_dot_v(ls.cst(a, &KArgs::closure), ls.cst(a, &KArgs::c), Enew, ls.F(0, k), ls.F(1, k),
                   ls.F(2, k), s.v, Pv);
    const double iden = rcp_nr(1.0 + cdt * c.chiF[k]);  // >= 1
    const double q = (1.0 + ac) * chE;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double f0 = LS::kKeep0 ? ls.F0(d, k) : a.F[((int64_t)d * ng + g) * n + i];  // F_g^(t)
      const double f = (f0 + cdt * (s.v[d] * c.emit[k] + q * Pv[d])) * iden;
      ls.F(d, k) = f;  // F_k+1 replaces F_k (v_k . F_k stays in s.vF)
      dmom[d] += f - f0;
    }
  }
  const double ccc = ls.cst(a, &KArgs::iccc);
  const double irho = s.ircv * ls.cst(a, &KArgs::cv);
  double vn[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    dmom[d] = cell_sum<LPC>(dmom[d], s.lpc);
    const double v0 = LS::kKeep0 ? ls.v0(d) : a.v[(int64_t)d * n + i];  // v^(t)
    vn[d] = (s.rho * v0 - dmom[d] * ccc) * irho;  // momentum update
  }
  // change of the velocity terms of eq. Rnew less 2^-46 of their size: the
  // change cannot be resolved below the terms' own rounding where they are
  // large against E_tot (tau v/c >> 1)
  double dW = 0.0;
#pragma unroll
  for (int k = 0; k < G; ++k) {
    const int g = gidx<LPC>(j, k, s.lpc);
    if (g >= ng) continue;
    const double vf_new = vn[0] * ls.F(0, k) + vn[1] * ls.F(1, k) + vn[2] * ls.F(2, k);
    const double kw = fabs((1.0 + (TD ? c.ac[k] : t.achi[g])) * c.chiF[k]);
    dW += kw * fma(-0x1p-46, fabs(vf_new), fabs(vf_new - s.vF[k]));
    s.vF[k] = vf_new;
  }
  dW = cell_sum<LPC>(dW, s.lpc) * ls.cst(a, &KArgs::cdt_ic2);
  const double ke_new = 0.5 * s.rho * (vn[0] * vn[0] + vn[1] * vn[1] + vn[2] * vn[2]);
  const double egas_new = s.egv;
  s.egv = egas_new + (ke_new - s.ke);
  s.ke = ke_new;
#pragma unroll
  for (int d = 0; d < 3; ++d) s.v[d] = vn[d];
  if (dW < ls.cst(a, &KArgs::eps_out) * s.etot) {
    finish_cell<G, LPC, FULL>(a, j, s, ls, true, egas_new);
    return false;
  }
  if (s.k_out + 1 >= ls.cst(a, &KArgs::max_outer)) {
    s.st |= MGRHD_ST_OUTER_MAXIT;
    finish_cell<G, LPC, FULL>(a, j, s, ls, true, egas_new);
    return false;
  }
  ++s.k_out;
  ++s.passes;
  s.polish_left = -1;
  s.phase = P_NEWTON;
  return true;
}

// The per-cell state machine of one wave over the cells [lo, hi): every cell
// group without a cell takes the next one; each trip performs one material
// evaluation for every active cell group, then the consumer of its phase (a
// Newton step, or the flux/momentum update of the outer stage followed by the
// first Newton step of the next pass at the same temperature).  Returns when
// every cell is done.  Shared by the single-table and the batched kernels.
// Where a wave takes its next cells from.  WaveRange: the cells [lo, hi)
// belong to this wave alone.  BlockQueue: the waves of a workgroup share the
// range through a counter in LDS, so the cells in flight in a workgroup stay
// within a narrow window of consecutive cells and share the cache lines of
// every SoA row between them.
struct WaveRange {
  int64_t next, hi;
  __device__ __forceinline__ int64_t take(int count) {  // wave-uniform
    const int64_t base = next;
    next += count;
    return base;
  }
};

struct BlockQueue {
  int* counter;  // LDS, zeroed before the first take
  int64_t lo, hi;
  __device__ __forceinline__ int64_t take(int count) {  // all lanes active
    int base = 0;
    if (__lane_id() == 0) base = atomicAdd(counter, count);
    return lo + __builtin_amdgcn_readfirstlane(base);
  }
};

template <int G, int LPC, int MODE, int NGM, bool TD = false, bool FULL = false, class LS,
          class Q>
__device__ __forceinline__ void run_cells(const KArgs& a, const Tables<NGM>& tab,
                                          const LS& ls_block, int lane, Q q) {
  static_assert(LPC >= 1 && LPC <= kWave && (LPC & (LPC - 1)) == 0, "lanes per cell");
  const int j = lane % LPC;
  // this cell's slot in the per-cell area: with room for a cell per lane
  // (CPB = kBlock, the batched kernels, whose waves may run different lane
  // counts) the slot of the cell's first lane, else the cell's rank in the
  // workgroup (every wave runs the same lane count)
  const LS ls = ls_block.at_cell(LS::kCPB == kBlock ? (int)threadIdx.x - j
                                                    : (int)threadIdx.x / LPC);
  CellState<G> s;
  s.phase = P_EMPTY;
  s.i = -1;
  s.lpc = LPC;
  Cache<G> c;
  const int64_t hi = q.hi;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  for (;;) {
    // refill: every cell group without a cell takes the next one of the queue
    const bool need = s.phase == P_EMPTY;
    const uint64_t m = __ballot(need && j == 0);
    if (m) {
      const int rank = __popcll(m & below);
      int64_t mine = q.take(__popcll(m)) + rank;
      mine = __shfl(mine, lane - j, kWave);
      if (need) {
        if (mine < hi) {
          load_cell<G, LPC, MODE, NGM, TD, FULL>(a, tab, j, mine, s, ls);
          if (s.phase == P_EMPTY) finish_cell<G, LPC, FULL>(a, j, s, ls, false);
        } else {
          s.phase = P_IDLE;
        }
      }
    }
    if (__ballot(s.phase == P_NEWTON || s.phase == P_FLUX) == 0) {
      if (__ballot(s.phase == P_EMPTY) == 0) break;  // range exhausted
      continue;
    }
    if (s.phase != P_NEWTON && s.phase != P_FLUX) continue;

    // one material evaluation at this cell's current temperature
    const double T = (s.egv - s.ke) * s.ircv;
    if (!(T > 0.0) || !isfinite(T)) {
      if (s.phase == P_NEWTON)
        newton_done<G, LPC, FULL>(a, j, s, ls, 2);
      else {
        s.st |= MGRHD_ST_INVALID;
        finish_cell<G, LPC, FULL>(a, j, s, ls, false);
      }
      continue;
    }
    double Ecur[G];
#pragma unroll
    for (int k = 0; k < G; ++k) Ecur[k] = s.E0[k] + s.R[k];
    const double aT4 = ls.cst(a, &KArgs::a) * (T * T) * (T * T);
    OpacityT ot{1.0, false};
    if (TD) {
      const double t_exp = ls.cst(a, &KArgs::t_exp);
      ot.fT = t_exp != 0.0 ? exp(t_exp * log(T * ls.cst(a, &KArgs::itref))) : 1.0;
      ot.stim = ls.cst(a, &KArgs::stim) != 0;
    }
    evaluate<G, LPC, MODE, NGM, TD>(tab, group_count<G, LPC, FULL>(a), j, s.lpc, T, aT4,
                                    ls.cst(a, &KArgs::hk), s.rho_kappa, Ecur, c, ot);

    if (s.phase == P_FLUX) {
      if (!flux_step<G, LPC, MODE, NGM, TD, FULL>(a, tab, j, s, ls, c)) continue;
      // the next inner pass starts at this temperature: fall through
    }
    if (s.elim) group_balance<G, LPC, MODE, NGM, TD, FULL>(a, tab, j, s, ls, c);
    newton_step<G, LPC, MODE, NGM, TD, FULL>(a, tab, j, s, ls, c);
  }
}

// WPE: minimum resident waves per SIMD the register allocation must allow

}  // namespace mgrhd
