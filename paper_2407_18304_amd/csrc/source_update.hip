// source_update.hip -- gfx950 kernels and C ABI of the multigroup
// matter-radiation source update (He, Wibking & Krumholz 2024, Sec. 3).
//
// Work decomposition: LPC consecutive lanes of a wavefront own one cell; lane
// j of the cell owns the G consecutive groups j*G .. j*G+G-1.  Each lane keeps
// its groups' state (R_g, E_g^(t)+S_g, F_g^(t), F_g of the current outer pass)
// in registers, evaluates its G+1 Planck edges, and the group sums of the
// Newton system (sum R_g, sum |F_R,g|, and the two sums of the arrowhead
// elimination) are formed with xor-butterfly shuffles inside the LPC lanes, so
// that every lane of a cell holds bit-identical scalars and takes the same
// branches.  The scalar part of the Newton step is repeated on the LPC lanes.
// Loads and stores are structure-of-arrays with the cell index fastest.
//
// Group tables (edges and the opacity table) are staged once per workgroup in
// LDS together with per-group constants (ln r_g, the powerlaw index, r_g^alpha,
// the PPL-fixed mean ratio, ln of the group width and of the log-centre).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/mgrhd.h"
#include "planck_device.hpp"

namespace mgrhd {

struct KArgs {
  double* E;
  double* F;
  const double* rho;
  double* egas;
  double* v;
  const double* kappa;
  const double* S;
  const double* guess;
  int32_t* iters;
  int32_t* outer;
  int32_t* status;
  const double* edges;
  const double* chi_lo;
  const double* alpha;
  const double* chi_hi;
  int64_t n;
  int32_t ng;
  int32_t closure;
  double dt, chat, c, a, hk, cv, eps, eps_out;
  int32_t max_newton, max_outer, polish, pad;
};

constexpr int kBlock = 256;

// LDS layout of the per-group tables (NGM = G * LPC groups at most).
template <int NGM>
struct Tables {
  double nu[NGM + 1];
  double lnr[NGM];    // ln(nu_g+ / nu_g-)
  double achi[NGM];   // opacity powerlaw index (0 in PC)
  double chat_[NGM];  // chi_lo table entry (per unit rho * kappa)
  double mfix[NGM];   // PPL-fixed mean ratio chi_0B/chi_0,g- = chi_0E/chi_0,g-
  double rac[NGM];    // r_g^alpha_chi
  double lndnu[NGM];  // ln(nu_g+ - nu_g-)
  double lnc[NGM];    // ln of the group's log-centre, (ln nu_g- + ln nu_g+)/2
  int bad;
};

template <int LPC>
__device__ __forceinline__ double cell_sum(double v) {
#pragma unroll
  for (int m = 1; m < LPC; m <<= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Stage and validate the tables.  Returns false (for every thread of the
// block) when the table is unusable.
template <int NGM, int MODE>
__device__ bool stage_tables(const KArgs& a, Tables<NGM>& t) {
  if (threadIdx.x == 0) t.bad = 0;
  __syncthreads();
  const int ng = a.ng;
  for (int g = threadIdx.x; g <= ng; g += blockDim.x) {
    const double nu = a.edges[g];
    t.nu[g] = nu;
    bool ok = nu >= 0.0;
    if (MODE != MGRHD_MEAN_PC) ok = ok && nu > 0.0 && isfinite(nu);
    if (!ok) atomicOr(&t.bad, 1);
  }
  __syncthreads();
  for (int g = threadIdx.x; g < ng; g += blockDim.x) {
    const double lo = t.nu[g], hi = t.nu[g + 1];
    const double chl = a.chi_lo[g];
    bool ok = hi > lo && chl > 0.0 && isfinite(chl);
    double L = 0.0, ac = 0.0, mf = 1.0, rac = 1.0, ldn = 0.0, lc = 0.0;
    if (MODE != MGRHD_MEAN_PC) {
      L = log(hi / lo);
      if (a.alpha) {
        ac = a.alpha[g];
      } else {
        const double chh = a.chi_hi[g];
        ok = ok && chh > 0.0 && isfinite(chh);
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
    t.chat_[g] = chl;
    t.mfix[g] = mf;
    t.rac[g] = rac;
    t.lndnu[g] = ldn;
    t.lnc[g] = lc;
    if (!ok) atomicOr(&t.bad, 1);
  }
  __syncthreads();
  return t.bad == 0;
}

// Group-mean opacities and Planck data of one group at temperature T.
struct GroupMat {
  double Bt, Dnu, dBdT;        // B~_g, Delta_g(nu B~), dB~_g/dT
  double chiB, chiE, chiF;     // means (per cell)
  double DchiB;                // Delta_g(nu chi_0 B~)
  double ac;                   // alpha_chi
};

// Slopes for PPL-free: fill lqB, lqE of this lane's groups.
template <int G>
struct FreeScratch {
  double b[G], elo[G], ehi[G], sig[G], scale[G], lqB[G], lqE[G], aB[G], aE[G];
};

template <int G, int LPC, int NGM>
__device__ __forceinline__ void slopes_free(const Tables<NGM>& t, int ng, int j, const double* lq,
                                            double* alpha) {
  // neighbours across the lane boundary of this cell
  const int lane = __lane_id();
  const double left = __shfl(lq[G - 1], lane - 1 < 0 ? 0 : lane - 1, 64);
  const double right = __shfl(lq[0], lane + 1 > 63 ? 63 : lane + 1, 64);
#pragma unroll
  for (int k = 0; k < G; ++k) {
    const int g = j * G + k;
    alpha[k] = -1.0;
    if (g <= 0 || g >= ng - 1) continue;
    const double lm = (k == 0) ? left : lq[k - 1];
    const double lp = (k == G - 1) ? right : lq[k + 1];
    const double sl = (lq[k] - lm) / (t.lnc[g] - t.lnc[g - 1]);
    const double sr = (lp - lq[k]) / (t.lnc[g + 1] - t.lnc[g]);
    if (isnan(sl) || isnan(sr)) continue;
    const double m = minmod(sl, sr);
    if (isfinite(m)) alpha[k] = m;
  }
}

// Evaluate the material state of this lane's G groups at temperature T.
// For PPL-free, Ecur holds the current group energies (slope of E_nu).
template <int G, int LPC, int MODE, int NGM>
__device__ __forceinline__ void material(const Tables<NGM>& t, int ng, int j, double T, double aT4,
                                         double hk, double rho_kappa, const double* Ecur,
                                         GroupMat* out) {
  Edge lo = planck_edge(hk * t.nu[min(j * G, ng)] / T);
  if (MODE != MGRHD_MEAN_PPL_FREE) {
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int g = j * G + k;
      if (g >= ng) break;
      const Edge hi = planck_edge(hk * t.nu[g + 1] / T);
      const GroupPlanck p = group_planck(lo, hi);
      lo = hi;
      GroupMat& m = out[k];
      m.Bt = aT4 * p.b * p.scale;
      m.Dnu = aT4 * (p.ehi - p.elo) * p.scale;
      m.dBdT = (4.0 * m.Bt - m.Dnu) / T;
      const double chl = rho_kappa * t.chat_[g];
      if (MODE == MGRHD_MEAN_PC) {
        m.chiB = m.chiE = m.chiF = chl;
        m.DchiB = chl * m.Dnu;
        m.ac = 0.0;
      } else {
        const double ac = t.achi[g];
        const double ch = chl * t.mfix[g];
        m.chiB = m.chiE = ch;
        const double dchib = chl * (t.rac[g] * p.ehi - p.elo);
        m.DchiB = aT4 * dchib * p.scale;
        const double num = (ch + ch / 3.0) * p.b + (ac * ch * p.b - dchib) / 3.0;
        const double den = (4.0 * p.b - (p.ehi - p.elo)) / 3.0;
        const double f = num / den;
        m.chiF = (den > 0.0 && isfinite(f)) ? f : ch;
        m.ac = ac;
      }
    }
  } else {
    FreeScratch<G> s;
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int g = j * G + k;
      s.lqB[k] = -INFINITY;
      s.lqE[k] = -INFINITY;
      if (g >= ng) continue;
      const Edge hi = planck_edge(hk * t.nu[g + 1] / T);
      const GroupPlanck p = group_planck(lo, hi);
      lo = hi;
      s.b[k] = p.b;
      s.elo[k] = p.elo;
      s.ehi[k] = p.ehi;
      s.sig[k] = p.sigma;
      s.scale[k] = p.scale;
      if (p.b > 0.0) s.lqB[k] = log(p.b) - p.sigma - t.lndnu[g];
      if (Ecur[k] > 0.0) s.lqE[k] = log(Ecur[k]) - t.lndnu[g];
    }
    slopes_free<G, LPC, NGM>(t, ng, j, s.lqB, s.aB);
    slopes_free<G, LPC, NGM>(t, ng, j, s.lqE, s.aE);
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int g = j * G + k;
      if (g >= ng) break;
      GroupMat& m = out[k];
      const double ac = t.achi[g], L = t.lnr[g];
      const double chl = rho_kappa * t.chat_[g];
      m.Bt = aT4 * s.b[k] * s.scale[k];
      m.Dnu = aT4 * (s.ehi[k] - s.elo[k]) * s.scale[k];
      m.dBdT = (4.0 * m.Bt - m.Dnu) / T;
      m.chiB = chl * mean_ratio(ac, s.aB[k], L);
      m.chiE = chl * mean_ratio(ac, s.aE[k], L);
      const double dchib = chl * (t.rac[g] * s.ehi[k] - s.elo[k]);
      m.DchiB = aT4 * dchib * s.scale[k];
      const double num = (m.chiB + m.chiE / 3.0) * s.b[k] + (ac * m.chiE * s.b[k] - dchib) / 3.0;
      const double den = (4.0 * s.b[k] - (s.ehi[k] - s.elo[k])) / 3.0;
      const double f = num / den;
      m.chiF = (den > 0.0 && isfinite(f)) ? f : m.chiE;
      m.ac = ac;
    }
  }
}

// P_g . v of the group closure (Sec. 2.1: M1 per group, or Eddington)
__device__ __forceinline__ void pressure_dot_v(int closure, double c, double E, double F0,
                                               double F1, double F2, const double* v,
                                               double* Pv) {
  if (!(E > 0.0)) {
    Pv[0] = Pv[1] = Pv[2] = 0.0;
    return;
  }
  const double fm = sqrt(F0 * F0 + F1 * F1 + F2 * F2);
  if (closure == MGRHD_CLOSURE_EDDINGTON || fm == 0.0) {
    Pv[0] = E * v[0] / 3.0;
    Pv[1] = E * v[1] / 3.0;
    Pv[2] = E * v[2] / 3.0;
    return;
  }
  double f = fm / (c * E);
  f = f > 1.0 ? 1.0 : f;
  const double chi = (3.0 + 4.0 * f * f) / (5.0 + 2.0 * sqrt(4.0 - 3.0 * f * f));
  const double n0 = F0 / fm, n1 = F1 / fm, n2 = F2 / fm;
  const double nv = n0 * v[0] + n1 * v[1] + n2 * v[2];
  const double p = 0.5 * (1.0 - chi), q = 0.5 * (3.0 * chi - 1.0);
  Pv[0] = E * (p * v[0] + q * n0 * nv);
  Pv[1] = E * (p * v[1] + q * n1 * nv);
  Pv[2] = E * (p * v[2] + q * n2 * nv);
}

template <int G>
struct LaneState {
  double R[G];     // Newton unknowns R_g
  double E0[G];    // E_g^(t) + S_g
  double F0[3][G]; // F_g^(t)
  double Fk[3][G]; // F_g of the current outer pass
};

// One inner stage.  0 converged, 1 max_newton, 2 T <= 0.
template <int G, int LPC, int MODE, int NGM>
__device__ int newton(const KArgs& a, const Tables<NGM>& t, int j, LaneState<G>& s, double rho,
                      double rho_kappa, double egas0, double etot, const double* v, double& egv,
                      int& steps) {
  const int ng = a.ng;
  const double cc = a.c / a.chat;
  const double ke = 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  const double rcv = rho * a.cv;
  const double cdt = a.chat * a.dt;
  const double ic2 = 1.0 / (a.c * a.c);
  int polish_left = -1;
  for (;;) {
    const double T = (egv - ke) / rcv;
    if (!(T > 0.0) || !isfinite(T)) return 2;
    const double aT4 = a.a * (T * T) * (T * T);
    double Ecur[G];
#pragma unroll
    for (int k = 0; k < G; ++k) Ecur[k] = s.E0[k] + s.R[k];
    GroupMat m[G];
    material<G, LPC, MODE, NGM>(t, ng, j, T, aT4, a.hk, rho_kappa, Ecur, m);

    double sumR = 0.0, sumAbs = 0.0, sumA = 0.0, sumB = 0.0;
    double ag[G], bg[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
      ag[k] = 0.0;
      bg[k] = 0.0;
      if (j * G + k >= ng) continue;
      const double vF = v[0] * s.Fk[0][k] + v[1] * s.Fk[1][k] + v[2] * s.Fk[2][k];
      const double tauE = cdt * m[k].chiE;
      const double W = cdt * (1.0 + m[k].ac) * m[k].chiF * vF * ic2;
      const double ratio = m[k].chiB / m[k].chiE;
      const double Eg = ratio * m[k].Bt + (W - s.R[k]) / tauE;
      const double FR = Eg - s.E0[k] - s.R[k];
      const double Jg0 = ratio * m[k].dBdT / rcv;
      const double Jgg = -1.0 / tauE - 1.0;
      ag[k] = FR / Jgg;
      bg[k] = Jg0 / Jgg;
      sumR += s.R[k];
      sumAbs += fabs(FR);
      sumA += ag[k];
      sumB += bg[k];
    }
    sumR = cell_sum<LPC>(sumR);
    sumAbs = cell_sum<LPC>(sumAbs);
    sumA = cell_sum<LPC>(sumA);
    sumB = cell_sum<LPC>(sumB);
    const double FG = egv - egas0 + cc * sumR;
    const bool conv = fabs(FG) / etot < a.eps && cc * sumAbs / etot < a.eps;
    if (polish_left < 0 && conv) polish_left = a.polish;
    if (polish_left == 0) return 0;
    if (polish_left < 0 && steps >= a.max_newton) return 1;

    // eq. matrix eliminated: dx0, then dx_g = -a_g - b_g dx0
    const double dx0 = (-FG + cc * sumA) / (1.0 - cc * sumB);
    double lam = 1.0;
    for (int h = 0; h < 30 && !(egv + lam * dx0 - ke > 0.0); ++h) lam *= 0.5;
    if (!(egv + lam * dx0 - ke > 0.0)) return 2;
    egv += lam * dx0;
#pragma unroll
    for (int k = 0; k < G; ++k) s.R[k] += lam * (-ag[k] - bg[k] * dx0);
    if (polish_left > 0)
      --polish_left;
    else
      ++steps;
    if (polish_left == 0) return 0;
  }
}

template <int G, int LPC, int MODE>
__global__ __launch_bounds__(kBlock) void k_source_update(KArgs a) {
  constexpr int NGM = G * LPC;
  __shared__ Tables<NGM> tab;
  const bool table_ok = stage_tables<NGM, MODE>(a, tab);

  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = tid / LPC;
  const int j = (int)(tid % LPC);
  if (i >= a.n) return;
  const int64_t n = a.n;
  const int ng = a.ng;
  const double cc = a.c / a.chat;
  const double cdt = a.chat * a.dt;

  int st = MGRHD_ST_OK, steps = 0, passes = 0;
  if (!table_ok) {
    if (j == 0 && a.status) a.status[i] = MGRHD_ST_BAD_TABLE;
    if (j == 0 && a.iters) a.iters[i] = 0;
    if (j == 0 && a.outer) a.outer[i] = 0;
    return;
  }

  const double rho = a.rho[i];
  const double egas0 = a.egas[i];
  const double v0[3] = {a.v[i], a.v[n + i], a.v[2 * n + i]};
  const double kap = a.kappa ? a.kappa[i] : 1.0;
  bool ok = rho > 0.0 && isfinite(rho) && kap > 0.0 && isfinite(kap) && isfinite(egas0) &&
            isfinite(v0[0]) && isfinite(v0[1]) && isfinite(v0[2]);

  LaneState<G> s;
  double sumE = 0.0;
#pragma unroll
  for (int k = 0; k < G; ++k) {
    const int g = j * G + k;
    s.R[k] = 0.0;
    s.E0[k] = 0.0;
    for (int d = 0; d < 3; ++d) s.F0[d][k] = s.Fk[d][k] = 0.0;
    if (g < ng) {
      const double e = a.E[(int64_t)g * n + i];
      const double sg = a.S ? a.S[(int64_t)g * n + i] : 0.0;
      ok = ok && e >= 0.0 && isfinite(e) && isfinite(sg);
      s.E0[k] = e + sg;
      sumE += e + sg;
      for (int d = 0; d < 3; ++d) {
        const double f = a.F[((int64_t)d * ng + g) * n + i];
        ok = ok && isfinite(f);
        s.F0[d][k] = s.Fk[d][k] = f;
      }
    }
  }
  // every lane of the cell must agree on validity
  sumE = cell_sum<LPC>(sumE);
  const double okf = cell_sum<LPC>(ok ? 0.0 : 1.0);
  const double ke0 = 0.5 * rho * (v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2]);
  const double etot = egas0 + (a.chat / a.c) * sumE;  // E_tot of Sec. 3
  ok = okf == 0.0 && (egas0 - ke0) > 0.0 && etot > 0.0;

  double egas_new = egas0;
  double v[3] = {v0[0], v0[1], v0[2]};
  if (!ok) {
    st = MGRHD_ST_INVALID;
  } else {
    const double rho_kappa = rho * kap;
    double egv = egas0;
    const bool warm = a.guess != nullptr;
    if (warm) {
      egv = a.guess[i];
#pragma unroll
      for (int k = 0; k < G; ++k) {
        const int g = j * G + k;
        s.R[k] = g < ng ? a.guess[(int64_t)(g + 1) * n + i] : 0.0;
      }
    }
    for (int k_out = 0;; ++k_out) {
      ++passes;
      int rc = newton<G, LPC, MODE, NGM>(a, tab, j, s, rho, rho_kappa, egas0, etot, v, egv, steps);
      if (k_out == 0 && warm && rc != 0) {
        st |= MGRHD_ST_FALLBACK;
        egv = egas0;
#pragma unroll
        for (int k = 0; k < G; ++k) s.R[k] = 0.0;
        rc = newton<G, LPC, MODE, NGM>(a, tab, j, s, rho, rho_kappa, egas0, etot, v, egv, steps);
      }
      if (rc == 1) st |= MGRHD_ST_NEWTON_MAXIT;
      if (rc == 2) {
        st |= MGRHD_ST_INVALID;
        break;
      }
      // conservative energy update
      double sumR = 0.0;
      double Enew[G];
#pragma unroll
      for (int k = 0; k < G; ++k) {
        Enew[k] = s.E0[k] + s.R[k];
        sumR += s.R[k];
      }
      sumR = cell_sum<LPC>(sumR);
      egas_new = egas0 - cc * sumR;

      // outer stage: material at the updated energies, outdated velocity
      const double ke = 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      const double T = (egas_new - ke) / (rho * a.cv);
      if (!(T > 0.0) || !isfinite(T)) {
        st |= MGRHD_ST_INVALID;
        break;
      }
      const double aT4 = a.a * (T * T) * (T * T);
      GroupMat m[G];
      material<G, LPC, MODE, NGM>(tab, ng, j, T, aT4, a.hk, rho_kappa, Enew, m);
      double dmom[3] = {0.0, 0.0, 0.0};
      double Fn[3][G];
#pragma unroll
      for (int k = 0; k < G; ++k) {
        for (int d = 0; d < 3; ++d) Fn[d][k] = 0.0;
        if (j * G + k >= ng) continue;
        double Pv[3];
        pressure_dot_v(a.closure, a.c, Enew[k], s.Fk[0][k], s.Fk[1][k], s.Fk[2][k], v, Pv);
        const double emit = m[k].chiB * m[k].Bt - m[k].DchiB / 3.0;
        const double den = 1.0 + cdt * m[k].chiF;
        for (int d = 0; d < 3; ++d) {
          // eq. numF1
          const double f =
              (s.F0[d][k] + cdt * (v[d] * emit + (1.0 + m[k].ac) * m[k].chiE * Pv[d])) / den;
          Fn[d][k] = f;
          dmom[d] += f - s.F0[d][k];
        }
      }
      const double ccc = 1.0 / (a.c * a.chat);
      double vn[3];
      for (int d = 0; d < 3; ++d) {
        dmom[d] = cell_sum<LPC>(dmom[d]);
        vn[d] = (rho * v0[d] - dmom[d] * ccc) / rho;  // momentum update
      }
      double dW = 0.0;
#pragma unroll
      for (int k = 0; k < G; ++k) {
        if (j * G + k >= ng) continue;
        const double vf_new = vn[0] * Fn[0][k] + vn[1] * Fn[1][k] + vn[2] * Fn[2][k];
        const double vf_old = v[0] * s.Fk[0][k] + v[1] * s.Fk[1][k] + v[2] * s.Fk[2][k];
        dW += fabs(cdt * (1.0 + m[k].ac) * m[k].chiF * (vf_new - vf_old)) / (a.c * a.c);
      }
      dW = cell_sum<LPC>(dW);
      // the next inner pass starts from this pass's temperature
      const double ke_new = 0.5 * rho * (vn[0] * vn[0] + vn[1] * vn[1] + vn[2] * vn[2]);
      egv += ke_new - ke;
      for (int d = 0; d < 3; ++d) v[d] = vn[d];
#pragma unroll
      for (int k = 0; k < G; ++k)
        for (int d = 0; d < 3; ++d) s.Fk[d][k] = Fn[d][k];
      if (dW < a.eps_out * etot) break;
      if (k_out + 1 >= a.max_outer) {
        st |= MGRHD_ST_OUTER_MAXIT;
        break;
      }
    }
    if (!(st & MGRHD_ST_INVALID)) {
      double bad = (isfinite(egas_new) && isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]))
                       ? 0.0 : 1.0;
#pragma unroll
      for (int k = 0; k < G; ++k) {
        if (j * G + k >= ng) continue;
        if (!isfinite(s.E0[k] + s.R[k])) bad = 1.0;
        for (int d = 0; d < 3; ++d)
          if (!isfinite(s.Fk[d][k])) bad = 1.0;
      }
      bad = cell_sum<LPC>(bad);
      if (bad != 0.0) {
        st |= MGRHD_ST_NONFINITE;
      } else {
#pragma unroll
        for (int k = 0; k < G; ++k) {
          const int g = j * G + k;
          if (g >= ng) continue;
          const double sg = a.S ? a.S[(int64_t)g * n + i] : 0.0;
          (void)sg;
          a.E[(int64_t)g * n + i] = s.E0[k] + s.R[k];
          for (int d = 0; d < 3; ++d) a.F[((int64_t)d * ng + g) * n + i] = s.Fk[d][k];
        }
        if (j == 0) {
          a.egas[i] = egas_new;
          a.v[i] = v[0];
          a.v[n + i] = v[1];
          a.v[2 * n + i] = v[2];
        }
      }
    }
  }
  if (j == 0) {
    if (a.status) a.status[i] = st;
    if (a.iters) a.iters[i] = steps;
    if (a.outer) a.outer[i] = passes;
  }
}

// ---------------------------------------------------------------------------
// Variant table
using KernelFn = void (*)(KArgs);

struct Variant {
  int lpc, g;
  KernelFn fn[3];
};

#define MGRHD_VARIANT(G_, LPC_)                                                   \
  {                                                                               \
    LPC_, G_, {                                                                   \
      k_source_update<G_, LPC_, MGRHD_MEAN_PC>,                                   \
          k_source_update<G_, LPC_, MGRHD_MEAN_PPL_FIXED>,                        \
          k_source_update<G_, LPC_, MGRHD_MEAN_PPL_FREE>                          \
    }                                                                             \
  }

static const Variant kVariants[] = {
    MGRHD_VARIANT(4, 1),  MGRHD_VARIANT(4, 2),  MGRHD_VARIANT(4, 4),  MGRHD_VARIANT(4, 8),
    MGRHD_VARIANT(4, 16), MGRHD_VARIANT(4, 32), MGRHD_VARIANT(4, 64), MGRHD_VARIANT(2, 2),
    MGRHD_VARIANT(2, 4),  MGRHD_VARIANT(2, 8),  MGRHD_VARIANT(2, 16), MGRHD_VARIANT(2, 32),
    MGRHD_VARIANT(8, 1),  MGRHD_VARIANT(8, 2),  MGRHD_VARIANT(8, 4),  MGRHD_VARIANT(8, 8),
    MGRHD_VARIANT(8, 16), MGRHD_VARIANT(1, 4),
};

// user overrides per group count (0 = built-in choice)
static int g_override_lpc[MGRHD_MAX_GROUPS + 1];
static int g_override_g[MGRHD_MAX_GROUPS + 1];

static const Variant* find_variant(int lpc, int g) {
  for (const Variant& v : kVariants)
    if (v.lpc == lpc && v.g == g) return &v;
  return nullptr;
}

static const Variant* choose_variant(int ng) {
  if (g_override_lpc[ng]) {
    const Variant* v = find_variant(g_override_lpc[ng], g_override_g[ng]);
    if (v && v->lpc * v->g >= ng) return v;
  }
  // default: 4 groups per lane, enough lanes to cover N_g
  int lpc = 1;
  while (lpc * 4 < ng) lpc <<= 1;
  return find_variant(lpc, 4);
}

}  // namespace mgrhd

using namespace mgrhd;

extern "C" {

const char* mgrhd_version(void) { return "mgrhd 0.1 (gfx950, fp64)"; }

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
  o->max_outer = 10;
  o->closure = MGRHD_CLOSURE_M1;
  o->polish = 0;
}

int mgrhd_get_variant(int32_t n_groups, int32_t mean_mode, int32_t* lpc, int32_t* gpl) {
  (void)mean_mode;
  if (n_groups < 1 || n_groups > MGRHD_MAX_GROUPS) return MGRHD_E_SIZE;
  const Variant* v = choose_variant(n_groups);
  if (!v) return MGRHD_E_OPTION;
  if (lpc) *lpc = v->lpc;
  if (gpl) *gpl = v->g;
  return 0;
}

int mgrhd_set_variant(int32_t n_groups, int32_t lpc, int32_t gpl) {
  if (n_groups < 1 || n_groups > MGRHD_MAX_GROUPS) return MGRHD_E_SIZE;
  if (lpc == 0 && gpl == 0) {
    g_override_lpc[n_groups] = g_override_g[n_groups] = 0;
    return 0;
  }
  const Variant* v = find_variant(lpc, gpl);
  if (!v || v->lpc * v->g < n_groups) return MGRHD_E_OPTION;
  g_override_lpc[n_groups] = lpc;
  g_override_g[n_groups] = gpl;
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
  if (n_cells == 0) return 0;
  if (!E_g || !F_g || !rho || !e_gas || !v || !group_edges || !op->chi_lo) return MGRHD_E_NULL;
  if (op->mean_mode != MGRHD_MEAN_PC && !op->alpha_chi && !op->chi_hi) return MGRHD_E_TABLE;
  auto pos = [](double x) { return x > 0.0 && std::isfinite(x); };
  if (!pos(dt) || !pos(c_hat) || !pos(opt->c) || !pos(opt->a_rad) || !pos(opt->h_over_k) ||
      !pos(opt->c_v))
    return MGRHD_E_SCALAR;
  if (!pos(opt->eps_newton) || !pos(opt->eps_outer) || opt->max_newton < 1 ||
      opt->max_outer < 1 || opt->polish < 0 || opt->polish > 4)
    return MGRHD_E_OPTION;

  const Variant* var = choose_variant(ng);
  if (!var) return MGRHD_E_OPTION;

  KArgs a;
  std::memset(&a, 0, sizeof(a));
  a.E = E_g;
  a.F = F_g;
  a.rho = rho;
  a.egas = e_gas;
  a.v = v;
  a.kappa = op->kappa_scale;
  a.S = opt->S_g;
  a.guess = opt->guess;
  a.iters = opt->iters;
  a.outer = opt->outer;
  a.status = opt->status;
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

  const int64_t threads = n_cells * var->lpc;
  const int64_t blocks = (threads + kBlock - 1) / kBlock;
  if (blocks > 0x7fffffffLL) return MGRHD_E_SIZE;
  hipLaunchKernelGGL(var->fn[op->mean_mode], dim3((unsigned)blocks), dim3(kBlock), 0,
                     (hipStream_t)stream, a);
  const hipError_t err = hipGetLastError();
  return err == hipSuccess ? 0 : (int)err;
}

}  // extern "C"
