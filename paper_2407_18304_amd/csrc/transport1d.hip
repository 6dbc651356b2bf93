// transport1d.hip -- the explicit stage of the two-stage IMEX integrator
// (He, Wibking & Krumholz 2024, Sec. 2.3, eqs. dysf, ysf, imex1, imex2) for a
// 1D column of cells: the M1 transport of every group's energy and x-flux,
//   dE_g/dt = -(c_hat/c) dF_g/dx,   dF_g/dt = -c_hat c dP_g/dx,
//   P_g = chi(f) E_g (Levermore's M1 factor along x, f = |F_g|/(c E_g) <= 1),
// in finite volumes with the local Lax-Friedrichs flux (wave speeds -+c_hat)
// at each face, the dissipation of the energy flux scaled by
// min(1, 1/tau)^2 with tau = dx (chi_L + chi_R)/2, so that optically thick
// cells move energy by the flux the implicit source has relaxed towards its
// diffusion value rather than by numerical diffusion.  Ghost cells hold given
// boundary energies and zero flux.
//
// One launch writes  out = a U0 + b U1 + dt_T T(U1)  for the radiation and
// out = a U0 + b U1 for the gas energy and velocity: stage 1 of a step is
// (a, b, dt_T) = (0, 1, dt) on U^n, stage 2 is (1/2, 1/2, dt/2) with
// U0 = U^n and U1 = U^(n+1/2).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/mgrhd.h"

namespace mgrhd {
namespace {

constexpr int kTBlock = 256;

struct TArgs {
  double *Eo, *Fo, *ego, *vo;
  const double *E1, *F1, *eg1, *v1;
  const double *E0, *F0, *eg0, *v0;
  const double *rho, *chi_mid, *El, *Er;
  double a, b, dx, dtT, c, chat;
  int64_t n;
  int32_t ng;
};

__device__ __forceinline__ double m1_factor(double E, double F, double c) {
  double f = E > 0.0 ? fabs(F) / (c * E) : 0.0;
  f = f < 1.0 ? f : 1.0;
  const double f2 = f * f;
  return (3.0 + 4.0 * f2) / (5.0 + 2.0 * sqrt(4.0 - 3.0 * f2));
}

// energy and x-flux of cell i (ghosts at i = -1 and i = n)
__device__ __forceinline__ void cell(const TArgs& a, int g, int64_t i, double& E, double& F,
                                     double& chi) {
  const int64_t n = a.n;
  const int64_t ic = i < 0 ? 0 : (i >= n ? n - 1 : i);
  chi = a.rho[ic] * a.chi_mid[g];
  if (i < 0) {
    E = a.El[g];
    F = 0.0;
  } else if (i >= n) {
    E = a.Er[g];
    F = 0.0;
  } else {
    E = a.E1[(int64_t)g * n + i];
    F = a.F1[(int64_t)g * n + i];  // x-component: row d = 0 of [3][N_g][n]
  }
}

__device__ __forceinline__ void face_flux(const TArgs& a, double EL, double FL, double chiL,
                                          double ER, double FR, double chiR, double& phE,
                                          double& phF) {
  const double PL = m1_factor(EL, FL, a.c) * EL;
  const double PR = m1_factor(ER, FR, a.c) * ER;
  const double tau = a.dx * 0.5 * (chiL + chiR);
  const double eps = tau > 1.0 ? 1.0 / (tau * tau) : 1.0;
  phE = (a.chat / a.c) * 0.5 * (FL + FR) - eps * a.chat * 0.5 * (ER - EL);
  phF = a.chat * a.c * 0.5 * (PL + PR) - a.chat * 0.5 * (FR - FL);
}

__global__ __launch_bounds__(kTBlock) void k_transport_stage(TArgs a) {
  const int64_t n = a.n;
  const int64_t t = (int64_t)blockIdx.x * kTBlock + threadIdx.x;
  if (t >= n * a.ng) return;
  const int g = (int)(t / n);
  const int64_t i = t - (int64_t)g * n;
  double Em, Fm, cm, E, F, c0, Ep, Fp, cp;
  cell(a, g, i - 1, Em, Fm, cm);
  cell(a, g, i, E, F, c0);
  cell(a, g, i + 1, Ep, Fp, cp);
  double phEl, phFl, phEr, phFr;
  face_flux(a, Em, Fm, cm, E, F, c0, phEl, phFl);
  face_flux(a, E, F, c0, Ep, Fp, cp, phEr, phFr);
  const double dE = -(phEr - phEl) / a.dx;
  const double dF = -(phFr - phFl) / a.dx;
  const int64_t gi = (int64_t)g * n + i;
  const int64_t stride = (int64_t)a.ng * n;  // one flux component
  const bool u0 = a.a != 0.0;
  a.Eo[gi] = a.b * E + (u0 ? a.a * a.E0[gi] : 0.0) + a.dtT * dE;
  a.Fo[gi] = a.b * F + (u0 ? a.a * a.F0[gi] : 0.0) + a.dtT * dF;
#pragma unroll
  for (int d = 1; d < 3; ++d)
    a.Fo[d * stride + gi] = a.b * a.F1[d * stride + gi] + (u0 ? a.a * a.F0[d * stride + gi] : 0.0);
  if (g == 0) {
    a.ego[i] = a.b * a.eg1[i] + (u0 ? a.a * a.eg0[i] : 0.0);
#pragma unroll
    for (int d = 0; d < 3; ++d)
      a.vo[d * n + i] = a.b * a.v1[d * n + i] + (u0 ? a.a * a.v0[d * n + i] : 0.0);
  }
}

}  // namespace
}  // namespace mgrhd

using namespace mgrhd;

extern "C" int mgrhd_transport1d_stage(double* E_out, double* F_out, double* e_gas_out,
                                       double* v_out, const double* E1, const double* F1,
                                       const double* e_gas1, const double* v1, const double* E0,
                                       const double* F0, const double* e_gas0, const double* v0,
                                       double a, double b, int64_t n_cells, int32_t n_groups,
                                       double dx, double dt_T, double c, double c_hat,
                                       const double* rho, const double* chi_mid,
                                       const double* E_left, const double* E_right,
                                       mgrhd_stream_t stream) {
  if (n_cells < 0 || n_groups < 1 || n_groups > MGRHD_MAX_GROUPS) return MGRHD_E_SIZE;
  if (n_cells == 0) return 0;
  if (!E_out || !F_out || !e_gas_out || !v_out || !E1 || !F1 || !e_gas1 || !v1 || !rho ||
      !chi_mid || !E_left || !E_right)
    return MGRHD_E_NULL;
  if (a != 0.0 && (!E0 || !F0 || !e_gas0 || !v0)) return MGRHD_E_NULL;
  auto pos = [](double x) { return x > 0.0 && std::isfinite(x); };
  if (!pos(dx) || !pos(c) || !pos(c_hat) || !std::isfinite(a) || !std::isfinite(b) ||
      !std::isfinite(dt_T) || dt_T < 0.0)
    return MGRHD_E_SCALAR;
  // the stencil reads neighbouring cells of U1: the output must not overlap it
  if (E_out == E1 || F_out == F1) return MGRHD_E_OPTION;
  TArgs t{E_out, F_out, e_gas_out, v_out, E1, F1, e_gas1, v1, E0, F0, e_gas0, v0,
          rho, chi_mid, E_left, E_right, a, b, dx, dt_T, c, c_hat, n_cells, n_groups};
  const int64_t threads = n_cells * n_groups;
  const int64_t blocks = (threads + kTBlock - 1) / kTBlock;
  hipLaunchKernelGGL(k_transport_stage, dim3((unsigned)blocks), dim3(kTBlock), 0,
                     (hipStream_t)stream, t);
  const hipError_t err = hipGetLastError();
  return err == hipSuccess ? 0 : (int)err;
}
