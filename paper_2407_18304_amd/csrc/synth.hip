// synth.hip -- device generator of the seeded synthetic source-update inputs.
//
// Test and benchmark infrastructure: it draws inputs only and holds none of
// the source-update arithmetic.  It implements the counter-based hash and the
// transforms of paper_2407_18304_amd/workloads.py cell by cell, so that any
// cell generated here equals the host generator's cell up to the last-bit
// differences of exp/log/cos between the two math libraries:
//
//   splitmix64(z): z += 0x9E3779B97F4A7C15; z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9;
//                  z = (z ^ (z >> 27)) * 0x94D049BB133111EB; return z ^ (z >> 31)
//   draw(seed, field, cell, sub) = splitmix64(splitmix64(splitmix64(splitmix64(seed)
//                                  ^ field) ^ cell) ^ sub);  uniform = (draw >> 11) 2^-53
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace {

enum { F_T = 0, F_TRAD = 2, F_V = 3, F_KAPPA = 4, F_FLUX = 5, F_DIR = 6 };

__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double uniform(uint64_t s0 /* splitmix64(seed) */, uint64_t field,
                                          uint64_t cell, uint64_t sub) {
  uint64_t z = splitmix64(s0 ^ field);
  z = splitmix64(z ^ cell);
  z = splitmix64(z ^ sub);
  return (double)(z >> 11) * 0x1.0p-53;
}

struct SynthArgs {
  double* E;       // [ng][n]
  double* F;       // [3][ng][n]
  double* rho;     // [n]
  double* egas;    // [n]
  double* v;       // [3][n]
  double* kappa;   // [n]
  double* T;       // [n] or null
  const double* edges;  // [ng+1] device
  const double* gl;     // [2*nq] Gauss-Legendre nodes then weights on [-1, 1]
  int64_t n, cell0;     // cells cell0 .. cell0+n-1 of the workload
  uint64_t seed;
  int32_t ng, nq;
  int32_t t_kind;       // 0: T = exp(s N(0,1)), 1: T = 10^U(p0, p1)
  int32_t k_kind;       // 0: kappa log-uniform [p0, p1], 1: tau = 10^U(p0,p1), kappa = tau*kscale
  double t_p0, t_p1, k_p0, k_p1, k_scale;
  double trad_lo, trad_hi, vmax, c, a_rad, c_v;
};

__global__ void k_synth(SynthArgs a) {
  const int64_t li = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (li >= a.n) return;
  const uint64_t cell = (uint64_t)(a.cell0 + li);
  const uint64_t s0 = splitmix64(a.seed);
  const double pi = 3.14159265358979323846;
  double T;
  if (a.t_kind == 0) {
    const double u1 = uniform(s0, F_T, cell, 0), u2 = uniform(s0, F_T, cell, 1);
    const double z = sqrt(-2.0 * log1p(-u1)) * cos(2.0 * pi * u2);
    T = exp(a.t_p1 * z);
  } else {
    T = pow(10.0, a.t_p0 + (a.t_p1 - a.t_p0) * uniform(s0, F_T, cell, 0));
  }
  double kap;
  const double uk = uniform(s0, F_KAPPA, cell, 0);
  if (a.k_kind == 0) {
    kap = exp(log(a.k_p0) + (log(a.k_p1) - log(a.k_p0)) * uk);
  } else {
    kap = pow(10.0, a.k_p0 + (a.k_p1 - a.k_p0) * uk) * a.k_scale;
  }
  const double trad = T * (a.trad_lo + (a.trad_hi - a.trad_lo) * uniform(s0, F_TRAD, cell, 0));
  double v[3];
  for (int d = 0; d < 3; ++d) v[d] = (2.0 * uniform(s0, F_V, cell, d) - 1.0) * a.vmax * a.c;
  const double rho = 1.0;
  const int64_t n = a.n;
  const double lnT = log(trad);
  const double T4 = a.a_rad * (trad * trad) * (trad * trad) * (15.0 / (pi * pi * pi * pi));
  for (int g = 0; g < a.ng; ++g) {
    const double lo = log(a.edges[g]), hi = log(a.edges[g + 1]);
    const double half = 0.5 * (hi - lo), mid = 0.5 * (hi + lo);
    double acc = 0.0;
    for (int q = 0; q < a.nq; ++q) {
      const double u = mid + half * a.gl[q] - lnT;   // ln t
      const double t = exp(u);
      double f = exp(4.0 * u - t) / (-expm1(-t));     // t^4/(e^t - 1)
      if (!isfinite(f)) f = 0.0;
      acc += (a.gl[a.nq + q] * half) * f;
    }
    const double E = T4 * acc;
    const double fr = 0.5 * uniform(s0, F_FLUX, cell, (uint64_t)g);
    const double zc = 2.0 * uniform(s0, F_DIR, cell, 2 * (uint64_t)g) - 1.0;
    const double ph = 2.0 * pi * uniform(s0, F_DIR, cell, 2 * (uint64_t)g + 1);
    const double s = sqrt(fmax(0.0, 1.0 - zc * zc));
    a.E[(int64_t)g * n + li] = E;
    const double amp = fr * a.c * E;
    a.F[((int64_t)0 * a.ng + g) * n + li] = amp * (s * cos(ph));
    a.F[((int64_t)1 * a.ng + g) * n + li] = amp * (s * sin(ph));
    a.F[((int64_t)2 * a.ng + g) * n + li] = amp * zc;
  }
  a.rho[li] = rho;
  a.egas[li] = rho * a.c_v * T + 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  for (int d = 0; d < 3; ++d) a.v[(int64_t)d * n + li] = v[d];
  a.kappa[li] = kap;
  if (a.T) a.T[li] = T;
}

}  // namespace

extern "C" int mgrhd_synth_state(double* E, double* F, double* rho, double* egas, double* v,
                                 double* kappa, double* T, const double* edges, const double* gl,
                                 int64_t n, int64_t cell0, uint64_t seed, int32_t ng, int32_t nq,
                                 int32_t t_kind, double t_p0, double t_p1, int32_t k_kind,
                                 double k_p0, double k_p1, double k_scale, double trad_lo,
                                 double trad_hi, double vmax, double c, double a_rad, double c_v,
                                 void* stream) {
  if (n <= 0) return 0;
  if (!E || !F || !rho || !egas || !v || !kappa || !edges || !gl || ng < 1 || nq < 1) return -1;
  SynthArgs a{E, F, rho, egas, v, kappa, T, edges, gl, n, cell0, seed, ng, nq, t_kind, k_kind,
              t_p0, t_p1, k_p0, k_p1, k_scale, trad_lo, trad_hi, vmax, c, a_rad, c_v};
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_synth, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}
