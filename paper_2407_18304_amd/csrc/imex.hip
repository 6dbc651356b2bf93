// imex.hip -- one step of the two-stage IMEX integrator (Sec. 2.3, eqs. imex1
// and imex2) restricted to the source terms: with no transport, the first
// stage is the source update from U^(n) with theta dt = dt, and the second is
// the source update with theta dt = dt/2 from the midpoint (U^(n) +
// U^(n+1/2))/2 (eq. imex2 with dt S(U^(n+1/2)) = U^(n+1/2) - U^(n)).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "../../include/mgrhd.h"

namespace mgrhd {
namespace imex {

// Library-owned U^(n+1/2) for mgrhd_imex_step_noalloc: a file-scope
// device array (one per GPU the library runs on, held until the process
// ends).  Host code never uses this name as an address: it takes the array's
// device address per device from hipGetSymbolAddress (scratch_ptr below).
__device__ __align__(256) double scratch[MGRHD_IMEX_SCRATCH_DOUBLES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch[kMaxDevices];

// Device address of `scratch` on the current device, looked up once per
// device; NULL if the lookup fails.
void* scratch_ptr(hipError_t* err) {
  int dev = 0;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return nullptr;
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

// The four state arrays of one side of the midpoint.
struct State4 {
  double *E, *F, *eg, *v;
};

// y <- (x + w) / 2 over the four arrays, w laid end to end in the workspace
// order (E_g, F_g, e_gas, v); y may be x (in place)
__global__ void k_midpoint(State4 y, State4 x, const double* __restrict__ w, int64_t nE,
                           int64_t n) {
  const int64_t total = 4 * nE + 4 * n;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
       k += (int64_t)gridDim.x * blockDim.x) {
    double *dst, *src;
    int64_t o;
    if (k < nE) {
      dst = y.E, src = x.E;
      o = k;
    } else if (k < 4 * nE) {
      dst = y.F, src = x.F;
      o = k - nE;
    } else if (k < 4 * nE + n) {
      dst = y.eg, src = x.eg;
      o = k - 4 * nE;
    } else {
      dst = y.v, src = x.v;
      o = k - 4 * nE - n;
    }
    dst[o] = 0.5 * (src[o] + w[k]);
  }
}

}  // namespace imex
}  // namespace mgrhd

extern "C" {

size_t mgrhd_imex_workspace_bytes(int64_t n_cells, int32_t n_groups) {
  if (n_cells < 0 || n_groups < 1) return 0;
  return sizeof(double) * (size_t)n_cells * (4 * (size_t)n_groups + 4);
}

int mgrhd_imex_step_noalloc(double* E_g, double* F_g, const double* rho, double* e_gas,
                            double* v, int64_t n_cells, const double* group_edges,
                            const mgrhd_opacity_params* opacity, double dt, double c_hat,
                            mgrhd_stream_t stream, const mgrhd_options* opt) {
  if (!opacity) return MGRHD_E_NULL;
  if (n_cells < 0 || opacity->n_groups < 1 || opacity->n_groups > MGRHD_MAX_GROUPS)
    return MGRHD_E_SIZE;
  const int n_out = opt ? !!opt->E_g_out + !!opt->F_g_out + !!opt->e_gas_out + !!opt->v_out : 0;
  if (n_out != 0 && n_out != 4) return MGRHD_E_NULL;  // out of place needs all four
  const size_t need = mgrhd_imex_workspace_bytes(n_cells, opacity->n_groups);
  if (need > sizeof(double) * (size_t)MGRHD_IMEX_SCRATCH_DOUBLES) return MGRHD_E_SIZE;
  hipError_t err = hipSuccess;
  void* w = mgrhd::imex::scratch_ptr(&err);
  if (!w) return err != hipSuccess ? (int)err : MGRHD_E_DEVICE;
  return mgrhd_imex_step(E_g, F_g, rho, e_gas, v, n_cells, group_edges, opacity, dt, c_hat,
                         stream, opt, w, sizeof(double) * (size_t)MGRHD_IMEX_SCRATCH_DOUBLES);
}

int mgrhd_imex_step(double* E_g, double* F_g, const double* rho, double* e_gas, double* v,
                    int64_t n_cells, const double* group_edges,
                    const mgrhd_opacity_params* opacity, double dt, double c_hat,
                    mgrhd_stream_t stream, const mgrhd_options* opt, void* work,
                    size_t work_bytes) {
  if (!opacity || !work) return MGRHD_E_NULL;
  if (n_cells < 0 || opacity->n_groups < 1 || opacity->n_groups > MGRHD_MAX_GROUPS)
    return MGRHD_E_SIZE;
  const int n_out = opt ? !!opt->E_g_out + !!opt->F_g_out + !!opt->e_gas_out + !!opt->v_out : 0;
  if (n_out != 0 && n_out != 4) return MGRHD_E_NULL;  // out of place needs all four
  if (work_bytes < mgrhd_imex_workspace_bytes(n_cells, opacity->n_groups)) return MGRHD_E_SIZE;
  if (!(dt > 0.0)) return MGRHD_E_SCALAR;
  if (n_cells == 0) return 0;
  if (!E_g || !F_g || !e_gas || !v) return MGRHD_E_NULL;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = n_cells, nE = n * opacity->n_groups;
  double* w = (double*)work;
  mgrhd_options o1;
  if (opt)
    o1 = *opt;
  else
    mgrhd_default_options(&o1);
  // where U^(n+1) goes: the caller's arrays (in place) or the outputs
  const mgrhd::imex::State4 un{E_g, F_g, e_gas, v};
  const mgrhd::imex::State4 un1 =
      n_out ? mgrhd::imex::State4{o1.E_g_out, o1.F_g_out, o1.e_gas_out, o1.v_out} : un;
  // first stage, out of place: U^(n+1/2) = U^(n) + dt S(U^(n+1/2)) into the
  // workspace (E_g, F_g, e_gas, v end to end), U^(n) left in the caller's arrays
  o1.E_g_out = w;
  o1.F_g_out = w + nE;
  o1.e_gas_out = w + 4 * nE;
  o1.v_out = w + 4 * nE + n;
  int rc = mgrhd_source_update(E_g, F_g, rho, e_gas, v, n, group_edges, opacity, dt, c_hat,
                               stream, &o1);
  if (rc) return rc;
  // second stage from the midpoint (U^(n) + U^(n+1/2))/2, formed where
  // U^(n+1) goes, with theta dt = dt / 2, in place there
  int64_t blocks = (4 * nE + 4 * n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(mgrhd::imex::k_midpoint, dim3((unsigned)blocks), dim3(256), 0, s, un1, un,
                     (const double*)w, nE, n);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  mgrhd_options o2 = o1;
  o2.E_g_out = o2.F_g_out = o2.e_gas_out = o2.v_out = nullptr;
  return mgrhd_source_update(un1.E, un1.F, rho, un1.eg, un1.v, n, group_edges, opacity,
                             0.5 * dt, c_hat, stream, &o2);
}

}  // extern "C"
