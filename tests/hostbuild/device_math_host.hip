// Host build of the device math of the source-update kernels, so that the CPU
// test suite can pin it against mpmath without a GPU.  Test infrastructure.
#include "../../paper_2407_18304_amd/csrc/planck_device.hpp"

extern "C" {
void dm_edge(double x, double* out) {
  const mgrhd::Edge e = mgrhd::planck_edge(x);
  out[0] = e.val;
  out[1] = e.eps;
  out[2] = e.u;
  out[3] = e.wien ? 1.0 : 0.0;
}
void dm_edge_low(double x, double* out) {
  const mgrhd::Edge e = mgrhd::planck_edge_low(x);
  out[0] = e.val;
  out[1] = e.eps;
  out[2] = e.u;
  out[3] = e.wien ? 1.0 : 0.0;
}
void dm_group(double xl, double xh, double* out) {
  const mgrhd::GroupPlanck p = mgrhd::group_planck(mgrhd::planck_edge(xl), mgrhd::planck_edge(xh));
  out[0] = p.b;
  out[1] = p.elo;
  out[2] = p.ehi;
  out[3] = p.sigma;
  out[4] = p.scale;
}
double dm_mean_ratio(double ac, double aq, double L) { return mgrhd::mean_ratio(ac, aq, L); }
double dm_exp_neg(double x) { return mgrhd::exp_neg(x); }
}
