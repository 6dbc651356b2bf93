// source_update_tdep.hip -- the single-table source-update kernels for an
// opacity that depends on temperature, (T/T_ref)^t_exp [1 - e^{-x}]^stim,
// evaluated at every Newton iterate.  Same variants as source_update.hip.
#include "solver_kernel.hpp"

namespace mgrhd {

KernelFn tdep_kernel(int k, int mode) {
#define MGRHD_TDEP_VARIANT(G_, LPC_, WPE_) MGRHD_VARIANT_MODES(G_, LPC_, WPE_, true),
  static const KernelFn fns[][3] = {MGRHD_FOR_EACH_VARIANT(MGRHD_TDEP_VARIANT)};
#undef MGRHD_TDEP_VARIANT
  constexpr int n = (int)(sizeof(fns) / sizeof(fns[0]));
  if (k < 0 || k >= n || mode < 0 || mode > 2) return nullptr;
  return fns[k][mode];
}

}  // namespace mgrhd
