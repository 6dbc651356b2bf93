// source_update_tdep.hip -- the single-table source-update kernels for an
// opacity that depends on temperature, (T/T_ref)^t_exp [1 - e^{-x}]^stim,
// evaluated at every Newton iterate.  Same variants as source_update.hip.
#include "solver_kernel.hpp"

namespace mgrhd {

#define MGRHD_TABLE_ROW(G_, LPC_, WPE_) MGRHD_VARIANT_MODES(G_, LPC_, WPE_, true, false),
MGRHD_DEFINE_KERNEL_TABLE(tdep_kernel)
#undef MGRHD_TABLE_ROW

}  // namespace mgrhd
