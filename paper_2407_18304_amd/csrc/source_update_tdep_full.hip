// source_update_tdep_full.hip -- the single-table source-update kernels for
// a temperature-dependent opacity and N_g = LPC * G.  Same variants as
// source_update.hip.
#include "solver_kernel.hpp"

namespace mgrhd {

#define MGRHD_TABLE_ROW(G_, LPC_, WPE_) MGRHD_VARIANT_MODES(G_, LPC_, WPE_, true, true),
MGRHD_DEFINE_KERNEL_TABLE(tdep_full_kernel)
#undef MGRHD_TABLE_ROW

}  // namespace mgrhd
