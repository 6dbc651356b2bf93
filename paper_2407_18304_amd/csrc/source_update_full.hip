// source_update_full.hip -- the single-table source-update kernels for
// N_g = LPC * G (every slot of every lane holds a group, so the per-slot group
// checks compile away).  Same variants as source_update.hip.
#include "solver_kernel.hpp"

namespace mgrhd {

#define MGRHD_TABLE_ROW(G_, LPC_, WPE_) MGRHD_VARIANT_MODES(G_, LPC_, WPE_, false, true),
MGRHD_DEFINE_KERNEL_TABLE(full_kernel)
#undef MGRHD_TABLE_ROW

}  // namespace mgrhd
