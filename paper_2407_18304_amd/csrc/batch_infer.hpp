// batch_infer.hpp -- what the batched launch and the warm-start network share:
// the work items of a batch of patches and the fused inference over a range
// of them (one launch per group count), so that a batch can run its
// warm-start inference and its solve in one captured graph.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "solver_device.hpp"

struct mgrhd_mlp;

namespace mgrhd {

// cells [c0, c1) of patch `patch`
struct BatchItem {
  int32_t patch;
  int32_t pad;
  int64_t c0, c1;
};

// 0 if the network m fits patches of n_groups groups (inputs 2 + 3 N_g,
// outputs 1 + N_g, the fused path's hidden width), else MGRHD_E_SIZE.
int mlp_check_patches(const mgrhd_mlp* m, int32_t n_groups);

// Enqueue on s the fused inference of m over the items [lo, hi) of a batch
// (device arrays of the patches' arguments and of the items; every patch of
// the range has n_groups groups and a guess buffer of the layout of `kind`):
// each patch's guess is written into its guess buffer.  Allocates nothing.
int mlp_infer_items(mgrhd_mlp* m, const KArgs* d_patches, const BatchItem* d_items, int64_t lo,
                    int64_t hi, int32_t n_groups, int32_t kind, const float* x_mean,
                    const float* x_istd, const float* y_mean, const float* y_std, hipStream_t s);

}  // namespace mgrhd
