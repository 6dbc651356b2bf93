// solver_kernel.hpp -- the single-table source-update kernel and the list of
// its compiled variants, shared by the four translation units that
// instantiate it (T-independent or T-dependent opacity, any N_g or
// N_g = LPC * G: source_update.hip, source_update_tdep.hip,
// source_update_full.hip, source_update_tdep_full.hip, compiled in parallel).
#pragma once
#include <hip/hip_runtime.h>

#include "solver_device.hpp"

namespace mgrhd {

// TD: the opacity depends on temperature (evaluated at every iterate).
// FULL: N_g = LPC * G (the launcher checks), every slot holds a group.
template <int G, int LPC, int MODE, int WPE, bool TD, bool FULL>
__global__ __launch_bounds__(kBlock, WPE) void k_source_update(KArgs a) {
  constexpr int NGM = G * LPC;
  __shared__ Tables<NGM> tab;
  using LS = LaneStore<G, true, kBlock / LPC>;
  __shared__ double lane_lds[LS::kSlots * kBlock];
  __shared__ double cell_lds[LS::kCellWords];
  // the arguments as the device reads them in place (a is the only argument)
  const KArgsRef ap = (KArgsRef)__builtin_amdgcn_kernarg_segment_ptr();
  const LS ls{lane_lds + threadIdx.x, cell_lds, ap};
  __shared__ int taken;  // cells of this workgroup's range handed out so far
  if (threadIdx.x == 0) taken = 0;
  const bool table_ok = stage_tables<NGM, MODE>(a, tab);  // (its barriers publish `taken`)

  const int lane = threadIdx.x % kWave;
  // each workgroup owns a contiguous range of cells, shared by its waves
  const int64_t lo = a.n * blockIdx.x / gridDim.x, hi = a.n * (blockIdx.x + 1) / gridDim.x;

  if (!table_ok) {
    // the table is unusable: report every cell of this workgroup's range
    for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
      copy_through(a, state_ptrs(ap), i, 0, 1);
      if (a.status) a.status[i] = MGRHD_ST_BAD_TABLE;
      if (a.iters) a.iters[i] = 0;
      if (a.outer) a.outer[i] = 0;
      if (a.trace)
        for (int k = 0; k < a.max_outer; ++k) a.trace[(int64_t)k * a.n + i] = -1;
    }
    return;
  }

  run_cells<G, LPC, MODE, NGM, TD, FULL>(a, tab, ls, lane, BlockQueue{&taken, lo, hi});
}

using KernelFn = void (*)(KArgs);

// (groups per lane, lanes per cell, minimum waves per SIMD) of every compiled
// variant.  The first entry of each (lanes per cell, groups per lane) pair is
// its default register budget; the others trade registers (spills) for waves.
#define MGRHD_FOR_EACH_VARIANT(X)                                                 \
  X(4, 1, 2) X(4, 2, 2) X(4, 4, 2) X(4, 8, 2) X(4, 16, 2) X(4, 32, 2) X(4, 64, 2) \
  X(2, 2, 3) X(2, 4, 3) X(2, 8, 3) X(2, 16, 3) X(2, 32, 3)                        \
  X(1, 4, 4) X(1, 8, 4) X(1, 16, 4) X(1, 32, 4) X(1, 64, 4)                       \
  X(2, 8, 4) X(2, 32, 4)

// the three mean modes of one variant
#define MGRHD_VARIANT_MODES(G_, LPC_, WPE_, TD_, FULL_)                            \
  {                                                                               \
    k_source_update<G_, LPC_, MGRHD_MEAN_PC, WPE_, TD_, FULL_>,                   \
        k_source_update<G_, LPC_, MGRHD_MEAN_PPL_FIXED, WPE_, TD_, FULL_>,        \
        k_source_update<G_, LPC_, MGRHD_MEAN_PPL_FREE, WPE_, TD_, FULL_>          \
  }

// A kernel table: the kernel of variant k (in MGRHD_FOR_EACH_VARIANT order)
// and mean mode, or nullptr; the including file defines MGRHD_TABLE_ROW.
#define MGRHD_DEFINE_KERNEL_TABLE(NAME)                                            \
  KernelFn NAME(int k, int mode) {                                                \
    static const KernelFn fns[][3] = {MGRHD_FOR_EACH_VARIANT(MGRHD_TABLE_ROW)};   \
    constexpr int n = (int)(sizeof(fns) / sizeof(fns[0]));                        \
    if (k < 0 || k >= n || mode < 0 || mode > 2) return nullptr;                  \
    return fns[k][mode];                                                          \
  }

// The kernels of the other three translation units, by variant and mode.
KernelFn tdep_kernel(int k, int mode);       // TD, any N_g (source_update_tdep.hip)
KernelFn full_kernel(int k, int mode);       // N_g = LPC * G (source_update_full.hip)
KernelFn tdep_full_kernel(int k, int mode);  // both (source_update_tdep_full.hip)

}  // namespace mgrhd
