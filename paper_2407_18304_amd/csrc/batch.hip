// batch.hip -- one persistent launch over many AMR-like patches, each with its
// own cell count, group count, group edges and opacity table (the patch
// layout of an adaptive mesh, where every patch holds its own SoA block).
//
// Work list: the patches are cut into items of at most `chunk` cells, ordered
// by decreasing group count (the costliest work first, so the tail of the
// launch is made of cheap items).  A wave takes the next item with one atomic
// increment of a global counter, stages that patch's tables in its own LDS
// slot, sets its lane count per cell to the next power of two >= N_g/G, and
// runs the same per-cell state machine as the single-table kernel (cell
// groups refill from the item's cells as their cells finish).  A tiny kernel
// clears the counter before the persistent kernel, so the pair can be
// captured in a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/mgrhd.h"
#include "batch_infer.hpp"
#include "solver_device.hpp"

namespace mgrhd {

constexpr int kBatchNGM = 128;  // group capacity of a wave's LDS table slot

using Item = BatchItem;

struct BatchArgs {
  const KArgs* patches;  // device array, one KArgs per patch
  const Item* items;     // device array
  int32_t* counter;      // device, cleared before each launch
  int64_t n_items;
};

__global__ void k_clear_counter(int32_t* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Stage the tables of one patch into this wave's LDS slot (wave scope).
template <int MODE, int NGM>
__device__ __forceinline__ bool stage_tables_wave(const KArgs& a, Tables<NGM>& t, int lane) {
  if (lane == 0) t.bad = 0;
  wave_sync();
  const int ng = a.ng;
  if (ng > NGM) {
    t.bad = 1;
    wave_sync();
    return false;
  }
  for (int g = lane; g <= ng; g += kWave)
    if (!table_edge<NGM, MODE>(a, t, g)) atomicOr(&t.bad, 1);
  wave_sync();
  for (int g = lane; g < ng; g += kWave)
    if (!table_group<NGM, MODE>(a, t, g)) atomicOr(&t.bad, 1);
  wave_sync();
  return t.bad == 0;
}

// A copy of *p in scalar registers: every lane reads the same words and the
// first lane's value is taken, so the compiler knows the fields are uniform.
template <class T>
__device__ __forceinline__ T load_uniform(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "whole words");
  constexpr int kWords = sizeof(T) / 4;
  int w[kWords];
  const int* src = reinterpret_cast<const int*>(p);
#pragma unroll
  for (int k = 0; k < kWords; ++k) w[k] = __builtin_amdgcn_readfirstlane(src[k]);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}

// Lanes per cell for N_g groups at G groups per lane: the next power of two
// >= N_g / G.  The state machine is compiled for each.
template <int G, int MODE, int NGM, bool FULL, class LS, class Q>
__device__ __forceinline__ void run_item_lpc(const KArgs& a, const Tables<NGM>& tab,
                                             const LS& ls, int lane, Q q, int lpc) {
  switch (lpc) {
    case 1: run_cells<G, 1, MODE, NGM, false, FULL>(a, tab, ls, lane, q); break;
    case 2: run_cells<G, 2, MODE, NGM, false, FULL>(a, tab, ls, lane, q); break;
    case 4: run_cells<G, 4, MODE, NGM, false, FULL>(a, tab, ls, lane, q); break;
    case 8: run_cells<G, 8, MODE, NGM, false, FULL>(a, tab, ls, lane, q); break;
    case 16: run_cells<G, 16, MODE, NGM, false, FULL>(a, tab, ls, lane, q); break;
    case 32: run_cells<G, 32, MODE, NGM, false, FULL>(a, tab, ls, lane, q); break;
    default:  // a patch wider than 32 lanes of G groups
      if constexpr (G * 32 < NGM) run_cells<G, kWave, MODE, NGM, false, FULL>(a, tab, ls, lane, q);
      break;
  }
}

// TRY_FULL: items whose N_g fills every slot (N_g = lanes per cell x G) run
// the state machine compiled for that case (no per-slot group checks).
template <int G, int MODE, int NGM, bool TRY_FULL, class LS, class Q>
__device__ __forceinline__ void run_item(const KArgs& a, const Tables<NGM>& tab,
                                         const LS& ls_block, int lane, Q q) {
  // a is an entry of the batch's device array of patch arguments
  const LS ls = ls_block.with_args((KArgsRef)&a);
  int lpc = 1;
  while (lpc * G < a.ng) lpc <<= 1;
  if (TRY_FULL && lpc * G == a.ng)
    run_item_lpc<G, MODE, NGM, true>(a, tab, ls, lane, q, lpc);
  else
    run_item_lpc<G, MODE, NGM, false>(a, tab, ls, lane, q, lpc);
}

// 2 groups per lane leave room in LDS for the old-time fluxes and velocity
// (re-reading them from HBM in the outer stage, or a table slot narrower than
// 128 groups to fit a third workgroup per CU, measured slower: the extra
// registers spill); with 4 they are re-read from HBM by the outer stage.
template <int G, int MODE, int NGM>
__global__ __launch_bounds__(kBlock, 2) void k_batch(BatchArgs b) {
  static_assert(G * kWave >= NGM, "a wave holds the widest patch");
  __shared__ Tables<NGM> tabs[kBlock / kWave];
  using LS = LaneStore<G, G == 2, kBlock, true>;  // constants read where used
  __shared__ double lane_lds[LS::kSlots * kBlock];
  __shared__ double cell_lds[LS::kCellWords];
  const LS ls{lane_lds + threadIdx.x, cell_lds, nullptr};  // run_item sets the arguments
  const int lane = threadIdx.x % kWave;
  Tables<NGM>& tab = tabs[threadIdx.x / kWave];
  int cur_patch = -1;
  bool table_ok = false;
  for (;;) {
    // the wave takes the next work item (all lanes are active here)
    int it = 0;
    if (lane == 0) it = atomicAdd(b.counter, 1);
    it = __builtin_amdgcn_readfirstlane(it);
    if (it >= b.n_items) break;
    const Item item = load_uniform(b.items + it);
    const KArgs& a = b.patches[item.patch];
    if (item.patch != cur_patch) {
      table_ok = stage_tables_wave<MODE, NGM>(a, tab, lane);
      cur_patch = item.patch;
    }
    if (!table_ok) {
      for (int64_t i = item.c0 + lane; i < item.c1; i += kWave) {
        copy_through(a, state_ptrs((KArgsRef)&a), i, 0, 1);  // out of place: inputs
        if (a.status) a.status[i] = MGRHD_ST_BAD_TABLE;
        if (a.iters) a.iters[i] = 0;
        if (a.outer) a.outer[i] = 0;
        if (a.trace)
          for (int k = 0; k < a.max_outer; ++k) a.trace[(int64_t)k * a.n + i] = -1;
      }
      continue;
    }
    run_item<G, MODE, NGM, false>(a, tab, ls, lane, WaveRange{item.c0, item.c1});
  }
}

// Items per workgroup: the four waves of a workgroup take one item together,
// share one LDS table slot (so LDS leaves room for 3 workgroups per CU) and
// take the item's cells through an LDS counter, so the cells in flight in a
// workgroup share the cache lines of every SoA row.  Waves that run out of
// cells wait at the item's end for the others.
// WPE: waves per SIMD the register allocation must allow (LDS allows 3 at 2
// groups per lane; at 3 a few registers spill, at 2 none do).
template <int G, int MODE, int NGM, int WPE>
__global__ __launch_bounds__(kBlock, WPE) void k_batch_wg(BatchArgs b) {
  static_assert(G * kWave >= NGM, "a wave holds the widest patch");
  __shared__ Tables<NGM> tab;
  __shared__ int item_s, taken;
  using LS = LaneStore<G, G == 2, kBlock, true>;  // constants read where used
  __shared__ double lane_lds[LS::kSlots * kBlock];
  __shared__ double cell_lds[LS::kCellWords];
  const LS ls{lane_lds + threadIdx.x, cell_lds, nullptr};  // run_item sets the arguments
  const int lane = threadIdx.x % kWave;
  int cur_patch = -1;
  bool table_ok = false;
  for (;;) {
    if (threadIdx.x == 0) {
      item_s = atomicAdd(b.counter, 1);
      taken = 0;
    }
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(item_s);
    if (it >= b.n_items) break;
    const Item item = load_uniform(b.items + it);
    const KArgs& a = b.patches[item.patch];
    if (item.patch != cur_patch) {  // uniform over the workgroup
      table_ok = stage_tables<NGM, MODE>(a, tab);
      cur_patch = item.patch;
    }
    if (!table_ok) {
      for (int64_t i = item.c0 + threadIdx.x; i < item.c1; i += kBlock) {
        copy_through(a, state_ptrs((KArgsRef)&a), i, 0, 1);  // out of place: inputs
        if (a.status) a.status[i] = MGRHD_ST_BAD_TABLE;
        if (a.iters) a.iters[i] = 0;
        if (a.outer) a.outer[i] = 0;
        if (a.trace)
          for (int k = 0; k < a.max_outer; ++k) a.trace[(int64_t)k * a.n + i] = -1;
      }
    } else {
      run_item<G, MODE, NGM, true>(a, tab, ls, lane, BlockQueue{&taken, item.c0, item.c1});
    }
    __syncthreads();  // the item is done before the next one resets the counter
  }
}

using BatchFn = void (*)(BatchArgs);
// the kernel for g groups per lane, mean mode, and items per wave (scope 0) or
// per workgroup (scope 1: register budget for 3 waves per SIMD at 2 groups
// per lane; scope 2: for 2 waves)
static BatchFn batch_fn(int g, int mode, int scope) {
  static const BatchFn wave[2][3] = {
      {k_batch<2, MGRHD_MEAN_PC, kBatchNGM>, k_batch<2, MGRHD_MEAN_PPL_FIXED, kBatchNGM>,
       k_batch<2, MGRHD_MEAN_PPL_FREE, kBatchNGM>},
      {k_batch<4, MGRHD_MEAN_PC, kBatchNGM>, k_batch<4, MGRHD_MEAN_PPL_FIXED, kBatchNGM>,
       k_batch<4, MGRHD_MEAN_PPL_FREE, kBatchNGM>}};
  static const BatchFn wg3[3] = {k_batch_wg<2, MGRHD_MEAN_PC, kBatchNGM, 3>,
                                 k_batch_wg<2, MGRHD_MEAN_PPL_FIXED, kBatchNGM, 3>,
                                 k_batch_wg<2, MGRHD_MEAN_PPL_FREE, kBatchNGM, 3>};
  static const BatchFn wg2[2][3] = {
      {k_batch_wg<2, MGRHD_MEAN_PC, kBatchNGM, 2>, k_batch_wg<2, MGRHD_MEAN_PPL_FIXED, kBatchNGM, 2>,
       k_batch_wg<2, MGRHD_MEAN_PPL_FREE, kBatchNGM, 2>},
      {k_batch_wg<4, MGRHD_MEAN_PC, kBatchNGM, 2>, k_batch_wg<4, MGRHD_MEAN_PPL_FIXED, kBatchNGM, 2>,
       k_batch_wg<4, MGRHD_MEAN_PPL_FREE, kBatchNGM, 2>}};
  const int gi = g == 4 ? 1 : 0;
  if (scope == 0) return wave[gi][mode];
  if (scope == 1 && g == 2) return wg3[mode];
  return wg2[gi][mode];
}

}  // namespace mgrhd

using namespace mgrhd;

struct mgrhd_batch {
  int32_t n_patches = 0;
  int32_t mode = 0;
  int64_t n_cells = 0;
  int32_t max_groups = 0;
  KArgs* d_patches = nullptr;
  Item* d_items = nullptr;
  int32_t* d_counter = nullptr;
  int64_t n_items = 0;
  std::vector<KArgs> h_patches;
  // tuning
  int32_t groups_per_lane = 2;
  int32_t scope = 1;          // 0: items per wave, 1 | 2: items per workgroup
  int32_t blocks_per_cu = 0;  // 0 = all resident
  int64_t chunk = 256;
  bool items_dirty = true;
  // [first, last) item of each group count (the work list is sorted by
  // decreasing N_g), rebuilt with the work list
  std::vector<std::pair<int32_t, std::pair<int64_t, int64_t>>> ng_items;
  // warm-start networks attached per group count (inference enqueued before
  // the solve)
  struct Net {
    int32_t ng;
    mgrhd_mlp* m;
    const float *x_mean, *x_istd, *y_mean, *y_std;
  };
  std::vector<Net> nets;
  int32_t guess_kind = 0;
  // graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static int build_items(mgrhd_batch* bt) {
  std::vector<Item> items;
  std::vector<int32_t> order(bt->n_patches);
  for (int32_t p = 0; p < bt->n_patches; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    return bt->h_patches[x].ng > bt->h_patches[y].ng;
  });
  bt->ng_items.clear();
  for (int32_t p : order) {
    const int64_t n = bt->h_patches[p].n;
    const int32_t ng = bt->h_patches[p].ng;
    if (bt->ng_items.empty() || bt->ng_items.back().first != ng)
      bt->ng_items.push_back({ng, {(int64_t)items.size(), (int64_t)items.size()}});
    for (int64_t c0 = 0; c0 < n; c0 += bt->chunk)
      items.push_back(Item{p, 0, c0, std::min(n, c0 + bt->chunk)});
    bt->ng_items.back().second.second = (int64_t)items.size();
  }
  if (bt->d_items) (void)hipFree(bt->d_items);
  bt->d_items = nullptr;
  bt->n_items = (int64_t)items.size();
  if (!items.empty()) {
    if (hipMalloc(&bt->d_items, sizeof(Item) * items.size()) != hipSuccess) return MGRHD_E_DEVICE;
    if (hipMemcpy(bt->d_items, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice) !=
        hipSuccess)
      return MGRHD_E_DEVICE;
  }
  bt->items_dirty = false;
  return 0;
}

static void drop_graph(mgrhd_batch* bt) {
  if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  bt->exec = nullptr;
  bt->graph = nullptr;
}

extern "C" {

int mgrhd_batch_create(const mgrhd_patch* patches, int32_t n_patches, int32_t mean_mode,
                       const mgrhd_options* opt_in, mgrhd_batch** out) {
  if (!out) return MGRHD_E_NULL;
  *out = nullptr;
  if (n_patches < 0 || (n_patches > 0 && !patches)) return MGRHD_E_NULL;
  if (mean_mode < 0 || mean_mode > 2) return MGRHD_E_MODE;
  mgrhd_options defaults;
  mgrhd_default_options(&defaults);
  const mgrhd_options* opt = opt_in ? opt_in : &defaults;
  if (opt->closure < 0 || opt->closure > 1) return MGRHD_E_MODE;
  if (opt->E_g_out || opt->F_g_out || opt->e_gas_out || opt->v_out)
    return MGRHD_E_OPTION;  // outputs are given per patch
  auto pos = [](double x) { return x > 0.0 && std::isfinite(x); };
  if (!pos(opt->c) || !pos(opt->a_rad) || !pos(opt->h_over_k) || !pos(opt->c_v))
    return MGRHD_E_SCALAR;
  if (!pos(opt->eps_newton) || !pos(opt->eps_outer) || opt->max_newton < 1 ||
      opt->max_outer < 1 || opt->polish < 0 || opt->polish > 4 || opt->guess_kind < 0 ||
      opt->guess_kind > 1)
    return MGRHD_E_OPTION;
  mgrhd_batch* bt = new (std::nothrow) mgrhd_batch();
  if (!bt) return MGRHD_E_DEVICE;
  bt->n_patches = n_patches;
  bt->mode = mean_mode;
  bt->guess_kind = opt->guess_kind;
  bt->h_patches.resize(n_patches);
  for (int32_t p = 0; p < n_patches; ++p) {
    const mgrhd_patch& q = patches[p];
    if (q.n_cells < 0 || q.n_groups < 1 || q.n_groups > kBatchNGM) {
      delete bt;
      return MGRHD_E_SIZE;
    }
    if (q.n_cells > 0 && (!q.E_g || !q.F_g || !q.rho || !q.e_gas || !q.v || !q.group_edges ||
                          !q.chi_lo)) {
      delete bt;
      return MGRHD_E_NULL;
    }
    if (mean_mode != MGRHD_MEAN_PC && !q.alpha_chi && !q.chi_hi) {
      delete bt;
      return MGRHD_E_TABLE;
    }
    if (!pos(q.dt) || !pos(q.c_hat)) {
      delete bt;
      return MGRHD_E_SCALAR;
    }
    const int n_out = !!q.E_g_out + !!q.F_g_out + !!q.e_gas_out + !!q.v_out;
    if (n_out != 0 && n_out != 4) {  // out of place needs all four
      delete bt;
      return MGRHD_E_NULL;
    }
    KArgs& a = bt->h_patches[p];
    std::memset(&a, 0, sizeof(a));
    a.E = q.E_g;
    a.F = q.F_g;
    a.rho = q.rho;
    a.egas = q.e_gas;
    a.v = q.v;
    a.kappa = q.kappa_scale;
    a.S = q.S_g;
    a.guess = q.guess;
    a.guess_kind = opt->guess_kind;
    a.iters = q.iters;
    a.outer = q.outer;
    a.status = q.status;
    a.trace = q.trace;
    a.Eo = q.E_g_out;  // NULL: set_derived points them at the inputs (in place)
    a.Fo = q.F_g_out;
    a.egaso = q.e_gas_out;
    a.vo = q.v_out;
    a.edges = q.group_edges;
    a.chi_lo = q.chi_lo;
    a.alpha = q.alpha_chi;
    a.chi_hi = q.chi_hi;
    a.n = q.n_cells;
    a.ng = q.n_groups;
    a.closure = opt->closure;
    a.dt = q.dt;
    a.chat = q.c_hat;
    a.c = opt->c;
    a.a = opt->a_rad;
    a.hk = opt->h_over_k;
    a.cv = opt->c_v;
    a.eps = opt->eps_newton;
    a.eps_out = opt->eps_outer;
    a.max_newton = opt->max_newton;
    a.max_outer = opt->max_outer;
    a.polish = opt->polish;
    set_derived(a);
    bt->n_cells += q.n_cells;
    bt->max_groups = std::max(bt->max_groups, q.n_groups);
  }
  if (n_patches > 0) {
    if (hipMalloc(&bt->d_patches, sizeof(KArgs) * n_patches) != hipSuccess ||
        hipMemcpy(bt->d_patches, bt->h_patches.data(), sizeof(KArgs) * n_patches,
                  hipMemcpyHostToDevice) != hipSuccess) {
      mgrhd_batch_destroy(bt);
      return MGRHD_E_DEVICE;
    }
  }
  if (hipMalloc(&bt->d_counter, sizeof(int32_t)) != hipSuccess) {
    mgrhd_batch_destroy(bt);
    return MGRHD_E_DEVICE;
  }
  const int rc = build_items(bt);
  if (rc) {
    mgrhd_batch_destroy(bt);
    return rc;
  }
  *out = bt;
  return 0;
}

int mgrhd_batch_set_tuning(mgrhd_batch* bt, int32_t groups_per_lane, int32_t blocks_per_cu,
                           int64_t chunk_cells) {
  if (!bt) return MGRHD_E_NULL;
  if (groups_per_lane != 2 && groups_per_lane != 4) return MGRHD_E_OPTION;
  if (blocks_per_cu < 0 || chunk_cells < 1) return MGRHD_E_OPTION;
  if (bt->max_groups > groups_per_lane * 64) return MGRHD_E_OPTION;
  const bool changed = groups_per_lane != bt->groups_per_lane ||
                       blocks_per_cu != bt->blocks_per_cu || chunk_cells != bt->chunk;
  if (changed) drop_graph(bt);
  bt->groups_per_lane = groups_per_lane;
  bt->blocks_per_cu = blocks_per_cu;
  if (chunk_cells != bt->chunk) {
    // the work list is rebuilt here, never inside run / capture / launch
    bt->chunk = chunk_cells;
    bt->items_dirty = true;
    return build_items(bt);
  }
  return 0;
}

int mgrhd_batch_set_item_scope(mgrhd_batch* bt, int32_t per_workgroup) {
  if (!bt) return MGRHD_E_NULL;
  if (per_workgroup < 0 || per_workgroup > 2) return MGRHD_E_OPTION;
  if (per_workgroup != bt->scope) {
    bt->scope = per_workgroup;
    drop_graph(bt);
  }
  return 0;
}

int32_t mgrhd_batch_get_item_scope(const mgrhd_batch* bt) {
  return bt ? bt->scope : MGRHD_E_NULL;
}

int mgrhd_batch_get_tuning(const mgrhd_batch* bt, int32_t* groups_per_lane,
                           int32_t* blocks_per_cu, int64_t* chunk_cells) {
  if (!bt) return MGRHD_E_NULL;
  if (groups_per_lane) *groups_per_lane = bt->groups_per_lane;
  if (blocks_per_cu) *blocks_per_cu = bt->blocks_per_cu;
  if (chunk_cells) *chunk_cells = bt->chunk;
  return 0;
}

// the attached networks' inference, one launch per group count
static int enqueue_infer(mgrhd_batch* bt, hipStream_t stream) {
  for (const auto& net : bt->nets)
    for (const auto& r : bt->ng_items)
      if (r.first == net.ng) {
        const int rc = mlp_infer_items(net.m, bt->d_patches, bt->d_items, r.second.first,
                                       r.second.second, net.ng, bt->guess_kind, net.x_mean,
                                       net.x_istd, net.y_mean, net.y_std, stream);
        if (rc) return rc;
      }
  return 0;
}

static int enqueue(mgrhd_batch* bt, hipStream_t stream) {
  if (bt->items_dirty) return MGRHD_E_DEVICE;  // the last rebuild of the work list failed
  if (bt->n_items == 0) return 0;
  if (const int rc = enqueue_infer(bt, stream)) return rc;
  BatchFn fn = batch_fn(bt->groups_per_lane, bt->mode, bt->scope);
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kBlock, 0) != hipSuccess || nb < 1)
    nb = 1;
  if (bt->blocks_per_cu > 0 && bt->blocks_per_cu < nb) nb = bt->blocks_per_cu;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  int64_t blocks = (int64_t)cus * nb;
  // never more takers than items: waves (scope 0) or workgroups (scope 1)
  if (bt->scope) {
    if (blocks > bt->n_items) blocks = bt->n_items;
  } else if (blocks * (kBlock / kWave) > bt->n_items) {
    blocks = (bt->n_items + 3) / 4;
  }
  hipLaunchKernelGGL(k_clear_counter, dim3(1), dim3(64), 0, stream, bt->d_counter);
  BatchArgs args{bt->d_patches, bt->d_items, bt->d_counter, bt->n_items};
  hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(kBlock), 0, stream, args);
  const hipError_t err = hipGetLastError();
  return err == hipSuccess ? 0 : (int)err;
}

int mgrhd_batch_run(mgrhd_batch* bt, mgrhd_stream_t stream) {
  if (!bt) return MGRHD_E_NULL;
  return enqueue(bt, (hipStream_t)stream);
}

int mgrhd_batch_attach_mlp(mgrhd_batch* bt, int32_t n_groups, mgrhd_mlp* m,
                           const float* x_mean, const float* x_istd, const float* y_mean,
                           const float* y_std) {
  if (!bt || !m || !x_mean || !x_istd || !y_mean || !y_std) return MGRHD_E_NULL;
  if (const int rc = mlp_check_patches(m, n_groups)) return rc;
  bool any = false;
  for (const KArgs& a : bt->h_patches)
    if (a.ng == n_groups) {
      if (!a.guess) return MGRHD_E_NULL;  // the inference writes the patch's guess buffer
      any = true;
    }
  if (!any) return MGRHD_E_SIZE;
  for (auto& net : bt->nets)
    if (net.ng == n_groups) {
      net = {n_groups, m, x_mean, x_istd, y_mean, y_std};
      drop_graph(bt);
      return 0;
    }
  bt->nets.push_back({n_groups, m, x_mean, x_istd, y_mean, y_std});
  drop_graph(bt);
  return 0;
}

int mgrhd_batch_infer(mgrhd_batch* bt, mgrhd_stream_t stream) {
  if (!bt) return MGRHD_E_NULL;
  if (bt->items_dirty) return MGRHD_E_DEVICE;
  return enqueue_infer(bt, (hipStream_t)stream);
}

int mgrhd_batch_capture(mgrhd_batch* bt, mgrhd_stream_t stream) {
  if (!bt) return MGRHD_E_NULL;
  drop_graph(bt);
  if (bt->items_dirty) return MGRHD_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return (int)e;
  const int rc = enqueue(bt, st);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(st, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return (int)e;
  bt->graph = g;
  e = hipGraphInstantiate(&bt->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(bt);
    return (int)e;
  }
  return 0;
}

int mgrhd_batch_launch(mgrhd_batch* bt, mgrhd_stream_t stream) {
  if (!bt) return MGRHD_E_NULL;
  if (!bt->exec) {
    const int rc = mgrhd_batch_capture(bt, stream);
    if (rc) return rc;
  }
  const hipError_t e = hipGraphLaunch(bt->exec, (hipStream_t)stream);
  return e == hipSuccess ? 0 : (int)e;
}

int64_t mgrhd_batch_cells(const mgrhd_batch* bt) { return bt ? bt->n_cells : -1; }

void mgrhd_batch_destroy(mgrhd_batch* bt) {
  if (!bt) return;
  drop_graph(bt);
  if (bt->d_patches) (void)hipFree(bt->d_patches);
  if (bt->d_items) (void)hipFree(bt->d_items);
  if (bt->d_counter) (void)hipFree(bt->d_counter);
  delete bt;
}

// ---------------------------------------------------------------------------
// Autotuner: every candidate launch shape runs on copies of the first
// kTuneCells cells of every patch (restored before each run), timed with HIP
// events; the fastest is kept.  The caller's arrays are only read.
static constexpr int64_t kTuneCells = 1024;

namespace {
struct TuneCandidate {
  int32_t groups_per_lane, scope;
  int64_t chunk;
};
constexpr TuneCandidate kTuneCandidates[] = {
    {2, 0, 1024}, {4, 0, 1024}, {2, 1, 256}, {2, 1, 1024}, {2, 2, 256}, {4, 2, 1024}};

struct TuneBuffers {
  double* pristine = nullptr;
  double* work = nullptr;
  int32_t* ints = nullptr;
  ~TuneBuffers() {
    if (pristine) (void)hipFree(pristine);
    if (work) (void)hipFree(work);
    if (ints) (void)hipFree(ints);
  }
};
}  // namespace

int mgrhd_batch_tune(mgrhd_batch* bt, mgrhd_stream_t stream) {
  if (!bt) return MGRHD_E_NULL;
  if (bt->items_dirty) return MGRHD_E_DEVICE;
  if (bt->n_cells == 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  // sample layout: per patch the first ns cells of every row of every field
  const int32_t np = bt->n_patches;
  std::vector<int64_t> ns(np), off(np);
  int64_t nd = 0, ni = 0;
  auto doubles_of = [&](const KArgs& a, int64_t m) {
    int64_t d = (int64_t)a.ng * m * 4 + m * 5;  // E_g, F_g, rho, e_gas, v
    if (a.kappa) d += m;
    if (a.S) d += (int64_t)a.ng * m;
    if (a.guess) d += a.guess_kind == 1 ? m : (int64_t)(a.ng + 1) * m;
    return d;
  };
  for (int32_t p = 0; p < np; ++p) {
    const KArgs& a = bt->h_patches[p];
    ns[p] = std::min<int64_t>(a.n, kTuneCells);
    off[p] = nd;
    nd += doubles_of(a, ns[p]);
    ni += 3 * ns[p];
  }
  TuneBuffers buf;
  if (hipMalloc(&buf.pristine, sizeof(double) * nd) != hipSuccess ||
      hipMalloc(&buf.work, sizeof(double) * nd) != hipSuccess ||
      hipMalloc(&buf.ints, sizeof(int32_t) * ni) != hipSuccess)
    return MGRHD_E_DEVICE;
  // the sample batch: the same patches over the work copies
  mgrhd_batch tmp;
  tmp.n_patches = np;
  tmp.mode = bt->mode;
  tmp.max_groups = bt->max_groups;
  tmp.h_patches = bt->h_patches;
  int64_t io = 0;
  hipError_t e = hipSuccess;
  for (int32_t p = 0; p < np && e == hipSuccess; ++p) {
    const KArgs& a = bt->h_patches[p];
    KArgs& t = tmp.h_patches[p];
    const int64_t m = ns[p];
    double* w = buf.work + off[p];
    double* q = buf.pristine + off[p];
    // copy `rows` rows of m cells (row pitch a.n) of field src into the sample
    auto take = [&](const double* src, int64_t rows) -> double* {
      if (e == hipSuccess && m > 0)
        e = hipMemcpy2DAsync(q, sizeof(double) * m, src, sizeof(double) * a.n,
                             sizeof(double) * m, rows, hipMemcpyDeviceToDevice, st);
      double* here = w;
      w += rows * m;
      q += rows * m;
      return here;
    };
    t.n = m;
    t.E = take(a.E, a.ng);
    t.F = take(a.F, 3 * (int64_t)a.ng);
    t.rho = take(a.rho, 1);
    t.egas = take(a.egas, 1);
    t.v = take(a.v, 3);
    t.Eo = t.E;  // the trial runs update the copies in place
    t.Fo = t.F;
    t.egaso = t.egas;
    t.vo = t.v;
    t.kappa = a.kappa ? take(a.kappa, 1) : nullptr;
    t.S = a.S ? take(a.S, a.ng) : nullptr;
    t.guess = a.guess ? take(a.guess, a.guess_kind == 1 ? 1 : a.ng + 1) : nullptr;
    t.iters = buf.ints + io;
    t.outer = buf.ints + io + m;
    t.status = buf.ints + io + 2 * m;
    t.trace = nullptr;
    io += 3 * m;
    tmp.n_cells += m;
  }
  if (e != hipSuccess) return MGRHD_E_DEVICE;
  int rc = 0;
  if (hipMalloc(&tmp.d_patches, sizeof(KArgs) * np) != hipSuccess ||
      hipMemcpyAsync(tmp.d_patches, tmp.h_patches.data(), sizeof(KArgs) * np,
                     hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMalloc(&tmp.d_counter, sizeof(int32_t)) != hipSuccess)
    rc = MGRHD_E_DEVICE;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = MGRHD_E_DEVICE;
  float best_ms = 0.f;
  const TuneCandidate* best = nullptr;
  for (const TuneCandidate& c : kTuneCandidates) {
    if (rc) break;
    if (bt->max_groups > c.groups_per_lane * 64) continue;
    tmp.groups_per_lane = c.groups_per_lane;
    tmp.scope = c.scope;
    tmp.blocks_per_cu = bt->blocks_per_cu;
    if (c.chunk != tmp.chunk || tmp.items_dirty) {
      tmp.chunk = c.chunk;
      if (hipStreamSynchronize(st) != hipSuccess) { rc = MGRHD_E_DEVICE; break; }
      if ((rc = build_items(&tmp)) != 0) break;
    }
    float ms = 0.f;
    for (int rep = 0; rep < 2 && !rc; ++rep) {  // the first run warms up
      if (hipMemcpyAsync(buf.work, buf.pristine, sizeof(double) * nd, hipMemcpyDeviceToDevice,
                         st) != hipSuccess ||
          hipEventRecord(e0, st) != hipSuccess)
        rc = MGRHD_E_DEVICE;
      if (!rc) rc = enqueue(&tmp, st);
      if (!rc && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = MGRHD_E_DEVICE;
    }
    if (!rc && (!best || ms < best_ms)) {
      best = &c;
      best_ms = ms;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  if (tmp.d_patches) (void)hipFree(tmp.d_patches);
  if (tmp.d_items) (void)hipFree(tmp.d_items);
  if (tmp.d_counter) (void)hipFree(tmp.d_counter);
  if (rc) return rc;
  if (!best) return MGRHD_E_OPTION;
  rc = mgrhd_batch_set_tuning(bt, best->groups_per_lane, bt->blocks_per_cu, best->chunk);
  if (!rc) rc = mgrhd_batch_set_item_scope(bt, best->scope);
  return rc;
}

}  // extern "C"
