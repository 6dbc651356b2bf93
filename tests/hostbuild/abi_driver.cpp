// Host-side paths of the C ABI that return before anything touches a device
// (defaults, version, the variant table, the mean-mode recommendation,
// workspace sizes, argument checks of every entry point), for a build of the
// library's host code with AddressSanitizer and UndefinedBehaviorSanitizer.
// Exits non-zero on an unexpected return code.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "mgrhd.h"

static int bad = 0;
static void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("unexpected: %s\n", what);
    bad = 1;
  }
}

int main() {
  mgrhd_options o;
  mgrhd_default_options(&o);
  expect(o.max_outer == 20 && o.max_newton == 100 && o.polish == 0, "defaults");
  expect(std::strstr(mgrhd_version(), "gfx950") != nullptr, "version");
  const int nv = mgrhd_variant_count();
  for (int k = 0; k < nv; ++k) {
    int32_t l, g, w;
    expect(mgrhd_variant_info(k, &l, &g, &w) == 0 && l * g >= 1, "variant info");
  }
  expect(mgrhd_variant_info(nv, nullptr, nullptr, nullptr) == MGRHD_E_OPTION, "variant range");
  for (int ng = 1; ng <= MGRHD_MAX_GROUPS; ++ng) {
    int32_t l, g, w;
    expect(mgrhd_get_variant(ng, 1, &l, &g, &w) == 0 && l * g >= ng, "get variant");
  }
  expect(mgrhd_get_variant(0, 1, nullptr, nullptr, nullptr) == MGRHD_E_SIZE, "variant size");
  expect(mgrhd_set_variant(64, 4, 4, 0) == MGRHD_E_OPTION, "set variant too narrow");
  expect(mgrhd_set_variant(16, 8, 2, 0) == 0 && mgrhd_set_variant(16, 0, 0, 0) == 0,
         "set and reset variant");
  std::vector<double> e(129);
  for (int k = 0; k <= 128; ++k) e[k] = std::pow(10.0, -3.0 + 6.0 * k / 128.0);
  for (int ng : {1, 4, 10, 11, 128}) {
    std::vector<double> eg(ng + 1);
    for (int k = 0; k <= ng; ++k) eg[k] = std::pow(10.0, -3.0 + 6.0 * k / ng);
    const int m = mgrhd_recommend_mean_mode(ng, eg.data());
    expect(m == (ng <= 10 ? MGRHD_MEAN_PPL_FIXED : MGRHD_MEAN_PC), "recommendation");
  }
  double desc[3] = {1.0, 0.5, 2.0};
  expect(mgrhd_recommend_mean_mode(2, desc) == MGRHD_E_TABLE, "descending edges");
  expect(mgrhd_imex_workspace_bytes(1000, 16) == 8u * 1000 * 68, "workspace");
  // argument checks (pointers never dereferenced)
  double* f = reinterpret_cast<double*>(64);
  mgrhd_opacity_params op{};
  op.n_groups = 4;
  op.mean_mode = 1;
  expect(mgrhd_source_update(nullptr, nullptr, nullptr, nullptr, nullptr, 10, nullptr, nullptr,
                             1.0, 1.0, nullptr, &o) == MGRHD_E_NULL, "null opacity");
  op.n_groups = MGRHD_MAX_GROUPS + 1;
  expect(mgrhd_source_update(f, f, f, f, f, 10, f, &op, 1.0, 1.0, nullptr, &o) == MGRHD_E_SIZE,
         "group count");
  op.n_groups = 4;
  op.mean_mode = 9;
  expect(mgrhd_source_update(f, f, f, f, f, 10, f, &op, 1.0, 1.0, nullptr, &o) == MGRHD_E_MODE,
         "mode");
  op.mean_mode = 1;
  op.chi_lo = f;
  op.alpha_chi = f;
  op.t_exp = 1.5;
  op.t_ref = -1.0;
  expect(mgrhd_source_update(f, f, f, f, f, 10, f, &op, 1.0, 1.0, nullptr, &o) == MGRHD_E_TABLE,
         "temperature reference");
  op.t_exp = 0.0;
  mgrhd_options bado = o;
  bado.max_newton = 0;
  expect(mgrhd_source_update(f, f, f, f, f, 10, f, &op, 1.0, 1.0, nullptr, &bado) ==
             MGRHD_E_OPTION, "max_newton");
  expect(mgrhd_source_update(f, f, f, f, f, 10, f, &op, -1.0, 1.0, nullptr, &o) ==
             MGRHD_E_SCALAR, "dt");
  mgrhd_options outo = o;  // out of place: all four outputs or none
  outo.E_g_out = f;
  expect(mgrhd_source_update(f, f, f, f, f, 10, f, &op, 1.0, 1.0, nullptr, &outo) ==
             MGRHD_E_NULL, "one output of four");
  expect(mgrhd_imex_step(f, f, f, f, f, 10, f, &op, 1.0, 1.0, nullptr, &outo, f, 1 << 20) ==
             MGRHD_E_NULL, "imex: one output of four");
  expect(mgrhd_imex_step_noalloc(f, f, f, f, f, 10, f, &op, 1.0, 1.0, nullptr, &outo) ==
             MGRHD_E_NULL, "noalloc: one output of four");
  expect(mgrhd_imex_step(f, f, f, f, f, 10, f, &op, 1.0, 1.0, nullptr, &o, nullptr, 0) ==
             MGRHD_E_NULL, "imex workspace");
  expect(mgrhd_imex_step(f, f, f, f, f, 10, f, &op, 1.0, 1.0, nullptr, &o, f, 8) == MGRHD_E_SIZE,
         "imex workspace size");
  expect(mgrhd_imex_step_noalloc(f, f, f, f, f, 1 << 22, f, &op, 1.0, 1.0, nullptr, &o) ==
             MGRHD_E_SIZE, "noalloc limit");
  expect(mgrhd_transport1d_stage(f, f, f, f, f, f, f, f, nullptr, nullptr, nullptr, nullptr, 0.0,
                                 1.0, 10, 0, 1.0, 1.0, 1.0, 1.0, f, f, f, f, nullptr) ==
             MGRHD_E_SIZE, "transport groups");
  expect(mgrhd_transport1d_stage(f, f, f, f, f, f, f, f, nullptr, nullptr, nullptr, nullptr, 0.0,
                                 1.0, 10, 4, 0.0, 1.0, 1.0, 1.0, f, f, f, f, nullptr) ==
             MGRHD_E_SCALAR, "transport dx");
  expect(mgrhd_batch_create(nullptr, 3, 1, &o, nullptr) == MGRHD_E_NULL, "batch out");
  mgrhd_batch* b = reinterpret_cast<mgrhd_batch*>(1);
  expect(mgrhd_batch_create(nullptr, 3, 1, &o, &b) == MGRHD_E_NULL && b == nullptr, "batch null");
  expect(mgrhd_batch_set_item_scope(nullptr, 1) == MGRHD_E_NULL, "batch scope");
  expect(mgrhd_batch_tune(nullptr, nullptr) == MGRHD_E_NULL, "batch tune");
  expect(mgrhd_batch_create(nullptr, 0, 1, &outo, &b) == MGRHD_E_OPTION && b == nullptr,
         "batch out of place");
  mgrhd_mlp* m = nullptr;
  expect(mgrhd_mlp_create(0, 128, 5, 64, 1, &m) == MGRHD_E_SIZE && m == nullptr, "mlp dims");
  expect(mgrhd_mlp_create(10, 300, 5, 64, 1, &m) == MGRHD_E_SIZE, "mlp width");
  expect(mgrhd_mlp_set_fp32_products(nullptr, 1) == MGRHD_E_NULL, "mlp fp32");
  expect(mgrhd_mlp_save(nullptr, "/nonexistent") == MGRHD_E_NULL, "mlp save");
  expect(mgrhd_mlp_load(nullptr, "/nonexistent") == MGRHD_E_NULL, "mlp load");
  expect(mgrhd_mlp_gemm(nullptr, 1, 0, nullptr, 1, 0, nullptr, 1, 1, 1, 1, 0, nullptr) ==
             MGRHD_E_NULL, "gemm null");
  expect(mgrhd_mlp_gemm(reinterpret_cast<float*>(f), 1, 0, reinterpret_cast<float*>(f), 1, 0,
                        reinterpret_cast<float*>(f), 1, 1, 1, 1, 3, nullptr) == MGRHD_E_OPTION,
         "gemm precision");
  std::printf("abi driver: %s\n", bad ? "FAILED" : "ok");
  return bad;
}
