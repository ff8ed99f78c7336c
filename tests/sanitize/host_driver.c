/*
 * Driver of the library's host code for the sanitizer build (tests/test_sanitizers.py):
 * every C-ABI call on the paths that return before any device call (argument and parameter
 * validation, tuning-table queries, null handles), against a host-only build of
 * liblesmi with -fsanitize=address,undefined. Needs no GPU.
 */
#include <stdio.h>
#include <string.h>

#include "../../include/lesmi.h"

#define CHECK(expr, want)                                                    \
  do {                                                                       \
    long long rc_ = (long long)(expr);                                       \
    if (rc_ != (long long)(want)) {                                          \
      fprintf(stderr, "%s:%d: %s returned %lld, expected %lld\n", __FILE__, \
              __LINE__, #expr, rc_, (long long)(want));                      \
      return 1;                                                              \
    }                                                                        \
  } while (0)

static les_params jet(int ni, int nj, int nk) {
  les_params p;
  memset(&p, 0, sizeof p);
  p.ni = ni;
  p.nj = nj;
  p.nk = nk;
  int bc[6] = {LES_BC_JET_INFLOW, LES_BC_EXIT, LES_BC_AXIS, LES_BC_FARFIELD, LES_BC_PERIODIC,
               LES_BC_PERIODIC};
  memcpy(p.bc, bc, sizeof bc);
  p.gamma = 1.4;
  p.prandtl = 0.72;
  p.prandtl_sgs = 0.6;
  p.re_acoustic = 71428.57;
  p.cs = 0.18;
  p.k2 = 0.25;
  p.k4 = 0.016;
  return p;
}

int main(void) {
  double xyz[3] = {0, 0, 0};
  les_ctx* c = (les_ctx*)0;
  les_params p;
  /* parameter validation */
  CHECK(les_init_grid(NULL, xyz, &c), LES_EINVAL);
  p = jet(8, 8, 8);
  CHECK(les_init_grid(&p, NULL, &c), LES_EINVAL);
  CHECK(les_init_grid(&p, xyz, NULL), LES_EINVAL);
  p = jet(3, 8, 8);
  CHECK(les_init_grid(&p, xyz, &c), LES_EINVAL);
  p = jet(8, 8, 8);
  p.bc[1] = LES_BC_PERIODIC;
  CHECK(les_init_grid(&p, xyz, &c), LES_EINVAL);
  p = jet(8, 8, 8);
  p.bc[2] = LES_BC_FARFIELD;
  CHECK(les_init_grid(&p, xyz, &c), LES_EINVAL);
  p = jet(8, 8, 8);
  p.gamma = 1.0;
  CHECK(les_init_grid(&p, xyz, &c), LES_EINVAL);
  p = jet(8, 8, 8);
  p.precision = 7;
  CHECK(les_init_grid(&p, xyz, &c), LES_EINVAL);
  p = jet(8, 8, 8);
  p.closure = -1;
  CHECK(les_init_grid(&p, xyz, &c), LES_EINVAL);
  p = jet(1200, 600, 300);
  CHECK(les_init_grid(&p, xyz, &c), LES_EINVAL);
  if (c) return 1;
  /* null contexts */
  double buf[8];
  CHECK(les_residual(NULL, buf, buf, NULL), LES_EINVAL);
  CHECK(les_step(NULL, buf, 1, 0.5, 0.0, NULL, NULL), LES_EINVAL);
  CHECK(les_sgs_viscosity(NULL, buf, buf, NULL), LES_EINVAL);
  CHECK(les_apply_bc(NULL, buf, NULL), LES_EINVAL);
  CHECK(les_diagnostics(NULL, buf, buf, NULL), LES_EINVAL);
  CHECK(les_residual_norms(NULL, buf, buf, NULL), LES_EINVAL);
  CHECK(les_stats_reset(NULL), LES_EINVAL);
  CHECK(les_stats_accumulate(NULL, buf, NULL), LES_EINVAL);
  CHECK(les_stats_read(NULL, buf, buf, NULL, NULL), LES_EINVAL);
  CHECK(les_get_metrics(NULL, buf, buf, NULL), LES_EINVAL);
  CHECK(les_updated_nodes(NULL), 0);
  CHECK(les_set_tuning(NULL, 0, 8), LES_EINVAL);
  CHECK(les_profile(NULL, 1), LES_EINVAL);
  CHECK(les_profile_read(NULL, NULL, NULL, NULL), LES_EINVAL);
  CHECK(les_autotune(NULL, buf, NULL, NULL, NULL), LES_EINVAL);
  CHECK(les_mlp_set_network(NULL, NULL, NULL), LES_EINVAL);
  CHECK(les_mlp_fallback_count(NULL, NULL), LES_EINVAL);
  CHECK(les_mlp_features(NULL, buf, NULL, NULL, NULL), LES_EINVAL);
  les_destroy(NULL);
  if (strcmp(les_last_error(NULL), "null context") != 0) return 1;
  /* tuning table */
  int nt = les_tuning_count();
  if (nt < 1) return 1;
  for (int t = -2; t < nt + 2; ++t) {
    const char* name = les_tuning_name(t);
    if (!name || ((t < 0 || t >= nt) && name[0])) return 1;
  }
  /* learned-closure and batch argument checks */
  float f[8];
  les_mlp_norm norm;
  memset(&norm, 0, sizeof norm);
  CHECK(les_mlp_coefficient(NULL, &norm, 0.03f, f, f, 1, f, NULL, NULL), LES_EINVAL);
  CHECK(les_mlp_coefficient(f, &norm, 0.03f, f, f, -1, f, NULL, NULL), LES_EINVAL);
  CHECK(les_mlp_coefficient(f, &norm, 0.03f, f, f, 0, f, NULL, NULL), LES_OK);
  CHECK(les_mlp_loss_grad(f, &norm, f, 1, f, f, NULL, 1, 1.f, f, NULL, f, NULL), LES_EINVAL);
  CHECK(les_mlp_adam(f, f, f, f, 0, 1e-3f, 0.9f, 0.999f, 1e-8f, NULL), LES_EINVAL);
  CHECK(les_mlp_fit_norm(f, f, 0, 0.1f, &norm, NULL), LES_EINVAL);
  CHECK(les_filter_target(NULL, NULL, NULL, 1.f, NULL, NULL, NULL, NULL, NULL, NULL, NULL),
        LES_EINVAL);
  if (les_mlp_work_size(4096) < 1) return 1;
  les_batch* b = (les_batch*)0;
  CHECK(les_batch_create(NULL, 1, &b), LES_EINVAL);
  CHECK(les_batch_create((les_ctx* const*)&c, 0, &b), LES_EINVAL);
  CHECK(les_batch_create((les_ctx* const*)&c, 1, NULL), LES_EINVAL);
  CHECK(les_batch_set_tuning(NULL, 0, 8), LES_EINVAL);
  CHECK(les_batch_get_tuning(NULL, NULL, NULL), LES_EINVAL);
  CHECK(les_batch_set_graph(NULL, 1), LES_EINVAL);
  CHECK(les_batch_step(NULL, NULL, 1, 0.5, 0.0, NULL, NULL), LES_EINVAL);
  CHECK(les_batch_autotune(NULL, NULL, NULL, NULL, NULL), LES_EINVAL);
  les_batch_destroy(NULL);
  if (strcmp(les_batch_last_error(NULL), "null batch") != 0) return 1;
  printf("host driver ok\n");
  return 0;
}
