/*
 * Driver of the CPU oracle for the sanitizer build (tests/test_sanitizers.py): calls every
 * entry point of oracle/oracle.h on a small polar jet grid (entrance, exit, centreline, far
 * field, periodic azimuth) and on a skewed periodic box, plus the invalid-parameter paths,
 * and checks the return codes. Built with -fsanitize=address,undefined; any report fails.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/oracle.h"

#define CHECK(expr, want)                                                    \
  do {                                                                       \
    int rc_ = (expr);                                                        \
    if (rc_ != (want)) {                                                     \
      fprintf(stderr, "%s:%d: %s returned %d, expected %d\n", __FILE__,     \
              __LINE__, #expr, rc_, (want));                                 \
      return 1;                                                              \
    }                                                                        \
  } while (0)

static void base_params(or_params* p, int ni, int nj, int nk) {
  memset(p, 0, sizeof *p);
  p->ni = ni;
  p->nj = nj;
  p->nk = nk;
  p->gamma = 1.4;
  p->prandtl = 0.72;
  p->prandtl_sgs = 0.6;
  p->re_acoustic = 1000.0;
  p->suth_s1 = 110.4 / 288.15;
  p->cs = 0.18;
  p->k2 = 0.25;
  p->k4 = 0.016;
  p->mach_jet = 1.4;
  p->jet_radius = 0.5;
  p->rho_inf = 1.0;
  p->u_inf[0] = 0.05;
  p->p_inf = 1.0 / 1.4;
}

static void fill_state(const or_params* p, const double* xyz, double* q) {
  long N = (long)p->ni * p->nj * p->nk;
  for (long id = 0; id < N; ++id) {
    double x = xyz[id], y = xyz[N + id], z = xyz[2 * N + id];
    double r = sqrt(y * y + z * z);
    double rho = 1.0 + 0.02 * sin(x + y);
    double u = 0.05 + 1.35 * 0.5 * (1.0 - tanh((r - 0.5) / 0.1)) + 0.01 * cos(z + x);
    double v = 0.01 * sin(2.0 * x), w = 0.01 * cos(y - x);
    double pr = 1.0 / 1.4 + 0.01 * cos(x - z);
    q[id] = rho;
    q[N + id] = rho * u;
    q[2 * N + id] = rho * v;
    q[3 * N + id] = rho * w;
    q[4 * N + id] = pr / 0.4 + 0.5 * rho * (u * u + v * v + w * w);
  }
}

static int run_case(or_params* p, const double* xyz) {
  long N = (long)p->ni * p->nj * p->nk;
  double* S = calloc(9 * N, sizeof(double));
  double* jinv = calloc(N, sizeof(double));
  double* q = calloc(5 * N, sizeof(double));
  double* rhs = calloc(5 * N, sizeof(double));
  double* mut = calloc(N, sizeof(double));
  double* grad = calloc(9 * N, sizeof(double));
  double* T = calloc(N, sizeof(double));
  double* mu = calloc(N, sizeof(double));
  double diag[6], dt = 0.0, dt_last = 0.0;
  if (!S || !jinv || !q || !rhs || !mut || !grad || !T || !mu) return 1;
  CHECK(or_metrics(p, xyz, S, jinv), 0);
  fill_state(p, xyz, q);
  CHECK(or_apply_bc(p, xyz, S, jinv, q), 0);
  CHECK(or_residual(p, S, jinv, q, rhs), 0);
  CHECK(or_sgs_viscosity(p, S, jinv, q, mut), 0);
  CHECK(or_residual_mut(p, S, jinv, q, mut, rhs), 0);
  CHECK(or_velocity_gradient(p, S, jinv, q, grad), 0);
  for (long i = 0; i < N; ++i) T[i] = 0.5 + (double)(i % 7) * 0.25;
  CHECK(or_sutherland(p, (int)N, T, mu), 0);
  CHECK(or_dt(p, S, jinv, q, 0.5, &dt), 0);
  CHECK(or_step(p, xyz, S, jinv, q, 3, 0.5, 0.0, &dt_last), 0);
  CHECK(or_step(p, xyz, S, jinv, q, 1, 0.0, 0.5 * dt_last, NULL), 0);
  CHECK(or_diagnostics(p, jinv, q, diag), 0);
  p->metric_form = 1;
  CHECK(or_metrics(p, xyz, S, jinv), 0);
  p->metric_form = 0;
  for (long i = 0; i < 5 * N; ++i)
    if (!isfinite(q[i])) return 1;
  free(S); free(jinv); free(q); free(rhs); free(mut); free(grad); free(T); free(mu);
  return 0;
}

int main(void) {
  /* Polar jet grid: x axial, r from the axis (j = 0) outwards, nk azimuthal nodes. */
  or_params p;
  int ni = 10, nj = 8, nk = 8;
  base_params(&p, ni, nj, nk);
  int jet_bc[6] = {OR_BC_JET_INFLOW, OR_BC_EXIT, OR_BC_AXIS, OR_BC_FARFIELD, OR_BC_PERIODIC,
                   OR_BC_PERIODIC};
  memcpy(p.bc, jet_bc, sizeof jet_bc);
  long N = (long)ni * nj * nk;
  double* xyz = malloc(3 * N * sizeof(double));
  if (!xyz) return 1;
  for (int k = 0; k < nk; ++k)
    for (int j = 0; j < nj; ++j)
      for (int i = 0; i < ni; ++i) {
        long id = i + (long)ni * (j + (long)nj * k);
        double th = 2.0 * M_PI * k / nk, r = 0.15 * j;
        xyz[id] = 0.3 * i;
        xyz[N + id] = r * cos(th);
        xyz[2 * N + id] = r * sin(th);
      }
  if (run_case(&p, xyz)) return 1;

  /* Skewed triply periodic box. */
  or_params b;
  int n = 6;
  base_params(&b, n, n, n);
  for (int d = 0; d < 3; ++d) b.period_shift[d][d] = 2.0 * M_PI;
  long M = (long)n * n * n;
  double* bx = malloc(3 * M * sizeof(double));
  if (!bx) return 1;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        long id = i + (long)n * (j + (long)n * k);
        double s1 = 2 * M_PI * i / n, s2 = 2 * M_PI * j / n, s3 = 2 * M_PI * k / n;
        bx[id] = s1 + 0.3 * sin(s2) * sin(s3);
        bx[M + id] = s2 + 0.3 * sin(s3) * sin(s1);
        bx[2 * M + id] = s3 + 0.3 * sin(s1) * sin(s2);
      }
  if (run_case(&b, bx)) return 1;

  /* Invalid parameter sets are refused. */
  double dummy[16] = {0};
  or_params bad = b;
  bad.ni = 3;
  CHECK(or_metrics(&bad, dummy, dummy, dummy), -1);
  bad = b;
  bad.bc[0] = OR_BC_AXIS;
  CHECK(or_residual(&bad, dummy, dummy, dummy, dummy), -1);
  bad = b;
  bad.gamma = 1.0;
  CHECK(or_dt(&bad, dummy, dummy, dummy, 0.5, dummy), -1);
  CHECK(or_step(&b, bx, dummy, dummy, dummy, -1, 0.5, 0.0, NULL), -1);
  free(xyz);
  free(bx);
  printf("oracle driver ok\n");
  return 0;
}
