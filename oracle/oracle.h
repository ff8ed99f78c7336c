/*
 * Plain FP64 CPU oracle for the LES residual and time stepping of
 * Junqueira-Junior, Yamouni, Azevedo & Wolf, "Large Eddy Simulations of Supersonic Jet
 * Flows for Aeroacoustic Applications" (arXiv 2212.12365).
 *
 * TEST INFRASTRUCTURE ONLY. This library is what the GPU library is checked against.
 * Only the test suite, the package smoke check and the benchmark's CPU-baseline leg may
 * load it. It shares no code, header, table or helper with the GPU library.
 *
 * Layout: a field f of a grid with ni x nj x nk nodes is stored f[c][k][j][i] (i fastest);
 * node (i,j,k) has offset i + ni*(j + nj*k). Directions d = 0,1,2 are xi (i), eta (j),
 * zeta (k). Metric arrays S[9][N] hold S_d^c = J^-1 * d(xi_d)/d(x_c) at index 3*d + c.
 *
 * Every function returns 0 on success or a negative code:
 *   -1 invalid parameters, -2 out of memory, -3 bad grid (J^-1 <= 0 away from the axis),
 *   -5 non-finite value or non-positive density/pressure after a step.
 */
#ifndef LES_ORACLE_H
#define LES_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_BC_PERIODIC = 0, OR_BC_AXIS = 1, OR_BC_JET_INFLOW = 2, OR_BC_FARFIELD = 3,
       OR_BC_EXIT = 4 };

typedef struct {
  int ni, nj, nk;
  int bc[6];                  /* faces i-, i+, j-, j+, k-, k+ */
  double period_shift[3][3];  /* [direction][x,y,z]: coordinate jump across a periodic wrap */
  double gamma, prandtl, prandtl_sgs;
  double re_acoustic;         /* rho_ref a_ref L / mu_ref; 0 = no molecular viscosity */
  double suth_s1;             /* Sutherland constant over the reference temperature */
  double cs, k2, k4;
  double mach_jet, jet_radius, rho_inf, u_inf[3], p_inf;
  int metric_form;            /* 0 conservative (Thomas-Lombard), 1 plain cross products */
} or_params;

int or_metrics(const or_params* P, const double* xyz, double* S, double* jinv);
int or_sutherland(const or_params* P, int n, const double* T, double* mu);
int or_sgs_viscosity(const or_params* P, const double* S, const double* jinv,
                     const double* q, double* mu_t);
/* Residual with the eddy viscosity mu_t [N] given instead of computed. */
int or_residual_mut(const or_params* P, const double* S, const double* jinv, const double* q,
                    const double* mu_t, double* rhs);
/* grad [9][N]: d u_m / d x_n at index 3m + n (0 where J^-1 <= 0). */
int or_velocity_gradient(const or_params* P, const double* S, const double* jinv,
                         const double* q, double* grad);
int or_residual(const or_params* P, const double* S, const double* jinv, const double* q,
                double* rhs);
int or_apply_bc(const or_params* P, const double* xyz, const double* S, const double* jinv,
                double* q);
int or_dt(const or_params* P, const double* S, const double* jinv, const double* q,
          double cfl, double* dt);
int or_step(const or_params* P, const double* xyz, const double* S, const double* jinv,
            double* q, int nsteps, double cfl, double dt_fixed, double* dt_last);
int or_diagnostics(const or_params* P, const double* jinv, const double* q, double* out);

#ifdef __cplusplus
}
#endif
#endif
