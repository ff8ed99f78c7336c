/*
 * Plain FP64 CPU oracle for the LES hot path of arXiv 2212.12365
 * ("Large Eddy Simulations of Supersonic Jet Flows for Aeroacoustic Applications").
 *
 * TEST INFRASTRUCTURE ONLY: the reference the GPU library is checked against. It is written
 * for clarity, not speed: one array per quantity, one loop per formula, the steps in the
 * order the paper gives them. OpenMP is used over k-planes only, for independent per-node
 * work; every sum is taken in a fixed sequential order.
 *
 * Section names below are those of the paper. Where the paper is silent, garbled or
 * ambiguous, the comment states the reading taken.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_EGRID (-3)
#define OR_ENONFINITE (-5)

typedef struct {
  const or_params* P;
  int n[3];      /* nodes per direction */
  int per[3];    /* 1 if the direction is periodic */
  long N;
} Grid;

static long ID(const Grid* G, const int* ix) {
  return ix[0] + (long)G->n[0] * (ix[1] + (long)G->n[1] * ix[2]);
}

static int setup(Grid* G, const or_params* P) {
  G->P = P;
  G->n[0] = P->ni; G->n[1] = P->nj; G->n[2] = P->nk;
  for (int d = 0; d < 3; ++d) {
    if (G->n[d] < 4) return OR_EINVAL;
    int lo = P->bc[2 * d], hi = P->bc[2 * d + 1];
    if ((lo == OR_BC_PERIODIC) != (hi == OR_BC_PERIODIC)) return OR_EINVAL;
    G->per[d] = (lo == OR_BC_PERIODIC);
  }
  /* Supported boundary sets: a triply periodic box, or the jet of the paper's boundary
   * conditions section (entrance i-, exit i+, centreline j-, far field j+, periodic k). */
  int all_periodic = G->per[0] && G->per[1] && G->per[2];
  int jet = P->bc[0] == OR_BC_JET_INFLOW && P->bc[1] == OR_BC_EXIT &&
            P->bc[2] == OR_BC_AXIS && P->bc[3] == OR_BC_FARFIELD && G->per[2];
  if (!all_periodic && !jet) return OR_EINVAL;
  if (!(P->gamma > 1.0)) return OR_EINVAL;
  G->N = (long)G->n[0] * G->n[1] * G->n[2];
  return OR_OK;
}

/* A node is updated by the time integration unless it lies on a non-periodic face; nodes
 * on such faces are set by the boundary conditions. */
static int updated(const Grid* G, const int* ix) {
  for (int d = 0; d < 3; ++d)
    if (!G->per[d] && (ix[d] == 0 || ix[d] == G->n[d] - 1)) return 0;
  return 1;
}

static void unflat(const Grid* G, long id, int* ix) {
  ix[0] = (int)(id % G->n[0]);
  ix[1] = (int)((id / G->n[0]) % G->n[1]);
  ix[2] = (int)(id / ((long)G->n[0] * G->n[1]));
}

/* ---------------------------------------------------------------------------------------
 * Differences. delta_d f at a node is the centred difference (f[m+1] - f[m-1])/2; at the
 * first and last node of a non-periodic direction it is the second-order one-sided
 * difference. Index spacing is 1 (the paper's Delta xi = Delta eta = Delta zeta = 1).
 * ------------------------------------------------------------------------------------- */
static double dfield(const Grid* G, const double* f, int d, const int* ix) {
  int n = G->n[d], m = ix[d];
  int a[3] = {ix[0], ix[1], ix[2]}, b[3] = {ix[0], ix[1], ix[2]}, c[3] = {ix[0], ix[1], ix[2]};
  if (G->per[d]) {
    a[d] = (m + 1) % n;
    b[d] = (m - 1 + n) % n;
    return 0.5 * (f[ID(G, a)] - f[ID(G, b)]);
  }
  if (m == 0) {
    a[d] = 0; b[d] = 1; c[d] = 2;
    return 0.5 * (-3.0 * f[ID(G, a)] + 4.0 * f[ID(G, b)] - f[ID(G, c)]);
  }
  if (m == n - 1) {
    a[d] = n - 1; b[d] = n - 2; c[d] = n - 3;
    return 0.5 * (3.0 * f[ID(G, a)] - 4.0 * f[ID(G, b)] + f[ID(G, c)]);
  }
  a[d] = m + 1;
  b[d] = m - 1;
  return 0.5 * (f[ID(G, a)] - f[ID(G, b)]);
}

/* ---------------------------------------------------------------------------------------
 * Grid metrics (paper, Transformation of Coordinates).
 * Coordinates are read through X(), which accepts indices one or two nodes past either end
 * of a periodic direction and adds the period translation for each wrap.
 * ------------------------------------------------------------------------------------- */
static double X(const Grid* G, const double* xyz, int c, const int* ix) {
  int w[3];
  double s = 0.0;
  for (int d = 0; d < 3; ++d) {
    int m = ix[d], n = G->n[d], q = 0;
    while (m < 0) { m += n; q -= 1; }
    while (m >= n) { m -= n; q += 1; }
    w[d] = m;
    s += q * G->P->period_shift[d][c];
  }
  return xyz[(long)c * G->N + ID(G, w)] + s;
}

/* delta_e of coordinate c at a (possibly unwrapped) index. */
static double dX(const Grid* G, const double* xyz, int c, int e, const int* ix) {
  int n = G->n[e], m = ix[e];
  int a[3] = {ix[0], ix[1], ix[2]}, b[3] = {ix[0], ix[1], ix[2]}, cc[3] = {ix[0], ix[1], ix[2]};
  if (G->per[e] || (m > 0 && m < n - 1)) {
    a[e] = m + 1;
    b[e] = m - 1;
    return 0.5 * (X(G, xyz, c, a) - X(G, xyz, c, b));
  }
  if (m == 0) {
    a[e] = 0; b[e] = 1; cc[e] = 2;
    return 0.5 * (-3.0 * X(G, xyz, c, a) + 4.0 * X(G, xyz, c, b) - X(G, xyz, c, cc));
  }
  a[e] = n - 1; b[e] = n - 2; cc[e] = n - 3;
  return 0.5 * (3.0 * X(G, xyz, c, a) - 4.0 * X(G, xyz, c, b) + X(G, xyz, c, cc));
}

/* g = x_{c2} * delta_e x_{c1} at a (possibly unwrapped) index. */
static double Gprod(const Grid* G, const double* xyz, int c2, int c1, int e, const int* ix) {
  return X(G, xyz, c2, ix) * dX(G, xyz, c1, e, ix);
}

/* delta_d of g = x_{c2} delta_e x_{c1}. */
static double dGprod(const Grid* G, const double* xyz, int c2, int c1, int e, int d,
                     const int* ix) {
  int n = G->n[d], m = ix[d];
  int a[3] = {ix[0], ix[1], ix[2]}, b[3] = {ix[0], ix[1], ix[2]}, cc[3] = {ix[0], ix[1], ix[2]};
  if (G->per[d] || (m > 0 && m < n - 1)) {
    a[d] = m + 1;
    b[d] = m - 1;
    return 0.5 * (Gprod(G, xyz, c2, c1, e, a) - Gprod(G, xyz, c2, c1, e, b));
  }
  if (m == 0) {
    a[d] = 0; b[d] = 1; cc[d] = 2;
    return 0.5 * (-3.0 * Gprod(G, xyz, c2, c1, e, a) + 4.0 * Gprod(G, xyz, c2, c1, e, b) -
                  Gprod(G, xyz, c2, c1, e, cc));
  }
  a[d] = n - 1; b[d] = n - 2; cc[d] = n - 3;
  return 0.5 * (3.0 * Gprod(G, xyz, c2, c1, e, a) - 4.0 * Gprod(G, xyz, c2, c1, e, b) +
                Gprod(G, xyz, c2, c1, e, cc));
}

int or_metrics(const or_params* P, const double* xyz, double* S, double* jinv) {
  Grid G;
  int rc = setup(&G, P);
  if (rc) return rc;
  int bad = 0;
#pragma omp parallel for reduction(| : bad)
  for (int k = 0; k < G.n[2]; ++k)
    for (int j = 0; j < G.n[1]; ++j)
      for (int i = 0; i < G.n[0]; ++i) {
        int ix[3] = {i, j, k};
        long id = ID(&G, ix);
        double r[3][3]; /* r[d][c] = d x_c / d(direction d) */
        for (int d = 0; d < 3; ++d)
          for (int c = 0; c < 3; ++c) r[d][c] = dX(&G, xyz, c, d, ix);
        /* J^-1: the determinant in the paper's six-term form (x_xi y_eta z_zeta + ...). */
        double xx = r[0][0], xe = r[1][0], xz = r[2][0];
        double yx = r[0][1], ye = r[1][1], yz = r[2][1];
        double zx = r[0][2], ze = r[1][2], zz = r[2][2];
        double det = xx * ye * zz + xe * yz * zx + xz * yx * ze - xx * yz * ze - xe * yx * zz -
                     xz * ye * zx;
        jinv[id] = det;
        for (int d = 0; d < 3; ++d) {
          int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
          for (int c = 0; c < 3; ++c) {
            int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            double s;
            if (P->metric_form == 0) {
              /* Conservative (Thomas-Lombard) form of S_d = r_{d+1} x r_{d+2}:
               * S_d^c = delta_{d+2}(x_{c+2} delta_{d+1} x_{c+1})
               *       - delta_{d+1}(x_{c+2} delta_{d+2} x_{c+1}).
               * Equal to the paper's cross products analytically; discretely it satisfies
               * sum_d delta_d S_d = 0, so a uniform flow gives a zero residual. */
              s = dGprod(&G, xyz, c2, c1, d1, d2, ix) - dGprod(&G, xyz, c2, c1, d2, d1, ix);
            } else {
              /* The paper's products of centred coordinate differences, e.g.
               * J^-1 xi_x = y_eta z_zeta - y_zeta z_eta (eta row read with zeta, see notes). */
              s = r[d1][c1] * r[d2][c2] - r[d1][c2] * r[d2][c1];
            }
            S[(long)(3 * d + c) * G.N + id] = s;
          }
        }
        if (updated(&G, ix) && !(det > 0.0)) bad |= 1;
      }
  return bad ? OR_EGRID : OR_OK;
}

/* Sutherland's law in reference units: mu* = T*^(3/2) (1 + S1*)/(T* + S1*), so mu*(1) = 1
 * (paper, LES formulation; the reference temperature takes the place of T_0 and T_inf). */
static double sutherland(const or_params* P, double T) {
  return pow(T, 1.5) * (1.0 + P->suth_s1) / (T + P->suth_s1);
}

int or_sutherland(const or_params* P, int n, const double* T, double* mu) {
  for (int i = 0; i < n; ++i) mu[i] = sutherland(P, T[i]);
  return OR_OK;
}

/* ---------------------------------------------------------------------------------------
 * Per-node quantities.
 * ------------------------------------------------------------------------------------- */
typedef struct {
  double *rho, *u, *v, *w, *p, *T, *mu, *mut;
  double* dq[3][4]; /* delta_d of (u, v, w, T) */
  double* lam[3];   /* J^-1 lambda_d = |S_d . u| + a |S_d| */
  double* lbar[3];  /* J^-1 times the anisotropic scaled radius */
  double* nu[3];    /* pressure sensor along d */
  double* H[3][5];  /* total numerical flux on the face between a node and its + neighbour */
  double* block;
} Work;

static int work_alloc(Work* W, long N) {
  int count = 8 + 12 + 3 + 3 + 3 + 15;
  W->block = (double*)calloc((size_t)count * N, sizeof(double));
  if (!W->block) return OR_ENOMEM;
  double* b = W->block;
  W->rho = b; b += N; W->u = b; b += N; W->v = b; b += N; W->w = b; b += N;
  W->p = b; b += N; W->T = b; b += N; W->mu = b; b += N; W->mut = b; b += N;
  for (int d = 0; d < 3; ++d)
    for (int f = 0; f < 4; ++f) { W->dq[d][f] = b; b += N; }
  for (int d = 0; d < 3; ++d) { W->lam[d] = b; b += N; }
  for (int d = 0; d < 3; ++d) { W->lbar[d] = b; b += N; }
  for (int d = 0; d < 3; ++d) { W->nu[d] = b; b += N; }
  for (int d = 0; d < 3; ++d)
    for (int c = 0; c < 5; ++c) { W->H[d][c] = b; b += N; }
  return OR_OK;
}

static void work_free(Work* W) { free(W->block); }

/* Primitive variables from the conserved ones (paper, LES formulation: equation of state
 * and System-I total energy; dimensionless formulation). In reference units
 * p = (gamma-1)(e - rho|u|^2/2), T = gamma p / rho, a = sqrt(T). */
static void primitives(const Grid* G, const double* q, Work* W) {
  const or_params* P = G->P;
  long N = G->N;
#pragma omp parallel for
  for (int k = 0; k < G->n[2]; ++k)
    for (long id = (long)k * G->n[0] * G->n[1]; id < (long)(k + 1) * G->n[0] * G->n[1]; ++id) {
      double rho = q[id];
      double u = q[N + id] / rho, v = q[2 * N + id] / rho, w = q[3 * N + id] / rho;
      double p = (P->gamma - 1.0) * (q[4 * N + id] - 0.5 * rho * (u * u + v * v + w * w));
      double T = P->gamma * p / rho;
      W->rho[id] = rho; W->u[id] = u; W->v[id] = v; W->w[id] = w;
      W->p[id] = p; W->T[id] = T;
      W->mu[id] = sutherland(P, T);
    }
}

static void node_differences(const Grid* G, Work* W) {
  const double* f[4] = {W->u, W->v, W->w, W->T};
#pragma omp parallel for
  for (int k = 0; k < G->n[2]; ++k)
    for (int j = 0; j < G->n[1]; ++j)
      for (int i = 0; i < G->n[0]; ++i) {
        int ix[3] = {i, j, k};
        long id = ID(G, ix);
        for (int d = 0; d < 3; ++d)
          for (int v = 0; v < 4; ++v) W->dq[d][v][id] = dfield(G, f[v], d, ix);
      }
}

/* Classical Smagorinsky eddy viscosity (paper, Subgrid Scale Viscosity):
 * mu_sgs = rho (C_s Delta)^2 (2 S_ij S_ij)^(1/2), with S_ij from the node velocity gradient
 * du_m/dx_n = J sum_e S_e^n delta_e u_m. Reading: the filter width Delta is the cube root of
 * the local cell volume J^-1; mu_sgs = 0 where J^-1 = 0 (the jet axis). */
static void smagorinsky(const Grid* G, const double* S, const double* jinv, Work* W) {
  const or_params* P = G->P;
  long N = G->N;
#pragma omp parallel for
  for (int k = 0; k < G->n[2]; ++k)
    for (long id = (long)k * G->n[0] * G->n[1]; id < (long)(k + 1) * G->n[0] * G->n[1]; ++id) {
      if (!(jinv[id] > 0.0)) {
        W->mut[id] = 0.0;
        continue;
      }
      double J = 1.0 / jinv[id];
      double g[3][3]; /* g[m][n] = d u_m / d x_n */
      for (int m = 0; m < 3; ++m)
        for (int n = 0; n < 3; ++n) {
          double s = 0.0;
          for (int e = 0; e < 3; ++e) s += S[(long)(3 * e + n) * N + id] * W->dq[e][m][id];
          g[m][n] = J * s;
        }
      double ss = 0.0;
      for (int m = 0; m < 3; ++m)
        for (int n = 0; n < 3; ++n) {
          double smn = 0.5 * (g[m][n] + g[n][m]);
          ss += smn * smn;
        }
      double smag = sqrt(2.0 * ss);
      double delta = cbrt(jinv[id]);
      W->mut[id] = W->rho[id] * (P->cs * delta) * (P->cs * delta) * smag;
    }
}

/* Spectral radii and their anisotropic scaling (paper, Spatial Discretization).
 * Reading: lambda_xi = |U| + a |grad xi|, and likewise for eta and zeta with their own
 * metric norms; everything is carried multiplied by J^-1, so
 * Lam_d = |S_d . u| + a |S_d| and Lambar_xi = Lam_xi + sqrt(Lam_xi Lam_eta)
 * + sqrt(Lam_xi Lam_zeta) (identical to lambda_xi[1 + (lambda_eta/lambda_xi)^0.5 + ...]
 * times J^-1, and finite where J^-1 = 0). */
static void spectral_radii(const Grid* G, const double* S, Work* W) {
  long N = G->N;
#pragma omp parallel for
  for (int k = 0; k < G->n[2]; ++k)
    for (long id = (long)k * G->n[0] * G->n[1]; id < (long)(k + 1) * G->n[0] * G->n[1]; ++id) {
      double a = sqrt(W->T[id]);
      for (int d = 0; d < 3; ++d) {
        double sx = S[(long)(3 * d) * N + id], sy = S[(long)(3 * d + 1) * N + id],
               sz = S[(long)(3 * d + 2) * N + id];
        double un = sx * W->u[id] + sy * W->v[id] + sz * W->w[id];
        W->lam[d][id] = fabs(un) + a * sqrt(sx * sx + sy * sy + sz * sz);
      }
      for (int d = 0; d < 3; ++d) {
        int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
        W->lbar[d][id] = W->lam[d][id] + sqrt(W->lam[d][id] * W->lam[d1][id]) +
                         sqrt(W->lam[d][id] * W->lam[d2][id]);
      }
    }
}

/* Pressure sensor (paper, Spatial Discretization). Reading: the standard Jameson form
 * |p+ - 2p + p-| / (p+ + 2p + p-) along the face direction; on the first and last node of a
 * non-periodic direction the value of the adjacent interior node is used. */
static void sensor(const Grid* G, Work* W) {
#pragma omp parallel for
  for (int k = 0; k < G->n[2]; ++k)
    for (int j = 0; j < G->n[1]; ++j)
      for (int i = 0; i < G->n[0]; ++i) {
        int ix[3] = {i, j, k};
        long id = ID(G, ix);
        for (int d = 0; d < 3; ++d) {
          int n = G->n[d], m = ix[d];
          int c[3] = {i, j, k};
          if (!G->per[d]) {
            if (m == 0) c[d] = 1;
            if (m == n - 1) c[d] = n - 2;
          }
          int a[3] = {c[0], c[1], c[2]}, b[3] = {c[0], c[1], c[2]};
          a[d] = (c[d] + 1) % n;
          b[d] = (c[d] - 1 + n) % n;
          double pp = W->p[ID(G, a)], p0 = W->p[ID(G, c)], pm = W->p[ID(G, b)];
          W->nu[d][id] = fabs(pp - 2.0 * p0 + pm) / (pp + 2.0 * p0 + pm);
        }
      }
}

/* The dissipated vector W = (rho, rho u, rho v, rho w, e + p) (paper, Spatial
 * Discretization). Reading: W is built from the physical conserved vector, not from
 * J^-1 Q; J^-1 enters the dissipation once, through Lambar. */
static double Wvec(const Grid* G, const double* q, const Work* W, int c, long id) {
  double val = q[(long)c * G->N + id];
  if (c == 4) val += W->p[id];
  return val;
}

/* Inviscid flux along d at a node (paper, Transformation of Coordinates: inviscid flux
 * vectors, stationary grid so xi_t = 0): J^-1 E_e = {rho U', rho u U' + p S_x, ...,
 * (e + p) U'} with U' = S_d . u. */
static void inviscid_node_flux(const Grid* G, const double* S, const double* q,
                               const Work* W, int d, long id, double* F) {
  long N = G->N;
  double sx = S[(long)(3 * d) * N + id], sy = S[(long)(3 * d + 1) * N + id],
         sz = S[(long)(3 * d + 2) * N + id];
  double un = sx * W->u[id] + sy * W->v[id] + sz * W->w[id];
  double p = W->p[id];
  F[0] = q[id] * un;
  F[1] = q[N + id] * un + p * sx;
  F[2] = q[2 * N + id] * un + p * sy;
  F[3] = q[3 * N + id] * un + p * sz;
  F[4] = (q[4 * N + id] + p) * un;
}

/* Artificial dissipation on the face m+1/2 along d (paper, Spatial Discretization, the
 * Turkel-Vatsa terms; near-boundary treatment from the Centerline Boundary Condition).
 * Reading of the garbled operator: D = Lam_f [eps2 (W_{m+1} - W_m) - eps4 Delta^3 W] with
 * Delta^3 W = W_{m+2} - 3 W_{m+1} + 3 W_m - W_{m-1}. On the first and last face of a
 * non-periodic direction the missing difference is extrapolated as
 * (Delta W)_outside = -(Delta W)_inside, which the paper gives for the centreline and this
 * oracle applies at every non-periodic face. */
static void dissipation(const Grid* G, const double* q, const Work* W, int d, const int* ixA,
                        double* D) {
  int n = G->n[d], m = ixA[d];
  int iA[3] = {ixA[0], ixA[1], ixA[2]}, iB[3], iM[3], iP[3];
  memcpy(iB, iA, sizeof iB); memcpy(iM, iA, sizeof iM); memcpy(iP, iA, sizeof iP);
  iB[d] = (m + 1) % n;
  long a = ID(G, iA), b = ID(G, iB);
  double lamf = 0.5 * (W->lbar[d][a] + W->lbar[d][b]);
  double nA = W->nu[d][a], nB = W->nu[d][b];
  double eps2 = G->P->k2 * (nA > nB ? nA : nB);
  double eps4 = G->P->k4 - eps2;
  if (eps4 < 0.0) eps4 = 0.0;
  for (int c = 0; c < 5; ++c) {
    double wA = Wvec(G, q, W, c, a), wB = Wvec(G, q, W, c, b);
    double d1 = wB - wA;
    double d3;
    if (G->per[d]) {
      iM[d] = (m - 1 + n) % n;
      iP[d] = (m + 2) % n;
      d3 = Wvec(G, q, W, c, ID(G, iP)) - 3.0 * wB + 3.0 * wA - Wvec(G, q, W, c, ID(G, iM));
    } else if (m == 0) {
      /* (Delta W)_{-1/2} = -(Delta W)_{1/2}: Delta^3 = (Delta W)_{3/2} - 3 (Delta W)_{1/2} */
      iP[d] = 2;
      double d32 = Wvec(G, q, W, c, ID(G, iP)) - wB;
      d3 = d32 - 3.0 * d1;
    } else if (m == n - 2) {
      /* (Delta W)_{n-1/2} = -(Delta W)_{n-3/2}: Delta^3 = -3 (Delta W)_{n-3/2} + (Delta W)_{n-5/2} */
      iM[d] = n - 3;
      double dlo = wA - Wvec(G, q, W, c, ID(G, iM));
      d3 = -3.0 * d1 + dlo;
    } else {
      iM[d] = m - 1;
      iP[d] = m + 2;
      d3 = Wvec(G, q, W, c, ID(G, iP)) - 3.0 * wB + 3.0 * wA - Wvec(G, q, W, c, ID(G, iM));
    }
    D[c] = lamf * (eps2 * d1 - eps4 * d3);
  }
}

/* Viscous and subgrid flux on the face m+1/2 along d (paper, Transformation of
 * Coordinates: viscous flux vectors; Subgrid Scale Modeling; LES formulation).
 * Readings: the face uses two neighbouring nodes, so the derivative along d is the compact
 * difference phi_{m+1} - phi_m and the two other derivatives are the averages of the nodal
 * centred differences; metrics, J^-1, mu, mu_sgs and velocity are face averages and
 * J_f = 1 / J^-1_f. The stress is
 * tau = 2 (mu/Re + mu_sgs)(S_ij - delta_ij S_kk / 3), and the heat flux obeys Fourier's law
 * q = -kappa grad T with kappa = [mu/(Re Pr) + mu_sgs/Pr_sgs]/(gamma - 1) in reference units
 * (Eidson's SGS conductivity models B1 + B2; B4..B7 are neglected). */
static void viscous(const Grid* G, const double* S, const double* jinv, const Work* W, int d,
                    const int* ixA, double* Fv) {
  const or_params* P = G->P;
  long N = G->N;
  int n = G->n[d];
  int iB[3] = {ixA[0], ixA[1], ixA[2]};
  iB[d] = (ixA[d] + 1) % n;
  long a = ID(G, ixA), b = ID(G, iB);
  double Sf[3][3];
  for (int e = 0; e < 3; ++e)
    for (int c = 0; c < 3; ++c)
      Sf[e][c] = 0.5 * (S[(long)(3 * e + c) * N + a] + S[(long)(3 * e + c) * N + b]);
  double Jf = 1.0 / (0.5 * (jinv[a] + jinv[b]));
  const double* f[4] = {W->u, W->v, W->w, W->T};
  double grad[4][3]; /* grad[var][x_n] */
  for (int v = 0; v < 4; ++v) {
    double dphi[3];
    for (int e = 0; e < 3; ++e)
      dphi[e] = (e == d) ? (f[v][b] - f[v][a]) : 0.5 * (W->dq[e][v][a] + W->dq[e][v][b]);
    for (int c = 0; c < 3; ++c)
      grad[v][c] = Jf * (Sf[0][c] * dphi[0] + Sf[1][c] * dphi[1] + Sf[2][c] * dphi[2]);
  }
  double inv_re = P->re_acoustic > 0.0 ? 1.0 / P->re_acoustic : 0.0;
  double muf = 0.5 * (W->mu[a] + W->mu[b]);
  double mutf = 0.5 * (W->mut[a] + W->mut[b]);
  double visc = muf * inv_re + mutf;
  double kappa = (muf * inv_re / P->prandtl + mutf / P->prandtl_sgs) / (P->gamma - 1.0);
  double div = grad[0][0] + grad[1][1] + grad[2][2];
  double tau[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      tau[r][c] = visc * (grad[r][c] + grad[c][r] - (r == c ? 2.0 / 3.0 * div : 0.0));
  double ub[3] = {0.5 * (W->u[a] + W->u[b]), 0.5 * (W->v[a] + W->v[b]),
                  0.5 * (W->w[a] + W->w[b])};
  double beta[3];
  for (int r = 0; r < 3; ++r) {
    double heat = -kappa * grad[3][r];
    beta[r] = tau[r][0] * ub[0] + tau[r][1] * ub[1] + tau[r][2] * ub[2] - heat;
  }
  Fv[0] = 0.0;
  for (int c = 0; c < 3; ++c)
    Fv[1 + c] = Sf[d][0] * tau[0][c] + Sf[d][1] * tau[1][c] + Sf[d][2] * tau[2][c];
  Fv[4] = Sf[d][0] * beta[0] + Sf[d][1] * beta[1] + Sf[d][2] * beta[2];
}

/* Numerical flux on every face (paper, Spatial Discretization: central interface flux
 * with artificial dissipation, minus the viscous flux). */
static void face_fluxes(const Grid* G, const double* S, const double* jinv, const double* q,
                        Work* W) {
#pragma omp parallel for
  for (int k = 0; k < G->n[2]; ++k)
    for (int j = 0; j < G->n[1]; ++j)
      for (int i = 0; i < G->n[0]; ++i) {
        int ix[3] = {i, j, k};
        long id = ID(G, ix);
        for (int d = 0; d < 3; ++d) {
          if (!G->per[d] && ix[d] == G->n[d] - 1) {
            for (int c = 0; c < 5; ++c) W->H[d][c][id] = 0.0;
            continue;
          }
          int iB[3] = {i, j, k};
          iB[d] = (ix[d] + 1) % G->n[d];
          double FA[5], FB[5], D[5], Fv[5];
          inviscid_node_flux(G, S, q, W, d, id, FA);
          inviscid_node_flux(G, S, q, W, d, ID(G, iB), FB);
          dissipation(G, q, W, d, ix, D);
          viscous(G, S, jinv, W, d, ix, Fv);
          for (int c = 0; c < 5; ++c) W->H[d][c][id] = 0.5 * (FA[c] + FB[c]) - D[c] - Fv[c];
        }
      }
}

static void node_state(const Grid* G, const double* S, const double* jinv, const double* q,
                       Work* W) {
  primitives(G, q, W);
  node_differences(G, W);
  smagorinsky(G, S, jinv, W);
  spectral_radii(G, S, W);
  sensor(G, W);
}

/* RHS_ijk = sum over directions of the face-flux differences (paper, Spatial
 * Discretization; the directions are summed). Written at updated nodes, 0 elsewhere. */
static void residual_from_work(const Grid* G, const Work* W, double* rhs) {
  long N = G->N;
#pragma omp parallel for
  for (int k = 0; k < G->n[2]; ++k)
    for (int j = 0; j < G->n[1]; ++j)
      for (int i = 0; i < G->n[0]; ++i) {
        int ix[3] = {i, j, k};
        long id = ID(G, ix);
        if (!updated(G, ix)) {
          for (int c = 0; c < 5; ++c) rhs[(long)c * N + id] = 0.0;
          continue;
        }
        for (int c = 0; c < 5; ++c) {
          double r = 0.0;
          for (int d = 0; d < 3; ++d) {
            int im[3] = {i, j, k};
            im[d] = (ix[d] - 1 + G->n[d]) % G->n[d];
            r += W->H[d][c][id] - W->H[d][c][ID(G, im)];
          }
          rhs[(long)c * N + id] = r;
        }
      }
}

int or_residual(const or_params* P, const double* S, const double* jinv, const double* q,
                double* rhs) {
  Grid G;
  int rc = setup(&G, P);
  if (rc) return rc;
  Work W;
  if (work_alloc(&W, G.N)) return OR_ENOMEM;
  node_state(&G, S, jinv, q, &W);
  face_fluxes(&G, S, jinv, q, &W);
  residual_from_work(&G, &W, rhs);
  work_free(&W);
  return OR_OK;
}

/* The same residual with a given eddy viscosity mu_t [N] in place of the Smagorinsky value
 * (for closures that predict the model coefficient). */
int or_residual_mut(const or_params* P, const double* S, const double* jinv, const double* q,
                    const double* mu_t, double* rhs) {
  Grid G;
  int rc = setup(&G, P);
  if (rc) return rc;
  Work W;
  if (work_alloc(&W, G.N)) return OR_ENOMEM;
  node_state(&G, S, jinv, q, &W);
  memcpy(W.mut, mu_t, sizeof(double) * G.N);
  face_fluxes(&G, S, jinv, q, &W);
  residual_from_work(&G, &W, rhs);
  work_free(&W);
  return OR_OK;
}

int or_sgs_viscosity(const or_params* P, const double* S, const double* jinv, const double* q,
                     double* mu_t) {
  Grid G;
  int rc = setup(&G, P);
  if (rc) return rc;
  Work W;
  if (work_alloc(&W, G.N)) return OR_ENOMEM;
  primitives(&G, q, &W);
  node_differences(&G, &W);
  smagorinsky(&G, S, jinv, &W);
  memcpy(mu_t, W.mut, sizeof(double) * G.N);
  work_free(&W);
  return OR_OK;
}

/* Velocity gradient g[3m + n] = d u_m / d x_n = J sum_e S_e^n delta_e u_m at every node,
 * from the same nodal differences as the Smagorinsky viscosity (paper, Subgrid Scale
 * Viscosity: the strain rate of the resolved field); 0 where J^-1 <= 0. */
int or_velocity_gradient(const or_params* P, const double* S, const double* jinv,
                         const double* q, double* grad) {
  Grid G;
  int rc = setup(&G, P);
  if (rc) return rc;
  Work W;
  if (work_alloc(&W, G.N)) return OR_ENOMEM;
  primitives(&G, q, &W);
  node_differences(&G, &W);
  long N = G.N;
#pragma omp parallel for
  for (int k = 0; k < G.n[2]; ++k)
    for (long id = (long)k * G.n[0] * G.n[1]; id < (long)(k + 1) * G.n[0] * G.n[1]; ++id) {
      double J = jinv[id] > 0.0 ? 1.0 / jinv[id] : 0.0;
      for (int m = 0; m < 3; ++m)
        for (int n = 0; n < 3; ++n) {
          double s = 0.0;
          for (int e = 0; e < 3; ++e) s += S[(long)(3 * e + n) * N + id] * W.dq[e][m][id];
          grad[(long)(3 * m + n) * N + id] = J * s;
        }
    }
  work_free(&W);
  return OR_OK;
}

/* ---------------------------------------------------------------------------------------
 * Boundary conditions (paper, Boundary Conditions).
 * ------------------------------------------------------------------------------------- */
static void conserved(double gamma, double rho, const double* u, double p, double* qo) {
  qo[0] = rho;
  qo[1] = rho * u[0];
  qo[2] = rho * u[1];
  qo[3] = rho * u[2];
  qo[4] = p / (gamma - 1.0) + 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
}

static void get_q(const Grid* G, const double* q, long id, double* qo) {
  for (int c = 0; c < 5; ++c) qo[c] = q[(long)c * G->N + id];
}

static void set_q(const Grid* G, double* q, long id, const double* qi) {
  for (int c = 0; c < 5; ++c) q[(long)c * G->N + id] = qi[c];
}

/* Far-field Riemann-invariant state (paper, Far Field Boundary). qe is the adjacent
 * interior node, n the unit outward normal at the boundary node. Readings: the interior
 * invariant is R+ = q_ne + 2 a_e/(gamma-1) (the only sign consistent with the printed a_f);
 * the velocity correction is along the unit normal; q_ne/a_e = 0 counts as outflow, = 1 as
 * supersonic outflow, = -1 as supersonic inflow. */
static void farfield_state(const or_params* P, const double* qe, const double* n, double* qb) {
  double g = P->gamma;
  double rho_e = qe[0];
  double ue[3] = {qe[1] / rho_e, qe[2] / rho_e, qe[3] / rho_e};
  double pe = (g - 1.0) * (qe[4] - 0.5 * rho_e * (ue[0] * ue[0] + ue[1] * ue[1] + ue[2] * ue[2]));
  double ae = sqrt(g * pe / rho_e);
  double ainf = sqrt(g * P->p_inf / P->rho_inf);
  double qne = ue[0] * n[0] + ue[1] * n[1] + ue[2] * n[2];
  double qninf = P->u_inf[0] * n[0] + P->u_inf[1] * n[1] + P->u_inf[2] * n[2];
  double rplus = qne + 2.0 * ae / (g - 1.0);
  double rminus = qninf - 2.0 * ainf / (g - 1.0);
  double qnf = 0.5 * (rplus + rminus);
  double af = 0.25 * (g - 1.0) * (rplus - rminus);
  double mn = qne / ae;
  double uf[3], rhof, pf;
  if (mn >= 1.0) { /* supersonic exit: everything from the interior */
    for (int c = 0; c < 5; ++c) qb[c] = qe[c];
    return;
  } else if (mn >= 0.0) { /* subsonic exit: entropy from the interior */
    for (int c = 0; c < 3; ++c) uf[c] = ue[c] + (qnf - qne) * n[c];
    rhof = pow(pow(rho_e, g) * af * af / (g * pe), 1.0 / (g - 1.0));
    pf = rhof * af * af / g;
  } else if (mn > -1.0) { /* subsonic entrance: entropy from the free stream */
    for (int c = 0; c < 3; ++c) uf[c] = P->u_inf[c] + (qnf - qninf) * n[c];
    rhof = pow(pow(P->rho_inf, g) * af * af / (g * P->p_inf), 1.0 / (g - 1.0));
    pf = rhof * af * af / g;
  } else { /* supersonic entrance: free stream */
    for (int c = 0; c < 3; ++c) uf[c] = P->u_inf[c];
    rhof = P->rho_inf;
    pf = P->p_inf;
  }
  conserved(g, rhof, uf, pf, qb);
}

static void unit_metric(const Grid* G, const double* S, int d, long id, double sign, double* n) {
  double sx = S[(long)(3 * d) * G->N + id], sy = S[(long)(3 * d + 1) * G->N + id],
         sz = S[(long)(3 * d + 2) * G->N + id];
  double m = sqrt(sx * sx + sy * sy + sz * sz);
  n[0] = sign * sx / m;
  n[1] = sign * sy / m;
  n[2] = sign * sz / m;
}

/* Boundary nodes are set from the stage's updated nodes. Reading (the paper gives no
 * order): far field, then centreline, then entrance, then exit; the i faces own the corner
 * nodes and read the values the j faces have just set. */
int or_apply_bc(const or_params* P, const double* xyz, const double* S, const double* jinv,
                double* q) {
  Grid G;
  int rc = setup(&G, P);
  (void)jinv;
  if (rc) return rc;
  if (G.per[0]) return OR_OK; /* periodic box: no boundary nodes */
  int ni = G.n[0], nj = G.n[1], nk = G.n[2];
  double g = P->gamma;
  /* Far field, j = nj-1, 1 <= i <= ni-2, normal S_eta/|S_eta|. */
  for (int k = 0; k < nk; ++k)
    for (int i = 1; i <= ni - 2; ++i) {
      int ib[3] = {i, nj - 1, k}, ie[3] = {i, nj - 2, k};
      double qe[5], qb[5], n[3];
      get_q(&G, q, ID(&G, ie), qe);
      unit_metric(&G, S, 1, ID(&G, ib), 1.0, n);
      farfield_state(P, qe, n, qb);
      set_q(&G, q, ID(&G, ib), qb);
    }
  /* Centreline, j = 0, 1 <= i <= ni-2 (paper, Centerline Boundary Condition): the
   * azimuthal average of the first ring, summed in k order. */
  for (int i = 1; i <= ni - 2; ++i) {
    double sum[5] = {0, 0, 0, 0, 0};
    for (int k = 0; k < nk; ++k) {
      int ie[3] = {i, 1, k};
      for (int c = 0; c < 5; ++c) sum[c] += q[(long)c * G.N + ID(&G, ie)];
    }
    for (int c = 0; c < 5; ++c) sum[c] /= (double)nk;
    for (int k = 0; k < nk; ++k) {
      int ib[3] = {i, 0, k};
      set_q(&G, q, ID(&G, ib), sum);
    }
  }
  /* Entrance, i = 0 (paper, Entrance Boundary): inside the jet, r <= D/2, the supersonic
   * jet state rho = 1, u = (M_j, 0, 0), p = 1/gamma; outside, the far-field procedure with
   * the xi direction as normal (outward normal -S_xi/|S_xi|). */
  for (int k = 0; k < nk; ++k)
    for (int j = 0; j < nj; ++j) {
      int ib[3] = {0, j, k}, ie[3] = {1, j, k};
      long b = ID(&G, ib);
      double y = xyz[G.N + b], z = xyz[2 * G.N + b];
      double r = sqrt(y * y + z * z);
      double qb[5];
      if (r <= P->jet_radius) {
        double uj[3] = {P->mach_jet, 0.0, 0.0};
        conserved(g, 1.0, uj, 1.0 / g, qb);
      } else {
        double qe[5], n[3];
        get_q(&G, q, ID(&G, ie), qe);
        unit_metric(&G, S, 0, b, -1.0, n);
        farfield_state(P, qe, n, qb);
      }
      set_q(&G, q, b, qb);
    }
  /* Exit, i = ni-1 (paper, Exit Boundary Condition). Supersonic (u.n/a >= 1): all from
   * i = ni-2. Subsonic: p = p_inf, velocity and internal energy per unit mass
   * e_i = p/((gamma-1) rho) from i = ni-2, rho = p_inf/((gamma-1) e_i). */
  for (int k = 0; k < nk; ++k)
    for (int j = 0; j < nj; ++j) {
      int ib[3] = {ni - 1, j, k}, ie[3] = {ni - 2, j, k}, in[3] = {ni - 1, j == 0 ? 1 : j, k};
      long b = ID(&G, ib);
      double qe[5], qb[5], n[3];
      get_q(&G, q, ID(&G, ie), qe);
      /* The xi metric vanishes on the axis; the axis node takes the normal of j = 1. */
      unit_metric(&G, S, 0, ID(&G, in), 1.0, n);
      double rho_e = qe[0];
      double ue[3] = {qe[1] / rho_e, qe[2] / rho_e, qe[3] / rho_e};
      double pe = (g - 1.0) * (qe[4] - 0.5 * rho_e * (ue[0] * ue[0] + ue[1] * ue[1] + ue[2] * ue[2]));
      double ae = sqrt(g * pe / rho_e);
      double mn = (ue[0] * n[0] + ue[1] * n[1] + ue[2] * n[2]) / ae;
      if (mn >= 1.0) {
        for (int c = 0; c < 5; ++c) qb[c] = qe[c];
      } else {
        double eint = pe / ((g - 1.0) * rho_e);
        double rho_b = P->p_inf / ((g - 1.0) * eint);
        conserved(g, rho_b, ue, P->p_inf, qb);
      }
      set_q(&G, q, b, qb);
    }
  return OR_OK;
}

/* ---------------------------------------------------------------------------------------
 * Time step and Runge-Kutta (paper, Time Marching Method).
 * ------------------------------------------------------------------------------------- */

/* Reading: one global step dt = CFL min over updated nodes of J^-1/(Lam_xi + Lam_eta +
 * Lam_zeta) (inviscid spectral radii), recomputed from Q^n at the start of every step. */
int or_dt(const or_params* P, const double* S, const double* jinv, const double* q, double cfl,
          double* dt) {
  Grid G;
  int rc = setup(&G, P);
  if (rc) return rc;
  Work W;
  if (work_alloc(&W, G.N)) return OR_ENOMEM;
  primitives(&G, q, &W);
  spectral_radii(&G, S, &W);
  double best = INFINITY;
  for (long id = 0; id < G.N; ++id) {
    int ix[3];
    unflat(&G, id, ix);
    if (!updated(&G, ix)) continue;
    double r = jinv[id] / (W.lam[0][id] + W.lam[1][id] + W.lam[2][id]);
    if (r < best) best = r;
  }
  *dt = cfl * best;
  work_free(&W);
  return OR_OK;
}

static int state_ok(const Grid* G, const double* q) {
  long N = G->N;
  for (long id = 0; id < N; ++id) {
    double rho = q[id];
    double e = q[4 * N + id];
    double ke = 0.5 * (q[N + id] * q[N + id] + q[2 * N + id] * q[2 * N + id] +
                       q[3 * N + id] * q[3 * N + id]) / rho;
    double pr = e - ke;
    if (!isfinite(rho) || !isfinite(e) || !(rho > 0.0) || !(pr > 0.0)) return 0;
    for (int c = 1; c < 4; ++c)
      if (!isfinite(q[(long)c * N + id])) return 0;
  }
  return 1;
}

/* Jameson's five-stage scheme with alpha = (1/4, 1/6, 3/8, 1/2, 1):
 * Q^(l) = Q^(0) - alpha_l dt J RHS(Q^(l-1)) at updated nodes, then the boundary conditions.
 * Reading: the integrated variable is J^-1 Q on a stationary grid, so the physical state is
 * advanced with J = 1/J^-1; the step is global (the LES uses a constant dt). */
int or_step(const or_params* P, const double* xyz, const double* S, const double* jinv,
            double* q, int nsteps, double cfl, double dt_fixed, double* dt_last) {
  static const double alpha[5] = {0.25, 1.0 / 6.0, 0.375, 0.5, 1.0};
  Grid G;
  int rc = setup(&G, P);
  if (rc) return rc;
  if (nsteps < 0) return OR_EINVAL;
  long N = G.N;
  double* q0 = (double*)malloc(sizeof(double) * 5 * N);
  double* rhs = (double*)malloc(sizeof(double) * 5 * N);
  if (!q0 || !rhs) { free(q0); free(rhs); return OR_ENOMEM; }
  Work W;
  if (work_alloc(&W, N)) { free(q0); free(rhs); return OR_ENOMEM; }
  double dt = dt_fixed;
  for (int s = 0; s < nsteps; ++s) {
    if (cfl > 0.0) {
      rc = or_dt(P, S, jinv, q, cfl, &dt);
      if (rc) break;
    }
    memcpy(q0, q, sizeof(double) * 5 * N);
    for (int l = 0; l < 5; ++l) {
      node_state(&G, S, jinv, q, &W);
      face_fluxes(&G, S, jinv, q, &W);
      residual_from_work(&G, &W, rhs);
#pragma omp parallel for
      for (int k = 0; k < G.n[2]; ++k)
        for (int j = 0; j < G.n[1]; ++j)
          for (int i = 0; i < G.n[0]; ++i) {
            int ix[3] = {i, j, k};
            long id = ID(&G, ix);
            if (!updated(&G, ix)) continue;
            double J = 1.0 / jinv[id];
            for (int c = 0; c < 5; ++c)
              q[(long)c * N + id] = q0[(long)c * N + id] - alpha[l] * dt * J * rhs[(long)c * N + id];
          }
      or_apply_bc(P, xyz, S, jinv, q);
    }
  }
  if (dt_last) *dt_last = dt;
  if (!rc && !state_ok(&G, q)) rc = OR_ENONFINITE;
  work_free(&W);
  free(q0);
  free(rhs);
  return rc;
}

/* Diagnostics over updated nodes, summed in index order:
 * out[0] = sum J^-1 rho|u|^2/2 / sum J^-1 (volume-weighted kinetic energy),
 * out[1..5] = sum J^-1 Q_c (the discrete totals conserved on a periodic grid). */
int or_diagnostics(const or_params* P, const double* jinv, const double* q, double* out) {
  Grid G;
  int rc = setup(&G, P);
  if (rc) return rc;
  long N = G.N;
  double vol = 0.0, ke = 0.0, tot[5] = {0, 0, 0, 0, 0};
  for (long id = 0; id < N; ++id) {
    int ix[3];
    unflat(&G, id, ix);
    if (!updated(&G, ix)) continue;
    double rho = q[id];
    double m2 = q[N + id] * q[N + id] + q[2 * N + id] * q[2 * N + id] + q[3 * N + id] * q[3 * N + id];
    vol += jinv[id];
    ke += jinv[id] * 0.5 * m2 / rho;
    for (int c = 0; c < 5; ++c) tot[c] += jinv[id] * q[(long)c * N + id];
  }
  out[0] = ke / vol;
  for (int c = 0; c < 5; ++c) out[1 + c] = tot[c];
  return OR_OK;
}
