// Device-side arithmetic of the LES residual (gfx950). Every function works on values in
// registers; the kernels decide where the values come from (HBM, LDS or a neighbour's
// registers). Equations follow Junqueira-Junior et al., arXiv 2212.12365; the section named
// in each comment is the paper's.
#pragma once

#include <hip/hip_runtime.h>

namespace lesmi {

struct Phys {
  double gamma, gm1, inv_gm1;  // gamma, gamma - 1, 1/(gamma - 1)
  double inv_re;               // 1 / Re_acoustic (0: no molecular viscosity)
  double inv_pr, inv_prs;      // 1/Pr, 1/Pr_sgs
  double s1, s1p1;             // Sutherland constant S1* and 1 + S1*
  double cs2;                  // C_s^2
  double k2, k4;
};

// Primitive variables of a node (paper, LES formulation: equation of state and System-I
// energy, in reference units): p = (gamma-1)(e - rho|u|^2/2), T = gamma p / rho, a^2 = T.
struct Prim {
  double rho, u, v, w, p, T;
};

__device__ __forceinline__ Prim prim_from_q(double r, double mu_, double mv, double mw,
                                            double e, const Phys& P) {
  Prim s;
  double ir = 1.0 / r;
  s.rho = r;
  s.u = mu_ * ir;
  s.v = mv * ir;
  s.w = mw * ir;
  s.p = P.gm1 * (e - 0.5 * r * (s.u * s.u + s.v * s.v + s.w * s.w));
  s.T = P.gamma * s.p * ir;
  return s;
}

// Sutherland's law in reference units, mu*(T*) = T*^(3/2) (1 + S1*)/(T* + S1*).
__device__ __forceinline__ double sutherland(double T, const Phys& P) {
  return T * sqrt(T) * P.s1p1 / (T + P.s1);
}

// J^-1 lambda_d = |S_d . u| + a |S_d| (paper, Spatial Discretization, spectral radii).
__device__ __forceinline__ double spectral(double sx, double sy, double sz, double u, double v,
                                           double w, double a) {
  return fabs(sx * u + sy * v + sz * w) + a * sqrt(sx * sx + sy * sy + sz * sz);
}

// Anisotropic scaling, carried times J^-1: Lb_d = L_d + sqrt(L_d L_e) + sqrt(L_d L_f).
__device__ __forceinline__ void scaled_radii(double l0, double l1, double l2, double* lb) {
  double s01 = sqrt(l0 * l1), s02 = sqrt(l0 * l2), s12 = sqrt(l1 * l2);
  lb[0] = l0 + s01 + s02;
  lb[1] = l1 + s01 + s12;
  lb[2] = l2 + s02 + s12;
}

// Jameson pressure sensor |p+ - 2p + p-| / (p+ + 2p + p-).
__device__ __forceinline__ double sensor(double pm, double p0, double pp) {
  return fabs(pp - 2.0 * p0 + pm) / (pp + 2.0 * p0 + pm);
}

// Smagorinsky eddy viscosity rho C_s^2 Delta^2 |S| with Delta^3 = J^-1, from the nodal
// differences delta_e u_m (d[e][m]) and metrics S_e^n (s[3e+n]) (paper, Subgrid Scale
// Viscosity). The gradient is du_m/dx_n = J sum_e S_e^n delta_e u_m.
__device__ __forceinline__ double smagorinsky(const double* s, const double d[3][3], double rho,
                                              double jinv, const Phys& P) {
  if (!(jinv > 0.0)) return 0.0;
  double J = 1.0 / jinv;
  double g[3][3];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int n = 0; n < 3; ++n)
      g[m][n] = J * (s[n] * d[0][m] + s[3 + n] * d[1][m] + s[6 + n] * d[2][m]);
  double ss = g[0][0] * g[0][0] + g[1][1] * g[1][1] + g[2][2] * g[2][2];
  double a01 = 0.5 * (g[0][1] + g[1][0]);
  double a02 = 0.5 * (g[0][2] + g[2][0]);
  double a12 = 0.5 * (g[1][2] + g[2][1]);
  ss += 2.0 * (a01 * a01 + a02 * a02 + a12 * a12);
  double smag = sqrt(2.0 * ss);
  double delta = cbrt(jinv);
  return rho * P.cs2 * delta * delta * smag;
}

// Inviscid node flux along direction d with metric row (sx, sy, sz) (paper, Transformation
// of Coordinates, inviscid flux vectors on a stationary grid).
__device__ __forceinline__ void inviscid_flux(double sx, double sy, double sz, const double* q,
                                              const Prim& s, double* F) {
  double un = sx * s.u + sy * s.v + sz * s.w;
  F[0] = q[0] * un;
  F[1] = q[1] * un + s.p * sx;
  F[2] = q[2] * un + s.p * sy;
  F[3] = q[3] * un + s.p * sz;
  F[4] = (q[4] + s.p) * un;
}

// Turkel-Vatsa dissipation on a face: D = Lf (eps2 dW - eps4 d3W), with
// eps2 = k2 max(nuA, nuB), eps4 = max(0, k4 - eps2) (paper, Spatial Discretization).
__device__ __forceinline__ void dissipation(double lf, double nuA, double nuB, const double* dW,
                                            const double* d3W, const Phys& P, double* D) {
  double eps2 = P.k2 * fmax(nuA, nuB);
  double eps4 = fmax(0.0, P.k4 - eps2);
#pragma unroll
  for (int c = 0; c < 5; ++c) D[c] = lf * (eps2 * dW[c] - eps4 * d3W[c]);
}

// Viscous + SGS face flux (paper, Transformation of Coordinates: viscous flux vectors;
// Subgrid Scale Modeling). Inputs are face values: Sf[9] face-averaged metrics, jinvf the
// face-averaged J^-1, grad_xi[v][e] the derivative of variable v in {u,v,w,T} along
// direction e, muf and mutf face-averaged molecular and eddy viscosities, ub the face
// velocity. d is the face direction. Output F[1..4] (the mass component is zero).
__device__ __forceinline__ void viscous_flux(const double* Sf, double jinvf,
                                             const double gxi[4][3], double muf, double mutf,
                                             const double* ub, int d, const Phys& P,
                                             double* F) {
  double Jf = 1.0 / jinvf;
  double g[4][3];  // d(var)/dx_n
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int n = 0; n < 3; ++n)
      g[v][n] = Jf * (Sf[n] * gxi[v][0] + Sf[3 + n] * gxi[v][1] + Sf[6 + n] * gxi[v][2]);
  double visc = muf * P.inv_re + mutf;
  double kappa = (muf * P.inv_re * P.inv_pr + mutf * P.inv_prs) * P.inv_gm1;
  double div = g[0][0] + g[1][1] + g[2][2];
  double t00 = visc * (2.0 * g[0][0] - (2.0 / 3.0) * div);
  double t11 = visc * (2.0 * g[1][1] - (2.0 / 3.0) * div);
  double t22 = visc * (2.0 * g[2][2] - (2.0 / 3.0) * div);
  double t01 = visc * (g[0][1] + g[1][0]);
  double t02 = visc * (g[0][2] + g[2][0]);
  double t12 = visc * (g[1][2] + g[2][1]);
  double bx = t00 * ub[0] + t01 * ub[1] + t02 * ub[2] + kappa * g[3][0];
  double by = t01 * ub[0] + t11 * ub[1] + t12 * ub[2] + kappa * g[3][1];
  double bz = t02 * ub[0] + t12 * ub[1] + t22 * ub[2] + kappa * g[3][2];
  const double* sd = Sf + 3 * d;
  F[1] = sd[0] * t00 + sd[1] * t01 + sd[2] * t02;
  F[2] = sd[0] * t01 + sd[1] * t11 + sd[2] * t12;
  F[3] = sd[0] * t02 + sd[1] * t12 + sd[2] * t22;
  F[4] = sd[0] * bx + sd[1] * by + sd[2] * bz;
}

}  // namespace lesmi
