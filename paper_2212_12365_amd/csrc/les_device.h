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
  // Pressure carried as p - p_ref in the node records (0 in FP64). The dropped p_ref S_d
  // terms sum to p_ref * sum_d delta_d S_d, which the conservative metrics make vanish at
  // every updated node.
  double p_ref;
  // Reference dissipated vector (rho, rho u, rho v, rho w, e + p) of the free stream,
  // subtracted in FP64 before the FP32 cast in the mixed form (0 in FP64). Differences of
  // W are unchanged; the FP32 rounding error of W then scales with |W - W_ref| rather than
  // |W|, which keeps the fourth-difference dissipation of a near-uniform free stream free
  // of rounding noise.
  double wref[5];
};

// The same constants in the arithmetic type of a kernel (double, or float for the mixed
// form).
template <typename R>
struct PhysT {
  R gamma, gm1, inv_gm1, inv_re, inv_pr, inv_prs, s1, s1p1, cs2, k2, k4;
  R wref[5];
  __device__ __host__ explicit PhysT(const Phys& P)
      : gamma((R)P.gamma), gm1((R)P.gm1), inv_gm1((R)P.inv_gm1), inv_re((R)P.inv_re),
        inv_pr((R)P.inv_pr), inv_prs((R)P.inv_prs), s1((R)P.s1), s1p1((R)P.s1p1),
        cs2((R)P.cs2), k2((R)P.k2), k4((R)P.k4) {
    for (int c = 0; c < 5; ++c) wref[c] = (R)P.wref[c];
  }
};

// a * b + c with one rounding. The flux formulas spell out their fused products with it
// (the translation units are compiled without automatic contraction), so every evaluation
// context of a face rounds the same way.
template <typename R>
__device__ __forceinline__ R fmadd(R a, R b, R c) {
  if constexpr (sizeof(R) == sizeof(float))
    return __builtin_fmaf(a, b, c);
  else
    return __builtin_fma(a, b, c);
}

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
  s.p = P.gm1 * fmadd(-0.5 * r, fmadd(s.w, s.w, fmadd(s.v, s.v, s.u * s.u)), e);
  s.T = P.gamma * s.p * ir;
  return s;
}

// Sutherland's law in reference units, mu*(T*) = T*^(3/2) (1 + S1*)/(T* + S1*).
template <typename R, typename PP>
__device__ __forceinline__ R sutherland(R T, const PP& P) {
  return T * sqrt(T) * (R)P.s1p1 / (T + (R)P.s1);
}

// J^-1 lambda_d = |S_d . u| + a |S_d| (paper, Spatial Discretization, spectral radii).
template <typename R>
__device__ __forceinline__ R spectral(R sx, R sy, R sz, R u, R v, R w, R a) {
  return fabs(sx * u + sy * v + sz * w) + a * sqrt(sx * sx + sy * sy + sz * sz);
}

// Anisotropic scaling, carried times J^-1: Lb_d = L_d + sqrt(L_d L_e) + sqrt(L_d L_f).
template <typename R>
__device__ __forceinline__ void scaled_radii(R l0, R l1, R l2, R* lb) {
  R s01 = sqrt(l0 * l1), s02 = sqrt(l0 * l2), s12 = sqrt(l1 * l2);
  lb[0] = l0 + s01 + s02;
  lb[1] = l1 + s01 + s12;
  lb[2] = l2 + s02 + s12;
}

// Jameson pressure sensor |p+ - 2p + p-| / (p+ + 2p + p-).
template <typename R>
__device__ __forceinline__ R sensor(R pm, R p0, R pp) {
  return fabs(pp - (R)2 * p0 + pm) / (pp + (R)2 * p0 + pm);
}

// Smagorinsky eddy viscosity rho C_s^2 Delta^2 |S| with Delta^3 = J^-1, from the nodal
// differences delta_e u_m (d[e][m]) and metrics S_e^n (s[3e+n]) (paper, Subgrid Scale
// Viscosity). The gradient is du_m/dx_n = J sum_e S_e^n delta_e u_m.
template <typename R, typename PP>
__device__ __forceinline__ R smagorinsky(const R* s, const R d[3][3], R rho, R jinv,
                                         const PP& P) {
  if (!(jinv > (R)0)) return (R)0;
  R J = (R)1 / jinv;
  R g[3][3];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int n = 0; n < 3; ++n)
      g[m][n] = J * (s[n] * d[0][m] + s[3 + n] * d[1][m] + s[6 + n] * d[2][m]);
  R ss = g[0][0] * g[0][0] + g[1][1] * g[1][1] + g[2][2] * g[2][2];
  R a01 = (R)0.5 * (g[0][1] + g[1][0]);
  R a02 = (R)0.5 * (g[0][2] + g[2][0]);
  R a12 = (R)0.5 * (g[1][2] + g[2][1]);
  ss += (R)2 * (a01 * a01 + a02 * a02 + a12 * a12);
  R smag = sqrt((R)2 * ss);
  R delta = cbrt(jinv);
  return rho * (R)P.cs2 * delta * delta * smag;
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

// Turkel-Vatsa coefficients of a face (paper, Spatial Discretization): eps2 = k2 max(nuA, nuB)
// and eps4 = max(0, k4 - eps2); the face's dissipation is Lf (eps2 dW - eps4 d3W).
template <typename R, typename PP>
__device__ __forceinline__ void dissipation_coefficients(R nuA, R nuB, const PP& P, R* eps2,
                                                         R* eps4) {
  *eps2 = (R)P.k2 * (nuA > nuB ? nuA : nuB);
  const R e4 = (R)P.k4 - *eps2;
  *eps4 = e4 > (R)0 ? e4 : (R)0;
}

// Viscous + SGS face flux (paper, Transformation of Coordinates: viscous flux vectors;
// Subgrid Scale Modeling). The face metrics, J^-1, molecular and eddy viscosities are the
// averages of the two nodes' values; they are passed as sums (Ss[9] the metrics, js the J^-1,
// mus and muts the viscosities), and the halves are folded in exactly: J_f S_f = Ss / js in
// the gradient, and F_v = (S_f)_d . tau = (Ss)_d . (tau / 2), so the viscosities enter halved
// once more. grad_xi[v][e] is the derivative of variable v in {u,v,w,T} along direction e, ub
// the face velocity, d the face direction. Output F[1..4] (the mass component is zero).
template <typename R, typename PP>
__device__ __forceinline__ void viscous_flux(const R* Ss, R js, const R gxi[4][3], R mus,
                                             R muts, const R* ub, int d, const PP& P, R* F) {
  const R Jf = (R)1 / js;
  R g[4][3];  // d(var)/dx_n
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int n = 0; n < 3; ++n)
      g[v][n] = Jf * fmadd(Ss[6 + n], gxi[v][2], fmadd(Ss[3 + n], gxi[v][1], Ss[n] * gxi[v][0]));
  const R mi = mus * (R)P.inv_re;
  // Half the face values: visc = (mu/Re + mu_t)/2, kappa = [mu/(Re Pr) + mu_t/Pr_t]/(gamma-1)/2.
  R visc = (R)0.25 * (mi + muts);
  R kappa = (R)0.25 * fmadd(mi, (R)P.inv_pr, muts * (R)P.inv_prs) * (R)P.inv_gm1;
  R div = g[0][0] + g[1][1] + g[2][2];
  const R c23 = -((R)2 / (R)3);
  R t00 = visc * fmadd(c23, div, (R)2 * g[0][0]);
  R t11 = visc * fmadd(c23, div, (R)2 * g[1][1]);
  R t22 = visc * fmadd(c23, div, (R)2 * g[2][2]);
  R t01 = visc * (g[0][1] + g[1][0]);
  R t02 = visc * (g[0][2] + g[2][0]);
  R t12 = visc * (g[1][2] + g[2][1]);
  R bx = fmadd(kappa, g[3][0], fmadd(t02, ub[2], fmadd(t01, ub[1], t00 * ub[0])));
  R by = fmadd(kappa, g[3][1], fmadd(t12, ub[2], fmadd(t11, ub[1], t01 * ub[0])));
  R bz = fmadd(kappa, g[3][2], fmadd(t22, ub[2], fmadd(t12, ub[1], t02 * ub[0])));
  const R* sd = Ss + 3 * d;
  F[1] = fmadd(sd[2], t02, fmadd(sd[1], t01, sd[0] * t00));
  F[2] = fmadd(sd[2], t12, fmadd(sd[1], t11, sd[0] * t01));
  F[3] = fmadd(sd[2], t22, fmadd(sd[1], t12, sd[0] * t02));
  F[4] = fmadd(sd[2], bz, fmadd(sd[1], by, sd[0] * bx));
}

}  // namespace lesmi
