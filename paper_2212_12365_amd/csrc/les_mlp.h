// Learned subgrid closure: device-side pieces shared by the node kernel and les_mlp.hip.
//
// The closure keeps the paper's eddy-viscosity form mu_t = rho c Delta^2 |S| (Subgrid Scale
// Modeling) and predicts the coefficient c per node with a 6-64-64-1 network (GELU in its
// tanh form, softplus output) from six scale-free invariants of the resolved velocity
// gradient. Where an input is not finite, |S| = 0, or an input leaves the trained range,
// c = C_s^2 (plain Smagorinsky).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/lesmi.h"

namespace lesmi {

constexpr int kMlpIn = LES_MLP_INPUTS;
constexpr int kMlpH = LES_MLP_HIDDEN;
constexpr int kMlpP = LES_MLP_NPARAMS;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpH * kMlpIn;
constexpr int kOffW2 = kOffB1 + kMlpH;
constexpr int kOffB2 = kOffW2 + kMlpH * kMlpH;
constexpr int kOffW3 = kOffB2 + kMlpH;
constexpr int kOffB3 = kOffW3 + kMlpH;
static_assert(kOffB3 + 1 == kMlpP, "parameter layout");

// The network as the kernels see it: FP32 master parameters (device) and the input
// normalisation and trained range.
struct MlpNet {
  const float* theta;
  les_mlp_norm norm;
  float cs2;
};

// Velocity gradient g[m][n] = d u_m / d x_n = J sum_e S_e^n d[e][m] from the nodal
// differences d[e][m] = delta_e u_m and the metrics s[3e + n]; 0 where J^-1 <= 0.
template <typename R>
__device__ __forceinline__ void velocity_gradient(const R* s, const R d[3][3], R jinv,
                                                  R g[3][3]) {
  const R J = jinv > (R)0 ? (R)1 / jinv : (R)0;
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int n = 0; n < 3; ++n)
      g[m][n] = J * (s[n] * d[0][m] + s[3 + n] * d[1][m] + s[6 + n] * d[2][m]);
}

// The six inputs of the closure and |S| = (2 S:S)^(1/2) from g (f is left non-finite where
// |S| = 0, which selects the fallback).
template <typename R>
__device__ __forceinline__ R mlp_invariants(const R g[3][3], R* f) {
  R S[3][3], O[3][3];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      S[m][n] = (R)0.5 * (g[m][n] + g[n][m]);
      O[m][n] = (R)0.5 * (g[m][n] - g[n][m]);
    }
  const R trS = S[0][0] + S[1][1] + S[2][2];
  R ss = (R)0;
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int n = 0; n < 3; ++n) ss += S[m][n] * S[m][n];
  const R smag = sqrt((R)2 * ss);
  R Sd[3][3];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int n = 0; n < 3; ++n) Sd[m][n] = S[m][n] - (m == n ? trS / (R)3 : (R)0);
  R Sd2[3][3], O2[3][3];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      R a = (R)0, b = (R)0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        a += Sd[m][k] * Sd[k][n];
        b += O[m][k] * O[k][n];
      }
      Sd2[m][n] = a;
      O2[m][n] = b;
    }
  R t2 = (R)0, to = (R)0, t3 = (R)0, tso = (R)0, t22 = (R)0;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    t2 += Sd2[m][m];
    to += O2[m][m];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      t3 += Sd2[m][k] * Sd[k][m];
      tso += Sd[m][k] * O2[k][m];
      t22 += Sd2[m][k] * O2[k][m];
    }
  }
  const R i1 = (R)1 / smag;  // inf at |S| = 0: the inputs become non-finite
  const R i2 = i1 * i1;
  f[0] = trS * i1;
  f[1] = t2 * i2;
  f[2] = to * i2;
  f[3] = t3 * i2 * i1;
  f[4] = tso * i2 * i1;
  f[5] = t22 * i2 * i2;
  return smag;
}

// Launch of the closure over a context's nodes: reads the features and the scale
// rho Delta^2 |S| the node kernel wrote, and overwrites the eddy-viscosity record.
struct MlpClosureArgs {
  MlpNet net;
  const float* feat;   // [6][N]
  const float* scale;  // [N]
  long long n;
  void* mut_rec;       // record plane of mu_t (double or float)
  int mixed;           // 1: mut_rec is float
  double* mut_out;     // optional copy of mu_t [N]
  unsigned* fallback;  // optional count of fallback nodes
};
hipError_t launch_mlp_closure(const MlpClosureArgs& A, hipStream_t s);

}  // namespace lesmi
