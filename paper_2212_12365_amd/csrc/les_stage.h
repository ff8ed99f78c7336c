// Launch interface of the Runge-Kutta stage kernels (les_stage.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "les_common.h"

namespace lesmi {

// Node record fields, each a plane of N doubles.
enum {
  kRecU = 0, kRecV, kRecW, kRecT, kRecP, kRecMu, kRecMut,
  kRecLb,           // three planes: scaled spectral radius along xi, eta, zeta
  kRecNu = kRecLb + 3,  // three planes: pressure sensor along xi, eta, zeta
  kRecCount = kRecNu + 3
};

struct StageArgs {
  Dims D;
  Phys P;
  const double* q;     // stage input Q^(l-1) [5][N]
  const double* S;     // metrics [9][N]
  const double* jinv;  // [N]
  const double* jac;   // 1/J^-1 at updated nodes [N]
  double* rec;         // node records [kRecCount][N]
  double* mut_out;     // optional copy of the eddy viscosity [N] (k_nodes)
  // Mixed form: FP32 metrics and node records; the fluxes are evaluated in FP32.
  int mixed;
  const float* S32;    // [9][N]
  float* rec32;        // [kRecCount][N]
  // k_stage output: mode 0 -> residual into out; mode 1 -> out = q0 - alpha dt J RHS.
  int mode;
  double* out;
  const double* q0;
  const double* dt;
  double alpha;
  int tile;   // k_stage_planes tile shape, index into kTileNames
  int kmin;   // smallest z-chunk depth (0 = default)
};

constexpr int kNumTiles = 6;
extern const char* const kTileNames[kNumTiles];

hipError_t launch_nodes(const StageArgs& A, hipStream_t s);
hipError_t launch_stage(const StageArgs& A, hipStream_t s);

}  // namespace lesmi
