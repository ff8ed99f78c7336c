// Launch interface of the Runge-Kutta stage kernels (les_stage.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "les_common.h"
#include "les_mlp.h"

namespace lesmi {

// Node record fields, each a plane of N values (FP64, or FP32 in the mixed form). The
// primitive variables and the molecular viscosity are not stored: the face kernel forms them
// from the state it stages.
enum {
  kRecMut = 0,
  kRecLb,               // three planes: scaled spectral radius along xi, eta, zeta
  kRecNu = kRecLb + 3,  // three planes: pressure sensor along xi, eta, zeta
  kRecDz = kRecNu + 3,  // four planes: centred zeta differences (x_{k+1} - x_{k-1})/2 of
                        // u, v, w, T
  kRecCount = kRecDz + 4
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
  // k_stage output: mode 0 -> residual into out; mode 1 -> out = q0 - alpha dt J RHS;
  // mode 2 -> the dual-time update below.
  int mode;
  double* out;
  const double* q0;
  const double* dt;
  double alpha;
  // Time-step reduction in the node kernel (null: off): each updated node contributes
  // J^-1 / (sum of its three spectral radii) in FP64, the same operations on the same values
  // as the separate reduction; block b of the node kernel writes its minimum to dtpart[b],
  // and a non-positive density or pressure or a non-finite ratio sets bit 2 of *flag.
  double* dtpart;
  int* flag;
  // Local pseudo-time steps of dual time stepping (null: off): the node kernel writes
  // dtau_out[o] = cfl_tau J^-1 / (sum of the three spectral radii) in FP64 at updated nodes
  // and 0 elsewhere.
  double* dtau_out;
  double cfl_tau;
  // Dual time stepping's point-implicit update fused into the face kernel (mode 2, default
  // launch shapes): out = [q0 - alpha dtau (J RHS + hist/dt)] / (1 + alpha dtau a0/dt) at
  // updated nodes, hist = a1 Q^n + a2 Q^(n-1) (Q^(n-1) read only when a2 != 0).
  const double* dual_qn;
  const double* dual_qm;
  const double* dual_dtau;
  double dual_a0, dual_a1, dual_a2, dual_dt;
  int tile;   // k_stage_planes tile shape, index into kTileNames
  int kmin;   // smallest z-chunk depth (0 = default)
  // Learned closure (k_nodes): inputs [6][N], scale rho Delta^2 |S| [N] and |S| [N] of the
  // network; each may be null.
  float* feat;
  float* fscale;
  float* fsmag;
  // Learned closure evaluated inside the node kernel (mlp_fused != 0): the network's
  // coefficient replaces the Smagorinsky coefficient in the eddy-viscosity record, with no
  // inputs written out; fallback nodes are counted into *mlp_fallback (may be null).
  int mlp_fused;
  MlpNet mlp;
  unsigned* mlp_fallback;
};

constexpr int kNumTiles = 10;
// Default launch shapes (indices into kTileNames): 16x16 in FP64, 32x8 in the mixed form.
constexpr int kDefaultTileFp64 = 3, kDefaultTileMixed = 0;
extern const char* const kTileNames[kNumTiles];

hipError_t launch_nodes(const StageArgs& A, hipStream_t s);
// Number of blocks of the node kernel (the partial minima of its time-step reduction).
int nodes_blocks(const Dims& D);
hipError_t launch_stage(const StageArgs& A, hipStream_t s);

// Thread-tile extent of a tile index, and the z-chunk depth of the face kernel for it: at
// least kmin planes, chosen against the number of blocks resident at once (resident <= 0:
// chunks for about 1024 blocks, the form the persistent batch work lists use).
void tile_shape(int tile, int* tx, int* ty);
int kchunk_for(const Dims& D, int tx, int ty, int kmin, int resident);

// A persistent launch over a batch: `args` holds one StageArgs per member (device), `work`
// the work items (device). grid <= 0 asks for the kernel's resident blocks per CU instead
// (written to *occupancy).
struct BatchLaunch {
  const StageArgs* args;
  const int4* work;
  int nwork;
  int grid;
  int tile;
  bool mixed;
  int* occupancy;
  // Node kernel only: also write each item's time-step partial minimum (StageArgs::dtpart
  // of its member, at the item's slot).
  bool dt = false;
};
// Node-kernel items are (member, bx | by << 16, kbeg | kend << 16, slot) over 64 x 4 column
// tiles and z-chunks of nodes_kchunk planes; slot numbers the member's items.
hipError_t launch_nodes_batch(const BatchLaunch& B, hipStream_t s);
int nodes_kchunk(const Dims& D);

// Stage arguments of a context for input state q (lesmi.hip).
StageArgs stage_args_of(les_ctx* c, const double* q);

// Runge-Kutta stage coefficients alpha_1..alpha_5 (paper, Time Marching Method).
constexpr double kAlpha[5] = {0.25, 1.0 / 6.0, 0.375, 0.5, 1.0};
hipError_t launch_stage_batch(const BatchLaunch& B, hipStream_t s);

}  // namespace lesmi
