// Shared host/device definitions of the lesmi library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lesmi.h"
#include "les_device.h"

namespace lesmi {

// Grid extents, periodicity and derived sizes, passed by value to every kernel.
struct Dims {
  int n[3];
  int per[3];
  int jet;     // 1 for the jet boundary set, 0 for a periodic box
  long long N; // nodes
};

__device__ __host__ __forceinline__ long long nid(const Dims& D, int i, int j, int k) {
  return (long long)i + (long long)D.n[0] * ((long long)j + (long long)D.n[1] * k);
}

__device__ __host__ __forceinline__ bool is_updated(const Dims& D, int i, int j, int k) {
  if (!D.per[0] && (i == 0 || i == D.n[0] - 1)) return false;
  if (!D.per[1] && (j == 0 || j == D.n[1] - 1)) return false;
  if (!D.per[2] && (k == 0 || k == D.n[2] - 1)) return false;
  return true;
}

struct BcData {
  double* nff;    // [3][ni*nk] far-field outward unit normal at j = nj-1
  double* nin;    // [3][nj*nk] entrance outward unit normal at i = 0
  double* nex;    // [3][nj*nk] exit outward unit normal at i = ni-1 (axis node: j = 1's)
  int* jetmask;   // [nj*nk] entrance node lies inside the jet
  double* axis;   // [5][ni] centreline means
  double rho_inf, u_inf[3], p_inf, mach_jet;
};

}  // namespace lesmi

struct les_ctx {
  les_params params;
  lesmi::Dims dims;
  lesmi::Phys phys;
  long long n_updated = 0;
  int device = 0;
  std::string err;

  // Metrics (FP64): S[9][N], jinv[N], jac[N] = 1/jinv at updated nodes (0 elsewhere).
  double* S = nullptr;
  double* jinv = nullptr;
  double* jac = nullptr;
  lesmi::BcData bc{};

  // Runge-Kutta stage buffers [5][N] each.
  double* qa = nullptr;
  double* qb = nullptr;

  // Node records of the stage kernels [kRecCount][N] (FP64 form), or the mixed form's
  // FP32 records [kRecCount][N] and FP32 copy of the metrics.
  double* rec = nullptr;
  float* rec32 = nullptr;
  float* S32 = nullptr;
  // Stage kernel launch shape (index into the tile table) and smallest z-chunk depth.
  int tile = 0;
  int kmin = 8;

  // Scalars: dt, min-ratio bits, status flags, reduction partials.
  double* d_dt = nullptr;
  double* d_dtpart = nullptr;   // per-block minima of the time-step reduction
  int* d_flag = nullptr;
  double* d_partial = nullptr;  // [kMaxPartials * 7]
  double* d_diag = nullptr;     // [6]

  // Learned closure (closure == LES_MLP): network parameters (FP32) and input
  // normalisation, the per-node inputs and scale written by the node kernel, and a count of
  // nodes where the closure fell back to Smagorinsky.
  float* mlp_theta = nullptr;
  les_mlp_norm mlp_norm{};
  bool mlp_ready = false;
  float* mlp_feat = nullptr;   // [6][N]
  float* mlp_scale = nullptr;  // [N]
  unsigned* mlp_fallback = nullptr;

  // Running statistics: sums of (rho, u, v, w, p) and of their squares [5][N], samples.
  double* stat_sum = nullptr;
  double* stat_sq = nullptr;
  long long stat_n = 0;

  // Optional timing of the stage kernel launches with HIP events on the caller's stream.
  bool prof = false;
  std::vector<hipEvent_t> ev;
  size_t nrec = 0;

  // Dual time stepping: Q^n and Q^(n-1) [5][N], the residual of a stage [5][N], the local
  // pseudo-time steps [N] (allocated by the first les_dual_step), and the device record of
  // the unsteady residual norms.
  double* dual_qn = nullptr;
  double* dual_qm = nullptr;
  double* dual_rhs = nullptr;
  double* dual_dtau = nullptr;
  double* dual_res = nullptr;
  int dual_res_cap = 0;

  // One Runge-Kutta step captured in a HIP graph (on the context's own non-blocking stream)
  // and replayed on the caller's stream; recaptured when the state pointer, the time-step
  // mode or value, the launch tuning or the network normalisation changes.
  bool use_graph = true;
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  const double* graph_q = nullptr;
  double graph_cfl = 0.0, graph_dt = 0.0;
  int graph_tile = -1, graph_kmin = -1;
};
