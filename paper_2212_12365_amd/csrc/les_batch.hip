// Batched ensembles: several independent grids (contexts) advanced together. Every kernel
// of a Runge-Kutta step is one persistent launch over a work list that spans all members,
// so small grids fill the GPU together; a whole step is captured once in a HIP graph and
// replayed. The stage-kernel launch shape comes from an autotuner that times the candidate
// shapes on the batch itself. The arithmetic per node and face is that of the single-grid
// path (the same device functions), so each member's result equals its single-grid run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "les_bcdt.h"
#include "les_common.h"
#include "les_stage.h"

using namespace lesmi;

namespace {

// Per-member data of the boundary, time-step and check kernels (device table).
struct MemberArgs {
  Dims D;
  Phys P;
  BcData B;
  const double* S;
  const double* jinv;
  double* dtpart;  // per-block minima of the time-step reduction
  int ndt;
  double* dt;
  int* flag;
};

constexpr int kRows = 6;  // stage rows 0..4 of a step, then the residual row of the tuner

// ---------------------------------------------------------------------------------------
// Persistent kernels. Items are int4: (member, ...).
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_batch_dt_final(const MemberArgs* __restrict__ M,
                                                        double cfl) {
  __shared__ double red[256];
  const MemberArgs& m = M[blockIdx.x];
  dt_final_block(m.dtpart, m.ndt, cfl, m.dt, red);
}

__global__ void k_batch_set_dt(const MemberArgs* __restrict__ M, int n, double dt) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < n) M[m].dt[0] = dt;
}

__global__ void k_batch_clear_flags(const MemberArgs* __restrict__ M, int n) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < n) M[m].flag[0] = 0;
}

__global__ void k_batch_gather(const MemberArgs* __restrict__ M, int n, double* __restrict__ dts,
                               int* __restrict__ flags) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < n) {
    dts[m] = M[m].dt[0];
    flags[m] = M[m].flag[0];
  }
}

// Boundary conditions of the stage output; items (member, i, 1): the centreline station i
// (with the entrance and exit nodes on the axis); items (member, block, 0): 256 of the other
// boundary nodes.
__global__ void __launch_bounds__(256) k_batch_bc(const StageArgs* __restrict__ row,
                                                  const MemberArgs* __restrict__ M,
                                                  const int4* __restrict__ work, int nwork) {
  __shared__ double ring[5][kAxisChunk];
  __shared__ double mean[5];
  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int4 it = work[w];
    const MemberArgs& m = M[it.x];
    if (it.z)
      bc_station_block(m.D, m.P, m.B, row[it.x].out, it.y, ring, mean);
    else
      bc_node(m.D, m.P, m.B, row[it.x].out, (long long)it.y * 256 + threadIdx.x);
  }
}

// State check of each member's state; items are (member, bx, by, k) over 64 x 4 blocks.
__global__ void __launch_bounds__(256) k_batch_check(const StageArgs* __restrict__ row0,
                                                     const MemberArgs* __restrict__ M,
                                                     const int4* __restrict__ work, int nwork) {
  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int4 it = work[w];
    const MemberArgs& m = M[it.x];
    check_node(m.D, m.P, row0[it.x].q, it.y * 64 + threadIdx.x, it.z * 4 + threadIdx.y, it.w,
               m.flag);
  }
}

template <class T>
hipError_t upload(T** d, const std::vector<T>& h) {
  if (*d) {
    (void)hipFree(*d);
    *d = nullptr;
  }
  if (h.empty()) return hipSuccess;
  hipError_t e = hipMalloc((void**)d, h.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
}

}  // namespace

struct les_batch {
  std::vector<les_ctx*> m;
  bool mixed = false;
  int tile = 0, kmin = 8;
  int cus = 256;
  int occ_nodes = 1, occ_faces = 1;  // resident blocks per CU of the two stage kernels
  int occ_bc = 1;                     // and of the boundary kernel
  std::string err;

  StageArgs* d_args = nullptr;  // [kRows][n]
  MemberArgs* d_mem = nullptr;  // [n]
  // Work lists: node kernel (tile, z-chunk), checks (64 x 4 block, plane), face kernel,
  // axis means, boundary nodes, time-step partials.
  int4 *d_wnodes = nullptr, *d_wcheck = nullptr, *d_wfaces = nullptr, *d_wbc = nullptr;
  int nwnodes = 0, nwcheck = 0, nwfaces = 0, nwbc = 0;
  double* d_dts = nullptr;
  int* d_flags = nullptr;

  std::vector<const double*> qbaked;  // state pointers written into d_args
  bool args_valid = false;

  bool use_graph = true;
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  double graph_cfl = 0.0, graph_dt = 0.0;
};

namespace {

int bfail(les_batch* b, int code, const std::string& msg) {
  if (b) b->err = msg;
  return code;
}

#define BHIP(b, expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return bfail(b, LES_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

void drop_graph(les_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
}

// Persistent grid: enough blocks to fill every CU at the kernel's occupancy, a multiple of
// 8 so that block b stays on XCD b % 8, and no more than the work needs (rounded up to 8).
int persistent_grid(les_batch* b, int occupancy, int nwork) {
  long long full = (long long)b->cus * std::max(occupancy, 1);
  long long need = ((long long)nwork + 7) / 8 * 8;
  long long g = std::min(full, need);
  g = std::max(8LL, g / 8 * 8);
  return (int)g;
}

int occupancy_of(les_batch* b, bool faces) {
  int occ = 1;
  BatchLaunch L{nullptr, nullptr, 0, 0, b->tile, b->mixed, &occ};
  hipError_t e = faces ? launch_stage_batch(L, nullptr) : launch_nodes_batch(L, nullptr);
  return e == hipSuccess ? occ : 1;
}

// Face-kernel work list for the current tile and kmin: one item per (member, column tile,
// z-chunk), members in order, tiles i-fastest within a chunk.
int build_face_work(les_batch* b) {
  int tx, ty;
  tile_shape(b->tile, &tx, &ty);
  std::vector<int4> w;
  for (int mi = 0; mi < (int)b->m.size(); ++mi) {
    const Dims& D = b->m[mi]->dims;
    const int gx = (D.n[0] + tx - 1) / tx, gy = (D.n[1] + ty - 1) / ty;
    const int kc = kchunk_for(D, tx, ty, b->kmin, 0);
    for (int k0 = 0; k0 < D.n[2]; k0 += kc)
      for (int by = 0; by < gy; ++by)
        for (int bx = 0; bx < gx; ++bx)
          w.push_back(make_int4(mi, bx | (by << 16), k0, std::min(k0 + kc, D.n[2])));
  }
  b->nwfaces = (int)w.size();
  b->occ_faces = occupancy_of(b, true);
  BHIP(b, upload(&b->d_wfaces, w));
  return LES_OK;
}

int build_static_work(les_batch* b) {
  std::vector<int4> wn, wc, wb;
  std::vector<MemberArgs> mem;
  for (int mi = 0; mi < (int)b->m.size(); ++mi) {
    les_ctx* c = b->m[mi];
    const Dims& D = c->dims;
    const int gx = (D.n[0] + 63) / 64, gy = (D.n[1] + 3) / 4;
    for (int k = 0; k < D.n[2]; ++k)
      for (int by = 0; by < gy; ++by)
        for (int bx = 0; bx < gx; ++bx) wc.push_back(make_int4(mi, bx, by, k));
    const int kc = nodes_kchunk(D);
    int slot = 0;  // the member's node items number its time-step partial minima
    for (int k0 = 0; k0 < D.n[2]; k0 += kc)
      for (int by = 0; by < gy; ++by)
        for (int bx = 0; bx < gx; ++bx)
          wn.push_back(make_int4(mi, bx | (by << 16), k0 | (std::min(k0 + kc, D.n[2]) << 16),
                                 slot++));
    if (D.jet) {  // the centreline stations first: they take longest
      for (int i = 1; i <= D.n[0] - 2; ++i) wb.push_back(make_int4(mi, i, 1, 0));
      for (long long blk = 0; blk * 256 < bc_count(D); ++blk)
        wb.push_back(make_int4(mi, (int)blk, 0, 0));
    }
    MemberArgs M{};
    M.D = D;
    M.P = c->phys;
    M.B = c->bc;
    M.S = c->S;
    M.jinv = c->jinv;
    M.dtpart = c->d_dtpart;
    M.ndt = slot;
    M.dt = c->d_dt;
    M.flag = c->d_flag;
    mem.push_back(M);
  }
  b->nwnodes = (int)wn.size();
  b->nwcheck = (int)wc.size();
  b->occ_nodes = occupancy_of(b, false);
  b->nwbc = (int)wb.size();
  BHIP(b, upload(&b->d_wnodes, wn));
  BHIP(b, upload(&b->d_wcheck, wc));
  BHIP(b, upload(&b->d_wbc, wb));
  BHIP(b, upload(&b->d_mem, mem));
  return LES_OK;
}

// Stage rows for the given member states: row l reads in_l and writes out_l exactly as the
// single-grid step does (stage buffers qa, qb; the last stage writes q).
int bake_args(les_batch* b, double* const* q) {
  const int n = (int)b->m.size();
  bool same = b->args_valid;
  for (int mi = 0; same && mi < n; ++mi) same = b->qbaked[mi] == q[mi];
  if (same) return LES_OK;
  std::vector<StageArgs> rows((size_t)kRows * n);
  for (int mi = 0; mi < n; ++mi) {
    les_ctx* c = b->m[mi];
    const double* in = q[mi];
    for (int l = 0; l < 5; ++l) {
      double* out = l == 4 ? q[mi] : (l % 2 == 0 ? c->qa : c->qb);
      StageArgs A = stage_args_of(c, in);
      A.mode = 1;
      A.out = out;
      A.q0 = q[mi];
      A.dt = c->d_dt;
      A.alpha = kAlpha[l];
      A.dtpart = c->d_dtpart;  // the first stage's node kernel reduces the time step
      A.flag = c->d_flag;
      rows[(size_t)l * n + mi] = A;
      in = out;
    }
    StageArgs R = stage_args_of(c, q[mi]);
    R.mode = 0;
    R.out = c->qa;
    rows[(size_t)5 * n + mi] = R;
  }
  BHIP(b, hipMemcpy(b->d_args, rows.data(), rows.size() * sizeof(StageArgs),
                    hipMemcpyHostToDevice));
  b->qbaked.assign(q, q + n);
  b->args_valid = true;
  return LES_OK;
}

int check_launch(les_batch* b, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return bfail(b, LES_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return LES_OK;
}

// With cfl > 0 the node kernel also reduces each member's time step from this stage's input
// (block minima, then k_batch_dt_final) before the face kernel uses it.
int enqueue_stage_kernels(les_batch* b, int row, hipStream_t s, double cfl = 0.0) {
  const int n = (int)b->m.size();
  const StageArgs* args = b->d_args + (size_t)row * n;
  BatchLaunch Ln{args, b->d_wnodes, b->nwnodes, persistent_grid(b, b->occ_nodes, b->nwnodes),
                 b->tile, b->mixed, nullptr};
  Ln.dt = cfl > 0.0;
  BHIP(b, launch_nodes_batch(Ln, s));
  if (cfl > 0.0) hipLaunchKernelGGL(k_batch_dt_final, dim3(n), dim3(256), 0, s, b->d_mem, cfl);
  BatchLaunch Lf{args, b->d_wfaces, b->nwfaces, persistent_grid(b, b->occ_faces, b->nwfaces),
                 b->tile, b->mixed, nullptr};
  BHIP(b, launch_stage_batch(Lf, s));
  return LES_OK;
}

// One Runge-Kutta step of every member on stream s (no host synchronisation).
int enqueue_step(les_batch* b, double cfl, double dt_fixed, hipStream_t s) {
  const int n = (int)b->m.size();
  // no more blocks than are resident at once: a block beyond them would start its items only
  // after a resident block had finished all of its own
  const int small = persistent_grid(b, b->occ_bc, b->nwbc);
  if (!(cfl > 0.0))
    hipLaunchKernelGGL(k_batch_set_dt, dim3((n + 63) / 64), dim3(64), 0, s, b->d_mem, n, dt_fixed);
  int rc = check_launch(b, "batch time step");
  if (rc) return rc;
  for (int l = 0; l < 5; ++l) {
    rc = enqueue_stage_kernels(b, l, s, l == 0 ? cfl : 0.0);
    if (rc) return rc;
    if (b->nwbc) {
      const StageArgs* row = b->d_args + (size_t)l * n;
      hipLaunchKernelGGL(k_batch_bc, dim3(small), dim3(256), 0, s, row, b->d_mem, b->d_wbc,
                         b->nwbc);
      rc = check_launch(b, "batch boundary conditions");
      if (rc) return rc;
    }
  }
  return LES_OK;
}

int capture_step(les_batch* b, double cfl, double dt_fixed) {
  drop_graph(b);
  if (!b->cap) BHIP(b, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  BHIP(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  int rc = enqueue_step(b, cfl, dt_fixed, b->cap);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return bfail(b, LES_EHIP, std::string("capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->exec = nullptr;
    return bfail(b, LES_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
  }
  b->graph_cfl = cfl;
  b->graph_dt = dt_fixed;
  return LES_OK;
}

}  // namespace

extern "C" {

int les_batch_create(les_ctx* const* members, int n, les_batch** out) {
  if (!out) return LES_EINVAL;
  *out = nullptr;
  if (!members || n < 1) return LES_EINVAL;
  les_batch* b = new (std::nothrow) les_batch();
  if (!b) return LES_ENOMEM;
  for (int i = 0; i < n; ++i) {
    if (!members[i]) {
      delete b;
      return LES_EINVAL;
    }
    for (int j = 0; j < i; ++j)
      if (members[j] == members[i]) {
        delete b;
        return LES_EINVAL;
      }
    b->m.push_back(members[i]);
  }
  b->mixed = members[0]->params.precision == LES_MIXED;
  for (les_ctx* c : b->m)
    if ((c->params.precision == LES_MIXED) != b->mixed || c->device != members[0]->device ||
        c->params.closure != LES_SMAGORINSKY) {
      delete b;
      return LES_EINVAL;
    }
  b->tile = members[0]->tile;
  b->kmin = members[0]->kmin;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, members[0]->device) ==
          hipSuccess &&
      cus > 0)
    b->cus = cus;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batch_bc, 256, 0) == hipSuccess &&
      occ > 0)
    b->occ_bc = occ;
  int rc = build_static_work(b);
  if (!rc) rc = build_face_work(b);
  if (!rc && hipMalloc((void**)&b->d_args, (size_t)kRows * n * sizeof(StageArgs)) != hipSuccess)
    rc = LES_ENOMEM;
  if (!rc && hipMalloc((void**)&b->d_dts, n * sizeof(double)) != hipSuccess) rc = LES_ENOMEM;
  if (!rc && hipMalloc((void**)&b->d_flags, n * sizeof(int)) != hipSuccess) rc = LES_ENOMEM;
  if (rc) {
    *out = b;  // the caller may read les_batch_last_error, then destroys it
    return rc;
  }
  *out = b;
  return LES_OK;
}

int les_batch_set_tuning(les_batch* b, int tile, int kmin) {
  if (!b) return LES_EINVAL;
  if (tile < 0 || tile >= kNumTiles || kmin < 1) return bfail(b, LES_EINVAL, "bad tuning");
  if (tile == b->tile && kmin == b->kmin) return LES_OK;
  b->tile = tile;
  b->kmin = kmin;
  drop_graph(b);
  return build_face_work(b);
}

int les_batch_get_tuning(const les_batch* b, int* tile, int* kmin) {
  if (!b || !tile || !kmin) return LES_EINVAL;
  *tile = b->tile;
  *kmin = b->kmin;
  return LES_OK;
}

int les_batch_set_graph(les_batch* b, int enable) {
  if (!b) return LES_EINVAL;
  b->use_graph = enable != 0;
  if (!b->use_graph) drop_graph(b);
  return LES_OK;
}

int les_batch_step(les_batch* b, double* const* q, int nsteps, double cfl, double dt_fixed,
                   double* dt_last, void* stream) {
  if (!b || !q || nsteps < 0) return bfail(b, LES_EINVAL, "bad argument");
  if (!(cfl > 0.0) && !(dt_fixed > 0.0)) return bfail(b, LES_EINVAL, "need cfl > 0 or dt_fixed > 0");
  const int n = (int)b->m.size();
  for (int i = 0; i < n; ++i)
    if (!q[i]) return bfail(b, LES_EINVAL, "null member state");
  hipStream_t s = (hipStream_t)stream;
  int rc = bake_args(b, q);
  if (rc) return rc;
  if (!(cfl > 0.0)) cfl = 0.0;
  hipLaunchKernelGGL(k_batch_clear_flags, dim3((n + 63) / 64), dim3(64), 0, s, b->d_mem, n);
  if (b->use_graph && nsteps > 0) {
    if (!b->exec || b->graph_cfl != cfl || (cfl == 0.0 && b->graph_dt != dt_fixed)) {
      rc = capture_step(b, cfl, dt_fixed);
      if (rc) return rc;
    }
    for (int t = 0; t < nsteps; ++t) BHIP(b, hipGraphLaunch(b->exec, s));
  } else {
    for (int t = 0; t < nsteps; ++t) {
      rc = enqueue_step(b, cfl, dt_fixed, s);
      if (rc) return rc;
    }
  }
  const StageArgs* row0 = b->d_args;
  hipLaunchKernelGGL(k_batch_check, dim3(persistent_grid(b, 4, b->nwcheck)), dim3(64, 4), 0, s,
                     row0, b->d_mem, b->d_wcheck, b->nwcheck);
  hipLaunchKernelGGL(k_batch_gather, dim3((n + 63) / 64), dim3(64), 0, s, b->d_mem, n, b->d_dts,
                     b->d_flags);
  rc = check_launch(b, "batch check");
  if (rc) return rc;
  std::vector<double> dts(n);
  std::vector<int> flags(n);
  BHIP(b, hipMemcpyAsync(dts.data(), b->d_dts, n * sizeof(double), hipMemcpyDeviceToHost, s));
  BHIP(b, hipMemcpyAsync(flags.data(), b->d_flags, n * sizeof(int), hipMemcpyDeviceToHost, s));
  BHIP(b, hipStreamSynchronize(s));
  if (dt_last)
    for (int i = 0; i < n; ++i) dt_last[i] = dts[i];
  std::string bad;
  for (int i = 0; i < n; ++i)
    if (flags[i]) bad += (bad.empty() ? "" : ", ") + std::to_string(i);
  if (!bad.empty())
    return bfail(b, LES_ENONFINITE,
                 "non-finite value or non-positive density/pressure in member(s) " + bad);
  return LES_OK;
}

int les_batch_autotune(les_batch* b, double* const* q, int* tile_out, int* kmin_out,
                       void* stream) {
  if (!b || !q) return LES_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int rc = bake_args(b, q);
  if (rc) return rc;
  static const int kmins[] = {4, 8, 16};
  const int n = (int)b->m.size();
  drop_graph(b);  // the candidates replace the work list a captured step refers to
  hipEvent_t e0, e1;
  BHIP(b, hipEventCreate(&e0));
  BHIP(b, hipEventCreate(&e1));
  float best = INFINITY;
  int bt = b->tile, bk = b->kmin;
  // Each candidate runs the first two stages of a step (node and stage kernels): they read
  // q and write only the context buffers qa and qb, with dt = 0.
  hipLaunchKernelGGL(k_batch_set_dt, dim3((n + 63) / 64), dim3(64), 0, s, b->d_mem, n, 0.0);
  rc = check_launch(b, "autotune");
  for (int t = 0; !rc && t < kNumTiles; ++t)
    for (int km : kmins) {
      b->tile = t;
      b->kmin = km;
      rc = build_face_work(b);
      if (rc) break;
      float ms = INFINITY;
      for (int rep = 0; rep < 4 && !rc; ++rep) {
        if (hipEventRecord(e0, s) != hipSuccess) rc = LES_EHIP;
        for (int l = 0; l < 2 && !rc; ++l) rc = enqueue_stage_kernels(b, l, s);
        if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = LES_EHIP;
        if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = LES_EHIP;
        float x = 0.f;
        if (!rc && hipEventElapsedTime(&x, e0, e1) != hipSuccess) rc = LES_EHIP;
        if (rep > 0) ms = std::min(ms, x);  // the first run warms the caches
      }
      if (!rc && ms < best) {
        best = ms;
        bt = t;
        bk = km;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return bfail(b, LES_EHIP, "autotune launch failed");
  b->tile = -1;  // force the work list rebuild
  rc = les_batch_set_tuning(b, bt, bk);
  if (rc) return rc;
  if (tile_out) *tile_out = bt;
  if (kmin_out) *kmin_out = bk;
  return LES_OK;
}

void les_batch_destroy(les_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  drop_graph(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  void* ptrs[] = {b->d_args, b->d_mem, b->d_wnodes, b->d_wcheck, b->d_wfaces,
                  b->d_wbc,   b->d_dts,  b->d_flags};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete b;
}

const char* les_batch_last_error(const les_batch* b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
