// Runge-Kutta stage kernels of the LES residual (gfx950).
//
// A stage is two launches:
//  * k_nodes_tile: one thread per (i, j) column marches a chunk of z-planes and writes each
//    node's record (eddy viscosity, scaled spectral radii, pressure sensors and the centred
//    zeta differences of u, v, w, T); the in-plane neighbours come from an LDS tile.
//  * k_stage_planes: one block per column tile marches through a chunk of z-planes, stages
//    each plane's node data in LDS (forming the primitive variables and the molecular
//    viscosity from the state), computes every face flux of the plane once (paper, Spatial
//    Discretization), and each node sums its six face fluxes and either writes the
//    residual or applies the Runge-Kutta stage update (paper, Time Marching Method).
// Both run in FP64, or with FP32 face arithmetic in the mixed form.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "les_common.h"
#include "les_mlp.h"
#include "les_mlp_infer.h"
#include "les_stage.h"

namespace lesmi {

namespace {

// Wrap index m along a direction of n nodes if periodic; -1 when outside a non-periodic
// range.
__device__ __forceinline__ int wrap_or_out(int m, int n, int per) {
  if (m >= 0 && m < n) return m;
  if (!per) return -1;
  return m < 0 ? m + n : m - n;
}

__device__ __forceinline__ int off3(const Dims& D, int i, int j, int k) {
  return i + D.n[0] * (j + D.n[1] * k);
}

// ---------------------------------------------------------------------------------------
// Node records.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ Prim load_prim(const double* __restrict__ q, int N, int o,
                                          const Phys& P) {
  return prim_from_q(q[o], q[N + o], q[2 * N + o], q[3 * N + o], q[4 * N + o], P);
}

template <typename R>
__device__ __forceinline__ const R* metrics_of(const StageArgs& A);
template <>
__device__ __forceinline__ const double* metrics_of<double>(const StageArgs& A) { return A.S; }
template <>
__device__ __forceinline__ const float* metrics_of<float>(const StageArgs& A) { return A.S32; }
template <typename R>
__device__ __forceinline__ R* records_of(const StageArgs& A);
template <>
__device__ __forceinline__ double* records_of<double>(const StageArgs& A) { return A.rec; }
template <>
__device__ __forceinline__ float* records_of<float>(const StageArgs& A) { return A.rec32; }

// Face inputs formed from the state at one node: the dissipated vector W (less W_ref), p -
// p_ref, u, v, w, T and the molecular viscosity, each rounded to R from the FP64 primitive
// variables (the node kernel works from the same FP64 values).
template <typename R>
struct NodeState {
  R W[5], prel, f[4], mu;
};

template <typename R>
__device__ __forceinline__ NodeState<R> node_state(const StageArgs& A, unsigned o) {
  const int N = (int)A.D.N;
  const double* __restrict__ q = A.q;
  const double q0 = q[o], q1 = q[N + o], q2 = q[2 * N + o], q3 = q[3 * N + o],
               q4 = q[4 * N + o];
  const Prim s = prim_from_q(q0, q1, q2, q3, q4, A.P);
  NodeState<R> n;
  n.prel = (R)(s.p - A.P.p_ref);
  const double qc[5] = {q0, q1, q2, q3, q4};
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    double w = qc[c];
    if (c == 4) w += (double)n.prel + A.P.p_ref;
    if constexpr (sizeof(R) == sizeof(float)) w -= A.P.wref[c];
    n.W[c] = (R)w;
  }
  n.f[0] = (R)s.u;
  n.f[1] = (R)s.v;
  n.f[2] = (R)s.w;
  n.f[3] = (R)s.T;
  n.mu = sutherland<R>(n.f[3], PhysT<R>(A.P));
  return n;
}

// Node record of node (i, j, k). Primitive variables are formed in FP64 from the FP64
// state; the differences, eddy viscosity, spectral radii and sensors are evaluated in R.
// With kQueue the primitive variables of the node and of its zeta neighbours (periodic
// zeta) are given by the caller (zm, z0, zp); otherwise they are loaded here.
// With nl non-null, the centred xi and eta neighbours' u, v, w, p come from a plane tile in
// LDS: nl[f * kNodeTileN + npos +- 1] along xi and +- kNodeTileX along eta (f = u, v, w, p).
constexpr int kNodeTileX = 66, kNodeTileY = 6, kNodeTileN = kNodeTileX * kNodeTileY;

// With mlp_in non-null the eddy-viscosity record is left to the caller and the closure's
// inputs come back in mlp_in[0..5], its scale rho Delta^2 |S| in mlp_in[6] (as FP32, the
// values the inference kernel would read).
template <typename R, bool kQueue, bool kTau = false>
__device__ __forceinline__ void node_record(const StageArgs& A, int i, int j, int k,
                                            const Prim& zm, const Prim& z0, const Prim& zp,
                                            const R* nl = nullptr, int npos = 0,
                                            double* rdt = nullptr, float* mlp_in = nullptr) {
  const Dims& D = A.D;
  const PhysT<R> P(A.P);
  const int N = (int)D.N;
  const double* __restrict__ q = A.q;
  const R* __restrict__ Sm = metrics_of<R>(A);
  int ix[3] = {i, j, k};
  int o = off3(D, i, j, k);
  Prim s = kQueue ? z0 : load_prim(q, N, o, A.P);
  const R su = (R)s.u, sv = (R)s.v, sw = (R)s.w, sp = (R)s.p;
  // Velocity differences delta_e u_m (centred; one-sided at the ends of a non-periodic
  // direction) and pressure sensors along e.
  R du[3][3];
  R nu[3];
  R dzT = (R)0;  // centred zeta difference of T (zeta is periodic)
  for (int e = 0; e < 3; ++e) {
    int n = D.n[e], m = ix[e];
    int stride = e == 0 ? 1 : (e == 1 ? D.n[0] : D.n[0] * D.n[1]);
    bool interior = D.per[e] || (m > 0 && m < n - 1);
    if (kQueue && e == 2) {
      du[e][0] = (R)0.5 * ((R)zp.u - (R)zm.u);
      du[e][1] = (R)0.5 * ((R)zp.v - (R)zm.v);
      du[e][2] = (R)0.5 * ((R)zp.w - (R)zm.w);
      dzT = (R)0.5 * ((R)zp.T - (R)zm.T);
      nu[e] = sensor<R>((R)zm.p, sp, (R)zp.p);
    } else if (interior && nl && e < 2) {
      const int st = e == 0 ? 1 : kNodeTileX;
      const R* a = nl + npos + st;
      const R* b = nl + npos - st;
      du[e][0] = (R)0.5 * (a[0] - b[0]);
      du[e][1] = (R)0.5 * (a[kNodeTileN] - b[kNodeTileN]);
      du[e][2] = (R)0.5 * (a[2 * kNodeTileN] - b[2 * kNodeTileN]);
      nu[e] = sensor<R>(b[3 * kNodeTileN], sp, a[3 * kNodeTileN]);
    } else if (interior) {
      int mp = m + 1 == n ? 0 : m + 1, mm = m == 0 ? n - 1 : m - 1;
      Prim a = load_prim(q, N, o + (mp - m) * stride, A.P);
      Prim b = load_prim(q, N, o + (mm - m) * stride, A.P);
      du[e][0] = (R)0.5 * ((R)a.u - (R)b.u);
      du[e][1] = (R)0.5 * ((R)a.v - (R)b.v);
      du[e][2] = (R)0.5 * ((R)a.w - (R)b.w);
      if (e == 2) dzT = (R)0.5 * ((R)a.T - (R)b.T);
      nu[e] = sensor<R>((R)b.p, sp, (R)a.p);
    } else {
      int sg = m == 0 ? 1 : -1;  // towards the interior
      Prim a = load_prim(q, N, o + sg * stride, A.P);
      Prim b = load_prim(q, N, o + 2 * sg * stride, A.P);
      R h = (R)0.5 * (R)sg;
      du[e][0] = h * ((R)-3 * su + (R)4 * (R)a.u - (R)b.u);
      du[e][1] = h * ((R)-3 * sv + (R)4 * (R)a.v - (R)b.v);
      du[e][2] = h * ((R)-3 * sw + (R)4 * (R)a.w - (R)b.w);
      // The boundary node takes the sensor of its interior neighbour c (p at c-1, c, c+1).
      nu[e] = m == 0 ? sensor<R>(sp, (R)a.p, (R)b.p) : sensor<R>((R)b.p, (R)a.p, sp);
    }
  }
  R sm[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) sm[c] = Sm[c * N + o];
  const R jinv = (R)A.jinv[o];
  const R T = (R)s.T;
  const R mut = smagorinsky<R>(sm, du, (R)s.rho, jinv, P);
  const R a = sqrt(T);
  const R l0 = spectral<R>(sm[0], sm[1], sm[2], su, sv, sw, a);
  const R l1 = spectral<R>(sm[3], sm[4], sm[5], su, sv, sw, a);
  const R l2 = spectral<R>(sm[6], sm[7], sm[8], su, sv, sw, a);
  const bool upd = is_updated(D, i, j, k);
  if ((rdt && upd) || kTau) {
    // The node's term of the time-step reduction, or its local pseudo-time step: the sum of
    // the spectral radii in FP64 (from the FP64 metrics in the mixed form), the same
    // operations on the same values as the separate FP64 passes.
    double l;
    if constexpr (sizeof(R) == sizeof(double)) {
      l = l0 + l1 + l2;
    } else {
      const double* __restrict__ S64 = A.S;
      const double a64 = sqrt(s.T);
      l = spectral(S64[o], S64[N + o], S64[2 * N + o], s.u, s.v, s.w, a64) +
          spectral(S64[3 * N + o], S64[4 * N + o], S64[5 * N + o], s.u, s.v, s.w, a64) +
          spectral(S64[6 * N + o], S64[7 * N + o], S64[8 * N + o], s.u, s.v, s.w, a64);
    }
    if (rdt && upd) {
      const double r = A.jinv[o] / l;
      if (!(s.rho > 0.0) || !(s.p > 0.0) || !isfinite(r)) atomicOr(A.flag, 2);
      *rdt = fmin(*rdt, r);
    }
    if (kTau) A.dtau_out[o] = upd ? A.cfl_tau * A.jinv[o] / l : 0.0;
  }
  R lb[3];
  scaled_radii<R>(l0, l1, l2, lb);
  R* __restrict__ r = records_of<R>(A);
  if (!mlp_in) r[kRecMut * N + o] = mut;
  r[(kRecLb + 0) * N + o] = lb[0];
  r[(kRecLb + 1) * N + o] = lb[1];
  r[(kRecLb + 2) * N + o] = lb[2];
  r[(kRecNu + 0) * N + o] = nu[0];
  r[(kRecNu + 1) * N + o] = nu[1];
  r[(kRecNu + 2) * N + o] = nu[2];
  r[(kRecDz + 0) * N + o] = du[2][0];
  r[(kRecDz + 1) * N + o] = du[2][1];
  r[(kRecDz + 2) * N + o] = du[2][2];
  r[(kRecDz + 3) * N + o] = dzT;
  if (mlp_in) {  // inputs of the learned closure, kept in registers
    R g[3][3], f[kMlpIn];
    velocity_gradient<R>(sm, du, jinv, g);
    const R smag = mlp_invariants<R>(g, f);
#pragma unroll
    for (int c = 0; c < kMlpIn; ++c) mlp_in[c] = (float)f[c];
    const R dl = jinv > (R)0 ? cbrt(jinv) : (R)0;
    mlp_in[kMlpIn] = (float)((R)s.rho * dl * dl * smag);
    return;
  }
  if (A.mut_out) A.mut_out[o] = (double)mut;
  if (A.feat || A.fscale || A.fsmag) {  // inputs of the learned closure
    R g[3][3], f[kMlpIn];
    velocity_gradient<R>(sm, du, jinv, g);
    const R smag = mlp_invariants<R>(g, f);
    if (A.feat)
#pragma unroll
      for (int c = 0; c < kMlpIn; ++c) A.feat[c * N + o] = (float)f[c];
    const R dl = jinv > (R)0 ? cbrt(jinv) : (R)0;
    if (A.fscale) A.fscale[o] = (float)((R)s.rho * dl * dl * smag);
    if (A.fsmag) A.fsmag[o] = (float)smag;
  }
}

// Node records of the 64 x 4 column tile (bx, by) over the z-planes kbeg .. kend-1 (zeta
// periodic), one thread per (i, j) column in 64 x 4 blocks. The primitive variables of
// planes k-1, k, k+1 of the own column stay in registers; per plane, each thread stages its
// node's u, v, w, p in the LDS tile Lp and threads 0..135 those of the tile's one-node ring,
// so the centred xi and eta differences read the tile and each node's primitive variables
// are formed about 1.5 times per plane. One-sided differences at the ends of a non-periodic
// direction read global memory.
// LDS of the learned closure evaluated in the node kernel: per-lane weight fragments, the
// biases and output weights (b1, b2, w3, b3), and each wave's split h1 rows.
struct NodeMlpLds {
  bf16x8 F[kInferFrags * 64];
  float bs[196];
  __bf16 H[4][16 * HS];
  __bf16 Hl[4][16 * HS];
};

template <typename R, bool kDt = false, bool kMlp = false, bool kTau = false>
__device__ __forceinline__ void nodes_tile_block(const StageArgs& A, int bx, int by, int kbeg,
                                                 int kend, R* Lp, int slot = 0,
                                                 NodeMlpLds* ML = nullptr) {
  const Dims& D = A.D;
  const int ni = D.n[0], nj = D.n[1], nk = D.n[2], N = (int)D.N;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + 64 * ty;
  const int i0 = bx * 64, j0 = by * 4;
  const int i = i0 + tx, j = j0 + ty;
  const bool mine = i < ni && j < nj;
  const int pl = ni * nj;
  // Ring slot of this thread (threads 0..135): rows j0 - 1 and j0 + 4, then columns i0 - 1
  // and i0 + 64. A thread whose own node lies past the end of a periodic direction stages
  // the wrapped node in its own slot instead (ragged tiles).
  int hpos = -1, ho = -1;
  if (tid < 136) {
    int hx, hy;
    if (tid < 64) { hx = tid + 1; hy = 0; }
    else if (tid < 128) { hx = tid - 63; hy = kNodeTileY - 1; }
    else if (tid < 132) { hx = 0; hy = tid - 127; }
    else { hx = kNodeTileX - 1; hy = tid - 131; }
    const int ia = wrap_or_out(i0 - 1 + hx, ni, D.per[0]);
    const int ja = wrap_or_out(j0 - 1 + hy, nj, D.per[1]);
    if (ia >= 0 && ja >= 0) {
      hpos = hx + kNodeTileX * hy;
      ho = ia + ni * ja;
    }
  }
  const int own = (tx + 1) + kNodeTileX * (ty + 1);
  int wo = -1;  // wrapped node staged in the own slot by a thread outside the grid
  if (!mine) {
    const bool oki = i < ni || D.per[0], okj = j < nj || D.per[1];
    if (oki && okj) wo = (i % ni) + ni * (j % nj);
  }
  const int o0 = i + ni * j;
  double rdt = INFINITY;  // this column's minimum of the time-step reduction
  unsigned nfb = 0;       // closure nodes of this thread that fell back to C_s^2
  Prim zm{}, z0{};
  if (mine) {
    zm = load_prim(A.q, N, o0 + pl * (kbeg == 0 ? nk - 1 : kbeg - 1), A.P);
    z0 = load_prim(A.q, N, o0 + pl * kbeg, A.P);
  }
  for (int k = kbeg; k < kend; ++k) {
    Prim zp{}, h{}, w{};
    if (mine) zp = load_prim(A.q, N, o0 + pl * (k + 1 == nk ? 0 : k + 1), A.P);
    if (ho >= 0) h = load_prim(A.q, N, ho + pl * k, A.P);
    if (wo >= 0) w = load_prim(A.q, N, wo + pl * k, A.P);
    __syncthreads();  // the previous plane's tile has been read
    if (mine) {
      Lp[own] = (R)z0.u;
      Lp[kNodeTileN + own] = (R)z0.v;
      Lp[2 * kNodeTileN + own] = (R)z0.w;
      Lp[3 * kNodeTileN + own] = (R)z0.p;
    } else if (wo >= 0) {
      Lp[own] = (R)w.u;
      Lp[kNodeTileN + own] = (R)w.v;
      Lp[2 * kNodeTileN + own] = (R)w.w;
      Lp[3 * kNodeTileN + own] = (R)w.p;
    }
    if (ho >= 0) {
      Lp[hpos] = (R)h.u;
      Lp[kNodeTileN + hpos] = (R)h.v;
      Lp[2 * kNodeTileN + hpos] = (R)h.w;
      Lp[3 * kNodeTileN + hpos] = (R)h.p;
    }
    __syncthreads();
    // Indices pass through an empty asm statement: their derived addresses are formed on
    // each plane instead of holding registers across the loop.
    int il = i, jl = j, ol = own;
    asm volatile("" : "+v"(il), "+v"(jl), "+v"(ol));
    if constexpr (kMlp) {
      // The wave's 64 nodes of this plane (one row of the tile) are the 64 samples of one
      // inference pass, in the order and arithmetic of the inference kernel; lanes without
      // a node take part with zero inputs and write nothing.
      float fin[kMlpIn + 1];
#pragma unroll
      for (int c = 0; c <= kMlpIn; ++c) fin[c] = 0.f;
      if (mine)
        node_record<R, true, kTau>(A, il, jl, k, zm, z0, zp, Lp, ol, kDt ? &rdt : nullptr,
                                   fin);
      float x[kMlpIn];
      const bool ok = mlp_input(A.mlp, fin, fin[kMlpIn], x);
      const int lane = tx, g = lane >> 4, sl = lane & 15;
      float zmine = 0.f;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        float xs[kMlpIn];
#pragma unroll
        for (int c = 0; c < kMlpIn; ++c) xs[c] = __shfl(x[c], sl + 16 * t);
        const float z = forward16_split_lds(ML->bs, ML->F, xs, lane, ML->H[ty], ML->Hl[ty]);
        if (g == t) zmine = z;
      }
      if (mine) {
        const float cc = ok ? softplus_f(zmine) : A.mlp.cs2;
        nfb += ok ? 0u : 1u;
        const double mu = (double)fin[kMlpIn] * (double)cc;
        records_of<R>(A)[kRecMut * N + (il + ni * (jl + nj * k))] = (R)mu;
      }
    } else {
      if (mine)
        node_record<R, true, kTau>(A, il, jl, k, zm, z0, zp, Lp, ol, kDt ? &rdt : nullptr);
    }
    zm = z0;
    z0 = zp;
  }
  if constexpr (kMlp) {  // the wave's fallback count
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) nfb += __shfl_xor(nfb, o);
    if (tx == 0 && nfb && A.mlp_fallback) atomicAdd(A.mlp_fallback, nfb);
  }
  if constexpr (kDt) {  // the block's minimum (the tile is free now)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) rdt = fmin(rdt, __shfl_xor(rdt, o));
    __syncthreads();
    double* red = (double*)Lp;
    if ((tid & 63) == 0) red[tid >> 6] = rdt;
    __syncthreads();
    if (tid == 0) A.dtpart[slot] = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
  }
}

// kDt: also the time-step reduction's block minima (A.dtpart); kTau: also the local
// pseudo-time steps (A.dtau_out).
template <typename R, bool kDt = false, bool kTau = false>
__global__ void __launch_bounds__(256) k_nodes_tile(StageArgs A, int kchunk) {
  __shared__ R Lp[4 * kNodeTileN];
  const int kbeg = blockIdx.z * kchunk;
  nodes_tile_block<R, kDt, false, kTau>(
      A, blockIdx.x, blockIdx.y, kbeg, min(kbeg + kchunk, A.D.n[2]), Lp,
      blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z));
}

// The same with the learned closure evaluated for each plane's nodes (StageArgs.mlp_fused):
// the block first lays the network's weight fragments into LDS.
template <typename R, bool kDt = false, bool kTau = false>
__global__ void __launch_bounds__(256) k_nodes_tile_mlp(StageArgs A, int kchunk) {
  __shared__ R Lp[4 * kNodeTileN];
  __shared__ NodeMlpLds ML;
  const float* __restrict__ th = A.mlp.theta;
  infer_frags_to_lds(th, ML.F, threadIdx.y, 4, threadIdx.x);
  const int t = threadIdx.x + 64 * threadIdx.y;
  if (t < 64) {
    ML.bs[t] = th[kOffB1 + t];
    ML.bs[64 + t] = th[kOffB2 + t];
    ML.bs[128 + t] = th[kOffW3 + t];
  } else if (t == 64) {
    ML.bs[192] = th[kOffB3];
  }
  __syncthreads();
  const int kbeg = blockIdx.z * kchunk;
  nodes_tile_block<R, kDt, true, kTau>(
      A, blockIdx.x, blockIdx.y, kbeg, min(kbeg + kchunk, A.D.n[2]), Lp,
      blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), &ML);
}

// Persistent form over the members of a batch: item = (member, bx | by << 16,
// kbeg | kend << 16, slot of the member's time-step partial minima).
template <typename R, bool kDt = false>
__global__ void __launch_bounds__(256) k_nodes_tile_batch(const StageArgs* __restrict__ args,
                                                          const int4* __restrict__ work,
                                                          int nwork) {
  __shared__ R Lp[4 * kNodeTileN];
  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int4 it = work[w];
    const StageArgs A = args[it.x];
    nodes_tile_block<R, kDt>(A, it.y & 0xffff, it.y >> 16, it.z & 0xffff, it.z >> 16, Lp, it.w);
  }
}

// Maps the dispatch order onto tiles so that each XCD (blocks are dealt round-robin to the
// 8 XCDs) works on one contiguous run of tiles, whose shared halo data then stays in that
// XCD's L2.
__device__ __forceinline__ int xcd_tile(int lin, int nblk) {
  const int full = (nblk / 8) * 8;
  if (lin >= full) return lin;
  return (lin % 8) * (full / 8) + lin / 8;
}

// ---------------------------------------------------------------------------------------
// Plane-staged stage kernel. One block per TX x TY column tile marches through a chunk of
// z-planes. Each plane's node data is loaded once into LDS (the dissipated vector over a
// two-node ring, the other face inputs over a one-node ring); the xi and eta faces of the
// plane are computed from LDS, the zeta face from the column's previous-plane values kept
// in registers. For every face an updated node uses, the tangential differences are
// centred (their nodes never lie on a non-periodic end in a tangential direction), so they
// are taken straight from the ring.
// ---------------------------------------------------------------------------------------
enum { sU = 0, sV, sWv, sT, sMu, sMut, sS0, sJinv = sS0 + 9, sDz, sNF = sDz + 4 };

template <int TX, int TY, typename R>
struct PlaneLds {
  static constexpr int RX2 = TX + 4, RY2 = TY + 4, RX1 = TX + 2, RY1 = TY + 2;
  static constexpr int NW = RX2 * RY2, N1 = RX1 * RY1;
  static constexpr int NX = (TX + 1) * TY, NY = TX * (TY + 1);
  // Staging of one plane. Once its faces are computed the same space holds the face
  // fluxes (xi then eta), 5 * (NX + NY) values.
  union {
    struct {
      R W[6][NW];    // W0..W4 and p over the two-node ring
      R F[sNF][N1];  // other face inputs over the one-node ring
      R DX[2][(TX + 2) * TY];  // scaled spectral radius and sensor along xi, xi-face nodes
      R DY[2][TX * (TY + 2)];  // the same along eta, eta-face nodes
    } in;
    R H[5][NX + NY];
  };
};

// Face inputs of a node staged in LDS, read at the point of use. Tangential differences
// are centred in-plane and staged along zeta; lb/nu along d are given by the caller (staged
// in LDS for xi and eta faces, prefetched into registers for zeta faces).
template <int TX, int TY, int d, typename R>
struct LdsNode {
  using PL = PlaneLds<TX, TY, R>;
  const PL& L;
  int p1, p2;
  R lb_, nu_;
  __device__ R W(int c) const { return L.in.W[c][p2]; }
  __device__ R p() const { return L.in.W[5][p2]; }
  __device__ R f(int v) const { return L.in.F[sU + v][p1]; }  // u, v, w, T
  __device__ R mu() const { return L.in.F[sMu][p1]; }
  __device__ R mut() const { return L.in.F[sMut][p1]; }
  __device__ R S(int c) const { return L.in.F[sS0 + c][p1]; }
  __device__ R jinv() const { return L.in.F[sJinv][p1]; }
  __device__ R lb() const { return lb_; }
  __device__ R nu() const { return nu_; }
  // Difference along the e-th tangential direction (in increasing direction order).
  __device__ R dt(int e, int v) const {
    const int dir = e == 0 ? (d == 0 ? 1 : 0) : (d == 2 ? 1 : 2);
    if (dir == 0) return (R)0.5 * (L.in.F[sU + v][p1 + 1] - L.in.F[sU + v][p1 - 1]);
    if (dir == 1) return (R)0.5 * (L.in.F[sU + v][p1 + PL::RX1] - L.in.F[sU + v][p1 - PL::RX1]);
    return L.in.F[sDz + v][p1];
  }
};

// Face inputs of node (i, j, k) from global memory (the zeta faces at the ends of a chunk):
// the state-derived inputs are formed from the state as in the staging, the others read
// from the records, metrics and J^-1; xi and eta differences are centred.
template <typename R>
struct GlobalNodeZ {
  const StageArgs& A;
  unsigned o, ip, im, jp, jm;
  int N;
  const R* __restrict__ rec;
  const R* __restrict__ Sm;
  NodeState<R> n;
  __device__ GlobalNodeZ(const StageArgs& A_, int i, int j, int k)
      : A(A_), N((int)A_.D.N), rec(records_of<R>(A_)), Sm(metrics_of<R>(A_)) {
    const int ni = A.D.n[0], nj = A.D.n[1];
    o = (unsigned)(i + ni * (j + nj * k));
    ip = i + 1 == ni ? o - (unsigned)(ni - 1) : o + 1;
    im = i == 0 ? o + (unsigned)(ni - 1) : o - 1;
    jp = j + 1 == nj ? o - (unsigned)((nj - 1) * ni) : o + ni;
    jm = j == 0 ? o + (unsigned)((nj - 1) * ni) : o - ni;
    n = node_state<R>(A, o);
  }
  __device__ R p() const { return n.prel; }
  __device__ R W(int c) const { return n.W[c]; }
  __device__ R f(int v) const { return n.f[v]; }
  __device__ R mu() const { return n.mu; }
  __device__ R mut() const { return rec[kRecMut * N + o]; }
  __device__ R S(int c) const { return Sm[c * N + o]; }
  __device__ R jinv() const { return (R)A.jinv[o]; }
  __device__ R lb() const { return rec[(kRecLb + 2) * N + o]; }
  __device__ R nu() const { return rec[(kRecNu + 2) * N + o]; }
  __device__ R dt(int e, int v) const {
    const NodeState<R> a = node_state<R>(A, e == 0 ? ip : jp);
    const NodeState<R> b = node_state<R>(A, e == 0 ? im : jm);
    return (R)0.5 * (a.f[v] - b.f[v]);
  }
};

// Face inputs of one node held in registers: the lower node of a zeta face, taken from
// LDS while its own plane is staged and used when the plane above is staged. With kMetRegs
// false the metrics and J^-1 are read again from global memory at the point of use (FP64,
// where registers are short).
template <typename R, bool kMetRegs>
struct RegNode {
  R w[5], pp, fv[4], mu_, mut_, s[kMetRegs ? 9 : 1], ji, d[2][4], lb_, nu_;
  const R* Sm;
  const double* jg;
  unsigned o;
  int N;
  __device__ R W(int c) const { return w[c]; }
  __device__ R p() const { return pp; }
  __device__ R f(int v) const { return fv[v]; }
  __device__ R mu() const { return mu_; }
  __device__ R mut() const { return mut_; }
  __device__ R S(int c) const {
    if constexpr (kMetRegs) return s[c];
    else return Sm[c * N + o];
  }
  __device__ R jinv() const {
    if constexpr (kMetRegs) return ji;
    else return (R)jg[o];
  }
  __device__ R lb() const { return lb_; }
  __device__ R nu() const { return nu_; }
  __device__ R dt(int e, int v) const { return d[e][v]; }
  // Takes the inputs of node offset o_ from accessor n.
  template <typename NodeT>
  __device__ __forceinline__ void take(const NodeT& n, const StageArgs& A, unsigned o_) {
#pragma unroll
    for (int c = 0; c < 5; ++c) w[c] = n.W(c);
    pp = n.p();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      fv[v] = n.f(v);
      d[0][v] = n.dt(0, v);
      d[1][v] = n.dt(1, v);
    }
    mu_ = n.mu();
    mut_ = n.mut();
    if constexpr (kMetRegs) {
#pragma unroll
      for (int c = 0; c < 9; ++c) s[c] = n.S(c);
      ji = n.jinv();
    } else {
      Sm = metrics_of<R>(A);
      jg = A.jinv;
      o = o_;
      N = (int)A.D.N;
    }
    lb_ = n.lb();
    nu_ = n.nu();
  }
};

// Total numerical flux H = (F_A + F_B)/2 - D - F_v on a face along d (paper, Spatial
// Discretization: interface flux with the Turkel-Vatsa terms; viscous flux from the two
// nodes of the interface), evaluated from node accessors a (A) and b (B = A + e_d) in the
// order the oracle evaluates it. Wm = W(A - e_d), Wp = W(B + e_d); m is A's index along d.
template <int d, typename R, typename NA, typename NB>
__device__ __forceinline__ void face_eval(const NA& a, const NB& b, const R* Wm, const R* Wp,
                                          int m, int n, bool per, const PhysT<R>& Ph, R* H) {
  {  // central inviscid part
    const R una = fmadd(a.S(3 * d + 2), a.f(2), fmadd(a.S(3 * d + 1), a.f(1), a.S(3 * d) * a.f(0)));
    const R unb = fmadd(b.S(3 * d + 2), b.f(2), fmadd(b.S(3 * d + 1), b.f(1), b.S(3 * d) * b.f(0)));
    // Each node's flux is rounded on its own, identically in the node's two faces along d,
    // so that it cancels exactly from the node's flux difference.
    const R pa = a.p(), pb = b.p();
    H[0] = (R)0.5 * (a.W(0) * una + b.W(0) * unb);
#pragma unroll
    for (int c = 1; c < 4; ++c)
      H[c] = (R)0.5 * (fmadd(a.W(c), una, pa * a.S(3 * d + c - 1)) +
                       fmadd(b.W(c), unb, pb * b.S(3 * d + c - 1)));
    H[4] = (R)0.5 * (a.W(4) * una + b.W(4) * unb);
    if constexpr (sizeof(R) == sizeof(float)) {  // the W_ref part of W U
      const R us = (R)0.5 * (una + unb);
#pragma unroll
      for (int c = 0; c < 5; ++c) H[c] = fmadd(Ph.wref[c], us, H[c]);
    }
  }
  {  // artificial dissipation: H -= Lam_f (eps2 dW - eps4 d3W)
    R dW[5], d3W[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) dW[c] = b.W(c) - a.W(c);
    // The third difference is summed left to right with rounded products: it is a small
    // difference of O(1) values on smooth fields, and this order is the one whose rounding
    // the residual's cancelling components are held to.
    if (per || (m > 0 && m < n - 2)) {
#pragma unroll
      for (int c = 0; c < 5; ++c) d3W[c] = Wp[c] - (R)3 * b.W(c) + (R)3 * a.W(c) - Wm[c];
    } else if (m == 0) {
#pragma unroll
      for (int c = 0; c < 5; ++c) d3W[c] = (Wp[c] - b.W(c)) - (R)3 * dW[c];
    } else {
#pragma unroll
      for (int c = 0; c < 5; ++c) d3W[c] = (R)-3 * dW[c] + (a.W(c) - Wm[c]);
    }
    const R lf = (R)0.5 * (a.lb() + b.lb());
    R eps2, eps4;
    dissipation_coefficients<R>(a.nu(), b.nu(), Ph, &eps2, &eps4);
#pragma unroll
    for (int c = 0; c < 5; ++c) H[c] = fmadd(-lf, fmadd(eps2, dW[c], -(eps4 * d3W[c])), H[c]);
  }
  {  // viscous and subgrid part (face averages passed as sums of the two nodes' values)
    R Ss[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) Ss[c] = a.S(c) + b.S(c);
    const R js = a.jinv() + b.jinv();
    constexpr int e1 = d == 0 ? 1 : 0, e2 = d == 2 ? 1 : 2;
    R gxi[4][3];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      gxi[v][d] = b.f(v) - a.f(v);
      gxi[v][e1] = (R)0.5 * (a.dt(0, v) + b.dt(0, v));
      gxi[v][e2] = (R)0.5 * (a.dt(1, v) + b.dt(1, v));
    }
    const R mus = a.mu() + b.mu();
    const R muts = a.mut() + b.mut();
    const R ub[3] = {(R)0.5 * (a.f(0) + b.f(0)), (R)0.5 * (a.f(1) + b.f(1)),
                     (R)0.5 * (a.f(2) + b.f(2))};
    R Fv[5];
    viscous_flux<R>(Ss, js, gxi, mus, muts, ub, d, Ph, Fv);
#pragma unroll
    for (int c = 1; c < 5; ++c) H[c] = H[c] - Fv[c];
    H[0] = H[0] - (R)0;
  }
}

// Residual of node (i, j, k) from the sum of its xi and eta face differences (part) and its
// zeta faces above (hu) and below (hd): written out (mode 0) or applied as the Runge-Kutta
// stage update Q = Q0 - alpha dt J R (mode 1). Nodes that are not updated get a zero
// residual in mode 0 and are left alone in mode 1. pq and pj, when given, are the node's
// Q0 and J loaded earlier by the caller.
template <typename R, bool kDual = false>
__device__ __forceinline__ void finish_node(const StageArgs& A, int i, int j, int k,
                                            const R* part, const R* hu, const R* hd,
                                            const double* pq = nullptr, double pj = 0.0,
                                            double pt = 0.0) {
  const Dims& D = A.D;
  const int N = (int)D.N;
  const int o = i + D.n[0] * (j + D.n[1] * k);
  if constexpr (kDual) {  // mode 2; pt is the node's pseudo-time step when pq is given
    if (!is_updated(D, i, j, k)) return;
    const double J = pq ? pj : A.jac[o], dtau = pq ? pt : A.dual_dtau[o];
    const double den = 1.0 + A.alpha * dtau * A.dual_a0 / A.dual_dt;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      R rr = part[c];
      rr += hu[c] - hd[c];
      const int e = c * N + o;
      const double jr = J * (double)rr;
      const double hist = A.dual_a2 != 0.0 ? A.dual_a1 * A.dual_qn[e] + A.dual_a2 * A.dual_qm[e]
                                           : A.dual_a1 * A.dual_qn[e];
      A.out[e] = ((pq ? pq[c] : A.q0[e]) - A.alpha * dtau * (jr + hist / A.dual_dt)) / den;
    }
    return;
  }
  if (is_updated(D, i, j, k)) {
    double fac = 0.0;
    if (A.mode == 1) fac = A.alpha * A.dt[0] * (pq ? pj : A.jac[o]);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      R rr = part[c];
      rr += hu[c] - hd[c];
      if (A.mode == 0)
        A.out[c * N + o] = (double)rr;
      else
        A.out[c * N + o] = (pq ? pq[c] : A.q0[c * N + o]) - fac * (double)rr;
    }
  } else if (A.mode == 0) {
#pragma unroll
    for (int c = 0; c < 5; ++c) A.out[c * N + o] = 0.0;
  }
}

// One block per TX x TY column tile marches a chunk of z-planes (z is periodic). R is the
// arithmetic type of the fluxes (double; float in the mixed form, where the state, the
// Runge-Kutta update, J^-1 and J stay FP64).
// Column tile (bx, by) over the z-planes kbeg .. kend-1, with the block's LDS L.
// The zeta face between planes k-1 and k is evaluated while plane k is staged: its upper node
// comes from LDS and its lower node from registers (taken from LDS one plane earlier), so the
// update of the column's node on plane k-1 completes one plane late. The faces below the
// first and above the last plane of the chunk read their outer node from global memory.
template <int TX, int TY, typename R, bool kDual = false>
__device__ __forceinline__ void stage_block(const StageArgs& A, int bx, int by, int kbeg,
                                            int kend, PlaneLds<TX, TY, R>& L) {
  using PL = PlaneLds<TX, TY, R>;
  constexpr int NT = TX * TY;
  constexpr int MW = (PL::NW + NT - 1) / NT;  // staging slots per thread
  constexpr int M1 = (PL::N1 + NT - 1) / NT;
  constexpr int MX = (PL::NX + NT - 1) / NT;  // face slots per thread
  constexpr int MY = (PL::NY + NT - 1) / NT;
  constexpr int NDX = (TX + 2) * TY, NDY = TX * (TY + 2);
  constexpr int MDX = (NDX + NT - 1) / NT;  // lb/nu staging slots per thread
  constexpr int MDY = (NDY + NT - 1) / NT;
  // FP64 loads the xi/eta lb and nu with the first staging group; in the mixed form they
  // go with the second, since the first would take the kernel past 168 VGPRs (3 waves/SIMD).
  constexpr bool kDxyEarly = sizeof(R) == sizeof(double);
  // Face slots: slot 0 of thread t is face t; slot 1 holds the faces NT.. of a direction,
  // taken by the first lanes of wave WX (xi) or WY (eta). -1: no face.
  constexpr int NWAVE = NT / 64, WX = 1 % NWAVE, WY = 2 % NWAVE;
  static_assert(NT % 64 == 0 && MX == 2 && MY == 2 && PL::NX - NT <= 64 && PL::NY - NT <= 64,
                "face slot layout");
  auto xi_slot = [](int t, int r) {
    const int e = t - 64 * WX;
    return r == 0 ? t : (e >= 0 && e < PL::NX - NT ? NT + e : -1);
  };
  auto eta_slot = [](int t, int r) {
    const int e = t - 64 * WY;
    return r == 0 ? t : (e >= 0 && e < PL::NY - NT ? NT + e : -1);
  };
  const Dims& D = A.D;
  const PhysT<R> Ph(A.P);
  const int N = (int)D.N;
  const int ni = D.n[0], nj = D.n[1], nk = D.n[2];
  const int i0 = bx * TX, j0 = by * TY;
  const int tid = threadIdx.x;
  const int a = tid % TX, b = tid / TX;
  const int i = i0 + a, j = j0 + b;
  const bool mine = i < ni && j < nj;
  const R* __restrict__ rec = records_of<R>(A);
  const R* __restrict__ S = metrics_of<R>(A);

  // State of the column between planes: the zeta face below the pending node (hz_lo), the
  // pending node's xi/eta flux sum (part) and face inputs (lo), and W one plane below it.
  R hz_lo[5] = {0, 0, 0, 0, 0};
  R Wm[5] = {0, 0, 0, 0, 0};
  R part[5] = {0, 0, 0, 0, 0};
  RegNode<R, sizeof(R) == sizeof(float)> lo;
  if (mine) {  // zeta face below the chunk
    const int kl = kbeg == 0 ? nk - 1 : kbeg - 1;
    const int kl2 = kl == 0 ? nk - 1 : kl - 1;
    const GlobalNodeZ<R> na(A, i, j, kl), nb(A, i, j, kbeg);
    const int kp = kbeg + 1 == nk ? 0 : kbeg + 1;
    const unsigned om = (unsigned)(i + ni * (j + nj * kl2));
    const unsigned op = (unsigned)(i + ni * (j + nj * kp));
    const NodeState<R> sm = node_state<R>(A, om), sp = node_state<R>(A, op);
    face_eval<2, R>(na, nb, sm.W, sp.W, kl, nk, true, Ph, hz_lo);
#pragma unroll
    for (int c = 0; c < 5; ++c) Wm[c] = na.W(c);
  }

  for (int k = kbeg; k < kend; ++k) {
    const bool pending = mine && k > kbeg;  // the node on plane k-1 awaits its upper face
    // The thread index passed through an empty asm statement: the staging addresses derived
    // from it are then formed anew on each plane instead of being hoisted out of the loop
    // (where they would hold registers across the face arithmetic).
    int tl = tid;
    asm volatile("" : "+v"(tl));
    // Staging loads of slot s of the two-node ring (W and p) and of the one-node ring (the
    // other face inputs); nodes outside a non-periodic range stage zeros.
    // A slot of the two-node ring inside the one-node ring also supplies that ring's u, v,
    // w, T and molecular viscosity (v[6..10]).
    auto load_w = [&](int s, R(&v)[11]) {
      const int ia = wrap_or_out(i0 - 2 + s % PL::RX2, ni, D.per[0]);
      const int ja = wrap_or_out(j0 - 2 + s / PL::RX2, nj, D.per[1]);
#pragma unroll
      for (int c = 0; c < 11; ++c) v[c] = (R)0;
      if (s < PL::NW && ia >= 0 && ja >= 0) {
        const NodeState<R> n = node_state<R>(A, (unsigned)(ia + ni * (ja + nj * k)));
#pragma unroll
        for (int c = 0; c < 5; ++c) v[c] = n.W[c];
        v[5] = n.prel;
#pragma unroll
        for (int c = 0; c < 4; ++c) v[6 + c] = n.f[c];
        v[10] = n.mu;
      }
    };
    auto load_f = [&](int s, R(&v)[sNF]) {
      const int ia = wrap_or_out(i0 - 1 + s % PL::RX1, ni, D.per[0]);
      const int ja = wrap_or_out(j0 - 1 + s / PL::RX1, nj, D.per[1]);
#pragma unroll
      for (int c = 0; c < sNF; ++c) v[c] = (R)0;
      if (s < PL::N1 && ia >= 0 && ja >= 0) {
        const unsigned o = (unsigned)(ia + ni * (ja + nj * k));
        v[sMut] = rec[kRecMut * N + o];
#pragma unroll
        for (int c = 0; c < 9; ++c) v[sS0 + c] = S[c * N + o];
        v[sJinv] = (R)A.jinv[o];
#pragma unroll
        for (int c = 0; c < 4; ++c) v[sDz + c] = rec[(kRecDz + c) * N + o];
      }
    };
    // Scaled spectral radius and sensor of the xi- and eta-face nodes (DX, DY).
    auto load_dxy = [&](R(&vdx)[MDX][2], R(&vdy)[MDY][2]) {
#pragma unroll
      for (int r = 0; r < MDX; ++r) {
        const int s = tl + r * NT;
        const int ia = wrap_or_out(i0 - 1 + s % (TX + 2), ni, D.per[0]);
        const int ja = wrap_or_out(j0 + s / (TX + 2), nj, D.per[1]);
        vdx[r][0] = vdx[r][1] = (R)0;
        if (s < NDX && ia >= 0 && ja >= 0) {
          const unsigned o = (unsigned)(ia + ni * (ja + nj * k));
          vdx[r][0] = rec[kRecLb * N + o];
          vdx[r][1] = rec[kRecNu * N + o];
        }
      }
#pragma unroll
      for (int r = 0; r < MDY; ++r) {
        const int s = tl + r * NT;
        const int ia = wrap_or_out(i0 + s % TX, ni, D.per[0]);
        const int ja = wrap_or_out(j0 - 1 + s / TX, nj, D.per[1]);
        vdy[r][0] = vdy[r][1] = (R)0;
        if (s < NDY && ia >= 0 && ja >= 0) {
          const unsigned o = (unsigned)(ia + ni * (ja + nj * k));
          vdy[r][0] = rec[(kRecLb + 1) * N + o];
          vdy[r][1] = rec[(kRecNu + 1) * N + o];
        }
      }
    };
    auto write_dxy = [&](const R(&vdx)[MDX][2], const R(&vdy)[MDY][2]) {
#pragma unroll
      for (int r = 0; r < MDX; ++r) {
        const int s = tl + r * NT;
        if (s < NDX) {
          L.in.DX[0][s] = vdx[r][0];
          L.in.DX[1][s] = vdx[r][1];
        }
      }
#pragma unroll
      for (int r = 0; r < MDY; ++r) {
        const int s = tl + r * NT;
        if (s < NDY) {
          L.in.DY[0][s] = vdy[r][0];
          L.in.DY[1][s] = vdy[r][1];
        }
      }
    };
    // The plane is staged in two groups of loads, each written to LDS as it arrives.
    // Group 1: the two-node ring, the first slot of the one-node ring, the own node's zeta
    // spectral radius and sensor, W one plane above the own node (outer node of the
    // pending zeta face), and in FP64 the xi/eta lb and nu.
    R zl[2] = {0, 0}, wp[5] = {0, 0, 0, 0, 0};
    // Q^(0) and J of the pending node for its stage update, loaded with the staging so that
    // their latency is hidden behind it rather than exposed after the zeta face.
    double pq[5] = {0, 0, 0, 0, 0}, pj = 0.0, pt = 0.0;
    if (pending && (kDual || A.mode == 1)) {
      const unsigned o1 = (unsigned)(i + ni * (j + nj * (k - 1)));
#pragma unroll
      for (int c = 0; c < 5; ++c) pq[c] = A.q0[c * N + o1];
      pj = A.jac[o1];
      if constexpr (kDual) pt = A.dual_dtau[o1];
    }
    {
      R vw[MW][11], vf[sNF], vdx[MDX][2], vdy[MDY][2];
#pragma unroll
      for (int r = 0; r < MW; ++r) load_w(tl + r * NT, vw[r]);
      load_f(tl, vf);
      if constexpr (kDxyEarly) load_dxy(vdx, vdy);
      if (mine) {
        const unsigned o = (unsigned)(i + ni * (j + nj * k));
        zl[0] = rec[(kRecLb + 2) * N + o];
        zl[1] = rec[(kRecNu + 2) * N + o];
      }
      if (pending) {
        const int kp = k + 1 == nk ? 0 : k + 1;
        const unsigned o2 = (unsigned)(i + ni * (j + nj * kp));
#pragma unroll
        for (int c = 0; c < 5; ++c) wp[c] = node_state<R>(A, o2).W[c];
      }
#pragma unroll
      for (int r = 0; r < MW; ++r) {
        const int s = tl + r * NT;
        if (s < PL::NW)
#pragma unroll
          for (int c = 0; c < 6; ++c) L.in.W[c][s] = vw[r][c];
        const int x1 = s % PL::RX2 - 1, y1 = s / PL::RX2 - 1;  // one-node ring position
        if (s < PL::NW && x1 >= 0 && x1 < PL::RX1 && y1 >= 0 && y1 < PL::RY1)
#pragma unroll
          for (int c = 0; c < 5; ++c) L.in.F[sU + c][x1 + PL::RX1 * y1] = vw[r][6 + c];
      }
      if (tl < PL::N1)
#pragma unroll
        for (int c = sMut; c < sNF; ++c) L.in.F[c][tl] = vf[c];
      if constexpr (kDxyEarly) write_dxy(vdx, vdy);
    }
    // Group 2: the other slots of the one-node ring, and in the mixed form the xi/eta lb
    // and nu.
    {
      constexpr int M1b = M1 > 1 ? M1 - 1 : 1;
      R vf[M1b][sNF], vdx[MDX][2], vdy[MDY][2];
#pragma unroll
      // The extra one-ring slots count down from the last thread, so they land on the waves
      // that the extra two-ring slots (counting up from thread 0) leave idle.
      for (int r = 1; r < M1; ++r) load_f(r * NT + (NT - 1 - tl), vf[r - 1]);
      if constexpr (!kDxyEarly) load_dxy(vdx, vdy);
#pragma unroll
      for (int r = 1; r < M1; ++r) {
        const int s = r * NT + (NT - 1 - tl);
        if (s < PL::N1)
#pragma unroll
          for (int c = sMut; c < sNF; ++c) L.in.F[c][s] = vf[r - 1][c];
      }
      if constexpr (!kDxyEarly) write_dxy(vdx, vdy);
    }
    __syncthreads();

    // Zeta face between planes k-1 and k, and the update of the node on plane k-1.
    int tf = tid;  // laundered again for the face phase
    asm volatile("" : "+v"(tf));
    const int own1 = tf % TX + 1 + PL::RX1 * (tf / TX + 1);
    const int own2 = tf % TX + 2 + PL::RX2 * (tf / TX + 2);
    if (pending) {
      const LdsNode<TX, TY, 2, R> nb{L, own1, own2, zl[0], zl[1]};
      R hz[5];
      face_eval<2, R>(lo, nb, Wm, wp, k - 1, nk, true, Ph, hz);
      finish_node<R, kDual>(A, i, j, k - 1, part, hz, hz_lo, pq, pj, pt);
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        hz_lo[c] = hz[c];
        Wm[c] = lo.w[c];
      }
    }

    // Faces of the plane, held in registers until the staging space is free. Slot 0 of
    // every thread takes one xi and one eta face; the TY extra xi faces and TX extra eta
    // faces (slot 1) go to the lanes of two different waves, so that no wave evaluates more
    // than four faces per plane (the wave with the most faces sets the time to the barrier).
    R hx[MX][5], hy[MY][5];
#pragma unroll
    for (int r = 0; r < MX; ++r) {
      const int s = xi_slot(tf, r);
#pragma unroll
      for (int c = 0; c < 5; ++c) hx[r][c] = (R)0;
      // Slot 0 (s < NT = TX*TY) takes the first TX faces of each row, a row per TX lanes,
      // so the lanes of an LDS access read consecutive words; slot 1 the rows' last faces.
      int fx = r == 0 ? s % TX : TX, fy = r == 0 ? s / TX : s - NT;
      asm volatile("" : "+v"(fx), "+v"(fy));
      const int ia = wrap_or_out(i0 - 1 + fx, ni, D.per[0]);
      const int ja = wrap_or_out(j0 + fy, nj, D.per[1]);
      if (s >= 0 && ia >= 0 && ja >= 0 && (D.per[0] || ia < ni - 1)) {
        const int da = fx + (TX + 2) * fy;
        const LdsNode<TX, TY, 0, R> na{L, fx + PL::RX1 * (fy + 1), (fx + 1) + PL::RX2 * (fy + 2),
                                       L.in.DX[0][da], L.in.DX[1][da]};
        const LdsNode<TX, TY, 0, R> nb{L, fx + 1 + PL::RX1 * (fy + 1),
                                       (fx + 2) + PL::RX2 * (fy + 2), L.in.DX[0][da + 1],
                                       L.in.DX[1][da + 1]};
        R wm[5], wq[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          wm[c] = L.in.W[c][fx + PL::RX2 * (fy + 2)];
          wq[c] = L.in.W[c][fx + 3 + PL::RX2 * (fy + 2)];
        }
        face_eval<0, R>(na, nb, wm, wq, ia, ni, D.per[0], Ph, hx[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < MY; ++r) {
      const int s = eta_slot(tf, r);
#pragma unroll
      for (int c = 0; c < 5; ++c) hy[r][c] = (R)0;
      int fx = s % TX, fy = s / TX;
      asm volatile("" : "+v"(fx), "+v"(fy));
      const int ia = wrap_or_out(i0 + fx, ni, D.per[0]);
      const int ja = wrap_or_out(j0 - 1 + fy, nj, D.per[1]);
      if (s >= 0 && ia >= 0 && ja >= 0 && (D.per[1] || ja < nj - 1)) {
        const int da = fx + TX * fy;
        const LdsNode<TX, TY, 1, R> na{L, fx + 1 + PL::RX1 * fy, (fx + 2) + PL::RX2 * (fy + 1),
                                       L.in.DY[0][da], L.in.DY[1][da]};
        const LdsNode<TX, TY, 1, R> nb{L, fx + 1 + PL::RX1 * (fy + 1),
                                       (fx + 2) + PL::RX2 * (fy + 2), L.in.DY[0][da + TX],
                                       L.in.DY[1][da + TX]};
        R wm[5], wq[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          wm[c] = L.in.W[c][fx + 2 + PL::RX2 * fy];
          wq[c] = L.in.W[c][fx + 2 + PL::RX2 * (fy + 3)];
        }
        face_eval<1, R>(na, nb, wm, wq, ja, nj, D.per[1], Ph, hy[r]);
      }
    }
    // The own node becomes the lower node of the next zeta face.
    if (mine)
      lo.take(LdsNode<TX, TY, 2, R>{L, own1, own2, zl[0], zl[1]}, A,
              (unsigned)(i + ni * (j + nj * k)));
    __syncthreads();  // staging reads done: the space now takes the face fluxes
#pragma unroll
    for (int r = 0; r < MX; ++r) {
      const int s = xi_slot(tf, r);
      const int hs = r == 0 ? s + s / TX : (TX + 1) * (s - NT) + TX;  // row-major index
      if (s >= 0)
#pragma unroll
        for (int c = 0; c < 5; ++c) L.H[c][hs] = hx[r][c];
    }
#pragma unroll
    for (int r = 0; r < MY; ++r) {
      const int s = eta_slot(tf, r);
      if (s >= 0)
#pragma unroll
        for (int c = 0; c < 5; ++c) L.H[c][PL::NX + s] = hy[r][c];
    }
    __syncthreads();
    if (mine) {
      const int sx = a + (TX + 1) * b, sy = PL::NX + a + TX * b;
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        R rr = (R)0;
        rr += L.H[c][sx + 1] - L.H[c][sx];
        rr += L.H[c][sy + TX] - L.H[c][sy];
        part[c] = rr;
      }
    }
    __syncthreads();  // the face fluxes have been consumed: the space takes the next plane
  }
  if (mine && kend > kbeg) {  // zeta face above the chunk, upper node from global memory
    const int kt = kend == nk ? 0 : kend;
    const int kt2 = kt + 1 == nk ? 0 : kt + 1;
    const GlobalNodeZ<R> nb(A, i, j, kt);
    const unsigned o2 = (unsigned)(i + ni * (j + nj * kt2));
    R wp[5], hz[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) wp[c] = node_state<R>(A, o2).W[c];
    face_eval<2, R>(lo, nb, Wm, wp, kend - 1, nk, true, Ph, hz);
    finish_node<R, kDual>(A, i, j, kend - 1, part, hz, hz_lo);
  }
}

// Minimum waves per EU asked of the compiler for the persistent batch kernels: the launch
// shape's hint, and at least 3 in the mixed form, whose batch kernels otherwise come out a
// few registers above the 168 of 3 waves; never more than the block's LDS lets a CU
// (160 KB) hold. (The single-grid mixed kernels reach 3 waves unasked, and measured slower
// when asked.)
template <int TX, int TY, int WPE, typename R>
constexpr int min_waves() {
  constexpr int want = sizeof(R) == sizeof(float) && WPE < 3 ? 3 : WPE;
  constexpr int lds = (160 * 1024 / (int)sizeof(PlaneLds<TX, TY, R>)) * (TX * TY / 64) / 4;
  return want < lds ? want : (lds > 1 ? lds : 1);
}

// kDual: the dual-time update (mode 2) in place of the residual or Runge-Kutta epilogue.
template <int TX, int TY, int WPE, typename R, bool kDual = false>
__global__ void __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
k_stage_planes(StageArgs A, int kchunk) {
  __shared__ PlaneLds<TX, TY, R> L;
  const int gx = gridDim.x, gy = gridDim.y;
  const int lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int t = xcd_tile(lin, gx * gy * gridDim.z);
  const int bx = t % gx, by = (t / gx) % gy, bz = t / (gx * gy);
  const int kbeg = bz * kchunk;
  stage_block<TX, TY, R, kDual>(A, bx, by, kbeg, min(kbeg + kchunk, A.D.n[2]), L);
}

// Persistent form over the members of a batch: item = (member, bx | by << 16, kbeg, kend).
// The grid is a multiple of 8 blocks, so block b stays on XCD b % 8 and its items, remapped
// by xcd_tile, form one contiguous run of the work list per XCD.
template <int TX, int TY, int WPE, typename R>
__global__ void __launch_bounds__(TX * TY)
    __attribute__((amdgpu_waves_per_eu(min_waves<TX, TY, WPE, R>(), 8)))
    k_stage_batch(const StageArgs* __restrict__ args, const int4* __restrict__ work, int nwork) {
  __shared__ PlaneLds<TX, TY, R> L;
  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int4 it = work[xcd_tile(w, nwork)];
    const StageArgs A = args[it.x];
    stage_block<TX, TY, R>(A, it.y & 0xffff, it.y >> 16, it.z, it.w, L);
  }
}

}  // namespace

int nodes_kchunk(const Dims& D) {
  // z-chunks of about 8 planes, at least 2048 blocks in all
  const int gx = (D.n[0] + 63) / 64, gy = (D.n[1] + 3) / 4;
  const int nz = std::max(1, std::min(D.n[2], std::max(D.n[2] / 8, 2048 / (gx * gy))));
  return (D.n[2] + nz - 1) / nz;
}

int nodes_blocks(const Dims& D) {
  const int kchunk = nodes_kchunk(D);
  return ((D.n[0] + 63) / 64) * ((D.n[1] + 3) / 4) * ((D.n[2] + kchunk - 1) / kchunk);
}

hipError_t launch_nodes(const StageArgs& A, hipStream_t s) {
  const int gx = (A.D.n[0] + 63) / 64, gy = (A.D.n[1] + 3) / 4;
  const int kchunk = nodes_kchunk(A.D);
  const dim3 grid(gx, gy, (A.D.n[2] + kchunk - 1) / kchunk), block(64, 4, 1);
  if (A.dtau_out) {  // dual time stepping: no time-step reduction beside it
    if (A.dtpart) return hipErrorInvalidValue;
    if (A.mlp_fused && A.mixed)
      hipLaunchKernelGGL((k_nodes_tile_mlp<float, false, true>), grid, block, 0, s, A, kchunk);
    else if (A.mlp_fused)
      hipLaunchKernelGGL((k_nodes_tile_mlp<double, false, true>), grid, block, 0, s, A, kchunk);
    else if (A.mixed)
      hipLaunchKernelGGL((k_nodes_tile<float, false, true>), grid, block, 0, s, A, kchunk);
    else
      hipLaunchKernelGGL((k_nodes_tile<double, false, true>), grid, block, 0, s, A, kchunk);
    return hipGetLastError();
  }
  if (A.mlp_fused) {
    if (A.mixed && A.dtpart)
      hipLaunchKernelGGL((k_nodes_tile_mlp<float, true>), grid, block, 0, s, A, kchunk);
    else if (A.mixed)
      hipLaunchKernelGGL(k_nodes_tile_mlp<float>, grid, block, 0, s, A, kchunk);
    else if (A.dtpart)
      hipLaunchKernelGGL((k_nodes_tile_mlp<double, true>), grid, block, 0, s, A, kchunk);
    else
      hipLaunchKernelGGL(k_nodes_tile_mlp<double>, grid, block, 0, s, A, kchunk);
    return hipGetLastError();
  }
  if (A.mixed && A.dtpart)
    hipLaunchKernelGGL((k_nodes_tile<float, true>), grid, block, 0, s, A, kchunk);
  else if (A.mixed)
    hipLaunchKernelGGL(k_nodes_tile<float>, grid, block, 0, s, A, kchunk);
  else if (A.dtpart)
    hipLaunchKernelGGL((k_nodes_tile<double, true>), grid, block, 0, s, A, kchunk);
  else
    hipLaunchKernelGGL(k_nodes_tile<double>, grid, block, 0, s, A, kchunk);
  return hipGetLastError();
}

const char* const kTileNames[kNumTiles] = {"32x8", "32x4", "16x8", "16x16", "16x8/w2",
                                           "16x16/w2", "32x8/w3", "16x16/w3", "32x8/w4",
                                           "16x16/w4"};

template <int TX, int TY, int WPE = 1, typename R = double, bool kDual = false>
hipError_t launch_planes(const StageArgs& A, hipStream_t s, int kmin) {
  const int gx = (A.D.n[0] + TX - 1) / TX, gy = (A.D.n[1] + TY - 1) / TY;
  // Blocks resident at once on the device (occupancy query, kept after the first call).
  static int resident = 0;
  if (resident <= 0) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu,
                                                     k_stage_planes<TX, TY, WPE, R, kDual>,
                                                     TX * TY, 0) == hipSuccess &&
        hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      resident = per_cu * cus;
  }
  const int kchunk = kchunk_for(A.D, TX, TY, kmin, resident);
  const int nz = (A.D.n[2] + kchunk - 1) / kchunk;
  hipLaunchKernelGGL((k_stage_planes<TX, TY, WPE, R, kDual>), dim3(gx, gy, nz), dim3(TX * TY), 0,
                     s, A, kchunk);
  return hipGetLastError();
}

void tile_shape(int tile, int* tx, int* ty) {
  static const int shapes[kNumTiles][2] = {{32, 8}, {32, 4}, {16, 8}, {16, 16}, {16, 8},
                                           {16, 16}, {32, 8}, {16, 16}, {32, 8}, {16, 16}};
  const int t = tile >= 0 && tile < kNumTiles ? tile : 0;
  *tx = shapes[t][0];
  *ty = shapes[t][1];
}

int kchunk_for(const Dims& D, int tx, int ty, int kmin, int resident) {
  const int gx = (D.n[0] + tx - 1) / tx, gy = (D.n[1] + ty - 1) / ty;
  const long long tiles = (long long)gx * gy;
  const int nk = D.n[2], nzmax = max(1, nk / max(kmin, 1));
  if (resident <= 0) {  // about 1024 blocks
    const int nz = max(1, min((int)((1024 + tiles - 1) / tiles), nzmax));
    return (nk + nz - 1) / nz;
  }
  // Every block of a chunk takes about (depth + 1) plane times (the extra plane: the two
  // zeta faces at the chunk ends, which read their outer node from global memory), and the
  // blocks run in waves of `resident`: pick the chunk count with the least waves x depth.
  int best = (nk + nzmax - 1) / nzmax;
  long long best_cost = -1;
  for (int nz = 1; nz <= nzmax; ++nz) {
    const int kc = (nk + nz - 1) / nz;
    const long long waves = (tiles * ((nk + kc - 1) / kc) + resident - 1) / resident;
    const long long cost = waves * (kc + 1);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = kc;
    }
  }
  return best;
}

namespace {

template <int TX, int TY, int WPE, typename R>
hipError_t batch_stage(const BatchLaunch& B, hipStream_t s) {
  auto k = k_stage_batch<TX, TY, WPE, R>;
  if (B.grid <= 0) {  // occupancy query only
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, TX * TY, 0);
    *B.occupancy = nb;
    return e;
  }
  hipLaunchKernelGGL(k, dim3(B.grid), dim3(TX * TY), 0, s, B.args, B.work, B.nwork);
  return hipGetLastError();
}

template <typename R>
hipError_t batch_stage_tile(const BatchLaunch& B, hipStream_t s) {
  switch (B.tile) {
    case 1: return batch_stage<32, 4, 1, R>(B, s);
    case 2: return batch_stage<16, 8, 1, R>(B, s);
    case 3: return batch_stage<16, 16, 1, R>(B, s);
    case 4: return batch_stage<16, 8, 2, R>(B, s);
    case 5: return batch_stage<16, 16, 2, R>(B, s);
    case 6: return batch_stage<32, 8, 3, R>(B, s);
    case 7: return batch_stage<16, 16, 3, R>(B, s);
    case 8: return batch_stage<32, 8, 4, R>(B, s);
    case 9: return batch_stage<16, 16, 4, R>(B, s);
    default: return batch_stage<32, 8, 1, R>(B, s);
  }
}

}  // namespace

hipError_t launch_stage_batch(const BatchLaunch& B, hipStream_t s) {
  return B.mixed ? batch_stage_tile<float>(B, s) : batch_stage_tile<double>(B, s);
}

hipError_t launch_nodes_batch(const BatchLaunch& B, hipStream_t s) {
  if (B.grid <= 0) {
    int nb = 0;
    hipError_t e = B.mixed
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_nodes_tile_batch<float>, 256, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_nodes_tile_batch<double>, 256, 0);
    *B.occupancy = nb;
    return e;
  }
  const dim3 g(B.grid), blk(64, 4);
  if (B.mixed && B.dt)
    hipLaunchKernelGGL((k_nodes_tile_batch<float, true>), g, blk, 0, s, B.args, B.work, B.nwork);
  else if (B.mixed)
    hipLaunchKernelGGL(k_nodes_tile_batch<float>, g, blk, 0, s, B.args, B.work, B.nwork);
  else if (B.dt)
    hipLaunchKernelGGL((k_nodes_tile_batch<double, true>), g, blk, 0, s, B.args, B.work, B.nwork);
  else
    hipLaunchKernelGGL(k_nodes_tile_batch<double>, g, blk, 0, s, B.args, B.work, B.nwork);
  return hipGetLastError();
}

hipError_t launch_stage(const StageArgs& A, hipStream_t s) {
  const int kmin = A.kmin > 0 ? A.kmin : 8;
  if (A.mode == 2) {  // the dual-time update: default launch shapes only
    if (A.tile != (A.mixed ? kDefaultTileMixed : kDefaultTileFp64)) return hipErrorInvalidValue;
    // (the mixed form asks for 3 waves/EU: its longer epilogue would otherwise cost one)
    return A.mixed ? launch_planes<32, 8, 3, float, true>(A, s, kmin)
                   : launch_planes<16, 16, 1, double, true>(A, s, kmin);
  }
  if (A.mixed) switch (A.tile) {
      case 1: return launch_planes<32, 4, 1, float>(A, s, kmin);
      case 2: return launch_planes<16, 8, 1, float>(A, s, kmin);
      case 3: return launch_planes<16, 16, 1, float>(A, s, kmin);
      case 4: return launch_planes<16, 8, 2, float>(A, s, kmin);
      case 5: return launch_planes<16, 16, 2, float>(A, s, kmin);
      case 6: return launch_planes<32, 8, 3, float>(A, s, kmin);
      case 7: return launch_planes<16, 16, 3, float>(A, s, kmin);
      case 8: return launch_planes<32, 8, 4, float>(A, s, kmin);
      case 9: return launch_planes<16, 16, 4, float>(A, s, kmin);
      default: return launch_planes<32, 8, 1, float>(A, s, kmin);
    }
  switch (A.tile) {
    case 1: return launch_planes<32, 4>(A, s, kmin);
    case 2: return launch_planes<16, 8>(A, s, kmin);
    case 3: return launch_planes<16, 16>(A, s, kmin);
    case 4: return launch_planes<16, 8, 2>(A, s, kmin);
    case 5: return launch_planes<16, 16, 2>(A, s, kmin);
    case 6: return launch_planes<32, 8, 3>(A, s, kmin);
    case 7: return launch_planes<16, 16, 3>(A, s, kmin);
    case 8: return launch_planes<32, 8, 4>(A, s, kmin);
    case 9: return launch_planes<16, 16, 4>(A, s, kmin);
    default: return launch_planes<32, 8>(A, s, kmin);
  }
}

}  // namespace lesmi
