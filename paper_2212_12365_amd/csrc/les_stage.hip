// Runge-Kutta stage kernels of the LES residual (gfx950, FP64).
//
// A stage is two launches:
//  * k_nodes: one thread per node writes a node record (primitive variables, molecular and
//    eddy viscosity, scaled spectral radii and pressure sensors); the eddy viscosity and the
//    sensors read the neighbouring nodes through the cache.
//  * k_stage: one block per 16x4x4 tile of nodes. Every face of the tile (and the faces on
//    its lower halo) is computed once into LDS, then each node sums its six face fluxes
//    (paper, Spatial Discretization) and either writes the residual or applies the
//    Runge-Kutta stage update (paper, Time Marching Method).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "les_common.h"
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

__global__ void __launch_bounds__(256) k_nodes(StageArgs A) {
  const Dims& D = A.D;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y * blockDim.y + threadIdx.y;
  int k = blockIdx.z;
  if (i >= D.n[0] || j >= D.n[1]) return;
  const int N = (int)D.N;
  const double* __restrict__ q = A.q;
  int ix[3] = {i, j, k};
  int o = off3(D, i, j, k);
  Prim s = load_prim(q, N, o, A.P);
  // Velocity differences delta_e u_m (centred; one-sided at the ends of a non-periodic
  // direction) and pressure sensors along e.
  double du[3][3];
  double nu[3];
  for (int e = 0; e < 3; ++e) {
    int n = D.n[e], m = ix[e];
    int stride = e == 0 ? 1 : (e == 1 ? D.n[0] : D.n[0] * D.n[1]);
    bool interior = D.per[e] || (m > 0 && m < n - 1);
    if (interior) {
      int mp = m + 1 == n ? 0 : m + 1, mm = m == 0 ? n - 1 : m - 1;
      Prim a = load_prim(q, N, o + (mp - m) * stride, A.P);
      Prim b = load_prim(q, N, o + (mm - m) * stride, A.P);
      du[e][0] = 0.5 * (a.u - b.u);
      du[e][1] = 0.5 * (a.v - b.v);
      du[e][2] = 0.5 * (a.w - b.w);
      nu[e] = sensor(b.p, s.p, a.p);
    } else {
      int sg = m == 0 ? 1 : -1;  // towards the interior
      Prim a = load_prim(q, N, o + sg * stride, A.P);
      Prim b = load_prim(q, N, o + 2 * sg * stride, A.P);
      double h = 0.5 * sg;
      du[e][0] = h * (-3.0 * s.u + 4.0 * a.u - b.u);
      du[e][1] = h * (-3.0 * s.v + 4.0 * a.v - b.v);
      du[e][2] = h * (-3.0 * s.w + 4.0 * a.w - b.w);
      // The boundary node takes the sensor of its interior neighbour c (p at c-1, c, c+1).
      nu[e] = m == 0 ? sensor(s.p, a.p, b.p) : sensor(b.p, a.p, s.p);
    }
  }
  double sm[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) sm[c] = A.S[c * N + o];
  double jinv = A.jinv[o];
  double mut = smagorinsky(sm, du, s.rho, jinv, A.P);
  double a = sqrt(s.T);
  double l0 = spectral(sm[0], sm[1], sm[2], s.u, s.v, s.w, a);
  double l1 = spectral(sm[3], sm[4], sm[5], s.u, s.v, s.w, a);
  double l2 = spectral(sm[6], sm[7], sm[8], s.u, s.v, s.w, a);
  double lb[3];
  scaled_radii(l0, l1, l2, lb);
  double* __restrict__ r = A.rec;
  r[kRecU * N + o] = s.u;
  r[kRecV * N + o] = s.v;
  r[kRecW * N + o] = s.w;
  r[kRecT * N + o] = s.T;
  r[kRecP * N + o] = s.p;
  r[kRecMu * N + o] = sutherland(s.T, A.P);
  r[kRecMut * N + o] = mut;
  r[(kRecLb + 0) * N + o] = lb[0];
  r[(kRecLb + 1) * N + o] = lb[1];
  r[(kRecLb + 2) * N + o] = lb[2];
  r[(kRecNu + 0) * N + o] = nu[0];
  r[(kRecNu + 1) * N + o] = nu[1];
  r[(kRecNu + 2) * N + o] = nu[2];
  if (A.mut_out) A.mut_out[o] = mut;
}

// ---------------------------------------------------------------------------------------
// Face fluxes.
// ---------------------------------------------------------------------------------------

// Field planes of the inputs, as wave-uniform base pointers.
struct Planes {
  const double* q[5];
  const double* u[4];  // record u, v, w, T
  const double* p;
  const double* mu;
  const double* mut;
  const double* lb;
  const double* nu;
  const double* S[9];
  const double* jinv;
};

__device__ __forceinline__ Planes make_planes(const StageArgs& A, int d) {
  const int N = (int)A.D.N;
  Planes P;
#pragma unroll
  for (int c = 0; c < 5; ++c) P.q[c] = A.q + c * N;
  P.u[0] = A.rec + kRecU * N;
  P.u[1] = A.rec + kRecV * N;
  P.u[2] = A.rec + kRecW * N;
  P.u[3] = A.rec + kRecT * N;
  P.p = A.rec + kRecP * N;
  P.mu = A.rec + kRecMu * N;
  P.mut = A.rec + kRecMut * N;
  P.lb = A.rec + (kRecLb + d) * N;
  P.nu = A.rec + (kRecNu + d) * N;
#pragma unroll
  for (int c = 0; c < 9; ++c) P.S[c] = A.S + c * N;
  P.jinv = A.jinv;
  return P;
}

template <int e>
__device__ __forceinline__ int dir_stride(const Dims& D) {
  return e == 0 ? 1 : (e == 1 ? D.n[0] : D.n[0] * D.n[1]);
}

// Nodal difference along e of (u, v, w, T) at node offset o whose index along e is m:
// centred, wrapped if periodic, second-order one-sided at the ends otherwise.
template <int e>
__device__ __forceinline__ void node_diff4(const Dims& D, const Planes& P, int m, unsigned o,
                                           double* out) {
  const int n = D.n[e];
  const unsigned st = dir_stride<e>(D);
  if (D.per[e] || (m > 0 && m < n - 1)) {
    unsigned op = m + 1 == n ? o - (unsigned)(n - 1) * st : o + st;
    unsigned om = m == 0 ? o + (unsigned)(n - 1) * st : o - st;
#pragma unroll
    for (int v = 0; v < 4; ++v) out[v] = 0.5 * (P.u[v][op] - P.u[v][om]);
  } else if (m == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
      out[v] = 0.5 * (-3.0 * P.u[v][o] + 4.0 * P.u[v][o + st] - P.u[v][o + 2 * st]);
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v)
      out[v] = 0.5 * (3.0 * P.u[v][o] - 4.0 * P.u[v][o - st] + P.u[v][o - 2 * st]);
  }
}

// Total numerical flux H = (F_A + F_B)/2 - D - F_v on the face between node A = (ia, ja, ka)
// and its + neighbour B along d (paper, Spatial Discretization: interface flux with the
// Turkel-Vatsa terms; viscous flux from the two nodes of the interface). B must exist.
template <int d>
__device__ __forceinline__ void face_flux(const StageArgs& A, int ia, int ja, int ka,
                                          double* H) {
  const Dims& D = A.D;
  const Phys& Ph = A.P;
  const Planes P = make_planes(A, d);
  const int ix[3] = {ia, ja, ka};
  const int n = D.n[d], m = ix[d];
  const unsigned st = dir_stride<d>(D);
  const unsigned oa = (unsigned)(ia + D.n[0] * (ja + D.n[1] * ka));
  const unsigned ob = m + 1 == n ? oa - (unsigned)(n - 1) * st : oa + st;
  const int mb = m + 1 == n ? 0 : m + 1;

  double qa[5], qb[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    qa[c] = P.q[c][oa];
    qb[c] = P.q[c][ob];
  }
  Prim sa{qa[0], P.u[0][oa], P.u[1][oa], P.u[2][oa], P.p[oa], P.u[3][oa]};
  Prim sb{qb[0], P.u[0][ob], P.u[1][ob], P.u[2][ob], P.p[ob], P.u[3][ob]};
  double Sa[9], Sb[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    Sa[c] = P.S[c][oa];
    Sb[c] = P.S[c][ob];
  }
  double FA[5], FB[5];
  inviscid_flux(Sa[3 * d], Sa[3 * d + 1], Sa[3 * d + 2], qa, sa, FA);
  inviscid_flux(Sb[3 * d], Sb[3 * d + 1], Sb[3 * d + 2], qb, sb, FB);

  // Dissipated vector W = Q + (0,0,0,0,p); at the first and last face of a non-periodic
  // direction the outside difference is the negated inside one.
  double wa[5], wb[5], dW[5], d3W[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    wa[c] = qa[c];
    wb[c] = qb[c];
  }
  wa[4] += sa.p;
  wb[4] += sb.p;
#pragma unroll
  for (int c = 0; c < 5; ++c) dW[c] = wb[c] - wa[c];
  if (D.per[d] || (m > 0 && m < n - 2)) {
    const unsigned om = m == 0 ? oa + (unsigned)(n - 1) * st : oa - st;
    const unsigned op = mb + 1 == n ? ob - (unsigned)(n - 1) * st : ob + st;
    double wm[5], wp[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      wm[c] = P.q[c][om];
      wp[c] = P.q[c][op];
    }
    wm[4] += P.p[om];
    wp[4] += P.p[op];
#pragma unroll
    for (int c = 0; c < 5; ++c) d3W[c] = wp[c] - 3.0 * wb[c] + 3.0 * wa[c] - wm[c];
  } else if (m == 0) {
    const unsigned op = ob + st;
    double wp[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) wp[c] = P.q[c][op];
    wp[4] += P.p[op];
#pragma unroll
    for (int c = 0; c < 5; ++c) d3W[c] = (wp[c] - wb[c]) - 3.0 * dW[c];
  } else {  // m == n - 2
    const unsigned om = oa - st;
    double wm[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) wm[c] = P.q[c][om];
    wm[4] += P.p[om];
#pragma unroll
    for (int c = 0; c < 5; ++c) d3W[c] = -3.0 * dW[c] + (wa[c] - wm[c]);
  }
  const double lf = 0.5 * (P.lb[oa] + P.lb[ob]);
  double Dd[5];
  dissipation(lf, P.nu[oa], P.nu[ob], dW, d3W, Ph, Dd);

  // Viscous flux: compact difference along d, averaged nodal differences across.
  double Sf[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) Sf[c] = 0.5 * (Sa[c] + Sb[c]);
  const double jf = 0.5 * (P.jinv[oa] + P.jinv[ob]);
  double gxi[4][3];
  gxi[0][d] = sb.u - sa.u;
  gxi[1][d] = sb.v - sa.v;
  gxi[2][d] = sb.w - sa.w;
  gxi[3][d] = sb.T - sa.T;
  {
    constexpr int e = d == 0 ? 1 : 0;
    double da[4], db[4];
    node_diff4<e>(D, P, ix[e], oa, da);
    node_diff4<e>(D, P, ix[e], ob, db);
#pragma unroll
    for (int v = 0; v < 4; ++v) gxi[v][e] = 0.5 * (da[v] + db[v]);
  }
  {
    constexpr int e = d == 2 ? 1 : 2;
    double da[4], db[4];
    node_diff4<e>(D, P, ix[e], oa, da);
    node_diff4<e>(D, P, ix[e], ob, db);
#pragma unroll
    for (int v = 0; v < 4; ++v) gxi[v][e] = 0.5 * (da[v] + db[v]);
  }
  const double muf = 0.5 * (P.mu[oa] + P.mu[ob]);
  const double mutf = 0.5 * (P.mut[oa] + P.mut[ob]);
  const double ub[3] = {0.5 * (sa.u + sb.u), 0.5 * (sa.v + sb.v), 0.5 * (sa.w + sb.w)};
  double Fv[5];
  viscous_flux(Sf, jf, gxi, muf, mutf, ub, d, Ph, Fv);
  Fv[0] = 0.0;
#pragma unroll
  for (int c = 0; c < 5; ++c) H[c] = 0.5 * (FA[c] + FB[c]) - Dd[c] - Fv[c];
}

// Maps the dispatch order onto tiles so that each XCD (blocks are dealt round-robin to the
// 8 XCDs) works on one contiguous run of tiles, whose shared halo data then stays in that
// XCD's L2.
__device__ __forceinline__ int xcd_tile(int lin, int nblk) {
  const int full = (nblk / 8) * 8;
  if (lin >= full) return lin;
  return (lin % 8) * (full / 8) + lin / 8;
}

// One block per TX x TY column tile and chunk of z-planes. Per plane, the xi and eta faces of
// the plane (including the tile's lower edge faces) go to LDS once; each thread carries the
// zeta face below its node in registers; then every node sums its six faces and applies
// the epilogue (residual, or the Runge-Kutta stage update of the paper's Time Marching
// Method).
template <int TX, int TY, int WPE>
__global__ void __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
k_stage(StageArgs A, int kchunk) {
  constexpr int NT = TX * TY;
  constexpr int NX = (TX + 1) * TY;
  constexpr int NY = TX * (TY + 1);
  __shared__ double hx[5][NX];
  __shared__ double hy[5][NY];
  const Dims& D = A.D;
  const int N = (int)D.N;
  const int gx = gridDim.x, gy = gridDim.y;
  const int lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int t = xcd_tile(lin, gx * gy * gridDim.z);
  const int bx = t % gx, by = (t / gx) % gy, bz = t / (gx * gy);
  const int i0 = bx * TX, j0 = by * TY;
  const int kbeg = bz * kchunk;
  const int kend = min(kbeg + kchunk, D.n[2]);
  const int tid = threadIdx.x;
  const int a = tid % TX, b = tid / TX;
  const int i = i0 + a, j = j0 + b;
  const bool mine = i < D.n[0] && j < D.n[1];

  // Zeta face below the chunk's first plane.
  double hz_lo[5] = {0, 0, 0, 0, 0};
  if (mine) {
    int kl = wrap_or_out(kbeg - 1, D.n[2], D.per[2]);
    if (kl >= 0) face_flux<2>(A, i, j, kl, hz_lo);
  }
  for (int k = kbeg; k < kend; ++k) {
    for (int s = tid; s < NX; s += NT) {
      int ia = wrap_or_out(i0 + s % (TX + 1) - 1, D.n[0], D.per[0]);
      int ja = wrap_or_out(j0 + s / (TX + 1), D.n[1], D.per[1]);
      if (ia >= 0 && ja >= 0 && (D.per[0] || ia < D.n[0] - 1)) {
        double H[5];
        face_flux<0>(A, ia, ja, k, H);
#pragma unroll
        for (int c = 0; c < 5; ++c) hx[c][s] = H[c];
      }
    }
    for (int s = tid; s < NY; s += NT) {
      int ia = wrap_or_out(i0 + s % TX, D.n[0], D.per[0]);
      int ja = wrap_or_out(j0 + s / TX - 1, D.n[1], D.per[1]);
      if (ia >= 0 && ja >= 0 && (D.per[1] || ja < D.n[1] - 1)) {
        double H[5];
        face_flux<1>(A, ia, ja, k, H);
#pragma unroll
        for (int c = 0; c < 5; ++c) hy[c][s] = H[c];
      }
    }
    double hz_hi[5] = {0, 0, 0, 0, 0};
    if (mine && (D.per[2] || k < D.n[2] - 1)) face_flux<2>(A, i, j, k, hz_hi);
    __syncthreads();
    if (mine) {
      const int o = i + D.n[0] * (j + D.n[1] * k);
      if (is_updated(D, i, j, k)) {
        const int sx = a + (TX + 1) * b, sy = a + TX * b;
        double fac = 0.0;
        if (A.mode == 1) fac = A.alpha * A.dt[0] * A.jac[o];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          double rr = 0.0;
          rr += hx[c][sx + 1] - hx[c][sx];
          rr += hy[c][sy + TX] - hy[c][sy];
          rr += hz_hi[c] - hz_lo[c];
          if (A.mode == 0)
            A.out[c * N + o] = rr;
          else
            A.out[c * N + o] = A.q0[c * N + o] - fac * rr;
        }
      } else if (A.mode == 0) {
#pragma unroll
        for (int c = 0; c < 5; ++c) A.out[c * N + o] = 0.0;
      }
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) hz_lo[c] = hz_hi[c];
    __syncthreads();
  }
}

template <int TX, int TY, int WPE = 2>
hipError_t launch_tile(const StageArgs& A, hipStream_t s, int kmin) {
  const int gx = (A.D.n[0] + TX - 1) / TX, gy = (A.D.n[1] + TY - 1) / TY;
  // Enough z-chunks for about 1024 blocks, each chunk at least kmin planes deep.
  int nz = (1024 + gx * gy - 1) / (gx * gy);
  nz = max(1, min(nz, A.D.n[2] / kmin));
  const int kchunk = (A.D.n[2] + nz - 1) / nz;
  nz = (A.D.n[2] + kchunk - 1) / kchunk;
  hipLaunchKernelGGL((k_stage<TX, TY, WPE>), dim3(gx, gy, nz), dim3(TX * TY), 0, s, A, kchunk);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_nodes(const StageArgs& A, hipStream_t s) {
  dim3 block(64, 4, 1);
  dim3 grid((A.D.n[0] + 63) / 64, (A.D.n[1] + 3) / 4, A.D.n[2]);
  hipLaunchKernelGGL(k_nodes, grid, block, 0, s, A);
  return hipGetLastError();
}

const char* const kTileNames[kNumTiles] = {"32x8", "64x4", "16x16", "32x4", "64x2",
                                           "128x2", "32x8/w3", "64x4/w3", "32x8/w4",
                                           "64x4/w4"};

hipError_t launch_stage(const StageArgs& A, hipStream_t s) {
  const int kmin = A.kmin > 0 ? A.kmin : 8;
  switch (A.tile) {
    case 1: return launch_tile<64, 4>(A, s, kmin);
    case 2: return launch_tile<16, 16>(A, s, kmin);
    case 3: return launch_tile<32, 4>(A, s, kmin);
    case 4: return launch_tile<64, 2>(A, s, kmin);
    case 5: return launch_tile<128, 2>(A, s, kmin);
    case 6: return launch_tile<32, 8, 3>(A, s, kmin);
    case 7: return launch_tile<64, 4, 3>(A, s, kmin);
    case 8: return launch_tile<32, 8, 4>(A, s, kmin);
    case 9: return launch_tile<64, 4, 4>(A, s, kmin);
    default: return launch_tile<32, 8>(A, s, kmin);
  }
}

}  // namespace lesmi
