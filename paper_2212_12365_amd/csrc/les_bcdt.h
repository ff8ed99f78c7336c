// Boundary-condition, time-step and state-check device functions of the lesmi library
// (gfx950), shared by the single-grid kernels and the persistent batch kernels. Each
// function covers one block's or one thread's part of the work, given its coordinates.
#pragma once

#include <hip/hip_runtime.h>

#include "les_common.h"

namespace lesmi {

// ---------------------------------------------------------------------------------------
// Boundary conditions (paper, Boundary Conditions).
// ---------------------------------------------------------------------------------------

// Far-field Riemann state from the interior state qe and the unit outward normal n.
__device__ void farfield_state(const Phys& P, const BcData& B, const double* qe,
                               const double* n, double* qo) {
  double g = P.gamma;
  double re = qe[0];
  double ue[3] = {qe[1] / re, qe[2] / re, qe[3] / re};
  double pe = P.gm1 * (qe[4] - 0.5 * re * (ue[0] * ue[0] + ue[1] * ue[1] + ue[2] * ue[2]));
  double ae = sqrt(g * pe / re);
  double ainf = sqrt(g * B.p_inf / B.rho_inf);
  double qne = ue[0] * n[0] + ue[1] * n[1] + ue[2] * n[2];
  double qninf = B.u_inf[0] * n[0] + B.u_inf[1] * n[1] + B.u_inf[2] * n[2];
  double rp = qne + 2.0 * ae * P.inv_gm1;
  double rm = qninf - 2.0 * ainf * P.inv_gm1;
  double qnf = 0.5 * (rp + rm);
  double af = 0.25 * P.gm1 * (rp - rm);
  double mn = qne / ae;
  double uf[3], rf, pf;
  if (mn >= 1.0) {
    for (int c = 0; c < 5; ++c) qo[c] = qe[c];
    return;
  } else if (mn > -1.0) {
    // Subsonic: the entropy p / rho^gamma of the interior (outflow) or of the free stream
    // (inflow) with the face sound speed af gives the density; along an isentrope
    // rho_f = rho_ref (af / a_ref)^(2 / (gamma - 1)), one power instead of two.
    const bool out = mn >= 0.0;
    const double rr = out ? re : B.rho_inf, ar = out ? ae : ainf;
    const double* ub = out ? ue : B.u_inf;
    const double qb = out ? qne : qninf;
    for (int c = 0; c < 3; ++c) uf[c] = ub[c] + (qnf - qb) * n[c];
    rf = rr * pow(af / ar, 2.0 * P.inv_gm1);
    pf = rf * af * af / g;
  } else {
    for (int c = 0; c < 3; ++c) uf[c] = B.u_inf[c];
    rf = B.rho_inf;
    pf = B.p_inf;
  }
  qo[0] = rf;
  qo[1] = rf * uf[0];
  qo[2] = rf * uf[1];
  qo[3] = rf * uf[2];
  qo[4] = pf * P.inv_gm1 + 0.5 * rf * (uf[0] * uf[0] + uf[1] * uf[1] + uf[2] * uf[2]);
}

// Centreline means of the first ring, summed in k order (paper, Centerline Boundary
// Condition). One 256-thread block per axial station i: the ring is staged through LDS in
// chunks of C and five threads add it up sequentially, so the sum order is k = 0, 1, ...,
// nk-1 for any C.
// The means go to axis[c * ni + i] and, with mean non-null, to mean[0..4] (LDS) for the
// whole block.
constexpr int kAxisChunk = 256;
template <int C = kAxisChunk>
__device__ __forceinline__ void axis_mean_block(const Dims& D, const double* __restrict__ q,
                                                double* __restrict__ axis, int i,
                                                double (&ring)[5][C], double* mean = nullptr) {
  const long long N = D.N;
  const int nk = D.n[2];
  double sum = 0.0;  // thread c < 5 accumulates component c
  constexpr int kPer = (5 * C + 255) / 256;  // ring values per thread of a 256-thread block
  for (int kb = 0; kb < nk; kb += C) {
    const int len = min(C, nk - kb);
    double v[kPer];  // all of the thread's loads are issued before the first LDS store
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int t = threadIdx.x + 256 * r;
      if (t < 5 * len) v[r] = q[(long long)(t / len) * N + nid(D, i, 1, kb + t % len)];
    }
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int t = threadIdx.x + 256 * r;
      if (t < 5 * len) ring[t / len][t % len] = v[r];
    }
    __syncthreads();
    if (threadIdx.x < 5)
      for (int k = 0; k < len; ++k) sum += ring[threadIdx.x][k];
    __syncthreads();
  }
  if (threadIdx.x < 5) {
    const double m = sum / (double)nk;
    axis[(long long)threadIdx.x * D.n[0] + i] = m;
    if (mean) mean[threadIdx.x] = m;
  }
  if (mean) __syncthreads();
}

__device__ __forceinline__ void load_q(const double* q, long long N, long long id, double* o) {
  for (int c = 0; c < 5; ++c) o[c] = q[(long long)c * N + id];
}

// Entrance node (0, j, k), o = j + nj k: the jet state inside the jet, else the far-field
// state from qe, the state of node (1, j, k) after the far field and centreline conditions.
__device__ __forceinline__ void entrance_state(const Phys& P, const BcData& B, long long nface,
                                               long long o, const double* qe, double* qo) {
  if (B.jetmask[o]) {
    const double uj = B.mach_jet;
    qo[0] = 1.0;
    qo[1] = uj;
    qo[2] = 0.0;
    qo[3] = 0.0;
    qo[4] = (1.0 / P.gamma) * P.inv_gm1 + 0.5 * uj * uj;
  } else {
    const double n[3] = {B.nin[o], B.nin[nface + o], B.nin[2 * nface + o]};
    farfield_state(P, B, qe, n, qo);
  }
}

// Exit node (ni-1, j, k), o = j + nj k, from qe, the state of node (ni-2, j, k) after the far
// field and centreline conditions: extrapolated where the normal Mach number is supersonic,
// else p_inf with the interior's velocity and internal energy per unit mass.
__device__ __forceinline__ void exit_state(const Phys& P, const BcData& B, long long nface,
                                           long long o, const double* qe, double* qo) {
  const double n[3] = {B.nex[o], B.nex[nface + o], B.nex[2 * nface + o]};
  const double re = qe[0];
  const double ue[3] = {qe[1] / re, qe[2] / re, qe[3] / re};
  const double pe = P.gm1 * (qe[4] - 0.5 * re * (ue[0] * ue[0] + ue[1] * ue[1] + ue[2] * ue[2]));
  const double ae = sqrt(P.gamma * pe / re);
  const double mn = (ue[0] * n[0] + ue[1] * n[1] + ue[2] * n[2]) / ae;
  if (mn >= 1.0) {
    for (int c = 0; c < 5; ++c) qo[c] = qe[c];
  } else {
    const double eint = pe / (P.gm1 * re);
    const double rb = B.p_inf / (P.gm1 * eint);
    qo[0] = rb;
    qo[1] = rb * ue[0];
    qo[2] = rb * ue[1];
    qo[3] = rb * ue[2];
    qo[4] = B.p_inf * P.inv_gm1 + 0.5 * rb * (ue[0] * ue[0] + ue[1] * ue[1] + ue[2] * ue[2]);
  }
}

// Boundary nodes other than the centreline's, one thread each: far field (j = nj-1,
// 1 <= i <= ni-2), entrance (i = 0) and exit (i = ni-1), the last two without their j = 0
// nodes, which take the centreline means (bc_station_block). Each value is composed from
// updated nodes only, reproducing the order far field -> centreline -> entrance -> exit.
__device__ __host__ __forceinline__ long long bc_count(const Dims& D) {
  return (long long)(D.n[0] - 2) * D.n[2] + 2LL * D.n[1] * D.n[2];
}

__device__ __forceinline__ void bc_node(const Dims& D, const Phys& P, const BcData& B,
                                        double* __restrict__ q, long long t) {
  const int ni = D.n[0], nj = D.n[1];
  const long long N = D.N;
  const long long nrow = (long long)(ni - 2) * D.n[2];
  const long long nface = (long long)nj * D.n[2];
  double qe[5], qo[5];
  // Far-field state of node (i, nj-1, k), from its interior neighbour.
  auto farfield_node = [&](int i, int k, double* o) {
    double qi[5];
    load_q(q, N, nid(D, i, nj - 2, k), qi);
    const long long s = (long long)ni * D.n[2], off = i + (long long)ni * k;
    const double nn[3] = {B.nff[off], B.nff[s + off], B.nff[2 * s + off]};
    farfield_state(P, B, qi, nn, o);
  };
  // State of node (i, j, k), 1 <= j <= nj-1, after the far field condition.
  auto after_j = [&](int i, int j, int k, double* o) {
    if (j == nj - 1)
      farfield_node(i, k, o);
    else
      load_q(q, N, nid(D, i, j, k), o);
  };
  long long id;
  if (t < nrow) {  // far field
    const int i = 1 + (int)(t % (ni - 2)), k = (int)(t / (ni - 2));
    farfield_node(i, k, qo);
    id = nid(D, i, nj - 1, k);
  } else if (t < nrow + nface) {  // entrance
    const long long o = t - nrow;
    const int j = (int)(o % nj), k = (int)(o / nj);
    if (j == 0) return;
    id = nid(D, 0, j, k);
    if (!B.jetmask[o]) after_j(1, j, k, qe);
    entrance_state(P, B, nface, o, qe, qo);
  } else if (t < nrow + 2 * nface) {  // exit
    const long long o = t - nrow - nface;
    const int j = (int)(o % nj), k = (int)(o / nj);
    if (j == 0) return;
    id = nid(D, ni - 1, j, k);
    after_j(ni - 2, j, k, qe);
    exit_state(P, B, nface, o, qe, qo);
  } else {
    return;
  }
  for (int c = 0; c < 5; ++c) q[(long long)c * N + id] = qo[c];
}

// Centreline nodes of axial station i, 1 <= i <= ni-2 (one block): the means of ring j = 1
// (also left in B.axis), written to nodes (i, 0, k); station 1's block also writes the
// entrance nodes (0, 0, k) and station ni-2's the exit nodes (ni-1, 0, k), whose interior
// neighbours are those centreline nodes.
template <int C>
__device__ __forceinline__ void bc_station_block(const Dims& D, const Phys& P, const BcData& B,
                                                 double* __restrict__ q, int i,
                                                 double (&ring)[5][C], double* mean) {
  axis_mean_block<C>(D, q, B.axis, i, ring, mean);
  const int ni = D.n[0], nj = D.n[1], nk = D.n[2];
  const long long N = D.N, nface = (long long)nj * nk;
  double m[5];
  for (int c = 0; c < 5; ++c) m[c] = mean[c];
  for (int k = threadIdx.x; k < nk; k += blockDim.x) {
    const long long id = nid(D, i, 0, k);
    for (int c = 0; c < 5; ++c) q[(long long)c * N + id] = m[c];
    double qo[5];
    const long long o = (long long)nj * k;
    if (i == 1) {
      entrance_state(P, B, nface, o, m, qo);
      const long long e = nid(D, 0, 0, k);
      for (int c = 0; c < 5; ++c) q[(long long)c * N + e] = qo[c];
    }
    if (i == ni - 2) {
      exit_state(P, B, nface, o, m, qo);
      const long long e = nid(D, ni - 1, 0, k);
      for (int c = 0; c < 5; ++c) q[(long long)c * N + e] = qo[c];
    }
  }
}

// ---------------------------------------------------------------------------------------
// Time step (paper, Time Marching Method): dt = CFL min over updated nodes of
// J^-1 / sum_d Lam_d. The node kernel of a step's first stage writes per-block minima.
// ---------------------------------------------------------------------------------------
// dt = CFL times the minimum of the block minima (exact in any order).
__device__ __forceinline__ void dt_final_block(const double* __restrict__ part, int nparts,
                                               double cfl, double* __restrict__ dt,
                                               double* red) {
  double r = INFINITY;
  for (int b = threadIdx.x; b < nparts; b += 256) r = fmin(r, part[b]);
  red[threadIdx.x] = r;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) dt[0] = cfl * red[0];
  __syncthreads();
}

// Non-finite or non-positive density/pressure at node (i, j, k) sets flag bit 2.
__device__ __forceinline__ void check_node(const Dims& D, const Phys& P,
                                           const double* __restrict__ q, int i, int j, int k,
                                           int* __restrict__ flag) {
  if (i >= D.n[0] || j >= D.n[1]) return;
  const int N = (int)D.N;
  const int id = i + D.n[0] * (j + D.n[1] * k);
  Prim s = prim_from_q(q[id], q[N + id], q[2 * N + id], q[3 * N + id], q[4 * N + id], P);
  bool ok = s.rho > 0.0 && s.p > 0.0 && isfinite(s.u) && isfinite(s.v) && isfinite(s.w) &&
            isfinite(q[4 * N + id]);
  if (!ok) atomicOr(flag, 2);
}

}  // namespace lesmi
