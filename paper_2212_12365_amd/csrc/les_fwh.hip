// Far-field noise by the Ffowcs Williams-Hawkings analogy from a permeable control surface
// around the jet (gfx950). The paper names this analogy as the route from its LES to far-field
// acoustics (Introduction; Concluding Remarks) and gives no formulation; the one used is
// Farassat's formulation 1A for a stationary surface in a medium at rest, the viscous stresses
// left out of the loading:
//   Q_n = rho u . n,  L_i = (p - p0) n_i + rho u_i (u . n),
//   4 pi p'(x, t) = sum over surface nodes of dS [ dQ_n/dtau / r + dL_r/dtau / (c0 r)
//                                                  + L_r / r^2 ] at tau = t - r/c0,
// with r = |x - y|, L_r = L . (x - y)/r.
//
// Three steps, all on the device:
//  * les_fwh_create: the surface nodes (lateral cylinder j = js, optional end caps), their
//    unit normals and areas from the metric vectors (S_eta, -/+ S_xi), with half weights on
//    patch edges;
//  * les_fwh_sample: one gather kernel per sample, (rho, u, v, w, p) of every surface node into
//    the sample history [m][5][ns];
//  * les_fwh_pressure: the sources Q_n, L_i of every sample and their time derivatives
//    (central differences, second-order one-sided at both ends), then one block per
//    observer and group of observer times: the block's threads take the surface nodes in a
//    fixed strided order, interpolate each node's term linearly at its retarded time, and
//    the block sums the terms of each time in a fixed tree order, so the result does not
//    depend on scheduling.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "les_common.h"

using namespace lesmi;

struct les_fwh {
  les_ctx* ctx = nullptr;
  int ns = 0;            // surface nodes
  int capacity = 0;      // samples the history holds
  int count = 0;         // samples taken
  double dtau = 0.0;     // sampling interval
  int* ids = nullptr;    // [ns] flat node numbers
  double* geo = nullptr; // [7][ns]: y (3), n (3), dS
  double* hist = nullptr;  // [capacity][5][ns] rho, u, v, w, p
  double* src = nullptr;   // [capacity][7][ns] dQ_n/dtau, L (3), dL/dtau (3)
  int src_count = -1;      // samples the sources were formed from
  double src_p0 = 0.0;
  double* d_obs = nullptr;  // observer positions, times and per-(observer, time) skipped
                            // counts (as doubles) of the last call
  long long obs_cap = 0;
  std::string err;
};

namespace {

constexpr int kFwhBlock = 256;

int ffail(les_fwh* f, int code, const std::string& msg) {
  if (f) f->err = msg;
  return code;
}

#define FHIP(f, expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ffail(f, LES_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

// Surface node s: metric row (0 = S_xi, 1 = S_eta) and sign of its area vector, quadrature
// weight, and position (host-built).
struct FwhNodeSpec {
  int row;
  double sign, weight;
};

__global__ void k_fwh_geometry(long long N, int ns, const int* __restrict__ ids,
                               const int* __restrict__ rows, const double* __restrict__ signs,
                               const double* __restrict__ weights, const double* __restrict__ S,
                               double* __restrict__ geo) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  const long long o = ids[s];
  const int d = rows[s];
  const double ax = signs[s] * S[(3 * d) * N + o], ay = signs[s] * S[(3 * d + 1) * N + o],
               az = signs[s] * S[(3 * d + 2) * N + o];
  const double m = sqrt(ax * ax + ay * ay + az * az);
  const double inv = m > 0.0 ? 1.0 / m : 0.0;
  geo[3 * ns + s] = ax * inv;
  geo[4 * ns + s] = ay * inv;
  geo[5 * ns + s] = az * inv;
  geo[6 * ns + s] = m * weights[s];
}

// (rho, u, v, w, p) of the surface nodes from the state q, into one sample of the history.
__global__ void k_fwh_sample(long long N, int ns, const int* __restrict__ ids, double gamma,
                             const double* __restrict__ q, double* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  const long long o = ids[s];
  const double r = q[o];
  const double u = q[N + o] / r, v = q[2 * N + o] / r, w = q[3 * N + o] / r;
  const double p = (gamma - 1.0) * (q[4 * N + o] - 0.5 * r * (u * u + v * v + w * w));
  out[s] = r;
  out[ns + s] = u;
  out[2 * ns + s] = v;
  out[3 * ns + s] = w;
  out[4 * ns + s] = p;
}

// Sources of sample m at node s: Q_n and L_i from the sample.
__device__ __forceinline__ void fwh_sources(const double* __restrict__ hist,
                                            const double* __restrict__ geo, int ns, int m, int s,
                                            double p0, double* qn, double* L) {
  const double* h = hist + (size_t)m * 5 * ns;
  const double r = h[s], u[3] = {h[ns + s], h[2 * ns + s], h[3 * ns + s]}, p = h[4 * ns + s];
  const double n[3] = {geo[3 * ns + s], geo[4 * ns + s], geo[5 * ns + s]};
  const double un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
  *qn = r * un;
  for (int c = 0; c < 3; ++c) L[c] = (p - p0) * n[c] + r * u[c] * un;
}

// src[m][0] = dQ_n/dtau, src[m][1..3] = L, src[m][4..6] = dL/dtau at every sample and node.
__global__ void k_fwh_prepare(int ns, int M, double dtau, double p0,
                              const double* __restrict__ hist, const double* __restrict__ geo,
                              double* __restrict__ src) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)M * ns) return;
  const int m = (int)(t / ns), s = (int)(t % ns);
  double q0, L0[3], q1, L1[3], q2, L2[3];
  double* out = src + (size_t)m * 7 * ns;
  fwh_sources(hist, geo, ns, m, s, p0, &q0, L0);
  // time derivative: central inside, second-order one-sided at the first and last sample
  double dq, dL[3];
  if (m > 0 && m < M - 1) {
    fwh_sources(hist, geo, ns, m - 1, s, p0, &q1, L1);
    fwh_sources(hist, geo, ns, m + 1, s, p0, &q2, L2);
    dq = (q2 - q1) / (2.0 * dtau);
    for (int c = 0; c < 3; ++c) dL[c] = (L2[c] - L1[c]) / (2.0 * dtau);
  } else if (m == 0) {
    fwh_sources(hist, geo, ns, 1, s, p0, &q1, L1);
    fwh_sources(hist, geo, ns, 2, s, p0, &q2, L2);
    dq = (-3.0 * q0 + 4.0 * q1 - q2) / (2.0 * dtau);
    for (int c = 0; c < 3; ++c) dL[c] = (-3.0 * L0[c] + 4.0 * L1[c] - L2[c]) / (2.0 * dtau);
  } else {
    fwh_sources(hist, geo, ns, M - 2, s, p0, &q1, L1);
    fwh_sources(hist, geo, ns, M - 3, s, p0, &q2, L2);
    dq = (3.0 * q0 - 4.0 * q1 + q2) / (2.0 * dtau);
    for (int c = 0; c < 3; ++c) dL[c] = (3.0 * L0[c] - 4.0 * L1[c] + L2[c]) / (2.0 * dtau);
  }
  out[s] = dq;
  for (int c = 0; c < 3; ++c) {
    out[(1 + c) * ns + s] = L0[c];
    out[(4 + c) * ns + s] = dL[c];
  }
}

// Observer times per block of the integration kernel.
constexpr int kFwhTimes = 8;

// One block per (observer a, group of kFwhTimes consecutive observer times): p'[a][b], the
// sum of the absolute terms (scale) and the number of nodes whose retarded time lies outside
// the samples, for each time b of the group. A node's term is linear in its seven sources,
// g_m = dS (dQ_n/dtau / r + dL_r/dtau / (c0 r) + L_r / r^2) at sample m, and the linear
// interpolation at the retarded time commutes with that combination, so each thread forms
// the node's seven coefficients once and then g_m of the samples the group's retarded times
// fall between, keeping the last pair: for times a fraction of a sample apart, consecutive
// times reuse one or both values instead of gathering 14 sources each. For every (a, b) the
// nodes are summed in the same strided order and the same tree as with one block per (a, b).
__global__ void __launch_bounds__(kFwhBlock)
    k_fwh_integrate(int ns, int M, double tau0, double dtau, double c0,
                    const double* __restrict__ geo, const double* __restrict__ src,
                    const double* __restrict__ obs, int no, const double* __restrict__ times,
                    int nt, double* __restrict__ pout, double* __restrict__ scale,
                    double* __restrict__ skipped) {
  __shared__ double red[3][kFwhBlock];
  // Work item of the block: blocks are dealt to the 8 XCDs in turn (block b on XCD b % 8), so
  // each XCD takes a contiguous run of items; consecutive items share a group of observer
  // times (observer fastest), so the blocks that run together on one XCD gather the sources
  // of nearby retarded samples through its L2.
  const int nblk = gridDim.x, full = nblk / 8 * 8;
  const int item = (int)blockIdx.x >= full ? (int)blockIdx.x
                                           : (blockIdx.x % 8) * (full / 8) + blockIdx.x / 8;
  const int a = item % no, b0 = (item / no) * kFwhTimes;
  const int nb = nt - b0 < kFwhTimes ? nt - b0 : kFwhTimes;
  const double x = obs[3 * a], y = obs[3 * a + 1], z = obs[3 * a + 2];
  double tb[kFwhTimes], sum[kFwhTimes], abs_sum[kFwhTimes];
  int skip[kFwhTimes];
#pragma unroll
  for (int u = 0; u < kFwhTimes; ++u) {
    tb[u] = u < nb ? times[b0 + u] : 0.0;
    sum[u] = abs_sum[u] = 0.0;
    skip[u] = 0;
  }
  const double ic0 = 1.0 / c0;
  for (int s = threadIdx.x; s < ns; s += kFwhBlock) {
    const double dx = x - geo[s], dy = y - geo[ns + s], dz = z - geo[2 * ns + s];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    const double ir = 1.0 / r;
    const double rc = r / c0;  // the retarded time is formed as the oracle forms it
    const double area = geo[6 * ns + s];
    // g_m = cq dQ_n/dtau + cl . L + cd . dL/dtau
    const double cq = area * ir, cr2 = cq * ir, ccr = cq * ic0;
    const double rh[3] = {dx * ir, dy * ir, dz * ir};
    const double cl[3] = {cr2 * rh[0], cr2 * rh[1], cr2 * rh[2]};
    const double cd[3] = {ccr * rh[0], ccr * rh[1], ccr * rh[2]};
    auto g_at = [&](int m) {
      const double* sm = src + (size_t)m * 7 * ns + s;
      double g = cq * sm[0];
#pragma unroll
      for (int c = 0; c < 3; ++c) g = fma(cl[c], sm[(1 + c) * ns], g);
#pragma unroll
      for (int c = 0; c < 3; ++c) g = fma(cd[c], sm[(4 + c) * ns], g);
      return g;
    };
    // Interval m_u and weight of each time of the group (the same division and floor as
    // one time at a time, so the interval decisions do not depend on the grouping).
    double wt[kFwhTimes];
    int mu[kFwhTimes];
    bool ok[kFwhTimes];
#pragma unroll
    for (int u = 0; u < kFwhTimes; ++u) {
      const double sm = (tb[u] - rc - tau0) / dtau;
      int m = (int)floor(sm);
      bool in = u < nb && m >= 0 && m + 1 <= M - 1;
      if (u < nb && m == M - 1 && sm == (double)(M - 1)) {  // exactly on the last sample
        m = M - 2;
        in = true;
      }
      ok[u] = in;
      mu[u] = in ? m : 0;
      wt[u] = in ? sm - m : 0.0;
    }
    // Regular node: every retarded time inside the samples from the first on, each at most
    // one interval past the previous one (times less than a sample apart, in order). Then
    // g at m_0 and at m_u + 1 for every u are all the values needed, and their loads do not
    // wait on one another.
    bool regular = true;
#pragma unroll
    for (int u = 1; u < kFwhTimes; ++u) {
      const int d = mu[u] - mu[u - 1];
      if (ok[u] && (!ok[u - 1] || d < 0 || d > 1)) regular = false;
    }
    if (regular) {
      // Row m_u + 1 is gathered only by the lanes whose interval changed at u (the others
      // take g_{m_u + 1} from u - 1): all gathers are issued before any of them is used.
      double v[kFwhTimes][7], gn[kFwhTimes];
      const double g0 = g_at(mu[0]);
#pragma unroll
      for (int u = 0; u < kFwhTimes; ++u)
        if (u == 0 || mu[u] != mu[u - 1]) {
          const double* sm = src + (size_t)(mu[u] + 1) * 7 * ns + s;
#pragma unroll
          for (int c = 0; c < 7; ++c) v[u][c] = sm[(size_t)c * ns];
        }
#pragma unroll
      for (int u = 0; u < kFwhTimes; ++u) {
        if (u == 0 || mu[u] != mu[u - 1]) {
          double g = cq * v[u][0];
#pragma unroll
          for (int c = 0; c < 3; ++c) g = fma(cl[c], v[u][1 + c], g);
#pragma unroll
          for (int c = 0; c < 3; ++c) g = fma(cd[c], v[u][4 + c], g);
          gn[u] = g;
        } else {
          gn[u] = gn[u - 1];
        }
      }
      double g_lo = g0;
#pragma unroll
      for (int u = 0; u < kFwhTimes; ++u) {
        if (u > 0 && mu[u] == mu[u - 1] + 1) g_lo = gn[u - 1];
        const double term = (1.0 - wt[u]) * g_lo + wt[u] * gn[u];
        if (ok[u]) {
          sum[u] += term;
          abs_sum[u] += fabs(term);
        } else if (u < nb) {
          skip[u] += 1;
        }
      }
    } else {  // times out of order, far apart or partly outside: the last pair is kept
      int cm = -2;  // g_lo = g_cm, g_hi = g_{cm+1}
      double g_lo = 0.0, g_hi = 0.0;
#pragma unroll
      for (int u = 0; u < kFwhTimes; ++u) {
        if (u >= nb) break;
        if (!ok[u]) {
          skip[u] += 1;
          continue;
        }
        const int m = mu[u];
        if (m != cm) {
          const double lo = m == cm + 1 ? g_hi : g_at(m);
          g_hi = g_at(m + 1);
          g_lo = lo;
          cm = m;
        }
        const double term = (1.0 - wt[u]) * g_lo + wt[u] * g_hi;
        sum[u] += term;
        abs_sum[u] += fabs(term);
      }
    }
  }
  const double k = 1.0 / (4.0 * M_PI);
  for (int u = 0; u < nb; ++u) {
    red[0][threadIdx.x] = sum[u];
    red[1][threadIdx.x] = abs_sum[u];
    red[2][threadIdx.x] = (double)skip[u];
    __syncthreads();
    for (int h = kFwhBlock / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h)
        for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const size_t o = (size_t)a * nt + b0 + u;
      pout[o] = red[0][0] * k;
      if (scale) scale[o] = red[1][0] * k;
      skipped[o] = red[2][0];
    }
    __syncthreads();
  }
}

void free_fwh(les_fwh* f) {
  void* ptrs[] = {f->ids, f->geo, f->hist, f->src, f->d_obs};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

}  // namespace

extern "C" {

int les_fwh_create(les_ctx* ctx, const double* xyz, int i1, int i2, int js, int caps,
                   int capacity, double dtau, les_fwh** out) {
  if (!out) return LES_EINVAL;
  *out = nullptr;
  if (!ctx || !xyz || capacity < 3 || !(dtau > 0.0)) return LES_EINVAL;
  const Dims& D = ctx->dims;
  if (!D.jet) return LES_EINVAL;
  const int ni = D.n[0], nj = D.n[1], nk = D.n[2];
  if (i1 < 0 || i2 <= i1 || i2 > ni - 1 || js < 1 || js > nj - 1 || caps < 0 || caps > 3)
    return LES_EINVAL;
  les_fwh* f = new (std::nothrow) les_fwh();
  if (!f) return LES_ENOMEM;
  *out = f;
  f->ctx = ctx;
  f->capacity = capacity;
  f->dtau = dtau;
  // Nodes: lateral (k, then i), upstream cap (k, then j), downstream cap (k, then j).
  std::vector<int> ids, rows;
  std::vector<double> signs, weights;
  for (int k = 0; k < nk; ++k)
    for (int i = i1; i <= i2; ++i) {
      ids.push_back(i + ni * (js + nj * k));
      rows.push_back(1);
      signs.push_back(1.0);
      weights.push_back(i == i1 || i == i2 ? 0.5 : 1.0);
    }
  for (int cap = 0; cap < 2; ++cap) {
    if (!(caps & (1 << cap))) continue;
    const int i = cap == 0 ? i1 : i2;
    for (int k = 0; k < nk; ++k)
      for (int j = 0; j <= js; ++j) {
        ids.push_back(i + ni * (j + nj * k));
        rows.push_back(0);
        signs.push_back(cap == 0 ? -1.0 : 1.0);
        weights.push_back(j == js ? 0.5 : 1.0);
      }
  }
  const int ns = (int)ids.size();
  f->ns = ns;
  std::vector<double> pos(3 * (size_t)ns);
  for (int s = 0; s < ns; ++s)
    for (int c = 0; c < 3; ++c) pos[(size_t)c * ns + s] = xyz[(size_t)c * D.N + ids[s]];
  int* d_rows = nullptr;
  double *d_signs = nullptr, *d_w = nullptr;
  auto bail = [&](int code, const char* msg) {
    if (d_rows) (void)hipFree(d_rows);
    if (d_signs) (void)hipFree(d_signs);
    if (d_w) (void)hipFree(d_w);
    return ffail(f, code, msg);
  };
  if (hipMalloc((void**)&f->ids, sizeof(int) * ns) != hipSuccess ||
      hipMalloc((void**)&f->geo, sizeof(double) * 7 * ns) != hipSuccess ||
      hipMalloc((void**)&f->hist, sizeof(double) * 5 * ns * (size_t)capacity) != hipSuccess ||
      hipMalloc((void**)&f->src, sizeof(double) * 7 * ns * (size_t)capacity) != hipSuccess ||
      hipMalloc((void**)&d_rows, sizeof(int) * ns) != hipSuccess ||
      hipMalloc((void**)&d_signs, sizeof(double) * ns) != hipSuccess ||
      hipMalloc((void**)&d_w, sizeof(double) * ns) != hipSuccess)
    return bail(LES_ENOMEM, "hipMalloc");
  if (hipMemcpy(f->ids, ids.data(), sizeof(int) * ns, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d_rows, rows.data(), sizeof(int) * ns, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d_signs, signs.data(), sizeof(double) * ns, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d_w, weights.data(), sizeof(double) * ns, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(f->geo, pos.data(), sizeof(double) * 3 * ns, hipMemcpyHostToDevice) != hipSuccess)
    return bail(LES_EHIP, "hipMemcpy");
  hipLaunchKernelGGL(k_fwh_geometry, dim3((ns + 255) / 256), dim3(256), 0, 0, D.N, ns, f->ids,
                     d_rows, d_signs, d_w, ctx->S, f->geo);
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess)
    return bail(LES_EHIP, "surface geometry kernel");
  (void)hipFree(d_rows);
  (void)hipFree(d_signs);
  (void)hipFree(d_w);
  d_rows = nullptr;
  d_signs = d_w = nullptr;
  return LES_OK;
}

int les_fwh_nodes(const les_fwh* f) { return f ? f->ns : 0; }

int les_fwh_samples(const les_fwh* f) { return f ? f->count : 0; }

int les_fwh_geometry(les_fwh* f, double* geo, void* stream) {
  if (!f || !geo) return ffail(f, LES_EINVAL, "null argument");
  FHIP(f, hipMemcpyAsync(geo, f->geo, sizeof(double) * 7 * f->ns, hipMemcpyDeviceToDevice,
                         (hipStream_t)stream));
  return LES_OK;
}

int les_fwh_sample(les_fwh* f, const double* q, void* stream) {
  if (!f || !q) return ffail(f, LES_EINVAL, "null argument");
  if (f->count >= f->capacity) return ffail(f, LES_ESTATE, "sample history is full");
  const Dims& D = f->ctx->dims;
  hipLaunchKernelGGL(k_fwh_sample, dim3((f->ns + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                     D.N, f->ns, f->ids, f->ctx->params.gamma, q,
                     f->hist + (size_t)f->count * 5 * f->ns);
  if (hipGetLastError() != hipSuccess) return ffail(f, LES_EHIP, "sample kernel");
  f->count += 1;
  return LES_OK;
}

int les_fwh_reset(les_fwh* f) {
  if (!f) return LES_EINVAL;
  f->count = 0;
  f->src_count = -1;
  return LES_OK;
}

int les_fwh_pressure(les_fwh* f, const double* observers, int no, const double* times, int nt,
                     double c0, double p0, double tau0, double* p_out, double* scale_out,
                     long long* skipped, void* stream) {
  if (!f || !observers || !times || !p_out || no < 1 || nt < 1 || !(c0 > 0.0))
    return ffail(f, LES_EINVAL, "bad argument");
  if (f->count < 3) return ffail(f, LES_ESTATE, "fewer than three samples");
  hipStream_t s = (hipStream_t)stream;
  const int M = f->count, ns = f->ns;
  if (f->src_count != M || f->src_p0 != p0) {
    const long long n = (long long)M * ns;
    hipLaunchKernelGGL(k_fwh_prepare, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ns, M,
                       f->dtau, p0, f->hist, f->geo, f->src);
    if (hipGetLastError() != hipSuccess) return ffail(f, LES_EHIP, "source kernel");
    f->src_count = M;
    f->src_p0 = p0;
  }
  const long long need = 3LL * no + nt + (long long)no * nt;
  if (need > (1LL << 28)) return ffail(f, LES_EINVAL, "too many observers x times");
  if (need > f->obs_cap) {
    if (f->d_obs) (void)hipFree(f->d_obs);
    f->d_obs = nullptr;
    f->obs_cap = 0;
    FHIP(f, hipMalloc((void**)&f->d_obs, sizeof(double) * need));
    f->obs_cap = need;
  }
  double* d_o = f->d_obs;
  double* d_t = d_o + 3 * no;
  double* d_skip = d_t + nt;
  FHIP(f, hipMemcpyAsync(d_o, observers, sizeof(double) * 3 * no, hipMemcpyHostToDevice, s));
  FHIP(f, hipMemcpyAsync(d_t, times, sizeof(double) * nt, hipMemcpyHostToDevice, s));
  const long long blocks = (long long)no * ((nt + kFwhTimes - 1) / kFwhTimes);
  if (blocks > 0x7fffffffLL) return ffail(f, LES_EINVAL, "too many observers x times");
  hipLaunchKernelGGL(k_fwh_integrate, dim3((unsigned)blocks), dim3(kFwhBlock), 0, s, ns, M, tau0,
                     f->dtau, c0, f->geo, f->src, d_o, no, d_t, nt, p_out, scale_out, d_skip);
  if (hipGetLastError() != hipSuccess) return ffail(f, LES_EHIP, "integration kernel");
  std::vector<double> sk((size_t)no * nt);
  FHIP(f, hipMemcpyAsync(sk.data(), d_skip, sizeof(double) * no * nt, hipMemcpyDeviceToHost, s));
  FHIP(f, hipStreamSynchronize(s));
  if (skipped) {
    long long tot = 0;
    for (double v : sk) tot += (long long)v;
    *skipped = tot;
  }
  return LES_OK;
}

void les_fwh_destroy(les_fwh* f) {
  if (!f) return;
  (void)hipDeviceSynchronize();
  free_fwh(f);
  delete f;
}

const char* les_fwh_last_error(const les_fwh* f) { return f ? f->err.c_str() : "null surface"; }

}  // extern "C"
