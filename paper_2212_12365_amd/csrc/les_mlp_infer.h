// Inference of the learned closure's network on gfx950, shared by les_mlp.hip (the
// inference kernel) and the node kernel (the closure evaluated where the features are
// formed). Matrix products use v_mfma_f32_16x16x32_bf16 (FP32 accumulate) with each operand
// split into two BF16 parts (three products per matrix product, about 16 significant bits).
// Fragments, per lane l of a wave (g = l / 16, s = l % 16): A (16 x 32) holds row s,
// k = 8g .. 8g+7; B (32 x 16) holds column s, k = 8g .. 8g+7; the 16 x 16 result holds
// column s, rows 4g .. 4g+3. The network is evaluated transposed: hidden units are rows and
// samples columns, so each lane owns one sample and, per 16-unit tile, four hidden units.
#pragma once

#include <hip/hip_runtime.h>

#include "les_mlp.h"

namespace lesmi {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int HS = 72;  // LDS stride (bf16) of a sample-major row of 64 hidden values

constexpr float kG0 = 0.7978845608028654f;  // sqrt(2/pi)
constexpr float kG1 = 0.044715f;

__device__ __forceinline__ f32x4 mfma16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// GELU in its tanh form, written through 0.5 (1 + tanh y) = 1 / (1 + exp(-2y)) with the
// hardware exponential and reciprocal (v_exp_f32, v_rcp_f32: about 1 ulp each, far below the
// BF16 rounding of the products): gelu(x) = x s, s = 1 / (1 + exp(-2 k0 (x + k1 x^3))).
// With exp(-2y) = 2^(x (c1 + c2 x^2)), c1 = -2 k0 log2(e), c2 = c1 k1, the sigmoid takes a
// square, one fused multiply-add, a product, the base-2 exponential and a reciprocal.
constexpr float kGc1 = -2.f * kG0 * 1.4426950408889634f;
constexpr float kGc2 = kGc1 * kG1;
__device__ __forceinline__ float gelu_sig(float x) {
  const float u = __builtin_fmaf(kGc2, x * x, kGc1);
  return __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(x * u));
}

__device__ __forceinline__ float gelu_f(float x) { return x * gelu_sig(x); }

__device__ __forceinline__ float softplus_f(float z) {
  return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z)));
}

// Split of an FP32 value into two BF16 parts hi + lo (hi = v rounded, lo = the rounded
// remainder): products of split operands taken as hi*hi + hi*lo + lo*hi carry about 16
// significant bits instead of 8.
__device__ __forceinline__ void split_bf16(float v, __bf16& hi, __bf16& lo) {
  hi = (__bf16)v;
  lo = (__bf16)(v - (float)hi);
}

__device__ __forceinline__ void split_frag(const float* v, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    __bf16 h, l;
    split_bf16(v[i], h, l);
    hi[i] = h;
    lo[i] = l;
  }
}

__device__ __forceinline__ void w1_frag_split(const float* __restrict__ th, int t, int lane,
                                              bf16x8& hi, bf16x8& lo) {
  const int g = lane >> 4, r = 16 * t + (lane & 15);
  float v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = (g == 0 && i < kMlpIn) ? th[kOffW1 + r * kMlpIn + i] : 0.f;
  split_frag(v, hi, lo);
}

__device__ __forceinline__ void w2_frag_split(const float* __restrict__ th, int t, int kb,
                                              int lane, bf16x8& hi, bf16x8& lo) {
  const int r = 16 * t + (lane & 15), k0 = 32 * kb + 8 * (lane >> 4);
  float v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = th[kOffW2 + r * kMlpH + k0 + i];
  split_frag(v, hi, lo);
}

// Normalised inputs x of one sample and whether the network applies there.
__device__ __forceinline__ bool mlp_input(const MlpNet& net, const float* f, float pos,
                                          float* x) {
  bool ok = pos > 0.f && isfinite(pos);
#pragma unroll
  for (int c = 0; c < kMlpIn; ++c) {
    const float v = f[c];
    const bool fin = isfinite(v);
    ok = ok && fin && v >= net.norm.lo[c] && v <= net.norm.hi[c];
    x[c] = ((fin ? v : 0.f) - net.norm.mean[c]) * net.norm.inv_std[c];
  }
  return ok;
}

// The forward pass of the 16 samples of a wave (sample s in lanes s, s+16, s+32, s+48,
// inputs x from lanes 0..15) with split-BF16 products (three MFMAs per product: hi*hi,
// hi*lo, lo*hi): w1h/w1l, w2h/w2l are the split weights, H and Hl the split h1.
// The wave's own LDS rows carry h1 from layer 1 to layer 2; LDS operations of one wave
// complete in order, so a wave-scope fence (which waits for the writes) replaces a block
// barrier. bs holds b1, b2, w3 and b3 in LDS.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float forward16_split(const float* bs,
                                                 const bf16x8 (&w1h)[4], const bf16x8 (&w1l)[4],
                                                 const bf16x8 (&w2h)[4][2],
                                                 const bf16x8 (&w2l)[4][2], const float* x,
                                                 int lane, __bf16* H, __bf16* Hl) {
  const int g = lane >> 4, s = lane & 15;
  float xv[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) xv[i] = (g == 0 && i < kMlpIn) ? x[i] : 0.f;
  bf16x8 bxh, bxl;
  split_frag(xv, bxh, bxl);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    // The bias seeds the accumulator.
    f32x4 a = mfma16(w1l[t], bxh, *(const f32x4*)&bs[16 * t + 4 * g]);
    a = mfma16(w1h[t], bxl, a);
    a = mfma16(w1h[t], bxh, a);
    bf16x4 hh, hl;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      __bf16 p, q;
      split_bf16(gelu_f(a[i]), p, q);
      hh[i] = p;
      hl[i] = q;
    }
    *(bf16x4*)&H[s * HS + 16 * t + 4 * g] = hh;
    *(bf16x4*)&Hl[s * HS + 16 * t + 4 * g] = hl;
  }
  wave_lds_fence();
  float z = 0.f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = *(const f32x4*)&bs[64 + 16 * t + 4 * g];  // the bias seeds the accumulator
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      const bf16x8 bh = *(const bf16x8*)&H[s * HS + 32 * kb + 8 * g];
      const bf16x8 bl = *(const bf16x8*)&Hl[s * HS + 32 * kb + 8 * g];
      acc = mfma16(w2l[t][kb], bh, acc);
      acc = mfma16(w2h[t][kb], bl, acc);
      acc = mfma16(w2h[t][kb], bh, acc);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) z += bs[128 + 16 * t + 4 * g + i] * gelu_f(acc[i]);
  }
  z += __shfl_xor(z, 16);
  z += __shfl_xor(z, 32);
  wave_lds_fence();  // this tile's reads of H end before the next tile writes it
  return z + bs[192];
}


// The inference weights as per-lane fragments in LDS, for kernels that cannot hold them in
// registers: F[f * 64 + lane], f = t (W1 hi), 4 + t (W1 lo), 8 + 2t + kb (W2 hi),
// 16 + 2t + kb (W2 lo), t = 0..3, kb = 0..1 (24 fragments, 24 KB).
constexpr int kInferFrags = 24;

// Wave `wave` of `nwaves` builds its share of the fragments for its own lane.
__device__ __forceinline__ void infer_frags_to_lds(const float* __restrict__ th, bf16x8* F,
                                                   int wave, int nwaves, int lane) {
  for (int p = wave; p < 12; p += nwaves) {  // 4 (t) W1 pairs, then 8 (t, kb) W2 pairs
    bf16x8 hi, lo;
    if (p < 4) {
      w1_frag_split(th, p, lane, hi, lo);
      F[p * 64 + lane] = hi;
      F[(4 + p) * 64 + lane] = lo;
    } else {
      const int t = (p - 4) >> 1, kb = (p - 4) & 1;
      w2_frag_split(th, t, kb, lane, hi, lo);
      F[(8 + 2 * t + kb) * 64 + lane] = hi;
      F[(16 + 2 * t + kb) * 64 + lane] = lo;
    }
  }
}

// forward16_split with the weight fragments read from LDS at the point of use: the same
// products in the same order, so the same z.
__device__ __forceinline__ float forward16_split_lds(const float* bs, const bf16x8* F,
                                                     const float* x, int lane, __bf16* H,
                                                     __bf16* Hl) {
  const int g = lane >> 4, s = lane & 15;
  float xv[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) xv[i] = (g == 0 && i < kMlpIn) ? x[i] : 0.f;
  bf16x8 bxh, bxl;
  split_frag(xv, bxh, bxl);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const bf16x8 w1h = F[t * 64 + lane], w1l = F[(4 + t) * 64 + lane];
    f32x4 a = mfma16(w1l, bxh, *(const f32x4*)&bs[16 * t + 4 * g]);
    a = mfma16(w1h, bxl, a);
    a = mfma16(w1h, bxh, a);
    bf16x4 hh, hl;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      __bf16 p, q;
      split_bf16(gelu_f(a[i]), p, q);
      hh[i] = p;
      hl[i] = q;
    }
    *(bf16x4*)&H[s * HS + 16 * t + 4 * g] = hh;
    *(bf16x4*)&Hl[s * HS + 16 * t + 4 * g] = hl;
  }
  wave_lds_fence();
  float z = 0.f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = *(const f32x4*)&bs[64 + 16 * t + 4 * g];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      const bf16x8 bh = *(const bf16x8*)&H[s * HS + 32 * kb + 8 * g];
      const bf16x8 bl = *(const bf16x8*)&Hl[s * HS + 32 * kb + 8 * g];
      const bf16x8 w2h = F[(8 + 2 * t + kb) * 64 + lane], w2l = F[(16 + 2 * t + kb) * 64 + lane];
      acc = mfma16(w2l, bh, acc);
      acc = mfma16(w2h, bl, acc);
      acc = mfma16(w2h, bh, acc);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) z += bs[128 + 16 * t + 4 * g + i] * gelu_f(acc[i]);
  }
  z += __shfl_xor(z, 16);
  z += __shfl_xor(z, 32);
  wave_lds_fence();
  return z + bs[192];
}

}  // namespace lesmi
