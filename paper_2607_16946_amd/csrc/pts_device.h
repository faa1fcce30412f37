// pts_device.h -- device helpers shared by the evaluation and gradient sweeps.
#pragma once

#include "pts_internal.h"

namespace pts {

__device__ __forceinline__ float hw_sqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ float hw_exp2(float v) { return __builtin_amdgcn_exp2f(v); }
__device__ __forceinline__ float hw_rcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ float hw_rsq(float v) { return __builtin_amdgcn_rsqf(v); }

// 1/sqrt(v) for v > 1e-30, else 0.  With it, v * safe_rsq(v) is sqrt(v) (0 for
// v <= 1e-30, i.e. below 1e-15) and a factor 1/sqrt(v) it supplies vanishes
// there (the subgradient convention at a torus's axis, its core circle and a
// query on a point): one transcendental gives a length and its reciprocal.
// The cut stays clear of FP32 denormals, which the hardware flushes to 0.
__device__ __forceinline__ float safe_rsq(float v) { return v > 1e-30f ? hw_rsq(v) : 0.f; }

struct QueryIn {
  float x, y, z;
  bool valid;
};

// Query q relative to the cloud origin (record coordinates).
__device__ __forceinline__ QueryIn load_query(const float* __restrict__ x, int64_t q, int64_t Q, const Header* h) {
  QueryIn r{0.f, 0.f, 0.f, false};
  if (q < Q) {
    r.x = x[3 * q] - h->origin[0];
    r.y = x[3 * q + 1] - h->origin[1];
    r.z = x[3 * q + 2] - h->origin[2];
    r.valid = true;
  }
  return r;
}

// Split-major order of a sweep's workgroups over S point splits (S a
// multiple of 8 and above 8).  The dispatcher places consecutive workgroups
// on consecutive XCDs (8 of them), so with workgroup b taking split
// b % 8 + 8 (b / 8 / nqb) and query block b / 8 % nqb, XCD k runs splits k,
// k + 8, ... one after the other, each for every query block: its resident
// workgroups then read one split's records, which stay in that XCD's L2.
// Sweeps with fewer splits take split b % S and query block b / S, which for
// S = 8 is the same order; they do so in code of their own (a template
// flag), as hipcc schedules the pair loop worse when this mapping precedes
// it (2% on the blend, 10% on the gradient sweep, measured).
__host__ __device__ __forceinline__ bool split_major(int S) { return S > 8 && S % 8 == 0; }

__device__ __forceinline__ void split_block(int S, int& split, int64_t& qb) {
  // a grid holds fewer than 2^32 workgroups: 32-bit arithmetic throughout
  const unsigned b = blockIdx.x, nqb = gridDim.x / unsigned(S), i = b / 8u;
  split = int(b % 8u + 8u * (i / nqb));
  qb = int64_t(i % nqb);
}

// M and -lambda' = -lambda log2(e) of a query from the per-split maxima of
// |x - p|^2 (Eq. RelationshipBetweenLambdaAndRadius: lambda_x = 2C/M).
__device__ __forceinline__ void far_of(const float* __restrict__ far2, int S, int64_t Q, int64_t q, float C2,
                                       float& M, float& nlam) {
  float m2 = -3.0e38f;
  for (int s = 0; s < S; ++s) m2 = fmaxf(m2, far2[int64_t(s) * Q + q]);
  M = sqrtf(fmaxf(m2, 0.f));
  // with M = 0 every point sits at the query and the weights are uniform
  nlam = M > 0.f ? -2.f * C2 / M : 0.f;
}

// One pair, direct torus form: <x-c,.> from stored dot products, then
// rho = |((x-c).m, (x-c).k)|, |q| = |(rho - R, (x-c).u)|, g = sign (|q| - r)
// (Eq. SingleTorusSDF and the sign of Eq. TorusSigns).
__device__ __forceinline__ float g_direct(float x, float y, float z, const float4& U, const float4& Mv,
                                          const float4& K, const float4& G) {
  const float vu = fmaf(z, U.z, fmaf(y, U.y, fmaf(x, U.x, U.w)));
  const float vm = fmaf(z, Mv.z, fmaf(y, Mv.y, fmaf(x, Mv.x, Mv.w)));
  const float vk = fmaf(z, K.z, fmaf(y, K.y, fmaf(x, K.x, K.w)));
  const float rho = hw_sqrt(fmaf(vm, vm, vk * vk));
  const float b = rho - G.x;
  const float qn = hw_sqrt(fmaf(b, b, vu * vu));
  return fmaf(G.z, qn, G.w);
}

// One pair, anchored form for large radii L (nearly flat directions): with
// y = x - o and t = y.m + L (= (x-c).m),
//   rho - L = alpha / (rho + L),  alpha = y.m (t + L) + (y.k)^2,
//   rho - R = (rho - L) + zeta r,
//   |q| - r = ((rho-L)(rho-L + 2 zeta r) + (y.u)^2) / (|q| + r),
// which avoids subtracting quantities of size L (and r).
__device__ __forceinline__ float g_anchored(float x, float y, float z, float L, const float4& U,
                                            const float4& Mv, const float4& K, const float4& G) {
  const float yu = fmaf(z, U.z, fmaf(y, U.y, fmaf(x, U.x, U.w)));
  const float ym = fmaf(z, Mv.z, fmaf(y, Mv.y, fmaf(x, Mv.x, Mv.w)));
  const float yk = fmaf(z, K.z, fmaf(y, K.y, fmaf(x, K.x, K.w)));
  const float t = ym + L;
  const float yk2 = yk * yk;
  const float rho = hw_sqrt(fmaf(t, t, yk2));
  const float alpha = fmaf(ym, t + L, yk2);
  const float beta = alpha * hw_rcp(rho + L);
  const float b = beta + G.y;
  const float yu2 = yu * yu;
  const float qn = hw_sqrt(fmaf(b, b, yu2));
  const float num = fmaf(beta, b + G.y, yu2);
  const float den = fmaf(G.z, qn, -G.w);   // sign (|q| + r)
  return num * hw_rcp(den);
}

// Torus quantities of one pair needed by the derivatives: g, the components
// (vu, vm, vk) of x - c in the frame (u, m, k), rho, b = rho - R, |q|^2, |q|,
// and 1/rho, 1/|q| (0 where rho, |q| vanish; rho and |q| from safe_rsq).
struct Geo {
  float g, vu, vm, vk, rho, b, qn2, qn, irho, iqn;
};

__device__ __forceinline__ Geo geo_direct(float x, float y, float z, const float4& U, const float4& Mv,
                                          const float4& K, const float4& G) {
  Geo r;
  r.vu = fmaf(z, U.z, fmaf(y, U.y, fmaf(x, U.x, U.w)));
  r.vm = fmaf(z, Mv.z, fmaf(y, Mv.y, fmaf(x, Mv.x, Mv.w)));
  r.vk = fmaf(z, K.z, fmaf(y, K.y, fmaf(x, K.x, K.w)));
  const float rho2 = fmaf(r.vm, r.vm, r.vk * r.vk);
  r.irho = safe_rsq(rho2);
  r.rho = rho2 * r.irho;
  r.b = r.rho - G.x;
  r.qn2 = fmaf(r.b, r.b, r.vu * r.vu);
  r.iqn = safe_rsq(r.qn2);
  r.qn = r.qn2 * r.iqn;
  r.g = fmaf(G.z, r.qn, G.w);
  return r;
}

__device__ __forceinline__ Geo geo_anchored(float x, float y, float z, float L, const float4& U, const float4& Mv,
                                            const float4& K, const float4& G) {
  Geo r;
  r.vu = fmaf(z, U.z, fmaf(y, U.y, fmaf(x, U.x, U.w)));
  const float ym = fmaf(z, Mv.z, fmaf(y, Mv.y, fmaf(x, Mv.x, Mv.w)));
  r.vk = fmaf(z, K.z, fmaf(y, K.y, fmaf(x, K.x, K.w)));
  r.vm = ym + L;
  const float yk2 = r.vk * r.vk;
  const float rho2 = fmaf(r.vm, r.vm, yk2);
  r.irho = safe_rsq(rho2);
  r.rho = rho2 * r.irho;
  const float alpha = fmaf(ym, r.vm + L, yk2);
  const float beta = alpha * hw_rcp(r.rho + L);
  r.b = beta + G.y;
  const float yu2 = r.vu * r.vu;
  r.qn2 = fmaf(r.b, r.b, yu2);
  r.iqn = safe_rsq(r.qn2);
  r.qn = r.qn2 * r.iqn;
  const float num = fmaf(beta, r.b + G.y, yu2);
  r.g = num * hw_rcp(fmaf(G.z, r.qn, -G.w));
  return r;
}

// A query's S split partials (sum w g, sum w) summed in a fixed order: in
// split order by one lane (combine_seq), or by one wavefront (combine_wave),
// lane l summing splits l, l + 64, ... in order, then a butterfly over the 64
// lane sums (each step adds a pair of values in both lanes of the pair, and
// addition is commutative, so every lane ends with the same bits).  Every
// lane of the wave calls combine_wave; lanes with q >= Q only contribute 0.
__device__ __forceinline__ float2 combine_seq(const float2* __restrict__ part, int S, int64_t Q, int64_t q) {
  float num = 0.f, den = 0.f;
  for (int s = 0; s < S; ++s) {
    const float2 v = part[int64_t(s) * Q + q];
    num += v.x;
    den += v.y;
  }
  return make_float2(num, den);
}

__device__ __forceinline__ float2 combine_wave(const float2* __restrict__ part, int S, int64_t Q, int64_t q,
                                               int lane) {
  float num = 0.f, den = 0.f;
  if (q < Q)
    for (int s = lane; s < S; s += 64) {
      const float2 v = part[int64_t(s) * Q + q];
      num += v.x;
      den += v.y;
    }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    num += __shfl_xor(num, o, 64);
    den += __shfl_xor(den, o, 64);
  }
  return make_float2(num, den);
}

// Fold of a query's S per-split maxima into row 0 of far2 (exact in any
// order; a NaN row 0 stays NaN, as the comparisons v > m never take a value
// over it): by one lane, or, for many rows, by one wavefront (lane l taking
// rows l, l + 64, ..., lane 0 starting from row 0, then a butterfly); only
// lane 0 of the wave holds the result.
__device__ __forceinline__ float fold_seq(const float* __restrict__ far2, int S, int64_t Q, int64_t q) {
  float m = far2[q];
  for (int s = 1; s < S; ++s) {
    const float v = far2[int64_t(s) * Q + q];
    m = v > m ? v : m;
  }
  return m;
}

__device__ __forceinline__ float fold_wave(const float* __restrict__ far2, int S, int64_t Q, int64_t q, int lane) {
  float m = -3.0e38f;
  if (q < Q) {
    if (lane == 0) m = far2[q];
    for (int s = lane == 0 ? 64 : lane; s < S; s += 64) {
      const float v = far2[int64_t(s) * Q + q];
      m = v > m ? v : m;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const float v = __shfl_xor(m, o, 64);
    m = v > m ? v : m;
  }
  return m;
}

// 1/v, or 0 where v is 0 (the derivative factors it scales vanish there; a
// subgradient on the torus axis, its core circle, and at the points).
__device__ __forceinline__ float safe_rcp(float v) { return v > 0.f ? hw_rcp(v) : 0.f; }

}  // namespace pts
