// pts_eval.hip -- inference stage of Algorithm 1 on gfx950 (Sec. 4.2).
//
//   phi(x) = sum_i g_i(x) w_i / sum_i w_i,  w_i = exp(-lambda_x (|x-p_i| - sigma_x)),
//   sigma_x = M/2, lambda_x = C/sigma_x = 2C/M, M = max_i |x - p_i|
//   (Eqs. BasicFormulaShifted, RelationshipBetweenLambdaAndRadius).
//
// lambda_x is only known once the farthest point is, so each query takes two
// sweeps over the points: k_far (M) and k_blend (the weighted sums).  Both use
// one query per lane (qpl queries per lane), point tiles staged in LDS and
// read by every lane at the same address (broadcast), and FP32 VALU math with
// the hardware square root / exp2 / reciprocal.  There is no matrix-core work:
// nothing here is a dense contraction.
//
// The point range is split S ways.  Workgroup b handles split b % S of query
// block b / S; dispatch places consecutive workgroups on consecutive XCDs, so
// with S a multiple of 8 each XCD only ever reads its own slice of the
// records, which then stays resident in that XCD's L2.  Partial results of the
// splits are combined in a fixed order (k_combine), so results are
// deterministic and depend on S only through rounding.
//
// Weights are computed with the shift of Eq. (BasicFormulaShifted):
//   w = 2^(C log2e - lambda_x log2e |x - p|)  in [2^-C log2e, 2^C log2e],
// and the sums are accumulated per tile and then per split (two-level), which
// bounds FP32 accumulation error by ~(tile + N/(S tile)) ulp.

#include "pts_internal.h"

namespace pts {
namespace {

__device__ __forceinline__ float hw_sqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ float hw_exp2(float v) { return __builtin_amdgcn_exp2f(v); }
__device__ __forceinline__ float hw_rcp(float v) { return __builtin_amdgcn_rcpf(v); }

struct QueryIn {
  float x, y, z;
  bool valid;
};

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

// ---------------------------------------------------------------------------
// Sweep 1: squared distance to the farthest point, per split.
//   |x-p|^2 = |x|^2 + |p|^2 - 2<x,p>; the max is taken over (|p|^2 - 2<x,p>)
//   (three FMAs and a max per pair) and |x|^2 is added once at the end.
// ---------------------------------------------------------------------------
template <int QPL>
__global__ __launch_bounds__(kBlock) void k_far(const Header* __restrict__ h, const float4* __restrict__ pos4,
                                                const float* __restrict__ x, int64_t Q, int S, int64_t per_split,
                                                float* __restrict__ far2) {
  __shared__ float4 tile[kTile1];
  const int split = int(blockIdx.x % unsigned(S));
  const int64_t qb = blockIdx.x / unsigned(S);
  const int64_t N = h->N;
  float qx[QPL], qy[QPL], qz[QPL], acc[QPL];
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    QueryIn qi = load_query(x, qb * (kBlock * QPL) + k * kBlock + threadIdx.x, Q, h);
    qx[k] = qi.x; qy[k] = qi.y; qz[k] = qi.z;
    acc[k] = -3.0e38f;
  }
  const int64_t beg = int64_t(split) * per_split;
  const int64_t end = min(N, beg + per_split);
  for (int64_t t0 = beg; t0 < end; t0 += kTile1) {
    const int cnt = int(min<int64_t>(kTile1, end - t0));
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += kBlock) tile[j] = pos4[t0 + j];
    __syncthreads();
    int j = 0;
    for (; j + 1 < cnt; j += 2) {
      const float4 P0 = tile[j], P1 = tile[j + 1];
#pragma unroll
      for (int k = 0; k < QPL; ++k) {
        const float a0 = fmaf(qz[k], P0.z, fmaf(qy[k], P0.y, fmaf(qx[k], P0.x, P0.w)));
        const float a1 = fmaf(qz[k], P1.z, fmaf(qy[k], P1.y, fmaf(qx[k], P1.x, P1.w)));
        acc[k] = fmaxf(acc[k], fmaxf(a0, a1));
      }
    }
    if (j < cnt) {
      const float4 P0 = tile[j];
#pragma unroll
      for (int k = 0; k < QPL; ++k)
        acc[k] = fmaxf(acc[k], fmaf(qz[k], P0.z, fmaf(qy[k], P0.y, fmaf(qx[k], P0.x, P0.w))));
    }
  }
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int64_t q = qb * (kBlock * QPL) + k * kBlock + threadIdx.x;
    if (q < Q) far2[int64_t(split) * Q + q] = acc[k] + fmaf(qz[k], qz[k], fmaf(qy[k], qy[k], qx[k] * qx[k]));
  }
}

// M and lambda' = lambda log2(e) of a query from the per-split maxima.
__device__ __forceinline__ void far_of(const float* __restrict__ far2, int S, int64_t Q, int64_t q, float C2,
                                       float& M, float& nlam) {
  float m2 = -3.0e38f;
  for (int s = 0; s < S; ++s) m2 = fmaxf(m2, far2[int64_t(s) * Q + q]);
  M = sqrtf(fmaxf(m2, 0.f));
  // lambda_x = 2C/M; with M = 0 every point sits at the query and the
  // weights are uniform (lambda does not matter).
  nlam = M > 0.f ? -2.f * C2 / M : 0.f;
}

// One pair, direct torus form: <x-c,.> from stored dot products, then
// rho = |((x-c).m, (x-c).k)|, |q| = |(rho - R, (x-c).u)|, g = sign (|q| - r).
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

// ---------------------------------------------------------------------------
// Sweep 2: partial (sum w g, sum w) per split.
// ---------------------------------------------------------------------------
template <int QPL>
__global__ __launch_bounds__(kBlock) void k_blend(const Header* __restrict__ h, const float4* __restrict__ rec,
                                                  const float* __restrict__ x, int64_t Q, int S, int64_t per_split,
                                                  const float* __restrict__ far2, float C2,
                                                  float2* __restrict__ part) {
  __shared__ float4 tile[kTile2 * kRecF4];
  const int split = int(blockIdx.x % unsigned(S));
  const int64_t qb = blockIdx.x / unsigned(S);
  const int64_t N = h->N;
  const int64_t nd = h->n_direct;
  float qx[QPL], qy[QPL], qz[QPL], nl[QPL], num[QPL], den[QPL];
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int64_t q = qb * (kBlock * QPL) + k * kBlock + threadIdx.x;
    QueryIn qi = load_query(x, q, Q, h);
    qx[k] = qi.x; qy[k] = qi.y; qz[k] = qi.z;
    float M = 0.f;
    nl[k] = 0.f;
    if (qi.valid) far_of(far2, S, Q, q, C2, M, nl[k]);
    num[k] = 0.f;
    den[k] = 0.f;
  }
  const float c2 = C2;
  const int64_t beg = int64_t(split) * per_split;
  const int64_t end = min(N, beg + per_split);
  for (int64_t t0 = beg; t0 < end; t0 += kTile2) {
    const int cnt = int(min<int64_t>(kTile2, end - t0));
    __syncthreads();
    for (int j = threadIdx.x; j < cnt * kRecF4; j += kBlock) tile[j] = rec[t0 * kRecF4 + j];
    __syncthreads();
    const int jd = int(max<int64_t>(0, min<int64_t>(cnt, nd - t0)));  // [0, jd) direct form
    float tn[QPL], td[QPL];
#pragma unroll
    for (int k = 0; k < QPL; ++k) { tn[k] = 0.f; td[k] = 0.f; }
    for (int j = 0; j < jd; ++j) {
      const float4 P = tile[j * kRecF4 + 0], U = tile[j * kRecF4 + 1], Mv = tile[j * kRecF4 + 2],
                   K = tile[j * kRecF4 + 3], G = tile[j * kRecF4 + 4];
#pragma unroll
      for (int k = 0; k < QPL; ++k) {
        const float dx = qx[k] - P.x, dy = qy[k] - P.y, dz = qz[k] - P.z;
        const float d = hw_sqrt(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
        const float w = hw_exp2(fmaf(d, nl[k], c2));
        const float g = g_direct(qx[k], qy[k], qz[k], U, Mv, K, G);
        tn[k] = fmaf(w, g, tn[k]);
        td[k] += w;
      }
    }
    for (int j = jd; j < cnt; ++j) {
      const float4 P = tile[j * kRecF4 + 0], U = tile[j * kRecF4 + 1], Mv = tile[j * kRecF4 + 2],
                   K = tile[j * kRecF4 + 3], G = tile[j * kRecF4 + 4];
#pragma unroll
      for (int k = 0; k < QPL; ++k) {
        const float dx = qx[k] - P.x, dy = qy[k] - P.y, dz = qz[k] - P.z;
        const float d = hw_sqrt(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
        const float w = hw_exp2(fmaf(d, nl[k], c2));
        const float g = g_anchored(qx[k], qy[k], qz[k], P.w, U, Mv, K, G);
        tn[k] = fmaf(w, g, tn[k]);
        td[k] += w;
      }
    }
#pragma unroll
    for (int k = 0; k < QPL; ++k) { num[k] += tn[k]; den[k] += td[k]; }
  }
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int64_t q = qb * (kBlock * QPL) + k * kBlock + threadIdx.x;
    if (q < Q) part[int64_t(split) * Q + q] = make_float2(num[k], den[k]);
  }
}

// Fixed-order combine of the split partials; optional (M, W, phi) statistics.
__global__ __launch_bounds__(kBlock) void k_combine(const float2* __restrict__ part, const float* __restrict__ far2,
                                                    int S, int64_t Q, float C2, float* __restrict__ sdf,
                                                    float* __restrict__ stats) {
  const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= Q) return;
  float num = 0.f, den = 0.f;
  for (int s = 0; s < S; ++s) {
    const float2 v = part[int64_t(s) * Q + q];
    num += v.x;
    den += v.y;
  }
  const float phi = num / den;
  sdf[q] = phi;
  if (stats) {
    float M, nlam;
    far_of(far2, S, Q, q, C2, M, nlam);
    stats[3 * q] = M;
    stats[3 * q + 1] = den;
    stats[3 * q + 2] = phi;
  }
}

template <int QPL>
void launch_sweeps(const Header* h, const float4* pos4, const float4* rec, const float* x, int64_t Q,
                   const Plan& plan, float* far2, float2* part, float C2, hipStream_t st, int stages) {
  const dim3 grid(unsigned(plan.nqb * plan.S));
  if (stages & kStageFar)
    hipLaunchKernelGGL(k_far<QPL>, grid, dim3(kBlock), 0, st, h, pos4, x, Q, plan.S, plan.per_split, far2);
  if (stages & kStageBlend)
    hipLaunchKernelGGL(k_blend<QPL>, grid, dim3(kBlock), 0, st, h, rec, x, Q, plan.S, plan.per_split, far2, C2,
                       part);
}

}  // namespace

size_t eval_ws_bytes(const Plan& plan, int64_t Q) {
  return align256(size_t(plan.S) * size_t(Q) * sizeof(float)) +
         align256(size_t(plan.S) * size_t(Q) * sizeof(float2));
}

int launch_eval(const void* rec, int64_t N, const float* x, int64_t Q, float* sdf, float* grad, float* stats,
                float C, const Plan& plan, void* ws, hipStream_t st, int stages) {
  (void)grad;
  const Layout L(N);
  const char* base = static_cast<const char*>(rec);
  const Header* h = reinterpret_cast<const Header*>(base);
  const float4* pos4 = reinterpret_cast<const float4*>(base + L.pos);
  const float4* recs = reinterpret_cast<const float4*>(base + L.rec);
  char* w = static_cast<char*>(ws);
  float* far2 = reinterpret_cast<float*>(w);
  float2* part = reinterpret_cast<float2*>(w + align256(size_t(plan.S) * size_t(Q) * sizeof(float)));
  const float C2 = C * kLog2e;
  switch (plan.qpl) {
    case 1: launch_sweeps<1>(h, pos4, recs, x, Q, plan, far2, part, C2, st, stages); break;
    case 2: launch_sweeps<2>(h, pos4, recs, x, Q, plan, far2, part, C2, st, stages); break;
    case 8: launch_sweeps<8>(h, pos4, recs, x, Q, plan, far2, part, C2, st, stages); break;
    default: launch_sweeps<4>(h, pos4, recs, x, Q, plan, far2, part, C2, st, stages); break;
  }
  if (stages & kStageCombine)
    hipLaunchKernelGGL(k_combine, dim3(unsigned((Q + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, part, far2,
                       plan.S, Q, C2, sdf, stats);
  return check_hip(hipGetLastError(), "eval kernels");
}

}  // namespace pts
