// pts_baseline.hip -- the two point-based baselines the paper compares against
// (Sec. 5.2, "Signed distance accuracy"), on the skeleton of the blend:
//   the culled farthest-point sweep gives M, hence sigma_x = M/2 and
//   lambda_x = 2C/M (Eq. RelationshipBetweenLambdaAndRadius); one weighted
//   sweep over LDS-staged point tiles, split over S point ranges; a
//   fixed-order combine of the splits.
// With w_i = A_i exp(-lambda_x (d_i - sigma_x)), d_i = |x - p_i| and the
// planar distance t_i = <x - p_i, n_i / |n_i|>:
//   smoothed signed planar distance, Eq. (SmoothedSignedPlanarDistance):
//     phi = sum w_i t_i / sum w_i
//   signed Hopf-Cole distance, Eq. (ScreenedWindingNumber):
//     s   = sum w_i (lambda_x d_i + 1) t_i / (2 pi d_i^3)
//     phi = sign(s) (-log|s| / lambda_x + sigma_x),  sign(0) = +1
// A query on a point (d_i = 0) gives NaN for the Hopf-Cole distance.  The
// shift keeps each weight in [e^-C, e^C]; the Hopf-Cole terms add the factor
// (lambda d + 1) / d^2, so a query within ~1e-5 of the cloud's diagonal of a
// point can overflow FP32 to an infinite distance.
//
// Point record (base section, 2 x float4 per slot, record coordinates):
//   (p, A) and (n / |n|, -<p, n / |n|>); A = 1 unless set by pts_set_areas.
#include "pts_device.h"

namespace pts {
namespace {

constexpr int kTileB = 256;                     // points per LDS tile (8 KB)
constexpr float kInv2Pi = 0.15915494309189535f;

template <int QPL, int KIND>
__global__ __launch_bounds__(kBlock) void k_base(const Header* __restrict__ h, const float4* __restrict__ bas,
                                                 const float* __restrict__ x, int64_t Q, int S, int64_t per_split,
                                                 const float* __restrict__ far2, float C, float2* __restrict__ part) {
  __shared__ float4 tile[kTileB * 2];
  // split = b % S: the blend's split-major order (split_block) is not worth
  // the slower pair-loop schedule hipcc gives this sweep with it
  const int split = int(blockIdx.x % unsigned(S));
  const int64_t qb = blockIdx.x / unsigned(S);
  const int64_t N = h->N;
  const float C2 = C * kLog2e, S2 = shift2_of(C);
  float qx[QPL], qy[QPL], qz[QPL], nl[QPL], lam[QPL], num[QPL], den[QPL];
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int64_t q = qb * (kBlock * QPL) + k * kBlock + threadIdx.x;
    const QueryIn qi = load_query(x, q, Q, h);
    qx[k] = qi.x; qy[k] = qi.y; qz[k] = qi.z;
    float M = 0.f;
    nl[k] = 0.f;
    if (qi.valid) far_of(far2, 1, Q, q, C2, M, nl[k]);
    lam[k] = M > 0.f ? 2.f * C / M : 0.f;
    num[k] = 0.f;
    den[k] = 0.f;
  }
  const int64_t beg = int64_t(split) * per_split;
  const int64_t end = min(N, beg + per_split);
  for (int64_t t0 = beg; t0 < end; t0 += kTileB) {
    const int cnt = int(min<int64_t>(kTileB, end - t0));
    __syncthreads();
    for (int j = threadIdx.x; j < cnt * 2; j += kBlock) tile[j] = bas[t0 * 2 + j];
    __syncthreads();
    float tn[QPL], td[QPL];
#pragma unroll
    for (int k = 0; k < QPL; ++k) { tn[k] = 0.f; td[k] = 0.f; }
    for (int j = 0; j < cnt; ++j) {
      const float4 P = tile[2 * j], Nv = tile[2 * j + 1];
#pragma unroll
      for (int k = 0; k < QPL; ++k) {
        const float dx = qx[k] - P.x, dy = qy[k] - P.y, dz = qz[k] - P.z;
        const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        const float t = fmaf(dz, Nv.z, fmaf(dy, Nv.y, dx * Nv.x));
        if (KIND == PTS_BASELINE_SSPD) {
          const float d = hw_sqrt(d2);
          const float w = hw_exp2(fmaf(d, nl[k], S2)) * P.w;
          tn[k] = fmaf(w, t, tn[k]);
          td[k] += w;
        } else {
          // d and 1/d from one rsqrt; at d = 0 (rsqrt = inf) d is NaN and so is the sum
          const float rd = hw_rsq(d2);
          const float d = d2 * rd;
          const float w = hw_exp2(fmaf(d, nl[k], S2)) * P.w;
          const float hv = d > 0.f ? fmaf(lam[k], d, 1.f) * t * (rd * rd * rd) * kInv2Pi : __builtin_nanf("");
          tn[k] = fmaf(w, hv, tn[k]);
        }
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

template <int KIND>
__global__ __launch_bounds__(kBlock) void k_base_combine(const float2* __restrict__ part,
                                                         const float* __restrict__ far2, int S, int64_t Q, float C,
                                                         float* __restrict__ sdf, float offset) {
  const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= Q) return;
  float num = 0.f, den = 0.f;
  for (int s = 0; s < S; ++s) {
    const float2 v = part[int64_t(s) * Q + q];
    num += v.x;
    den += v.y;
  }
  if (KIND == PTS_BASELINE_SSPD) {
    sdf[q] = num / den - offset;
  } else {
    const float M = sqrtf(fmaxf(far2[q], 0.f));
    const float sg = num < 0.f ? -1.f : 1.f;
    // the weights carry the factor e^s, s = min(C, 64), i.e. -log adds s / lambda_x = s M / (2C) (= M/2 for s = C)
    const float back = C <= kShiftMaxC ? 0.5f * M : kShiftMaxC * M / (2.f * C);
    sdf[q] = sg * (-logf(fabsf(num)) * M / (2.f * C) + back) - offset;
  }
}

__global__ __launch_bounds__(kBlock) void k_areas(const int32_t* __restrict__ perm, const float* __restrict__ area,
                                                  int64_t N, float4* __restrict__ bas) {
  const int64_t slot = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (slot >= N) return;
  bas[2 * slot].w = area ? area[perm[slot]] : 1.f;
}

template <int QPL, int KIND>
void launch_base_q(const Header* h, const float4* bas, const float* x, int64_t Q, const Plan& plan,
                   const float* far2, float C, float2* part, hipStream_t st) {
  hipLaunchKernelGGL((k_base<QPL, KIND>), dim3(unsigned(plan.nqb * plan.S)), dim3(kBlock), 0, st, h, bas, x, Q,
                     plan.S, plan.per_split, far2, C, part);
}

template <int KIND>
void launch_base_kind(const Header* h, const float4* bas, const float* x, int64_t Q, const Plan& plan,
                      const float* far2, float C, float2* part, float* sdf, float offset, hipStream_t st) {
  switch (plan.qpl) {
    case 1: launch_base_q<1, KIND>(h, bas, x, Q, plan, far2, C, part, st); break;
    case 2: launch_base_q<2, KIND>(h, bas, x, Q, plan, far2, C, part, st); break;
    default: launch_base_q<4, KIND>(h, bas, x, Q, with_qpl(plan, 4, Q), far2, C, part, st); break;
  }
  hipLaunchKernelGGL(k_base_combine<KIND>, dim3(unsigned((Q + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, part,
                     far2, plan.S, Q, C, sdf, offset);
}

}  // namespace

int launch_set_areas(void* rec, int64_t N, const float* area, hipStream_t st) {
  const Layout L(N);
  char* base = static_cast<char*>(rec);
  hipLaunchKernelGGL(k_areas, dim3(unsigned((N + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     reinterpret_cast<const int32_t*>(base + L.perm), area, N,
                     reinterpret_cast<float4*>(base + L.base));
  return check_hip(hipGetLastError(), "area kernel");
}

int launch_baseline(const void* rec, int64_t N, const float* x, int64_t Q, int kind, float C, const Plan& plan,
                    const WsView& ws, float* sdf, hipStream_t st, float offset) {
  const Layout L(N);
  const char* base = static_cast<const char*>(rec);
  const Header* h = reinterpret_cast<const Header*>(base);
  const float4* bas = reinterpret_cast<const float4*>(base + L.base);
  if (int rc = launch_far_cull(rec, N, x, Q, plan.qpl, ws.far2, nullptr, st)) return rc;
  if (kind == PTS_BASELINE_SSPD)
    launch_base_kind<PTS_BASELINE_SSPD>(h, bas, x, Q, plan, ws.far2, C, ws.part, sdf, offset, st);
  else
    launch_base_kind<PTS_BASELINE_SHC>(h, bas, x, Q, plan, ws.far2, C, ws.part, sdf, offset, st);
  return check_hip(hipGetLastError(), "baseline kernels");
}

}  // namespace pts
