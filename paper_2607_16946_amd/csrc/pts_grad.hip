// pts_grad.hip -- derivative of phi with respect to the query point on gfx950.
//
// With W = sum_i w_i, d_i = |x - p_i|, e_i = (x - p_i)/d_i and lambda = 2C/M,
// App. D gives, for fixed lambda,
//   grad phi = (1/W) [ sum_i w_i grad g_i - lambda sum_i w_i (g_i - phi) e_i ];
// lambda_x = 2C/M(x) also moves with x through the farthest point p_*
// (grad M = e_*), which adds
//   (2C/M^2) e_* (1/W) sum_i w_i (g_i - phi) d_i.
// For one torus (Eq. SingleTorusSDF), with v = x - c in the frame (u, m, k),
// rho = |(v.m, v.k)|, b = rho - R, |q| = |(b, v.u)|:
//   grad g = sign / |q| [ (b / rho) ((v.m) m + (v.k) k) + (v.u) u ].
// The factors 1/rho, 1/|q|, 1/d are taken as 0 where they vanish (torus axis,
// core circle, query on a point): a subgradient of the nonsmooth sets.
//
// Kernels:
//   (farthest-point sweep that also records the farthest slot: the culled
//    sweep of pts_eval.hip with argmax tracking)
//   k_combine_stats  phi and the statistics (M, W, phi, e_*) of each query
//   k_grad           third sweep: per split, sum w grad g, sum w (g-phi) e,
//                    sum w (g-phi) d (seven accumulators per query)
//   k_grad_combine   fixed-order sum over splits, grad phi (times an optional
//                    upstream gradient)
#include "pts_device.h"

namespace pts {
namespace {

// phi = sum num / sum den over splits (fixed order) and stats (M, W, phi, e_*)
// from the farthest-point sweep's M^2 and farthest slot of each query.
__global__ __launch_bounds__(kBlock) void k_combine_stats(const Header* __restrict__ h, const float4* __restrict__ pos4,
                                                          const float* __restrict__ x, const float2* __restrict__ part,
                                                          const float* __restrict__ far2,
                                                          const int32_t* __restrict__ farix, int S, int64_t Q,
                                                          float* __restrict__ sdf, float* __restrict__ stats,
                                                          float offset) {
  const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= Q) return;
  float num = 0.f, den = 0.f;
  for (int s = 0; s < S; ++s) {
    const float2 v = part[int64_t(s) * Q + q];
    num += v.x;
    den += v.y;
  }
  const float m2 = far2[q];
  const int32_t slot = farix[q];
  const float phi = num / den;
  if (sdf) sdf[q] = phi - offset;   // the statistics keep phi itself
  const float M = sqrtf(fmaxf(m2, 0.f));
  float e[3] = {0.f, 0.f, 0.f};
  if (slot >= 0 && M > 0.f) {
    const QueryIn qi = load_query(x, q, Q, h);
    const float4 P = pos4[slot];   // (-2p, |p|^2)
    const float inv = 1.f / M;
    e[0] = (qi.x + 0.5f * P.x) * inv;
    e[1] = (qi.y + 0.5f * P.y) * inv;
    e[2] = (qi.z + 0.5f * P.z) * inv;
  }
  float* o = stats + 6 * q;
  o[0] = M;
  o[1] = den;
  o[2] = phi;
  o[3] = e[0];
  o[4] = e[1];
  o[5] = e[2];
}

// kFull = false: only D (the weight sweep of the point backward).
template <bool kDirect, bool kFull>
__device__ __forceinline__ void grad_pair(float qx, float qy, float qz, float nl, float S2, float phi,
                                          const float4& P, const float4& U, const float4& Mv, const float4& K,
                                          const float4& G, float* A, float* B, float& D) {
  const float dx = qx - P.x, dy = qy - P.y, dz = qz - P.z;
  const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
  if (!kFull) {  // the weight sweep needs neither reciprocals nor grad g: the blend's forms
    const float d = hw_sqrt(d2);
    const float w = hw_exp2(fmaf(d, nl, S2));
    const float g = kDirect ? g_direct(qx, qy, qz, U, Mv, K, G) : g_anchored(qx, qy, qz, P.w, U, Mv, K, G);
    D = fmaf(w * (g - phi), d, D);
    return;
  }
  const float id = safe_rsq(d2);                   // 1/d
  const float d = d2 * id;
  const float w = hw_exp2(fmaf(d, nl, S2));
  const Geo r = kDirect ? geo_direct(qx, qy, qz, U, Mv, K, G) : geo_anchored(qx, qy, qz, P.w, U, Mv, K, G);
  const float we = w * (r.g - phi);
  const float sq = G.z * r.iqn;
  const float f1 = sq * r.b * r.irho;
  const float f2 = sq * r.vu;
  const float a1 = f1 * r.vm, a2 = f1 * r.vk;
  const float gx = fmaf(a1, Mv.x, fmaf(a2, K.x, f2 * U.x));
  const float gy = fmaf(a1, Mv.y, fmaf(a2, K.y, f2 * U.y));
  const float gz = fmaf(a1, Mv.z, fmaf(a2, K.z, f2 * U.z));
  A[0] = fmaf(w, gx, A[0]);
  A[1] = fmaf(w, gy, A[1]);
  A[2] = fmaf(w, gz, A[2]);
  const float c = we * id;
  B[0] = fmaf(c, dx, B[0]);
  B[1] = fmaf(c, dy, B[1]);
  B[2] = fmaf(c, dz, B[2]);
  D = fmaf(we, d, D);
}

// kFull: the seven accumulators of grad phi into gpart; otherwise only
// sum w (g - phi) d into vpart [S][Q].
template <int QPL, bool kFull>
__global__ __launch_bounds__(kBlock) void k_grad(const Header* __restrict__ h, const float4* __restrict__ rec,
                                                 const float* __restrict__ x, int64_t Q, int S, int64_t per_split,
                                                 const float* __restrict__ stats, float C2, float S2,
                                                 float4* __restrict__ gpart, float* __restrict__ vpart) {
  __shared__ float4 tile[kTile2 * kRecF4];
  // split = b % S: the blend's split-major order (split_block) is not worth
  // the slower pair-loop schedule hipcc gives this sweep with it (10%)
  const int split = int(blockIdx.x % unsigned(S));
  const int64_t qb = blockIdx.x / unsigned(S);
  const int64_t N = h->N;
  const int64_t nd = h->n_direct;
  float qx[QPL], qy[QPL], qz[QPL], nl[QPL], ph[QPL];
  float A[QPL][3], B[QPL][3], D[QPL];
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int64_t q = qb * (kBlock * QPL) + k * kBlock + threadIdx.x;
    QueryIn qi = load_query(x, q, Q, h);
    qx[k] = qi.x; qy[k] = qi.y; qz[k] = qi.z;
    nl[k] = 0.f;
    ph[k] = 0.f;
    if (qi.valid) {
      const float M = stats[6 * q];
      nl[k] = M > 0.f ? -2.f * C2 / M : 0.f;
      ph[k] = stats[6 * q + 2];
    }
    for (int c = 0; c < 3; ++c) { A[k][c] = 0.f; B[k][c] = 0.f; }
    D[k] = 0.f;
  }
  const int64_t beg = int64_t(split) * per_split;
  const int64_t end = min(N, beg + per_split);
  for (int64_t t0 = beg; t0 < end; t0 += kTile2) {
    const int cnt = int(min<int64_t>(kTile2, end - t0));
    __syncthreads();
    for (int j = threadIdx.x; j < cnt * kRecF4; j += kBlock) tile[j] = rec[t0 * kRecF4 + j];
    __syncthreads();
    const int jd = int(max<int64_t>(0, min<int64_t>(cnt, nd - t0)));
    float tA[QPL][3], tB[QPL][3], tD[QPL];
#pragma unroll
    for (int k = 0; k < QPL; ++k) {
      for (int c = 0; c < 3; ++c) { tA[k][c] = 0.f; tB[k][c] = 0.f; }
      tD[k] = 0.f;
    }
    for (int j = 0; j < jd; ++j) {
      const float4 P = tile[j * kRecF4 + 0], U = tile[j * kRecF4 + 1], Mv = tile[j * kRecF4 + 2],
                   K = tile[j * kRecF4 + 3], G = tile[j * kRecF4 + 4];
#pragma unroll
      for (int k = 0; k < QPL; ++k) grad_pair<true, kFull>(qx[k], qy[k], qz[k], nl[k], S2, ph[k], P, U, Mv, K, G, tA[k], tB[k], tD[k]);
    }
    for (int j = jd; j < cnt; ++j) {
      const float4 P = tile[j * kRecF4 + 0], U = tile[j * kRecF4 + 1], Mv = tile[j * kRecF4 + 2],
                   K = tile[j * kRecF4 + 3], G = tile[j * kRecF4 + 4];
#pragma unroll
      for (int k = 0; k < QPL; ++k) grad_pair<false, kFull>(qx[k], qy[k], qz[k], nl[k], S2, ph[k], P, U, Mv, K, G, tA[k], tB[k], tD[k]);
    }
#pragma unroll
    for (int k = 0; k < QPL; ++k) {
      for (int c = 0; c < 3; ++c) { A[k][c] += tA[k][c]; B[k][c] += tB[k][c]; }
      D[k] += tD[k];
    }
  }
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int64_t q = qb * (kBlock * QPL) + k * kBlock + threadIdx.x;
    if (q < Q) {
      if (kFull) {
        float4* o = gpart + 2 * (int64_t(split) * Q + q);
        o[0] = make_float4(A[k][0], A[k][1], A[k][2], D[k]);
        o[1] = make_float4(B[k][0], B[k][1], B[k][2], 0.f);
      } else {
        vpart[int64_t(split) * Q + q] = D[k];
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_grad_combine(const float4* __restrict__ gpart,
                                                         const float* __restrict__ stats, int S, int64_t Q, float C,
                                                         const float* __restrict__ gout, float* __restrict__ gx) {
  const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= Q) return;
  float A[3] = {0.f, 0.f, 0.f}, B[3] = {0.f, 0.f, 0.f}, D = 0.f;
  for (int s = 0; s < S; ++s) {
    const float4* p = gpart + 2 * (int64_t(s) * Q + q);
    const float4 a = p[0], b = p[1];
    A[0] += a.x; A[1] += a.y; A[2] += a.z; D += a.w;
    B[0] += b.x; B[1] += b.y; B[2] += b.z;
  }
  const float* st = stats + 6 * q;
  const float M = st[0], W = st[1];
  const float iw = 1.f / W;
  const float lam = M > 0.f ? 2.f * C / M : 0.f;
  const float cm = M > 0.f ? 2.f * C / (M * M) * D : 0.f;
  const float s = gout ? gout[q] : 1.f;
  for (int c = 0; c < 3; ++c) gx[3 * q + c] = s * (iw * (A[c] - lam * B[c] + cm * st[3 + c]));
}

template <int QPL, bool kFull>
void launch_grad_sweep(const Header* h, const float4* rec, const float* x, int64_t Q, const Plan& plan,
                       const float* stats, float C, float4* gpart, float* vpart, hipStream_t st) {
  hipLaunchKernelGGL((k_grad<QPL, kFull>), dim3(unsigned(plan.nqb * plan.S)), dim3(kBlock), 0, st, h, rec, x, Q,
                     plan.S, plan.per_split, stats, C * kLog2e, shift2_of(C), gpart, vpart);
}

}  // namespace

int launch_far_arg(const void* rec, int64_t N, const float* x, int64_t Q, const Plan& plan, const WsView& ws,
                   hipStream_t st) {
  return launch_far_cull(rec, N, x, Q, plan.qpl, ws.far2, ws.farix, st, plan.S, plan.per_split);
}

int launch_combine_stats(const void* rec, int64_t N, const float* x, int64_t Q, const Plan& plan, const WsView& ws,
                         float* sdf, float* stats, hipStream_t st, float offset) {
  const Layout L(N);
  const char* base = static_cast<const char*>(rec);
  hipLaunchKernelGGL(k_combine_stats, dim3(unsigned((Q + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     reinterpret_cast<const Header*>(base), reinterpret_cast<const float4*>(base + L.pos), x,
                     ws.part, ws.far2, ws.farix, plan.S, Q, sdf, stats, offset);
  return check_hip(hipGetLastError(), "combine (stats) kernel");
}

int launch_grad(const void* rec, int64_t N, const float* x, int64_t Q, const float* stats, const float* gout,
                float* gx, float C, const Plan& plan, const WsView& ws, hipStream_t st) {
  const Layout L(N);
  const char* base = static_cast<const char*>(rec);
  const Header* h = reinterpret_cast<const Header*>(base);
  const float4* recs = reinterpret_cast<const float4*>(base + L.rec);
  const int qpl = plan.qpl > 2 ? 2 : plan.qpl;
  const Plan p = with_qpl(plan, qpl, Q);
  switch (qpl) {
    case 1: launch_grad_sweep<1, true>(h, recs, x, Q, p, stats, C, ws.gpart, nullptr, st); break;
    default: launch_grad_sweep<2, true>(h, recs, x, Q, p, stats, C, ws.gpart, nullptr, st); break;
  }
  hipLaunchKernelGGL(k_grad_combine, dim3(unsigned((Q + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, ws.gpart,
                     stats, plan.S, Q, C, gout, gx);
  return check_hip(hipGetLastError(), "gradient kernels");
}

int launch_vsum(const void* rec, int64_t N, const float* x, int64_t Q, const float* stats, float C,
                const Plan& plan, float* vpart, hipStream_t st) {
  const Layout L(N);
  const char* base = static_cast<const char*>(rec);
  const Header* h = reinterpret_cast<const Header*>(base);
  const float4* recs = reinterpret_cast<const float4*>(base + L.rec);
  const int qpl = plan.qpl > 2 ? 2 : plan.qpl;
  const Plan p = with_qpl(plan, qpl, Q);
  switch (qpl) {
    case 1: launch_grad_sweep<1, false>(h, recs, x, Q, p, stats, C, nullptr, vpart, st); break;
    default: launch_grad_sweep<2, false>(h, recs, x, Q, p, stats, C, nullptr, vpart, st); break;
  }
  return check_hip(hipGetLastError(), "weight sweep kernel");
}

}  // namespace pts
