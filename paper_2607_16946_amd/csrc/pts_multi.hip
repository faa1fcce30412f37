// pts_multi.hip -- packed evaluation of many requests in one launch (serving).
//
// Each workgroup reads a work descriptor naming its request (cloud record,
// queries, workspace), its query block and its point split, and then runs the
// same farthest-point / blend code as the single-request kernels.  A request's
// split count is a function of the request alone (its cloud's N and its query
// count), and a query's sums depend only on the split and tile boundaries, so
// a request gets bit-identical results whether it is launched alone or packed
// with others.
#include "pts_farcull.h"
#include "pts_multi.h"

namespace pts {
namespace {

constexpr int kQpl = 2;
// Farthest point per query and point split, culled (pts_farcull.h) within
// the split: the lower bound comes from the extreme points of a fixed sample
// of the cloud's units (a split whose block spheres cannot reach it stops
// there) and of the split's own units, and only the split's units that can
// reach it are swept.  A split may then miss its own maximum,
// but never the cloud's: the unit holding the farthest point is always swept,
// with the same arithmetic as a full sweep, and the blend reads only the
// maximum over splits, so M is bitwise that of a full sweep.
__global__ __launch_bounds__(kBlock) void k_far_multi(const WorkDesc* __restrict__ descs) {
  __shared__ FarLds L;
  const WorkDesc d = descs[blockIdx.x];
  const Header* h = reinterpret_cast<const Header*>(d.rec);
  const int64_t N = h->N, Q = d.Q;
  const Layout lay(N);
  const float4* pos4 = reinterpret_cast<const float4*>(d.rec + d.pos_off);
  const float4* ub = reinterpret_cast<const float4*>(d.rec + lay.ub);
  const int64_t U = lay.nunit;
  float qx[kQpl], qy[kQpl], qz[kQpl], acc[kQpl], lb[kQpl];
  int32_t ix[kQpl];
  bool ok[kQpl];
#pragma unroll
  for (int k = 0; k < kQpl; ++k) {
    QueryIn qi = load_query(d.x, int64_t(d.qb) * (kBlock * kQpl) + k * kBlock + threadIdx.x, Q, h);
    qx[k] = qi.x; qy[k] = qi.y; qz[k] = qi.z;
    ok[k] = qi.valid;
    acc[k] = -3.0e38f;
    ix[k] = -1;
    lb[k] = -1.f;
  }
  const int64_t beg = int64_t(d.split) * d.per_split;
  const int64_t end = min(N, beg + d.per_split);
  if (d.per_split <= kFarPlainMax) {  // a short split: swept whole, as the bound would cost more
    far_sweep_plain<kQpl, false>(pos4, beg, end, qx, qy, qz, acc, ix, L);
  } else {
    const int64_t u_lo = beg / kUnit, u_hi = max(u_lo, (end + kUnit - 1) / kUnit);
    // 1. lower bound: extreme points of sampled units and, if the split's
    // block spheres reach it, of the split's units; 2./3. the split's units
    // that can reach it
    const float4* bb = reinterpret_cast<const float4*>(d.rec + lay.bb);
    if (far_bound_split_reach<kQpl>(ub, bb, U, u_lo, u_hi, qx, qy, qz, ok, lb, L)) {
      far_threshold<kQpl>(lb, ok);
      far_sweep<kQpl, false>(pos4, ub, u_lo, u_hi, end, qx, qy, qz, ok, lb, acc, ix, L);
    }
  }
#pragma unroll
  for (int k = 0; k < kQpl; ++k) {
    const int64_t q = int64_t(d.qb) * (kBlock * kQpl) + k * kBlock + threadIdx.x;
    if (q < Q) d.far2[int64_t(d.split) * Q + q] = acc[k] + fmaf(qz[k], qz[k], fmaf(qy[k], qy[k], qx[k] * qx[k]));
  }
}

__global__ __launch_bounds__(kBlock) void k_blend_multi(const WorkDesc* __restrict__ descs, float C2, float S2) {
  __shared__ float4 tile[kTileBlend * kRecF4];
  const WorkDesc d = descs[blockIdx.x];
  const Header* h = reinterpret_cast<const Header*>(d.rec);
  const float4* rec = reinterpret_cast<const float4*>(d.rec + d.rec_off);
  const int64_t N = h->N, Q = d.Q;
  const int64_t nd = h->n_direct;
  const int S = d.S;
  float qx[kQpl], qy[kQpl], qz[kQpl], nl[kQpl], num[kQpl], den[kQpl];
#pragma unroll
  for (int k = 0; k < kQpl; ++k) {
    const int64_t q = int64_t(d.qb) * (kBlock * kQpl) + k * kBlock + threadIdx.x;
    QueryIn qi = load_query(d.x, q, Q, h);
    qx[k] = qi.x; qy[k] = qi.y; qz[k] = qi.z;
    float M = 0.f;
    nl[k] = 0.f;
    if (qi.valid) far_of(d.far2, S <= kLaneSplitsMax ? S : 1, Q, q, C2, M, nl[k]);
    num[k] = 0.f;
    den[k] = 0.f;
  }
  const int64_t beg = int64_t(d.split) * d.per_split;
  const int64_t end = min(N, beg + d.per_split);
  for (int64_t t0 = beg; t0 < end; t0 += kTileBlend) {
    const int cnt = int(min<int64_t>(kTileBlend, end - t0));
    __syncthreads();
    for (int j = threadIdx.x; j < cnt * kRecF4; j += kBlock) tile[j] = rec[t0 * kRecF4 + j];
    __syncthreads();
    const int jd = int(max<int64_t>(0, min<int64_t>(cnt, nd - t0)));
    float tn[kQpl], td[kQpl];
#pragma unroll
    for (int k = 0; k < kQpl; ++k) { tn[k] = 0.f; td[k] = 0.f; }
    for (int j = 0; j < jd; ++j) {
      const float4 P = tile[j * kRecF4 + 0], U = tile[j * kRecF4 + 1], Mv = tile[j * kRecF4 + 2],
                   K = tile[j * kRecF4 + 3], G = tile[j * kRecF4 + 4];
#pragma unroll
      for (int k = 0; k < kQpl; ++k) {
        const float dx = qx[k] - P.x, dy = qy[k] - P.y, dz = qz[k] - P.z;
        const float dd = hw_sqrt(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
        const float w = hw_exp2(fmaf(dd, nl[k], S2));
        const float g = g_direct(qx[k], qy[k], qz[k], U, Mv, K, G);
        tn[k] = fmaf(w, g, tn[k]);
        td[k] += w;
      }
    }
    for (int j = jd; j < cnt; ++j) {
      const float4 P = tile[j * kRecF4 + 0], U = tile[j * kRecF4 + 1], Mv = tile[j * kRecF4 + 2],
                   K = tile[j * kRecF4 + 3], G = tile[j * kRecF4 + 4];
#pragma unroll
      for (int k = 0; k < kQpl; ++k) {
        const float dx = qx[k] - P.x, dy = qy[k] - P.y, dz = qz[k] - P.z;
        const float dd = hw_sqrt(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
        const float w = hw_exp2(fmaf(dd, nl[k], S2));
        const float g = g_anchored(qx[k], qy[k], qz[k], P.w, U, Mv, K, G);
        tn[k] = fmaf(w, g, tn[k]);
        td[k] += w;
      }
    }
#pragma unroll
    for (int k = 0; k < kQpl; ++k) { num[k] += tn[k]; den[k] += td[k]; }
  }
#pragma unroll
  for (int k = 0; k < kQpl; ++k) {
    const int64_t q = int64_t(d.qb) * (kBlock * kQpl) + k * kBlock + threadIdx.x;
    if (q < Q) d.part[int64_t(d.split) * Q + q] = make_float2(num[k], den[k]);
  }
}

// Between the two sweeps, for requests with more than kLaneSplitsMax splits:
// their per-split maxima folded into row 0 over the combine's descriptors,
// as the combine partitions the queries (a lane or a wavefront per query).
__global__ __launch_bounds__(kBlock) void k_fold_multi(const CombDesc* __restrict__ descs) {
  const CombDesc c = descs[blockIdx.x];
  if (c.S <= kLaneSplitsMax) return;
  if (!combine_by_wave(c.S, c.Q)) {  // this descriptor covers kBlock queries: one lane each
    const int64_t q = int64_t(c.qb) * kBlock + threadIdx.x;
    if (q < c.Q) c.far2[q] = fold_seq(c.far2, c.S, c.Q, q);
    return;
  }
  const int64_t q = int64_t(c.qb) * (kBlock / 64) + threadIdx.x / 64;
  const int lane = int(threadIdx.x & 63);
  const float m = fold_wave(c.far2, c.S, c.Q, q, lane);
  if (lane == 0 && q < c.Q) c.far2[q] = m;
}

// One workgroup per (request, block of queries): the fixed-order combine of
// pts_device.h, as k_combine / k_combine_wave do it -- kBlock queries one per
// lane, or, when combine_by_wave, kBlock / 64 queries one per wave.
__global__ __launch_bounds__(kBlock) void k_combine_multi(const CombDesc* __restrict__ descs) {
  const CombDesc c = descs[blockIdx.x];
  if (!combine_by_wave(c.S, c.Q)) {
    const int64_t q = int64_t(c.qb) * kBlock + threadIdx.x;
    if (q >= c.Q) return;
    const float2 v = combine_seq(c.part, c.S, c.Q, q);
    c.out[q] = v.x / v.y;
  } else {
    const int64_t q = int64_t(c.qb) * (kBlock / 64) + threadIdx.x / 64;
    const int lane = int(threadIdx.x & 63);
    const float2 v = combine_wave(c.part, c.S, c.Q, q, lane);
    if (lane == 0 && q < c.Q) c.out[q] = v.x / v.y;
  }
}

}  // namespace

int launch_multi(const WorkDesc* d_work, int64_t n_work, const CombDesc* d_comb, int64_t n_comb, float C,
                 bool fold, hipStream_t st) {
  if (n_work > 0) {
    hipLaunchKernelGGL(k_far_multi, dim3(unsigned(n_work)), dim3(kBlock), 0, st, d_work);
    if (fold && n_comb > 0) hipLaunchKernelGGL(k_fold_multi, dim3(unsigned(n_comb)), dim3(kBlock), 0, st, d_comb);
    hipLaunchKernelGGL(k_blend_multi, dim3(unsigned(n_work)), dim3(kBlock), 0, st, d_work, C * kLog2e,
                       shift2_of(C));
  }
  if (n_comb > 0) hipLaunchKernelGGL(k_combine_multi, dim3(unsigned(n_comb)), dim3(kBlock), 0, st, d_comb);
  return check_hip(hipGetLastError(), "packed eval kernels");
}

int multi_qpl() { return kQpl; }

}  // namespace pts
