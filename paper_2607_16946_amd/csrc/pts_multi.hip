// pts_multi.hip -- packed evaluation of many requests in one launch (serving).
//
// Each workgroup reads a work descriptor naming its request (cloud record,
// queries, workspace), its query block and its point split, and then runs the
// same farthest-point / blend code as the single-request kernels.  A request's
// split count is a function of its cloud's N only, and a query's sums depend
// only on the split and tile boundaries, so a request gets bit-identical
// results whether it is launched alone or packed with others.
#include "pts_device.h"
#include "pts_multi.h"

namespace pts {
namespace {

constexpr int kQpl = 2;

__global__ __launch_bounds__(kBlock) void k_far_multi(const WorkDesc* __restrict__ descs) {
  __shared__ float4 tile[kTile1];
  const WorkDesc d = descs[blockIdx.x];
  const Header* h = reinterpret_cast<const Header*>(d.rec);
  const float4* pos4 = reinterpret_cast<const float4*>(d.rec + d.pos_off);
  const int64_t N = h->N, Q = d.Q;
  float qx[kQpl], qy[kQpl], qz[kQpl], acc[kQpl];
#pragma unroll
  for (int k = 0; k < kQpl; ++k) {
    QueryIn qi = load_query(d.x, int64_t(d.qb) * (kBlock * kQpl) + k * kBlock + threadIdx.x, Q, h);
    qx[k] = qi.x; qy[k] = qi.y; qz[k] = qi.z;
    acc[k] = -3.0e38f;
  }
  const int64_t beg = int64_t(d.split) * d.per_split;
  const int64_t end = min(N, beg + d.per_split);
  for (int64_t t0 = beg; t0 < end; t0 += kTile1) {
    const int cnt = int(min<int64_t>(kTile1, end - t0));
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += kBlock) tile[j] = pos4[t0 + j];
    __syncthreads();
    int j = 0;
    for (; j + 1 < cnt; j += 2) {
      const float4 P0 = tile[j], P1 = tile[j + 1];
#pragma unroll
      for (int k = 0; k < kQpl; ++k) {
        const float a0 = fmaf(qz[k], P0.z, fmaf(qy[k], P0.y, fmaf(qx[k], P0.x, P0.w)));
        const float a1 = fmaf(qz[k], P1.z, fmaf(qy[k], P1.y, fmaf(qx[k], P1.x, P1.w)));
        acc[k] = fmaxf(acc[k], fmaxf(a0, a1));
      }
    }
    if (j < cnt) {
      const float4 P0 = tile[j];
#pragma unroll
      for (int k = 0; k < kQpl; ++k)
        acc[k] = fmaxf(acc[k], fmaf(qz[k], P0.z, fmaf(qy[k], P0.y, fmaf(qx[k], P0.x, P0.w))));
    }
  }
#pragma unroll
  for (int k = 0; k < kQpl; ++k) {
    const int64_t q = int64_t(d.qb) * (kBlock * kQpl) + k * kBlock + threadIdx.x;
    if (q < Q) d.far2[int64_t(d.split) * Q + q] = acc[k] + fmaf(qz[k], qz[k], fmaf(qy[k], qy[k], qx[k] * qx[k]));
  }
}

__global__ __launch_bounds__(kBlock) void k_blend_multi(const WorkDesc* __restrict__ descs, float C2) {
  __shared__ float4 tile[kTile2 * kRecF4];
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
    if (qi.valid) far_of(d.far2, S, Q, q, C2, M, nl[k]);
    num[k] = 0.f;
    den[k] = 0.f;
  }
  const int64_t beg = int64_t(d.split) * d.per_split;
  const int64_t end = min(N, beg + d.per_split);
  for (int64_t t0 = beg; t0 < end; t0 += kTile2) {
    const int cnt = int(min<int64_t>(kTile2, end - t0));
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
        const float w = hw_exp2(fmaf(dd, nl[k], C2));
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
        const float w = hw_exp2(fmaf(dd, nl[k], C2));
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

// One workgroup per (request, block of kBlock queries): fixed-order combine.
__global__ __launch_bounds__(kBlock) void k_combine_multi(const CombDesc* __restrict__ descs) {
  const CombDesc c = descs[blockIdx.x];
  const int64_t q = int64_t(c.qb) * kBlock + threadIdx.x;
  if (q >= c.Q) return;
  float num = 0.f, den = 0.f;
  for (int s = 0; s < c.S; ++s) {
    const float2 v = c.part[int64_t(s) * c.Q + q];
    num += v.x;
    den += v.y;
  }
  c.out[q] = num / den;
}

}  // namespace

int launch_multi(const WorkDesc* d_work, int64_t n_work, const CombDesc* d_comb, int64_t n_comb, float C,
                 hipStream_t st) {
  if (n_work > 0) {
    hipLaunchKernelGGL(k_far_multi, dim3(unsigned(n_work)), dim3(kBlock), 0, st, d_work);
    hipLaunchKernelGGL(k_blend_multi, dim3(unsigned(n_work)), dim3(kBlock), 0, st, d_work, C * kLog2e);
  }
  if (n_comb > 0) hipLaunchKernelGGL(k_combine_multi, dim3(unsigned(n_comb)), dim3(kBlock), 0, st, d_comb);
  return check_hip(hipGetLastError(), "packed eval kernels");
}

int multi_qpl() { return kQpl; }

}  // namespace pts
