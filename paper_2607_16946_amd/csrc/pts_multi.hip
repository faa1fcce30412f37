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
constexpr int kChunkU = 256;              // units whose bounds are staged in LDS at once
constexpr int kBatchU = kTile1 / kUnit;   // units per LDS tile of points
constexpr int kSampleU = 64;              // units of the whole cloud that seed the lower bound

// Farthest point per query and point split, culled exactly as the
// single-request sweep but within the split: with LB <= M the largest
// distance from the query to the extreme points of a fixed sample of the
// cloud's units and of this split's units, only the split's units whose
// bounding sphere can reach LB (1 - 1e-5) for some query of the workgroup are
// swept.  A split may then miss its own maximum, but never the cloud's: the
// unit holding the farthest point is always swept, with the same arithmetic as
// a full sweep, and the blend reads only the maximum over splits, so M is
// bitwise that of a full sweep.
__global__ __launch_bounds__(kBlock) void k_far_multi(const WorkDesc* __restrict__ descs) {
  __shared__ float4 sb[kChunkU];
  __shared__ uint32_t smask[kChunkU / 32];
  __shared__ int32_t slist[kChunkU];
  __shared__ int32_t scount;
  __shared__ float4 tile[kTile1];
  const WorkDesc d = descs[blockIdx.x];
  const Header* h = reinterpret_cast<const Header*>(d.rec);
  const int64_t N = h->N, Q = d.Q;
  const Layout L(N);
  const float4* pos4 = reinterpret_cast<const float4*>(d.rec + d.pos_off);
  const float4* ub = reinterpret_cast<const float4*>(d.rec + L.ub);
  const int64_t U = L.nunit;
  float qx[kQpl], qy[kQpl], qz[kQpl], acc[kQpl], lb[kQpl];
  bool ok[kQpl];
#pragma unroll
  for (int k = 0; k < kQpl; ++k) {
    QueryIn qi = load_query(d.x, int64_t(d.qb) * (kBlock * kQpl) + k * kBlock + threadIdx.x, Q, h);
    qx[k] = qi.x; qy[k] = qi.y; qz[k] = qi.z;
    ok[k] = qi.valid;
    acc[k] = -3.0e38f;
    lb[k] = -1.f;
  }
  const int64_t beg = int64_t(d.split) * d.per_split;
  const int64_t end = min(N, beg + d.per_split);
  const int64_t u_lo = beg / kUnit, u_hi = max(u_lo, (end + kUnit - 1) / kUnit);
  // 1. lower bound: extreme points of every stride-th unit, then of the split's units
  const int64_t stride = (U + kSampleU - 1) / kSampleU;
  const int64_t n_samp = (U + stride - 1) / stride;
  const int64_t n_lb = n_samp + (u_hi - u_lo);
  for (int64_t c0 = 0; c0 < n_lb; c0 += kChunkU) {
    const int cnt = int(min<int64_t>(kChunkU, n_lb - c0));
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += kBlock) {
      const int64_t i = c0 + j;
      sb[j] = ub[2 * (i < n_samp ? i * stride : u_lo + (i - n_samp)) + 1];
    }
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const float4 E = sb[j];
#pragma unroll
      for (int k = 0; k < kQpl; ++k) {
        const float dx = qx[k] - E.x, dy = qy[k] - E.y, dz = qz[k] - E.z;
        lb[k] = fmaxf(lb[k], fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kQpl; ++k) {
    ok[k] = ok[k] && lb[k] >= 0.f;              // a query with a NaN coordinate needs no unit: M is NaN
    lb[k] = sqrtf(fmaxf(lb[k], 0.f)) * (1.f - 1e-5f);
  }
  // 2./3. per chunk of the split's units: mark the needed ones, list them, sweep their points
  for (int64_t c0 = u_lo; c0 < u_hi; c0 += kChunkU) {
    const int cnt = int(min<int64_t>(kChunkU, u_hi - c0));
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += kBlock) sb[j] = ub[2 * (c0 + j)];
    for (int j = threadIdx.x; j < kChunkU / 32; j += kBlock) smask[j] = 0u;
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const float4 C = sb[j];
      bool need = false;
#pragma unroll
      for (int k = 0; k < kQpl; ++k) {
        const float t = lb[k] - C.w;
        const float dx = qx[k] - C.x, dy = qy[k] - C.y, dz = qz[k] - C.z;
        const float dc2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        need = need || (ok[k] && (t <= 0.f || !(dc2 < t * t)));
      }
      if (__ballot(need) != 0ull && (threadIdx.x & 63) == 0) atomicOr(&smask[j >> 5], 1u << (j & 31));
    }
    __syncthreads();
    if (threadIdx.x < 64) {  // ascending list of the needed units (first wave)
      const int w = int(threadIdx.x);
      const uint32_t bits = w < kChunkU / 32 ? smask[w] : 0u;
      const int pc = __popc(bits);
      int incl = pc;
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o);
        if (w >= o) incl += t;
      }
      int pos = incl - pc;
      for (uint32_t b = bits; b != 0u; b &= b - 1u) slist[pos++] = int32_t(c0) + w * 32 + (__ffs(b) - 1);
      if (w == 63) scount = incl;
    }
    __syncthreads();
    const int nlist = scount;
    for (int b0 = 0; b0 < nlist; b0 += kBatchU) {
      const int nbu = min(kBatchU, nlist - b0);
      const int cntp = nbu * kUnit;
      __syncthreads();
      for (int t = threadIdx.x; t < cntp; t += kBlock) {
        const int64_t sl = int64_t(slist[b0 + t / kUnit]) * kUnit + (t % kUnit);
        tile[t] = sl < end ? pos4[sl] : make_float4(0.f, 0.f, 0.f, -3.0e38f);
      }
      __syncthreads();
      for (int j = 0; j < cntp; j += 2) {
        const float4 P0 = tile[j], P1 = tile[j + 1];
#pragma unroll
        for (int k = 0; k < kQpl; ++k) {
          const float a0 = fmaf(qz[k], P0.z, fmaf(qy[k], P0.y, fmaf(qx[k], P0.x, P0.w)));
          const float a1 = fmaf(qz[k], P1.z, fmaf(qy[k], P1.y, fmaf(qx[k], P1.x, P1.w)));
          acc[k] = fmaxf(acc[k], fmaxf(a0, a1));
        }
      }
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
