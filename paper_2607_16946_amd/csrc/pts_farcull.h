// pts_farcull.h -- exact culling of the farthest-point sweep (the maximum of
// Eq. RelationshipBetweenLambdaAndRadius), shared by the single-request sweep
// (pts_eval.hip) and the packed serving sweep (pts_multi.hip).
//
// With LB <= M the largest distance from a query to some actual points (the
// extreme points e_u of chosen 64-slot units), a unit whose bounding sphere
// (c, r) has |x - c| + r < LB (1 - 1e-5) for every query of the workgroup
// cannot hold the farthest point: its points are at least 1e-5 M nearer than
// M, far above FP32 rounding of the swept values.  Only the other units are
// swept, in ascending slot order, so the maximum (and, with kArg, the first
// slot attaining it) is exactly that of a full sweep over the same points.
#pragma once

#include "pts_device.h"

namespace pts {

constexpr int kChunkU = 256;             // units whose bounds are staged in LDS at once
constexpr int kBatchU = kTile1 / kUnit;  // units per LDS tile of points
constexpr int kSampleU = 64;             // units sampled across a cloud when a sweep covers one point split

// LDS of one workgroup's culled sweep.
struct FarLds {
  float4 sb[kChunkU];
  uint32_t smask[kChunkU / 32];
  int32_t slist[kChunkU];
  int32_t scount;
  float4 tile[kTile1];
};

// lb[k] = max(lb[k], largest squared distance from query k to the extreme
// points of the units unit_of(i), i in [0, n)).
template <int QPL, class UnitOf>
__device__ __forceinline__ void far_bound(const float4* __restrict__ ub, int64_t n, UnitOf unit_of,
                                          const float (&qx)[QPL], const float (&qy)[QPL], const float (&qz)[QPL],
                                          float (&lb)[QPL], FarLds& L) {
  for (int64_t c0 = 0; c0 < n; c0 += kChunkU) {
    const int cnt = int(min<int64_t>(kChunkU, n - c0));
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += kBlock) L.sb[j] = ub[2 * unit_of(c0 + j) + 1];
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const float4 E = L.sb[j];
#pragma unroll
      for (int k = 0; k < QPL; ++k) {
        const float dx = qx[k] - E.x, dy = qy[k] - E.y, dz = qz[k] - E.z;
        lb[k] = fmaxf(lb[k], fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
      }
    }
  }
}

// The bound of a sweep over the point split [u_lo, u_hi) of a cloud of U
// units, in two steps so that a split no query can reach costs only the
// sample: the extreme points of kSampleU units sampled across the cloud
// first; then, only if some block sphere (bb) over the split's units
// [u_lo, u_hi) reaches that bound's threshold for some query of the
// workgroup, those of the split's own units.  Returns false (uniform across
// the workgroup) when none does: the split then holds no point at any
// query's farthest distance, and nothing of it needs sweeping.
template <int QPL>
__device__ __forceinline__ bool far_bound_split_reach(const float4* __restrict__ ub, const float4* __restrict__ bb,
                                                      int64_t U, int64_t u_lo, int64_t u_hi, const float (&qx)[QPL],
                                                      const float (&qy)[QPL], const float (&qz)[QPL],
                                                      const bool (&ok)[QPL], float (&lb)[QPL], FarLds& L) {
  const int64_t stride = (U + kSampleU - 1) / kSampleU;
  const int64_t n_samp = (U + stride - 1) / stride;
  far_bound<QPL>(ub, n_samp, [=](int64_t i) { return i * stride; }, qx, qy, qz, lb, L);
  bool reach = false;
  for (int64_t b = u_lo / kBlkU; b < (u_hi + kBlkU - 1) / kBlkU; ++b) {
    const float4 C = bb[b];
#pragma unroll
    for (int k = 0; k < QPL; ++k) {
      const float t = sqrtf(fmaxf(lb[k], 0.f)) * (1.f - 1e-5f) - C.w;
      const float dx = qx[k] - C.x, dy = qy[k] - C.y, dz = qz[k] - C.z;
      const float dc2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
      reach = reach || (ok[k] && lb[k] >= 0.f && (t <= 0.f || !(dc2 < t * t)));
    }
  }
  if (!__syncthreads_or(reach)) return false;
  far_bound<QPL>(ub, u_hi - u_lo, [=](int64_t i) { return u_lo + i; }, qx, qy, qz, lb, L);
  return true;
}

// The squared bound becomes the cull threshold LB (1 - 1e-5); a query with a
// NaN coordinate needs no unit (its M is NaN whatever is swept).
template <int QPL>
__device__ __forceinline__ void far_threshold(float (&lb)[QPL], bool (&ok)[QPL]) {
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    ok[k] = ok[k] && lb[k] >= 0.f;
    lb[k] = sqrtf(fmaxf(lb[k], 0.f)) * (1.f - 1e-5f);
  }
}

// The spheres sb[0, cnt) (staged in LDS, mask cleared, both behind a barrier)
// that some query of the workgroup can reach beyond its threshold lb
// (|x - c| + r >= lb), as the ascending list of i0 + j in list[0, *count).
// Ends behind a barrier.
template <int QPL>
__device__ __forceinline__ void far_mark(const float4* sb, int cnt, int32_t i0, const float (&qx)[QPL],
                                         const float (&qy)[QPL], const float (&qz)[QPL], const bool (&ok)[QPL],
                                         const float (&lb)[QPL], uint32_t* mask, int32_t* list, int32_t* count) {
  for (int j = 0; j < cnt; ++j) {
    const float4 C = sb[j];
    bool need = false;
#pragma unroll
    for (int k = 0; k < QPL; ++k) {
      const float t = lb[k] - C.w;
      const float dx = qx[k] - C.x, dy = qy[k] - C.y, dz = qz[k] - C.z;
      const float dc2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
      need = need || (ok[k] && (t <= 0.f || !(dc2 < t * t)));
    }
    if (__ballot(need) != 0ull && (threadIdx.x & 63) == 0) atomicOr(&mask[j >> 5], 1u << (j & 31));
  }
  __syncthreads();
  if (threadIdx.x < 64) {  // ascending list (first wave)
    const int w = int(threadIdx.x);
    const uint32_t bits = w < kChunkU / 32 ? mask[w] : 0u;
    const int pc = __popc(bits);
    int incl = pc;
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o);
      if (w >= o) incl += t;
    }
    int pos = incl - pc;
    for (uint32_t b = bits; b != 0u; b &= b - 1u) list[pos++] = i0 + w * 32 + (__ffs(b) - 1);
    if (w == 63) *count = incl;
  }
  __syncthreads();
}

// Sweep the units of [u_lo, u_hi) that some query of the workgroup needs:
// acc[k] = max over their points of |p|^2 - 2<x,p> (slots >= slot_end are
// padding), and with kArg ix[k] the first slot attaining it.
template <int QPL, bool kArg>
__device__ __forceinline__ void far_sweep(const float4* __restrict__ pos4, const float4* __restrict__ ub,
                                          int64_t u_lo, int64_t u_hi, int64_t slot_end, const float (&qx)[QPL],
                                          const float (&qy)[QPL], const float (&qz)[QPL], const bool (&ok)[QPL],
                                          const float (&lb)[QPL], float (&acc)[QPL], int32_t (&ix)[QPL],
                                          FarLds& L) {
  for (int64_t c0 = u_lo; c0 < u_hi; c0 += kChunkU) {
    const int cnt = int(min<int64_t>(kChunkU, u_hi - c0));
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += kBlock) L.sb[j] = ub[2 * (c0 + j)];
    for (int j = threadIdx.x; j < kChunkU / 32; j += kBlock) L.smask[j] = 0u;
    __syncthreads();
    far_mark<QPL>(L.sb, cnt, int32_t(c0), qx, qy, qz, ok, lb, L.smask, L.slist, &L.scount);
    // sweep their points, a tile of kBatchU units at a time
    const int nlist = L.scount;
    for (int b0 = 0; b0 < nlist; b0 += kBatchU) {
      const int nbu = min(kBatchU, nlist - b0);
      const int cntp = nbu * kUnit;
      __syncthreads();
      for (int t = threadIdx.x; t < cntp; t += kBlock) {
        const int64_t sl = int64_t(L.slist[b0 + t / kUnit]) * kUnit + (t % kUnit);
        L.tile[t] = sl < slot_end ? pos4[sl] : make_float4(0.f, 0.f, 0.f, -3.0e38f);
      }
      __syncthreads();
      if (kArg) {
        for (int u = 0; u < nbu; ++u) {
          const int32_t base = L.slist[b0 + u] * kUnit;
          for (int j = 0; j < kUnit; ++j) {
            const float4 P = L.tile[u * kUnit + j];
#pragma unroll
            for (int k = 0; k < QPL; ++k) {  // branch-free: the first slot attaining the maximum
              const float a = fmaf(qz[k], P.z, fmaf(qy[k], P.y, fmaf(qx[k], P.x, P.w)));
              const bool gt = a > acc[k];
              acc[k] = gt ? a : acc[k];
              ix[k] = gt ? base + j : ix[k];
            }
          }
        }
      } else {
        for (int j = 0; j < cntp; j += 2) {
          const float4 P0 = L.tile[j], P1 = L.tile[j + 1];
#pragma unroll
          for (int k = 0; k < QPL; ++k) {
            const float a0 = fmaf(qz[k], P0.z, fmaf(qy[k], P0.y, fmaf(qx[k], P0.x, P0.w)));
            const float a1 = fmaf(qz[k], P1.z, fmaf(qy[k], P1.y, fmaf(qx[k], P1.x, P1.w)));
            acc[k] = fmaxf(acc[k], fmaxf(a0, a1));
          }
        }
      }
    }
  }
}

// The needed blocks of one chunk of block spheres (far_tree).
struct FarBlkLds {
  uint32_t mask[kChunkU / 32];
  int32_t list[kChunkU];
  int32_t count;
};

// The sweep over all U units of a cloud, through the blocks of kBlkU units
// whose spheres bb enclose their units' spheres.  The bound starts from the
// extreme points of kSampleU units sampled across the cloud and is raised by
// those of every unit of each block that can reach it; the unit attaining the
// largest extreme-point distance lies in such a block, so the bound ends equal
// to the one over every unit.  The blocks that can reach the final threshold
// are then swept in ascending order (far_sweep over their units); a block
// that cannot holds no unit that could, so the maximum (and, with kArg, the
// first slot attaining it) is that of far_sweep over [0, U).
template <int QPL, bool kArg>
__device__ __forceinline__ void far_tree(const float4* __restrict__ pos4, const float4* __restrict__ ub,
                                         const float4* __restrict__ bb, int64_t U, int64_t slot_end,
                                         const float (&qx)[QPL], const float (&qy)[QPL], const float (&qz)[QPL],
                                         bool (&ok)[QPL], float (&acc)[QPL], int32_t (&ix)[QPL], FarLds& L,
                                         FarBlkLds& B) {
  const int64_t NB = (U + kBlkU - 1) / kBlkU;
  const int64_t stride = (U + kSampleU - 1) / kSampleU;
  float lb[QPL];
#pragma unroll
  for (int k = 0; k < QPL; ++k) lb[k] = -1.f;
  far_bound<QPL>(ub, (U + stride - 1) / stride, [=](int64_t i) { return i * stride; }, qx, qy, qz, lb, L);
  // pass 0 raises the bound over the blocks that reach it; pass 1 sweeps the
  // blocks that reach the final threshold
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) far_threshold<QPL>(lb, ok);
    for (int64_t c0 = 0; c0 < NB; c0 += kChunkU) {
      const int cnt = int(min<int64_t>(kChunkU, NB - c0));
      float thr[QPL];
      bool okt[QPL];
#pragma unroll
      for (int k = 0; k < QPL; ++k) {
        okt[k] = pass == 1 ? ok[k] : (ok[k] && lb[k] >= 0.f);
        thr[k] = pass == 1 ? lb[k] : sqrtf(fmaxf(lb[k], 0.f)) * (1.f - 1e-5f);
      }
      __syncthreads();
      for (int j = threadIdx.x; j < cnt; j += kBlock) L.sb[j] = bb[c0 + j];
      for (int j = threadIdx.x; j < kChunkU / 32; j += kBlock) B.mask[j] = 0u;
      __syncthreads();
      far_mark<QPL>(L.sb, cnt, int32_t(c0), qx, qy, qz, okt, thr, B.mask, B.list, &B.count);
      const int nl = B.count;
      for (int i = 0; i < nl; ++i) {
        const int64_t u0 = int64_t(B.list[i]) * kBlkU, u1 = min(U, u0 + kBlkU);
        if (pass == 0)
          far_bound<QPL>(ub, u1 - u0, [=](int64_t t) { return u0 + t; }, qx, qy, qz, lb, L);
        else
          far_sweep<QPL, kArg>(pos4, ub, u0, u1, slot_end, qx, qy, qz, ok, lb, acc, ix, L);
      }
    }
  }
}

// Splits of at most this many points are swept whole: the bound and marking
// phases (three rounds of loads and barriers) cost more than the sweep they
// save.
constexpr int64_t kFarPlainMax = 1024;

// The same maximum (and first slot attaining it) over every point of
// [beg, end), without culling.
template <int QPL, bool kArg>
__device__ __forceinline__ void far_sweep_plain(const float4* __restrict__ pos4, int64_t beg, int64_t end,
                                                const float (&qx)[QPL], const float (&qy)[QPL],
                                                const float (&qz)[QPL], float (&acc)[QPL], int32_t (&ix)[QPL],
                                                FarLds& L) {
  for (int64_t t0 = beg; t0 < end; t0 += kTile1) {
    const int cnt = int(min<int64_t>(kTile1, end - t0));
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += kBlock) L.tile[t] = pos4[t0 + t];
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const float4 P = L.tile[j];
#pragma unroll
      for (int k = 0; k < QPL; ++k) {
        const float a = fmaf(qz[k], P.z, fmaf(qy[k], P.y, fmaf(qx[k], P.x, P.w)));
        if (kArg) {
          const bool gt = a > acc[k];
          acc[k] = gt ? a : acc[k];
          ix[k] = gt ? int32_t(t0 + j) : ix[k];
        } else {
          acc[k] = fmaxf(acc[k], a);
        }
      }
    }
  }
}

}  // namespace pts
