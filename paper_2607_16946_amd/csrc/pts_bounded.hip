// pts_bounded.hip -- phi of Eq. (BasicFormulaShifted) with far point units
// skipped under a proven bound on the change of phi.
//
// The bound.  Every torus passes through its anchor o_i = p_i + a00_i n_i
// (Sec. 4.1), so |g_i(x)| <= |x - o_i| <= |x - p_i| + A with A = max |a00|.
// For a unit of n points whose distances to a query x lie in [d_lo, d_hi],
// every weight is at most w_u = exp(-lambda_x (d_lo - sigma_x)) and every
// |g_i| at most d_hi + A, so the unit adds at most
//   d_u = n w_u  to the denominator,  g_u = d_u (d_hi + A)  to |numerator|.
// A 4096-point block takes d_lo = max(s - r, 0), d_hi = s + r from its
// bounding sphere (c, r), s = |x - c|; a 64-point unit takes them from its
// oriented box (the build's unit boxes, first axis along the unit's mean
// normal): with t_k = |<x - c, a_k>| and half-extents e_k,
// d_lo = |max(t - e, 0)| and d_hi = |t + e|.  Surface patches are thin along
// their normal, so the box's d_lo is well above the sphere's for queries off
// the surface.
// If the skipped units' totals are D_s <= sum d_u and G_s <= sum g_u and the
// kept sums give phi' = N_k / D_k, then
//   |phi - phi'| = |N_s - phi' D_s| / (D_k + D_s) <= (G_s + |phi'| D_s) / D_k,
// and |phi'| <= Phi = M + A (every |g_i| <= |x - p_i| + A <= M + A).  A unit
// is skipped only while G_s + Phi D_s (totals including it) stays within
// eps D_run, the kept denominator so far; D_run <= D_k, so the final bound
// (G_s + |phi'| D_s) / D_k <= eps.  The kernel reports that bound per query.
// Which skips to take is free within that rule: a unit's skip may also spend
// no more than a quarter of the budget still left, so that early, expensive
// skips do not use up what the many cheap far units would need.
// Bounds carry a relative slack of 1e-4 for FP32 rounding of s, the exponent
// and D_run, and the budget gives up U 2^-23 (U units) for the bounds that
// the FP32 running sums of G_s and D_s absorb; the returned phi' itself has
// the rounding of the plain blend.
//
// Making skips pay.  A unit's work is skipped by a whole wave or not at all,
// so the wave's queries must agree: queries are processed in Morton order of
// the cloud's bbox (a radix sort of the query keys on the device) and each
// lane takes QPL consecutive sorted queries, so a wave covers a compact brick
// of 64 QPL queries.  Each workgroup is one wave, which stages into LDS only
// the units it keeps: no wave waits on units only another keeps.  D_run must
// be large early: each wave starts its sweep at the unit nearest to its first
// query and wraps around its point range.
//
// Splits.  The path has its own plan: one point range per query block unless
// that leaves fewer than ~2048 workgroups, then S ranges.  A range far from
// its queries keeps only tiny weights, so its own kept denominator would
// allow few skips; instead every workgroup of a query block first computes the
// weights W_seed of one shared seed unit (the unit nearest the block's first
// query).  The range holding it sweeps it first and always keeps it (nothing is
// skipped against an empty denominator); every other range skips against
// W_seed plus its own kept sum, each with budget eps / (S + 1).  Summed over
// ranges the skipped bounds are at most eps / (S + 1) (S W_seed + D_k) <= eps D_k.
//
//   k_qkeys    Morton key (3 x 8 bits over the cloud's bbox) of every query
//   (radix sort of the keys, pts_build.hip)
//   k_bwork    per query block: a work estimate (seen from the block's first
//              query, the units whose skip bound exceeds a 1/(10 U) share of
//              the budget eps W, W summed from the unit centres; both sums
//              over every fourth unit, scaled up), sorted by
//              half-octave buckets of it so that heavy blocks launch first
//              and the tail of the launch is light, neighbouring blocks
//              staying together within a bucket (ordering only: a block's
//              result does not depend on when it runs)
//   k_bounded  the sweep: a wave votes per block of 64 units (4096 points)
//              and, in blocks it keeps, per 64-point unit; kept units are
//              staged and run the blend's pair arithmetic
//   k_bcombine fixed-order sum over splits, phi', the bound, kept counts
#include "pts_device.h"

#include <algorithm>

namespace pts {
namespace {

constexpr float kSlack = 1e-4f;

__device__ inline uint32_t spread3_8(uint32_t v) {
  uint32_t r = 0;
  for (int k = 0; k < 8; ++k) r |= ((v >> k) & 1u) << (3 * k);
  return r;
}

__global__ __launch_bounds__(kBlock) void k_qkeys(const Header* __restrict__ h, const float* __restrict__ x,
                                                  int64_t Q, uint32_t* __restrict__ key, int32_t* __restrict__ idx) {
  const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= Q) return;
  uint32_t m = 0;
  for (int k = 0; k < 3; ++k) {
    const float lo = h->lo[k], ext = h->hi[k] - h->lo[k];
    float t = ext > 0.f ? (x[3 * q + k] - lo) / ext * 256.f : 0.f;
    t = t < 0.f ? 0.f : (t > 255.f ? 255.f : t);   // NaN compares false: stays NaN -> below
    int c = t == t ? int(t) : 0;
    m |= spread3_8(uint32_t(c)) << k;
  }
  key[q] = m;
  idx[q] = int32_t(q);
}

template <bool kDirect>
__device__ __forceinline__ void pair(float qx, float qy, float qz, float nl, float S2, const float4& P,
                                     const float4& U, const float4& Mv, const float4& K, const float4& G, float& tn,
                                     float& td) {
  const float dx = qx - P.x, dy = qy - P.y, dz = qz - P.z;
  const float d = hw_sqrt(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
  const float w = hw_exp2(fmaf(d, nl, S2));
  const float g = kDirect ? g_direct(qx, qy, qz, U, Mv, K, G) : g_anchored(qx, qy, qz, P.w, U, Mv, K, G);
  tn = fmaf(w, g, tn);
  td += w;
}

// Blocks taken nearest-first at the start of a wave's sweep.
constexpr int kNear = 8;

// One wavefront per workgroup: waves sweep, vote and stage independently (a
// wave never waits on units only another wave keeps).
constexpr int kBW = 64;

// Unit nearest (by sphere lower bound) to (rx, ry, rz) among units [u0, u1);
// ties to the lower index.  Wave-wide.
__device__ int64_t nearest_unit(const float4* __restrict__ ub, int64_t u0, int64_t u1, float rx, float ry, float rz,
                                float* red_v, int32_t* red_i) {
  float best = 3.0e38f;
  int32_t bi = int32_t(u0);
  for (int64_t u = u0 + threadIdx.x; u < u1; u += kBW) {
    const float4 cb = ub[2 * u];
    const float ex = rx - cb.x, ey = ry - cb.y, ez = rz - cb.z;
    const float lb = sqrtf(fmaf(ez, ez, fmaf(ey, ey, ex * ex))) - cb.w;
    if (lb < best) { best = lb; bi = int32_t(u); }
  }
  __syncthreads();
  red_v[threadIdx.x] = best;
  red_i[threadIdx.x] = bi;
  __syncthreads();
  for (int o = kBW / 2; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) {
      const float v2 = red_v[threadIdx.x + o];
      const int32_t i2 = red_i[threadIdx.x + o];
      if (v2 < red_v[threadIdx.x] || (v2 == red_v[threadIdx.x] && i2 < red_i[threadIdx.x])) {
        red_v[threadIdx.x] = v2;
        red_i[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  return red_i[0];
}

// The queries in Morton order: the sweeps below read them, and M, by sorted
// position.
__global__ __launch_bounds__(kBlock) void k_gather(const float* __restrict__ x, const int32_t* __restrict__ order,
                                                   int64_t Q, float* __restrict__ xs) {
  const int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (j >= Q) return;
  const int64_t q = order[j];
  xs[3 * j] = x[3 * q];
  xs[3 * j + 1] = x[3 * q + 1];
  xs[3 * j + 2] = x[3 * q + 2];
}

// Threads per workgroup of k_bwork: small, so its few thousand threads spread
// over every compute unit.
constexpr int kWorkBlock = 64;
// k_bwork looks at every kWorkStride-th unit and scales the sums back up: the
// estimate only orders the blocks, and a quarter of the units orders them as
// well as all of them.
constexpr int kWorkStride = 4;

__global__ __launch_bounds__(kWorkBlock) void k_bwork(const Header* __restrict__ h, const float4* __restrict__ ub,
                                                      const float* __restrict__ xs,
                                                      int64_t Q, int64_t nqb, int qpl, const float* __restrict__ far2,
                                                      float C2, float S2, float eps, uint32_t* __restrict__ key,
                                                      int32_t* __restrict__ idx) {
  const int64_t b = int64_t(blockIdx.x) * kWorkBlock + threadIdx.x;
  if (b >= nqb) return;
  const int64_t j = b * kBW * qpl;  // the block's first sorted position
  const QueryIn r = load_query(xs, j, Q, h);
  float M = 0.f, nl = 0.f;
  far_of(far2, 1, Q, j, C2, M, nl);
  const float A = __uint_as_float(h->a00max_bits);
  const int64_t nunit = (h->N + kUnit - 1) / kUnit;
  // W from the unit centres, then the units whose skip bound (as the vote
  // prices it) exceeds a share eps W / (10 U) of the budget: those the sweep
  // must evaluate, about; both over every kWorkStride-th unit
  float W = 0.f;
  for (int64_t u = 0; u < nunit; u += kWorkStride) {
    const float4 cb = ub[2 * u];
    const float ex = r.x - cb.x, ey = r.y - cb.y, ez = r.z - cb.z;
    W += hw_exp2(fmaf(hw_sqrt(fmaf(ez, ez, fmaf(ey, ey, ex * ex))), nl, S2));
  }
  const float thr = eps * (float(kWorkStride) * W) / (10.f * float(nunit));
  uint32_t cnt = 0;
  for (int64_t u = 0; u < nunit; u += kWorkStride) {
    const float4 cb = ub[2 * u];
    const float ex = r.x - cb.x, ey = r.y - cb.y, ez = r.z - cb.z;
    const float s = hw_sqrt(fmaf(ez, ez, fmaf(ey, ey, ex * ex)));
    const float du = hw_exp2(fmaf(fmaxf(s - cb.w, 0.f), nl, S2));
    cnt += du * (s + cb.w + M + 2.f * A) > thr ? 1u : 0u;
  }
  // half-octave buckets of the estimate, heaviest first; the sort is stable
  // and bricks come in Morton order, so within a bucket they stay in it
  key[b] = 63u - min(63u, uint32_t(2.f * log2f(float(kWorkStride * cnt) + 1.f)));
  idx[b] = int32_t(b);
}

// The wave's vote on skipping n points inside the sphere sb = (c, r): true
// (and the skipped bounds added) if every live query's budget allows it.
template <int QPL>
__device__ __forceinline__ bool vote(const float4& sb, float n, const float* qx, const float* qy, const float* qz,
                                     const float* nl, float S2, float A, const float* phimax, float* gs, float* ds,
                                     const float* den, const float* wseed, float eps, const bool* live) {
  float du[QPL], gu[QPL];
  bool ok = true;
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const float ex = qx[k] - sb.x, ey = qy[k] - sb.y, ez = qz[k] - sb.z;
    const float s = hw_sqrt(fmaf(ez, ez, fmaf(ey, ey, ex * ex)));
    const float dmin = fmaxf(s * (1.f - kSlack) - sb.w * (1.f + kSlack), 0.f);
    du[k] = n * hw_exp2(fmaf(dmin, nl[k], S2)) * (1.f + kSlack);
    gu[k] = du[k] * (s + sb.w + A) * (1.f + kSlack);
    const bool skip = (gs[k] + gu[k]) + phimax[k] * (ds[k] + du[k]) <= eps * (den[k] * (1.f - kSlack) + wseed[k]);
    ok = ok && (skip || !live[k]);
  }
  if (__ballot(!ok) != 0ull) return false;
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    gs[k] += gu[k];
    ds[k] += du[k];
  }
  return true;
}

// The largest share of the remaining budget one unit's skip may spend.
constexpr float kSkipShare = 0.25f;

// The same vote for the n points of a unit inside the oriented box B[0..3]
// (center, then axis and half-extent per axis): with t_k = |<x - c, a_k>|,
// every point is at least |max(t - e, 0)| and at most |t + e| from x.  The
// lower bound gives up kSlack of the upper one for the FP32 rounding of t.
template <int QPL>
__device__ __forceinline__ bool vote_box(const float4* __restrict__ B, float n, const float* qx, const float* qy,
                                         const float* qz, const float* nl, float S2, float A, const float* phimax,
                                         float* gs, float* ds, const float* den, const float* wseed, float eps,
                                         const bool* live) {
  const float4 C = B[0], A0 = B[1], A1 = B[2], A2 = B[3];
  float du[QPL], gu[QPL];
  bool ok = true;
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const float ex = qx[k] - C.x, ey = qy[k] - C.y, ez = qz[k] - C.z;
    const float t0 = fabsf(fmaf(ez, A0.z, fmaf(ey, A0.y, ex * A0.x)));
    const float t1 = fabsf(fmaf(ez, A1.z, fmaf(ey, A1.y, ex * A1.x)));
    const float t2 = fabsf(fmaf(ez, A2.z, fmaf(ey, A2.y, ex * A2.x)));
    const float l0 = fmaxf(t0 - A0.w, 0.f), l1 = fmaxf(t1 - A1.w, 0.f), l2 = fmaxf(t2 - A2.w, 0.f);
    const float h0 = t0 + A0.w, h1 = t1 + A1.w, h2 = t2 + A2.w;
    const float dmax = hw_sqrt(fmaf(h2, h2, fmaf(h1, h1, h0 * h0))) * (1.f + kSlack);
    const float dmin = fmaxf(hw_sqrt(fmaf(l2, l2, fmaf(l1, l1, l0 * l0))) - kSlack * dmax, 0.f);
    du[k] = n * hw_exp2(fmaf(dmin, nl[k], S2)) * (1.f + kSlack);
    gu[k] = du[k] * (dmax + A) * (1.f + kSlack);
    const float budget = eps * (den[k] * (1.f - kSlack) + wseed[k]);
    const bool fits = (gs[k] + gu[k]) + phimax[k] * (ds[k] + du[k]) <= budget;
    // and no more than kSkipShare of what is left of the budget (or a share
    // of it below FP32 resolution): skips that would spend much of it are
    // kept, so the budget lasts for the many cheap units further out
    const float cost = gu[k] + phimax[k] * du[k];
    const bool share = cost <= kSkipShare * (budget - (gs[k] + phimax[k] * ds[k])) || cost <= 1e-7f * budget;
    ok = ok && ((fits && share) || !live[k]);
  }
  if (__ballot(!ok) != 0ull) return false;
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    gs[k] += gu[k];
    ds[k] += du[k];
  }
  return true;
}

template <int QPL>
// 8 waves per SIMD (at most 64 VGPRs)
__global__ __launch_bounds__(kBW, 8) void k_bounded(const Header* __restrict__ h, const float4* __restrict__ rec,
                                                 const float4* __restrict__ ub, const float4* __restrict__ bb,
                                                 const float4* __restrict__ ob,
                                                 const float* __restrict__ xs, const int32_t* __restrict__ border,
                                                 int64_t Q, int S, int64_t per_split,
                                                 const float* __restrict__ far2, float C2, float S2, float eps_total,
                                                 float4* __restrict__ part, int32_t* __restrict__ kpart) {
  // 5 KB of LDS per wave (8 waves per SIMD); the seed searches' reductions
  // use the unit tile, which holds nothing yet (every tile write is preceded
  // by a barrier that also orders the reductions' reads)
  __shared__ float4 tile[kUnit * kRecF4];
  float* red_v = reinterpret_cast<float*>(tile);
  int32_t* red_i = reinterpret_cast<int32_t*>(tile) + kBW;
  const int split = int(blockIdx.x % unsigned(S));
  const int64_t qb = border[blockIdx.x / unsigned(S)];
  const int64_t N = h->N;
  const int64_t nd = h->n_direct;
  const float A = __uint_as_float(h->a00max_bits);
  const int64_t j0 = qb * (kBW * QPL);          // first sorted position of the wave
  float qx[QPL], qy[QPL], qz[QPL], nl[QPL], phimax[QPL], num[QPL], den[QPL], gs[QPL], ds[QPL], wseed[QPL];
  bool live[QPL];
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int64_t j = j0 + int64_t(threadIdx.x) * QPL + k;
    live[k] = j < Q;
    const QueryIn qi = load_query(xs, j, live[k] ? Q : 0, h);
    qx[k] = qi.x; qy[k] = qi.y; qz[k] = qi.z;
    // a query with a non-finite coordinate (its phi is NaN) takes no part in
    // the votes, which its NaN bounds would otherwise block for the wave
    live[k] = live[k] && isfinite(qi.x) && isfinite(qi.y) && isfinite(qi.z);
    float M = 0.f;
    nl[k] = 0.f;
    if (qi.valid) far_of(far2, 1, Q, j, C2, M, nl[k]);
    phimax[k] = M + A;
    num[k] = den[k] = gs[k] = ds[k] = wseed[k] = 0.f;
  }
  const int64_t beg = int64_t(split) * per_split;
  const int64_t end = min(N, beg + per_split);
  const int64_t u_beg = beg / kUnit, u_end = (end + kUnit - 1) / kUnit;
  // every skip adds its bounds to FP32 sums, and each addition may lose up
  // to 2^-24 of the sum it lands in; with at most one addition per unit and
  // per block, the budget gives that up front (U 2^-23, U units)
  const float absorb = fminf(0.5f, float((N + kUnit - 1) / kUnit) * 0x1p-23f);
  const float eps = (S > 1 ? eps_total / float(S + 1) : eps_total) * (1.f - absorb);
  // the wave's first query with finite coordinates (in lane order; the first
  // query if none is), in record coordinates: it seeds the sweep's order
  QueryIn r0 = load_query(xs, j0, Q, h);
  {
    const unsigned long long fin = __ballot(live[0]);
    if (fin != 0ull) {
      const int src = __builtin_ctzll(fin);
      r0.x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(qx[0]), src));
      r0.y = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(qy[0]), src));
      r0.z = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(qz[0]), src));
    }
  }
  const int64_t useed = nearest_unit(ub, 0, (N + kUnit - 1) / kUnit, r0.x, r0.y, r0.z, red_v, red_i);
  int64_t ustart = useed;
  if (useed < u_beg || useed >= u_end) {
    // W_seed per query (the range holding the seed keeps it), then this range's own nearest unit
    const int64_t s0 = useed * kUnit, s1 = min(N, s0 + kUnit);
    for (int64_t sl = s0; sl < s1; ++sl) {
      const float4 P = rec[sl * kRecF4];
#pragma unroll
      for (int k = 0; k < QPL; ++k) {
        const float dx = qx[k] - P.x, dy = qy[k] - P.y, dz = qz[k] - P.z;
        const float d = hw_sqrt(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
        wseed[k] += hw_exp2(fmaf(d, nl[k], S2));
      }
    }
#pragma unroll
    for (int k = 0; k < QPL; ++k) wseed[k] *= (1.f - kSlack);
    ustart = nearest_unit(ub, u_beg, u_end, r0.x, r0.y, r0.z, red_v, red_i);
  }
  int32_t kept = 0;
  // Blocks of kBlkU units (their bounding spheres from the build): the block
  // of the first unit, then the kNear - 1 blocks nearest to the wave's first
  // query (by sphere lower bound, ties to the lower index), nearest first,
  // then the others from the first unit's block on, wrapping.  The kept
  // denominator is then close to its final value before far blocks are voted
  // on.  Within the first block the sweep starts at the first unit.
  const int64_t b_beg = u_beg / kBlkU, b_end = (u_end + kBlkU - 1) / kBlkU, nbk = b_end - b_beg;
  const int64_t bstart = ustart / kBlkU;
  // (eps = 0 skips nothing: index order, whose shared walk keeps the records
  // that neighbouring waves read in L2)
  const int n_near = eps_total > 0.f ? int(min<int64_t>(kNear, nbk)) : 1;
  // the list: lane t holds entry t (read back with readlane, no LDS)
  int32_t near_l = int32_t(bstart);
  for (int t = 1; t < n_near; ++t) {
    float best = 3.0e38f;
    int32_t bi = INT32_MAX;
    for (int64_t b = b_beg + threadIdx.x; b < b_end; b += kBW) {
      bool taken = false;
      for (int i = 0; i < t; ++i) taken = taken || __builtin_amdgcn_readlane(near_l, i) == int32_t(b);
      if (taken) continue;
      const float4 cb = bb[b];
      const float ex = r0.x - cb.x, ey = r0.y - cb.y, ez = r0.z - cb.z;
      float lb = hw_sqrt(fmaf(ez, ez, fmaf(ey, ey, ex * ex))) - cb.w;
      // a NaN or overflowing bound (seed not finite, or too far out) counts as
      // the largest: such blocks tie and the lowest index wins, so every
      // round of the search picks a block
      lb = lb < 3.0e38f ? lb : 3.0e38f;
      if (lb < best || (lb == best && int32_t(b) < bi)) { best = lb; bi = int32_t(b); }
    }
#pragma unroll
    for (int o = kBW / 2; o > 0; o >>= 1) {
      const float v2 = __shfl_xor(best, o, kBW);
      const int32_t i2 = __shfl_xor(bi, o, kBW);
      if (v2 < best || (v2 == best && i2 < bi)) { best = v2; bi = i2; }
    }
    if (int(threadIdx.x) == t) near_l = bi;
  }
  for (int64_t ib = 0, iw = 0; ib < nbk; ++ib) {
    int64_t b;
    if (ib < n_near) {
      b = __builtin_amdgcn_readlane(near_l, int(ib));
    } else {
      for (;;) {  // the next block in wrap order not visited among the nearest
        b = bstart + iw++;
        if (b >= b_end) b -= nbk;
        bool taken = false;
        for (int i = 0; i < n_near; ++i) taken = taken || __builtin_amdgcn_readlane(near_l, i) == int32_t(b);
        if (!taken) break;
      }
      b = __builtin_amdgcn_readfirstlane(int32_t(b));
    }
    const int64_t bu0 = max(b * kBlkU, u_beg), bu1 = min(b * kBlkU + kBlkU, u_end);
    if (ib > 0 && vote<QPL>(bb[b], float(min(end, bu1 * kUnit) - bu0 * kUnit), qx, qy, qz, nl, S2, A, phimax, gs, ds, den,
                       wseed, eps, live)) continue;
    const int64_t nub = bu1 - bu0;
    const int64_t us = ib == 0 ? ustart : bu0;
    for (int64_t iu = 0; iu < nub; ++iu) {
      int64_t u = us + iu;
      if (u >= bu1) u -= nub;
      const int64_t t0 = u * kUnit;
      const int cnt = int(min<int64_t>(kUnit, end - t0));
      if (vote_box<QPL>(ob + 4 * u, float(cnt), qx, qy, qz, nl, S2, A, phimax, gs, ds, den, wseed, eps, live))
        continue;
      kept += cnt;
      __syncthreads();                 // the previous unit is read
      for (int j = threadIdx.x; j < cnt * kRecF4; j += kBW) tile[j] = rec[t0 * kRecF4 + j];
      __syncthreads();
      const int jd = int(max<int64_t>(0, min<int64_t>(cnt, nd - t0)));
      float tn[QPL], td[QPL];
#pragma unroll
      for (int k = 0; k < QPL; ++k) { tn[k] = 0.f; td[k] = 0.f; }
#pragma unroll 2
      for (int j = 0; j < jd; ++j) {
        const float4 P = tile[j * kRecF4 + 0], U = tile[j * kRecF4 + 1], Mv = tile[j * kRecF4 + 2],
                     K = tile[j * kRecF4 + 3], G = tile[j * kRecF4 + 4];
#pragma unroll
        for (int k = 0; k < QPL; ++k) pair<true>(qx[k], qy[k], qz[k], nl[k], S2, P, U, Mv, K, G, tn[k], td[k]);
      }
#pragma unroll 2
      for (int j = jd; j < cnt; ++j) {
        const float4 P = tile[j * kRecF4 + 0], U = tile[j * kRecF4 + 1], Mv = tile[j * kRecF4 + 2],
                     K = tile[j * kRecF4 + 3], G = tile[j * kRecF4 + 4];
#pragma unroll
        for (int k = 0; k < QPL; ++k) pair<false>(qx[k], qy[k], qz[k], nl[k], S2, P, U, Mv, K, G, tn[k], td[k]);
      }
#pragma unroll
      for (int k = 0; k < QPL; ++k) { num[k] += tn[k]; den[k] += td[k]; }
    }
  }
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int64_t j = j0 + int64_t(threadIdx.x) * QPL + k;
    if (j < Q) {
      part[int64_t(split) * Q + j] = make_float4(num[k], den[k], gs[k], ds[k]);
      kpart[int64_t(split) * Q + j] = kept;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_bcombine(const float4* __restrict__ part,
                                                     const int32_t* __restrict__ kpart,
                                                     const int32_t* __restrict__ order, int S, int64_t Q,
                                                     float* __restrict__ sdf, float* __restrict__ bound,
                                                     int32_t* __restrict__ kept, float offset) {
  const int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (j >= Q) return;
  float num = 0.f, den = 0.f, gs = 0.f, ds = 0.f;
  int32_t kc = 0;
  for (int s = 0; s < S; ++s) {
    const float4 v = part[int64_t(s) * Q + j];
    num += v.x;
    den += v.y;
    gs += v.z;
    ds += v.w;
    kc += kpart[int64_t(s) * Q + j];
  }
  const int64_t q = order[j];
  const float phi = num / den;
  sdf[q] = phi - offset;
  if (bound) bound[q] = (gs + fabsf(phi) * ds) / den;
  if (kept) kept[q] = kc;
}

template <int QPL>
void launch_bounded_q(const Header* h, const float4* rec, const float4* ub, const float4* bb, const float4* ob,
                      const float* xs, const int32_t* border, int64_t Q, const Plan& plan, const float* far2,
                      float C2, float S2, float eps, float4* part, int32_t* kpart, hipStream_t st) {
  hipLaunchKernelGGL(k_bounded<QPL>, dim3(unsigned(plan.nqb * plan.S)), dim3(kBW), 0, st, h, rec, ub, bb, ob, xs,
                     border, Q, plan.S, plan.per_split, far2, C2, S2, eps, part, kpart);
}

// Workspace: far2 [Q], partials float4 [S][Q], kept int32 [S][Q], keys and
// indices [2][Q] each, radix histograms.
struct BoundedWs {
  float* xs;    // the queries in Morton order [Q][3]
  float* far2;  // M^2 per sorted position
  float4* part;
  int32_t* kpart;
  uint32_t* key[2];
  int32_t* idx[2];
  int32_t* rhist;
  uint32_t* bkey[2];
  int32_t* bidx[2];
  size_t bytes;
};

}  // namespace

// The bounded path's plan: one query per lane (a wave votes for 64 queries;
// measured slightly faster than two per lane), one wavefront per
// workgroup, one point range per query block unless that leaves fewer than
// 8192 workgroups, then up to 64 ranges (multiples of a 64-point unit, at
// least 512 points each).
Plan bounded_plan(int64_t N, int64_t Q) {
  Plan p;
  p.qpl = 1;
  p.nqb = (Q + int64_t(kBW) * p.qpl - 1) / (int64_t(kBW) * p.qpl);
  int S = 1;
  while (S < 64 && p.nqb * S < 8192 && (N + 2 * S - 1) / (2 * S) >= 512) S *= 2;
  p.per_split = ((N + S - 1) / S + kUnit - 1) / kUnit * kUnit;
  p.S = int((N + p.per_split - 1) / p.per_split);
  return p;
}

namespace {

BoundedWs bounded_ws(const Plan& plan, int64_t Q, void* ws) {
  char* c = static_cast<char*>(ws);
  BoundedWs v;
  size_t o = 0;
  auto take = [&](size_t b) {
    char* r = c ? c + o : nullptr;
    o += align256(b);
    return r;
  };
  v.xs = reinterpret_cast<float*>(take(size_t(Q) * 12));
  v.far2 = reinterpret_cast<float*>(take(size_t(Q) * 4));
  v.part = reinterpret_cast<float4*>(take(size_t(plan.S) * size_t(Q) * 16));
  v.kpart = reinterpret_cast<int32_t*>(take(size_t(plan.S) * size_t(Q) * 4));
  for (int i = 0; i < 2; ++i) v.key[i] = reinterpret_cast<uint32_t*>(take(size_t(Q) * 4));
  for (int i = 0; i < 2; ++i) v.idx[i] = reinterpret_cast<int32_t*>(take(size_t(Q) * 4));
  v.rhist = reinterpret_cast<int32_t*>(take(size_t((Q + kBlock - 1) / kBlock) * 16 * 4));
  for (int i = 0; i < 2; ++i) v.bkey[i] = reinterpret_cast<uint32_t*>(take(size_t(plan.nqb) * 4));
  for (int i = 0; i < 2; ++i) v.bidx[i] = reinterpret_cast<int32_t*>(take(size_t(plan.nqb) * 4));
  v.bytes = o;
  return v;
}

}  // namespace

size_t bounded_ws_bytes(const Plan& plan, int64_t Q) { return bounded_ws(plan, Q, nullptr).bytes; }

// The largest workspace of any query count 1..R.  Every section but the
// partials grows with Q; the partials are S x Q, with S constant while the
// query block count nqb stays in [2^k, 2^(k+1) - 1] (bounded_plan doubles S
// while nqb S < 8192), so the largest Q of each such range, and R, cover it.
size_t bounded_ws_max(int64_t N, int64_t R) {
  size_t m = bounded_ws_bytes(bounded_plan(N, R), R);
  for (int64_t nb = 1; nb <= 2 * 8192; nb *= 2) {
    const int64_t q = std::min<int64_t>(R, (2 * nb - 1) * int64_t(kBW));
    m = std::max(m, bounded_ws_bytes(bounded_plan(N, q), q));
  }
  return m;
}

int launch_query_order(const void* rec, const float* x, int64_t Q, uint32_t* key[2], int32_t* idx[2],
                       int32_t* rhist, hipStream_t st, const int32_t** order) {
  const Header* h = static_cast<const Header*>(rec);
  hipLaunchKernelGGL(k_qkeys, dim3(unsigned((Q + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, h, x, Q, key[0],
                     idx[0]);
  if (int rc = check_hip(hipGetLastError(), "query key kernel")) return rc;
  int cur = 0;
  if (int rc = launch_radix_sort(key, idx, Q, 6, rhist, st, &cur)) return rc;
  *order = idx[cur];
  return PTS_OK;
}

int launch_bounded(const void* rec, int64_t N, const float* x, int64_t Q, float eps, float C, const Plan& plan,
                   void* ws, float* sdf, float* bound, int32_t* kept, hipStream_t st, float offset) {
  const Layout L(N);
  const char* base = static_cast<const char*>(rec);
  const Header* h = reinterpret_cast<const Header*>(base);
  const float4* recs = reinterpret_cast<const float4*>(base + L.rec);
  const float4* ub = reinterpret_cast<const float4*>(base + L.ub);
  const float4* bb = reinterpret_cast<const float4*>(base + L.bb);
  const float4* ob = reinterpret_cast<const float4*>(base + L.ob);
  BoundedWs v = bounded_ws(plan, Q, ws);
  const unsigned qblocks = unsigned((Q + kBlock - 1) / kBlock);
  const int32_t* order = nullptr;
  if (int rc = launch_query_order(rec, x, Q, v.key, v.idx, v.rhist, st, &order)) return rc;
  hipLaunchKernelGGL(k_gather, dim3(qblocks), dim3(kBlock), 0, st, x, order, Q, v.xs);
  // M of the sorted queries at up to 4 per lane (exact in any order; the
  // compact Morton blocks let the culling skip more units than the input's
  // order would)
  if (int rc = launch_far_cull(rec, N, v.xs, Q, 4, v.far2, nullptr, st)) return rc;
  // heavy query blocks first
  const float C2 = C * kLog2e, S2 = shift2_of(C);
  hipLaunchKernelGGL(k_bwork, dim3(unsigned((plan.nqb + kWorkBlock - 1) / kWorkBlock)), dim3(kWorkBlock), 0, st, h, ub,
                     v.xs, Q, plan.nqb, plan.qpl, v.far2, C2, S2, eps, v.bkey[0], v.bidx[0]);
  int bcur = 0;
  if (int rc = launch_radix_sort(v.bkey, v.bidx, plan.nqb, 2, v.rhist, st, &bcur)) return rc;
  const int32_t* border = v.bidx[bcur];
  // one query per lane (bounded_plan); the kernel is written for QPL queries
  // per lane, but more than one needs more than 64 VGPRs at 8 waves per SIMD
  if (plan.qpl != 1) return fail(PTS_EINVAL, "bounded evaluation plans one query per lane");
  launch_bounded_q<1>(h, recs, ub, bb, ob, v.xs, border, Q, plan, v.far2, C2, S2, eps, v.part, v.kpart, st);
  hipLaunchKernelGGL(k_bcombine, dim3(qblocks), dim3(kBlock), 0, st, v.part, v.kpart, order, plan.S, Q, sdf, bound,
                     kept, offset);
  return check_hip(hipGetLastError(), "bounded evaluation kernels");
}

}  // namespace pts
