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
// Weights are computed with the shift of Eq. (BasicFormulaShifted), capped at
// 64 (shift2_of in pts_internal.h; the paper's C = 64 is not capped):
//   w = 2^((s - lambda_x |x - p|) log2e)  in [e^(s - 2C), e^s],
// and the sums are accumulated per tile and then per split (two-level), which
// bounds FP32 accumulation error by ~(tile + N/(S tile)) ulp.

#include "pts_farcull.h"

namespace pts {
namespace {

// ---------------------------------------------------------------------------
// Sweep 1: squared distance to the farthest point, M^2 = max_i |x - p_i|^2.
//   |x-p|^2 = |x|^2 + |p|^2 - 2<x,p>; the max is taken over (|p|^2 - 2<x,p>)
//   (three FMAs and a max per pair) and |x|^2 is added once at the end.
// Exact culling by units of kUnit consecutive slots (spatially sorted at
// build time, with bounding spheres and extreme points; pts_farcull.h), the
// units reached through the blocks of kBlkU units and the lower bound equal to
// the one over every unit's extreme point, so M^2 (and, with kArg, the first
// slot attaining it) is exactly what a sweep over every point gives.
// ---------------------------------------------------------------------------
template <int QPL, bool kArg>
__global__ __launch_bounds__(kBlock) void k_far_cull(const Header* __restrict__ h, const float4* __restrict__ pos4,
                                                     const float4* __restrict__ ub, const float4* __restrict__ bb,
                                                     const float* __restrict__ x, int64_t Q,
                                                     float* __restrict__ far2, int32_t* __restrict__ farix) {
  __shared__ FarLds L;
  __shared__ FarBlkLds B;
  const int64_t N = h->N;
  const int64_t U = (N + kUnit - 1) / kUnit;
  const int64_t qb = blockIdx.x;
  float qx[QPL], qy[QPL], qz[QPL], acc[QPL];
  int32_t ix[QPL];
  bool ok[QPL];
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const QueryIn qi = load_query(x, qb * (kBlock * QPL) + k * kBlock + threadIdx.x, Q, h);
    qx[k] = qi.x; qy[k] = qi.y; qz[k] = qi.z;
    ok[k] = qi.valid;
    acc[k] = -3.0e38f;
    ix[k] = -1;
  }
  far_tree<QPL, kArg>(pos4, ub, bb, U, N, qx, qy, qz, ok, acc, ix, L, B);
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int64_t q = qb * (kBlock * QPL) + k * kBlock + threadIdx.x;
    if (q < Q) {
      far2[q] = acc[k] + fmaf(qz[k], qz[k], fmaf(qy[k], qy[k], qx[k] * qx[k]));
      if (kArg) farix[q] = ix[k];
    }
  }
}

// The same sweep for calls with few query blocks, over the blend's point
// splits as well: workgroup b covers split b % S of query block b / S, with
// the bound of pts_farcull.h's far_bound_split_reach (splits of at most
// kFarPlainMax points are swept whole), and writes row `split` of far2 (and
// farix).  A split may miss its own maximum but never the cloud's;
// k_far_fold keeps the largest row and, among equal ones, the first split
// (the lowest slots), so row 0 ends up bitwise what k_far_cull writes.
template <int QPL, bool kArg>
__global__ __launch_bounds__(kBlock) void k_far_split(const Header* __restrict__ h, const float4* __restrict__ pos4,
                                                      const float4* __restrict__ ub, const float4* __restrict__ bb,
                                                      const float* __restrict__ x,
                                                      int64_t Q, int S, int64_t per_split, float* __restrict__ far2,
                                                      int32_t* __restrict__ farix) {
  __shared__ FarLds L;
  const int split = int(blockIdx.x % unsigned(S));
  const int64_t qb = blockIdx.x / unsigned(S);
  const int64_t N = h->N;
  const int64_t U = (N + kUnit - 1) / kUnit;
  float qx[QPL], qy[QPL], qz[QPL], acc[QPL], lb[QPL];
  int32_t ix[QPL];
  bool ok[QPL];
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const QueryIn qi = load_query(x, qb * (kBlock * QPL) + k * kBlock + threadIdx.x, Q, h);
    qx[k] = qi.x; qy[k] = qi.y; qz[k] = qi.z;
    ok[k] = qi.valid;
    acc[k] = -3.0e38f;
    ix[k] = -1;
    lb[k] = -1.f;
  }
  const int64_t beg = int64_t(split) * per_split;
  const int64_t end = min(N, beg + per_split);
  if (per_split <= kFarPlainMax) {  // uniform across the grid
    far_sweep_plain<QPL, kArg>(pos4, beg, end, qx, qy, qz, acc, ix, L);
  } else {
    const int64_t u_lo = beg / kUnit, u_hi = max(u_lo, (end + kUnit - 1) / kUnit);
    if (far_bound_split_reach<QPL>(ub, bb, U, u_lo, u_hi, qx, qy, qz, ok, lb, L)) {
      far_threshold<QPL>(lb, ok);
      far_sweep<QPL, kArg>(pos4, ub, u_lo, u_hi, end, qx, qy, qz, ok, lb, acc, ix, L);
    }
  }
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int64_t q = qb * (kBlock * QPL) + k * kBlock + threadIdx.x;
    if (q < Q) {
      far2[int64_t(split) * Q + q] = acc[k] + fmaf(qz[k], qz[k], fmaf(qy[k], qy[k], qx[k] * qx[k]));
      if (kArg) farix[int64_t(split) * Q + q] = ix[k];
    }
  }
}

// Rows 1..S-1 of far2 (and farix) folded into row 0: the largest value, the
// first row among equal ones (a NaN row 0 stays).
__global__ __launch_bounds__(kBlock) void k_far_fold(float* __restrict__ far2, int32_t* __restrict__ farix, int S,
                                                     int64_t Q) {
  const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= Q) return;
  float m = far2[q];
  int32_t ix = farix ? farix[q] : -1;
  for (int s = 1; s < S; ++s) {
    const float v = far2[int64_t(s) * Q + q];
    if (v > m) {
      m = v;
      if (farix) ix = farix[int64_t(s) * Q + q];
    }
  }
  far2[q] = m;
  if (farix) farix[q] = ix;
}

// The same fold for many rows (plain sweeps only, no slots): one wavefront per
// query (fold_wave, pts_device.h).
__global__ __launch_bounds__(kBlock) void k_far_fold_wave(float* __restrict__ far2, int S, int64_t Q) {
  const int64_t q = int64_t(blockIdx.x) * (kBlock / 64) + threadIdx.x / 64;
  const int lane = int(threadIdx.x & 63);
  const float m = fold_wave(far2, S, Q, q, lane);
  if (lane == 0 && q < Q) far2[q] = m;
}

// ---------------------------------------------------------------------------
// Sweep 2: partial (sum w g, sum w) per split.
// ---------------------------------------------------------------------------
// far_rows: rows of far2 holding per-split maxima (1 once k_far_fold has
// folded them); the blend takes their maximum itself when the fold is skipped.
// kMajor: split_major(S), workgroups in split-major order (split_block).
template <int QPL, bool kMajor>
__global__ __launch_bounds__(kBlock) void k_blend(const Header* __restrict__ h, const float4* __restrict__ rec,
                                                  const float* __restrict__ x, int64_t Q, int S, int64_t per_split,
                                                  const float* __restrict__ far2, int far_rows, float C2, float S2,
                                                  float2* __restrict__ part) {
  __shared__ float4 tile[kTileBlend * kRecF4];
  int split;
  int64_t qb;
  if constexpr (kMajor) {
    split_block(S, split, qb);
  } else {
    split = int(blockIdx.x % unsigned(S));
    qb = blockIdx.x / unsigned(S);
  }
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
    if (qi.valid) far_of(far2, far_rows, Q, q, C2, M, nl[k]);
    num[k] = 0.f;
    den[k] = 0.f;
  }
  const float c2 = S2;
  const int64_t beg = int64_t(split) * per_split;
  const int64_t end = min(N, beg + per_split);
  for (int64_t t0 = beg; t0 < end; t0 += kTileBlend) {
    const int cnt = int(min<int64_t>(kTileBlend, end - t0));
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

// Fixed-order combine of the split partials (pts_device.h): one lane per
// query, or one wavefront per query for many splits and few queries
// (combine_by_wave).
__global__ __launch_bounds__(kBlock) void k_combine(const float2* __restrict__ part, int S, int64_t Q,
                                                    float* __restrict__ sdf, float offset) {
  const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= Q) return;
  const float2 v = combine_seq(part, S, Q, q);
  sdf[q] = v.x / v.y - offset;
}

__global__ __launch_bounds__(kBlock) void k_combine_wave(const float2* __restrict__ part, int S, int64_t Q,
                                                         float* __restrict__ sdf, float offset) {
  const int64_t q = int64_t(blockIdx.x) * (kBlock / 64) + threadIdx.x / 64;
  const int lane = int(threadIdx.x & 63);
  const float2 v = combine_wave(part, S, Q, q, lane);
  if (lane == 0 && q < Q) sdf[q] = v.x / v.y - offset;
}

// fold = false: the split rows are left for the blend to take the maximum of
// (worth it for a few rows only: every blend workgroup of a query reads them).
template <int QPL, bool kArg>
void launch_far_q(const Header* h, const float4* pos4, const float4* ub, const float4* bb, const float* x,
                  int64_t Q, int64_t nqb,
                  int S, int64_t per_split, float* far2, int32_t* farix, hipStream_t st, bool fold) {
  if (S > 1) {
    hipLaunchKernelGGL((k_far_split<QPL, kArg>), dim3(unsigned(nqb * S)), dim3(kBlock), 0, st, h, pos4, ub, bb, x, Q,
                       S, per_split, far2, farix);
    if (fold && (farix || !combine_by_wave(S, Q)))
      hipLaunchKernelGGL(k_far_fold, dim3(unsigned((Q + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, far2, farix, S,
                         Q);
    else if (fold)
      hipLaunchKernelGGL(k_far_fold_wave, dim3(unsigned((Q + kBlock / 64 - 1) / (kBlock / 64))), dim3(kBlock), 0, st,
                         far2, S, Q);
  } else {
    hipLaunchKernelGGL((k_far_cull<QPL, kArg>), dim3(unsigned(nqb)), dim3(kBlock), 0, st, h, pos4, ub, bb, x, Q,
                       far2, farix);
  }
}

template <int QPL>
void launch_blend_q(const Header* h, const float4* rec, const float* x, int64_t Q, const Plan& plan,
                    const float* far2, int far_rows, float2* part, float C2, float S2, hipStream_t st) {
  if (split_major(plan.S))
    hipLaunchKernelGGL((k_blend<QPL, true>), dim3(unsigned(plan.nqb * plan.S)), dim3(kBlock), 0, st, h, rec, x, Q,
                       plan.S, plan.per_split, far2, far_rows, C2, S2, part);
  else
    hipLaunchKernelGGL((k_blend<QPL, false>), dim3(unsigned(plan.nqb * plan.S)), dim3(kBlock), 0, st, h, rec, x, Q,
                       plan.S, plan.per_split, far2, far_rows, C2, S2, part);
}

// The farthest-point sweep's launch shape for an evaluation plan: queries per
// lane lowered (from at most 4) until there are >= 2048 workgroups, and split
// over the plan's point ranges when there are fewer than 1024 query blocks.
struct FarShape {
  int q;
  int64_t nqb;
  int S;
};
FarShape far_shape(int qpl, int64_t Q, int S, int64_t per_split) {
  FarShape f;
  f.q = qpl >= 4 ? 4 : (qpl == 2 ? 2 : 1);
  while (f.q > 1 && (Q + int64_t(kBlock) * f.q - 1) / (int64_t(kBlock) * f.q) < 2048) f.q /= 2;
  f.nqb = (Q + int64_t(kBlock) * f.q - 1) / (int64_t(kBlock) * f.q);
  f.S = (f.nqb >= 1024 || per_split <= 0) ? 1 : S;
  return f;
}

}  // namespace

size_t eval_ws_bytes(const Plan& plan, int64_t Q) {
  const size_t sq = size_t(plan.S) * size_t(Q);
  return align256(sq * sizeof(float)) + align256(sq * sizeof(float2)) + align256(sq * sizeof(int32_t));
}

size_t grad_ws_bytes(const Plan& plan, int64_t Q) {
  const size_t sq = size_t(plan.S) * size_t(Q);
  return eval_ws_bytes(plan, Q) + align256(size_t(Q) * 6 * sizeof(float)) + align256(sq * 2 * sizeof(float4));
}

WsView ws_view(const Plan& plan, int64_t Q, void* ws) {
  const size_t sq = size_t(plan.S) * size_t(Q);
  char* w = static_cast<char*>(ws);
  WsView v;
  v.far2 = reinterpret_cast<float*>(w);
  w += align256(sq * sizeof(float));
  v.part = reinterpret_cast<float2*>(w);
  w += align256(sq * sizeof(float2));
  v.farix = reinterpret_cast<int32_t*>(w);
  w += align256(sq * sizeof(int32_t));
  v.stats = reinterpret_cast<float*>(w);
  w += align256(size_t(Q) * 6 * sizeof(float));
  v.gpart = reinterpret_cast<float4*>(w);
  return v;
}

int launch_far_cull(const void* rec, int64_t N, const float* x, int64_t Q, int qpl, float* far2, int32_t* farix,
                    hipStream_t st, int S, int64_t per_split) {
  const Layout L(N);
  const char* base = static_cast<const char*>(rec);
  const Header* h = reinterpret_cast<const Header*>(base);
  const float4* pos4 = reinterpret_cast<const float4*>(base + L.pos);
  const float4* ub = reinterpret_cast<const float4*>(base + L.ub);
  const float4* bb = reinterpret_cast<const float4*>(base + L.bb);
  // one workgroup per query block: keep at least 2048 of them (8 per CU) when
  // there are queries enough, by lowering the queries per lane; with fewer
  // than 1024 query blocks, sweep the point splits as separate workgroups (the
  // caller's far2 / farix then hold S rows)
  const FarShape f = far_shape(qpl, Q, S, per_split);
  if (farix) {
    switch (f.q) {
      case 1: launch_far_q<1, true>(h, pos4, ub, bb, x, Q, f.nqb, f.S, per_split, far2, farix, st, true); break;
      case 2: launch_far_q<2, true>(h, pos4, ub, bb, x, Q, f.nqb, f.S, per_split, far2, farix, st, true); break;
      default: launch_far_q<4, true>(h, pos4, ub, bb, x, Q, f.nqb, f.S, per_split, far2, farix, st, true); break;
    }
  } else {
    switch (f.q) {
      case 1: launch_far_q<1, false>(h, pos4, ub, bb, x, Q, f.nqb, f.S, per_split, far2, nullptr, st, true); break;
      case 2: launch_far_q<2, false>(h, pos4, ub, bb, x, Q, f.nqb, f.S, per_split, far2, nullptr, st, true); break;
      default: launch_far_q<4, false>(h, pos4, ub, bb, x, Q, f.nqb, f.S, per_split, far2, nullptr, st, true); break;
    }
  }
  return check_hip(hipGetLastError(), "farthest-point kernel");
}

int launch_far(const void* rec, int64_t N, const float* x, int64_t Q, const Plan& plan, const WsView& ws,
               hipStream_t st) {
  return launch_far_cull(rec, N, x, Q, plan.qpl, ws.far2, nullptr, st, plan.S, plan.per_split);
}

int launch_blend(const void* rec, int64_t N, const float* x, int64_t Q, float C, const Plan& plan,
                 const WsView& ws, hipStream_t st) {
  const Layout L(N);
  const char* base = static_cast<const char*>(rec);
  const Header* h = reinterpret_cast<const Header*>(base);
  const float4* recs = reinterpret_cast<const float4*>(base + L.rec);
  const float C2 = C * kLog2e, S2 = shift2_of(C);
  switch (plan.qpl) {
    case 1: launch_blend_q<1>(h, recs, x, Q, plan, ws.far2, 1, ws.part, C2, S2, st); break;
    case 2: launch_blend_q<2>(h, recs, x, Q, plan, ws.far2, 1, ws.part, C2, S2, st); break;
    case 8: launch_blend_q<8>(h, recs, x, Q, plan, ws.far2, 1, ws.part, C2, S2, st); break;
    default: launch_blend_q<4>(h, recs, x, Q, plan, ws.far2, 1, ws.part, C2, S2, st); break;
  }
  return check_hip(hipGetLastError(), "blend kernel");
}

int launch_eval_plain(const void* rec, int64_t N, const float* x, int64_t Q, float C, const Plan& plan,
                      const WsView& ws, float* sdf, hipStream_t st, float offset) {
  const Layout L(N);
  const char* base = static_cast<const char*>(rec);
  const Header* h = reinterpret_cast<const Header*>(base);
  const float4* pos4 = reinterpret_cast<const float4*>(base + L.pos);
  const float4* ub = reinterpret_cast<const float4*>(base + L.ub);
  const float4* bb = reinterpret_cast<const float4*>(base + L.bb);
  const float4* recs = reinterpret_cast<const float4*>(base + L.rec);
  const FarShape f = far_shape(plan.qpl, Q, plan.S, plan.per_split);
  const bool fold = f.S > kLaneSplitsMax;
  const int rows = fold ? 1 : f.S;
  switch (f.q) {
    case 1: launch_far_q<1, false>(h, pos4, ub, bb, x, Q, f.nqb, f.S, plan.per_split, ws.far2, nullptr, st, fold); break;
    case 2: launch_far_q<2, false>(h, pos4, ub, bb, x, Q, f.nqb, f.S, plan.per_split, ws.far2, nullptr, st, fold); break;
    default: launch_far_q<4, false>(h, pos4, ub, bb, x, Q, f.nqb, f.S, plan.per_split, ws.far2, nullptr, st, fold); break;
  }
  if (int rc = check_hip(hipGetLastError(), "farthest-point kernel")) return rc;
  const float C2 = C * kLog2e, S2 = shift2_of(C);
  switch (plan.qpl) {
    case 1: launch_blend_q<1>(h, recs, x, Q, plan, ws.far2, rows, ws.part, C2, S2, st); break;
    case 2: launch_blend_q<2>(h, recs, x, Q, plan, ws.far2, rows, ws.part, C2, S2, st); break;
    case 8: launch_blend_q<8>(h, recs, x, Q, plan, ws.far2, rows, ws.part, C2, S2, st); break;
    default: launch_blend_q<4>(h, recs, x, Q, plan, ws.far2, rows, ws.part, C2, S2, st); break;
  }
  if (int rc = check_hip(hipGetLastError(), "blend kernel")) return rc;
  return launch_combine(Q, plan, ws, sdf, st, offset);
}

int launch_combine(int64_t Q, const Plan& plan, const WsView& ws, float* sdf, hipStream_t st, float offset) {
  if (!combine_by_wave(plan.S, Q))
    hipLaunchKernelGGL(k_combine, dim3(unsigned((Q + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, ws.part, plan.S,
                       Q, sdf, offset);
  else
    hipLaunchKernelGGL(k_combine_wave, dim3(unsigned((Q + kBlock / 64 - 1) / (kBlock / 64))), dim3(kBlock), 0, st,
                       ws.part, plan.S, Q, sdf, offset);
  return check_hip(hipGetLastError(), "combine kernel");
}

}  // namespace pts
