// pts_trace.hip -- sphere tracing of the point-cloud SDF (Sec. 5.3, "Direct
// visualization of point cloud surfaces").
//
// Per ray (origin o, unit direction d): t = 0; up to `steps` times evaluate
// phi(o + t d); stop with a hit when |phi| < eps; otherwise t += phi and stop
// with a miss when t > tmax.  At hits the unit normal grad phi / |grad phi| is
// returned.  Each step evaluates all still-active rays with the evaluation
// kernels (farthest-point and blend sweeps, split combine), then a small
// kernel advances the rays and a deterministic stream compaction keeps the
// active ones.  The point splits (of the march, and of the normals' gradient
// sweep) are functions of N only, so every ray's phi and normal are computed in
// the same order whatever the other rays do.
#include "pts_device.h"

#include <algorithm>

namespace pts {
namespace {

// Positions of the active rays.
__global__ __launch_bounds__(kBlock) void k_positions(const int32_t* __restrict__ act, int64_t na,
                                                      const float* __restrict__ org, const float* __restrict__ dir,
                                                      const float* __restrict__ t, float* __restrict__ xq) {
  const int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (j >= na) return;
  const int64_t r = act[j];
  const float tr = t[r];
  for (int c = 0; c < 3; ++c) xq[3 * j + c] = fmaf(tr, dir[3 * r + c], org[3 * r + c]);
}

// Advance the active rays by one step; keep[j] = 1 if ray act[j] continues.
__global__ __launch_bounds__(kBlock) void k_advance(const int32_t* __restrict__ act, int64_t na,
                                                    const float* __restrict__ phi, float eps, float tmax, int step,
                                                    float* __restrict__ t, int32_t* __restrict__ hit,
                                                    int32_t* __restrict__ nsteps, int32_t* __restrict__ keep) {
  const int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (j >= na) return;
  const int64_t r = act[j];
  const float f = phi[j];
  int k = 0;
  if (fabsf(f) < eps) {
    hit[r] = 1;
    nsteps[r] = step;
  } else {
    const float tn = t[r] + f;
    t[r] = tn;
    if (tn > tmax || !(tn == tn)) {
      nsteps[r] = step;
    } else {
      k = 1;
    }
  }
  keep[j] = k;
}

__global__ __launch_bounds__(kBlock) void k_init_rays(int64_t R, int steps, float* __restrict__ t,
                                                      int32_t* __restrict__ hit, int32_t* __restrict__ nsteps,
                                                      int32_t* __restrict__ act, float* __restrict__ nrm) {
  const int64_t r = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (r >= R) return;
  t[r] = 0.f;
  hit[r] = 0;
  nsteps[r] = steps;
  act[r] = int32_t(r);
  if (nrm) { nrm[3 * r] = 0.f; nrm[3 * r + 1] = 0.f; nrm[3 * r + 2] = 0.f; }
}

// Compaction, pass 1: per-block counts of keep flags.
__global__ __launch_bounds__(kBlock) void k_count(const int32_t* __restrict__ keep, int64_t n,
                                                  int32_t* __restrict__ blk) {
  const int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int v = j < n ? keep[j] : 0;
  const int c = __syncthreads_count(v);
  if (threadIdx.x == 0) blk[blockIdx.x] = c;
}

// Compaction, pass 2: exclusive scan of the block counts by one wavefront
// (a 64-lane shuffle scan per 64 counts, carried in a register), total
// written to *count.  One wave and no LDS, so it finds a slot at once beside
// large concurrent launches.
__global__ __launch_bounds__(64) void k_scan_counts(const int32_t* __restrict__ blk, int64_t nb,
                                                    int32_t* __restrict__ off, int32_t* __restrict__ count) {
  const int lane = int(threadIdx.x);
  int32_t carry = 0;
  for (int64_t base = 0; base < nb; base += 64) {
    const int64_t i = base + lane;
    const int32_t v = i < nb ? blk[i] : 0;
    int32_t incl = v;
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t t = __shfl_up(incl, o);
      if (lane >= o) incl += t;
    }
    if (i < nb) off[i] = carry + incl - v;
    carry += __shfl(incl, 63);
  }
  if (lane == 0) *count = carry;
}

// Compaction, pass 3: stable scatter of the kept entries.
__global__ __launch_bounds__(kBlock) void k_scatter(const int32_t* __restrict__ keep, const int32_t* __restrict__ src,
                                                    int64_t n, const int32_t* __restrict__ off,
                                                    int32_t* __restrict__ dst) {
  __shared__ int32_t wsum[kBlock / 64];
  const int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int v = j < n ? keep[j] : 0;
  const uint64_t ball = __ballot(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int below = __popcll(ball & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
  if (lane == 0) wsum[wave] = __popcll(ball);
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wave; ++w) before += wsum[w];
  if (v) dst[off[blockIdx.x] + before + below] = src[j];
}

// Normals from gradients of the hit rays.
__global__ __launch_bounds__(kBlock) void k_normals(const int32_t* __restrict__ act, int64_t na,
                                                    const float* __restrict__ g, float* __restrict__ nrm) {
  const int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (j >= na) return;
  const int64_t r = act[j];
  const float gx = g[3 * j], gy = g[3 * j + 1], gz = g[3 * j + 2];
  const float l = sqrtf(gx * gx + gy * gy + gz * gz);
  const float il = l > 0.f ? 1.f / l : 0.f;
  nrm[3 * r] = gx * il;
  nrm[3 * r + 1] = gy * il;
  nrm[3 * r + 2] = gz * il;
}

__global__ __launch_bounds__(kBlock) void k_iota(int32_t* __restrict__ out, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) out[i] = int32_t(i);
}

inline unsigned nblk(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

struct TraceWs {
  int32_t *act0, *act1, *keep, *blk, *off, *count, *nsteps;
  float *xq, *phi, *g;
  void* eval;
  size_t eval_bytes;
};

size_t trace_fixed_bytes(int64_t R) {
  const int64_t nb = (R + kBlock - 1) / kBlock;
  return 4 * align256(size_t(R) * 4) + 2 * align256(size_t(nb) * 4) + 256 + align256(size_t(R) * 12) +
         align256(size_t(R) * 4) + align256(size_t(R) * 12) + align256(size_t(R) * 4);
}

TraceWs trace_ws(void* ws, int64_t R, size_t total) {
  const int64_t nb = (R + kBlock - 1) / kBlock;
  char* w = static_cast<char*>(ws);
  TraceWs v;
  auto take = [&](size_t b) { char* p = w; w += align256(b); return p; };
  v.act0 = reinterpret_cast<int32_t*>(take(size_t(R) * 4));
  v.act1 = reinterpret_cast<int32_t*>(take(size_t(R) * 4));
  v.keep = reinterpret_cast<int32_t*>(take(size_t(R) * 4));
  v.nsteps = reinterpret_cast<int32_t*>(take(size_t(R) * 4));
  v.blk = reinterpret_cast<int32_t*>(take(size_t(nb) * 4));
  v.off = reinterpret_cast<int32_t*>(take(size_t(nb) * 4));
  v.count = reinterpret_cast<int32_t*>(take(256));
  v.xq = reinterpret_cast<float*>(take(size_t(R) * 12));
  v.phi = reinterpret_cast<float*>(take(size_t(R) * 4));
  v.g = reinterpret_cast<float*>(take(size_t(R) * 12));
  take(size_t(R) * 4);
  v.eval = w;
  v.eval_bytes = total - size_t(w - static_cast<char*>(ws));
  return v;
}

// Compact act_in by keep into act_out; returns the new count (reads it back).
int compact(const int32_t* keep, const int32_t* act_in, int64_t n, int32_t* act_out, const TraceWs& v, int64_t* out,
            hipStream_t st) {
  const unsigned nb = nblk(n);
  hipLaunchKernelGGL(k_count, dim3(nb), dim3(kBlock), 0, st, keep, n, v.blk);
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(64), 0, st, v.blk, int64_t(nb), v.off, v.count);
  hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kBlock), 0, st, keep, act_in, n, v.off, act_out);
  int32_t c = 0;
  if (int rc = check_hip(hipMemcpyAsync(&c, v.count, sizeof(c), hipMemcpyDeviceToHost, st), "read count")) return rc;
  if (int rc = check_hip(hipStreamSynchronize(st), "trace step")) return rc;
  *out = c;
  return PTS_OK;
}

}  // namespace

// Point split of the march: the largest power of two <= 64 that leaves every
// split at least two farthest-point tiles.  A function of N only, so a ray's
// phi does not depend on which other rays are still active.
int march_splits(int64_t N, int cap) {
  const int64_t tiles = (N + kTile1 - 1) / kTile1;
  int S = 1;
  while (S < cap && tiles >= int64_t(4) * S) S *= 2;
  return S;
}

Plan march_plan(int64_t N, int64_t Q, const pts_params& P, int cap) {
  pts_params F = P;
  if (F.splits == 0) F.splits = march_splits(N, cap);
  return make_plan(N, Q, &F);
}

// The normals' gradient sweep keeps at most 8 of the march's splits (its
// workspace grows by 32 bytes per ray and split); also a function of N only.
Plan normal_plan(int64_t N, int64_t Q, const pts_params& P) {
  pts_params F = P;
  F.splits = std::min(F.splits > 0 ? F.splits : march_splits(N, kMarchSplitCap), 8);
  return make_plan(N, Q, &F);
}

size_t trace_eval_ws_bytes(int64_t N, int64_t R, const pts_params& P, int cap) {
  return std::max(eval_ws_bytes(march_plan(N, R, P, cap), R), grad_ws_bytes(normal_plan(N, R, P), R));
}

size_t trace_ws_bytes(int64_t N, int64_t R, const pts_params& P) {
  return trace_fixed_bytes(R) + trace_eval_ws_bytes(N, R, P, kMarchSplitCap);
}

size_t trace_bounded_ws_bytes(int64_t N, int64_t R, const pts_params& P) {
  return trace_fixed_bytes(R) + std::max(bounded_ws_max(N, R), grad_ws_bytes(normal_plan(N, R, P), R));
}

int launch_trace(const void* rec, int64_t N, const float* org, const float* dir, int64_t R, int steps, float eps,
                 float tmax, float* t, float* nrm, int32_t* hit, int32_t* nsteps_out, const pts_params& P, void* ws,
                 size_t ws_bytes, hipStream_t st, float eval_eps) {
  const TraceWs v = trace_ws(ws, R, ws_bytes);
  int32_t* nsteps = nsteps_out ? nsteps_out : v.nsteps;
  hipLaunchKernelGGL(k_init_rays, dim3(nblk(R)), dim3(kBlock), 0, st, R, steps, t, hit, nsteps, v.act0, nrm);
  int32_t* act = v.act0;
  int32_t* nxt = v.act1;
  int64_t na = R;
  for (int k = 0; k < steps && na > 0; ++k) {
    hipLaunchKernelGGL(k_positions, dim3(nblk(na)), dim3(kBlock), 0, st, act, na, org, dir, t, v.xq);
    if (eval_eps >= 0.f) {
      const Plan plan = bounded_plan(N, na);
      if (int rc = launch_bounded(rec, N, v.xq, na, eval_eps, P.C, plan, v.eval, v.phi, nullptr, nullptr, st,
                                  P.offset))
        return rc;
    } else {
      const Plan plan = march_plan(N, na, P, kMarchSplitCap);
      const WsView wv = ws_view(plan, na, v.eval);
      if (int rc = launch_eval_plain(rec, N, v.xq, na, P.C, plan, wv, v.phi, st, P.offset)) return rc;
    }
    hipLaunchKernelGGL(k_advance, dim3(nblk(na)), dim3(kBlock), 0, st, act, na, v.phi, eps, tmax, k, t, hit, nsteps,
                       v.keep);
    int64_t nn = 0;
    if (int rc = compact(v.keep, act, na, nxt, v, &nn, st)) return rc;
    int32_t* tmp = act;
    act = nxt;
    nxt = tmp;
    na = nn;
  }
  if (!nrm) return check_hip(hipGetLastError(), "trace kernels");
  // normals at the hits: compact the hit rays, evaluate grad phi there
  hipLaunchKernelGGL(k_iota, dim3(nblk(R)), dim3(kBlock), 0, st, nxt, R);
  int64_t nh = 0;
  if (int rc = compact(hit, nxt, R, act, v, &nh, st)) return rc;
  if (nh == 0) return PTS_OK;
  const Plan plan = normal_plan(N, nh, P);
  const WsView wv = ws_view(plan, nh, v.eval);
  hipLaunchKernelGGL(k_positions, dim3(nblk(nh)), dim3(kBlock), 0, st, act, nh, org, dir, t, v.xq);
  if (int rc = launch_far_arg(rec, N, v.xq, nh, plan, wv, st)) return rc;
  if (int rc = launch_blend(rec, N, v.xq, nh, P.C, plan, wv, st)) return rc;
  if (int rc = launch_combine_stats(rec, N, v.xq, nh, plan, wv, v.phi, wv.stats, st, P.offset)) return rc;
  if (int rc = launch_grad(rec, N, v.xq, nh, wv.stats, nullptr, v.g, P.C, plan, wv, st)) return rc;
  hipLaunchKernelGGL(k_normals, dim3(nblk(nh)), dim3(kBlock), 0, st, act, nh, v.g, nrm);
  return check_hip(hipGetLastError(), "trace normals");
}

// ---------------------------------------------------------------------------
// The same march driven one step at a time by the server, with nothing read
// back synchronously: the active count is left on the device.
// ---------------------------------------------------------------------------
int trace_init(int64_t R, int steps, float* t, int32_t* hit, int32_t* nsteps, int32_t* act, float* nrm,
               hipStream_t st) {
  hipLaunchKernelGGL(k_init_rays, dim3(nblk(R)), dim3(kBlock), 0, st, R, steps, t, hit, nsteps, act, nrm);
  return check_hip(hipGetLastError(), "trace init");
}

int trace_step_pre(const int32_t* act, int64_t na, const float* org, const float* dir, const float* t, float* xq,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_positions, dim3(nblk(na)), dim3(kBlock), 0, st, act, na, org, dir, t, xq);
  return check_hip(hipGetLastError(), "trace positions");
}

int trace_step_post(const int32_t* act, int64_t na, const float* phi, float eps, float tmax, int step, float* t,
                    int32_t* hit, int32_t* nsteps, int32_t* keep, int32_t* act_out, int32_t* blk, int32_t* off,
                    int32_t* count, hipStream_t st) {
  const unsigned nb = nblk(na);
  hipLaunchKernelGGL(k_advance, dim3(nb), dim3(kBlock), 0, st, act, na, phi, eps, tmax, step, t, hit, nsteps, keep);
  hipLaunchKernelGGL(k_count, dim3(nb), dim3(kBlock), 0, st, keep, na, blk);
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(64), 0, st, blk, int64_t(nb), off, count);
  hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kBlock), 0, st, keep, act, na, off, act_out);
  return check_hip(hipGetLastError(), "trace advance");
}

// Hit rays of a finished march, compacted on the device in ray order into
// act_out [0, *count); `iota` is scratch of R int32.  Nothing is read back.
int trace_hits(const int32_t* hit, int64_t R, int32_t* iota, int32_t* act_out, int32_t* blk, int32_t* off,
               int32_t* count, hipStream_t st) {
  const unsigned nb = nblk(R);
  hipLaunchKernelGGL(k_iota, dim3(nb), dim3(kBlock), 0, st, iota, R);
  hipLaunchKernelGGL(k_count, dim3(nb), dim3(kBlock), 0, st, hit, R, blk);
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(64), 0, st, blk, int64_t(nb), off, count);
  hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kBlock), 0, st, hit, iota, R, off, act_out);
  return check_hip(hipGetLastError(), "trace hit compaction");
}

// Normals at the nh hit rays act [0, nh) (from trace_hits), written to nrm at
// their ray index; the other rays' entries are left as they are (0 from
// trace_init).  plan = normal_plan(N, nh, ...): its splits depend on N only,
// so the normals are bitwise those pts_trace computes.
int trace_normals_hits(const void* rec, int64_t N, const float* org, const float* dir, const float* t,
                       const int32_t* act, int64_t nh, float* xq, float* phi, float* g, float* nrm, const Plan& plan,
                       float C, void* ws, hipStream_t st) {
  if (nh == 0) return PTS_OK;
  const WsView wv = ws_view(plan, nh, ws);
  hipLaunchKernelGGL(k_positions, dim3(nblk(nh)), dim3(kBlock), 0, st, act, nh, org, dir, t, xq);
  if (int rc = launch_far_arg(rec, N, xq, nh, plan, wv, st)) return rc;
  if (int rc = launch_blend(rec, N, xq, nh, C, plan, wv, st)) return rc;
  if (int rc = launch_combine_stats(rec, N, xq, nh, plan, wv, phi, wv.stats, st)) return rc;
  if (int rc = launch_grad(rec, N, xq, nh, wv.stats, nullptr, g, C, plan, wv, st)) return rc;
  hipLaunchKernelGGL(k_normals, dim3(nblk(nh)), dim3(kBlock), 0, st, act, nh, g, nrm);
  return check_hip(hipGetLastError(), "trace normals");
}

}  // namespace pts
