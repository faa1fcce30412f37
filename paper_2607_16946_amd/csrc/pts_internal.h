// pts_internal.h -- record layout and launch helpers shared by the HIP sources
// of libpts (gfx950).  Not part of the public ABI (include/pts.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "pts.h"

namespace pts {

constexpr uint32_t kMagic = 0x31535450u;  // "PTS1"
constexpr int kRecordVersion = 4;
constexpr int kBlock = 256;               // threads per workgroup (4 waves of 64)
constexpr int kTile2 = 128;               // points per LDS tile of the derivative sweeps (80 B each)
// Points per LDS tile of the blend (k_blend, and k_blend_multi, which must sum
// in the same order): 20 KB, half the barriers of 128 (0.6% on the blend; the
// query-gradient sweep lost 3% with it, so it keeps kTile2).
constexpr int kTileBlend = 256;
constexpr int kTile1 = 512;               // points per LDS tile, farthest-point pass (16 B each)
constexpr int kRecF4 = 5;                 // float4 per point record
constexpr float kLog2e = 1.4426950408889634f;
// Screening constant C (Eq. RelationshipBetweenLambdaAndRadius) and the
// additive shift of the weights.  The paper shifts every exponent by
// lambda_x sigma_x = C (Eq. BasicFormulaShifted), so the weights lie in
// [e^-C, e^C]; phi does not depend on the shift, only the FP32 range of the
// sums does.  The kernels shift by s = min(C, 64): the largest weight is then
// at most e^64, so sums over N points of w |g| stay below FLT_MAX while
// N max|g| < 5e10, and the smallest, e^(s - 2C), stays a normal FP32 number
// (>= 2^-126) for every C <= 75.  s = C for the paper's C = 64.
constexpr float kShiftMaxC = 64.0f;
constexpr float kCMax = 75.0f;
// Smallest relative curvature floor: torus radii reach D / kfloor_rel, and the
// anchored form squares them (t^2 with t ~ L), so L must stay well below
// sqrt(FLT_MAX) ~ 1.8e19 for clouds up to D ~ 1e6.
constexpr float kKfloorRelMin = 1e-12f;
__host__ __device__ inline float shift2_of(float C) { return (C < kShiftMaxC ? C : kShiftMaxC) * kLog2e; }
constexpr double kDirectMaxL = 4.0;       // direct torus form when L <= 4 D
constexpr int kUnit = 64;                 // points per culling unit of the farthest-point pass
constexpr int kBlkU = 64;                 // units per block of the two-level sphere hierarchy
constexpr int kSortBits = 4;              // radix of the build's spatial sort (16 buckets per pass)
constexpr int kSortPasses = 7;            // 25-bit keys: form bit + 3 x 8 Morton bits

// Cloud header (first 256 bytes of the record buffer).
struct alignas(256) Header {
  uint32_t magic;
  int32_t version;
  int64_t N;
  int64_t n_direct;     // points [0, n_direct) use the direct torus form
  int64_t n_anchored;   // points [n_direct, N) use the anchored form (L > 4 D)
  float origin[3];      // record coordinates are relative to this point (bbox center)
  float diag;           // bbox diagonal D
  float kfloor;         // curvature floor
  float lmax_direct;    // 4 D
  float lo[3];
  float hi[3];
  uint32_t lo_bits[3];  // order-preserving encodings used by the bbox reduction
  uint32_t hi_bits[3];
  int32_t status;       // bit 0: zero normal, bit 1: non-finite input
  int32_t pad0;
  double kfloor64;      // curvature floor used by the fit (FP64)
  // radius-limited evaluation (set by pts_radius_prepare)
  double rl_D;          // mean distance to the 64 nearest other points
  float rl_lambda;      // 1e3 / rl_D
  float rl_reval;       // 2 C / rl_lambda
  int32_t rl_ready;     // 1 once the three values above are set
  float rl_shift;       // min(C, 64) / rl_lambda: the exponent shift (a distance) of the radius branch
  uint32_t a00max_bits; // bits of max_i |a00_i| (non-negative, so integer order is float order)
  int32_t pad2;
};
static_assert(sizeof(Header) == 256, "header is 256 bytes");

constexpr int32_t kStatusZeroNormal = 1;
constexpr int32_t kStatusNonFinite = 2;

__host__ __device__ inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Byte offsets of the sections of a record buffer for N points.
//   pos4  [N]     float4 (-2 p, |p|^2), farthest-point pass
//   rec   [N][5]  float4 torus record, blend passes (layout in pts_build.hip)
//   perm  [N]     int32 original index of each slot
//   ub    [U][2]  float4 bounds of each kUnit-point unit of slots, U = ceil(N / kUnit):
//                 (center c, radius r) and (the unit's point farthest from c, 0)
//   bb    [B]     float4 (center, radius) of each block of kBlkU units, B = ceil(U / kBlkU)
//   ob    [U][4]  float4 oriented box of each unit: (center c, 0), then (a_k, e_k) for
//                 k = 0..2, axes a_k (a_0 the unit's mean normal) and half-extents e_k with
//                 |<p - c, a_k>| <= e_k for every point p of the unit
//   base  [N][2]  float4 (p, A) and (n / |n|, -<p, n / |n|>): the baseline evaluators'
//                 point record (A = area weight, 1 unless set by pts_set_areas)
//   flag  [N]     int32 build scratch (direct-form flag)
//   blk   [2*nb]  int32 build scratch (per-block counts and offsets)
//   key, idx [2][N] uint32 / int32 build scratch (sort keys and indices, ping-pong)
//   rhist [16*nb] int32 build scratch (radix histograms)
struct Layout {
  size_t pos, rec, perm, ub, bb, ob, base, flag, blk, key, idx, rhist, total;
  int64_t nblk, nunit, nbk;
  __host__ __device__ explicit Layout(int64_t N) {
    nblk = (N + kBlock - 1) / kBlock;
    nunit = (N + kUnit - 1) / kUnit;
    nbk = (nunit + kBlkU - 1) / kBlkU;
    pos = 256;
    rec = pos + align256(size_t(N) * 16);
    perm = rec + align256(size_t(N) * 16 * kRecF4);
    ub = perm + align256(size_t(N) * 4);
    bb = ub + align256(size_t(nunit) * 32);
    ob = bb + align256(size_t(nbk) * 16);
    base = ob + align256(size_t(nunit) * 64);
    flag = base + align256(size_t(N) * 32);
    blk = flag + align256(size_t(N) * 4);
    key = blk + align256(size_t(nblk) * 8);
    idx = key + 2 * align256(size_t(N) * 4);
    rhist = idx + 2 * align256(size_t(N) * 4);
    total = rhist + align256(size_t(nblk) * 16 * 4);
  }
};

// Split of the point range of one evaluation (a pure function of N, Q and the
// parameters, so that a request gives the same result alone or batched).
struct Plan {
  int qpl;            // queries per lane
  int S;              // point splits
  int64_t per_split;  // points per split (multiple of kUnit)
  int64_t nqb;        // query blocks of kBlock * qpl queries
};
// max_auto_splits bounds the automatic split count (prm->splits == 0): the
// plain evaluation (phi only: pts_eval without gradient or statistics, its
// staged calls, the server's query requests) allows kPlainSplitMax, every
// other path kAutoSplitMax (their combine kernels sum a query's splits in
// one lane).
constexpr int kAutoSplitMax = 64;
constexpr int kPlainSplitMax = 1024;
// The plain evaluation's per-query reductions over splits -- the fold of the
// farthest-point sweep's per-split maxima and the combine of the blend's
// partials -- run in one lane up to kLaneSplitsMax splits (the blend then
// reads the unfolded maxima itself), in one wavefront beyond.
constexpr int kLaneSplitsMax = 16;
// The combine, though, stays one lane per query from kLaneCombineMinQ queries
// on, whatever the split count: a wavefront per query reads a column of the
// partials (one 8-byte value per 128-byte line), which only pays when there
// are too few queries to occupy the lanes.
constexpr int64_t kLaneCombineMinQ = 32768;
__host__ __device__ inline bool combine_by_wave(int S, int64_t Q) { return S > kLaneSplitsMax && Q < kLaneCombineMinQ; }
Plan make_plan(int64_t N, int64_t Q, const pts_params* prm, int max_auto_splits = kAutoSplitMax);
// The same split with a different number of queries per lane.
inline Plan with_qpl(Plan p, int qpl, int64_t Q) {
  p.qpl = qpl;
  p.nqb = (Q + int64_t(kBlock) * qpl - 1) / (int64_t(kBlock) * qpl);
  return p;
}

// Workspace of one evaluation: per-split maxima and blend partials, the slot
// of each split's farthest point, and (gradients only) the statistics of the
// queries and the per-split gradient partials.
struct WsView {
  float* far2;     // [S][Q] (the farthest-point sweep fills row 0; packed launches use all rows)
  float2* part;    // [S][Q]
  int32_t* farix;  // [S][Q] (row 0 used)
  float* stats;    // [Q][6]    (gradient workspace only)
  float4* gpart;   // [S][Q][2] (gradient workspace only)
};
size_t eval_ws_bytes(const Plan& plan, int64_t Q);
size_t grad_ws_bytes(const Plan& plan, int64_t Q);
WsView ws_view(const Plan& plan, int64_t Q, void* ws);

// Error reporting (thread-local message, returned status).
int fail(int code, const std::string& msg);
int check_hip(hipError_t e, const char* what);

// Kernel launchers (defined in the .hip files).
int launch_build(const float* p, const float* n, const float* a, int64_t N, float kfloor_rel,
                 void* rec, hipStream_t st);
int launch_decode(const void* rec, int64_t N, float* out, hipStream_t st);
// Stable LSD radix sort of (key, index) pairs, kSortBits per pass, `passes`
// passes from the lowest digit; key[0]/idx[0] hold the input and the result
// ends in key[*out]/idx[*out].  rhist: 16 * ceil(n / kBlock) int32 of scratch.
int launch_radix_sort(uint32_t* key[2], int32_t* idx[2], int64_t n, int passes, int32_t* rhist, hipStream_t st,
                      int* out);

// Plain evaluation (phi only) with the workspace in a static device array
// (pts_noalloc.hip): no allocation of any kind; rejects plans whose workspace
// exceeds noalloc_scratch_bytes().
size_t noalloc_scratch_bytes();
int eval_noalloc(const void* rec, int64_t N, const float* x, int64_t Q, float* sdf, const pts_params& P,
                 const Plan& plan, hipStream_t st);

// Queries in Morton order of the cloud's bbox (3 x 8 bits; pts_bounded.hip):
// keys into key[0], a stable radix sort, and *order = the sorted query indices
// (one of idx[0], idx[1]).  key, idx: [2][Q]; rhist: 16 * ceil(Q / kBlock) int32.
int launch_query_order(const void* rec, const float* x, int64_t Q, uint32_t* key[2], int32_t* idx[2],
                       int32_t* rhist, hipStream_t st, const int32_t** order);

// Error-bounded evaluation (pts_bounded.hip): the blend with point units
// skipped while a proven bound on the change of phi stays within eps.
Plan bounded_plan(int64_t N, int64_t Q);
size_t bounded_ws_bytes(const Plan& plan, int64_t Q);
size_t bounded_ws_max(int64_t N, int64_t R);  // over every query count 1..R
int launch_bounded(const void* rec, int64_t N, const float* x, int64_t Q, float eps, float C, const Plan& plan,
                   void* ws, float* sdf, float* bound, int32_t* kept, hipStream_t st, float offset = 0.f);

// Baseline evaluators (pts_baseline.hip): smoothed signed planar distance and
// signed Hopf-Cole distance over the record's base section.
int launch_set_areas(void* rec, int64_t N, const float* area, hipStream_t st);
int launch_baseline(const void* rec, int64_t N, const float* x, int64_t Q, int kind, float C, const Plan& plan,
                    const WsView& ws, float* sdf, hipStream_t st, float offset = 0.f);
// Elementwise compositions of signed distances (pts_compose.hip).
int launch_compose(const float* a, const float* b, int64_t n, int op, float c, float* out, hipStream_t st);
// Radius-limited evaluation (pts_radius.hip).
int launch_blocks(void* rec, int64_t N, hipStream_t st);
int launch_radius_prepare(void* rec, int64_t N, float C, hipStream_t st);
size_t eval_radius_ws_bytes(int64_t Q);
int launch_eval_radius(const void* rec, int64_t N, const float* x, int64_t Q, float* sdf, int32_t* count,
                       void* ws, hipStream_t st);
// Farthest-point sweep (culled by units): M^2 per query into far2[Q] and, if
// farix is non-null, the first slot attaining it into farix[Q].  With S > 1
// and per_split > 0 (an evaluation plan's point split) a call with few query
// blocks also sweeps the splits as separate workgroups; far2 and farix must
// then hold S rows of Q, and row 0 gets the result (bitwise the same).
int launch_far_cull(const void* rec, int64_t N, const float* x, int64_t Q, int qpl, float* far2, int32_t* farix,
                    hipStream_t st, int S = 1, int64_t per_split = 0);
int launch_far(const void* rec, int64_t N, const float* x, int64_t Q, const Plan& plan, const WsView& ws,
               hipStream_t st);
int launch_blend(const void* rec, int64_t N, const float* x, int64_t Q, float C, const Plan& plan,
                 const WsView& ws, hipStream_t st);
// The whole plain evaluation (phi only): the farthest-point sweep (with few
// split rows left unfolded for the blend sweep to take their maximum), the
// blend sweep and the combine.  Bitwise equal to launch_far + launch_blend +
// launch_combine, one launch fewer when the farthest-point sweep runs split
// over at most 16 splits.
int launch_eval_plain(const void* rec, int64_t N, const float* x, int64_t Q, float C, const Plan& plan,
                      const WsView& ws, float* sdf, hipStream_t st, float offset = 0.f);
// sdf = num / den - offset (the offset surface phi = offset; 0 leaves phi bitwise unchanged)
int launch_combine(int64_t Q, const Plan& plan, const WsView& ws, float* sdf, hipStream_t st, float offset = 0.f);
int launch_far_arg(const void* rec, int64_t N, const float* x, int64_t Q, const Plan& plan, const WsView& ws,
                   hipStream_t st);
int launch_combine_stats(const void* rec, int64_t N, const float* x, int64_t Q, const Plan& plan,
                         const WsView& ws, float* sdf, float* stats, hipStream_t st, float offset = 0.f);
int launch_grad(const void* rec, int64_t N, const float* x, int64_t Q, const float* stats, const float* gout,
                float* gx, float C, const Plan& plan, const WsView& ws, hipStream_t st);

// Laplacian, gradient and eikonal residual from one query-major sweep (pts_lap.hip).
size_t lap_ws_bytes(const Plan& plan, int64_t Q);
int launch_lap(const void* rec, int64_t N, const float* x, int64_t Q, const float* stats, float* lap, float* grad,
               float* eik, float C, const Plan& plan, void* ws, hipStream_t st);

// Parameter backward: point blocks x query ranges.
struct BackPlan {
  int Sq;          // query ranges
  int64_t per_qs;  // queries per range (multiple of the query tile)
  int64_t pbs;     // point blocks of kBlock points
};
BackPlan make_back_plan(int64_t N, int64_t Q);
size_t back_ws_bytes(int64_t N, int64_t Q);  // dL/da and dL/dn only
// Workspace of the backward with dL/dp: per-range point partials (12 floats),
// M^2 and farthest slot per query, weight-sweep partials [S][Q] and the query
// records [Q][3] float4.  With ws = nullptr only `bytes` is meaningful.
struct BackPointsWs {
  float* gpp;
  float* far2;
  int32_t* farix;
  float* vpart;
  float4* qrec;
  size_t bytes;
};
BackPointsWs back_points_ws(int64_t N, int64_t Q, const Plan& plan, void* ws);
// sum_j w_j (g_j - phi) d_j per query and point split into vpart [S][Q].
int launch_vsum(const void* rec, int64_t N, const float* x, int64_t Q, const float* stats, float C,
                const Plan& plan, float* vpart, hipStream_t st);
// ga [N,6], gp [N,3], gn [N,3]: each may be null.  With gp, ws is a
// BackPointsWs of the plan; otherwise back_ws_bytes.
int launch_backward(const void* rec, int64_t N, const float* p, const float* n, const float* a, const float* x,
                    int64_t Q, const float* gout, const float* stats, float* ga, float* gp, float* gn, float C,
                    const Plan& plan, void* ws, hipStream_t st);

// Sphere tracing (point splits fixed by N so that rays do not affect each other).
// The march's split: the largest power of two <= cap leaving each split two
// 512-point tiles; pts_trace and the server both cap it at 64.  With the
// blend's split-major order a full-ray sweep costs the same at 16 or 64
// splits, and the late steps, with few rays still marching, need the
// parallelism (a walk of one split is their latency).
constexpr int kMarchSplitCap = 64;
int march_splits(int64_t N, int cap);
Plan march_plan(int64_t N, int64_t Q, const pts_params& P, int cap);
Plan normal_plan(int64_t N, int64_t Q, const pts_params& P);
size_t trace_eval_ws_bytes(int64_t N, int64_t R, const pts_params& P, int cap);  // evaluation part of the workspace
size_t trace_ws_bytes(int64_t N, int64_t R, const pts_params& P);
// eval_eps < 0: every step evaluates phi exactly (pts_eval's kernels); >= 0:
// with the error-bounded evaluation at that eps (workspace trace_bounded_ws_bytes).
size_t trace_bounded_ws_bytes(int64_t N, int64_t R, const pts_params& P);
int launch_trace(const void* rec, int64_t N, const float* org, const float* dir, int64_t R, int steps, float eps,
                 float tmax, float* t, float* nrm, int32_t* hit, int32_t* nsteps, const pts_params& P, void* ws,
                 size_t ws_bytes, hipStream_t st, float eval_eps = -1.f);
// Single steps of the march with the active-ray count left on the device.
int trace_init(int64_t R, int steps, float* t, int32_t* hit, int32_t* nsteps, int32_t* act, float* nrm,
               hipStream_t st);
int trace_step_pre(const int32_t* act, int64_t na, const float* org, const float* dir, const float* t, float* xq,
                   hipStream_t st);
int trace_step_post(const int32_t* act, int64_t na, const float* phi, float eps, float tmax, int step, float* t,
                    int32_t* hit, int32_t* nsteps, int32_t* keep, int32_t* act_out, int32_t* blk, int32_t* off,
                    int32_t* count, hipStream_t st);
int trace_hits(const int32_t* hit, int64_t R, int32_t* iota, int32_t* act_out, int32_t* blk, int32_t* off,
               int32_t* count, hipStream_t st);
int trace_normals_hits(const void* rec, int64_t N, const float* org, const float* dir, const float* t,
                       const int32_t* act, int64_t nh, float* xq, float* phi, float* g, float* nrm, const Plan& plan,
                       float C, void* ws, hipStream_t st);

}  // namespace pts
