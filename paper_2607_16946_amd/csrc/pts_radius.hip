// pts_radius.hip -- radius-limited evaluation (Sec. 4.2, "Acceleration and
// adaptive lambda").
//
// The paper's accelerated evaluation keeps lambda constant for a cloud:
//   D      = mean over points of the mean distance to their 64 nearest other
//            points,
//   lambda = 1e3 / D,   R_eval = 2C / lambda   (sigma = R_eval / 2, so that
//            lambda = C / sigma as in Eq. RelationshipBetweenLambdaAndRadius),
// and blends Eq. (BasicFormulaShifted) only over the points within R_eval of
// the query; if there are none, over the 32 nearest points (then shifted by
// the nearest distance, which keeps the largest weight at 1; phi does not
// depend on the shift).
//
// Queries are taken in Morton order of the cloud's bbox (a radix sort of
// their keys on the device), so that neighbouring lanes walk the same part of
// the hierarchy instead of the union of 64 unrelated walks.
//
// Search structure: the build orders points spatially and bounds every unit
// of kUnit slots and every block of kBlkU units by a sphere.  Each lane owns one
// query and walks the blocks and units in slot order, skipping every sphere
// that cannot reach the current search radius; the k nearest squared
// distances are kept in registers, sorted, with a branch-free insertion.  The
// k-nearest search is seeded with the unit whose center is nearest within the
// block whose center is nearest, so the radius is finite from the start.
//
// Sphere tests use a relative margin of 1e-5 on the radius (units and blocks
// never skip a point FP32 rounding could bring inside); point tests use the
// FP32 squared distance itself, so the selected set is exactly the points
// whose computed distance passes.
#include "pts_device.h"

namespace pts {
namespace {

constexpr int kKnnD = 64;   // neighbours in the mean-distance heuristic
constexpr int kKnnFb = 32;  // nearest points of the fallback
constexpr float kInf = 3.0e38f;

struct Tree {
  const float4* pos4;  // (-2p, |p|^2) per slot
  const float4* ub;    // per unit: (c, r), (e, 0)
  const float4* bb;    // per block: (c, r)
  const float4* ob;    // per unit: oriented box (c, 0), (a_k, e_k)
  int64_t N, nunit, nbk;
};

__device__ __forceinline__ Tree tree_of(const void* rec, int64_t N) {
  const Layout L(N);
  const char* base = static_cast<const char*>(rec);
  Tree t;
  t.pos4 = reinterpret_cast<const float4*>(base + L.pos);
  t.ub = reinterpret_cast<const float4*>(base + L.ub);
  t.bb = reinterpret_cast<const float4*>(base + L.bb);
  t.ob = reinterpret_cast<const float4*>(base + L.ob);
  t.N = N;
  t.nunit = L.nunit;
  t.nbk = L.nbk;
  return t;
}

// |x - p|^2 from the stored (-2p, |p|^2): x - p = x + (-2p)/2 (exact halving).
__device__ __forceinline__ float dist2(float x, float y, float z, const float4& P) {
  const float dx = fmaf(0.5f, P.x, x), dy = fmaf(0.5f, P.y, y), dz = fmaf(0.5f, P.z, z);
  return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

// Can a sphere (c, r) hold a point within radius `rad` of x?  (margin 1e-5)
__device__ __forceinline__ bool reaches(float x, float y, float z, const float4& S, float rad) {
  const float dx = x - S.x, dy = y - S.y, dz = z - S.z;
  const float lim = fmaf(rad, 1.00001f, S.w);
  return fmaf(dz, dz, fmaf(dy, dy, dx * dx)) <= lim * lim;
}

// The same question for a unit's oriented box B[0..3] (center, then axis and
// half-extent per axis): its nearest distance is |max(t - e, 0)| with
// t_k = |<x - c, a_k>|.  Asked after the sphere test passes; the limit adds
// 1e-6 of the farthest distance for the FP32 rounding of t.
__device__ __forceinline__ bool reaches_box(float x, float y, float z, const float4* __restrict__ B, float rad) {
  const float4 C = B[0], A0 = B[1], A1 = B[2], A2 = B[3];
  const float ex = x - C.x, ey = y - C.y, ez = z - C.z;
  const float t0 = fabsf(fmaf(ez, A0.z, fmaf(ey, A0.y, ex * A0.x)));
  const float t1 = fabsf(fmaf(ez, A1.z, fmaf(ey, A1.y, ex * A1.x)));
  const float t2 = fabsf(fmaf(ez, A2.z, fmaf(ey, A2.y, ex * A2.x)));
  const float l0 = fmaxf(t0 - A0.w, 0.f), l1 = fmaxf(t1 - A1.w, 0.f), l2 = fmaxf(t2 - A2.w, 0.f);
  const float hsum = (t0 + A0.w) + (t1 + A1.w) + (t2 + A2.w);
  const float lim = fmaf(rad, 1.00001f, 1e-6f * hsum);
  return fmaf(l2, l2, fmaf(l1, l1, l0 * l0)) <= lim * lim;
}

template <int K>
__device__ __forceinline__ void list_insert(float (&a)[K], float v) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const float lo = fminf(a[i], v);
    v = fmaxf(a[i], v);
    a[i] = lo;
  }
}

// The K smallest squared distances from x to the points (slot `self` excluded),
// ascending in a[]; entries stay kInf when there are fewer than K points.
// kSeedFirst walks the seed's block before the others (the order does not
// change the result): measured faster for the per-point search of the
// preparation (every query on the surface), slower for the evaluation's
// lattice queries, whose waves then split over different seed blocks.
template <int K, bool kSeedFirst>
__device__ void knn(const Tree& T, float x, float y, float z, int64_t self, float (&a)[K]) {
#pragma unroll
  for (int i = 0; i < K; ++i) a[i] = kInf;
  // seed: nearest block center, then nearest unit center inside it
  int64_t sb = 0;
  float best = kInf;
  for (int64_t b = 0; b < T.nbk; ++b) {
    const float4 S = T.bb[b];
    const float dx = x - S.x, dy = y - S.y, dz = z - S.z;
    const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    if (d2 < best) { best = d2; sb = b; }
  }
  const int64_t u0 = sb * kBlkU, u1 = min(T.nunit, u0 + kBlkU);
  int64_t su = u0;
  best = kInf;
  for (int64_t u = u0; u < u1; ++u) {
    const float4 S = T.ub[2 * u];
    const float dx = x - S.x, dy = y - S.y, dz = z - S.z;
    const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    if (d2 < best) { best = d2; su = u; }
  }
  const int64_t s1 = min(T.N, (su + 1) * kUnit);
  for (int64_t s = su * kUnit; s < s1; ++s) {
    if (s == self) continue;
    const float d2 = dist2(x, y, z, T.pos4[s]);
    if (d2 < a[K - 1]) list_insert(a, d2);
  }
  float rad = a[K - 1] < kInf ? sqrtf(a[K - 1]) : kInf;
  // every other unit the current radius can reach, in slot order (with
  // kSeedFirst the seed's block first, so that the radius is near its final
  // value before the other blocks are tested)
  auto walk = [&](int64_t b) {
    if (!reaches(x, y, z, T.bb[b], rad)) return;
    const int64_t v1 = min(T.nunit, (b + 1) * kBlkU);
    for (int64_t u = b * kBlkU; u < v1; ++u) {
      if (u == su || !reaches(x, y, z, T.ub[2 * u], rad) || !reaches_box(x, y, z, T.ob + 4 * u, rad)) continue;
      const int64_t e = min(T.N, (u + 1) * kUnit);
      for (int64_t s = u * kUnit; s < e; ++s) {
        if (s == self) continue;
        const float d2 = dist2(x, y, z, T.pos4[s]);
        if (d2 < a[K - 1]) {
          list_insert(a, d2);
          if (a[K - 1] < kInf) rad = sqrtf(a[K - 1]);
        }
      }
    }
  };
  if (kSeedFirst) walk(sb);
  for (int64_t b = 0; b < T.nbk; ++b)
    if (!kSeedFirst || b != sb) walk(b);
}

// Blend over every point with squared distance <= lim2:
// w = 2^((sigma - d) lambda log2e), num += w g, den += w; returns the count.
__device__ int blend_within(const Tree& T, const float4* rec, int64_t nd, float x, float y, float z, float lim2,
                            float sigma, float lam2, float& num, float& den) {
  const float rad = sqrtf(lim2);
  int cnt = 0;
  for (int64_t b = 0; b < T.nbk; ++b) {
    if (!reaches(x, y, z, T.bb[b], rad)) continue;
    const int64_t v1 = min(T.nunit, (b + 1) * kBlkU);
    for (int64_t u = b * kBlkU; u < v1; ++u) {
      if (!reaches(x, y, z, T.ub[2 * u], rad) || !reaches_box(x, y, z, T.ob + 4 * u, rad)) continue;
      const int64_t e = min(T.N, (u + 1) * kUnit);
      for (int64_t s = u * kUnit; s < e; ++s) {
        const float d2 = dist2(x, y, z, T.pos4[s]);
        if (!(d2 <= lim2)) continue;
        const float4* R = rec + s * kRecF4;
        const float4 P = R[0], U = R[1], Mv = R[2], K = R[3], G = R[4];
        const float g = s < nd ? g_direct(x, y, z, U, Mv, K, G) : g_anchored(x, y, z, P.w, U, Mv, K, G);
        // |x - p| in FP64 from the FP32 coordinates (their differences are exact):
        // lambda = 1e3 / D is large, so the FP32 rounding of a distance of, say,
        // half the cloud would reach the exponent as lambda eps d ~ 1e-3
        const double ex = double(x) - double(P.x), ey = double(y) - double(P.y), ez = double(z) - double(P.z);
        const double dd = sqrt(fma(ez, ez, fma(ey, ey, ex * ex)));
        const float w = hw_exp2(float((double(sigma) - dd) * double(lam2)));
        num = fmaf(w, g, num);
        den += w;
        ++cnt;
      }
    }
  }
  return cnt;
}

// Block spheres enclosing their units' spheres.
__global__ __launch_bounds__(kBlock) void k_blocks(const float4* __restrict__ ub, int64_t nunit, int64_t nbk,
                                                   float4* __restrict__ bb) {
  const int64_t b = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (b >= nbk) return;
  const int64_t u0 = b * kBlkU, u1 = min(nunit, u0 + kBlkU);
  float lo[3] = {kInf, kInf, kInf}, hi[3] = {-kInf, -kInf, -kInf};
  for (int64_t u = u0; u < u1; ++u) {
    const float4 S = ub[2 * u];
    const float c[3] = {S.x, S.y, S.z};
    for (int k = 0; k < 3; ++k) {
      lo[k] = fminf(lo[k], c[k] - S.w);
      hi[k] = fmaxf(hi[k], c[k] + S.w);
    }
  }
  const float cx = 0.5f * (lo[0] + hi[0]), cy = 0.5f * (lo[1] + hi[1]), cz = 0.5f * (lo[2] + hi[2]);
  double r = 0.0;
  for (int64_t u = u0; u < u1; ++u) {
    const float4 S = ub[2 * u];
    const double dx = double(S.x) - cx, dy = double(S.y) - cy, dz = double(S.z) - cz;
    r = fmax(r, sqrt(dx * dx + dy * dy + dz * dz) + double(S.w));
  }
  bb[b] = make_float4(cx, cy, cz, float(r * (1.0 + 1e-6)) + 1e-30f);
}

// Per point: mean distance to its 64 nearest other points (FP64 out).
__global__ __launch_bounds__(kBlock) void k_knn_mean(const Header* __restrict__ h, const void* __restrict__ rec,
                                                     int64_t N, double* __restrict__ mean) {
  const int64_t s = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (s >= N) return;
  const Tree T = tree_of(rec, N);
  const float4 P = T.pos4[s];
  float a[kKnnD];
  knn<kKnnD, true>(T, -0.5f * P.x, -0.5f * P.y, -0.5f * P.z, s, a);
  const int kk = int(min<int64_t>(kKnnD, N - 1));
  double sum = 0.0;
  for (int i = 0; i < kKnnD; ++i)
    if (i < kk) sum += sqrt(double(a[i]));
  mean[s] = sum / double(kk);
  (void)h;
}

// D = (sum of per-point means in slot order, fixed tree) / N; lambda and R_eval
// into the header.  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_knn_finish(Header* __restrict__ h, const double* __restrict__ mean,
                                                     int64_t N, float C) {
  __shared__ double s[1024];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += 1024) acc += mean[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < unsigned(o)) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double D = N > 1 ? s[0] / double(N) : 1.0;
    const double lam = 1e3 / D;
    h->rl_D = D;
    h->rl_lambda = float(lam);
    h->rl_reval = float(2.0 * double(C) / lam);
    h->rl_shift = float(double(C < kShiftMaxC ? C : kShiftMaxC) / lam);  // = rl_reval / 2 for C <= 64
    h->rl_ready = 1;
  }
}

// phi at queries: points within R_eval, else the 32 nearest.  Lane i takes the
// i-th query in Morton order (order[i]), so a wavefront's queries are a compact
// brick and its lanes walk nearly the same blocks and units; results go back to
// the query's own index.
__global__ __launch_bounds__(kBlock) void k_eval_radius(const Header* __restrict__ h, const void* __restrict__ recb,
                                                        const float* __restrict__ x, int64_t Q,
                                                        const int32_t* __restrict__ order,
                                                        float* __restrict__ sdf, int32_t* __restrict__ count) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= Q) return;
  const int64_t q = order[i];
  const int64_t N = h->N;
  const QueryIn qi = load_query(x, q, Q, h);
  const bool finite = isfinite(qi.x) && isfinite(qi.y) && isfinite(qi.z);
  if (!h->rl_ready || !finite) {
    sdf[q] = __builtin_nanf("");
    if (count) count[q] = 0;
    return;
  }
  const Tree T = tree_of(recb, N);
  const float4* rec = reinterpret_cast<const float4*>(static_cast<const char*>(recb) + Layout(N).rec);
  const float lam2 = h->rl_lambda * kLog2e, reval = h->rl_reval;
  float num = 0.f, den = 0.f;
  int cnt = blend_within(T, rec, h->n_direct, qi.x, qi.y, qi.z, reval * reval, h->rl_shift, lam2, num, den);
  if (cnt == 0) {
    float a[kKnnFb];
    knn<kKnnFb, false>(T, qi.x, qi.y, qi.z, -1, a);
    const float lim2 = a[kKnnFb - 1];            // kInf when N < 32: every point
    cnt = -blend_within(T, rec, h->n_direct, qi.x, qi.y, qi.z, lim2, sqrtf(a[0]), lam2, num, den);
  }
  sdf[q] = num / den;
  if (count) count[q] = cnt;
}

}  // namespace

int launch_blocks(void* rec, int64_t N, hipStream_t st) {
  const Layout L(N);
  char* base = static_cast<char*>(rec);
  hipLaunchKernelGGL(k_blocks, dim3(unsigned((L.nbk + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     reinterpret_cast<const float4*>(base + L.ub), L.nunit, L.nbk,
                     reinterpret_cast<float4*>(base + L.bb));
  return check_hip(hipGetLastError(), "block bounds kernel");
}

int launch_radius_prepare(void* rec, int64_t N, float C, hipStream_t st) {
  const Layout L(N);
  char* base = static_cast<char*>(rec);
  Header* h = reinterpret_cast<Header*>(base);
  // per-point means in the build's sort scratch (2 x 4N bytes of keys, 8N needed)
  double* mean = reinterpret_cast<double*>(base + L.key);
  hipLaunchKernelGGL(k_knn_mean, dim3(unsigned((N + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, h, rec, N, mean);
  hipLaunchKernelGGL(k_knn_finish, dim3(1), dim3(1024), 0, st, h, mean, N, C);
  return check_hip(hipGetLastError(), "radius prepare kernels");
}

// Workspace: Morton keys and query indices [2][Q] each, radix histograms.
namespace {
struct RadiusWs {
  uint32_t* key[2];
  int32_t* idx[2];
  int32_t* rhist;
  size_t bytes;
};
RadiusWs radius_ws(int64_t Q, void* ws) {
  char* c = static_cast<char*>(ws);
  RadiusWs v;
  size_t o = 0;
  auto take = [&](size_t b) {
    char* r = c ? c + o : nullptr;
    o += align256(b);
    return r;
  };
  for (int k = 0; k < 2; ++k) v.key[k] = reinterpret_cast<uint32_t*>(take(size_t(Q) * 4));
  for (int k = 0; k < 2; ++k) v.idx[k] = reinterpret_cast<int32_t*>(take(size_t(Q) * 4));
  v.rhist = reinterpret_cast<int32_t*>(take(size_t((Q + kBlock - 1) / kBlock) * 16 * 4));
  v.bytes = o;
  return v;
}
}  // namespace

size_t eval_radius_ws_bytes(int64_t Q) { return radius_ws(Q, nullptr).bytes; }

int launch_eval_radius(const void* rec, int64_t N, const float* x, int64_t Q, float* sdf, int32_t* count,
                       void* ws, hipStream_t st) {
  (void)N;
  RadiusWs v = radius_ws(Q, ws);
  const int32_t* order = nullptr;
  if (int rc = launch_query_order(rec, x, Q, v.key, v.idx, v.rhist, st, &order)) return rc;
  hipLaunchKernelGGL(k_eval_radius, dim3(unsigned((Q + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     static_cast<const Header*>(rec), rec, x, Q, order, sdf, count);
  return check_hip(hipGetLastError(), "radius evaluation kernel");
}

}  // namespace pts
