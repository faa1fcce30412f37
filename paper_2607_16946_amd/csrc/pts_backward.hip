// pts_backward.hip -- derivatives of L = sum_q gout_q phi(x_q) with respect to
// the per-point coefficients a_i, points p_i and normals n_i (the paper's
// representation is "fully differentiable", Sec. 6).
//
// Through the torus.  The torus of point i is parameterised by its anchor
// o = Q*(0,0) (on the equator), the orientation of its frame (u, m, k) (a
// rotation omega about o), L = 1/|kappa_min| and r, with c = o - L m and
// R = L - zeta r.  Unlike (c, u, R, r), these keep the derivatives well
// conditioned when L is large (nearly flat directions), where moving c and R
// would cancel to O(1/L^2).  With v = x - c in the frame (vu, vm, vk),
// rho = |(vm, vk)|, b = rho - R, |q| = |(b, vu)|, g = sign (|q| - r)
// (Eq. SingleTorusSDF) and delta = rho - vm (= vk^2 / (rho + vm) for vm > 0):
//   dg/do     = -grad g = -(sign/|q|) (vu, (b/rho) vm, (b/rho) vk)      [frame u, m, k]
//   dg/domega = -(x - o) x grad g
//             = (sign/|q|) ( b vk L / rho, -vu vk R / rho, -vu (L delta + vm zeta r) / rho )
//   dg/dL     = -sign b delta / (rho |q|)
//   dg/dr     =  sign (zeta b / |q| - 1)  (= -sign vu^2 / (|q| (|q| + zeta b)))
// and dL/dtheta_i = sum_q gout_q (w_qi / W_q) dg_i(x_q)/dtheta_i for theta
// = a_i, n_i (the weights do not depend on them).  The anchor o = p + a00 n
// moves rigidly with p, so the torus part of dL/dp_i is the force on o.
//
// Through the weights (dL/dp only).  With d_i = |x - p_i|, e_i = (x - p_i)/d_i
// and lambda = 2C/M (Eq. RelationshipBetweenLambdaAndRadius), the weight
// exp(-lambda (d_i - sigma)) of Eq. (BasicFormulaShifted) gives
//   d phi / d p_i  +=  (w_i / W) lambda (g_i - phi) e_i,
// and the farthest point p_* of x sets M = d_*, so with
// V = (1/W) sum_j w_j (g_j - phi) d_j = -d phi / d lambda,
//   d phi / d p_*  +=  -(2C/M^2) V e_*.
//
//   (culled farthest-point sweep with the slot of p_*; pts_eval.hip)
//   k_vsum    query-major sweep of sum_j w_j (g_j - phi) d_j per point split
//             (pts_grad.hip)
//   k_qrec    per query: fixed-order sum of the splits, V, and the query record
//             the point sweep stages (x, -lambda log2 e; gout/W, phi, lambda,
//             slot of p_*; the farthest-point term)
//   k_backp   point-major sweep: one point per lane, query tiles staged in LDS
//             and read by every lane at the same address; 8 accumulators per
//             point (11 with the weight terms); the queries are split into Sq
//             ranges, each a separate workgroup.  A tile's queries whose p_* is
//             in the workgroup's point block are found with ballots and added
//             in query order (deterministic; no atomics).
//   k_chain   per point: fixed-order sum over the query ranges, then the chain
//             rule to the six coefficients (and the normal) through the torus
//             fit of Sec. 4.1 evaluated in FP64 on dual numbers (pts_fit.h):
//             do/dtheta, dL/dtheta, dr/dtheta, and omega_j = 1/2 sum_e e x
//             de/dtheta_j over the frame vectors e = u, m, k.  Results in the
//             caller's point order.
#include "pts_device.h"
#include "pts_fit.h"

#include <type_traits>

namespace pts {
namespace {

constexpr int kQTile = 256;

// Query record of the point sweep with the weight terms (three float4 per query).
__global__ __launch_bounds__(kBlock) void k_qrec(const Header* __restrict__ h, const float* __restrict__ x,
                                                 int64_t Q, const float* __restrict__ stats,
                                                 const float* __restrict__ vpart, int S,
                                                 const int32_t* __restrict__ farix, const float* __restrict__ gout,
                                                 float C, float4* __restrict__ qrec) {
  const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= Q) return;
  const float* st = stats + 6 * q;
  const float M = st[0], W = st[1], phi = st[2];
  float V = 0.f;
  for (int s = 0; s < S; ++s) V += vpart[int64_t(s) * Q + q];
  V /= W;
  const float go = gout ? gout[q] : 1.f;
  const float C2 = C * kLog2e;
  const float nlam = M > 0.f ? -2.f * C2 / M : 0.f;
  const float lam = M > 0.f ? 2.f * C / M : 0.f;
  const float f = M > 0.f ? -go * (2.f * C / (M * M)) * V : 0.f;
  const QueryIn qi = load_query(x, q, Q, h);
  qrec[3 * q] = make_float4(qi.x, qi.y, qi.z, nlam);
  qrec[3 * q + 1] = make_float4(go / W, phi, lam, __int_as_float(farix[q]));
  qrec[3 * q + 2] = make_float4(f * st[3], f * st[4], f * st[5], 0.f);
}

// Occupancy: the coefficient sweep fits 64 VGPRs (8 waves per SIMD, so the
// 2048-workgroup grid of the differentiation workload is one round); the sweep
// with the weight terms keeps its 70 at 7 waves (fitting 64 made it spill and
// ran 8% slower).
template <bool kW>
__global__ __launch_bounds__(kBlock, kW ? 7 : 8) void k_backp(const Header* __restrict__ h, const float4* __restrict__ rec,
                                                  const float* __restrict__ x, int64_t Q, int Sq, int64_t per_qs,
                                                  const float* __restrict__ stats, const float* __restrict__ gout,
                                                  const float4* __restrict__ qrec, float C2, float S2,
                                                  float* __restrict__ gpp) {
  constexpr int kStride = kW ? 12 : 8;
  __shared__ float4 qt[kQTile];
  __shared__ float qk[kW ? 1 : kQTile];
  __shared__ float4 qa[kW ? kQTile : 1];
  __shared__ float4 qf[kW ? kQTile : 1];
  __shared__ unsigned long long fmask[kW ? kQTile / 64 : 1];
  const int qs = int(blockIdx.x % unsigned(Sq));
  const int64_t pb = blockIdx.x / unsigned(Sq);
  const int64_t N = h->N, nd = h->n_direct;
  const int64_t base = pb * kBlock;
  const int64_t slot = base + threadIdx.x;
  const bool valid = slot < N;
  const bool direct = slot < nd;
  float4 P = make_float4(0.f, 0.f, 0.f, 1.f), U = make_float4(0.f, 0.f, 0.f, 0.f), Mv = U, K = U,
         G = make_float4(0.f, 0.f, 1.f, -1.f);
  if (valid) {
    const float4* r = rec + slot * kRecF4;
    P = r[0]; U = r[1]; Mv = r[2]; K = r[3]; G = r[4];
  }
  const bool wave_anchored = __ballot(valid && !direct) != 0ull;  // uniform across the wave
  float acc[kStride];
#pragma unroll
  for (int c = 0; c < kStride; ++c) acc[c] = 0.f;
  const int64_t qbeg = int64_t(qs) * per_qs;
  const int64_t qend = min(Q, qbeg + per_qs);
  for (int64_t q0 = qbeg; q0 < qend; q0 += kQTile) {
    const int cnt = int(min<int64_t>(kQTile, qend - q0));
    __syncthreads();
    if (kW) {
      bool far_here = false;
      if (int(threadIdx.x) < cnt) {
        const int64_t q = q0 + threadIdx.x;
        qt[threadIdx.x] = qrec[3 * q];
        const float4 A4 = qrec[3 * q + 1];
        qa[threadIdx.x] = A4;
        qf[threadIdx.x] = qrec[3 * q + 2];
        const int32_t fs = __float_as_int(A4.w);
        far_here = fs >= base && fs < base + kBlock;
      }
      const unsigned long long m = __ballot(far_here);
      if ((threadIdx.x & 63) == 0) fmask[threadIdx.x >> 6] = m;
    } else if (int(threadIdx.x) < cnt) {
      const int64_t q = q0 + threadIdx.x;
      const QueryIn qi = load_query(x, q, Q, h);
      const float M = stats[6 * q], W = stats[6 * q + 1];
      qt[threadIdx.x] = make_float4(qi.x, qi.y, qi.z, M > 0.f ? -2.f * C2 / M : 0.f);
      qk[threadIdx.x] = (gout ? gout[q] : 1.f) / W;
    }
    __syncthreads();
    float t[kStride];
#pragma unroll
    for (int c = 0; c < kStride; ++c) t[c] = 0.f;
    // One (query j, this lane's point) pair.  kMixed: the wave holds anchored
    // points (their own torus form, and the cancellation-free rho - vm);
    // waves of direct points only run the plain instance.
    auto pair = [&](int j, auto mixed) {
      constexpr bool kMixed = decltype(mixed)::value;
      const float4 X = qt[j];
      float kap, phi = 0.f, lam = 0.f;
      if constexpr (kW) {
        const float4 A4 = qa[j];
        kap = A4.x; phi = A4.y; lam = A4.z;
      } else {
        kap = qk[j];
      }
      const float dx = X.x - P.x, dy = X.y - P.y, dz = X.z - P.z;
      const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
      const float id = safe_rsq(d2);                     // 1/d (both variants form d alike)
      const float d = d2 * id;
      const float coef = hw_exp2(fmaf(d, X.w, S2)) * kap;
      const bool anch = kMixed && !direct;
      const Geo r = anch ? geo_anchored(X.x, X.y, X.z, P.w, U, Mv, K, G) : geo_direct(X.x, X.y, X.z, U, Mv, K, G);
      const float iq = r.iqn, ir = r.irho;
      const float sq = G.z * iq;                       // sign / |q|
      const float bir = r.b * ir;                      // b / rho
      const float L = P.w, zr = G.y;                   // L, zeta r
      // rho - vm cancels for vm > 0 near the plane vk = 0; its rounding error, about
      // eps rho, reaches the derivatives as eps L |vu| (dg/domega) and eps |b|
      // (dg/dL), which matters only for the large radii of anchored points (L > 4 D):
      // only they take the cancellation-free form (and its reciprocal)
      const float delta = anch && r.vm > 0.f ? r.vk * r.vk * safe_rcp(r.rho + r.vm) : r.rho - r.vm;
      const float c1 = coef * sq;
      t[0] = fmaf(-c1, r.vu, t[0]);                              // dg/do along u
      t[1] = fmaf(-c1, bir * r.vm, t[1]);                        //            m
      t[2] = fmaf(-c1, bir * r.vk, t[2]);                        //            k
      t[3] = fmaf(c1, bir * r.vk * L, t[3]);                     // dg/domega along u
      t[4] = fmaf(-c1, r.vu * r.vk * (G.x * ir), t[4]);          //                m (1 - b/rho = R/rho)
      t[5] = fmaf(-c1, r.vu * fmaf(L, delta, r.vm * zr) * ir, t[5]);  //           k
      t[6] = fmaf(-c1, r.b * delta * ir, t[6]);                  // dg/dL
      // dg/dr = sign (zeta b / |q| - 1) cancels where zeta b > 0 and |b| >> |vu|;
      // there it is -sign vu^2 / (|q| (|q| + zeta b)).  Its error is multiplied by
      // r^2 in dr/dkappa_max, so the anchored points (r up to L) take that form
      const float zb = copysignf(1.f, zr) * r.b;
      float dgr = fmaf(zb, iq, -1.f);
      // (|q| + zeta b as one explicit fma, so that both sweeps round it alike)
      if (anch && zb > 0.f) dgr = -(r.vu * r.vu) * iq * safe_rcp(fmaf(r.qn2, iq, zb));
      t[7] = fmaf(coef, G.z * dgr, t[7]);                        // dg/dr
      if constexpr (kW) {  // weight: (w/W) lambda (g - phi) e, e = (x - p)/d
        const float c3 = coef * lam * (r.g - phi) * id;
        t[8] = fmaf(c3, dx, t[8]);
        t[9] = fmaf(c3, dy, t[9]);
        t[10] = fmaf(c3, dz, t[10]);
      }
    };
    if (wave_anchored) {
      for (int j = 0; j < cnt; ++j) pair(j, std::true_type{});
    } else {
#pragma unroll 1
      for (int j = 0; j < cnt; ++j) pair(j, std::false_type{});
    }
    if (kW) {  // farthest-point terms of this tile, in query order
      for (int w = 0; w < kQTile / 64; ++w) {
        unsigned long long m = fmask[w];
        while (m) {
          const int j = w * 64 + __builtin_ctzll(m);
          m &= m - 1;
          if (__float_as_int(qa[j].w) == int32_t(slot)) {
            const float4 F = qf[j];
            t[8] += F.x;
            t[9] += F.y;
            t[10] += F.z;
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < kStride; ++c) acc[c] += t[c];
  }
  if (valid) {
    float4* o = reinterpret_cast<float4*>(gpp + kStride * (int64_t(qs) * N + slot));
    o[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
    o[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
    if (kW) o[2] = make_float4(acc[8], acc[9], acc[10], 0.f);
  }
}

// K = 6: derivatives in a; K = 9: in a and n.  kW: the sweep also produced the
// weight terms of dL/dp.
template <int K, bool kW>
__global__ __launch_bounds__(kBlock) void k_chain(const Header* __restrict__ h, const int32_t* __restrict__ perm,
                                                  const float* __restrict__ p, const float* __restrict__ n,
                                                  const float* __restrict__ a, int64_t N, int Sq,
                                                  const float* __restrict__ gpp, float* __restrict__ ga,
                                                  float* __restrict__ gp, float* __restrict__ gn) {
  using T = Dual<K>;
  constexpr int kStride = kW ? 12 : 8;
  const int64_t slot = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (slot >= N) return;
  double G[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int s = 0; s < Sq; ++s) {
    const float* g = gpp + kStride * (int64_t(s) * N + slot);
    for (int c = 0; c < kStride; ++c) G[c] += double(g[c]);
  }
  const int64_t i = perm[slot];
  double pd[3];
  T nd[3], ad[6];
  for (int k = 0; k < 3; ++k) {
    pd[k] = p[3 * i + k];
    nd[k] = dual<K>(n[3 * i + k]);
    if (K == 9) nd[k].d[6 + k] = 1.0;
  }
  for (int j = 0; j < 6; ++j) { ad[j] = dual<K>(a[6 * i + j]); ad[j].d[j] = 1.0; }
  const FitT<T> F = fit_point<T>(pd, nd, ad, h->kfloor64);
  // forces on o and torques about o, from frame (u, m, k) to world
  double go[3], gw[3];
  for (int k = 0; k < 3; ++k) {
    go[k] = G[0] * F.u[k].v + G[1] * F.m[k].v + G[2] * F.k[k].v;
    gw[k] = G[3] * F.u[k].v + G[4] * F.m[k].v + G[5] * F.k[k].v;
  }
  for (int j = 0; j < K; ++j) {
    // rotation of the frame per unit change of parameter j: omega = 1/2 sum_e e x de/dtheta_j
    double om[3] = {0.0, 0.0, 0.0};
    const T* fr[3] = {F.u, F.m, F.k};
    for (int e = 0; e < 3; ++e) {
      const T* E = fr[e];
      om[0] += 0.5 * (E[1].v * E[2].d[j] - E[2].v * E[1].d[j]);
      om[1] += 0.5 * (E[2].v * E[0].d[j] - E[0].v * E[2].d[j]);
      om[2] += 0.5 * (E[0].v * E[1].d[j] - E[1].v * E[0].d[j]);
    }
    double s = G[6] * F.L.d[j] + G[7] * F.r.d[j];
    for (int k = 0; k < 3; ++k) s += go[k] * F.o[k].d[j] + gw[k] * om[k];
    if (j < 6) {
      if (ga) ga[6 * i + j] = float(s);
    } else {
      gn[3 * i + (j - 6)] = float(s);
    }
  }
  // the anchor moves rigidly with p: torus part go, plus the weight terms
  if (kW && gp)
    for (int k = 0; k < 3; ++k) gp[3 * i + k] = float(go[k] + G[8 + k]);
}

__global__ __launch_bounds__(kBlock) void k_zero(float* __restrict__ out, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) out[i] = 0.f;
}

int zero(float* out, int64_t n, hipStream_t st) {
  if (!out || n == 0) return PTS_OK;
  hipLaunchKernelGGL(k_zero, dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, out, n);
  return check_hip(hipGetLastError(), "zero fill");
}

}  // namespace

BackPlan make_back_plan(int64_t N, int64_t Q) {
  BackPlan b;
  const int64_t pbs = (N + kBlock - 1) / kBlock;
  const int64_t qtiles = (Q + kQTile - 1) / kQTile;
  int Sq = 1;
  while (Sq < 256 && pbs * Sq < 2048 && qtiles >= int64_t(2) * Sq) Sq *= 2;
  b.per_qs = ((qtiles + Sq - 1) / Sq) * kQTile;
  b.Sq = int((Q + b.per_qs - 1) / b.per_qs);
  if (b.Sq < 1) b.Sq = 1;
  b.pbs = pbs;
  return b;
}

size_t back_ws_bytes(int64_t N, int64_t Q) {
  const BackPlan b = make_back_plan(N, Q);
  return align256(size_t(b.Sq) * size_t(N) * 8 * sizeof(float));
}

BackPointsWs back_points_ws(int64_t N, int64_t Q, const Plan& plan, void* ws) {
  const BackPlan b = make_back_plan(N, Q);
  char* c = static_cast<char*>(ws);
  BackPointsWs v;
  v.bytes = 0;
  v.gpp = reinterpret_cast<float*>(c);
  v.bytes += align256(size_t(b.Sq) * size_t(N) * 12 * sizeof(float));
  v.far2 = reinterpret_cast<float*>(c ? c + v.bytes : nullptr);
  v.bytes += align256(size_t(Q) * sizeof(float));
  v.farix = reinterpret_cast<int32_t*>(c ? c + v.bytes : nullptr);
  v.bytes += align256(size_t(Q) * sizeof(int32_t));
  v.vpart = reinterpret_cast<float*>(c ? c + v.bytes : nullptr);
  v.bytes += align256(size_t(plan.S) * size_t(Q) * sizeof(float));
  v.qrec = reinterpret_cast<float4*>(c ? c + v.bytes : nullptr);
  v.bytes += align256(size_t(Q) * 3 * sizeof(float4));
  return v;
}

int launch_backward(const void* rec, int64_t N, const float* p, const float* n, const float* a, const float* x,
                    int64_t Q, const float* gout, const float* stats, float* ga, float* gp, float* gn, float C,
                    const Plan& plan, void* ws, hipStream_t st) {
  const Layout L(N);
  const char* base = static_cast<const char*>(rec);
  const Header* h = reinterpret_cast<const Header*>(base);
  if (Q == 0) {  // no queries: every derivative is 0
    if (int rc = zero(ga, 6 * N, st)) return rc;
    if (int rc = zero(gp, 3 * N, st)) return rc;
    return zero(gn, 3 * N, st);
  }
  const BackPlan b = make_back_plan(N, Q);
  const float4* recs = reinterpret_cast<const float4*>(base + L.rec);
  const int32_t* perm = reinterpret_cast<const int32_t*>(base + L.perm);
  const float C2 = C * kLog2e, S2 = shift2_of(C);
  const unsigned gb = unsigned(b.pbs * b.Sq);
  if (gp) {
    const BackPointsWs v = back_points_ws(N, Q, plan, ws);
    if (int rc = launch_far_cull(rec, N, x, Q, plan.qpl, v.far2, v.farix, st)) return rc;
    if (int rc = launch_vsum(rec, N, x, Q, stats, C, plan, v.vpart, st)) return rc;
    hipLaunchKernelGGL(k_qrec, dim3(unsigned((Q + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, h, x, Q, stats,
                       v.vpart, plan.S, v.farix, gout, C, v.qrec);
    hipLaunchKernelGGL(k_backp<true>, dim3(gb), dim3(kBlock), 0, st, h, recs, x, Q, b.Sq, b.per_qs, stats, gout,
                       v.qrec, C2, S2, v.gpp);
    if (gn)
      hipLaunchKernelGGL((k_chain<9, true>), dim3(unsigned(b.pbs)), dim3(kBlock), 0, st, h, perm, p, n, a, N, b.Sq,
                         v.gpp, ga, gp, gn);
    else
      hipLaunchKernelGGL((k_chain<6, true>), dim3(unsigned(b.pbs)), dim3(kBlock), 0, st, h, perm, p, n, a, N, b.Sq,
                         v.gpp, ga, gp, gn);
  } else {
    float* gpp = static_cast<float*>(ws);
    hipLaunchKernelGGL(k_backp<false>, dim3(gb), dim3(kBlock), 0, st, h, recs, x, Q, b.Sq, b.per_qs, stats, gout,
                       nullptr, C2, S2, gpp);
    if (gn)
      hipLaunchKernelGGL((k_chain<9, false>), dim3(unsigned(b.pbs)), dim3(kBlock), 0, st, h, perm, p, n, a, N,
                         b.Sq, gpp, ga, gp, gn);
    else
      hipLaunchKernelGGL((k_chain<6, false>), dim3(unsigned(b.pbs)), dim3(kBlock), 0, st, h, perm, p, n, a, N,
                         b.Sq, gpp, ga, gp, gn);
  }
  return check_hip(hipGetLastError(), "backward kernels");
}

}  // namespace pts
