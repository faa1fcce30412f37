// pts_backward.hip -- derivative of L = sum_q gout_q phi(x_q) with respect to
// the per-point coefficients a_i (the paper's representation is "fully
// differentiable", Sec. 6).
//
// The weights of Eq. (BasicFormulaShifted) depend on the points, not on a, so
//   dL/d theta_i = sum_q gout_q (w_qi / W_q) d g_i(x_q) / d theta_i.
// The torus of point i is parameterised by its anchor o = Q*(0,0) (on the
// equator), the orientation of its frame (u, m, k) (a rotation omega about
// o), L = 1/|kappa_min| and r, with c = o - L m and R = L - zeta r.  Unlike
// (c, u, R, r), these keep the derivatives well conditioned when L is large
// (nearly flat directions), where moving c and R would cancel to O(1/L^2).
// With v = x - c in the frame (vu, vm, vk), rho = |(vm, vk)|, b = rho - R,
// |q| = |(b, vu)|, g = sign (|q| - r) (Eq. SingleTorusSDF) and
// delta = rho - vm = vk^2 / (rho + vm) (vm > 0):
//   dg/do     = -grad g = -(sign/|q|) (vu, (b/rho) vm, (b/rho) vk)      [frame u, m, k]
//   dg/domega = -(x - o) x grad g
//             = (sign/|q|) ( b vk L / rho, -vu vk (1 - b/rho), -vu (L delta + vm zeta r) / rho )
//   dg/dL     = -sign b delta / (rho |q|)
//   dg/dr     =  sign (zeta b / |q| - 1)
//
//   k_backp   point-major sweep: one point per lane, query tiles staged in LDS
//             and read by every lane at the same address; 8 accumulators per
//             point; the queries are split into Sq ranges, each a separate
//             workgroup.
//   k_chain   per point: fixed-order sum over the query ranges, then the chain
//             rule to the six coefficients through the torus fit of Sec. 4.1
//             evaluated in FP64 on dual numbers (pts_fit.h): do/da, dL/da,
//             dr/da, and omega_j = 1/2 sum_e e x de/da_j over the frame vectors
//             e = u, m, k.  Result in the caller's point order.
#include "pts_device.h"
#include "pts_fit.h"

namespace pts {
namespace {

constexpr int kQTile = 256;

__global__ __launch_bounds__(kBlock) void k_backp(const Header* __restrict__ h, const float4* __restrict__ rec,
                                                  const float* __restrict__ x, int64_t Q, int Sq, int64_t per_qs,
                                                  const float* __restrict__ stats, const float* __restrict__ gout,
                                                  float C2, float* __restrict__ gpp) {
  __shared__ float4 qt[kQTile];
  __shared__ float qk[kQTile];
  const int qs = int(blockIdx.x % unsigned(Sq));
  const int64_t pb = blockIdx.x / unsigned(Sq);
  const int64_t N = h->N, nd = h->n_direct;
  const int64_t slot = pb * kBlock + threadIdx.x;
  const bool valid = slot < N;
  const bool direct = slot < nd;
  float4 P = make_float4(0.f, 0.f, 0.f, 1.f), U = make_float4(0.f, 0.f, 0.f, 0.f), Mv = U, K = U,
         G = make_float4(0.f, 0.f, 1.f, -1.f);
  if (valid) {
    const float4* r = rec + slot * kRecF4;
    P = r[0]; U = r[1]; Mv = r[2]; K = r[3]; G = r[4];
  }
  float acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = 0.f;
  const int64_t qbeg = int64_t(qs) * per_qs;
  const int64_t qend = min(Q, qbeg + per_qs);
  for (int64_t q0 = qbeg; q0 < qend; q0 += kQTile) {
    const int cnt = int(min<int64_t>(kQTile, qend - q0));
    __syncthreads();
    if (int(threadIdx.x) < cnt) {
      const int64_t q = q0 + threadIdx.x;
      const QueryIn qi = load_query(x, q, Q, h);
      const float M = stats[6 * q], W = stats[6 * q + 1];
      qt[threadIdx.x] = make_float4(qi.x, qi.y, qi.z, M > 0.f ? -2.f * C2 / M : 0.f);
      qk[threadIdx.x] = (gout ? gout[q] : 1.f) / W;
    }
    __syncthreads();
    float t[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) t[c] = 0.f;
    for (int j = 0; j < cnt; ++j) {
      const float4 X = qt[j];
      const float kap = qk[j];
      const float dx = X.x - P.x, dy = X.y - P.y, dz = X.z - P.z;
      const float d = hw_sqrt(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
      const float coef = hw_exp2(fmaf(d, X.w, C2)) * kap;
      const Geo r = direct ? geo_direct(X.x, X.y, X.z, U, Mv, K, G) : geo_anchored(X.x, X.y, X.z, P.w, U, Mv, K, G);
      const float iq = safe_rcp(r.qn), ir = safe_rcp(r.rho);
      const float sq = G.z * iq;                       // sign / |q|
      const float bir = r.b * ir;                      // b / rho
      const float L = P.w, zr = G.y;                   // L, zeta r
      const float delta = r.vm > 0.f ? r.vk * r.vk * safe_rcp(r.rho + r.vm) : r.rho - r.vm;
      const float c1 = coef * sq;
      t[0] = fmaf(-c1, r.vu, t[0]);                              // dg/do along u
      t[1] = fmaf(-c1, bir * r.vm, t[1]);                        //            m
      t[2] = fmaf(-c1, bir * r.vk, t[2]);                        //            k
      t[3] = fmaf(c1, bir * r.vk * L, t[3]);                     // dg/domega along u
      t[4] = fmaf(-c1, r.vu * r.vk * (1.f - bir), t[4]);         //                m
      t[5] = fmaf(-c1, r.vu * fmaf(L, delta, r.vm * zr) * ir, t[5]);  //           k
      t[6] = fmaf(-c1, r.b * delta * ir, t[6]);                  // dg/dL
      t[7] = fmaf(coef, G.z * fmaf(copysignf(1.f, zr), r.b * iq, -1.f), t[7]);  // dg/dr
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] += t[c];
  }
  if (valid) {
    float4* o = reinterpret_cast<float4*>(gpp + 8 * (int64_t(qs) * N + slot));
    o[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
    o[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
  }
}

__global__ __launch_bounds__(kBlock) void k_chain(const Header* __restrict__ h, const int32_t* __restrict__ perm,
                                                  const float* __restrict__ p, const float* __restrict__ n,
                                                  const float* __restrict__ a, int64_t N, int Sq,
                                                  const float* __restrict__ gpp, float* __restrict__ ga) {
  const int64_t slot = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (slot >= N) return;
  double G[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int s = 0; s < Sq; ++s) {
    const float* g = gpp + 8 * (int64_t(s) * N + slot);
    for (int c = 0; c < 8; ++c) G[c] += double(g[c]);
  }
  const int64_t i = perm[slot];
  double pd[3], nd[3];
  D6 ad[6];
  for (int k = 0; k < 3; ++k) { pd[k] = p[3 * i + k]; nd[k] = n[3 * i + k]; }
  for (int j = 0; j < 6; ++j) { ad[j] = d6(a[6 * i + j]); ad[j].d[j] = 1.0; }
  const FitT<D6> F = fit_point<D6>(pd, nd, ad, h->kfloor64);
  // forces on o and torques about o, from frame (u, m, k) to world
  double go[3], gw[3];
  for (int k = 0; k < 3; ++k) {
    go[k] = G[0] * F.u[k].v + G[1] * F.m[k].v + G[2] * F.k[k].v;
    gw[k] = G[3] * F.u[k].v + G[4] * F.m[k].v + G[5] * F.k[k].v;
  }
  for (int j = 0; j < 6; ++j) {
    // rotation of the frame per unit change of a_j: omega = 1/2 sum_e e x de/da_j
    double om[3] = {0.0, 0.0, 0.0};
    const D6* fr[3] = {F.u, F.m, F.k};
    for (int e = 0; e < 3; ++e) {
      const D6* E = fr[e];
      om[0] += 0.5 * (E[1].v * E[2].d[j] - E[2].v * E[1].d[j]);
      om[1] += 0.5 * (E[2].v * E[0].d[j] - E[0].v * E[2].d[j]);
      om[2] += 0.5 * (E[0].v * E[1].d[j] - E[1].v * E[0].d[j]);
    }
    double s = G[6] * F.L.d[j] + G[7] * F.r.d[j];
    for (int k = 0; k < 3; ++k) s += go[k] * F.o[k].d[j] + gw[k] * om[k];
    ga[6 * i + j] = float(s);
  }
}

__global__ __launch_bounds__(kBlock) void k_zero(float* __restrict__ out, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) out[i] = 0.f;
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

int launch_backward(const void* rec, int64_t N, const float* p, const float* n, const float* a, const float* x,
                    int64_t Q, const float* gout, const float* stats, float* ga, float C, void* ws, hipStream_t st) {
  const Layout L(N);
  const char* base = static_cast<const char*>(rec);
  const Header* h = reinterpret_cast<const Header*>(base);
  if (Q == 0) {  // no queries: dL/da = 0
    hipLaunchKernelGGL(k_zero, dim3(unsigned((6 * N + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, ga, 6 * N);
    return check_hip(hipGetLastError(), "zero fill");
  }
  const BackPlan b = make_back_plan(N, Q);
  float* gpp = static_cast<float*>(ws);
  hipLaunchKernelGGL(k_backp, dim3(unsigned(b.pbs * b.Sq)), dim3(kBlock), 0, st, h,
                     reinterpret_cast<const float4*>(base + L.rec), x, Q, b.Sq, b.per_qs, stats, gout, C * kLog2e,
                     gpp);
  hipLaunchKernelGGL(k_chain, dim3(unsigned(b.pbs)), dim3(kBlock), 0, st, h,
                     reinterpret_cast<const int32_t*>(base + L.perm), p, n, a, N, b.Sq, gpp, ga);
  return check_hip(hipGetLastError(), "parameter backward kernels");
}

}  // namespace pts
