// pts_lap.hip -- Laplacian of phi, with its gradient and the eikonal residual
// |grad phi| - 1, at a set of queries (App. D gives the Laplacian for a fixed
// lambda; here lambda_x = 2C/M(x) moves with x as well).
//
// Write <h> = sum_i w_i h_i / W for the normalised weights of
// Eq. (BasicFormulaShifted), d_i = |x - p_i|, e_i = (x - p_i)/d_i, and
// F(x, lambda) = <g>.  With lambda fixed (App. D, written out in 3D):
//   grad F = <grad g> - lambda <(g - phi) e>
//   Lap  F = <Lap g> - 2 lambda <grad g . e> + 2 lambda <grad g> . <e>
//            - 2 lambda <(g - phi)/d> - 2 lambda^2 <(g - phi) e> . <e>.
// lambda_x = 2C/M with M = |x - p_*| (p_* the farthest point) has
// grad lambda = -kappa e_*, kappa = 2C/M^2, and Lap lambda = 0 (1/|x - p_*| is
// harmonic in 3D), so
//   Lap phi = Lap F + 2 grad F_lambda . grad lambda + F_lambda,lambda |grad lambda|^2
// with
//   F_lambda        = -V,  V = <(g - phi) d>
//   F_lambda,lambda = <(g - phi) d^2> - 2 <d> V
//   grad V          = <d grad g> + <(g - phi) e> - lambda <(g - phi) d e>
//                     + lambda V <e> - <d> grad F,
// i.e. Lap phi = Lap F + 2 kappa grad V . e_* + kappa^2 F_lambda,lambda, and
// grad phi = grad F + kappa V e_* (the gradient of pts_eval).
// For one torus (Eq. SingleTorusSDF), g = sign (|q| - r) with |q| = |(b, vu)|,
// b = rho - R, and in the torus's cylindrical coordinates
//   Lap g = sign (1 + b / rho) / |q|.
// The factors 1/rho, 1/|q|, 1/d are taken as 0 where they vanish (the same
// subgradient convention as the gradient sweeps).
//
//   k_lap          query-major sweep over point splits: 22 weighted sums per
//                  query (W itself and the moments above; only the e_*
//                  projections of the vectors that enter grad V . e_*).  The
//                  cancellations below need one set of weights and one phi:
//                  the forward's W and phi differ from this sweep's in their
//                  last bits, and 2 lambda^2 times such a difference is not
//                  small.  So the moments are normalised by this sweep's own
//                  W, and the (g - phi) sums, centred on the forward's phi to
//                  keep them small, are re-centred exactly on this sweep's
//                  phi with the extra moments <g - phi_fwd>, <1/d>,
//                  <d e . e_*> and <d^2>.  The formulas cancel terms
//                  of size lambda ~ 2C/M down to the O(1) Laplacian, so the
//                  sums run in FP32 over runs of kSub points and are carried
//                  in FP64 (a plain FP32 running sum over N points loses
//                  ~sqrt(N) eps of each term, ~1e-3 of the result at N ~ 2000);
//                  per-split partials are stored in FP64.
//   k_lap_combine  fixed-order FP64 sum over splits, then the formulas above
//                  in FP64; outputs rounded to FP32.
#include "pts_device.h"

namespace pts {
namespace {

constexpr int kLapAcc = 22;
constexpr int kLapD2 = 11;  // partials per (split, query): 22 doubles in 11 double2
constexpr int kSub = 16;    // points per FP32 run before the FP64 carry

template <bool kDirect>
__device__ __forceinline__ void lap_pair(float qx, float qy, float qz, float nl, float S2, float phi,
                                         float ex, float ey, float ez, const float4& P, const float4& U,
                                         const float4& Mv, const float4& K, const float4& G, float* a) {
  const float dx = qx - P.x, dy = qy - P.y, dz = qz - P.z;
  const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
  const float id = safe_rsq(d2);                                    // 1/d
  const float d = d2 * id;
  const float w = hw_exp2(fmaf(d, nl, S2));
  const Geo r = kDirect ? geo_direct(qx, qy, qz, U, Mv, K, G) : geo_anchored(qx, qy, qz, P.w, U, Mv, K, G);
  const float sq = G.z * r.iqn;
  const float bir = r.b * r.irho;
  const float f1 = sq * bir;
  const float f2 = sq * r.vu;
  const float a1 = f1 * r.vm, a2 = f1 * r.vk;
  const float gx = fmaf(a1, Mv.x, fmaf(a2, K.x, f2 * U.x));
  const float gy = fmaf(a1, Mv.y, fmaf(a2, K.y, f2 * U.y));
  const float gz = fmaf(a1, Mv.z, fmaf(a2, K.z, f2 * U.z));
  const float lapg = sq * (1.f + bir);
  const float ux = dx * id, uy = dy * id, uz = dz * id;            // e
  const float gdote = fmaf(gx, ux, fmaf(gy, uy, gz * uz));          // grad g . e
  const float gdots = fmaf(gx, ex, fmaf(gy, ey, gz * ez));          // grad g . e_*
  const float edots = fmaf(ux, ex, fmaf(uy, ey, uz * ez));          // e . e_*
  const float gm = w * (r.g - phi);                                 // w (g - phi)
  const float wd = w * d;
  const float gmd = gm * d;
  a[0] = fmaf(w, lapg, a[0]);
  a[1] = fmaf(w, gdote, a[1]);
  a[2] = fmaf(w, gx, a[2]);
  a[3] = fmaf(w, gy, a[3]);
  a[4] = fmaf(w, gz, a[4]);
  a[5] = fmaf(w, ux, a[5]);
  a[6] = fmaf(w, uy, a[6]);
  a[7] = fmaf(w, uz, a[7]);
  a[8] = fmaf(gm, id, a[8]);
  a[9] = fmaf(gm, ux, a[9]);
  a[10] = fmaf(gm, uy, a[10]);
  a[11] = fmaf(gm, uz, a[11]);
  a[12] = fmaf(wd, gdots, a[12]);
  a[13] = fmaf(gmd, edots, a[13]);
  a[14] += gmd;
  a[15] += wd;
  a[16] = fmaf(gmd, d, a[16]);
  a[17] += w;
  a[18] += gm;
  a[19] = fmaf(w, id, a[19]);
  a[20] = fmaf(wd, edots, a[20]);
  a[21] = fmaf(wd, d, a[21]);
}

template <int QPL>
__global__ __launch_bounds__(kBlock) void k_lap(const Header* __restrict__ h, const float4* __restrict__ rec,
                                                const float* __restrict__ x, int64_t Q, int S, int64_t per_split,
                                                const float* __restrict__ stats, float C2, float S2,
                                                double2* __restrict__ part) {
  __shared__ float4 tile[kTile2 * kRecF4];
  // split = b % S: the blend's split-major order (split_block) is not worth
  // the slower pair-loop schedule hipcc gives this sweep with it
  const int split = int(blockIdx.x % unsigned(S));
  const int64_t qb = blockIdx.x / unsigned(S);
  const int64_t N = h->N;
  const int64_t nd = h->n_direct;
  float qx[QPL], qy[QPL], qz[QPL], nl[QPL], ph[QPL], es[QPL][3];
  double A[QPL][kLapAcc];
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int64_t q = qb * (kBlock * QPL) + k * kBlock + threadIdx.x;
    const QueryIn qi = load_query(x, q, Q, h);
    qx[k] = qi.x; qy[k] = qi.y; qz[k] = qi.z;
    nl[k] = 0.f;
    ph[k] = 0.f;
    es[k][0] = es[k][1] = es[k][2] = 0.f;
    if (qi.valid) {
      const float* st = stats + 6 * q;
      const float M = st[0];
      nl[k] = M > 0.f ? -2.f * C2 / M : 0.f;
      ph[k] = st[2];
      es[k][0] = st[3]; es[k][1] = st[4]; es[k][2] = st[5];
    }
#pragma unroll
    for (int c = 0; c < kLapAcc; ++c) A[k][c] = 0.0;
  }
  const int64_t beg = int64_t(split) * per_split;
  const int64_t end = min(N, beg + per_split);
  for (int64_t t0 = beg; t0 < end; t0 += kTile2) {
    const int cnt = int(min<int64_t>(kTile2, end - t0));
    __syncthreads();
    for (int j = threadIdx.x; j < cnt * kRecF4; j += kBlock) tile[j] = rec[t0 * kRecF4 + j];
    __syncthreads();
    const int jd = int(max<int64_t>(0, min<int64_t>(cnt, nd - t0)));
    // direct-form points [0, jd), anchored [jd, cnt); FP32 runs of kSub points
    for (int j0 = 0; j0 < cnt; j0 += kSub) {
      const int j1 = min(j0 + kSub, cnt);
      float T[QPL][kLapAcc];
#pragma unroll
      for (int k = 0; k < QPL; ++k)
#pragma unroll
        for (int c = 0; c < kLapAcc; ++c) T[k][c] = 0.f;
      for (int j = j0; j < min(j1, jd); ++j) {
        const float4 P = tile[j * kRecF4 + 0], U = tile[j * kRecF4 + 1], Mv = tile[j * kRecF4 + 2],
                     K = tile[j * kRecF4 + 3], G = tile[j * kRecF4 + 4];
#pragma unroll
        for (int k = 0; k < QPL; ++k)
          lap_pair<true>(qx[k], qy[k], qz[k], nl[k], S2, ph[k], es[k][0], es[k][1], es[k][2], P, U, Mv, K, G, T[k]);
      }
      for (int j = max(j0, jd); j < j1; ++j) {
        const float4 P = tile[j * kRecF4 + 0], U = tile[j * kRecF4 + 1], Mv = tile[j * kRecF4 + 2],
                     K = tile[j * kRecF4 + 3], G = tile[j * kRecF4 + 4];
#pragma unroll
        for (int k = 0; k < QPL; ++k)
          lap_pair<false>(qx[k], qy[k], qz[k], nl[k], S2, ph[k], es[k][0], es[k][1], es[k][2], P, U, Mv, K, G, T[k]);
      }
#pragma unroll
      for (int k = 0; k < QPL; ++k)
#pragma unroll
        for (int c = 0; c < kLapAcc; ++c) A[k][c] += double(T[k][c]);
    }
  }
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int64_t q = qb * (kBlock * QPL) + k * kBlock + threadIdx.x;
    if (q < Q) {
      double2* o = part + kLapD2 * (int64_t(split) * Q + q);
#pragma unroll
      for (int c = 0; c < kLapD2; ++c) o[c] = make_double2(A[k][2 * c], A[k][2 * c + 1]);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_lap_combine(const double2* __restrict__ part,
                                                        const float* __restrict__ stats, int S, int64_t Q, float C,
                                                        float* __restrict__ lap, float* __restrict__ grad,
                                                        float* __restrict__ eik) {
  const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= Q) return;
  double a[2 * kLapD2];
  for (int c = 0; c < 2 * kLapD2; ++c) a[c] = 0.0;
  for (int s = 0; s < S; ++s) {
    const double2* p = part + kLapD2 * (int64_t(s) * Q + q);
    for (int c = 0; c < kLapD2; ++c) {
      const double2 v = p[c];
      a[2 * c] += v.x;
      a[2 * c + 1] += v.y;
    }
  }
  const float* st = stats + 6 * q;
  const double M = st[0];
  const double es[3] = {st[3], st[4], st[5]};
  const double iw = 1.0 / a[17];
  for (int c = 0; c < kLapAcc; ++c)
    if (c != 17) a[c] *= iw;
  // re-centre the (g - phi) moments on this sweep's phi = phi_fwd + <g - phi_fwd>
  const double dphi = a[18];
  a[8] -= dphi * a[19];
  for (int c = 0; c < 3; ++c) a[9 + c] -= dphi * a[5 + c];
  a[13] -= dphi * a[20];
  a[14] -= dphi * a[15];
  a[16] -= dphi * a[21];
  const double lam = M > 0.0 ? 2.0 * C / M : 0.0;
  const double kap = M > 0.0 ? 2.0 * C / (M * M) : 0.0;
  const double* gA = a + 2;   // <grad g>
  const double* E = a + 5;    // <e>
  const double* B = a + 9;    // <(g - phi) e>
  const double V = a[14], dbar = a[15];
  double gF[3], AE = 0.0, BE = 0.0, Bs = 0.0, Es = 0.0, gFs = 0.0;
  for (int c = 0; c < 3; ++c) {
    gF[c] = gA[c] - lam * B[c];
    AE += gA[c] * E[c];
    BE += B[c] * E[c];
    Bs += B[c] * es[c];
    Es += E[c] * es[c];
    gFs += gF[c] * es[c];
  }
  const double lapF = a[0] - 2.0 * lam * a[1] + 2.0 * lam * AE - 2.0 * lam * a[8] - 2.0 * lam * lam * BE;
  const double gVs = a[12] + Bs - lam * a[13] + lam * V * Es - dbar * gFs;   // grad V . e_*
  const double Fll = a[16] - 2.0 * dbar * V;
  if (lap) lap[q] = float(lapF + 2.0 * kap * gVs + kap * kap * Fll);
  double g2 = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double gc = gF[c] + kap * V * es[c];
    if (grad) grad[3 * q + c] = float(gc);
    g2 += gc * gc;
  }
  if (eik) eik[q] = float(sqrt(g2) - 1.0);
}

template <int QPL>
void launch_lap_sweep(const Header* h, const float4* rec, const float* x, int64_t Q, const Plan& plan,
                      const float* stats, float C, double2* part, hipStream_t st) {
  hipLaunchKernelGGL(k_lap<QPL>, dim3(unsigned(plan.nqb * plan.S)), dim3(kBlock), 0, st, h, rec, x, Q, plan.S,
                     plan.per_split, stats, C * kLog2e, shift2_of(C), part);
}

}  // namespace

size_t lap_ws_bytes(const Plan& plan, int64_t Q) {
  return align256(size_t(plan.S) * size_t(Q) * kLapD2 * sizeof(double2));
}

int launch_lap(const void* rec, int64_t N, const float* x, int64_t Q, const float* stats, float* lap, float* grad,
               float* eik, float C, const Plan& plan, void* ws, hipStream_t st) {
  const Layout L(N);
  const char* base = static_cast<const char*>(rec);
  const Header* h = reinterpret_cast<const Header*>(base);
  const float4* recs = reinterpret_cast<const float4*>(base + L.rec);
  double2* part = static_cast<double2*>(ws);
  const Plan p = with_qpl(plan, 1, Q);
  launch_lap_sweep<1>(h, recs, x, Q, p, stats, C, part, st);
  hipLaunchKernelGGL(k_lap_combine, dim3(unsigned((Q + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, part, stats,
                     plan.S, Q, C, lap, grad, eik);
  return check_hip(hipGetLastError(), "Laplacian kernels");
}

}  // namespace pts
