// pts_build.hip -- precomputation stage of Algorithm 1: one torus per point
// (Sec. 4.1), laid out for the evaluation kernels.
//
// Pipeline (all on `stream`, deterministic):
//   k_init     header defaults
//   k_bbox     bounding box + input validation (order-preserving atomics)
//   k_flags    per point: which torus form the blend kernels use; per-block counts
//   k_scan     exclusive scan of the per-block counts (one workgroup)
//   k_fit      per point: FP64 torus fit, FP32 record written to its slot
//
// Slots: points whose torus radius L = 1/|kappa_min| is at most 4 D (D = bbox
// diagonal) come first, in input order ("direct" form); the rest follow, in
// input order ("anchored" form, which stays accurate in FP32 for very large
// radii).  perm[slot] is the input index.
//
// Record of one point, 5 x float4, coordinates relative to the bbox center:
//   f0 = (p, L)                      L = 1/|kappa_min| (floored)
//   f1 = (u, -<o,u>)                 u = torus axis, o = Q*(0,0) = p + a00 n
//   f2 = (m, -<c,m>) direct form     m = (o - c)/L, unit, in the equatorial plane
//        (m, -<o,m>) anchored form
//   f3 = (k, -<o,k>)                 k = u x m
//   f4 = (R, zeta r, sign, -sign r)  zeta = sign(kappa_+ kappa_-)
// so that, for a query x, <x-c,u> = <x,u> - <o,u>, <x-c,k> = <x,k> - <o,k> and
// <x-c,m> = <x,m> - <c,m> = (<x,m> - <o,m>) + L.

#include "pts_internal.h"
#include "pts_fit.h"

#include <cmath>

namespace pts {
namespace {

__device__ inline uint32_t ordered_bits(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float from_ordered_bits(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__global__ void k_init(Header* h, int64_t N) {
  if (threadIdx.x != 0) return;
  h->magic = kMagic;
  h->version = kRecordVersion;
  h->N = N;
  h->n_direct = 0;
  h->n_anchored = 0;
  for (int k = 0; k < 3; ++k) {
    h->lo_bits[k] = 0xffffffffu;
    h->hi_bits[k] = 0u;
    h->origin[k] = 0.f;
    h->lo[k] = 0.f;
    h->hi[k] = 0.f;
  }
  h->diag = 0.f;
  h->kfloor = 0.f;
  h->lmax_direct = 0.f;
  h->status = 0;
  h->pad0 = 0;
  h->kfloor64 = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_bbox(const float* __restrict__ p, const float* __restrict__ n,
                                                 const float* __restrict__ a, int64_t N, Header* h) {
  __shared__ uint32_t s_lo[3], s_hi[3];
  __shared__ int32_t s_status;
  if (threadIdx.x < 3) { s_lo[threadIdx.x] = 0xffffffffu; s_hi[threadIdx.x] = 0u; }
  if (threadIdx.x == 0) s_status = 0;
  __syncthreads();
  uint32_t lo[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, hi[3] = {0u, 0u, 0u};
  int32_t st = 0;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += int64_t(gridDim.x) * kBlock) {
    float px = p[3 * i], py = p[3 * i + 1], pz = p[3 * i + 2];
    float nx = n[3 * i], ny = n[3 * i + 1], nz = n[3 * i + 2];
    bool finite = isfinite(px) && isfinite(py) && isfinite(pz) && isfinite(nx) && isfinite(ny) && isfinite(nz);
    for (int j = 0; j < 6; ++j) finite = finite && isfinite(a[6 * i + j]);
    if (!finite) { st |= kStatusNonFinite; continue; }
    double nn = double(nx) * nx + double(ny) * ny + double(nz) * nz;
    if (!(nn > 1e-40)) st |= kStatusZeroNormal;
    float c[3] = {px, py, pz};
    for (int k = 0; k < 3; ++k) {
      uint32_t b = ordered_bits(c[k]);
      lo[k] = min(lo[k], b);
      hi[k] = max(hi[k], b);
    }
  }
  for (int k = 0; k < 3; ++k) { atomicMin(&s_lo[k], lo[k]); atomicMax(&s_hi[k], hi[k]); }
  if (st) atomicOr(&s_status, st);
  __syncthreads();
  if (threadIdx.x < 3) {
    atomicMin(&h->lo_bits[threadIdx.x], s_lo[threadIdx.x]);
    atomicMax(&h->hi_bits[threadIdx.x], s_hi[threadIdx.x]);
  }
  if (threadIdx.x == 0 && s_status) atomicOr(&h->status, s_status);
}

// Scalars derived from the bounding box (same for every thread).
struct BoxInfo {
  double lo[3], hi[3], origin[3], diag, kfloor, lmax;
};
__device__ inline BoxInfo box_info(const Header* h, float kfloor_rel) {
  BoxInfo b;
  double s = 0.0;
  for (int k = 0; k < 3; ++k) {
    b.lo[k] = from_ordered_bits(h->lo_bits[k]);
    b.hi[k] = from_ordered_bits(h->hi_bits[k]);
    double e = b.hi[k] - b.lo[k];
    s += e * e;
    b.origin[k] = double(float(0.5 * (b.lo[k] + b.hi[k])));
  }
  b.diag = sqrt(s);
  double D = b.diag > 0.0 ? b.diag : 1.0;
  b.kfloor = double(kfloor_rel) / D;
  b.lmax = kDirectMaxL * D;
  return b;
}

__device__ inline double clampmag(double k, double floor_) { return floor_mag<double>(k, floor_); }

// L = 1/|kappa_min| only (for the form flag); same arithmetic as fit_point.
__device__ inline double radius_L(const float* aa, double kfloor) {
  const double a01 = aa[1], a10 = aa[2], a11 = aa[3], a02 = aa[4], a20 = aa[5];
  const double E = 1.0 + a10 * a10, G = 1.0 + a01 * a01, Fm = a10 * a01;
  const double A = sqrt(1.0 + a01 * a01 + a10 * a10);
  const double H = (a02 * E + a20 * G - a11 * Fm) / (A * A * A);
  const double K = (4.0 * a02 * a20 - a11 * a11) / (A * A * A * A);
  const double root = sqrt(fmax(H * H - K, 0.0));
  const double kp = H + root, km = H - root;
  const double kmin = fabs(kp) < fabs(km) ? kp : km;
  return 1.0 / fabs(clampmag(kmin, kfloor));
}

__global__ __launch_bounds__(kBlock) void k_flags(const float* __restrict__ a, int64_t N, float kfloor_rel,
                                                  Header* h, int32_t* flag, int32_t* blk) {
  const BoxInfo b = box_info(h, kfloor_rel);
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  int direct = 0;
  if (i < N) {
    direct = radius_L(a + 6 * i, b.kfloor) <= b.lmax ? 1 : 0;
    flag[i] = direct;
  }
  int cnt = __syncthreads_count(direct);
  if (threadIdx.x == 0) blk[blockIdx.x] = cnt;
}

// Exclusive scan of nb block counts in place into blk[nb + b]; header totals.
__global__ __launch_bounds__(1024) void k_scan(int32_t* blk, int64_t nb, int64_t N, float kfloor_rel, Header* h) {
  __shared__ int64_t s_part[1024];
  __shared__ int64_t s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += 1024) {
    int64_t i = base + threadIdx.x;
    int64_t v = i < nb ? blk[i] : 0;
    s_part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      int64_t t = threadIdx.x >= off ? s_part[threadIdx.x - off] : 0;
      __syncthreads();
      s_part[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nb) blk[nb + i] = int32_t(s_carry + s_part[threadIdx.x] - v);
    __syncthreads();
    if (threadIdx.x == 1023) s_carry += s_part[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const BoxInfo b = box_info(h, kfloor_rel);
    h->n_direct = s_carry;
    h->n_anchored = N - s_carry;
    for (int k = 0; k < 3; ++k) {
      h->lo[k] = float(b.lo[k]);
      h->hi[k] = float(b.hi[k]);
      h->origin[k] = float(b.origin[k]);
    }
    h->diag = float(b.diag);
    h->kfloor = float(b.kfloor);
    h->kfloor64 = b.kfloor;
    h->lmax_direct = float(b.lmax);
  }
}

__global__ __launch_bounds__(kBlock) void k_fit(const float* __restrict__ p, const float* __restrict__ n,
                                                const float* __restrict__ a, int64_t N, float kfloor_rel,
                                                const Header* __restrict__ h, const int32_t* __restrict__ flag,
                                                const int32_t* __restrict__ blk, int64_t nb,
                                                float4* __restrict__ pos4, float4* __restrict__ rec,
                                                int32_t* __restrict__ perm) {
  __shared__ int32_t s_wave[kBlock / 64];
  const BoxInfo b = box_info(h, kfloor_rel);
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int direct = i < N ? flag[i] : 0;
  // rank of this point among the direct points of its workgroup
  const uint64_t ball = __ballot(direct);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int below = __popcll(ball & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
  if (lane == 0) s_wave[wave] = __popcll(ball);
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wave; ++w) before += s_wave[w];
  if (i >= N) return;
  const int64_t direct_before = int64_t(blk[nb + blockIdx.x]) + before + below;
  const int64_t n_direct = h->n_direct;
  const int64_t slot = direct ? direct_before : n_direct + (i - direct_before);

  double pd[3], nd[3], ad[6];
  for (int k = 0; k < 3; ++k) { pd[k] = p[3 * i + k]; nd[k] = n[3 * i + k]; }
  for (int k = 0; k < 6; ++k) ad[k] = a[6 * i + k];
  const FitT<double> F = fit_point<double>(pd, nd, ad, b.kfloor);
  const double* O = b.origin;
  double pr[3], orel[3], crel[3];
  for (int k = 0; k < 3; ++k) {
    pr[k] = double(p[3 * i + k]) - O[k];
    orel[k] = F.o[k] - O[k];
    crel[k] = F.c[k] - O[k];
  }
  float px = float(pr[0]), py = float(pr[1]), pz = float(pr[2]);
  double pp = double(px) * px + double(py) * py + double(pz) * pz;
  pos4[slot] = make_float4(-2.f * px, -2.f * py, -2.f * pz, float(pp));

  auto dot = [](const double* x, const double* y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; };
  float4* R = rec + slot * kRecF4;
  R[0] = make_float4(px, py, pz, float(F.L));
  R[1] = make_float4(float(F.u[0]), float(F.u[1]), float(F.u[2]), float(-dot(orel, F.u)));
  R[2] = make_float4(float(F.m[0]), float(F.m[1]), float(F.m[2]),
                     float(direct ? -dot(crel, F.m) : -dot(orel, F.m)));
  R[3] = make_float4(float(F.k[0]), float(F.k[1]), float(F.k[2]), float(-dot(orel, F.k)));
  R[4] = make_float4(float(F.R), float(F.zeta * F.r), float(F.sgn), float(-F.sgn * F.r));
  perm[slot] = int32_t(i);
}

// Original-order view of the fitted tori (inspection and tests).
__global__ __launch_bounds__(kBlock) void k_decode(const Header* __restrict__ h, const float4* __restrict__ rec,
                                                   const int32_t* __restrict__ perm, int64_t N, float* out) {
  const int64_t slot = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (slot >= N || slot >= h->N) return;
  const float4* R = rec + slot * kRecF4;
  const float4 f0 = R[0], f1 = R[1], f2 = R[2], f3 = R[3], f4 = R[4];
  const bool direct = slot < h->n_direct;
  // c = o - L m, o from <o,u>, <o,m>, <o,k> in the orthonormal frame (u, m, k)
  const float ou = -f1.w, ok = -f3.w;
  const float om = direct ? (-f2.w + f0.w) : -f2.w;   // direct stores -<c,m> = -<o,m> + L
  const float cm = om - f0.w;
  float c[3];
  c[0] = ou * f1.x + cm * f2.x + ok * f3.x + h->origin[0];
  c[1] = ou * f1.y + cm * f2.y + ok * f3.y + h->origin[1];
  c[2] = ou * f1.z + cm * f2.z + ok * f3.z + h->origin[2];
  float* o = out + int64_t(perm[slot]) * 12;
  o[0] = c[0]; o[1] = c[1]; o[2] = c[2];
  o[3] = f1.x; o[4] = f1.y; o[5] = f1.z;
  o[6] = f4.x;
  o[7] = fabsf(f4.w);
  o[8] = f4.z;
  o[9] = f0.w;
  o[10] = direct ? 0.f : 1.f;
  o[11] = 0.f;
}

}  // namespace

int launch_build(const float* p, const float* n, const float* a, int64_t N, float kfloor_rel, void* rec,
                 hipStream_t st) {
  const Layout L(N);
  char* base = static_cast<char*>(rec);
  Header* h = reinterpret_cast<Header*>(base);
  int32_t* flag = reinterpret_cast<int32_t*>(base + L.flag);
  int32_t* blk = reinterpret_cast<int32_t*>(base + L.blk);
  const unsigned nb = unsigned(L.nblk);
  hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, st, h, N);
  const unsigned gb = unsigned(std::min<int64_t>(L.nblk, 2048));
  hipLaunchKernelGGL(k_bbox, dim3(gb), dim3(kBlock), 0, st, p, n, a, N, h);
  hipLaunchKernelGGL(k_flags, dim3(nb), dim3(kBlock), 0, st, a, N, kfloor_rel, h, flag, blk);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, blk, int64_t(nb), N, kfloor_rel, h);
  hipLaunchKernelGGL(k_fit, dim3(nb), dim3(kBlock), 0, st, p, n, a, N, kfloor_rel, h, flag, blk,
                     int64_t(nb), reinterpret_cast<float4*>(base + L.pos), reinterpret_cast<float4*>(base + L.rec),
                     reinterpret_cast<int32_t*>(base + L.perm));
  return check_hip(hipGetLastError(), "build kernels");
}

int launch_decode(const void* rec, int64_t N, float* out, hipStream_t st) {
  const Layout L(N);
  const char* base = static_cast<const char*>(rec);
  hipLaunchKernelGGL(k_decode, dim3(unsigned(L.nblk)), dim3(kBlock), 0, st, reinterpret_cast<const Header*>(base),
                     reinterpret_cast<const float4*>(base + L.rec), reinterpret_cast<const int32_t*>(base + L.perm),
                     N, out);
  return check_hip(hipGetLastError(), "decode kernel");
}

}  // namespace pts
