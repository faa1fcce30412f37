// pts_build.hip -- precomputation stage of Algorithm 1: one torus per point
// (Sec. 4.1), laid out for the evaluation kernels.
//
// Pipeline (all on `stream`, deterministic):
//   k_init     header defaults
//   k_bbox     bounding box + input validation (order-preserving atomics)
//   k_flags    per point: which torus form the blend kernels use, per-block
//              counts, and the sort key (form bit, then the 24-bit Morton code
//              of the point in a 256^3 grid over the bbox)
//   k_scan     exclusive scan of the per-block counts (one workgroup)
//   k_rhist / k_exscan / k_rscatter
//              stable LSD radix sort of (key, input index), 4 bits per pass
//   k_fit      per slot: FP64 torus fit of its point, FP32 record, and the
//              baseline record (p, 1), (unit normal, -<p, unit normal>)
//   k_units    bounding sphere and extreme point of every kUnit slots
//
// Slots: points whose torus radius L = 1/|kappa_min| is at most 4 D (D = bbox
// diagonal) come first ("direct" form), the rest ("anchored" form, which stays
// accurate in FP32 for very large radii) after; within each group points are
// in Morton order (ties in input order), so consecutive slots are close in
// space and a unit's bounding sphere is small.  perm[slot] is the input index.
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
  h->rl_D = 0.0;
  h->rl_lambda = 0.f;
  h->rl_reval = 0.f;
  h->rl_ready = 0;
  h->rl_shift = 0.f;
  h->a00max_bits = 0u;
  h->pad2 = 0;
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

// Spread the low 8 bits of v to every third bit.
__device__ inline uint32_t spread3(uint32_t v) {
  uint32_t r = 0;
  for (int k = 0; k < 8; ++k) r |= ((v >> k) & 1u) << (3 * k);
  return r;
}

__global__ __launch_bounds__(kBlock) void k_flags(const float* __restrict__ p, const float* __restrict__ a,
                                                  int64_t N, float kfloor_rel, Header* h, int32_t* flag,
                                                  int32_t* blk, uint32_t* key, int32_t* idx) {
  const BoxInfo b = box_info(h, kfloor_rel);
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  int direct = 0;
  if (i < N) {
    direct = radius_L(a + 6 * i, b.kfloor) <= b.lmax ? 1 : 0;
    flag[i] = direct;
    uint32_t m = 0;
    for (int k = 0; k < 3; ++k) {
      const double ext = b.hi[k] - b.lo[k];
      int c = ext > 0.0 ? int((double(p[3 * i + k]) - b.lo[k]) / ext * 256.0) : 0;
      c = c < 0 ? 0 : (c > 255 ? 255 : c);
      m |= spread3(uint32_t(c)) << k;
    }
    key[i] = (direct ? 0u : (1u << 24)) | m;
    idx[i] = int32_t(i);
  }
  int cnt = __syncthreads_count(direct);
  if (threadIdx.x == 0) blk[blockIdx.x] = cnt;
}

// Radix sort blocks: kSortPer chunks of kBlock keys (1024 keys), so that the
// digit-major histogram the scan walks has 16 entries per 1024 keys.
constexpr int kSortPer = 4;
constexpr int64_t kSortBlock = int64_t(kBlock) * kSortPer;

// Radix sort, pass histogram: counts of the 4-bit digit at `shift` in each
// block of kSortBlock keys, digit-major: hist[d * nb + block].
__global__ __launch_bounds__(kBlock) void k_rhist(const uint32_t* __restrict__ key, int64_t N, int shift,
                                                  int32_t* __restrict__ hist, int64_t nb) {
  __shared__ int32_t cnt[1 << kSortBits];
  if (threadIdx.x < (1 << kSortBits)) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t b0 = int64_t(blockIdx.x) * kSortBlock;
#pragma unroll
  for (int j = 0; j < kSortPer; ++j) {
    const int64_t i = b0 + int64_t(j) * kBlock + threadIdx.x;
    if (i < N) atomicAdd(&cnt[(key[i] >> shift) & ((1u << kSortBits) - 1)], 1);
  }
  __syncthreads();
  if (threadIdx.x < (1 << kSortBits)) hist[int64_t(threadIdx.x) * nb + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan of n int32 in place (one workgroup of 1024 threads).  Each
// round covers 8192 values, 8 consecutive ones per thread: the thread's total,
// an inclusive scan of the totals within each wavefront (shuffles), the 16
// wavefront totals through LDS, then the thread writes its 8 prefixes.
__global__ __launch_bounds__(1024) void k_exscan(int32_t* __restrict__ v, int64_t n) {
  constexpr int kPer = 8, kWaves = 1024 / 64;
  __shared__ int32_t wsum[kWaves];
  const int t = int(threadIdx.x), lane = t & 63, w = t >> 6;
  int32_t carry = 0;
  for (int64_t base = 0; base < n; base += int64_t(1024) * kPer) {
    const int64_t i0 = base + int64_t(t) * kPer;
    int32_t x[kPer];
    int32_t tot = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      x[k] = i0 + k < n ? v[i0 + k] : 0;
      tot += x[k];
    }
    int32_t inc = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t y = __shfl_up(inc, o, 64);
      if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
      const int32_t s = wsum[k];
      before += k < w ? s : 0;
      all += s;
    }
    int32_t run = carry + before + inc - tot;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      if (i0 + k < n) v[i0 + k] = run;
      run += x[k];
    }
    carry += all;
    __syncthreads();  // wsum is rewritten in the next round
  }
}

// Radix sort, pass scatter: each key goes to its digit's offset for its block
// plus its rank among the block's keys with the same digit (stable): the
// block's chunks are taken in index order, a key's rank counting the equal
// digits of the earlier chunks, of the earlier waves of its chunk and of the
// earlier lanes of its wave.
__global__ __launch_bounds__(kBlock) void k_rscatter(const uint32_t* __restrict__ kin, const int32_t* __restrict__ iin,
                                                     uint32_t* __restrict__ kout, int32_t* __restrict__ iout,
                                                     int64_t N, int shift, const int32_t* __restrict__ hist,
                                                     int64_t nb) {
  constexpr int kD = 1 << kSortBits;
  __shared__ int32_t wc[kBlock / 64][kD];
  __shared__ int32_t seen[kD];  // digits in the block's earlier chunks
  if (threadIdx.x < kD) seen[threadIdx.x] = 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t b0 = int64_t(blockIdx.x) * kSortBlock;
  for (int j = 0; j < kSortPer; ++j) {
    const int64_t i = b0 + int64_t(j) * kBlock + threadIdx.x;
    const bool valid = i < N;
    const uint32_t k = valid ? kin[i] : 0u;
    const int d = valid ? int((k >> shift) & (kD - 1)) : kD;
    int rank = 0;
    for (int v = 0; v < kD; ++v) {
      const uint64_t m = __ballot(d == v);
      if (lane == 0) wc[wave][v] = __popcll(m);
      if (d == v) rank = __popcll(m & lt);
    }
    __syncthreads();  // wc of this chunk, and seen from the chunks before it
    if (valid) {
      rank += seen[d];
      for (int w = 0; w < wave; ++w) rank += wc[w][d];
      const int64_t dst = int64_t(hist[int64_t(d) * nb + blockIdx.x]) + rank;
      kout[dst] = k;
      iout[dst] = iin[i];
    }
    __syncthreads();  // every read of seen and wc is done
    if (threadIdx.x < kD) {
      int32_t add = 0;
      for (int w = 0; w < kBlock / 64; ++w) add += wc[w][threadIdx.x];
      seen[threadIdx.x] += add;
    }
    __syncthreads();  // seen updated before the next chunk reads it; wc free
  }
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
                                                const Header* __restrict__ h, const int32_t* __restrict__ order,
                                                float4* __restrict__ pos4, float4* __restrict__ rec,
                                                int32_t* __restrict__ perm, float4* __restrict__ bas,
                                                Header* hw) {
  const BoxInfo b = box_info(h, kfloor_rel);
  const int64_t slot = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (slot >= N) return;
  const int64_t i = order[slot];
  const bool direct = slot < h->n_direct;

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
  const double nl = sqrt(nd[0] * nd[0] + nd[1] * nd[1] + nd[2] * nd[2]);
  double nh[3] = {0.0, 0.0, 0.0};
  if (nl > 0.0)
    for (int k = 0; k < 3; ++k) nh[k] = nd[k] / nl;
  // the torus passes through o = p + a00 n, so |g(x)| <= |x - p| + |a00|
  atomicMax(&hw->a00max_bits, __float_as_uint(fabsf(a[6 * i])));
  bas[2 * slot] = make_float4(px, py, pz, 1.f);
  bas[2 * slot + 1] = make_float4(float(nh[0]), float(nh[1]), float(nh[2]), float(-dot(pr, nh)));
}

// Bounds of each unit of kUnit consecutive slots (one wave per unit): center
// c = midpoint of the unit's box, radius r >= max |p - c| (FP64, rounded up),
// and the unit's point e farthest from c (lowest slot among ties); and the
// unit's oriented box (ob), whose first axis is the mean of its points' unit
// normals (each signed to agree with the first point's), the others completing
// an orthonormal frame, with its center and half-extents measured in FP64 from
// the stored FP32 center and axes and rounded up, so that every point lies in
// the box as stored.
__global__ __launch_bounds__(kBlock) void k_units(const float4* __restrict__ pos4, const float4* __restrict__ bas,
                                                  int64_t N, float4* __restrict__ ub, float4* __restrict__ ob) {
  const int64_t u = int64_t(blockIdx.x) * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t nunit = (N + kUnit - 1) / kUnit;
  if (u >= nunit) return;                       // whole wave leaves together
  const int64_t s = u * kUnit + lane;
  const bool valid = s < N;
  float px = 0.f, py = 0.f, pz = 0.f;
  if (valid) {
    const float4 P = pos4[s];
    px = -0.5f * P.x; py = -0.5f * P.y; pz = -0.5f * P.z;   // exact: pos4 holds -2p
  }
  float lo[3] = {valid ? px : 3.0e38f, valid ? py : 3.0e38f, valid ? pz : 3.0e38f};
  float hi[3] = {valid ? px : -3.0e38f, valid ? py : -3.0e38f, valid ? pz : -3.0e38f};
  for (int o = 32; o > 0; o >>= 1)
    for (int k = 0; k < 3; ++k) {
      lo[k] = fminf(lo[k], __shfl_xor(lo[k], o));
      hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], o));
    }
  const float cx = 0.5f * (lo[0] + hi[0]), cy = 0.5f * (lo[1] + hi[1]), cz = 0.5f * (lo[2] + hi[2]);
  const double dx = double(px) - cx, dy = double(py) - cy, dz = double(pz) - cz;
  double d = valid ? sqrt(dx * dx + dy * dy + dz * dz) : -1.0;
  int who = valid ? lane : 64;
  for (int o = 32; o > 0; o >>= 1) {
    const double od = __shfl_xor(d, o);
    const int ow = __shfl_xor(who, o);
    if (od > d || (od == d && ow < who)) { d = od; who = ow; }
  }
  const float ex = __shfl(px, who), ey = __shfl(py, who), ez = __shfl(pz, who);
  if (lane == 0) {
    ub[2 * u] = make_float4(cx, cy, cz, float(d * (1.0 + 1e-6)) + 1e-30f);
    ub[2 * u + 1] = make_float4(ex, ey, ez, 0.f);
  }
  // the oriented box
  float nx = 0.f, ny = 0.f, nz = 0.f;
  if (valid) {
    const float4 B = bas[2 * s + 1];
    nx = B.x; ny = B.y; nz = B.z;
  }
  const float fx = __shfl(nx, 0), fy = __shfl(ny, 0), fz = __shfl(nz, 0);
  const float sg = fx * nx + fy * ny + fz * nz < 0.f ? -1.f : 1.f;
  float m[3] = {sg * nx, sg * ny, sg * nz};
  for (int o = 32; o > 0; o >>= 1)
    for (int k = 0; k < 3; ++k) m[k] += __shfl_xor(m[k], o);
  float ax[3][3];
  const float mn = sqrtf(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
  if (mn > 1e-6f) {
    for (int k = 0; k < 3; ++k) ax[0][k] = m[k] / mn;
  } else {
    ax[0][0] = 0.f; ax[0][1] = 0.f; ax[0][2] = 1.f;
  }
  const float tx = fabsf(ax[0][0]) < 0.9f ? 1.f : 0.f, ty = 1.f - tx;  // (1,0,0) or (0,1,0)
  float c1[3] = {ax[0][1] * 0.f - ax[0][2] * ty, ax[0][2] * tx - ax[0][0] * 0.f, ax[0][0] * ty - ax[0][1] * tx};
  const float cn = sqrtf(c1[0] * c1[0] + c1[1] * c1[1] + c1[2] * c1[2]);
  for (int k = 0; k < 3; ++k) ax[1][k] = c1[k] / cn;
  ax[2][0] = ax[0][1] * ax[1][2] - ax[0][2] * ax[1][1];
  ax[2][1] = ax[0][2] * ax[1][0] - ax[0][0] * ax[1][2];
  ax[2][2] = ax[0][0] * ax[1][1] - ax[0][1] * ax[1][0];
  // center: the midpoint of the extents along the axes
  double plo[3], phi[3];
  for (int k = 0; k < 3; ++k) {
    const double t = double(px) * ax[k][0] + double(py) * ax[k][1] + double(pz) * ax[k][2];
    plo[k] = valid ? t : 1e300;
    phi[k] = valid ? t : -1e300;
  }
  for (int o = 32; o > 0; o >>= 1)
    for (int k = 0; k < 3; ++k) {
      plo[k] = fmin(plo[k], __shfl_xor(plo[k], o));
      phi[k] = fmax(phi[k], __shfl_xor(phi[k], o));
    }
  double cd[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) cd[j] += 0.5 * (plo[k] + phi[k]) * ax[k][j];
  const float bx = float(cd[0]), by = float(cd[1]), bz = float(cd[2]);
  // half-extents about the stored center along the stored axes
  double e[3];
  for (int k = 0; k < 3; ++k) {
    const double t = (double(px) - bx) * ax[k][0] + (double(py) - by) * ax[k][1] + (double(pz) - bz) * ax[k][2];
    e[k] = valid ? fabs(t) : 0.0;
  }
  for (int o = 32; o > 0; o >>= 1)
    for (int k = 0; k < 3; ++k) e[k] = fmax(e[k], __shfl_xor(e[k], o));
  if (lane == 0) {
    ob[4 * u] = make_float4(bx, by, bz, 0.f);
    for (int k = 0; k < 3; ++k)
      ob[4 * u + 1 + k] = make_float4(ax[k][0], ax[k][1], ax[k][2], float(e[k] * (1.0 + 1e-6)) + 1e-30f);
  }
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

int launch_radix_sort(uint32_t* key[2], int32_t* idx[2], int64_t n, int passes, int32_t* rhist, hipStream_t st,
                      int* out) {
  const unsigned nb = unsigned((n + kSortBlock - 1) / kSortBlock);  // callers size rhist for kBlock-key blocks
  int cur = 0;
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = pass * kSortBits;
    hipLaunchKernelGGL(k_rhist, dim3(nb), dim3(kBlock), 0, st, key[cur], n, shift, rhist, int64_t(nb));
    hipLaunchKernelGGL(k_exscan, dim3(1), dim3(1024), 0, st, rhist, int64_t(nb) << kSortBits);
    hipLaunchKernelGGL(k_rscatter, dim3(nb), dim3(kBlock), 0, st, key[cur], idx[cur], key[1 - cur], idx[1 - cur], n,
                       shift, rhist, int64_t(nb));
    cur = 1 - cur;
  }
  *out = cur;
  return check_hip(hipGetLastError(), "radix sort");
}

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
  uint32_t* key[2] = {reinterpret_cast<uint32_t*>(base + L.key),
                      reinterpret_cast<uint32_t*>(base + L.key + align256(size_t(N) * 4))};
  int32_t* idx[2] = {reinterpret_cast<int32_t*>(base + L.idx),
                     reinterpret_cast<int32_t*>(base + L.idx + align256(size_t(N) * 4))};
  int32_t* rhist = reinterpret_cast<int32_t*>(base + L.rhist);
  hipLaunchKernelGGL(k_flags, dim3(nb), dim3(kBlock), 0, st, p, a, N, kfloor_rel, h, flag, blk, key[0], idx[0]);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, blk, int64_t(nb), N, kfloor_rel, h);
  int cur = 0;
  if (int rc = launch_radix_sort(key, idx, N, kSortPasses, rhist, st, &cur)) return rc;
  float4* pos4 = reinterpret_cast<float4*>(base + L.pos);
  hipLaunchKernelGGL(k_fit, dim3(nb), dim3(kBlock), 0, st, p, n, a, N, kfloor_rel, h, idx[cur], pos4,
                     reinterpret_cast<float4*>(base + L.rec), reinterpret_cast<int32_t*>(base + L.perm),
                     reinterpret_cast<float4*>(base + L.base), h);
  hipLaunchKernelGGL(k_units, dim3(unsigned((L.nunit + 3) / 4)), dim3(kBlock), 0, st, pos4,
                     reinterpret_cast<const float4*>(base + L.base), N, reinterpret_cast<float4*>(base + L.ub),
                     reinterpret_cast<float4*>(base + L.ob));
  if (int rc = check_hip(hipGetLastError(), "build kernels")) return rc;
  return launch_blocks(rec, N, st);
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
