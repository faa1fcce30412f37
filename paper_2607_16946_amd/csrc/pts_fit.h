// pts_fit.h -- torus fitting of one point (Sec. 4.1), templated on the scalar
// type so that the build kernel runs it on double and the backward sweeps run
// it on forward-mode dual numbers with K tangent directions (the six
// coefficients, and optionally the three components of the normal).  Device
// code only.
#pragma once

#include <hip/hip_runtime.h>

namespace pts {

// Forward-mode dual number with K tangent directions.
template <int K>
struct Dual {
  double v;
  double d[K];
};
template <int K>
__device__ __forceinline__ Dual<K> dual(double v) {
  Dual<K> r;
  r.v = v;
  for (int k = 0; k < K; ++k) r.d[k] = 0.0;
  return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator+(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r; r.v = a.v + b.v; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
template <int K>
__device__ __forceinline__ Dual<K> operator-(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r; r.v = a.v - b.v; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
template <int K>
__device__ __forceinline__ Dual<K> operator-(const Dual<K>& a) {
  Dual<K> r; r.v = -a.v; for (int k = 0; k < K; ++k) r.d[k] = -a.d[k]; return r; }
template <int K>
__device__ __forceinline__ Dual<K> operator*(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r; r.v = a.v * b.v; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
template <int K>
__device__ __forceinline__ Dual<K> operator/(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r; r.v = a.v / b.v;
  const double ib = 1.0 / b.v;
  for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
  return r; }
template <int K>
__device__ __forceinline__ Dual<K> operator+(const Dual<K>& a, double b) { Dual<K> r = a; r.v += b; return r; }
template <int K>
__device__ __forceinline__ Dual<K> operator+(double a, const Dual<K>& b) { return b + a; }
template <int K>
__device__ __forceinline__ Dual<K> operator-(const Dual<K>& a, double b) { Dual<K> r = a; r.v -= b; return r; }
template <int K>
__device__ __forceinline__ Dual<K> operator-(double a, const Dual<K>& b) { return -b + a; }
template <int K>
__device__ __forceinline__ Dual<K> operator*(const Dual<K>& a, double b) {
  Dual<K> r; r.v = a.v * b; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b; return r; }
template <int K>
__device__ __forceinline__ Dual<K> operator*(double a, const Dual<K>& b) { return b * a; }
template <int K>
__device__ __forceinline__ Dual<K> operator/(const Dual<K>& a, double b) { return a * (1.0 / b); }
template <int K>
__device__ __forceinline__ Dual<K> operator/(double a, const Dual<K>& b) { return dual<K>(a) / b; }

__device__ __forceinline__ double val(double x) { return x; }
template <int K>
__device__ __forceinline__ double val(const Dual<K>& x) { return x.v; }
__device__ __forceinline__ double sq_root(double x) { return sqrt(x); }
__device__ __forceinline__ double absval(double x) { return fabs(x); }
// d sqrt at 0 is taken as 0 (umbilic points, where the curvatures are not differentiable)
template <int K>
__device__ __forceinline__ Dual<K> sq_root(const Dual<K>& a) {
  Dual<K> r; r.v = sqrt(a.v);
  const double f = r.v > 0.0 ? 0.5 / r.v : 0.0;
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * f;
  return r; }
template <int K>
__device__ __forceinline__ Dual<K> absval(const Dual<K>& a) { return a.v < 0.0 ? -a : a; }

template <class T> struct Lift;
template <> struct Lift<double> { __device__ static double of(double x) { return x; } };
template <int K> struct Lift<Dual<K>> { __device__ static Dual<K> of(double x) { return dual<K>(x); } };
template <class T> __device__ __forceinline__ T lift(double x) { return Lift<T>::of(x); }

// |kappa| <- max(|kappa|, floor), sign kept, sign(0) = -1
template <class T>
__device__ __forceinline__ T floor_mag(const T& k, double fl) {
  if (fabs(val(k)) >= fl) return k;
  return lift<T>(val(k) > 0.0 ? fl : -fl);
}

template <class T>
struct FitT {
  T c[3], u[3], m[3], k[3], o[3];
  T L, R, r;
  double zeta, sgn;
};

// p, n: point and (not necessarily unit) normal; a = (a00, a01, a10, a11, a02, a20).
template <class T>
__device__ FitT<T> fit_point(const double* p, const T* nin, const T* a, double kfloor) {
  FitT<T> F;
  const T &a00 = a[0], &a01 = a[1], &a10 = a[2], &a11 = a[3], &a02 = a[4], &a20 = a[5];
  // unit normal and the tangent frame (s, t, n): s from the axis e = x-hat
  // unless |n_x| >= 0.9 (then y-hat), with its normal component removed
  const T nl = sq_root(nin[0] * nin[0] + nin[1] * nin[1] + nin[2] * nin[2]);
  const T n[3] = {nin[0] / nl, nin[1] / nl, nin[2] / nl};
  const double ex = fabs(val(n[0])) < 0.9 ? 1.0 : 0.0, ey = 1.0 - ex;
  const T en = ex * n[0] + ey * n[1];
  T s[3] = {ex - en * n[0], ey - en * n[1], -(en * n[2])};
  const T sl = sq_root(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
  for (int i = 0; i < 3; ++i) s[i] = s[i] / sl;
  const T t[3] = {n[1] * s[2] - n[2] * s[1], n[2] * s[0] - n[0] * s[2], n[0] * s[1] - n[1] * s[0]};

  // mean and Gaussian curvature of the height polynomial at (0,0)
  const T E = 1.0 + a10 * a10, G = 1.0 + a01 * a01, Fm = a10 * a01;
  const T A = sq_root(1.0 + a01 * a01 + a10 * a10);
  const T A3 = A * A * A;
  const T H = (a02 * E + a20 * G - a11 * Fm) / A3;
  const T K = (4.0 * a02 * a20 - a11 * a11) / (A3 * A);
  T disc = H * H - K;
  if (val(disc) < 0.0) disc = lift<T>(0.0);
  const T root = sq_root(disc);
  const T kp = H + root, km = H - root;
  const bool plus_is_min = fabs(val(kp)) < fabs(val(km));
  const T kmin = plus_is_min ? kp : km;
  const T kmax = plus_is_min ? km : kp;

  // principal direction of kappa_min: rows of (II - kappa I) w = 0, longer one
  const T r1x = kmin * Fm * A - a11, r1y = 2.0 * a20 - kmin * E * A;
  const T r2x = 2.0 * a02 - kmin * G * A, r2y = kmin * Fm * A - a11;
  const double q1 = val(r1x) * val(r1x) + val(r1y) * val(r1y);
  const double q2 = val(r2x) * val(r2x) + val(r2y) * val(r2y);
  const bool row2 = q2 > q1;
  const T wx = row2 ? r2x : r1x, wy = row2 ? r2y : r1y;
  const double qw = row2 ? q2 : q1;
  const double scale = fabs(val(a11)) + 2.0 * fabs(val(a20)) + 2.0 * fabs(val(a02)) +
                       fabs(val(kmin)) * val(A) * (1.0 + val(a10) * val(a10) + val(a01) * val(a01));
  T v[3];
  if (sqrt(qw) > 1e-12 * scale) {
    for (int i = 0; i < 3; ++i) v[i] = wx * (s[i] + a10 * n[i]) + wy * (t[i] + a01 * n[i]);
    const T vl = sq_root(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int i = 0; i < 3; ++i) v[i] = v[i] / vl;
  } else {  // umbilic: any tangent direction
    for (int i = 0; i < 3; ++i) v[i] = s[i];
  }

  // polynomial normal n*(0,0)
  T ns[3];
  for (int i = 0; i < 3; ++i) ns[i] = (n[i] - a10 * s[i] - a01 * t[i]) / A;

  const T kminf = floor_mag(kmin, kfloor), kmaxf = floor_mag(kmax, kfloor);
  F.L = 1.0 / absval(kminf);
  F.r = 1.0 / absval(kmaxf);
  F.zeta = (val(kminf) * val(kmaxf) > 0.0) ? 1.0 : -1.0;
  F.R = F.L - F.zeta * F.r;
  F.sgn = (val(kmaxf) < 0.0) ? 1.0 : -1.0;

  for (int i = 0; i < 3; ++i) {
    F.o[i] = p[i] + a00 * n[i];
    F.c[i] = F.o[i] + ns[i] / kminf;
  }
  // axis u = n* x v_min (unit), m = (o - c)/L = -sign(kappa_min) n*, k = u x m
  T u[3] = {ns[1] * v[2] - ns[2] * v[1], ns[2] * v[0] - ns[0] * v[2], ns[0] * v[1] - ns[1] * v[0]};
  const T ul = sq_root(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  for (int i = 0; i < 3; ++i) F.u[i] = u[i] / ul;
  const double sm = val(kminf) > 0.0 ? -1.0 : 1.0;
  for (int i = 0; i < 3; ++i) F.m[i] = ns[i] * sm;
  F.k[0] = F.u[1] * F.m[2] - F.u[2] * F.m[1];
  F.k[1] = F.u[2] * F.m[0] - F.u[0] * F.m[2];
  F.k[2] = F.u[0] * F.m[1] - F.u[1] * F.m[0];
  return F;
}

}  // namespace pts
