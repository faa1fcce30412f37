// pts_oracle.cpp -- plain double-precision reference for the pointwise signed
// distance of "Points as Tori" (Feng, Gkioulekas, Crane; ACM TOG 45(4), 2026).
//
// TEST INFRASTRUCTURE ONLY.  The product library never links, loads or calls
// this file; only the test suite, the smoke check and the CPU-baseline leg of
// the benchmark do.  It shares no code, header, table or constant with the GPU
// path.
//
// Every step follows the paper in its own order and notation:
//   * torus fitting            Sec. 4.1, Eqs. (BivariatePolynomial),
//                              (MeanAndGaussCurvatures), (PrincipalDirections),
//                              (TorusSigns), (SingleTorusSDF); App. C
//   * blended evaluation       Sec. 4.2, Eqs. (BasicFormulaShifted),
//                              (RelationshipBetweenLambdaAndRadius)
//   * sphere tracing           Sec. 5.3 ("Direct visualization")
// There is no blocking, fusion or reordering beyond those definitions.
//
// Derivatives (d phi/dx, d phi/da, d phi/dp, d phi/dn, and the Laplacian of
// phi in x; Sec. 6 and App. D) are not hand-derived here: the same templated
// code is evaluated on forward-mode dual numbers (first derivatives) and
// hyper-dual numbers (exact second derivatives along one coordinate), so they
// are the exact derivatives of what this file computes.  The GPU path
// implements the closed forms of App. D (plus the x-dependence of lambda_x)
// instead.
//
// Readings of the paper where it is silent or inconsistent (kept identical on
// both sides; each is listed in the design notes):
//   R-frame   tangent frame: e = x-hat if |n_x| < 0.9 else y-hat;
//             s = normalize(e - <e,n>n), t = n x s.
//   R-disc    H^2 - K < 0 from rounding is clamped to 0.
//   R-tie     |kappa_+| == |kappa_-|  ->  kappa_min = kappa_-.
//   R-floor   |kappa| <- max(|kappa|, kappa_floor) keeping the sign,
//             sign(0) = -1; kappa_floor is an input (1e-6 / bbox diagonal).
//   R-umbilic principal direction from the longer of the two row solutions of
//             (II - kappa I) w = 0; if both vanish, v_min = s.
//   R-center  c = Q*(0,0) + n*/kappa_min with the signed, floored kappa_min.
//             (The printed c = Q* - sign(T)/|kappa_min| n* is kept as
//             center_mode = 1 for comparison; it disagrees on saddles.)
//   R-lambda  sum over all points with the per-query sigma_x, lambda_x;
//             if max distance is 0 the weights are uniform.
//   R-argmax  lambda_x depends on x through the farthest point; ties go to
//             the lowest index (first maximum).
//
// Radius-limited evaluation (Sec. 4.2, "Acceleration and adaptive lambda"):
//   R-rl-knn  D is the mean over points of the mean distance to their 64
//             nearest *other* points (fewer if N <= 64; D = 1 if N = 1).
//   R-rl-in   "within R_eval" includes distance = R_eval; sigma = R_eval/2,
//             so lambda = C/sigma as in Eq. (RelationshipBetweenLambdaAndRadius).
//   R-rl-fb   the fallback blends the 32 nearest points (the 32 smallest
//             distances, ties to the lower index) with the same lambda and the
//             shift sigma = their smallest distance (phi does not depend on
//             sigma; this keeps the largest weight at 1).

// Baselines of the accuracy comparison (Sec. 5.2, "Signed distance
// accuracy"): smoothed signed planar distance, Eq. (SmoothedSignedPlanarDistance),
// and signed Hopf-Cole distance, Eq. (ScreenedWindingNumber):
//   R-base-lambda  both use the per-query sigma_x = M/2 and lambda_x = C/sigma_x
//             of Eq. (RelationshipBetweenLambdaAndRadius), as the blend does
//             (the equations write sigma_x; lambda is the same heuristic).
//   R-base-A  area weights A_i are an input; absent, A_i = 1 (the library
//             Voronoi areas the paper uses are not computed here).
//   R-base-n  <x - p_i, n_i> uses the normal scaled to unit length.
//   R-shc-zero    a double-layer sum of exactly 0 gives +inf (sign(0) = +1).
//   R-shc-onpoint a query on a point (d_i = 0) gives NaN.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// Forward-mode dual numbers with K tangent directions.
// ---------------------------------------------------------------------------
template <int K>
struct Dual {
  double v;
  double d[K];
  Dual() : v(0.0) { for (int k = 0; k < K; ++k) d[k] = 0.0; }
  Dual(double x) : v(x) { for (int k = 0; k < K; ++k) d[k] = 0.0; }
};

template <int K> inline Dual<K> operator+(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r; r.v = a.v + b.v; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
template <int K> inline Dual<K> operator-(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r; r.v = a.v - b.v; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
template <int K> inline Dual<K> operator-(const Dual<K>& a) {
  Dual<K> r; r.v = -a.v; for (int k = 0; k < K; ++k) r.d[k] = -a.d[k]; return r; }
template <int K> inline Dual<K> operator*(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r; r.v = a.v * b.v; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
template <int K> inline Dual<K> operator/(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r; r.v = a.v / b.v;
  for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
  return r; }
template <int K> inline Dual<K> operator+(const Dual<K>& a, double b) { return a + Dual<K>(b); }
template <int K> inline Dual<K> operator+(double a, const Dual<K>& b) { return Dual<K>(a) + b; }
template <int K> inline Dual<K> operator-(const Dual<K>& a, double b) { return a - Dual<K>(b); }
template <int K> inline Dual<K> operator-(double a, const Dual<K>& b) { return Dual<K>(a) - b; }
template <int K> inline Dual<K> operator*(const Dual<K>& a, double b) { return a * Dual<K>(b); }
template <int K> inline Dual<K> operator*(double a, const Dual<K>& b) { return Dual<K>(a) * b; }
template <int K> inline Dual<K> operator/(const Dual<K>& a, double b) { return a / Dual<K>(b); }
template <int K> inline Dual<K> operator/(double a, const Dual<K>& b) { return Dual<K>(a) / b; }

// Hyper-dual numbers a + b e1 + c e2 + d e1 e2 (e1^2 = e2^2 = 0): with
// b = c = 1 along one coordinate, d is the exact second derivative along it.
struct HD {
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
  HD() = default;
  HD(double v) : a(v) {}
  HD(double a_, double b_, double c_, double d_) : a(a_), b(b_), c(c_), d(d_) {}
};
inline HD operator+(const HD& x, const HD& y) { return HD(x.a + y.a, x.b + y.b, x.c + y.c, x.d + y.d); }
inline HD operator-(const HD& x, const HD& y) { return HD(x.a - y.a, x.b - y.b, x.c - y.c, x.d - y.d); }
inline HD operator-(const HD& x) { return HD(-x.a, -x.b, -x.c, -x.d); }
inline HD operator*(const HD& x, const HD& y) {
  return HD(x.a * y.a, x.a * y.b + x.b * y.a, x.a * y.c + x.c * y.a, x.a * y.d + x.b * y.c + x.c * y.b + x.d * y.a);
}
// f(x) from f(a), f'(a), f''(a)
inline HD chain(const HD& x, double f0, double f1, double f2) {
  return HD(f0, f1 * x.b, f1 * x.c, f1 * x.d + f2 * x.b * x.c);
}
inline HD inv(const HD& y) { const double r = 1.0 / y.a; return chain(y, r, -r * r, 2.0 * r * r * r); }
inline HD operator/(const HD& x, const HD& y) { return x * inv(y); }
inline HD operator+(const HD& x, double y) { return x + HD(y); }
inline HD operator+(double x, const HD& y) { return HD(x) + y; }
inline HD operator-(const HD& x, double y) { return x - HD(y); }
inline HD operator-(double x, const HD& y) { return HD(x) - y; }
inline HD operator*(const HD& x, double y) { return HD(x.a * y, x.b * y, x.c * y, x.d * y); }
inline HD operator*(double x, const HD& y) { return y * x; }
inline HD operator/(const HD& x, double y) { return x * (1.0 / y); }
inline HD operator/(double x, const HD& y) { return HD(x) / y; }
inline double val(const HD& x) { return x.a; }
inline HD Sqrt(const HD& x) {
  if (x.a <= 0.0) return HD(0.0);  // no derivative at 0 (as for the dual numbers)
  const double s = std::sqrt(x.a);
  return chain(x, s, 0.5 / s, -0.25 / (s * x.a));
}
inline HD Exp(const HD& x) { const double e = std::exp(x.a); return chain(x, e, e, e); }
inline HD Abs(const HD& x) { return x.a < 0.0 ? -x : x; }

inline double val(double x) { return x; }
template <int K> inline double val(const Dual<K>& x) { return x.v; }

inline double Sqrt(double x) { return std::sqrt(x); }
inline double Exp(double x) { return std::exp(x); }
inline double Abs(double x) { return std::fabs(x); }
// At 0 the square root has no derivative; 0 is used (a subgradient choice).
template <int K> inline Dual<K> Sqrt(const Dual<K>& a) {
  Dual<K> r; r.v = std::sqrt(a.v);
  for (int k = 0; k < K; ++k) r.d[k] = (r.v > 0.0) ? a.d[k] / (2.0 * r.v) : 0.0;
  return r; }
template <int K> inline Dual<K> Exp(const Dual<K>& a) {
  Dual<K> r; r.v = std::exp(a.v); for (int k = 0; k < K; ++k) r.d[k] = r.v * a.d[k]; return r; }
template <int K> inline Dual<K> Abs(const Dual<K>& a) { return (a.v < 0.0) ? -a : a; }

template <class T> inline T dot3(const T* a, const T* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
template <class T> inline void cross3(const T* a, const T* b, T* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
template <class T> inline T norm3(const T* a) { return Sqrt(dot3(a, a)); }

// ---------------------------------------------------------------------------
// Torus fitted at one point (Sec. 4.1).
// ---------------------------------------------------------------------------
template <class T>
struct Torus {
  T c[3], u[3];       // center, unit axis of revolution
  T R, r;             // major, minor radius
  double sgn;         // sign(T_i), Eq. (TorusSigns)
  // diagnostics
  T kplus, kminus, kmin, kmax, kminf, kmaxf, H, K;
  T nstar[3], vmin[3], o[3];
  int umbilic;
};

// R-frame: the fixed orthonormal basis (s, t, n) at a point.
template <class T>
void local_frame(const T* n_in, T* nh, T* s, T* t) {
  T len = Sqrt(dot3(n_in, n_in));
  for (int k = 0; k < 3; ++k) nh[k] = n_in[k] / len;
  double e[3] = {0.0, 0.0, 0.0};
  if (std::fabs(val(nh[0])) < 0.9) e[0] = 1.0; else e[1] = 1.0;
  T en = e[0] * nh[0] + e[1] * nh[1] + e[2] * nh[2];
  for (int k = 0; k < 3; ++k) s[k] = e[k] - en * nh[k];
  T sl = norm3(s);
  for (int k = 0; k < 3; ++k) s[k] = s[k] / sl;
  cross3(nh, s, t);
}

// R-floor
template <class T> T floor_curvature(const T& k, double kfloor) {
  if (Abs(val(k)) >= kfloor) return k;
  if (val(k) > 0.0) return T(kfloor);
  return T(-kfloor);  // includes sign(0) = -1
}

// Torus fitting of Sec. 4.1 for one point.  a = (a00, a01, a10, a11, a02, a20).
// p, n and a may all carry derivatives (T = double or a dual number).
template <class T>
Torus<T> fit_torus(const T* p, const T* n_in, const T* a, double kfloor, int center_mode) {
  Torus<T> tor;
  const T& a00 = a[0]; const T& a01 = a[1]; const T& a10 = a[2];
  const T& a11 = a[3]; const T& a02 = a[4]; const T& a20 = a[5];
  T nh[3], s[3], t[3];
  local_frame(n_in, nh, s, t);

  // Fundamental forms at (0,0) and Eq. (MeanAndGaussCurvatures).
  T A = Sqrt(1.0 + a01 * a01 + a10 * a10);
  T A3 = A * A * A;
  T A4 = A3 * A;
  T H = (a02 * (1.0 + a10 * a10) + a20 * (1.0 + a01 * a01) - a11 * a10 * a01) / A3;
  T K = (4.0 * a02 * a20 - a11 * a11) / A4;
  T disc = H * H - K;
  if (val(disc) < 0.0) disc = T(0.0);  // R-disc
  T sq = Sqrt(disc);
  T kp = H + sq;
  T km = H - sq;
  tor.H = H; tor.K = K; tor.kplus = kp; tor.kminus = km;

  // kappa_min / kappa_max by magnitude; R-tie.
  T kmin, kmax;
  if (Abs(val(kp)) < Abs(val(km))) { kmin = kp; kmax = km; }
  else { kmin = km; kmax = kp; }
  tor.kmin = kmin; tor.kmax = kmax;

  // Eq. (PrincipalDirections) for kappa_min, both rows of (II - kappa I) w = 0.
  T w1x = kmin * a10 * a01 * A - a11;
  T w1y = 2.0 * a20 - kmin * (1.0 + a10 * a10) * A;
  T w2x = 2.0 * a02 - kmin * (1.0 + a01 * a01) * A;
  T w2y = kmin * a10 * a01 * A - a11;
  double n1 = val(w1x) * val(w1x) + val(w1y) * val(w1y);
  double n2 = val(w2x) * val(w2x) + val(w2y) * val(w2y);
  T wx = w1x, wy = w1y;
  double nw = n1;
  if (n2 > n1) { wx = w2x; wy = w2y; nw = n2; }
  double scale = std::fabs(val(a11)) + 2.0 * std::fabs(val(a20)) + 2.0 * std::fabs(val(a02)) +
                 std::fabs(val(kmin)) * val(A) * (1.0 + val(a10) * val(a10) + val(a01) * val(a01));
  T vmin[3];
  tor.umbilic = 0;
  if (!(std::sqrt(nw) > 1e-12 * scale)) {
    tor.umbilic = 1;  // R-umbilic
    for (int k = 0; k < 3; ++k) vmin[k] = s[k];
  } else {
    T v[3];
    for (int k = 0; k < 3; ++k) v[k] = wx * (s[k] + a10 * nh[k]) + wy * (t[k] + a01 * nh[k]);
    T vl = norm3(v);
    for (int k = 0; k < 3; ++k) vmin[k] = v[k] / vl;
  }

  // Polynomial normal n*(0,0).
  T nstar[3];
  for (int k = 0; k < 3; ++k) nstar[k] = (nh[k] - a10 * s[k] - a01 * t[k]) / A;

  // R-floor, radii, Eq. (TorusSigns).
  T kminf = floor_curvature(kmin, kfloor);
  T kmaxf = floor_curvature(kmax, kfloor);
  tor.kminf = kminf; tor.kmaxf = kmaxf;
  double sgn_prod = (val(kminf) * val(kmaxf) > 0.0) ? 1.0 : -1.0;
  tor.r = 1.0 / Abs(kmaxf);
  tor.R = 1.0 / Abs(kminf) - sgn_prod * tor.r;
  tor.sgn = (val(kmaxf) < 0.0) ? 1.0 : -1.0;

  // Center (R-center) and axis.
  T o[3];
  for (int k = 0; k < 3; ++k) o[k] = p[k] + a00 * nh[k];
  for (int k = 0; k < 3; ++k) {
    if (center_mode == 1) tor.c[k] = o[k] - (tor.sgn / Abs(kminf)) * nstar[k];
    else tor.c[k] = o[k] + nstar[k] / kminf;
  }
  cross3(nstar, vmin, tor.u);
  for (int k = 0; k < 3; ++k) { tor.nstar[k] = nstar[k]; tor.vmin[k] = vmin[k]; tor.o[k] = o[k]; }
  return tor;
}

// Eq. (SingleTorusSDF) and the signed g_i = sign(T_i) phi_T.
template <class T, class X>
auto torus_g(const Torus<T>& tor, const X* x) -> decltype(T() * X()) {
  using V = decltype(T() * X());
  V v[3], cr[3], u[3];
  for (int k = 0; k < 3; ++k) { v[k] = x[k] - tor.c[k]; u[k] = V(0.0) + tor.u[k]; }
  cross3(v, u, cr);
  V rho = norm3(cr);
  V h = dot3(v, u);
  V e = rho - tor.R;
  V q = Sqrt(e * e + h * h);
  return tor.sgn * (q - tor.r);
}

// Stored torus layout (doubles per point).
constexpr int TSTRIDE = 32;

void store_torus(const Torus<double>& t, double* o) {
  for (int k = 0; k < TSTRIDE; ++k) o[k] = 0.0;
  for (int k = 0; k < 3; ++k) { o[k] = t.c[k]; o[3 + k] = t.u[k]; }
  o[6] = t.R; o[7] = t.r; o[8] = t.sgn;
  o[9] = t.kmin; o[10] = t.kmax; o[11] = t.kminf; o[12] = t.kmaxf;
  for (int k = 0; k < 3; ++k) { o[13 + k] = t.nstar[k]; o[16 + k] = t.vmin[k]; o[19 + k] = t.o[k]; }
  o[22] = t.H; o[23] = t.K; o[24] = t.umbilic; o[25] = t.kplus; o[26] = t.kminus;
}

Torus<double> load_torus(const double* o) {
  Torus<double> t{};
  for (int k = 0; k < 3; ++k) { t.c[k] = o[k]; t.u[k] = o[3 + k]; }
  t.R = o[6]; t.r = o[7]; t.sgn = o[8];
  return t;
}

// Eq. (BasicFormulaShifted) with (RelationshipBetweenLambdaAndRadius) at one
// query, templated on the query type so that dual queries give d phi/dx.
template <class X>
X blend_at(int64_t N, const double* P, const std::vector<Torus<double>>& tori, const X* x,
           double C, double* M_out, double* W_out) {
  std::vector<X> d(N);
  int64_t imax = 0;
  for (int64_t i = 0; i < N; ++i) {
    X dv[3];
    for (int k = 0; k < 3; ++k) dv[k] = x[k] - P[3 * i + k];
    d[i] = norm3(dv);
    if (val(d[i]) > val(d[imax])) imax = i;  // R-argmax: first maximum
  }
  // NaN queries: propagate.
  bool bad = false;
  for (int k = 0; k < 3; ++k) if (!std::isfinite(val(x[k]))) bad = true;
  if (bad) { if (M_out) *M_out = NAN; if (W_out) *W_out = NAN; return X(NAN); }
  X M = d[imax];
  X sigma = 0.5 * M;
  X num(0.0), den(0.0);
  if (val(M) == 0.0) {
    for (int64_t i = 0; i < N; ++i) { num = num + torus_g(tori[i], x); den = den + 1.0; }
  } else {
    X lambda = C / sigma;
    for (int64_t i = 0; i < N; ++i) {
      X w = Exp(-lambda * (d[i] - sigma));
      num = num + w * torus_g(tori[i], x);
      den = den + w;
    }
  }
  if (M_out) *M_out = val(M);
  if (W_out) *W_out = val(den);
  return num / den;
}

// Mean distance from point i to its k nearest other points.
double knn_mean_of(int64_t N, const double* P, int64_t i, int k, std::vector<double>& d) {
  d.clear();
  for (int64_t j = 0; j < N; ++j) {
    if (j == i) continue;
    double dv[3];
    for (int c = 0; c < 3; ++c) dv[c] = P[3 * i + c] - P[3 * j + c];
    d.push_back(std::sqrt(dot3(dv, dv)));
  }
  const int64_t kk = std::min<int64_t>(k, (int64_t)d.size());
  std::nth_element(d.begin(), d.begin() + (kk - 1), d.end());
  std::sort(d.begin(), d.begin() + kk);
  double s = 0.0;
  for (int64_t j = 0; j < kk; ++j) s += d[j];
  return s / double(kk);
}

// Radius-limited phi at one query: the points within reval of x, or the kfb
// nearest if there are none.  *count = number blended (negative: fallback).
double blend_radius_at(int64_t N, const double* P, const std::vector<Torus<double>>& tori, const double* x,
                       double lambda, double reval, int kfb, int32_t* count) {
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(x[k])) { *count = 0; return NAN; }
  std::vector<double> d(N);
  for (int64_t i = 0; i < N; ++i) {
    double dv[3];
    for (int k = 0; k < 3; ++k) dv[k] = x[k] - P[3 * i + k];
    d[i] = std::sqrt(dot3(dv, dv));
  }
  double num = 0.0, den = 0.0;
  int64_t nin = 0;
  const double sigma = 0.5 * reval;
  for (int64_t i = 0; i < N; ++i) {
    if (!(d[i] <= reval)) continue;
    const double w = std::exp(-lambda * (d[i] - sigma));
    num += w * torus_g(tori[i], x);
    den += w;
    ++nin;
  }
  if (nin > 0) { *count = int32_t(nin); return num / den; }
  std::vector<int64_t> idx(N);
  for (int64_t i = 0; i < N; ++i) idx[i] = i;
  const int64_t kk = std::min<int64_t>(kfb, N);
  std::partial_sort(idx.begin(), idx.begin() + kk, idx.end(),
                    [&](int64_t a, int64_t b) { return d[a] < d[b] || (d[a] == d[b] && a < b); });
  const double s0 = d[idx[0]];
  for (int64_t j = 0; j < kk; ++j) {
    const int64_t i = idx[j];
    const double w = std::exp(-lambda * (d[i] - s0));
    num += w * torus_g(tori[i], x);
    den += w;
  }
  *count = -int32_t(kk);
  return num / den;
}

int set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  return omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

}  // namespace

extern "C" {

int orc_version(void) { return 1; }

int orc_threads(int nthreads) { return set_threads(nthreads); }

// Length of the diagonal of the axis-aligned bounding box of N points.
double orc_bbox_diag(int64_t N, const double* p) {
  if (N <= 0) return 0.0;
  double lo[3], hi[3];
  for (int k = 0; k < 3; ++k) lo[k] = hi[k] = p[k];
  for (int64_t i = 1; i < N; ++i)
    for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], p[3 * i + k]); hi[k] = std::max(hi[k], p[3 * i + k]); }
  double s = 0.0;
  for (int k = 0; k < 3; ++k) s += (hi[k] - lo[k]) * (hi[k] - lo[k]);
  return std::sqrt(s);
}

// The frame of R-frame for N normals: out is [N, 9] = (s, t, n-hat).
void orc_frame(int64_t N, const double* n, double* out) {
  for (int64_t i = 0; i < N; ++i) local_frame(n + 3 * i, out + 9 * i + 6, out + 9 * i, out + 9 * i + 3);
}

// Torus fitting (Sec. 4.1) for N points; out is [N, 32] (see store_torus).
int orc_fit(int64_t N, const double* p, const double* n, const double* a, double kfloor,
            int center_mode, double* out) {
  for (int64_t i = 0; i < N; ++i) {
    double nl = std::sqrt(n[3 * i] * n[3 * i] + n[3 * i + 1] * n[3 * i + 1] + n[3 * i + 2] * n[3 * i + 2]);
    if (!(nl > 0.0)) return 1;
    Torus<double> t = fit_torus<double>(p + 3 * i, n + 3 * i, a + 6 * i, kfloor, center_mode);
    store_torus(t, out + (size_t)TSTRIDE * i);
  }
  return 0;
}

// g_i(x_q) for all pairs: out is [Q, N].
void orc_torus_g(int64_t N, const double* tor, int64_t Q, const double* x, double* out) {
  std::vector<Torus<double>> tt(N);
  for (int64_t i = 0; i < N; ++i) tt[i] = load_torus(tor + (size_t)TSTRIDE * i);
  for (int64_t q = 0; q < Q; ++q)
    for (int64_t i = 0; i < N; ++i) out[q * N + i] = torus_g(tt[i], x + 3 * q);
}

// phi at Q queries (Eq. BasicFormulaShifted).  grad [Q,3] and stats [Q,3] =
// (max distance M, shifted weight sum W, phi) are optional (NULL).
int orc_eval(int64_t N, const double* p, const double* tor, int64_t Q, const double* x, double C,
             int nthreads, double* phi, double* grad, double* stats) {
  if (N <= 0) return 1;
  set_threads(nthreads);
  std::vector<Torus<double>> tt(N);
  for (int64_t i = 0; i < N; ++i) tt[i] = load_torus(tor + (size_t)TSTRIDE * i);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < Q; ++q) {
    double M, W;
    if (grad) {
      Dual<3> xd[3];
      for (int k = 0; k < 3; ++k) { xd[k] = Dual<3>(x[3 * q + k]); xd[k].d[k] = 1.0; }
      Dual<3> f = blend_at(N, p, tt, xd, C, &M, &W);
      phi[q] = f.v;
      for (int k = 0; k < 3; ++k) grad[3 * q + k] = f.d[k];
    } else {
      phi[q] = blend_at(N, p, tt, x + 3 * q, C, &M, &W);
    }
    if (stats) { stats[3 * q] = M; stats[3 * q + 1] = W; stats[3 * q + 2] = phi[q]; }
  }
  return 0;
}

// dL/da for L = sum_q gout_q phi(x_q): [N, 6].  The weights do not depend on a,
// so d phi_q / d a_i = (w_qi / W_q) d g_i(x_q) / d a_i, with the torus of
// point i refitted on dual coefficients.
int orc_grad_a(int64_t N, const double* p, const double* n, const double* a, double kfloor,
               int center_mode, int64_t Q, const double* x, double C, const double* gout,
               int nthreads, double* ga) {
  if (N <= 0) return 1;
  set_threads(nthreads);
  // Per-query M and W from the definition.
  std::vector<double> M(Q), W(Q);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < Q; ++q) {
    double m = -1.0;
    for (int64_t i = 0; i < N; ++i) {
      double dv[3] = {x[3 * q] - p[3 * i], x[3 * q + 1] - p[3 * i + 1], x[3 * q + 2] - p[3 * i + 2]};
      m = std::max(m, norm3(dv));
    }
    M[q] = m;
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i) {
      double dv[3] = {x[3 * q] - p[3 * i], x[3 * q + 1] - p[3 * i + 1], x[3 * q + 2] - p[3 * i + 2]};
      double di = norm3(dv);
      s += (m == 0.0) ? 1.0 : std::exp(-(C / (0.5 * m)) * (di - 0.5 * m));
    }
    W[q] = s;
  }
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < N; ++i) {
    Dual<6> ad[6];
    for (int j = 0; j < 6; ++j) { ad[j] = Dual<6>(a[6 * i + j]); ad[j].d[j] = 1.0; }
    Dual<6> pd[3], nd[3];
    for (int k = 0; k < 3; ++k) { pd[k] = Dual<6>(p[3 * i + k]); nd[k] = Dual<6>(n[3 * i + k]); }
    Torus<Dual<6>> t = fit_torus<Dual<6>>(pd, nd, ad, kfloor, center_mode);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t q = 0; q < Q; ++q) {
      if (gout[q] == 0.0) continue;
      double dv[3] = {x[3 * q] - p[3 * i], x[3 * q + 1] - p[3 * i + 1], x[3 * q + 2] - p[3 * i + 2]};
      double di = norm3(dv);
      double w = (M[q] == 0.0) ? 1.0 : std::exp(-(C / (0.5 * M[q])) * (di - 0.5 * M[q]));
      Dual<6> g = torus_g(t, x + 3 * q);
      double f = gout[q] * w / W[q];
      for (int j = 0; j < 6; ++j) acc[j] += f * g.d[j];
    }
    for (int j = 0; j < 6; ++j) ga[6 * i + j] = acc[j];
  }
  return 0;
}

// Sphere tracing (Sec. 5.3): march x = o + t d with step phi(x) until
// |phi| < eps (hit), t > tmax (miss) or `steps` evaluations.  Outputs the
// final t, a hit flag, the number of steps taken and, for hits, the unit
// normal grad phi / |grad phi| at the hit point.
int orc_trace(int64_t N, const double* p, const double* tor, int64_t Rn, const double* org,
              const double* dir, int steps, double eps, double tmax, double C, int nthreads,
              double* t_out, int* hit_out, int* nsteps_out, double* normal_out) {
  if (N <= 0) return 1;
  set_threads(nthreads);
  std::vector<Torus<double>> tt(N);
  for (int64_t i = 0; i < N; ++i) tt[i] = load_torus(tor + (size_t)TSTRIDE * i);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t r = 0; r < Rn; ++r) {
    double t = 0.0;
    int hit = 0, k = 0;
    double xq[3];
    for (k = 0; k < steps; ++k) {
      for (int j = 0; j < 3; ++j) xq[j] = org[3 * r + j] + t * dir[3 * r + j];
      double f = blend_at(N, p, tt, xq, C, nullptr, nullptr);
      if (std::fabs(f) < eps) { hit = 1; break; }
      t += f;
      if (t > tmax) break;
    }
    t_out[r] = t;
    hit_out[r] = hit;
    nsteps_out[r] = k;
    for (int j = 0; j < 3; ++j) normal_out[3 * r + j] = 0.0;
    if (hit) {
      Dual<3> xd[3];
      for (int j = 0; j < 3; ++j) { xd[j] = Dual<3>(org[3 * r + j] + t * dir[3 * r + j]); xd[j].d[j] = 1.0; }
      Dual<3> f = blend_at(N, p, tt, xd, C, nullptr, nullptr);
      double gl = std::sqrt(f.d[0] * f.d[0] + f.d[1] * f.d[1] + f.d[2] * f.d[2]);
      if (gl > 0.0) for (int j = 0; j < 3; ++j) normal_out[3 * r + j] = f.d[j] / gl;
    }
  }
  return 0;
}

// Smoothed signed planar distance (kind 0), Eq. (SmoothedSignedPlanarDistance),
// and signed Hopf-Cole distance (kind 1), Eq. (ScreenedWindingNumber), at Q
// queries.  area [N] may be null (A_i = 1).  lam_fixed > 0 replaces lambda_x
// by that constant with sigma = 0 (for the pins only).  raw [Q] (may be null)
// receives the weighted sum itself: the double-layer sum w(x) for kind 1,
// the numerator for kind 0; raw_abs [Q] (may be null) the sum of the absolute
// values of its terms (the scale of its rounding error in lower precision).
int orc_eval_baseline(int64_t N, const double* p, const double* n, const double* area, int64_t Q,
                      const double* x, double C, int kind, double lam_fixed, int nthreads, double* out,
                      double* raw, double* raw_abs) {
  if (N <= 0 || (kind != 0 && kind != 1)) return 1;
  set_threads(nthreads);
  std::vector<double> nh(3 * (size_t)N);
  for (int64_t i = 0; i < N; ++i) {
    const double l = std::sqrt(n[3 * i] * n[3 * i] + n[3 * i + 1] * n[3 * i + 1] + n[3 * i + 2] * n[3 * i + 2]);
    for (int k = 0; k < 3; ++k) nh[3 * i + k] = l > 0.0 ? n[3 * i + k] / l : 0.0;
  }
  const double two_pi = 2.0 * 3.14159265358979323846;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < Q; ++q) {
    const double* xq = x + 3 * q;
    double sigma = 0.0, lam = lam_fixed;
    if (lam_fixed <= 0.0) {
      double M = 0.0;
      for (int64_t i = 0; i < N; ++i) {
        const double dv[3] = {xq[0] - p[3 * i], xq[1] - p[3 * i + 1], xq[2] - p[3 * i + 2]};
        M = std::max(M, norm3(dv));
      }
      sigma = 0.5 * M;
      lam = M > 0.0 ? C / sigma : 0.0;
    }
    double num = 0.0, den = 0.0, nabs = 0.0;
    for (int64_t i = 0; i < N; ++i) {
      const double dv[3] = {xq[0] - p[3 * i], xq[1] - p[3 * i + 1], xq[2] - p[3 * i + 2]};
      const double d = norm3(dv);
      const double A = area ? area[i] : 1.0;
      const double w = A * std::exp(-lam * (d - sigma));
      const double planar = dot3(dv, &nh[3 * i]);
      double term;
      if (kind == 0) {
        term = w * planar;
        den += w;
      } else {
        term = (d > 0.0) ? w * (lam * d + 1.0) * planar / (two_pi * d * d * d) : std::nan("");
      }
      num += term;
      nabs += std::fabs(term);
    }
    if (raw) raw[q] = num;
    if (raw_abs) raw_abs[q] = nabs;
    if (kind == 0) {
      out[q] = num / den;
    } else {
      const double sg = num < 0.0 ? -1.0 : 1.0;
      out[q] = sg * (-std::log(std::fabs(num)) / lam + sigma);
    }
  }
  return 0;
}

// Laplacian of phi at Q queries: the exact sum of second derivatives of
// Eq. (BasicFormulaShifted) with sigma_x, lambda_x moving with x (App. D gives
// the fixed-lambda terms), one hyper-dual evaluation per coordinate.
int orc_laplacian(int64_t N, const double* p, const double* tor, int64_t Q, const double* x, double C,
                  int nthreads, double* lap) {
  if (N <= 0) return 1;
  set_threads(nthreads);
  std::vector<Torus<double>> tt(N);
  for (int64_t i = 0; i < N; ++i) tt[i] = load_torus(tor + (size_t)TSTRIDE * i);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < Q; ++q) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
      HD xh[3];
      for (int c = 0; c < 3; ++c) xh[c] = HD(x[3 * q + c]);
      xh[k].b = 1.0;
      xh[k].c = 1.0;
      s += blend_at(N, p, tt, xh, C, nullptr, nullptr).d;
    }
    lap[q] = s;
  }
  return 0;
}

// dL/da [N,6], dL/dp [N,3], dL/dn [N,3] for L = sum_q gout_q phi(x_q)
// (differentiable representation, Sec. 6): exact forward-mode derivatives of
// phi through each point's torus fit (a, p, n), its weight (p) and, for the
// queries whose farthest point it is, lambda_x = 2C/M (p).  The normal n is
// the input vector (not normalised), as in the fit.
int orc_grad_points(int64_t N, const double* p, const double* n, const double* a, double kfloor,
                    int center_mode, int64_t Q, const double* x, double C, const double* gout, int nthreads,
                    double* ga, double* gp, double* gn) {
  if (N <= 0) return 1;
  set_threads(nthreads);
  std::vector<Torus<double>> tt(N);
  for (int64_t i = 0; i < N; ++i) tt[i] = fit_torus<double>(p + 3 * i, n + 3 * i, a + 6 * i, kfloor, center_mode);
  // per query: M, its first farthest point, W and phi (Eq. BasicFormulaShifted)
  std::vector<double> M(Q), W(Q), PHI(Q);
  std::vector<int64_t> IM(Q);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < Q; ++q) {
    std::vector<double> d(N);
    int64_t im = 0;
    for (int64_t i = 0; i < N; ++i) {
      double dv[3];
      for (int k = 0; k < 3; ++k) dv[k] = x[3 * q + k] - p[3 * i + k];
      d[i] = norm3(dv);
      if (d[i] > d[im]) im = i;
    }
    const double m = d[im];
    double num = 0.0, den = 0.0;
    for (int64_t i = 0; i < N; ++i) {
      const double w = (m == 0.0) ? 1.0 : std::exp(-(C / (0.5 * m)) * (d[i] - 0.5 * m));
      num += w * torus_g(tt[i], x + 3 * q);
      den += w;
    }
    M[q] = m; IM[q] = im; W[q] = den; PHI[q] = num / den;
  }
  using D12 = Dual<12>;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < N; ++i) {
    D12 ad[6], pd[3], nd[3];
    for (int j = 0; j < 6; ++j) { ad[j] = D12(a[6 * i + j]); ad[j].d[j] = 1.0; }
    for (int k = 0; k < 3; ++k) {
      pd[k] = D12(p[3 * i + k]); pd[k].d[6 + k] = 1.0;
      nd[k] = D12(n[3 * i + k]); nd[k].d[9 + k] = 1.0;
    }
    const Torus<D12> t = fit_torus<D12>(pd, nd, ad, kfloor, center_mode);
    double acc[12] = {0};
    for (int64_t q = 0; q < Q; ++q) {
      if (gout[q] == 0.0) continue;
      const double* xq = x + 3 * q;
      D12 dv[3];
      for (int k = 0; k < 3; ++k) dv[k] = xq[k] - pd[k];
      const D12 di = norm3(dv);
      const D12 gi = torus_g(t, xq);
      D12 phi;
      if (M[q] == 0.0) {
        phi = gi / double(N);                      // R-M0: uniform weights (only g_i moves)
      } else if (IM[q] != i) {
        const double sig = 0.5 * M[q], lam = C / sig;
        const D12 wi = Exp(-lam * (di - sig));
        phi = (wi * gi - PHI[q] * wi) / W[q];      // d/dtheta of (num_rest + w g)/(W_rest + w)
      } else {                                     // point i fixes M, hence sigma_x and lambda_x
        const D12 sig = 0.5 * di, lam = C / sig;
        D12 num(0.0), den(0.0);
        for (int64_t j = 0; j < N; ++j) {
          if (j == i) {
            const D12 w = Exp(-lam * (di - sig));
            num = num + w * gi;
            den = den + w;
          } else {
            double dj[3];
            for (int k = 0; k < 3; ++k) dj[k] = xq[k] - p[3 * j + k];
            const D12 w = Exp(-lam * (norm3(dj) - sig));
            num = num + w * torus_g(tt[j], xq);
            den = den + w;
          }
        }
        phi = num / den;
      }
      for (int j = 0; j < 12; ++j) acc[j] += gout[q] * phi.d[j];
    }
    for (int j = 0; j < 6; ++j) ga[6 * i + j] = acc[j];
    for (int k = 0; k < 3; ++k) { gp[3 * i + k] = acc[6 + k]; gn[3 * i + k] = acc[9 + k]; }
  }
  return 0;
}

// D = mean over points of the mean distance to their k nearest other points
// (Sec. 4.2, "Acceleration and adaptive lambda"); 1 if N = 1.
int orc_knn_mean(int64_t N, const double* p, int k, int nthreads, double* out) {
  if (N <= 0 || k <= 0) return 1;
  if (N == 1) { *out = 1.0; return 0; }
  set_threads(nthreads);
  std::vector<double> m(N);
#pragma omp parallel
  {
    std::vector<double> d;
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < N; ++i) m[i] = knn_mean_of(N, p, i, k, d);
  }
  double s = 0.0;
  for (int64_t i = 0; i < N; ++i) s += m[i];
  *out = s / double(N);
  return 0;
}

// Radius-limited phi at Q queries with the constant lambda and radius reval;
// count[q] = points blended (negative: the kfb-nearest fallback; 0: NaN query).
int orc_eval_radius(int64_t N, const double* p, const double* tor, int64_t Q, const double* x, double lambda,
                    double reval, int kfb, int nthreads, double* phi, int32_t* count) {
  if (N <= 0 || kfb <= 0) return 1;
  set_threads(nthreads);
  std::vector<Torus<double>> tt(N);
  for (int64_t i = 0; i < N; ++i) tt[i] = load_torus(tor + (size_t)TSTRIDE * i);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < Q; ++q) phi[q] = blend_radius_at(N, p, tt, x + 3 * q, lambda, reval, kfb, count + q);
  return 0;
}

}  // extern "C"
