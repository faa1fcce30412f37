// pts_api.hip -- C ABI entry points of libpts: argument checks, launch plans,
// thread-local error messages.  All device work is in pts_build.hip and
// pts_eval.hip; this file only validates, sizes and dispatches.
#include "pts_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>

namespace pts {

namespace {
thread_local std::string g_last_error;

pts_params resolve(const pts_params* prm) {
  pts_params r;
  r.C = 64.0f;
  r.kfloor_rel = 1e-6f;
  r.splits = 0;
  r.offset = 0.0f;
  if (prm) {
    if (prm->C != 0.0f) r.C = prm->C;
    if (prm->kfloor_rel != 0.0f) r.kfloor_rel = prm->kfloor_rel;
    r.splits = prm->splits;
    r.offset = prm->offset;
  }
  return r;
}

int check_params(const pts_params& p) {
  if (!(p.C > 0.0f && p.C <= kCMax)) return fail(PTS_EINVAL, "C must be in (0, 75]");
  if (!(p.kfloor_rel >= kKfloorRelMin && std::isfinite(p.kfloor_rel)))
    return fail(PTS_EINVAL, "kfloor_rel must be finite and >= 1e-12");
  if (p.splits < 0 || p.splits > 64 || (p.splits & (p.splits - 1)) != 0)
    return fail(PTS_EINVAL, "splits must be 0 or a power of two <= 64");
  if (!std::isfinite(p.offset)) return fail(PTS_EINVAL, "offset must be finite");
  return PTS_OK;
}
}  // namespace

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return PTS_OK;
  return fail(PTS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

Plan make_plan(int64_t N, int64_t Q, const pts_params* prm, int max_auto_splits) {
  Plan p;
  // queries per lane: 4 once there are enough queries to fill the device
  p.qpl = Q >= 4 * 256 * kBlock ? 4 : (Q >= 2 * 64 * kBlock ? 2 : 1);
  if (const char* e = std::getenv("PTS_QPL")) {  // tuning knob: 1, 2, 4 or 8
    const int v = std::atoi(e);
    if (v == 1 || v == 2 || v == 4 || v == 8) p.qpl = v;
  }
  p.nqb = (Q + int64_t(kBlock) * p.qpl - 1) / (int64_t(kBlock) * p.qpl);
  const int64_t tiles = (N + kTile1 - 1) / kTile1;   // farthest-point tiles
  const int64_t gran = (N + kUnit - 1) / kUnit;      // 64-point units: the split granularity
  int S;
  if (prm && prm->splits > 0) {
    S = prm->splits;
  } else {
    // one split per XCD when there are enough points (each split >= 2
    // farthest-point tiles); then, while the grid has fewer than 4096
    // workgroups (16 waves per CU), more splits, down to one 64-point unit
    // each and at most max_auto_splits: a workgroup walks its split serially,
    // so for few queries the split length is the latency (about 0.12 us per
    // point)
    S = 1;
    while (S < 8 && tiles >= int64_t(2) * S * 2) S *= 2;
    // four splits per XCD when one XCD's eighth of the records would not fit
    // its 4 MiB L2: the blend takes an XCD's splits one after the other
    // (split_block), so its resident workgroups share a quarter of that
    if (S == 8 && max_auto_splits >= 32 && N * int64_t(kRecF4 * 16) / 8 > (int64_t(4) << 20)) S = 32;
    while (S < max_auto_splits && p.nqb * S < 4096 && gran >= int64_t(2) * S) S *= 2;
  }
  S = int(std::max<int64_t>(1, std::min<int64_t>(S, gran)));
  p.per_split = (gran + S - 1) / S * kUnit;
  // splits that would start past the last point are dropped; the remaining
  // S * per_split >= N cover every point
  p.S = int((N + p.per_split - 1) / p.per_split);
  return p;
}

}  // namespace pts

using namespace pts;

extern "C" {

int pts_version(void) { return 101; }

const char* pts_last_error(void) { return g_last_error.c_str(); }

int pts_record_bytes(int64_t N, size_t* out_bytes) {
  if (!out_bytes) return fail(PTS_EINVAL, "out_bytes is NULL");
  if (N < 1 || N > (int64_t(1) << 31) - 1) return fail(PTS_EINVAL, "N must be in [1, 2^31)");
  *out_bytes = Layout(N).total;
  return PTS_OK;
}

int pts_cloud_build(const float* p, const float* n, const float* a, int64_t N, const pts_params* prm, void* rec,
                    size_t rec_bytes, void* stream) {
  if (!p || !n || !a || !rec) return fail(PTS_EINVAL, "null pointer");
  if (N < 1 || N > (int64_t(1) << 31) - 1) return fail(PTS_EINVAL, "N must be in [1, 2^31)");
  if (reinterpret_cast<uintptr_t>(rec) % 256 != 0) return fail(PTS_EINVAL, "record buffer must be 256-byte aligned");
  const pts_params P = resolve(prm);
  if (int rc = check_params(P)) return rc;
  const Layout L(N);
  if (rec_bytes < L.total) return fail(PTS_EINVAL, "record buffer too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int rc = launch_build(p, n, a, N, P.kfloor_rel, rec, st)) return rc;
  int32_t status = 0;
  const Header* h = static_cast<const Header*>(rec);
  if (int rc = check_hip(hipMemcpyAsync(&status, &h->status, sizeof(status), hipMemcpyDeviceToHost, st),
                         "read build status"))
    return rc;
  if (int rc = check_hip(hipStreamSynchronize(st), "build")) return rc;
  if (status & kStatusNonFinite) return fail(PTS_EINVAL, "non-finite point, normal or coefficient");
  if (status & kStatusZeroNormal) return fail(PTS_EINVAL, "zero-length normal");
  return PTS_OK;
}

int pts_cloud_info_get(const void* rec, pts_cloud_info* out, void* stream) {
  if (!rec || !out) return fail(PTS_EINVAL, "null pointer");
  Header h;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int rc = check_hip(hipMemcpyAsync(&h, rec, sizeof(h), hipMemcpyDeviceToHost, st), "read header")) return rc;
  if (int rc = check_hip(hipStreamSynchronize(st), "read header")) return rc;
  if (h.magic != kMagic) return fail(PTS_EINVAL, "not a built record");
  std::memset(out, 0, sizeof(*out));
  out->N = h.N;
  out->n_direct = h.n_direct;
  out->n_anchored = h.n_anchored;
  for (int k = 0; k < 3; ++k) { out->bbox_lo[k] = h.lo[k]; out->bbox_hi[k] = h.hi[k]; }
  out->diag = h.diag;
  out->kfloor = h.kfloor;
  out->version = h.version;
  return PTS_OK;
}

int pts_cloud_decode(const void* rec, int64_t N, float* out, void* stream) {
  if (!rec || !out) return fail(PTS_EINVAL, "null pointer");
  if (N < 1) return fail(PTS_EINVAL, "N must be >= 1");
  return launch_decode(rec, N, out, static_cast<hipStream_t>(stream));
}

int pts_radius_prepare(void* rec, int64_t N, const pts_params* prm, void* stream) {
  if (!rec) return fail(PTS_EINVAL, "null pointer");
  if (N < 1) return fail(PTS_EINVAL, "N must be >= 1");
  const pts_params P = resolve(prm);
  if (int rc = check_params(P)) return rc;
  return launch_radius_prepare(rec, N, P.C, static_cast<hipStream_t>(stream));
}

int pts_radius_info_get(const void* rec, pts_radius_info* out, void* stream) {
  if (!rec || !out) return fail(PTS_EINVAL, "null pointer");
  Header h;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int rc = check_hip(hipMemcpyAsync(&h, rec, sizeof(h), hipMemcpyDeviceToHost, st), "read header")) return rc;
  if (int rc = check_hip(hipStreamSynchronize(st), "read header")) return rc;
  if (h.magic != kMagic) return fail(PTS_EINVAL, "not a built record");
  std::memset(out, 0, sizeof(*out));
  out->D = h.rl_D;
  out->lam = h.rl_lambda;
  out->reval = h.rl_reval;
  out->ready = h.rl_ready;
  return PTS_OK;
}

int pts_eval_radius_ws_bytes(int64_t N, int64_t Q, size_t* out_bytes) {
  if (!out_bytes) return fail(PTS_EINVAL, "out_bytes is NULL");
  if (N < 1 || Q < 0) return fail(PTS_EINVAL, "N must be >= 1 and Q >= 0");
  if (Q > (int64_t(1) << 31) - 1) return fail(PTS_EINVAL, "Q must be < 2^31");
  *out_bytes = Q == 0 ? 0 : eval_radius_ws_bytes(Q);
  return PTS_OK;
}

int pts_eval_radius(const void* rec, int64_t N, const float* x, int64_t Q, float* sdf, int32_t* count, void* ws,
                    size_t ws_bytes, void* stream) {
  if (N < 1 || Q < 0) return fail(PTS_EINVAL, "N must be >= 1 and Q >= 0");
  if (Q > (int64_t(1) << 31) - 1) return fail(PTS_EINVAL, "Q must be < 2^31");
  if (Q == 0) return PTS_OK;
  if (!rec || !x || !sdf || !ws) return fail(PTS_EINVAL, "null pointer");
  if (ws_bytes < eval_radius_ws_bytes(Q)) return fail(PTS_EINVAL, "workspace too small");
  return launch_eval_radius(rec, N, x, Q, sdf, count, ws, static_cast<hipStream_t>(stream));
}

int pts_eval_plan(int64_t N, int64_t Q, const pts_params* prm, int* qpl, int* splits, int64_t* per_split) {
  if (!qpl || !splits || !per_split) return fail(PTS_EINVAL, "null pointer");
  if (N < 1 || Q < 1) return fail(PTS_EINVAL, "N and Q must be >= 1");
  const pts_params P = resolve(prm);
  if (int rc = check_params(P)) return rc;
  const Plan plan = make_plan(N, Q, &P, kPlainSplitMax);
  *qpl = plan.qpl;
  *splits = plan.S;
  *per_split = plan.per_split;
  return PTS_OK;
}

int pts_eval_ws_bytes(int64_t N, int64_t Q, const pts_params* prm, size_t* out_bytes) {
  if (!out_bytes) return fail(PTS_EINVAL, "out_bytes is NULL");
  if (N < 1 || Q < 0) return fail(PTS_EINVAL, "N must be >= 1 and Q >= 0");
  const pts_params P = resolve(prm);
  if (int rc = check_params(P)) return rc;
  *out_bytes = Q == 0 ? 0 : eval_ws_bytes(make_plan(N, Q, &P, kPlainSplitMax), Q);
  return PTS_OK;
}

int pts_grad_ws_bytes(int64_t N, int64_t Q, const pts_params* prm, size_t* out_bytes) {
  if (!out_bytes) return fail(PTS_EINVAL, "out_bytes is NULL");
  if (N < 1 || Q < 0) return fail(PTS_EINVAL, "N must be >= 1 and Q >= 0");
  const pts_params P = resolve(prm);
  if (int rc = check_params(P)) return rc;
  *out_bytes = Q == 0 ? 0 : grad_ws_bytes(make_plan(N, Q, &P), Q);
  return PTS_OK;
}

namespace {
// Common checks; on success *plan and *P are set.  need_grad_ws selects the
// workspace size that the call requires.
int eval_checks(int64_t N, int64_t Q, const pts_params* prm, size_t ws_bytes, bool need_grad_ws, Plan* plan,
                pts_params* P, bool plain = false) {
  if (N < 1 || Q < 0) return fail(PTS_EINVAL, "N must be >= 1 and Q >= 0");
  if (Q > (int64_t(1) << 31) - 1) return fail(PTS_EINVAL, "Q must be < 2^31");
  *P = resolve(prm);
  if (int rc = check_params(*P)) return rc;
  if (Q == 0) return PTS_OK;
  *plan = make_plan(N, Q, P, plain ? kPlainSplitMax : kAutoSplitMax);
  const size_t need = need_grad_ws ? grad_ws_bytes(*plan, Q) : eval_ws_bytes(*plan, Q);
  if (ws_bytes < need) return fail(PTS_EINVAL, "workspace too small");
  return PTS_OK;
}
}  // namespace

int pts_eval(const void* rec, int64_t N, const float* x, int64_t Q, float* sdf, float* grad, float* stats,
             const pts_params* prm, void* ws, size_t ws_bytes, void* stream) {
  Plan plan;
  pts_params P;
  if (int rc = eval_checks(N, Q, prm, ws_bytes, grad != nullptr, &plan, &P, !grad && !stats)) return rc;
  if (Q == 0) return PTS_OK;
  if (!rec || !x || !sdf || !ws) return fail(PTS_EINVAL, "null pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const WsView v = ws_view(plan, Q, ws);
  if (!grad && !stats) return launch_eval_plain(rec, N, x, Q, P.C, plan, v, sdf, st, P.offset);
  float* st6 = stats ? stats : v.stats;
  if (int rc = launch_far_arg(rec, N, x, Q, plan, v, st)) return rc;
  if (int rc = launch_blend(rec, N, x, Q, P.C, plan, v, st)) return rc;
  if (int rc = launch_combine_stats(rec, N, x, Q, plan, v, sdf, st6, st, P.offset)) return rc;
  if (grad) return launch_grad(rec, N, x, Q, st6, nullptr, grad, P.C, plan, v, st);
  return PTS_OK;
}

int pts_eval_noalloc(const void* rec, int64_t N, const float* x, int64_t Q, float* sdf, const pts_params* prm,
                     void* stream) {
  if (N < 1 || Q < 0) return fail(PTS_EINVAL, "N must be >= 1 and Q >= 0");
  if (Q > (int64_t(1) << 31) - 1) return fail(PTS_EINVAL, "Q must be < 2^31");
  const pts_params P = resolve(prm);
  if (int rc = check_params(P)) return rc;
  if (Q == 0) return PTS_OK;
  if (!rec || !x || !sdf) return fail(PTS_EINVAL, "null pointer");
  // eval_noalloc refuses a plan whose workspace exceeds the static scratch
  return eval_noalloc(rec, N, x, Q, sdf, P, make_plan(N, Q, &P, kPlainSplitMax), static_cast<hipStream_t>(stream));
}

int pts_eval_far(const void* rec, int64_t N, const float* x, int64_t Q, const pts_params* prm, void* ws,
                 size_t ws_bytes, void* stream) {
  Plan plan;
  pts_params P;
  if (int rc = eval_checks(N, Q, prm, ws_bytes, false, &plan, &P, true)) return rc;
  if (Q == 0) return PTS_OK;
  if (!rec || !x || !ws) return fail(PTS_EINVAL, "null pointer");
  return launch_far(rec, N, x, Q, plan, ws_view(plan, Q, ws), static_cast<hipStream_t>(stream));
}

int pts_eval_blend(const void* rec, int64_t N, const float* x, int64_t Q, const pts_params* prm, void* ws,
                   size_t ws_bytes, void* stream) {
  Plan plan;
  pts_params P;
  if (int rc = eval_checks(N, Q, prm, ws_bytes, false, &plan, &P, true)) return rc;
  if (Q == 0) return PTS_OK;
  if (!rec || !x || !ws) return fail(PTS_EINVAL, "null pointer");
  return launch_blend(rec, N, x, Q, P.C, plan, ws_view(plan, Q, ws), static_cast<hipStream_t>(stream));
}

int pts_eval_combine(int64_t N, int64_t Q, float* sdf, const pts_params* prm, void* ws, size_t ws_bytes,
                     void* stream) {
  Plan plan;
  pts_params P;
  if (int rc = eval_checks(N, Q, prm, ws_bytes, false, &plan, &P, true)) return rc;
  if (Q == 0) return PTS_OK;
  if (!sdf || !ws) return fail(PTS_EINVAL, "null pointer");
  return launch_combine(Q, plan, ws_view(plan, Q, ws), sdf, static_cast<hipStream_t>(stream), P.offset);
}

int pts_eval_bounded_ws_bytes(int64_t N, int64_t Q, const pts_params* prm, size_t* out_bytes) {
  if (!out_bytes) return fail(PTS_EINVAL, "out_bytes is NULL");
  if (N < 1 || Q < 0) return fail(PTS_EINVAL, "N must be >= 1 and Q >= 0");
  const pts_params P = resolve(prm);
  if (int rc = check_params(P)) return rc;
  *out_bytes = Q == 0 ? 0 : bounded_ws_bytes(bounded_plan(N, Q), Q);
  return PTS_OK;
}

int pts_eval_bounded(const void* rec, int64_t N, const float* x, int64_t Q, float eps, float* sdf, float* bound,
                     int32_t* kept, const pts_params* prm, void* ws, size_t ws_bytes, void* stream) {
  if (N < 1 || Q < 0) return fail(PTS_EINVAL, "N must be >= 1 and Q >= 0");
  if (Q > (int64_t(1) << 31) - 1) return fail(PTS_EINVAL, "Q must be < 2^31");
  if (!(eps >= 0.f) || !(eps < 3.0e38f)) return fail(PTS_EINVAL, "eps must be finite and >= 0");
  const pts_params P = resolve(prm);
  if (int rc = check_params(P)) return rc;
  if (Q == 0) return PTS_OK;
  if (!rec || !x || !sdf || !ws) return fail(PTS_EINVAL, "null pointer");
  const Plan plan = bounded_plan(N, Q);
  if (ws_bytes < bounded_ws_bytes(plan, Q)) return fail(PTS_EINVAL, "workspace too small");
  return launch_bounded(rec, N, x, Q, eps, P.C, plan, ws, sdf, bound, kept, static_cast<hipStream_t>(stream),
                        P.offset);
}

int pts_set_areas(void* rec, int64_t N, const float* area, void* stream) {
  if (N < 1) return fail(PTS_EINVAL, "N must be >= 1");
  if (!rec) return fail(PTS_EINVAL, "null record");
  return launch_set_areas(rec, N, area, static_cast<hipStream_t>(stream));
}

int pts_eval_baseline(const void* rec, int64_t N, const float* x, int64_t Q, int kind, float* sdf,
                      const pts_params* prm, void* ws, size_t ws_bytes, void* stream) {
  if (kind != PTS_BASELINE_SSPD && kind != PTS_BASELINE_SHC) return fail(PTS_EINVAL, "unknown baseline kind");
  Plan plan;
  pts_params P;
  if (int rc = eval_checks(N, Q, prm, ws_bytes, false, &plan, &P)) return rc;
  if (Q == 0) return PTS_OK;
  if (!rec || !x || !sdf || !ws) return fail(PTS_EINVAL, "null pointer");
  return launch_baseline(rec, N, x, Q, kind, P.C, plan, ws_view(plan, Q, ws), sdf,
                         static_cast<hipStream_t>(stream), P.offset);
}

int pts_compose(const float* a, const float* b, int64_t n, int op, float c, float* out, void* stream) {
  if (n < 0) return fail(PTS_EINVAL, "n must be >= 0");
  if (op < PTS_OP_OFFSET || op > PTS_OP_SUBTRACT) return fail(PTS_EINVAL, "unknown composition");
  if (!std::isfinite(c)) return fail(PTS_EINVAL, "c must be finite");
  if (n == 0) return PTS_OK;
  if (!a || !out || (op != PTS_OP_OFFSET && !b)) return fail(PTS_EINVAL, "null pointer");
  return launch_compose(a, b, n, op, c, out, static_cast<hipStream_t>(stream));
}

int pts_grad_x(const void* rec, int64_t N, const float* x, int64_t Q, const float* gout, const float* stats,
               float* gx, const pts_params* prm, void* ws, size_t ws_bytes, void* stream) {
  Plan plan;
  pts_params P;
  if (int rc = eval_checks(N, Q, prm, ws_bytes, true, &plan, &P)) return rc;
  if (Q == 0) return PTS_OK;
  if (!rec || !x || !stats || !gx || !ws) return fail(PTS_EINVAL, "null pointer");
  return launch_grad(rec, N, x, Q, stats, gout, gx, P.C, plan, ws_view(plan, Q, ws),
                     static_cast<hipStream_t>(stream));
}

int pts_laplacian_ws_bytes(int64_t N, int64_t Q, const pts_params* prm, size_t* out_bytes) {
  if (!out_bytes) return fail(PTS_EINVAL, "out_bytes is NULL");
  if (N < 1 || Q < 0) return fail(PTS_EINVAL, "N must be >= 1 and Q >= 0");
  const pts_params P = resolve(prm);
  if (int rc = check_params(P)) return rc;
  *out_bytes = Q == 0 ? 0 : lap_ws_bytes(make_plan(N, Q, &P), Q);
  return PTS_OK;
}

int pts_laplacian(const void* rec, int64_t N, const float* x, int64_t Q, const float* stats, float* lap,
                  float* grad, float* eik, const pts_params* prm, void* ws, size_t ws_bytes, void* stream) {
  if (N < 1 || Q < 0) return fail(PTS_EINVAL, "N must be >= 1 and Q >= 0");
  if (Q > (int64_t(1) << 31) - 1) return fail(PTS_EINVAL, "Q must be < 2^31");
  if (!lap && !grad && !eik) return fail(PTS_EINVAL, "no output requested");
  const pts_params P = resolve(prm);
  if (int rc = check_params(P)) return rc;
  if (Q == 0) return PTS_OK;
  if (!rec || !x || !stats || !ws) return fail(PTS_EINVAL, "null pointer");
  const Plan plan = make_plan(N, Q, &P);
  if (ws_bytes < lap_ws_bytes(plan, Q)) return fail(PTS_EINVAL, "workspace too small");
  return launch_lap(rec, N, x, Q, stats, lap, grad, eik, P.C, plan, ws, static_cast<hipStream_t>(stream));
}

int pts_backward_ws_bytes(int64_t N, int64_t Q, const pts_params* prm, size_t* out_bytes) {
  if (!out_bytes) return fail(PTS_EINVAL, "out_bytes is NULL");
  if (N < 1 || Q < 0) return fail(PTS_EINVAL, "N must be >= 1 and Q >= 0");
  const pts_params P = resolve(prm);
  if (int rc = check_params(P)) return rc;
  *out_bytes = back_ws_bytes(N, Q == 0 ? 1 : Q);
  return PTS_OK;
}

int pts_backward_params(const void* rec, int64_t N, const float* p, const float* n, const float* a,
                        const float* x, int64_t Q, const float* gout, const float* stats, float* ga,
                        const pts_params* prm, void* ws, size_t ws_bytes, void* stream) {
  if (N < 1 || Q < 0) return fail(PTS_EINVAL, "N must be >= 1 and Q >= 0");
  if (Q > (int64_t(1) << 31) - 1) return fail(PTS_EINVAL, "Q must be < 2^31");
  if (!rec || !p || !n || !a || !ga || !ws) return fail(PTS_EINVAL, "null pointer");
  if (Q > 0 && (!x || !stats)) return fail(PTS_EINVAL, "null queries or statistics");
  const pts_params P = resolve(prm);
  if (int rc = check_params(P)) return rc;
  if (ws_bytes < back_ws_bytes(N, Q == 0 ? 1 : Q)) return fail(PTS_EINVAL, "workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  return launch_backward(rec, N, p, n, a, x, Q, gout, stats, ga, nullptr, nullptr, P.C, Plan{}, ws, st);
}

int pts_backward_points_ws_bytes(int64_t N, int64_t Q, const pts_params* prm, size_t* out_bytes) {
  if (!out_bytes) return fail(PTS_EINVAL, "out_bytes is NULL");
  if (N < 1 || Q < 0) return fail(PTS_EINVAL, "N must be >= 1 and Q >= 0");
  const pts_params P = resolve(prm);
  if (int rc = check_params(P)) return rc;
  const int64_t Qe = Q == 0 ? 1 : Q;
  const size_t wp = back_points_ws(N, Qe, make_plan(N, Qe, &P), nullptr).bytes;
  const size_t wa = back_ws_bytes(N, Qe);
  *out_bytes = wp > wa ? wp : wa;
  return PTS_OK;
}

int pts_backward_points(const void* rec, int64_t N, const float* p, const float* n, const float* a,
                        const float* x, int64_t Q, const float* gout, const float* stats, float* ga, float* gp,
                        float* gn, const pts_params* prm, void* ws, size_t ws_bytes, void* stream) {
  if (N < 1 || Q < 0) return fail(PTS_EINVAL, "N must be >= 1 and Q >= 0");
  if (Q > (int64_t(1) << 31) - 1) return fail(PTS_EINVAL, "Q must be < 2^31");
  if (!ga && !gp && !gn) return fail(PTS_EINVAL, "no output requested");
  if (!rec || !p || !n || !a || !ws) return fail(PTS_EINVAL, "null pointer");
  if (Q > 0 && (!x || !stats)) return fail(PTS_EINVAL, "null queries or statistics");
  const pts_params P = resolve(prm);
  if (int rc = check_params(P)) return rc;
  const int64_t Qe = Q == 0 ? 1 : Q;
  const Plan plan = make_plan(N, Qe, &P);
  const size_t need = gp ? back_points_ws(N, Qe, plan, nullptr).bytes : back_ws_bytes(N, Qe);
  if (ws_bytes < need) return fail(PTS_EINVAL, "workspace too small");
  return launch_backward(rec, N, p, n, a, x, Q, gout, stats, ga, gp, gn, P.C, plan, ws,
                         static_cast<hipStream_t>(stream));
}

int pts_trace_ws_bytes(int64_t N, int64_t R, const pts_params* prm, size_t* out_bytes) {
  if (!out_bytes) return fail(PTS_EINVAL, "out_bytes is NULL");
  if (N < 1 || R < 0) return fail(PTS_EINVAL, "N must be >= 1 and R >= 0");
  const pts_params P = resolve(prm);
  if (int rc = check_params(P)) return rc;
  *out_bytes = R == 0 ? 0 : trace_ws_bytes(N, R, P);
  return PTS_OK;
}

int pts_trace(const void* rec, int64_t N, const float* origin, const float* dir, int64_t R, int steps, float eps,
              float tmax, float* t_out, float* normal_out, int32_t* hit_out, int32_t* steps_out,
              const pts_params* prm, void* ws, size_t ws_bytes, void* stream) {
  if (N < 1 || R < 0) return fail(PTS_EINVAL, "N must be >= 1 and R >= 0");
  if (R > (int64_t(1) << 31) - 1) return fail(PTS_EINVAL, "R must be < 2^31");
  if (steps < 0) return fail(PTS_EINVAL, "steps must be >= 0");
  if (!(eps >= 0.f) || !(tmax >= 0.f)) return fail(PTS_EINVAL, "eps and tmax must be >= 0");
  if (R == 0) return PTS_OK;
  if (!rec || !origin || !dir || !t_out || !hit_out || !ws) return fail(PTS_EINVAL, "null pointer");
  const pts_params P = resolve(prm);
  if (int rc = check_params(P)) return rc;
  if (ws_bytes < trace_ws_bytes(N, R, P)) return fail(PTS_EINVAL, "workspace too small");
  return launch_trace(rec, N, origin, dir, R, steps, eps, tmax, t_out, normal_out, hit_out, steps_out, P, ws,
                      ws_bytes, static_cast<hipStream_t>(stream));
}

int pts_trace_bounded_ws_bytes(int64_t N, int64_t R, const pts_params* prm, size_t* out_bytes) {
  if (!out_bytes) return fail(PTS_EINVAL, "out_bytes is NULL");
  if (N < 1 || R < 0) return fail(PTS_EINVAL, "N must be >= 1 and R >= 0");
  if (R > (int64_t(1) << 31) - 1) return fail(PTS_EINVAL, "R must be < 2^31");
  const pts_params P = resolve(prm);
  if (int rc = check_params(P)) return rc;
  *out_bytes = R == 0 ? 0 : trace_bounded_ws_bytes(N, R, P);
  return PTS_OK;
}

int pts_trace_bounded(const void* rec, int64_t N, const float* origin, const float* dir, int64_t R, int steps,
                      float eps, float tmax, float eval_eps, float* t_out, float* normal_out, int32_t* hit_out,
                      int32_t* steps_out, const pts_params* prm, void* ws, size_t ws_bytes, void* stream) {
  if (N < 1 || R < 0) return fail(PTS_EINVAL, "N must be >= 1 and R >= 0");
  if (R > (int64_t(1) << 31) - 1) return fail(PTS_EINVAL, "R must be < 2^31");
  if (steps < 0) return fail(PTS_EINVAL, "steps must be >= 0");
  if (!(eps >= 0.f) || !(tmax >= 0.f)) return fail(PTS_EINVAL, "eps and tmax must be >= 0");
  if (!(eval_eps >= 0.f) || !std::isfinite(eval_eps)) return fail(PTS_EINVAL, "eval_eps must be finite and >= 0");
  if (R == 0) return PTS_OK;
  if (!rec || !origin || !dir || !t_out || !hit_out || !ws) return fail(PTS_EINVAL, "null pointer");
  const pts_params P = resolve(prm);
  if (int rc = check_params(P)) return rc;
  if (ws_bytes < trace_bounded_ws_bytes(N, R, P)) return fail(PTS_EINVAL, "workspace too small");
  return launch_trace(rec, N, origin, dir, R, steps, eps, tmax, t_out, normal_out, hit_out, steps_out, P, ws,
                      ws_bytes, static_cast<hipStream_t>(stream), eval_eps);
}

}  // extern "C"
