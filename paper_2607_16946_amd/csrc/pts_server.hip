// pts_server.hip -- continuous-batching SDF server: resident clouds, packed
// multi-request launches, admission by a device-memory budget, latency
// percentiles.
//
// Threads.  Client threads call the pts_server_* entry points; one scheduler
// thread owns every HIP call made for requests.  Shared state is guarded by
// one mutex; a request's device-side progress fields are touched only by the
// scheduler.
//
// Life of a request.  pts_server_submit validates it, copies its inputs into
// a pinned staging buffer and queues it.  The scheduler admits queued
// requests in arrival order while fewer than max_inflight run and the
// request's device buffers fit the arena (first fit; FIFO, so a large request
// is never overtaken), and uploads their inputs on the upload stream.  Each
// pass it packs runnable work -- admitted query requests first, then the next
// step of every trace request -- up to a quantum of pairs into the
// descriptors of one packed launch (pts_multi.hip) on whichever of the two
// launch streams is idle, so a second launch runs while the first is still on
// the device (launch_batch has the rules).  When a launch's
// end event has fired: query requests copy their results out and finish;
// trace requests take their new active-ray count and are packed again, or,
// once every ray has stopped or the step budget is spent, finish on the
// finishing stream: with normals, the hit rays are compacted and counted
// first (one more event), and the normals are evaluated at those rays only;
// then the results are copied back.
//
// Memory.  One device allocation of hbm_budget_bytes holds everything: cloud
// records, request buffers and the launch descriptors (reserved at creation).
// A request's region returns to the arena only after the device work that
// uses it has completed (observed through an event), so reuse never races.
//
// Determinism.  A query request's point splits are pts_eval's automatic plan
// for its (N, Q), a trace request's those of the tracer (march_splits /
// normal_plan: N only), and a query's sums depend only on the split and the
// tile boundaries, so results are bitwise the same alone or packed with any
// other requests, and equal to pts_eval's (default parameters) for query
// requests and to pts_trace's for trace requests.
//
// Mock mode.  With cfg.mock the scheduler runs unchanged without a device: a
// launch "takes" pairs / mock_pairs_per_s seconds and outputs are a pattern,
// so admission, packing, ordering, cancellation, failures and latency
// accounting are testable on a host without a GPU.
#include "pts_device.h"
#include "pts_multi.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace pts {
namespace {

using Clock = std::chrono::steady_clock;
double now_s() { return std::chrono::duration<double>(Clock::now().time_since_epoch()).count(); }

constexpr int kSlots = 2;  // launches in flight at once
constexpr double kDefaultQuantum = 4e9;  // query x point pairs per packed launch (~4 ms of device time)

// First-fit allocator over byte offsets [0, size) with coalescing.
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) {
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align256(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[*off + bytes] = rest;
      used_ += bytes;
      sizes_[*off] = bytes;
      return true;
    }
    return false;
  }
  void release(size_t off) {
    auto s = sizes_.find(off);
    if (s == sizes_.end()) return;
    size_t bytes = s->second;
    sizes_.erase(s);
    used_ -= bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  size_t size_, used_ = 0;
  std::map<size_t, size_t> free_;   // offset -> length of free runs
  std::map<size_t, size_t> sizes_;  // offset -> length of allocations
};

struct SCloud {
  int64_t N = 0;
  size_t off = 0, bytes = 0;
};

// Byte offsets of a request's buffers inside its arena block.
struct ReqLayout {
  // query requests
  size_t x = 0, out = 0, far2 = 0, part = 0;
  // trace requests (the step sweeps use the normals workspace's far2 / part)
  size_t org = 0, dir = 0, t = 0, hit = 0, nsteps = 0, nrm = 0, act = 0, nxt = 0, keep = 0, blk = 0, off = 0,
         cnt = 0, xq = 0, phi = 0, g = 0, nws = 0;
  size_t total = 0;
};

ReqLayout req_layout(int kind, int64_t n, const Plan& plan, const pts_params& P, int64_t N) {
  ReqLayout L;
  size_t w = 0;
  auto take = [&](size_t b) {
    const size_t o = w;
    w += align256(std::max<size_t>(b, 1));
    return o;
  };
  const size_t sq = size_t(plan.S) * size_t(n);
  if (kind == PTS_REQ_EVAL) {
    L.x = take(size_t(n) * 12);
    L.out = take(size_t(n) * 4);
    L.far2 = take(sq * 4);
    L.part = take(sq * 8);
  } else {
    const size_t nb = size_t((n + kBlock - 1) / kBlock);
    L.org = take(size_t(n) * 12);
    L.dir = take(size_t(n) * 12);
    L.t = take(size_t(n) * 4);
    L.hit = take(size_t(n) * 4);
    L.nsteps = take(size_t(n) * 4);
    L.nrm = take(size_t(n) * 12);
    L.act = take(size_t(n) * 4);
    L.nxt = take(size_t(n) * 4);
    L.keep = take(size_t(n) * 4);
    L.blk = take(nb * 4);
    L.off = take(nb * 4);
    L.cnt = take(4);
    L.xq = take(size_t(n) * 12);
    L.phi = take(size_t(n) * 4);
    L.g = take(size_t(n) * 12);
    L.nws = take(trace_eval_ws_bytes(N, n, P, kMarchSplitCap));
  }
  L.total = w;
  return L;
}

// Pinned staging bytes: inputs, then outputs.
size_t stage_bytes_of(int kind, int64_t n) { return size_t(n) * (kind == PTS_REQ_EVAL ? 16 : 48); }

enum {
  ST_QUEUED = PTS_STATE_QUEUED,
  ST_RUNNING = PTS_STATE_RUNNING,
  ST_DONE = PTS_STATE_DONE,
  ST_FAILED = PTS_STATE_FAILED,
  ST_CANCELLED = PTS_STATE_CANCELLED
};

struct Req {
  uint64_t ticket = 0;
  int waiters = 0;  // threads inside pts_server_wait on this request (release refuses meanwhile)
  pts_request r{};
  int state = ST_QUEUED;
  int status = PTS_OK;
  std::string msg;
  double t_submit = 0;
  // cloud and plan (copied at submit; a cloud cannot be removed under a request)
  size_t cloud_off = 0;
  int64_t N = 0;
  Plan plan{};   // split of query requests and of trace steps
  ReqLayout lay;
  size_t dev_off = 0;
  bool admitted = false;
  bool cancel = false;
  // device progress (scheduler thread only)
  int in_batch = -1;
  int64_t n_active = 0;
  int64_t next_blk = 0;   // first work block of the current evaluation / trace step not yet launched
  int step = 0;
  bool finalizing = false;
  bool fin_hits = false;  // normals asked for: the hit count is on its way to the host
  int final_rc = PTS_OK;
  hipEvent_t fin_ev = nullptr;
  int32_t *act = nullptr, *nxt = nullptr;
  // pinned staging
  char* stage = nullptr;
  size_t stage_cap = 0;
};

struct Batch {
  bool active = false;
  bool whole = false;  // one long request run whole, beyond the quantum
  int rc = PTS_OK;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::vector<Req*> reqs;
  std::vector<int64_t> blk0, blk1;  // each request's chunk of work blocks in this launch
  std::vector<char> last;           // the chunk ends the request's evaluation / trace step
  WorkDesc* h_work = nullptr;
  CombDesc* h_comb = nullptr;
  int32_t* h_counts = nullptr;
  size_t d_work_off = 0, d_comb_off = 0;
  double t_launch = 0, mock_done = 0;
};

// Linear interpolation between order statistics.
double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double idx = p * double(v.size() - 1);
  const size_t i = size_t(idx);
  const double f = idx - double(i);
  return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace

class Server {
 public:
  explicit Server(const pts_server_cfg& cfg) : cfg_(cfg), arena_(cfg.hbm_budget_bytes) {}
  ~Server() { shutdown(); }

  int init() {
    P_.C = cfg_.C > 0 ? cfg_.C : 64.0f;
    P_.kfloor_rel = cfg_.kfloor_rel > 0 ? cfg_.kfloor_rel : 1e-6f;
    P_.splits = 0;
    P_.offset = 0.0f;
    max_work_ = cfg_.max_batch_work;
    max_comb_ = cfg_.max_batch_work;
    quantum_ = cfg_.quantum_pairs > 0 ? cfg_.quantum_pairs : kDefaultQuantum;
    if (!cfg_.mock) {
      if (int rc = check_hip(hipGetDevice(&dev_), "server device")) return rc;
      if (hipMalloc(&base_, cfg_.hbm_budget_bytes) != hipSuccess) {
        base_ = nullptr;
        (void)hipGetLastError();
        return fail(PTS_ENOMEM, "cannot allocate the server budget");
      }
      hipStream_t* ss[] = {&up_stream_, &fin_stream_, &batches_[0].stream, &batches_[1].stream};
      for (hipStream_t* s : ss)
        if (int rc = check_hip(hipStreamCreateWithFlags(s, hipStreamNonBlocking), "server stream")) return rc;
      if (int rc = check_hip(hipEventCreateWithFlags(&up_ev_, hipEventDisableTiming), "server event")) return rc;
      for (auto& b : batches_) {
        if (int rc = check_hip(hipEventCreate(&b.ev0), "server event")) return rc;
        if (int rc = check_hip(hipEventCreate(&b.ev1), "server event")) return rc;
      }
    }
    for (auto& b : batches_) {
      if (!arena_.alloc(size_t(max_work_) * sizeof(WorkDesc), &b.d_work_off) ||
          !arena_.alloc(size_t(max_comb_) * sizeof(CombDesc), &b.d_comb_off))
        return fail(PTS_ENOMEM, "budget too small for the launch descriptors");
      b.h_work = static_cast<WorkDesc*>(host_alloc(size_t(max_work_) * sizeof(WorkDesc)));
      b.h_comb = static_cast<CombDesc*>(host_alloc(size_t(max_comb_) * sizeof(CombDesc)));
      b.h_counts = static_cast<int32_t*>(host_alloc(size_t(cfg_.max_inflight) * sizeof(int32_t)));
      if (!b.h_work || !b.h_comb || !b.h_counts) return fail(PTS_ENOMEM, "pinned descriptor allocation failed");
    }
    reserved_ = arena_.used();
    th_ = std::thread([this] { loop(); });
    started_ = true;
    return PTS_OK;
  }

  int add_cloud(const float* p, const float* n, const float* a, int64_t N, int* id) {
    if (!p || !n || !a || !id) return fail(PTS_EINVAL, "null pointer");
    if (N < 1 || N > (int64_t(1) << 31) - 1) return fail(PTS_EINVAL, "N must be in [1, 2^31)");
    const Layout L(N);
    const size_t in_bytes = align256(size_t(N) * 12) * 2 + align256(size_t(N) * 24);
    size_t off = 0, tmp = 0;
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stopping_) return fail(PTS_ECANCELLED, "server is shutting down");
      if (!arena_.alloc(L.total, &off)) return fail(PTS_EBUDGET, "cloud does not fit the server budget");
      if (!arena_.alloc(in_bytes, &tmp)) {
        arena_.release(off);
        return fail(PTS_EBUDGET, "no room to stage the cloud inputs");
      }
    }
    int rc = PTS_OK;
    if (!cfg_.mock) {
      int old = 0;
      (void)hipGetDevice(&old);
      (void)hipSetDevice(dev_);
      hipStream_t st = nullptr;
      rc = check_hip(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "cloud stream");
      char* d = base_ + tmp;
      float* dp = reinterpret_cast<float*>(d);
      float* dn = reinterpret_cast<float*>(d + align256(size_t(N) * 12));
      float* da = reinterpret_cast<float*>(d + 2 * align256(size_t(N) * 12));
      if (!rc) rc = check_hip(hipMemcpyAsync(dp, p, size_t(N) * 12, hipMemcpyHostToDevice, st), "cloud upload");
      if (!rc) rc = check_hip(hipMemcpyAsync(dn, n, size_t(N) * 12, hipMemcpyHostToDevice, st), "cloud upload");
      if (!rc) rc = check_hip(hipMemcpyAsync(da, a, size_t(N) * 24, hipMemcpyHostToDevice, st), "cloud upload");
      if (!rc) rc = pts_cloud_build(dp, dn, da, N, &P_, base_ + off, L.total, st);
      if (st) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
      }
      (void)hipSetDevice(old);
    }
    std::lock_guard<std::mutex> lk(mu_);
    arena_.release(tmp);
    if (rc) {
      arena_.release(off);
      return rc;
    }
    SCloud c;
    c.N = N;
    c.off = off;
    c.bytes = align256(L.total);
    const int cid = next_cloud_++;
    clouds_[cid] = c;
    resident_ += c.bytes;
    *id = cid;
    return PTS_OK;
  }

  int cloud_plan(int id, int64_t* N, int* splits) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = clouds_.find(id);
    if (it == clouds_.end()) return fail(PTS_ENOTFOUND, "unknown cloud");
    if (N) *N = it->second.N;
    if (splits) *splits = march_splits(it->second.N, kMarchSplitCap);
    return PTS_OK;
  }

  int remove_cloud(int id) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = clouds_.find(id);
    if (it == clouds_.end()) return fail(PTS_ENOTFOUND, "unknown cloud");
    for (auto& kv : reqs_)
      if (kv.second->r.cloud == id && kv.second->state <= ST_RUNNING)
        return fail(PTS_EBUSY, "cloud has queued or running requests");
    arena_.release(it->second.off);
    resident_ -= it->second.bytes;
    clouds_.erase(it);
    return PTS_OK;
  }

  int submit(const pts_request* r, uint64_t* ticket) {
    if (!r || !ticket) return fail(PTS_EINVAL, "null pointer");
    if (r->kind != PTS_REQ_EVAL && r->kind != PTS_REQ_TRACE) return fail(PTS_EINVAL, "unknown request kind");
    if (r->count < 0 || r->count > (int64_t(1) << 31) - 1) return fail(PTS_EINVAL, "count out of range");
    const bool trace = r->kind == PTS_REQ_TRACE;
    if (r->count > 0 && (!r->in0 || !r->out_sdf)) return fail(PTS_EINVAL, "null input or output");
    if (trace && r->count > 0 && (!r->in1 || !r->out_hit)) return fail(PTS_EINVAL, "trace needs dirs and hit output");
    if (trace && (r->steps < 0 || !(r->eps >= 0.f) || !(r->tmax >= 0.f)))
      return fail(PTS_EINVAL, "bad trace parameters");
    auto q = std::make_unique<Req>();
    q->r = *r;
    SCloud c;
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stopping_) return fail(PTS_ECANCELLED, "server is shutting down");
      auto it = clouds_.find(r->cloud);
      if (it == clouds_.end()) return fail(PTS_ENOTFOUND, "unknown cloud");
      c = it->second;
    }
    q->cloud_off = c.off;
    q->N = c.N;
    const int64_t n = r->count;
    if (n > 0) {
      // query requests: pts_eval's own plan (its results bit for bit), or, if
      // one launch cannot hold the workgroups of one block of queries, the
      // largest power-of-two split <= 64 that fits (pts_eval with
      // pts_params.splits set to it); trace requests: the march's split, a
      // function of N only.  Launches take a request in chunks of blocks.
      const int64_t bq = int64_t(kBlock) * multi_qpl();
      auto fits = [&](const Plan& pl) {
        return pl.S <= max_work_ && (bq + comb_per(pl.S, n) - 1) / comb_per(pl.S, n) <= max_comb_;
      };
      if (r->kind == PTS_REQ_EVAL) {
        q->plan = make_plan(c.N, n, &P_, kPlainSplitMax);
        for (int cap = kAutoSplitMax; cap >= 1 && !fits(q->plan); cap /= 2) {
          pts_params F = P_;
          F.splits = cap;
          q->plan = make_plan(c.N, n, &F);
        }
      } else {
        q->plan = march_plan(c.N, n, P_, kMarchSplitCap);
      }
      if (!fits(q->plan)) {
        std::lock_guard<std::mutex> lk(mu_);
        ++rejected_;
        return fail(PTS_EINVAL, "one block of the request needs more workgroups than a launch holds");
      }
      q->lay = req_layout(r->kind, n, q->plan, P_, c.N);
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (n > 0 && align256(q->lay.total) > arena_.size() - reserved_ - resident_) {
        ++rejected_;
        return fail(PTS_EBUDGET, "request can never fit next to the resident clouds");
      }
      if (int64_t(pending_.size()) >= cfg_.max_queue) {
        ++rejected_;
        return fail(PTS_EBUSY, "queue full");
      }
      if (n > 0) q->stage = stage_get_locked(stage_bytes_of(r->kind, n), &q->stage_cap);
    }
    if (n > 0 && !q->stage) return fail(PTS_ENOMEM, "pinned staging allocation failed");
    if (n > 0) {  // inputs are the server's from here on
      std::memcpy(q->stage, r->in0, size_t(n) * 12);
      if (trace) std::memcpy(q->stage + size_t(n) * 12, r->in1, size_t(n) * 12);
    }
    std::lock_guard<std::mutex> lk(mu_);
    if (stopping_ || !clouds_.count(r->cloud)) {  // cloud ids are never reused
      stage_put_locked(q->stage, q->stage_cap);
      return stopping_ ? fail(PTS_ECANCELLED, "server is shutting down") : fail(PTS_ENOTFOUND, "unknown cloud");
    }
    q->ticket = next_ticket_++;
    q->t_submit = now_s();
    *ticket = q->ticket;
    ++submitted_;
    Req* raw = q.get();
    reqs_[q->ticket] = std::move(q);
    if (n == 0) {
      finish_locked(raw, ST_DONE, PTS_OK, nullptr);
      return PTS_OK;
    }
    pending_.push_back(raw);
    cv_.notify_all();
    return PTS_OK;
  }

  int poll(uint64_t t, int* state) {
    if (!state) return fail(PTS_EINVAL, "null pointer");
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(t);
    if (it == reqs_.end()) return fail(PTS_ENOTFOUND, "unknown ticket");
    *state = it->second->state;
    return PTS_OK;
  }

  int wait(uint64_t t, int timeout_ms) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = reqs_.find(t);
    if (it == reqs_.end()) return fail(PTS_ENOTFOUND, "unknown ticket");
    Req* q = it->second.get();
    auto done = [q] { return q->state >= ST_DONE; };
    ++waiters_;  // shutdown waits for waiters to leave before the server is freed
    ++q->waiters;  // and release() for this request's waiters, so q stays valid
    bool ok = true;
    if (timeout_ms < 0) cv_done_.wait(lk, done);
    else ok = cv_done_.wait_for(lk, std::chrono::milliseconds(timeout_ms), done);
    --q->waiters;
    --waiters_;
    cv_done_.notify_all();
    if (!ok) return fail(PTS_ETIMEOUT, "request still queued or running");
    if (q->state == ST_DONE) return PTS_OK;
    return fail(q->status, q->msg);
  }

  int cancel(uint64_t t) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(t);
    if (it == reqs_.end()) return fail(PTS_ENOTFOUND, "unknown ticket");
    Req* q = it->second.get();
    if (q->state == ST_QUEUED) {
      pending_.erase(std::remove(pending_.begin(), pending_.end(), q), pending_.end());
      stage_put_locked(q->stage, q->stage_cap);
      q->stage = nullptr;
      finish_locked(q, ST_CANCELLED, PTS_ECANCELLED, "cancelled while queued");
    } else if (q->state == ST_RUNNING) {
      q->cancel = true;  // finishes once its device work in flight has completed
    }
    return PTS_OK;
  }

  int release(uint64_t t) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(t);
    if (it == reqs_.end()) return fail(PTS_ENOTFOUND, "unknown ticket");
    if (it->second->state < ST_DONE) return fail(PTS_EBUSY, "request has not finished");
    if (it->second->waiters > 0) return fail(PTS_EBUSY, "another thread is waiting on the request");
    reqs_.erase(it);
    return PTS_OK;
  }

  int get_stats(pts_server_stats* s) {
    if (!s) return fail(PTS_EINVAL, "null pointer");
    std::lock_guard<std::mutex> lk(mu_);
    std::memset(s, 0, sizeof(*s));
    s->submitted = submitted_;
    s->completed = completed_;
    s->failed = failed_;
    s->cancelled = cancelled_;
    s->rejected = rejected_;
    s->launches = launches_;
    s->overlapped_launches = overlapped_;
    s->max_batch_requests = max_batch_reqs_;
    s->pairs = pairs_;
    s->busy_s = busy_s_;
    s->p50_ms = 1e3 * percentile(lat_all_, 0.5);
    s->p99_ms = 1e3 * percentile(lat_all_, 0.99);
    s->max_ms = lat_all_.empty() ? 0.0 : 1e3 * *std::max_element(lat_all_.begin(), lat_all_.end());
    s->p50_eval_ms = 1e3 * percentile(lat_eval_, 0.5);
    s->p99_eval_ms = 1e3 * percentile(lat_eval_, 0.99);
    s->p50_trace_ms = 1e3 * percentile(lat_trace_, 0.5);
    s->p99_trace_ms = 1e3 * percentile(lat_trace_, 0.99);
    s->bytes_resident = resident_;
    s->bytes_reserved = reserved_;
    s->bytes_inflight = arena_.used() - resident_ - reserved_;
    s->inflight = int(running_.size());
    s->queued = int(pending_.size());
    return PTS_OK;
  }

  int reset_stats() {
    std::lock_guard<std::mutex> lk(mu_);
    submitted_ = completed_ = failed_ = cancelled_ = rejected_ = launches_ = overlapped_ = 0;
    max_batch_reqs_ = 0;
    pairs_ = busy_s_ = 0;
    lat_all_.clear();
    lat_eval_.clear();
    lat_trace_.clear();
    return PTS_OK;
  }

  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (shut_) return;
      shut_ = true;
      stopping_ = true;
      for (Req* q : pending_) {
        stage_put_locked(q->stage, q->stage_cap);
        q->stage = nullptr;
        finish_locked(q, ST_CANCELLED, PTS_ECANCELLED, "server destroyed");
      }
      pending_.clear();
      for (Req* q : running_) q->cancel = true;
      cv_.notify_all();
    }
    if (started_ && th_.joinable()) th_.join();
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_done_.wait(lk, [this] { return waiters_ == 0; });
    }
    if (!cfg_.mock) {
      hipStream_t ss[] = {up_stream_, fin_stream_, batches_[0].stream, batches_[1].stream};
      for (hipStream_t s : ss)
        if (s) (void)hipStreamSynchronize(s);
      for (auto& b : batches_) {
        if (b.ev0) (void)hipEventDestroy(b.ev0);
        if (b.ev1) (void)hipEventDestroy(b.ev1);
      }
      if (up_ev_) (void)hipEventDestroy(up_ev_);
      for (hipStream_t s : ss)
        if (s) (void)hipStreamDestroy(s);
    }
    for (auto& b : batches_) {
      host_free(b.h_work);
      host_free(b.h_comb);
      host_free(b.h_counts);
      b.h_work = nullptr;
      b.h_comb = nullptr;
      b.h_counts = nullptr;
    }
    for (auto& kv : pool_)
      for (char* p : kv.second) host_free(p);
    pool_.clear();
    if (base_) (void)hipFree(base_);
    base_ = nullptr;
  }

 private:
  // ---------------- host memory
  void* host_alloc(size_t bytes) {
    if (cfg_.mock) return std::malloc(bytes);
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  void host_free(void* p) {
    if (!p) return;
    if (cfg_.mock) std::free(p);
    else (void)hipHostFree(p);
  }
  // Pinned staging buffers pooled by power-of-two size (mu_ held).
  char* stage_get_locked(size_t bytes, size_t* cap) {
    size_t c = 4096;
    while (c < bytes) c <<= 1;
    *cap = c;
    auto& v = pool_[c];
    if (!v.empty()) {
      char* p = v.back();
      v.pop_back();
      return p;
    }
    return static_cast<char*>(host_alloc(c));
  }
  void stage_put_locked(char* p, size_t cap) {
    if (p) pool_[cap].push_back(p);
  }

  template <class T>
  T* dev(const Req* q, size_t off) const {
    return cfg_.mock ? nullptr : reinterpret_cast<T*>(base_ + q->dev_off + off);
  }

  // ---------------- state changes (mu_ held)
  void finish_locked(Req* q, int state, int status, const char* msg) {
    q->state = state;
    q->status = status;
    if (msg) q->msg = msg;
    if (state == ST_DONE) {
      ++completed_;
      const double l = now_s() - q->t_submit;
      lat_all_.push_back(l);
      (q->r.kind == PTS_REQ_EVAL ? lat_eval_ : lat_trace_).push_back(l);
    } else if (state == ST_CANCELLED) {
      ++cancelled_;
    } else {
      ++failed_;
    }
    cv_done_.notify_all();
  }

  // Return a finished request's device block and staging (its device work
  // has completed).
  void free_req_locked(Req* q) {
    if (q->admitted) arena_.release(q->dev_off);
    q->admitted = false;
    stage_put_locked(q->stage, q->stage_cap);
    q->stage = nullptr;
    running_.erase(std::remove(running_.begin(), running_.end(), q), running_.end());
  }

  // Admit queued requests in order while a slot is free and memory fits.
  void admit_locked(bool device_idle) {
    while (!pending_.empty() && int(running_.size()) < cfg_.max_inflight) {
      Req* q = pending_.front();
      size_t off = 0;
      if (!arena_.alloc(q->lay.total, &off)) {
        if (running_.empty() && device_idle) {  // nothing will free memory: it can never run
          pending_.pop_front();
          stage_put_locked(q->stage, q->stage_cap);
          q->stage = nullptr;
          finish_locked(q, ST_FAILED, PTS_EBUDGET, "request does not fit next to the resident clouds");
          continue;
        }
        break;  // FIFO: later requests wait too
      }
      pending_.pop_front();
      q->dev_off = off;
      q->admitted = true;
      q->state = ST_RUNNING;
      q->n_active = q->r.count;
      q->next_blk = 0;
      q->step = 0;
      running_.push_back(q);
      fresh_.push_back(q);
    }
  }

  // ---------------- the scheduler
  void loop() {
    if (!cfg_.mock) (void)hipSetDevice(dev_);
    for (;;) {
      std::vector<Req*> fresh;
      {
        std::unique_lock<std::mutex> lk(mu_);
        const bool dev_idle = !batches_[0].active && !batches_[1].active && finals_.empty();
        admit_locked(dev_idle);
        fresh.swap(fresh_);
        const bool idle = fresh.empty() && running_.empty() && pending_.empty() && dev_idle;
        if (idle && stopping_) break;
        if (idle) {
          cv_.wait_for(lk, std::chrono::milliseconds(5));
          continue;
        }
      }
      upload(fresh);
      bool progressed = !fresh.empty();
      progressed |= complete_batches();
      progressed |= complete_finals();
      progressed |= launch_batch();
      if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }

  // Upload newly admitted requests' inputs; later launches wait for them.
  void upload(const std::vector<Req*>& fresh) {
    if (fresh.empty()) return;
    if (!cfg_.mock) {
      for (Req* q : fresh) {
        const int64_t n = q->r.count;
        int rc = PTS_OK;
        if (q->r.kind == PTS_REQ_EVAL) {
          rc = check_hip(hipMemcpyAsync(dev<float>(q, q->lay.x), q->stage, size_t(n) * 12, hipMemcpyHostToDevice,
                                        up_stream_),
                         "request upload");
        } else {
          rc = check_hip(hipMemcpyAsync(dev<float>(q, q->lay.org), q->stage, size_t(n) * 12, hipMemcpyHostToDevice,
                                        up_stream_),
                         "request upload");
          if (!rc)
            rc = check_hip(hipMemcpyAsync(dev<float>(q, q->lay.dir), q->stage + size_t(n) * 12, size_t(n) * 12,
                                          hipMemcpyHostToDevice, up_stream_),
                           "request upload");
          if (!rc)
            rc = trace_init(n, q->r.steps, dev<float>(q, q->lay.t), dev<int32_t>(q, q->lay.hit),
                            dev<int32_t>(q, q->lay.nsteps), dev<int32_t>(q, q->lay.act), dev<float>(q, q->lay.nrm),
                            up_stream_);
          q->act = dev<int32_t>(q, q->lay.act);
          q->nxt = dev<int32_t>(q, q->lay.nxt);
        }
        if (rc) q->final_rc = rc;
      }
      (void)hipEventRecord(up_ev_, up_stream_);
      hipStream_t ss[] = {batches_[0].stream, batches_[1].stream, fin_stream_};
      for (hipStream_t s : ss) (void)hipStreamWaitEvent(s, up_ev_, 0);
    }
    std::lock_guard<std::mutex> lk(mu_);
    for (Req* q : fresh) {
      if (q->final_rc) {
        if (!cfg_.mock) (void)hipStreamSynchronize(up_stream_);  // the upload may still read the staging
        finish_locked(q, ST_FAILED, q->final_rc, "request upload failed");
        free_req_locked(q);
      } else if (q->r.kind == PTS_REQ_TRACE && q->r.steps == 0) {
        q->n_active = 0;
        start_final_locked(q);
      }
    }
  }

  bool batch_done(Batch& b) {
    if (cfg_.mock || b.rc != PTS_OK) return cfg_.mock ? now_s() >= b.mock_done : true;
    const hipError_t e = hipEventQuery(b.ev1);
    if (e == hipErrorNotReady) return false;
    if (e != hipSuccess) b.rc = check_hip(e, "packed launch");
    return true;
  }

  bool complete_batches() {
    bool any = false;
    for (int bi = 0; bi < kSlots; ++bi) {
      Batch& b = batches_[bi];
      if (!b.active || !batch_done(b)) continue;
      any = true;
      float ms = 0.f;
      if (!cfg_.mock && b.rc == PTS_OK) (void)hipEventElapsedTime(&ms, b.ev0, b.ev1);
      std::lock_guard<std::mutex> lk(mu_);
      busy_s_ += cfg_.mock ? (b.mock_done - b.t_launch) : double(ms) * 1e-3;
      for (size_t i = 0; i < b.reqs.size(); ++i) {
        Req* q = b.reqs[i];
        q->in_batch = -1;
        q->next_blk = b.last[i] ? 0 : b.blk1[i];
        const int64_t n = q->r.count;
        const bool mock_fail =
            cfg_.mock && q->r.kind == PTS_REQ_EVAL && cfg_.mock_fail_count > 0 && n == cfg_.mock_fail_count;
        if (q->cancel) {
          finish_locked(q, ST_CANCELLED, PTS_ECANCELLED, "cancelled while running");
          free_req_locked(q);
        } else if (b.rc != PTS_OK || mock_fail) {
          finish_locked(q, ST_FAILED, mock_fail ? PTS_EHIP : b.rc, mock_fail ? "mock failure" : "launch failed");
          free_req_locked(q);
        } else if (!b.last[i]) {
          // more chunks of this evaluation / step to launch
        } else if (q->r.kind == PTS_REQ_EVAL) {
          if (cfg_.mock) {
            for (int64_t j = 0; j < n; ++j) q->r.out_sdf[j] = float(q->r.cloud) + 1e-3f * float(j % 1000);
          } else {
            std::memcpy(q->r.out_sdf, q->stage + size_t(n) * 12, size_t(n) * 4);
          }
          finish_locked(q, ST_DONE, PTS_OK, nullptr);
          free_req_locked(q);
        } else {
          q->step += 1;
          if (cfg_.mock) {
            if (q->step >= std::min(q->r.steps, 3)) q->n_active = 0;
          } else {
            q->n_active = b.h_counts[i];
          }
          if (q->n_active == 0 || q->step >= q->r.steps) start_final_locked(q);
        }
      }
      b.reqs.clear();
      b.whole = false;
      b.blk0.clear();
      b.blk1.clear();
      b.last.clear();
      b.active = false;
      b.rc = PTS_OK;
    }
    return any;
  }

  // The end of a finished march (mu_ held; the request's last launch has
  // completed).  With normals, the hit rays are first compacted on the device
  // and their count copied to the host (complete_finals then evaluates the
  // normals at those rays only); otherwise the results are copied back.
  void start_final_locked(Req* q) {
    q->finalizing = true;
    finals_.push_back(q);
    if (cfg_.mock) return;
    const int64_t n = q->r.count;
    hipStream_t st = fin_stream_;
    int rc = PTS_OK;
    if (q->r.out_normal) {
      rc = trace_hits(dev<int32_t>(q, q->lay.hit), n, dev<int32_t>(q, q->lay.keep), dev<int32_t>(q, q->lay.act),
                      dev<int32_t>(q, q->lay.blk), dev<int32_t>(q, q->lay.off), dev<int32_t>(q, q->lay.cnt), st);
      // the staged inputs were uploaded before the march: their first bytes take the count
      if (!rc)
        rc = check_hip(hipMemcpyAsync(q->stage, dev<int32_t>(q, q->lay.cnt), sizeof(int32_t), hipMemcpyDeviceToHost,
                                      st),
                       "copy hit count");
      if (!rc) rc = check_hip(hipEventCreateWithFlags(&q->fin_ev, hipEventDisableTiming), "final event");
      if (!rc) rc = check_hip(hipEventRecord(q->fin_ev, st), "final event");
      q->fin_hits = true;
      q->final_rc = rc;
      return;
    }
    q->final_rc = enqueue_results_locked(q, false);
  }

  // Normals at the hit rays (their count is in the first bytes of the stage)
  // if `normals`, then the copy back of the results and an event after it.
  int enqueue_results_locked(Req* q, bool normals) {
    const int64_t n = q->r.count;
    hipStream_t st = fin_stream_;
    int rc = PTS_OK;
    if (normals) {
      int32_t nh = 0;
      std::memcpy(&nh, q->stage, sizeof(nh));
      if (nh < 0 || nh > n) return fail(PTS_EHIP, "hit count out of range");
      const Plan plan = normal_plan(q->N, nh, P_);
      rc = trace_normals_hits(base_ + q->cloud_off, q->N, dev<float>(q, q->lay.org), dev<float>(q, q->lay.dir),
                              dev<float>(q, q->lay.t), dev<int32_t>(q, q->lay.act), nh, dev<float>(q, q->lay.xq),
                              dev<float>(q, q->lay.phi), dev<float>(q, q->lay.g), dev<float>(q, q->lay.nrm), plan,
                              P_.C, dev<void>(q, q->lay.nws), st);
    }
    char* s = q->stage + size_t(n) * 24;
    if (!rc)
      rc = check_hip(hipMemcpyAsync(s, dev<float>(q, q->lay.t), size_t(n) * 4, hipMemcpyDeviceToHost, st), "copy t");
    if (!rc)
      rc = check_hip(hipMemcpyAsync(s + size_t(n) * 4, dev<int32_t>(q, q->lay.hit), size_t(n) * 4,
                                    hipMemcpyDeviceToHost, st),
                     "copy hits");
    if (!rc)
      rc = check_hip(hipMemcpyAsync(s + size_t(n) * 8, dev<int32_t>(q, q->lay.nsteps), size_t(n) * 4,
                                    hipMemcpyDeviceToHost, st),
                     "copy steps");
    if (!rc && q->r.out_normal)
      rc = check_hip(hipMemcpyAsync(s + size_t(n) * 12, dev<float>(q, q->lay.nrm), size_t(n) * 12,
                                    hipMemcpyDeviceToHost, st),
                     "copy normals");
    if (!rc) rc = check_hip(hipEventCreateWithFlags(&q->fin_ev, hipEventDisableTiming), "final event");
    if (!rc) rc = check_hip(hipEventRecord(q->fin_ev, st), "final event");
    return rc;
  }

  bool complete_finals() {
    bool any = false;
    std::lock_guard<std::mutex> lk(mu_);
    for (size_t i = 0; i < finals_.size();) {
      Req* q = finals_[i];
      int rc = q->final_rc;
      if (!cfg_.mock) {
        if (!rc && q->fin_ev) {
          const hipError_t e = hipEventQuery(q->fin_ev);
          if (e == hipErrorNotReady) {
            ++i;
            continue;
          }
          if (e != hipSuccess) rc = check_hip(e, "trace finish");
        } else {
          (void)hipStreamSynchronize(fin_stream_);  // drain what was enqueued before the error
        }
        if (q->fin_ev) (void)hipEventDestroy(q->fin_ev);
        q->fin_ev = nullptr;
        if (!rc && q->fin_hits && !q->cancel) {  // the hit count has arrived
          q->fin_hits = false;
          rc = enqueue_results_locked(q, true);
          q->final_rc = rc;
          if (!rc) {
            ++i;
            continue;
          }
          (void)hipStreamSynchronize(fin_stream_);  // drain what was enqueued before the error
        }
      }
      any = true;
      const int64_t n = q->r.count;
      if (q->cancel) {
        finish_locked(q, ST_CANCELLED, PTS_ECANCELLED, "cancelled while running");
      } else if (rc) {
        finish_locked(q, ST_FAILED, rc, "trace finish failed");
      } else {
        if (cfg_.mock) {
          for (int64_t j = 0; j < n; ++j) {
            q->r.out_sdf[j] = float(q->r.cloud);
            q->r.out_hit[j] = int32_t(j & 1);
            if (q->r.out_steps) q->r.out_steps[j] = std::min(q->r.steps, 3);
            if (q->r.out_normal) {
              q->r.out_normal[3 * j] = 0.f;
              q->r.out_normal[3 * j + 1] = 0.f;
              q->r.out_normal[3 * j + 2] = 0.f;
            }
          }
        } else {
          const char* s = q->stage + size_t(n) * 24;
          std::memcpy(q->r.out_sdf, s, size_t(n) * 4);
          std::memcpy(q->r.out_hit, s + size_t(n) * 4, size_t(n) * 4);
          if (q->r.out_steps) std::memcpy(q->r.out_steps, s + size_t(n) * 8, size_t(n) * 4);
          if (q->r.out_normal) std::memcpy(q->r.out_normal, s + size_t(n) * 12, size_t(n) * 12);
        }
        finish_locked(q, ST_DONE, PTS_OK, nullptr);
      }
      free_req_locked(q);
      finals_.erase(finals_.begin() + long(i));
    }
    return any;
  }

  // Queries per packed-combine workgroup, and the combine workgroups of work
  // blocks [k0, k1) of a request's current evaluation / step.
  static int64_t comb_per(int S, int64_t n) { return combine_by_wave(S, n) ? kBlock / 64 : kBlock; }
  static int64_t chunk_comb_descs(const Req* q, int64_t k0, int64_t k1) {
    const int64_t bq = int64_t(kBlock) * multi_qpl();
    const int64_t q0 = k0 * bq, q1 = std::min(q->n_active, k1 * bq);
    const int64_t per = comb_per(q->plan.S, q->n_active);
    return (q1 - q0 + per - 1) / per;
  }

  // Pack runnable requests (in admission order, chunks of at most a quantum
  // of work in all) into one launch on an idle slot.
  bool launch_batch() {
    int slot = -1;
    for (int bi = 0; bi < kSlots; ++bi)
      if (!batches_[bi].active) {
        slot = bi;
        break;
      }
    if (slot < 0) return false;
    Batch& b = batches_[slot];
    std::vector<Req*> work;
    int64_t nw = 0, nc = 0;
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (size_t i = 0; i < running_.size();) {  // cancelled and on no launch: finish now
        Req* q = running_[i];
        if (q->cancel && q->in_batch < 0 && !q->finalizing) {
          finish_locked(q, ST_CANCELLED, PTS_ECANCELLED, "cancelled while running");
          free_req_locked(q);
        } else {
          ++i;
        }
      }
      // Runnable requests are taken query requests first, then trace steps,
      // each in admission order (a trace runs for many launches anyway; a
      // query waits on each).  Each contributes a chunk of its work blocks
      // (kBlock * qpl queries each, from next_blk on): first one block for
      // every request in that order until a quantum of pairs is reached,
      // then the rest of the quantum to them in the same order.  A long
      // request is thus spread over several launches; requests beyond the
      // quantum are left to the other slot, so both launch slots stay busy;
      // and a request that arrives meanwhile joins the next launch on either
      // slot, waiting about one quantum.  One exception keeps a long request
      // fast when the device is not contended: if it is the only runnable
      // request, exceeds the quantum and the other slot does not hold such a
      // launch, it runs whole -- so at most one launch in flight exceeds the
      // quantum, and a request that arrives meanwhile runs in the other
      // slot.
      const int64_t bq = int64_t(kBlock) * multi_qpl();
      const bool other_whole = batches_[1 - slot].active && batches_[1 - slot].whole;
      std::vector<Req*> cand;  // runnable: query requests, then trace steps
      for (int kind : {int(PTS_REQ_EVAL), int(PTS_REQ_TRACE)})
        for (Req* q : running_)
          if (q->r.kind == kind && q->in_batch < 0 && !q->finalizing && q->n_active > 0) cand.push_back(q);
      const int64_t runnable = int64_t(cand.size());
      b.whole = false;
      std::vector<int64_t> take;
      auto nblk_of = [&](const Req* q) { return (q->n_active + bq - 1) / bq; };
      auto fits = [&](const Req* q, int64_t k) {
        return nw + k * q->plan.S <= max_work_ &&
               nc + chunk_comb_descs(q, q->next_blk, q->next_blk + k) <= max_comb_;
      };
      double budget = quantum_;
      for (Req* q : cand) {
        if (int64_t(work.size()) >= cfg_.max_inflight || budget <= 0.0) break;
        const int64_t rem = nblk_of(q) - q->next_blk;
        const double per = double(bq) * double(q->N);
        if (work.empty() && runnable == 1 && !other_whole && double(rem) * per > quantum_ && fits(q, rem)) {
          work.push_back(q);
          take.push_back(rem);
          b.whole = true;
          break;
        }
        if (!fits(q, 1)) break;  // leads the next launch
        nw += q->plan.S;
        nc += chunk_comb_descs(q, q->next_blk, q->next_blk + 1);
        budget -= per;
        work.push_back(q);
        take.push_back(1);
      }
      for (size_t i = 0; i < work.size() && !b.whole && budget > 0.0; ++i) {
        Req* q = work[i];
        const double per = double(bq) * double(q->N);
        const int64_t fit = int64_t(std::min(budget / per, 1e15));  // (a huge quantum must not overflow)
        int64_t more = std::min<int64_t>(nblk_of(q) - q->next_blk - take[i], fit);
        while (more > 0) {
          const int64_t w = more * q->plan.S;
          const int64_t c = chunk_comb_descs(q, q->next_blk, q->next_blk + take[i] + more) -
                            chunk_comb_descs(q, q->next_blk, q->next_blk + take[i]);
          if (nw + w <= max_work_ && nc + c <= max_comb_) {
            nw += w;
            nc += c;
            break;
          }
          more /= 2;
        }
        if (more <= 0) continue;
        take[i] += more;
        budget -= double(more) * per;
      }
      if (b.whole) {
        nw = take[0] * work[0]->plan.S;
        nc = chunk_comb_descs(work[0], work[0]->next_blk, work[0]->next_blk + take[0]);
      }
      for (size_t i = 0; i < work.size(); ++i) {
        Req* q = work[i];
        b.blk0.push_back(q->next_blk);
        b.blk1.push_back(q->next_blk + take[i]);
        b.last.push_back(q->next_blk + take[i] == nblk_of(q));
      }
    }
    if (work.empty()) return false;
    const bool other_active = batches_[1 - slot].active;
    const int qpl = multi_qpl();
    double pairs = 0;
    int64_t iw = 0, ic = 0;
    bool fold = false;
    for (size_t wi = 0; wi < work.size(); ++wi) {
      Req* q = work[wi];
      fold = fold || q->plan.S > kLaneSplitsMax;
      const int64_t n = q->n_active;
      const Layout L(q->N);
      const bool ev = q->r.kind == PTS_REQ_EVAL;
      float* far2 = nullptr;
      float2* part = nullptr;
      if (ev) {
        far2 = dev<float>(q, q->lay.far2);
        part = dev<float2>(q, q->lay.part);
      } else if (!cfg_.mock) {
        const WsView wv = ws_view(q->plan, q->r.count, dev<void>(q, q->lay.nws));
        far2 = wv.far2;
        part = wv.part;
      }
      const float* x = ev ? dev<float>(q, q->lay.x) : dev<float>(q, q->lay.xq);
      float* out = ev ? dev<float>(q, q->lay.out) : dev<float>(q, q->lay.phi);
      for (int64_t qb = b.blk0[wi]; qb < b.blk1[wi]; ++qb)
        for (int s = 0; s < q->plan.S; ++s) {
          WorkDesc& d = b.h_work[iw++];
          d.rec = cfg_.mock ? nullptr : base_ + q->cloud_off;
          d.x = x;
          d.far2 = far2;
          d.part = part;
          d.Q = n;
          d.per_split = q->plan.per_split;
          d.pos_off = int64_t(L.pos);
          d.rec_off = int64_t(L.rec);
          d.S = q->plan.S;
          d.qb = int32_t(qb);
          d.split = s;
          d.pad = 0;
        }
      const int64_t cper = comb_per(q->plan.S, n);
      const int64_t cb0 = b.blk0[wi] * (int64_t(kBlock) * qpl) / cper;
      const int64_t cb1 = cb0 + chunk_comb_descs(q, b.blk0[wi], b.blk1[wi]);
      for (int64_t qb = cb0; qb < cb1; ++qb) {
        CombDesc& cd = b.h_comb[ic++];
        cd.far2 = far2;
        cd.part = part;
        cd.out = out;
        cd.Q = n;
        cd.S = q->plan.S;
        cd.qb = int32_t(qb);
      }
      pairs += double(std::min(n, b.blk1[wi] * int64_t(kBlock) * qpl) - b.blk0[wi] * int64_t(kBlock) * qpl) *
               double(q->N);
    }
    b.reqs = work;
    b.rc = PTS_OK;
    b.t_launch = now_s();
    if (cfg_.mock) {
      b.mock_done = b.t_launch + pairs / (cfg_.mock_pairs_per_s > 0 ? cfg_.mock_pairs_per_s : 1e12);
    } else {
      hipStream_t st = b.stream;
      WorkDesc* d_work = reinterpret_cast<WorkDesc*>(base_ + b.d_work_off);
      CombDesc* d_comb = reinterpret_cast<CombDesc*>(base_ + b.d_comb_off);
      int rc = check_hip(hipEventRecord(b.ev0, st), "launch event");
      for (size_t i = 0; i < work.size(); ++i) {  // a trace step's positions, before its first chunk
        Req* q = work[i];
        if (!rc && q->r.kind == PTS_REQ_TRACE && b.blk0[i] == 0)
          rc = trace_step_pre(q->act, q->n_active, dev<float>(q, q->lay.org), dev<float>(q, q->lay.dir),
                              dev<float>(q, q->lay.t), dev<float>(q, q->lay.xq), st);
      }
      if (!rc)
        rc = check_hip(hipMemcpyAsync(d_work, b.h_work, size_t(nw) * sizeof(WorkDesc), hipMemcpyHostToDevice, st),
                       "descriptor upload");
      if (!rc)
        rc = check_hip(hipMemcpyAsync(d_comb, b.h_comb, size_t(nc) * sizeof(CombDesc), hipMemcpyHostToDevice, st),
                       "descriptor upload");
      if (!rc) rc = launch_multi(d_work, nw, d_comb, nc, P_.C, fold, st);
      for (size_t i = 0; i < work.size() && !rc; ++i) {
        Req* q = work[i];
        const int64_t n = q->r.count;
        if (!b.last[i]) continue;  // results and the step's end follow its last chunk
        if (q->r.kind == PTS_REQ_EVAL) {
          rc = check_hip(hipMemcpyAsync(q->stage + size_t(n) * 12, dev<float>(q, q->lay.out), size_t(n) * 4,
                                        hipMemcpyDeviceToHost, st),
                         "result copy");
        } else {
          rc = trace_step_post(q->act, q->n_active, dev<float>(q, q->lay.phi), q->r.eps, q->r.tmax, q->step,
                               dev<float>(q, q->lay.t), dev<int32_t>(q, q->lay.hit), dev<int32_t>(q, q->lay.nsteps),
                               dev<int32_t>(q, q->lay.keep), q->nxt, dev<int32_t>(q, q->lay.blk),
                               dev<int32_t>(q, q->lay.off), dev<int32_t>(q, q->lay.cnt), st);
          if (!rc)
            rc = check_hip(hipMemcpyAsync(b.h_counts + i, dev<int32_t>(q, q->lay.cnt), sizeof(int32_t),
                                          hipMemcpyDeviceToHost, st),
                           "count copy");
          std::swap(q->act, q->nxt);
        }
      }
      const hipError_t er = hipEventRecord(b.ev1, st);
      if (!rc && er != hipSuccess) rc = check_hip(er, "launch event");
      if (rc) {
        (void)hipStreamSynchronize(st);
        b.rc = rc;
      }
    }
    std::lock_guard<std::mutex> lk(mu_);
    for (Req* q : work) q->in_batch = slot;
    b.active = true;
    ++launches_;
    if (other_active) ++overlapped_;
    pairs_ += pairs;
    max_batch_reqs_ = std::max<int64_t>(max_batch_reqs_, int64_t(work.size()));
    return true;
  }

  pts_server_cfg cfg_;
  pts_params P_{};
  Arena arena_;
  int dev_ = 0;
  char* base_ = nullptr;
  int64_t max_work_ = 0, max_comb_ = 0;
  double quantum_ = 0;
  std::mutex mu_;
  std::condition_variable cv_, cv_done_;
  std::thread th_;
  bool started_ = false, stopping_ = false, shut_ = false;
  std::map<int, SCloud> clouds_;
  std::map<uint64_t, std::unique_ptr<Req>> reqs_;
  std::deque<Req*> pending_;
  std::vector<Req*> running_, fresh_, finals_;
  Batch batches_[kSlots];
  hipStream_t up_stream_ = nullptr, fin_stream_ = nullptr;
  hipEvent_t up_ev_ = nullptr;
  std::map<size_t, std::vector<char*>> pool_;
  size_t resident_ = 0, reserved_ = 0;
  int next_cloud_ = 1;
  uint64_t next_ticket_ = 1;
  uint64_t submitted_ = 0, completed_ = 0, failed_ = 0, cancelled_ = 0, rejected_ = 0, launches_ = 0,
           overlapped_ = 0;
  int64_t max_batch_reqs_ = 0;
  int waiters_ = 0;
  double pairs_ = 0, busy_s_ = 0;
  std::vector<double> lat_all_, lat_eval_, lat_trace_;
};

}  // namespace pts

struct pts_server {
  std::unique_ptr<pts::Server> s;
};

extern "C" {

int pts_server_create(const pts_server_cfg* cfg, pts_server** out) {
  using pts::fail;
  if (!out) return fail(PTS_EINVAL, "null pointer");
  *out = nullptr;
  pts_server_cfg c{};
  if (cfg) c = *cfg;
  if (c.hbm_budget_bytes == 0) c.hbm_budget_bytes = size_t(4) << 30;
  if (c.max_inflight <= 0) c.max_inflight = 64;
  if (c.max_queue <= 0) c.max_queue = 1 << 20;
  if (c.max_batch_work <= 0) c.max_batch_work = 131072;
  if (c.max_batch_work > (int64_t(1) << 24)) return fail(PTS_EINVAL, "max_batch_work must be <= 2^24");
  if (c.C != 0.f && !(c.C > 0.f && c.C <= pts::kCMax)) return fail(PTS_EINVAL, "C must be in (0, 75]");
  if (!(c.kfloor_rel == 0.f || (c.kfloor_rel >= pts::kKfloorRelMin && std::isfinite(c.kfloor_rel))))
    return fail(PTS_EINVAL, "kfloor_rel must be 0 (default) or in [1e-12, inf)");
  if (c.mock && !(c.mock_pairs_per_s >= 0)) return fail(PTS_EINVAL, "mock_pairs_per_s must be >= 0");
  if (!(c.quantum_pairs >= 0) || !std::isfinite(c.quantum_pairs))
    return fail(PTS_EINVAL, "quantum_pairs must be finite and >= 0");
  auto h = std::make_unique<pts_server>();
  h->s = std::make_unique<pts::Server>(c);
  if (int rc = h->s->init()) return rc;
  *out = h.release();
  return PTS_OK;
}

int pts_server_add_cloud(pts_server* s, const float* p, const float* n, const float* a, int64_t N, int* id) {
  if (!s) return pts::fail(PTS_EINVAL, "null server");
  return s->s->add_cloud(p, n, a, N, id);
}

int pts_server_cloud_plan(pts_server* s, int id, int64_t* N, int* splits) {
  if (!s) return pts::fail(PTS_EINVAL, "null server");
  return s->s->cloud_plan(id, N, splits);
}

int pts_server_remove_cloud(pts_server* s, int id) {
  if (!s) return pts::fail(PTS_EINVAL, "null server");
  return s->s->remove_cloud(id);
}

int pts_server_submit(pts_server* s, const pts_request* r, uint64_t* ticket) {
  if (!s) return pts::fail(PTS_EINVAL, "null server");
  return s->s->submit(r, ticket);
}

int pts_server_poll(pts_server* s, uint64_t ticket, int* state) {
  if (!s) return pts::fail(PTS_EINVAL, "null server");
  return s->s->poll(ticket, state);
}

int pts_server_wait(pts_server* s, uint64_t ticket, int timeout_ms) {
  if (!s) return pts::fail(PTS_EINVAL, "null server");
  return s->s->wait(ticket, timeout_ms);
}

int pts_server_cancel(pts_server* s, uint64_t ticket) {
  if (!s) return pts::fail(PTS_EINVAL, "null server");
  return s->s->cancel(ticket);
}

int pts_server_release(pts_server* s, uint64_t ticket) {
  if (!s) return pts::fail(PTS_EINVAL, "null server");
  return s->s->release(ticket);
}

int pts_server_stats_get(pts_server* s, pts_server_stats* out) {
  if (!s) return pts::fail(PTS_EINVAL, "null server");
  return s->s->get_stats(out);
}

int pts_server_stats_reset(pts_server* s) {
  if (!s) return pts::fail(PTS_EINVAL, "null server");
  return s->s->reset_stats();
}

int pts_server_destroy(pts_server* s) {
  if (!s) return PTS_OK;
  s->s->shutdown();
  delete s;
  return PTS_OK;
}

}  // extern "C"
