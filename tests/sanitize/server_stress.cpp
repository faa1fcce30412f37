// server_stress.cpp -- the server's scheduler under concurrent clients, on a
// host without a GPU (mock executor), for builds of the library's host code
// with AddressSanitizer + UndefinedBehaviorSanitizer or ThreadSanitizer.
//
// Scenarios (each checks the results it can: mock outputs follow a fixed
// pattern, cloud id + 1e-3 (j mod 1000) for query requests):
//   1. many client threads submit, wait and release query and trace
//      requests on several clouds, with cancellations mixed in;
//   2. several threads wait on the same ticket and race to release it (a
//      release while another thread still waits must be refused, not free
//      the request under it);
//   3. long requests spread over quantum-bounded launches while short ones
//      pass them;
//   4. destroy while requests are queued and running.
// Exit status 0 when every check passed.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "pts.h"

namespace {

std::atomic<int> g_fail{0};

#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      g_fail.fetch_add(1);                                            \
    }                                                                 \
  } while (0)

pts_server* make_server(double quantum, int64_t max_work, double rate) {
  pts_server_cfg cfg{};
  cfg.hbm_budget_bytes = size_t(512) << 20;
  cfg.max_inflight = 32;
  cfg.max_batch_work = max_work;
  cfg.mock = 1;
  cfg.mock_pairs_per_s = rate;
  cfg.quantum_pairs = quantum;
  pts_server* s = nullptr;
  CHECK(pts_server_create(&cfg, &s) == PTS_OK);
  return s;
}

int add_cloud(pts_server* s, int64_t N) {
  std::vector<float> p(size_t(N) * 3, 0.f), n(size_t(N) * 3, 0.f), a(size_t(N) * 6, 0.f);
  for (int64_t i = 0; i < N; ++i) {
    p[3 * i] = float(i % 97) * 0.01f;
    n[3 * i + 2] = 1.f;
  }
  int id = -1;
  CHECK(pts_server_add_cloud(s, p.data(), n.data(), a.data(), N, &id) == PTS_OK);
  return id;
}

bool pattern_ok(const std::vector<float>& out, int cloud) {
  for (size_t j = 0; j < out.size(); ++j)
    if (std::fabs(out[j] - (float(cloud) + 1e-3f * float(j % 1000))) > 1e-3f) return false;
  return true;
}

void clients(pts_server* s, const std::vector<int>& ids, int nthreads, int per_thread) {
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; ++t)
    th.emplace_back([&, t] {
      unsigned seed = 1234u + unsigned(t);
      for (int k = 0; k < per_thread; ++k) {
        seed = seed * 1103515245u + 12345u;
        const int cloud = ids[(seed >> 8) % ids.size()];
        const bool trace = ((seed >> 4) % 8) == 0;
        const int64_t count = trace ? 1 + int64_t((seed >> 12) % 3000) : int64_t((seed >> 12) % 5000);
        const size_t n = static_cast<size_t>(count);
        std::vector<float> in0(n * 3, 0.f), in1(n * 3, 0.f), out(n, -1.f), nrm(n * 3);
        std::vector<int32_t> hit(n), steps(n);
        for (int64_t j = 0; j < count; ++j) in1[3 * j + 2] = 1.f;
        pts_request r{};
        r.kind = trace ? PTS_REQ_TRACE : PTS_REQ_EVAL;
        r.cloud = cloud;
        r.count = count;
        r.in0 = in0.data();
        r.in1 = trace ? in1.data() : nullptr;
        r.out_sdf = out.data();
        r.out_normal = trace ? nrm.data() : nullptr;
        r.out_hit = trace ? hit.data() : nullptr;
        r.out_steps = trace ? steps.data() : nullptr;
        r.steps = 6;
        r.eps = 1e-3f;
        r.tmax = 5.f;
        uint64_t tk = 0;
        const int rc = pts_server_submit(s, &r, &tk);
        if (rc == PTS_EBUSY) continue;
        CHECK(rc == PTS_OK);
        if (rc != PTS_OK) continue;
        const bool cancel = ((seed >> 20) % 11) == 0;
        if (cancel) CHECK(pts_server_cancel(s, tk) == PTS_OK);
        const int w = pts_server_wait(s, tk, -1);
        CHECK(w == PTS_OK || (cancel && w == PTS_ECANCELLED));
        if (w == PTS_OK && !trace) CHECK(pattern_ok(out, cloud));
        if (w == PTS_OK && trace)
          for (int64_t j = 0; j < count; ++j) CHECK(out[size_t(j)] == float(cloud) && hit[size_t(j)] == (j & 1));
        CHECK(pts_server_release(s, tk) == PTS_OK);
      }
    });
  for (auto& x : th) x.join();
}

void shared_ticket(pts_server* s, int cloud) {
  for (int rep = 0; rep < 20; ++rep) {
    std::vector<float> in(size_t(3000) * 3, 0.f), out(3000);
    pts_request r{};
    r.kind = PTS_REQ_EVAL;
    r.cloud = cloud;
    r.count = 3000;
    r.in0 = in.data();
    r.out_sdf = out.data();
    uint64_t tk = 0;
    CHECK(pts_server_submit(s, &r, &tk) == PTS_OK);
    std::atomic<int> released{0};
    std::vector<std::thread> th;
    for (int t = 0; t < 4; ++t)
      th.emplace_back([&] {
        const int w = pts_server_wait(s, tk, -1);
        CHECK(w == PTS_OK || w == PTS_ENOTFOUND);
        const int rc = pts_server_release(s, tk);
        CHECK(rc == PTS_OK || rc == PTS_EBUSY || rc == PTS_ENOTFOUND);
        if (rc == PTS_OK) released.fetch_add(1);
      });
    for (auto& x : th) x.join();
    // the ticket may still be held if every release came while another waited
    if (released.load() == 0) CHECK(pts_server_release(s, tk) == PTS_OK);
    CHECK(pattern_ok(out, cloud));
  }
}

}  // namespace

int main() {
  {  // 1 + 2: mixed clients, shared tickets
    pts_server* s = make_server(0.0, 1 << 14, 2e9);
    std::vector<int> ids = {add_cloud(s, 1000), add_cloud(s, 5000), add_cloud(s, 20000)};
    std::thread sh([&] { shared_ticket(s, ids[1]); });
    clients(s, ids, 8, 40);
    sh.join();
    pts_server_stats st{};
    CHECK(pts_server_stats_get(s, &st) == PTS_OK);
    CHECK(st.failed == 0);
    CHECK(pts_server_destroy(s) == PTS_OK);
  }
  {  // 3: quantum-bounded launches
    const double quantum = 512.0 * 4000 * 4;
    pts_server* s = make_server(quantum, 1 << 16, quantum / 0.002);
    std::vector<int> ids = {add_cloud(s, 4000)};
    std::thread big([&] {
      for (int k = 0; k < 3; ++k) {
        std::vector<float> in(size_t(40000) * 3, 0.f), out(40000);
        pts_request r{};
        r.kind = PTS_REQ_EVAL;
        r.cloud = ids[0];
        r.count = 40000;
        r.in0 = in.data();
        r.out_sdf = out.data();
        uint64_t tk = 0;
        CHECK(pts_server_submit(s, &r, &tk) == PTS_OK);
        CHECK(pts_server_wait(s, tk, -1) == PTS_OK);
        CHECK(pattern_ok(out, ids[0]));
        CHECK(pts_server_release(s, tk) == PTS_OK);
      }
    });
    clients(s, ids, 4, 20);
    big.join();
    CHECK(pts_server_destroy(s) == PTS_OK);
  }
  {  // 4: destroy with requests queued and running (they finish cancelled; nothing leaks)
    pts_server* s = make_server(0.0, 1 << 14, 1e8);
    const int c = add_cloud(s, 5000);
    std::vector<std::vector<float>> ins(16, std::vector<float>(size_t(4000) * 3, 0.f)),
        outs(16, std::vector<float>(4000));
    for (int k = 0; k < 16; ++k) {
      pts_request r{};
      r.kind = PTS_REQ_EVAL;
      r.cloud = c;
      r.count = 4000;
      r.in0 = ins[size_t(k)].data();
      r.out_sdf = outs[size_t(k)].data();
      uint64_t tk = 0;
      CHECK(pts_server_submit(s, &r, &tk) == PTS_OK);
    }
    std::this_thread::sleep_for(std::chrono::milliseconds(5));
    CHECK(pts_server_destroy(s) == PTS_OK);
  }
  std::printf("server_stress: %s (%d failed checks)\n", g_fail.load() ? "FAILED" : "ok", g_fail.load());
  return g_fail.load() ? 1 : 0;
}
