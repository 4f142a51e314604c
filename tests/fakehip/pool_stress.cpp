// Drives the serving pool of the host runtime (gbees.cpp) on the fake HIP
// backend: many requests of two kinds and uneven capacities, groups of eight
// per driver thread, results fetched by several threads at once (some
// requests by two threads concurrently), releases, capacity failures that are
// rolled back and moved into larger slices, and requests that cannot grow
// because the arena is full.  Built with AddressSanitizer or ThreadSanitizer
// by tests/test_pool_host.py; exits non-zero on any inconsistency.
// TEST INFRASTRUCTURE ONLY.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gbees.h"

namespace {

gbees_config make_cfg(int k) {
  gbees_config c;
  std::memset(&c, 0, sizeof(c));
  const bool l96 = (k % 2) == 1;
  c.n = l96 ? 6 : 3;
  c.model = l96 ? GBEES_L96 : GBEES_L63;
  c.params[0] = l96 ? 4.0 : 10.0;
  c.params[1] = 28.0;
  c.params[2] = 8.0 / 3.0;
  for (int j = 0; j < c.n; ++j) {
    c.h[j] = 0.5;
    c.mean[j] = 1.0;
    c.cov[j * c.n + j] = 1.0 + 0.1 * (k % 7);
  }
  c.thresh_rel = 1e-4;
  c.cfl = 0.9;
  c.prune_every = 5;
  c.limiter = 1;
  c.precision = (k % 5) == 4 ? 1 : 0;
  // 3..20 bricks: the fake grid starts with 2..6 bricks and gains one every
  // third step, so the smaller capacities run out and must be enlarged.
  c.max_cells = 64 * (3 + (k * 7) % 18);
  return c;
}

int fail(const char* what, int64_t id, int code) {
  std::fprintf(stderr, "FAIL %s request %lld code %d\n", what, static_cast<long long>(id), code);
  std::exit(1);
}

}  // namespace

int main(int argc, char** argv) {
  const int nreq = argc > 1 ? std::atoi(argv[1]) : 240;
  const size_t bytes = size_t(160) << 20;
  void* arena = std::aligned_alloc(256, bytes);
  gbees_pool* pool = nullptr;
  if (gbees_pool_create(arena, bytes, 32, &pool) != GBEES_OK) return fail("create", 0, -1);
  if (gbees_pool_group_size(pool, 8) != GBEES_OK) return fail("group size", 0, -1);

  std::mutex qmu;
  std::deque<int64_t> ready;
  std::atomic<bool> done_submitting{false};
  std::atomic<int> finished{0}, failed{0}, resized{0};
  std::unordered_map<int64_t, std::atomic<int>*> pending_fetch;

  auto fetcher = [&] {
    while (true) {
      int64_t id = -1;
      {
        std::lock_guard<std::mutex> lk(qmu);
        if (!ready.empty()) {
          id = ready.front();
          ready.pop_front();
        }
      }
      if (id < 0) {
        if (done_submitting && finished + failed >= nreq) return;
        std::this_thread::yield();
        continue;
      }
      int64_t cnt = 0;
      int rc = gbees_pool_result(pool, id, 0, nullptr, nullptr, &cnt);
      if (rc != GBEES_E_BUFFER && rc != GBEES_OK) fail("result size", id, rc);
      std::vector<int32_t> idx(static_cast<size_t>(cnt) * 6);
      std::vector<double> P(static_cast<size_t>(cnt));
      rc = gbees_pool_result(pool, id, cnt, idx.data(), P.data(), &cnt);
      if (rc != GBEES_OK) fail("result", id, rc);
      if (cnt <= 0 || cnt % 64 != 0) fail("result count", id, static_cast<int>(cnt));
      std::atomic<int>* left;
      {
        std::lock_guard<std::mutex> lk(qmu);
        left = pending_fetch.at(id);
      }
      if (left->fetch_sub(1) == 1) {  // last fetcher of this request releases it
        rc = gbees_pool_release(pool, id);
        if (rc != GBEES_OK) fail("release", id, rc);
        ++finished;
      }
    }
  };
  std::vector<std::thread> th;
  for (int k = 0; k < 4; ++k) th.emplace_back(fetcher);

  std::vector<int64_t> live;
  std::vector<std::atomic<int>> counters(static_cast<size_t>(nreq));
  int submitted = 0;
  while (finished + failed < nreq) {
    for (int burst = 0; burst < 8 && submitted < nreq; ++burst, ++submitted) {
      const gbees_config c = make_cfg(submitted);
      gbees_meas m[3];
      const int nm = submitted % 4 == 3 ? 0 : submitted % 3 + 1;
      for (int q = 0; q < nm; ++q) m[q] = gbees_meas{0.05 * (q + 1), q % c.n, 1.0, 1.0};
      int64_t id = 0;
      const int rc = gbees_pool_submit(pool, &c, 0.2 + 0.01 * (submitted % 9), m, nm, &id);
      if (rc != GBEES_OK) fail("submit", submitted, rc);
      live.push_back(id);
    }
    if (submitted >= nreq) done_submitting = true;
    if (gbees_pool_progress(pool, nullptr, nullptr) != GBEES_OK) fail("progress", 0, -1);
    std::vector<int64_t> still;
    for (int64_t id : live) {
      gbees_req_info inf;
      if (gbees_pool_info(pool, id, &inf) != GBEES_OK) fail("info", id, -1);
      if (inf.status == 2) {
        resized += inf.resizes > 0 ? 1 : 0;
        const int fetchers = (id % 5 == 0) ? 2 : 1;  // every fifth request: two threads fetch it at once
        std::lock_guard<std::mutex> lk(qmu);
        std::atomic<int>* ctr = &counters[static_cast<size_t>(id - 1)];
        ctr->store(fetchers);
        pending_fetch[id] = ctr;
        for (int f = 0; f < fetchers; ++f) ready.push_back(id);
      } else if (inf.status < 0) {
        if (inf.status != GBEES_E_CAPACITY) fail("status", id, inf.status);
        if (gbees_pool_release(pool, id) != GBEES_OK) fail("release failed", id, -1);
        ++failed;
      } else {
        still.push_back(id);
      }
    }
    live.swap(still);
    std::this_thread::yield();
  }
  for (auto& t : th) t.join();
  if (gbees_pool_destroy(pool) != GBEES_OK) fail("destroy", 0, -1);
  std::free(arena);
  std::printf("pool_stress ok: %d finished (%d after a resize), %d out of capacity\n", finished.load(), resized.load(),
              failed.load());
  return 0;
}
