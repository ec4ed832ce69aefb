// Drives the serving loop's batch-formation policy (host-only header) through
// fixed scenarios and prints one "name value" line per result; the Python test
// checks the values.
#include <cstdio>
#include <vector>

#include "batcher.h"

using fps::CostModel;
using fps::PendingView;

static size_t prefix(const std::vector<PendingView> &p, uint64_t now, uint32_t maxq, bool cap,
                     const CostModel &cm) {
  return fps::batch_prefix(p.size(), [&](size_t i) { return p[i]; }, now, maxq, cap, cm);
}

static std::vector<PendingView> reqs(size_t n, uint32_t q, uint32_t k, uint64_t submit,
                                     uint32_t deadline_us) {
  std::vector<PendingView> v(n);
  for (auto &r : v) {
    r.q = q;
    r.k = k;
    r.submit_ns = submit;
    r.deadline_us = deadline_us;
  }
  return v;
}

int main() {
  // the fit recovers a linear law from batches of varying weight
  CostModel lin;
  for (int i = 0; i < 40; ++i) {
    const double x = 50.0 + 37.0 * (i % 9);
    lin.observe(x, 300.0 + 4.0 * x);
  }
  std::printf("fit_c0 %.6f\nfit_c1 %.6f\n", lin.c0_us(), lin.c1_us());
  // one repeated weight: proportional model
  CostModel flat;
  for (int i = 0; i < 10; ++i) flat.observe(100.0, 2000.0);
  std::printf("flat_c0 %.6f\nflat_c1 %.6f\n", flat.c0_us(), flat.c1_us());
  std::printf("weight_q10_k700 %.6f\n", CostModel::weight(10, 700));

  // model used below: 300 us + 4 us per unit of weight; requests of 10
  // queries at k = 0 weigh 10 (40 us each)
  const uint64_t now = 1000000000ull;
  // query cap alone
  std::printf("cap_only %zu\n", prefix(reqs(20, 10, 0, now, 0), now, 35, true, lin));
  std::printf("first_over_cap %zu\n", prefix(reqs(3, 50, 0, now, 0), now, 35, true, lin));
  std::printf("empty %zu\n", prefix({}, now, 35, true, lin));
  // deadline 10 ms from now: 300 + 40 n <= 10000 -> n <= 242
  std::printf("deadline %zu\n", prefix(reqs(400, 10, 0, now, 10000), now, 100000, true, lin));
  // the same with the cap off
  std::printf("deadline_off %zu\n", prefix(reqs(400, 10, 0, now, 10000), now, 100000, false, lin));
  // submitted 5 ms ago: 300 + 40 n <= 5000 -> n <= 117
  std::printf("deadline_aged %zu\n",
              prefix(reqs(400, 10, 0, now - 5000000ull, 10000), now, 100000, true, lin));
  // the head is already late: no deadline limit, the query cap rules
  std::printf("behind %zu\n",
              prefix(reqs(400, 10, 0, now - 20000000ull, 10000), now, 2000, true, lin));
  // a late head followed by fresh requests: the batch is behind from its first
  // request on, so it grows to the query cap
  {
    auto v = reqs(1, 10, 0, now - 20000000ull, 10000);
    auto w = reqs(300, 10, 0, now, 10000);
    v.insert(v.end(), w.begin(), w.end());
    std::printf("behind_mixed %zu\n", prefix(v, now, 2000, true, lin));
  }
  // requests without deadlines ahead of one with a deadline: the deadline one
  // joins only while it is still met (300 + 40 n <= 1000 -> n <= 17)
  {
    auto v = reqs(50, 10, 0, now, 0);
    v[30].deadline_us = 1000;
    std::printf("late_joiner %zu\n", prefix(v, now, 100000, true, lin));
    auto u = reqs(50, 10, 0, now, 0);
    u[10].deadline_us = 1000;
    std::printf("early_joiner %zu\n", prefix(u, now, 100000, true, lin));
  }
  // k raises the weight: k = 700 doubles it -> 300 + 80 n <= 10000 -> n <= 121
  std::printf("deadline_k700 %zu\n", prefix(reqs(400, 10, 700, now, 10000), now, 100000, true, lin));
  // behind: the head alone (300 + 40 us) misses its deadline
  {
    PendingView h;
    h.q = 10;
    h.k = 0;
    h.deadline_us = 10000;
    h.submit_ns = now - 9000000ull;  // 1 ms left: 340 us fit
    std::printf("behind_no %d\n", fps::queue_behind(h, now, lin) ? 1 : 0);
    h.submit_ns = now - 9800000ull;  // 200 us left: 340 us do not
    std::printf("behind_yes %d\n", fps::queue_behind(h, now, lin) ? 1 : 0);
    h.deadline_us = 0;  // no deadline: never behind
    std::printf("behind_none %d\n", fps::queue_behind(h, now, lin) ? 1 : 0);
    h.deadline_us = 10000;
    std::printf("reserve_full %d\n", fps::reserve_may_run(h, 1024, 1024, now, lin) ? 1 : 0);
    std::printf("reserve_short %d\n", fps::reserve_may_run(h, 1023, 1024, now, lin) ? 1 : 0);
    h.submit_ns = now;  // on time
    std::printf("reserve_on_time %d\n", fps::reserve_may_run(h, 5000, 1024, now, lin) ? 1 : 0);
  }
  return 0;
}
