// Batch formation of the serving loop: host-only policy, no device code (it is
// compiled by the host compiler alone in the CPU tests).
//
// A batch is a prefix of the first-come first-served queue.  It grows while
//   * its queries stay within the query cap, and
//   * with the deadline cap on: its predicted completion stays within the
//     earliest deadline among its requests.  A request that would push the
//     batch past a deadline the batch still meets waits for the next batch.
//     When even the batch without it misses its earliest deadline (the queue
//     is behind), the deadline no longer limits the batch: under overload the
//     larger batch clears the queue sooner.
// The caller then shrinks the prefix until its workspace fits a slot.
// Reserve slots (the last reserve_streams of the server's streams) take a
// batch only under overload (reserve_may_run): at light load fewer batches
// share the GPU and each finishes sooner; under overload the extra batch in
// flight fills the gaps between the phases of the others.
//
// Completion is predicted by a linear model of service time fitted online to
// the batches served so far: time = c0 + c1 * x, x = sum over requests of
// weight(q, k) = q * (1 + k / kWeightK).  Per query the scan costs the same
// for any k; candidate handling grows with k.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>

namespace fps {

struct PendingView {
  uint32_t q = 0, k = 0;
  uint64_t submit_ns = 0;
  uint32_t deadline_us = 0;  // 0: none
};

class CostModel {
 public:
  static constexpr double kWeightK = 700.0;
  static constexpr double kForget = 0.95;  // per observed batch

  static double weight(uint32_t q, uint32_t k) { return (double)q * (1.0 + (double)k / kWeightK); }

  // Predicted service time of a batch of total weight x, in ns.
  uint64_t predict_ns(double x) const {
    const double us = c0_ + c1_ * x;
    return us <= 0 ? 0 : (uint64_t)(us * 1000.0);
  }

  // One served batch: total weight x, service time us.  Weighted least squares
  // over the batches so far, older ones discounted by kForget each.
  void observe(double x, double us) {
    sw_ = kForget * sw_ + 1.0;
    sx_ = kForget * sx_ + x;
    sy_ = kForget * sy_ + us;
    sxx_ = kForget * sxx_ + x * x;
    sxy_ = kForget * sxy_ + x * us;
    const double mx = sx_ / sw_, my = sy_ / sw_;
    const double vx = sxx_ / sw_ - mx * mx, cxy = sxy_ / sw_ - mx * my;
    if (sw_ >= 3.0 && vx > 1e-3 * mx * mx && cxy > 0) {
      c1_ = cxy / vx;
      c0_ = std::max(0.0, my - c1_ * mx);
    } else if (mx > 0) {  // too little spread in x: proportional model
      c1_ = my / mx;
      c0_ = 0;
    }
  }

  double c0_us() const { return c0_; }
  double c1_us() const { return c1_; }

 private:
  // prior until batches are observed: 0.5 ms + 20 us per unit of weight
  double c0_ = 500.0, c1_ = 20.0;
  double sw_ = 0, sx_ = 0, sy_ = 0, sxx_ = 0, sxy_ = 0;
};

// The queue is behind when its first request would miss its deadline even if
// it were served alone starting now (requests without a deadline never are).
inline bool queue_behind(const PendingView &head, uint64_t now_ns, const CostModel &cm) {
  if (!head.deadline_us) return false;
  return now_ns + cm.predict_ns(CostModel::weight(head.q, head.k)) >
         head.submit_ns + 1000ull * head.deadline_us;
}

// A reserve slot takes a batch only under overload: the queue is behind and
// holds at least a full batch of queries (a late request alone, at light
// load, does not wake it).
inline bool reserve_may_run(const PendingView &head, uint64_t pending_queries,
                            uint32_t max_queries, uint64_t now_ns, const CostModel &cm) {
  return pending_queries >= max_queries && queue_behind(head, now_ns, cm);
}

// Length of the queue prefix that forms the next batch (at least 1 when the
// queue is not empty).  get(i) returns the PendingView of the i-th request.
template <class Get>
size_t batch_prefix(size_t count, Get get, uint64_t now_ns, uint32_t max_queries,
                    bool deadline_cap, const CostModel &cm) {
  size_t n = 0;
  uint64_t qs = 0, dl = UINT64_MAX;
  double x = 0;
  for (; n < count; ++n) {
    const PendingView r = get(n);
    if (n > 0 && qs + r.q > max_queries) break;
    const double x2 = x + CostModel::weight(r.q, r.k);
    const uint64_t dl2 =
        r.deadline_us ? std::min<uint64_t>(dl, r.submit_ns + 1000ull * r.deadline_us) : dl;
    if (deadline_cap && n > 0 && dl2 != UINT64_MAX) {
      const bool meets = dl == UINT64_MAX || now_ns + cm.predict_ns(x) <= dl;
      if (meets && now_ns + cm.predict_ns(x2) > dl2) break;
    }
    qs += r.q;
    x = x2;
    dl = dl2;
  }
  return n;
}

}  // namespace fps
