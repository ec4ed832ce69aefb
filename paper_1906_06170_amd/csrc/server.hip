// Continuous-batching request loop over a resident library.
//
// The paper decouples the user side from the long computation with a queue
// (Sections 3.1 and 4.4).  Here the queue feeds the GPU directly: requests are
// admitted while the workspace pool has room for their candidate buffers,
// coalesced first-come first-served into batches (capped by query count and,
// optionally, by the earliest deadline; batcher.h), and run on n_streams slots
// (one worker thread, one HIP stream and one workspace slice each), so a batch
// can start while others are still on the device.  The last reserve_streams
// slots run only under overload.  Each request keeps its own
// k and stride mask inside the batch; batching never changes a result, since
// every query of a batch is answered independently.
//
// Latency is counted from a request's arrival (given by the caller or stamped
// when submit is entered, before any wait for admission) to the moment its
// results are available.  No kernel is ever timed on the request path: the
// batch shapes named at creation are tuned there, and any other shape takes a
// fixed default kernel.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batcher.h"
#include "fps_internal.h"
#include "runtime.h"

namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  uint64_t ticket = 0;
  std::vector<uint64_t> queries;
  uint32_t q = 0, k = 0, mask = 0, deadline_us = 0;
  uint32_t keff = 0;  // min(k, records in the mask's strides): hits per query
  size_t bytes = 0;  // workspace the request needs on its own
  uint64_t arrival_ns = 0, submit_ns = 0, start_ns = 0, done_ns = 0;
  uint32_t batch_id = 0, batch_queries = 0;
  std::vector<fps_hit> hits;
  std::vector<uint64_t> offsets;
  fps_status status = FPS_OK;
  std::string error;
  bool done = false;
};

struct Slot {
  hipStream_t stream = nullptr;
  uint8_t *ws = nullptr;
  size_t ws_bytes = 0;
  SearchCtx ctx;
  std::thread worker;
  // batch buffers, kept across batches
  std::vector<uint64_t> qs, off;
  std::vector<uint32_t> kk, mm;
  std::vector<fps_hit> hits;
  ~Slot() {
    if (stream) (void)hipStreamDestroy(stream);
  }
};

}  // namespace

struct fps_server {
  fps_library *lib = nullptr;
  fps_server_config cfg{};
  std::vector<std::unique_ptr<Slot>> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_room;
  std::deque<std::shared_ptr<Request>> pending;
  uint64_t pending_q = 0;  // queries in pending
  std::unordered_map<uint64_t, std::shared_ptr<Request>> live;
  size_t admitted_bytes = 0;
  uint64_t next_ticket = 1;
  uint32_t next_batch = 1;
  bool stopping = false;
  fps::CostModel cost;  // service time of a batch (batcher.h)
  // statistics
  // latencies of the last kLatWindow requests (a ring once full)
  static constexpr size_t kLatWindow = size_t(1) << 20;
  std::vector<double> lat_us, admit_us;  // arrival -> done, arrival -> admission
  size_t lat_next = 0, admit_next = 0;
  uint64_t st_requests = 0, st_queries = 0, st_batches = 0, st_misses = 0, st_batch_q = 0,
           st_untuned = 0;
};

// Appends to a ring of the last fps_server::kLatWindow values.
static void ring_push(std::vector<double> &v, size_t &next, double x) {
  if (v.size() < fps_server::kLatWindow) {
    v.push_back(x);
  } else {
    v[next] = x;
    next = (next + 1) % fps_server::kLatWindow;
  }
}

static size_t request_bytes(fps_library *lib, uint32_t q, uint32_t k, uint32_t mask) {
  std::vector<uint32_t> kk(q, k), mm(q, mask);
  Plan P;
  if (fps_plan(lib, q, kk.data(), mm.data(), &P)) return (size_t)-1;
  return P.total_bytes;
}

static fps::PendingView view_of(const Request &r) {
  fps::PendingView v;
  v.q = r.q;
  v.k = r.keff;
  v.submit_ns = r.arrival_ns;  // deadlines run from arrival
  v.deadline_us = r.deadline_us;
  return v;
}

static void run_slot(fps_server *S, Slot *slot, bool reserve) {
  (void)hipSetDevice(S->lib->device);
  for (;;) {
    std::vector<std::shared_ptr<Request>> batch;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      auto ready = [&] {
        if (S->stopping || S->pending.empty()) return S->stopping;
        return !reserve || fps::reserve_may_run(view_of(*S->pending.front()), S->pending_q,
                                                S->cfg.max_batch_queries, now_ns(), S->cost);
      };
      if (reserve) {
        // the queue can fall behind without a notification: look again
        while (!ready()) S->cv_work.wait_for(lk, std::chrono::microseconds(500));
      } else {
        S->cv_work.wait(lk, ready);
      }
      if (S->pending.empty() && S->stopping) return;
      if (S->cfg.max_wait_us > 0) {
        // give a small batch a bounded chance to grow
        const uint64_t oldest = S->pending.front()->submit_ns;
        const uint64_t until = oldest + (uint64_t)S->cfg.max_wait_us * 1000ull;
        while (!S->stopping && S->pending_q < S->cfg.max_batch_queries) {
          const uint64_t now = now_ns();
          if (now >= until) break;
          S->cv_work.wait_for(lk, std::chrono::nanoseconds(until - now));
        }
        if (S->pending.empty()) continue;
      }
      // a prefix of the queue (batcher.h), shrunk until it fits the slot
      size_t n = fps::batch_prefix(
          S->pending.size(), [&](size_t i) { return view_of(*S->pending[i]); }, now_ns(),
          S->cfg.max_batch_queries, S->cfg.deadline_cap != 0, S->cost);
      auto fits = [&](size_t m) {
        slot->kk.clear();
        slot->mm.clear();
        for (size_t i = 0; i < m; ++i) {
          const Request &r = *S->pending[i];
          slot->kk.insert(slot->kk.end(), r.q, r.k);
          slot->mm.insert(slot->mm.end(), r.q, r.mask);
        }
        Plan P;
        try {
          return fps_plan(S->lib, (uint32_t)slot->kk.size(), slot->kk.data(), slot->mm.data(),
                          &P) == FPS_OK &&
                 P.total_bytes <= slot->ws_bytes;
        } catch (const std::bad_alloc &) {
          return false;
        }
      };
      if (n > 1 && !fits(n)) {
        // the longest prefix that fits (one request always does: admission)
        size_t lo = 1, hi = n - 1;
        while (lo < hi) {
          const size_t mid = (lo + hi + 1) / 2;
          if (fits(mid))
            lo = mid;
          else
            hi = mid - 1;
        }
        n = lo;
      }
      for (size_t i = 0; i < n; ++i) {
        S->pending_q -= S->pending.front()->q;
        batch.push_back(S->pending.front());
        S->pending.pop_front();
      }
      if (!S->pending.empty()) S->cv_work.notify_all();
    }
    // run the batch
    uint32_t qsum = 0;
    double weight = 0;
    for (auto &r : batch) {
      qsum += r->q;
      weight += fps::CostModel::weight(r->q, r->keff);
    }
    std::vector<uint64_t> &qs = slot->qs;
    std::vector<uint32_t> &kk = slot->kk, &mm = slot->mm;
    uint64_t cap = 0;
    for (auto &r : batch) cap += (uint64_t)r->q * r->keff;
    const uint64_t t0 = now_ns();
    uint32_t bid;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      bid = S->next_batch++;
    }
    fps_clear_error();
    fps_status rc = FPS_OK;
    std::string err;
    bool untuned = false;
    try {
      qs.clear();
      kk.clear();
      mm.clear();
      for (auto &r : batch) {
        qs.insert(qs.end(), r->queries.begin(), r->queries.end());
        kk.insert(kk.end(), r->q, r->k);
        mm.insert(mm.end(), r->q, r->mask);
      }
      if (slot->hits.size() < std::max<uint64_t>(cap, 1))
        slot->hits.resize(std::max<uint64_t>(cap, 1));
      if (slot->off.size() < (size_t)qsum + 1) slot->off.resize((size_t)qsum + 1);
      rc = fps_search_impl(S->lib, &slot->ctx, qs.data(), qsum, kk.data(), mm.data(), slot->ws,
                           slot->ws_bytes, slot->hits.data(), cap, slot->off.data(),
                           slot->stream, FPS_PATH_AUTO, false);
      if (rc) err = fps_last_error();
      untuned = slot->ctx.last_untuned;
    } catch (const std::bad_alloc &) {
      rc = FPS_E_NOMEM;
      err = "host allocation failed while running a batch";
    }
    const fps_hit *hits = slot->hits.data();
    const uint64_t *off = slot->off.data();
    const uint64_t t1 = now_ns();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      uint32_t base = 0;
      for (auto &r : batch) {
        r->start_ns = t0;
        r->done_ns = t1;
        r->batch_id = bid;
        r->batch_queries = qsum;
        r->status = rc;
        r->error = err;
        if (!rc) {
          try {
            r->offsets.resize(r->q + 1);
            const uint64_t h0 = off[base];
            for (uint32_t i = 0; i <= r->q; ++i) r->offsets[i] = off[base + i] - h0;
            r->hits.assign(hits + h0, hits + off[base + r->q]);
          } catch (const std::bad_alloc &) {
            r->status = FPS_E_NOMEM;
            r->error = "host allocation failed while copying a result";
            r->offsets.clear();
            r->hits.clear();
          }
        }
        base += r->q;
        r->done = true;
        S->admitted_bytes -= r->bytes;
        const double us = (double)(t1 - r->arrival_ns) / 1000.0;
        ring_push(S->lat_us, S->lat_next, us);
        S->st_requests++;
        S->st_queries += r->q;
        if (r->deadline_us && us > (double)r->deadline_us) S->st_misses++;
      }
      S->st_batches++;
      S->st_batch_q += qsum;
      S->st_untuned += untuned ? 1u : 0u;
      if (!rc) S->cost.observe(weight, (double)(t1 - t0) / 1000.0);
    }
    S->cv_done.notify_all();
    S->cv_room.notify_all();
  }
}

extern "C" fps_status fps_server_create(fps_library *lib, const fps_server_config *cfg,
                                        void *workspace, size_t ws_bytes, fps_server **out) {
  fps_clear_error();
  if (!lib || !cfg || !workspace || !out) return fps_fail(FPS_E_ARG, "NULL argument");
  if (cfg->n_streams < 1 || cfg->n_streams > 8)
    return fps_fail(FPS_E_ARG, "n_streams must be 1..8");
  if (cfg->max_batch_queries < 1) return fps_fail(FPS_E_ARG, "max_batch_queries must be >= 1");
  if (cfg->reserve_streams >= cfg->n_streams)
    return fps_fail(FPS_E_ARG, "reserve_streams must be below n_streams");
  if (cfg->pool_bytes == 0 || cfg->pool_bytes > ws_bytes)
    return fps_fail(FPS_E_ARG, "pool_bytes must be in 1..ws_bytes");
  if (((uintptr_t)workspace & 255) != 0)
    return fps_fail(FPS_E_ARG, "workspace must be 256-byte aligned");
  auto S = std::make_unique<fps_server>();
  S->lib = lib;
  S->cfg = *cfg;
  const size_t slot_bytes = (cfg->pool_bytes / cfg->n_streams) & ~(size_t)255;
  for (uint32_t i = 0; i < cfg->n_streams; ++i) {
    auto sl = std::make_unique<Slot>();
    if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess) {
      sl->stream = nullptr;
      return fps_fail(FPS_E_DEVICE, "hipStreamCreateWithFlags failed");
    }
    sl->ws = (uint8_t *)workspace + i * slot_bytes;
    sl->ws_bytes = slot_bytes;
    fps_status rc = sl->ctx.init();
    if (rc) return rc;
    S->slots.push_back(std::move(sl));
  }
  // Tune every batch shape of 1, 2, 4, ... queries up to max_batch_queries with
  // each expected k, on slot 0, before any request arrives.  A shape whose
  // workspace exceeds a slot never runs as one batch and is skipped.
  if (cfg->tune_k && cfg->n_tune_k && lib->path == FPS_PATH_AUTO) {
    Slot *s0 = S->slots[0].get();
    for (uint32_t t = 0; t < cfg->n_tune_k; ++t) {
      for (uint64_t q = 1;; q *= 2) {
        const uint32_t qq = (uint32_t)std::min<uint64_t>(q, cfg->max_batch_queries);
        std::vector<uint32_t> kk(qq, cfg->tune_k[t]);
        Plan P;
        fps_status rc = fps_plan(lib, qq, kk.data(), nullptr, &P);
        if (rc) return rc;
        if (P.total_bytes <= s0->ws_bytes) {
          rc = fps_tune_impl(lib, &s0->ctx, qq, kk.data(), nullptr, s0->ws, s0->ws_bytes,
                             s0->stream);
          if (rc) return rc;
        }
        if (qq >= cfg->max_batch_queries) break;
      }
    }
  }
  for (uint32_t i = 0; i < cfg->n_streams; ++i)
    S->slots[i]->worker = std::thread(run_slot, S.get(), S->slots[i].get(),
                                      i >= cfg->n_streams - cfg->reserve_streams);
  *out = S.release();
  return FPS_OK;
}

extern "C" uint64_t fps_clock_ns(void) { return now_ns(); }

extern "C" fps_status fps_server_submit(fps_server *srv, const uint64_t *queries, uint32_t q,
                                        uint32_t k, uint32_t mask, uint32_t deadline_us,
                                        uint64_t arrival_ns, int nonblocking, uint64_t *ticket) {
  const uint64_t entered = now_ns();
  fps_clear_error();
  if (!srv || !queries || !ticket || q == 0) return fps_fail(FPS_E_ARG, "bad argument");
  for (uint32_t i = 0; i < q; ++i)
    if ((queries[3 * i] & 1ull) || (queries[3 * i + 2] >> 39))
      return fps_fail(FPS_E_FINGERPRINT, "query %u has bit 0 or a bit above key 166 set", i);
  fps::RangeSet rs;
  {
    fps_status rc = fps_make_rangeset(srv->lib, mask, &rs);
    if (rc) return rc;
  }
  std::shared_ptr<Request> r;
  try {
    r = std::make_shared<Request>();
    r->queries.assign(queries, queries + 3 * (size_t)q);
  } catch (const std::bad_alloc &) {
    return fps_fail(FPS_E_NOMEM, "host allocation failed");
  }
  r->q = q;
  r->k = k;
  r->keff = (uint32_t)std::min<uint64_t>(k, rs.neff);
  r->mask = mask;
  r->deadline_us = deadline_us;
  r->arrival_ns = arrival_ns ? arrival_ns : entered;
  r->bytes = request_bytes(srv->lib, q, k, mask);
  if (r->bytes > srv->slots[0]->ws_bytes)
    return fps_fail(FPS_E_NOMEM, "request needs %zu workspace bytes, a slot has %zu", r->bytes,
                    srv->slots[0]->ws_bytes);
  std::unique_lock<std::mutex> lk(srv->mu);
  if (srv->stopping) return fps_fail(FPS_E_STATE, "server is stopping");
  auto fits = [&] { return srv->admitted_bytes + r->bytes <= srv->cfg.pool_bytes; };
  if (!fits()) {
    if (nonblocking) return fps_fail(FPS_E_BUSY, "admission pool is full");
    srv->cv_room.wait(lk, [&] { return fits() || srv->stopping; });
    if (srv->stopping) return fps_fail(FPS_E_STATE, "server is stopping");
  }
  srv->admitted_bytes += r->bytes;
  r->ticket = srv->next_ticket++;
  r->submit_ns = now_ns();
  ring_push(srv->admit_us, srv->admit_next,
            r->submit_ns > r->arrival_ns ? (double)(r->submit_ns - r->arrival_ns) / 1000.0 : 0.0);
  srv->live[r->ticket] = r;
  srv->pending.push_back(r);
  srv->pending_q += q;
  *ticket = r->ticket;
  lk.unlock();
  srv->cv_work.notify_all();  // a reserve slot may take the wake-up and stay idle
  return FPS_OK;
}

// The request of a ticket once it is done (waits); null for an unknown ticket.
static std::shared_ptr<Request> wait_done(fps_server *srv, std::unique_lock<std::mutex> &lk,
                                          uint64_t ticket) {
  auto it = srv->live.find(ticket);
  if (it == srv->live.end()) return nullptr;
  std::shared_ptr<Request> r = it->second;
  srv->cv_done.wait(lk, [&] { return r->done; });
  return r;
}

extern "C" fps_status fps_server_result_size(fps_server *srv, uint64_t ticket, uint32_t *q,
                                             uint64_t *n_hits) {
  fps_clear_error();
  if (!srv) return fps_fail(FPS_E_ARG, "NULL server");
  std::unique_lock<std::mutex> lk(srv->mu);
  std::shared_ptr<Request> r = wait_done(srv, lk, ticket);
  if (!r) return fps_fail(FPS_E_ARG, "unknown ticket %llu", (unsigned long long)ticket);
  if (q) *q = r->q;
  if (n_hits) *n_hits = r->status ? 0 : (uint64_t)r->hits.size();
  return FPS_OK;
}

extern "C" fps_status fps_server_wait(fps_server *srv, uint64_t ticket, fps_hit *out,
                                      uint64_t out_capacity, uint64_t *out_offset,
                                      uint64_t offset_capacity, fps_request_stats *stats) {
  fps_clear_error();
  if (!srv || !out_offset) return fps_fail(FPS_E_ARG, "NULL argument");
  std::shared_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(srv->mu);
    r = wait_done(srv, lk, ticket);
    if (!r) return fps_fail(FPS_E_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    if (!r->status) {
      // check every buffer before the ticket is consumed
      if (offset_capacity < (uint64_t)r->q + 1)
        return fps_fail(FPS_E_ARG, "out_offset holds %llu entries, %u needed",
                        (unsigned long long)offset_capacity, r->q + 1);
      if (out_capacity < r->hits.size())
        return fps_fail(FPS_E_ARG, "out holds %llu hits, %zu needed",
                        (unsigned long long)out_capacity, r->hits.size());
      if (!r->hits.empty() && !out) return fps_fail(FPS_E_ARG, "NULL out");
    }
    srv->live.erase(ticket);
  }
  if (r->status) return fps_fail(r->status, "%s", r->error.c_str());
  if (!r->hits.empty()) std::memcpy(out, r->hits.data(), r->hits.size() * sizeof(fps_hit));
  std::memcpy(out_offset, r->offsets.data(), r->offsets.size() * sizeof(uint64_t));
  if (stats) {
    stats->arrival_ns = r->arrival_ns;
    stats->submit_ns = r->submit_ns;
    stats->start_ns = r->start_ns;
    stats->done_ns = r->done_ns;
    stats->batch_id = r->batch_id;
    stats->batch_queries = r->batch_queries;
  }
  return FPS_OK;
}

extern "C" fps_status fps_server_stats_get(fps_server *srv, fps_server_stats *st, int reset) {
  fps_clear_error();
  if (!srv || !st) return fps_fail(FPS_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  std::memset(st, 0, sizeof *st);
  st->requests = srv->st_requests;
  st->queries = srv->st_queries;
  st->batches = srv->st_batches;
  st->deadline_misses = srv->st_misses;
  st->mean_batch_queries = srv->st_batches ? (double)srv->st_batch_q / srv->st_batches : 0.0;
  st->cost_fixed_us = srv->cost.c0_us();
  st->cost_per_weight_us = srv->cost.c1_us();
  st->untuned_batches = srv->st_untuned;
  auto pct = [](std::vector<double> v, double p) {
    std::sort(v.begin(), v.end());
    size_t i = (size_t)std::ceil(p * (double)v.size());
    if (i > 0) --i;
    return v[std::min(i, v.size() - 1)];
  };
  if (!srv->lat_us.empty()) {
    st->p50_us = pct(srv->lat_us, 0.50);
    st->p99_us = pct(srv->lat_us, 0.99);
    st->max_us = *std::max_element(srv->lat_us.begin(), srv->lat_us.end());
  }
  if (!srv->admit_us.empty()) {
    st->admit_p50_us = pct(srv->admit_us, 0.50);
    st->admit_p99_us = pct(srv->admit_us, 0.99);
  }
  if (reset) {
    srv->lat_us.clear();
    srv->admit_us.clear();
    srv->lat_next = srv->admit_next = 0;
    srv->st_requests = srv->st_queries = srv->st_batches = srv->st_misses = srv->st_batch_q = 0;
    srv->st_untuned = 0;
  }
  return FPS_OK;
}

extern "C" fps_status fps_server_destroy(fps_server *srv) {
  fps_clear_error();
  if (!srv) return FPS_OK;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
  }
  srv->cv_work.notify_all();
  srv->cv_room.notify_all();
  for (auto &sl : srv->slots)
    if (sl->worker.joinable()) sl->worker.join();
  for (auto &sl : srv->slots) {
    (void)hipStreamSynchronize(sl->stream);
    (void)hipStreamDestroy(sl->stream);
    sl->stream = nullptr;
  }
  delete srv;
  return FPS_OK;
}
