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
  size_t bytes = 0;  // workspace the request needs on its own
  uint64_t submit_ns = 0, start_ns = 0, done_ns = 0;
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
  std::vector<double> lat_us;
  size_t lat_next = 0;
  uint64_t st_requests = 0, st_queries = 0, st_batches = 0, st_misses = 0, st_batch_q = 0;
};

static size_t request_bytes(fps_library *lib, uint32_t q, uint32_t k, uint32_t mask) {
  std::vector<uint32_t> kk(q, k), mm(q, mask);
  Plan P;
  if (fps_plan(lib, q, kk.data(), mm.data(), &P)) return (size_t)-1;
  return P.total_bytes;
}

static fps::PendingView view_of(const Request &r) {
  fps::PendingView v;
  v.q = r.q;
  v.k = r.k;
  v.submit_ns = r.submit_ns;
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
        return fps_plan(S->lib, (uint32_t)slot->kk.size(), slot->kk.data(), slot->mm.data(),
                        &P) == FPS_OK &&
               P.total_bytes <= slot->ws_bytes;
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
      weight += fps::CostModel::weight(r->q, r->k);
    }
    std::vector<uint64_t> &qs = slot->qs;
    std::vector<uint32_t> &kk = slot->kk, &mm = slot->mm;
    qs.clear();
    kk.clear();
    mm.clear();
    uint64_t cap = 0;
    for (auto &r : batch) {
      qs.insert(qs.end(), r->queries.begin(), r->queries.end());
      kk.insert(kk.end(), r->q, r->k);
      mm.insert(mm.end(), r->q, r->mask);
      cap += (uint64_t)r->q * r->k;
    }
    if (slot->hits.size() < std::max<uint64_t>(cap, 1)) slot->hits.resize(std::max<uint64_t>(cap, 1));
    if (slot->off.size() < (size_t)qsum + 1) slot->off.resize((size_t)qsum + 1);
    fps_hit *hits = slot->hits.data();
    uint64_t *off = slot->off.data();
    const uint64_t t0 = now_ns();
    uint32_t bid;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      bid = S->next_batch++;
    }
    fps_clear_error();
    fps_status rc = fps_search_impl(S->lib, &slot->ctx, qs.data(), qsum, kk.data(), mm.data(),
                                    slot->ws, slot->ws_bytes, hits, cap, off, slot->stream,
                                    FPS_PATH_AUTO);
    const std::string err = rc ? std::string(fps_last_error()) : std::string();
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
          r->offsets.resize(r->q + 1);
          const uint64_t h0 = off[base];
          for (uint32_t i = 0; i <= r->q; ++i) r->offsets[i] = off[base + i] - h0;
          r->hits.assign(hits + h0, hits + off[base + r->q]);
        }
        base += r->q;
        r->done = true;
        S->admitted_bytes -= r->bytes;
        const double us = (double)(t1 - r->submit_ns) / 1000.0;
        if (S->lat_us.size() < fps_server::kLatWindow) {
          S->lat_us.push_back(us);
        } else {
          S->lat_us[S->lat_next] = us;
          S->lat_next = (S->lat_next + 1) % fps_server::kLatWindow;
        }
        S->st_requests++;
        S->st_queries += r->q;
        if (r->deadline_us && us > (double)r->deadline_us) S->st_misses++;
      }
      S->st_batches++;
      S->st_batch_q += qsum;
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
    if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess)
      return fps_fail(FPS_E_DEVICE, "hipStreamCreateWithFlags failed");
    sl->ws = (uint8_t *)workspace + i * slot_bytes;
    sl->ws_bytes = slot_bytes;
    fps_status rc = sl->ctx.init();
    if (rc) {
      (void)hipStreamDestroy(sl->stream);
      return rc;
    }
    S->slots.push_back(std::move(sl));
  }
  for (uint32_t i = 0; i < cfg->n_streams; ++i)
    S->slots[i]->worker = std::thread(run_slot, S.get(), S->slots[i].get(),
                                      i >= cfg->n_streams - cfg->reserve_streams);
  *out = S.release();
  return FPS_OK;
}

extern "C" fps_status fps_server_submit(fps_server *srv, const uint64_t *queries, uint32_t q,
                                        uint32_t k, uint32_t mask, uint32_t deadline_us,
                                        int nonblocking, uint64_t *ticket) {
  fps_clear_error();
  if (!srv || !queries || !ticket || q == 0) return fps_fail(FPS_E_ARG, "bad argument");
  for (uint32_t i = 0; i < q; ++i)
    if ((queries[3 * i] & 1ull) || (queries[3 * i + 2] >> 39))
      return fps_fail(FPS_E_FINGERPRINT, "query %u has bit 0 or a bit above key 166 set", i);
  {
    fps::RangeSet rs;
    fps_status rc = fps_make_rangeset(srv->lib, mask, &rs);
    if (rc) return rc;
  }
  auto r = std::make_shared<Request>();
  r->queries.assign(queries, queries + 3 * (size_t)q);
  r->q = q;
  r->k = k;
  r->mask = mask;
  r->deadline_us = deadline_us;
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
  srv->live[r->ticket] = r;
  srv->pending.push_back(r);
  srv->pending_q += q;
  *ticket = r->ticket;
  lk.unlock();
  srv->cv_work.notify_all();  // a reserve slot may take the wake-up and stay idle
  return FPS_OK;
}

extern "C" fps_status fps_server_wait(fps_server *srv, uint64_t ticket, fps_hit *out,
                                      uint64_t out_capacity, uint64_t *out_offset,
                                      fps_request_stats *stats) {
  fps_clear_error();
  if (!srv || !out_offset) return fps_fail(FPS_E_ARG, "NULL argument");
  std::shared_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->live.find(ticket);
    if (it == srv->live.end()) return fps_fail(FPS_E_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    r = it->second;
    srv->cv_done.wait(lk, [&] { return r->done; });
    srv->live.erase(ticket);
  }
  if (r->status) return fps_fail(r->status, "%s", r->error.c_str());
  if (out_capacity < r->hits.size())
    return fps_fail(FPS_E_ARG, "out holds %llu hits, %zu needed",
                    (unsigned long long)out_capacity, r->hits.size());
  if (!r->hits.empty()) {
    if (!out) return fps_fail(FPS_E_ARG, "NULL out");
    std::memcpy(out, r->hits.data(), r->hits.size() * sizeof(fps_hit));
  }
  std::memcpy(out_offset, r->offsets.data(), r->offsets.size() * sizeof(uint64_t));
  if (stats) {
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
  if (!srv->lat_us.empty()) {
    std::vector<double> v = srv->lat_us;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
      size_t i = (size_t)std::ceil(p * (double)v.size()) ;
      if (i > 0) --i;
      return v[std::min(i, v.size() - 1)];
    };
    st->p50_us = pct(0.50);
    st->p99_us = pct(0.99);
    st->max_us = v.back();
  }
  if (reset) {
    srv->lat_us.clear();
    srv->lat_next = 0;
    srv->st_requests = srv->st_queries = srv->st_batches = srv->st_misses = srv->st_batch_q = 0;
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
  }
  delete srv;
  return FPS_OK;
}
