// Host-side state of the C ABI shared by the runtime and the server.
#pragma once
#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

#include "fps_internal.h"


// Host state of one search in flight: pinned staging, timing events, counters.
// The handle owns one; every server slot owns its own, so slots can run
// concurrently on their own streams.
struct SearchCtx {
  void *h_params = nullptr;
  size_t h_params_bytes = 0;
  void *h_out = nullptr;
  size_t h_out_bytes = 0;
  void *h_out_dev = nullptr;     // device address of h_out (null: not mapped)
  const void *h_out_dev_of = nullptr;  // the h_out that h_out_dev belongs to
  // ev[0]/ev[1]: first and last kernel of a call; ev[2 + 2p], ev[3 + 2p]:
  // around the scan launches of phase p
  hipEvent_t ev[2 + 2 * fps::kMaxPhases] = {};
  fps_search_stats last{};
  uint32_t last_phases = 0;    // scan phases of the last launch sequence
  uint32_t last_timed = 0;     // bit p: the events around phase p were stamped
  uint32_t last_launches = 0;  // scan kernel launches of the last sequence
  bool last_untuned = false;   // the last call took the default kernel of an untimed shape
  bool last_total_timed = false;  // ev[0], ev[1] were stamped
  double sum_scan_ms = 0, sum_total_ms = 0;  // running sums since creation
  uint64_t sum_calls = 0, sum_launches = 0;
  // graph replay of repeated launch shapes (see run_search)
  static constexpr size_t kGraphs = 4, kSeen = 8;
  hipStream_t cap = nullptr;
  std::vector<std::pair<std::vector<uint64_t>, hipGraphExec_t>> graphs;
  std::vector<std::vector<uint64_t>> seen;
  uint32_t graph_failures = 0;
  fps_status init();
  ~SearchCtx();
};

// Batch shape for the autotuner: log2 of live queries, largest k, library size.
struct TuneKey {
  uint32_t q, k, n;
  bool operator<(const TuneKey &o) const { return std::tie(q, k, n) < std::tie(o.q, o.k, o.n); }
};

struct fps_library {
  uint64_t n = 0, np = 0;
  uint32_t nstrides = 0;
  uint64_t strides[FPS_MAX_STRIDES + 1] = {};
  uint64_t *dev = nullptr;  // caller-owned library arrays a, b, c, d (fps_internal.h)
  int device = 0;
  int cus = 256;
  fps_path path = FPS_PATH_AUTO;
  int variant = -1;  // matrix-core tile shape, -1 = tuner's choice
  double cand_scale = 1.0;
  uint64_t sample = fps::kDefaultBoundSample;  // records of the bound sample
  uint64_t phase_a = fps::kDefaultPhaseA;      // first phase boundary (0 = from the schedule)
  int force_fb = 0;
  bool timing = false;  // HIP events around the kernels of every call
  bool graphs = true;  // capture and replay repeated launch shapes
  SearchCtx ctx;  // staging of direct calls on this handle
  const uint64_t *ids = nullptr;  // caller-owned host id of every record (text loads), or null
  const uint64_t *ids_dev = nullptr;  // caller-owned device ids (text loads), or null
  // fps_hit_ids on a library whose ids stay in device memory: mapped pinned
  // staging of hit indices and ids (grown on demand), one call at a time
  std::mutex id_mu;
  void *id_stage = nullptr;
  size_t id_stage_bytes = 0;
  ~fps_library() {
    if (id_stage) (void)hipHostFree(id_stage);
  }
  std::mutex tune_mu;
  std::map<TuneKey, std::pair<fps_path, int>> tuned;
};

// A planned search: per-query parameters and the byte layout of the workspace.
struct Plan {
  uint32_t q = 0;
  std::vector<fps::RangeSet> rsets;
  std::vector<fps::QueryInfo> qinfo;
  std::vector<uint32_t> perm;
  std::vector<uint64_t> bounds;  // scan phase boundaries in records (last = UINT64_MAX)
  uint64_t total_cand = 0, total_out = 0, max_sample = 0, total_ctr = 0;
  size_t off_rsets = 0, off_qinfo = 0, off_perm = 0, off_qblocks = 0, off_qbitem = 0,
         off_bblocks = 0, params_bytes = 0;
  size_t off_bdone = 0, off_T = 0, off_ctr = 0, off_count = 0, off_flags = 0, off_hist = 0, off_cand = 0, off_out = 0,
         off_fbh = 0, off_fbo = 0, off_fbt = 0, total_bytes = 0;
};

fps_status fps_fail(fps_status s, const char *fmt, ...);
// Returns FPS_E_DEVICE with the HIP error text when a HIP call fails.
#define HIP_TRY(x)                                                                         \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) return fps_fail(FPS_E_DEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)
// A handle over caller-owned device memory for n records (strides validated,
// device queried, staging allocated); the records themselves are not written.
fps_status fps_library_new(uint64_t n, const uint64_t *stride_begin, uint32_t nstrides,
                           void *device_buf, size_t device_bytes, fps_library **out);
// Zeroes the padding records [n, np) of a new handle's arrays on stream s.
fps_status fps_library_zero_tail(fps_library *lib, hipStream_t s);
void fps_clear_error();
fps_status fps_make_rangeset(const fps_library *lib, uint32_t mask, fps::RangeSet *rs);
fps_status fps_plan(const fps_library *lib, uint32_t q, const uint32_t *k, const uint32_t *mask,
                    Plan *P);
fps_status fps_search_impl(fps_library *lib, SearchCtx *ctx, const uint64_t *queries, uint32_t q,
                           const uint32_t *k, const uint32_t *mask, void *workspace,
                           size_t ws_bytes, fps_hit *out, uint64_t out_capacity,
                           uint64_t *out_offset, hipStream_t s, fps_path forced,
                           bool may_tune);
// The autotuner for one batch shape (fps_tune) on the given context's stream.
fps_status fps_tune_impl(fps_library *lib, SearchCtx *ctx, uint32_t q, const uint32_t *k,
                         const uint32_t *mask, void *workspace, size_t ws_bytes, hipStream_t s);
