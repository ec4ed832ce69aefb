// Host runtime of the C ABI (include/fps.h): library upload, workspace
// planning, the launch sequence of a search, the exact fallback, statistics and
// the batch-path autotuner.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <map>
#include <string>
#include <vector>

#include "fps_internal.h"
#include "runtime.h"

using namespace fps;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string t_err;

fps_status fps_fail(fps_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_err = buf;
  return s;
}

void fps_clear_error() { t_err.clear(); }

extern "C" const char *fps_last_error(void) { return t_err.c_str(); }


static inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

static void tune_load(fps_library *lib);
static fps_status scratch_setup(int device);
// Pinned staging (parameters, results) allocated when a library is loaded;
// the allocation-free search must fit it.
static constexpr size_t kNoAllocStaging = size_t(1) << 16;

static bool bad_fingerprint(const uint64_t *w) {
  return (w[0] & 1ull) != 0 || (w[2] >> 39) != 0;
}

// ---------------------------------------------------------------------------
// pinned staging
// ---------------------------------------------------------------------------
static fps_status ensure_pinned(void **p, size_t *have, size_t need) {
  if (*have >= need && *p) return FPS_OK;
  if (*p) {
    (void)hipHostFree(*p);
    *p = nullptr;
    *have = 0;
  }
  size_t n = align_up(std::max<size_t>(need, 1 << 16), 1 << 16);
  HIP_TRY(hipHostMalloc(p, n, hipHostMallocDefault));
  *have = n;
  return FPS_OK;
}

// ---------------------------------------------------------------------------
// library
// ---------------------------------------------------------------------------
extern "C" size_t fps_library_device_bytes(uint64_t n) {
  const uint64_t np = (n + kRowAlign - 1) / kRowAlign * kRowAlign;
  return (size_t)(np * kBytesPerRecord);
}


static Lib lib_view(const fps_library *lib) {
  Lib L;
  L.a = lib->dev;
  L.b = lib->dev + lib->np;
  L.c = (const uint32_t *)(lib->dev + 2 * lib->np);
  L.d = (const uint8_t *)((const uint32_t *)(lib->dev + 2 * lib->np) + lib->np);
  L.n = lib->n;
  L.np = lib->np;
  return L;
}

SearchCtx::~SearchCtx() {
  for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
  if (cap) (void)hipStreamDestroy(cap);
  if (h_params) (void)hipHostFree(h_params);
  if (h_out) (void)hipHostFree(h_out);
  for (auto &e : ev)
    if (e) (void)hipEventDestroy(e);
}

fps_status SearchCtx::init() {
  for (auto &e : ev)
    if (!e) HIP_TRY(hipEventCreate(&e));
  if (!cap) HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  return FPS_OK;
}

fps_status fps_library_new(uint64_t n, const uint64_t *stride_begin, uint32_t nstrides,
                           void *device_buf, size_t device_bytes, fps_library **out) {
  if (!device_buf || !out) return fps_fail(FPS_E_ARG, "NULL argument");
  if (n == 0 || n >= (1ull << 32)) return fps_fail(FPS_E_ARG, "n = %llu out of range", (unsigned long long)n);
  if (device_bytes < fps_library_device_bytes(n))
    return fps_fail(FPS_E_ARG, "device buffer of %zu bytes < %zu needed", device_bytes,
                    fps_library_device_bytes(n));
  if (((uintptr_t)device_buf & 255) != 0)
    return fps_fail(FPS_E_ARG, "device buffer must be 256-byte aligned");
  std::vector<uint64_t> st;
  if (!stride_begin) {
    st = {0, n};
  } else {
    if (nstrides < 1 || nstrides > FPS_MAX_STRIDES)
      return fps_fail(FPS_E_ARG, "nstrides = %u out of range", nstrides);
    st.assign(stride_begin, stride_begin + nstrides + 1);
    if (st[0] != 0 || st[nstrides] != n)
      return fps_fail(FPS_E_ARG, "stride offsets must start at 0 and end at n");
    for (uint32_t s = 0; s < nstrides; ++s)
      if (st[s + 1] < st[s]) return fps_fail(FPS_E_ARG, "stride offsets must not decrease");
  }
  auto *L = new (std::nothrow) fps_library();
  if (!L) return fps_fail(FPS_E_NOMEM, "host allocation failed");
  L->n = n;
  L->np = (n + kRowAlign - 1) / kRowAlign * kRowAlign;
  L->nstrides = (uint32_t)st.size() - 1;
  std::copy(st.begin(), st.end(), L->strides);
  L->dev = (uint64_t *)device_buf;
  fps_status rc = FPS_OK;
  do {
    if (hipGetDevice(&L->device) != hipSuccess ||
        hipDeviceGetAttribute(&L->cus, hipDeviceAttributeMultiprocessorCount, L->device) !=
            hipSuccess) {
      rc = fps_fail(FPS_E_DEVICE, "cannot query the current device");
      break;
    }
    if ((rc = L->ctx.init())) break;
    // staging of the allocation-free search, sized once here
    if ((rc = ensure_pinned(&L->ctx.h_params, &L->ctx.h_params_bytes, kNoAllocStaging))) break;
    if ((rc = ensure_pinned(&L->ctx.h_out, &L->ctx.h_out_bytes, kNoAllocStaging))) break;
    if ((rc = scratch_setup(L->device))) break;
    tune_load(L);
  } while (0);
  if (rc) {
    delete L;
    return rc;
  }
  *out = L;
  return FPS_OK;
}

// Zeroes the records [n, np) of every array (they are scanned but never reported).
fps_status fps_library_zero_tail(fps_library *L, hipStream_t s) {
  uint8_t *da = (uint8_t *)L->dev, *db = da + 8 * L->np, *dc = db + 8 * L->np,
          *dd = dc + 4 * L->np;
  const uint64_t n = L->n, tail = L->np - n;
  if (tail &&
      (hipMemsetAsync(da + 8 * n, 0, 8 * tail, s) != hipSuccess ||
       hipMemsetAsync(db + 8 * n, 0, 8 * tail, s) != hipSuccess ||
       hipMemsetAsync(dc + 4 * n, 0, 4 * tail, s) != hipSuccess ||
       hipMemsetAsync(dd + n, 0, tail, s) != hipSuccess))
    return fps_fail(FPS_E_DEVICE, "hipMemsetAsync failed");
  return FPS_OK;
}

extern "C" fps_status fps_library_load(const uint64_t *host_words, uint64_t n,
                                       const uint64_t *stride_begin, uint32_t nstrides,
                                       void *device_buf, size_t device_bytes, void *stream,
                                       fps_library **out) {
  fps_clear_error();
  if (!host_words || !device_buf || !out) return fps_fail(FPS_E_ARG, "NULL argument");
  if (n < (1ull << 32))
    for (uint64_t i = 0; i < n; ++i)
      if (bad_fingerprint(host_words + 3 * i))
        return fps_fail(FPS_E_FINGERPRINT, "record %llu has bit 0 or a bit above key 166 set",
                        (unsigned long long)i);
  fps_library *L = nullptr;
  fps_status rc = fps_library_new(n, stride_begin, nstrides, device_buf, device_bytes, &L);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  do {
    // relabel and transpose record-major host words into the four device arrays
    const uint64_t CH = 1u << 20;
    void *pin = nullptr;
    size_t pin_bytes = 0;
    if ((rc = ensure_pinned(&pin, &pin_bytes, CH * kBytesPerRecord))) break;
    uint64_t *sa = (uint64_t *)pin, *sb = sa + CH;
    uint32_t *sc = (uint32_t *)(sb + CH);
    uint8_t *sd = (uint8_t *)(sc + CH);
    uint8_t *da = (uint8_t *)L->dev, *db = da + 8 * L->np, *dc = db + 8 * L->np,
            *dd = dc + 4 * L->np;
    for (uint64_t c0 = 0; c0 < n && !rc; c0 += CH) {
      const uint64_t c1 = std::min(n, c0 + CH), m = c1 - c0;
      if (hipStreamSynchronize(s) != hipSuccess) {
        rc = fps_fail(FPS_E_DEVICE, "stream synchronize failed");
        break;
      }
      for (uint64_t i = 0; i < m; ++i) {
        uint32_t c, d;
        relabel(host_words + 3 * (c0 + i), &sa[i], &sb[i], &c, &d);
        sc[i] = c;
        sd[i] = (uint8_t)d;
      }
      if (hipMemcpyAsync(da + 8 * c0, sa, 8 * m, hipMemcpyHostToDevice, s) != hipSuccess ||
          hipMemcpyAsync(db + 8 * c0, sb, 8 * m, hipMemcpyHostToDevice, s) != hipSuccess ||
          hipMemcpyAsync(dc + 4 * c0, sc, 4 * m, hipMemcpyHostToDevice, s) != hipSuccess ||
          hipMemcpyAsync(dd + c0, sd, m, hipMemcpyHostToDevice, s) != hipSuccess)
        rc = fps_fail(FPS_E_DEVICE, "upload failed");
    }
    if (!rc) rc = fps_library_zero_tail(L, s);
    if (!rc && hipStreamSynchronize(s) != hipSuccess)
      rc = fps_fail(FPS_E_DEVICE, "stream synchronize failed");
    (void)hipHostFree(pin);
  } while (0);
  if (rc) {
    delete L;
    return rc;
  }
  *out = L;
  return FPS_OK;
}

extern "C" fps_status fps_library_info(const fps_library *lib, uint64_t *n, uint32_t *nstrides,
                                       uint64_t *stride_begin) {
  fps_clear_error();
  if (!lib) return fps_fail(FPS_E_ARG, "NULL library");
  if (n) *n = lib->n;
  if (nstrides) *nstrides = lib->nstrides;
  if (stride_begin) std::copy(lib->strides, lib->strides + lib->nstrides + 1, stride_begin);
  return FPS_OK;
}

extern "C" fps_status fps_library_free(fps_library *lib) {
  fps_clear_error();
  delete lib;
  return FPS_OK;
}

extern "C" fps_status fps_set_path(fps_library *lib, fps_path path) {
  fps_clear_error();
  if (!lib) return fps_fail(FPS_E_ARG, "NULL library");
  if ((int)path < 0 || (int)path > (int)FPS_PATH_MFMA_F4)
    return fps_fail(FPS_E_ARG, "unknown path %d", (int)path);
  lib->path = path;
  return FPS_OK;
}

extern "C" fps_status fps_set_graphs(fps_library *lib, int enable) {
  fps_clear_error();
  if (!lib) return fps_fail(FPS_E_ARG, "NULL library");
  lib->graphs = enable != 0;
  return FPS_OK;
}

extern "C" fps_status fps_set_timing(fps_library *lib, int enable) {
  fps_clear_error();
  if (!lib) return fps_fail(FPS_E_ARG, "NULL library");
  lib->timing = enable != 0;
  return FPS_OK;
}

extern "C" fps_status fps_set_variant(fps_library *lib, int variant) {
  fps_clear_error();
  if (!lib) return fps_fail(FPS_E_ARG, "NULL library");
  if (variant < -1 || variant >= std::max(mfma_variants(), mfma_f4_variants()))
    return fps_fail(FPS_E_ARG, "variant %d out of range", variant);
  lib->variant = variant;
  return FPS_OK;
}

extern "C" fps_status fps_set_tuning(fps_library *lib, double candidate_scale,
                                     uint64_t sample_records, uint64_t phase_records,
                                     int force_fallback) {
  fps_clear_error();
  if (!lib) return fps_fail(FPS_E_ARG, "NULL library");
  if (!(candidate_scale > 0.0) || !std::isfinite(candidate_scale))
    return fps_fail(FPS_E_ARG, "candidate_scale must be positive");
  lib->cand_scale = candidate_scale;
  lib->sample = sample_records ? sample_records : kDefaultBoundSample;
  lib->phase_a = phase_records ? phase_records : kDefaultPhaseA;
  lib->force_fb = force_fallback;
  return FPS_OK;
}

extern "C" fps_status fps_last_search_stats(const fps_library *lib, fps_search_stats *stats) {
  fps_clear_error();
  if (!lib || !stats) return fps_fail(FPS_E_ARG, "NULL argument");
  *stats = lib->ctx.last;
  return FPS_OK;
}

// ---------------------------------------------------------------------------
// planning
// ---------------------------------------------------------------------------
fps_status fps_make_rangeset(const fps_library *lib, uint32_t mask, RangeSet *rs) {
  const uint32_t ns = lib->nstrides;
  uint32_t m = mask;
  if (mask == FPS_MASK_ALL) m = ns >= 32 ? 0xFFFFFFFFu : ((1u << ns) - 1u);
  if (m == 0) return fps_fail(FPS_E_ARG, "stride mask is zero");
  if (ns < 32 && (m >> ns) != 0)
    return fps_fail(FPS_E_ARG, "stride mask 0x%x names a stride the library lacks", mask);
  std::memset(rs, 0, sizeof *rs);
  rs->mask = m;
  for (uint32_t s = 0; s < ns; ++s) {
    if (!((m >> s) & 1u)) continue;
    const uint64_t b = lib->strides[s], e = lib->strides[s + 1];
    if (b == e) continue;
    if (rs->nranges > 0 && rs->end[rs->nranges - 1] == b) {
      rs->end[rs->nranges - 1] = e;  // adjacent strides form one range
    } else {
      rs->begin[rs->nranges] = b;
      rs->end[rs->nranges] = e;
      rs->nranges++;
    }
  }
  uint64_t v = 0, t1 = 0, tb = 0;
  for (uint32_t r = 0; r < rs->nranges; ++r) {
    rs->voff[r] = v;
    rs->t1off[r] = t1;
    rs->tboff[r] = tb;
    const uint64_t len = rs->end[r] - rs->begin[r];
    v += len;
    t1 += (rs->end[r] + kScanTile - 1) / kScanTile - rs->begin[r] / kScanTile;
    tb += (len + kBatchTile - 1) / kBatchTile;
  }
  for (uint32_t r = rs->nranges; r <= FPS_MAX_STRIDES; ++r) {
    rs->voff[r] = v;
    rs->t1off[r] = t1;
    rs->tboff[r] = tb;
  }
  rs->neff = v;
  return FPS_OK;
}

// Scan phases.  The first bound comes from a sample of S1 records.  When it is
// expected to admit few records (keff * neff / S1 <= kSinglePhaseAppends, at
// the largest keff and neff of the batch) one phase scans everything.
// Otherwise the scan proceeds in phases whose boundaries grow geometrically
// (b1 = G * S1, b2 = G * b1, ...), and after each phase the bound is refined to
// the keff-th smallest distance of the prefix scanned so far.  A phase
// [b_i, b_i+1) then appends about keff * (b_i+1 - b_i) / b_i records, times a
// small factor for ties at the bound.  G = A / keff clamped to Gmin..64, with
// A = 4096 and Gmin = 8 for batches of <= kSegQueries queries (appends are
// cheap there and a phase costs a launch) and A = 256, Gmin = 4 for larger
// batches, whose matrix-core scans pay for every append with a decode of the
// result tile.
static std::vector<uint64_t> phase_bounds(const fps_library *lib, uint64_t max_neff,
                                          uint64_t max_keff, uint64_t s1, uint32_t q) {
  std::vector<uint64_t> b{0};
  s1 = std::max<uint64_t>(s1, 1);
  if (!lib->phase_a && (double)max_keff * (double)max_neff <= (double)kSinglePhaseAppends * s1) {
    b.push_back(UINT64_MAX);
    return b;
  }
  const uint64_t A = q <= kSegQueries ? 4096 : 256;
  const uint64_t Gmin = q <= kSegQueries ? 8 : 4;
  const uint64_t G =
      std::min<uint64_t>(64, std::max<uint64_t>(Gmin, A / std::max<uint64_t>(max_keff, 1)));
  uint64_t a = lib->phase_a ? lib->phase_a : s1 * G;
  while (a < max_neff && b.size() < (size_t)kMaxPhases) {
    b.push_back(a);
    a = a > (UINT64_MAX / G) ? UINT64_MAX : a * G;
  }
  b.push_back(UINT64_MAX);
  return b;
}

// Candidate slots of a query: the expected appends of every phase (see
// phase_bounds), times 8 for distance ties, plus slack; at most neff.
static uint32_t capacity(const fps_library *lib, const std::vector<uint64_t> &bounds,
                         uint64_t keff, uint64_t neff, uint64_t sample) {
  if (keff == 0 || neff == 0) return 0;
  double expected = 0;
  for (size_t i = 0; i + 1 < bounds.size() && bounds[i] < neff; ++i) {
    const double lo = (double)bounds[i], hi = (double)std::min<uint64_t>(bounds[i + 1], neff);
    const double ref = i == 0 ? (double)std::max<uint64_t>(sample, 1) : lo;
    expected += (double)keff * (hi - lo) / ref;
  }
  double cap = lib->cand_scale * (8.0 * expected + 4096.0);
  cap = std::min(cap, (double)neff);
  cap = std::max(cap, 1.0);
  return (uint32_t)std::ceil(cap);
}

fps_status fps_plan(const fps_library *lib, uint32_t q, const uint32_t *k, const uint32_t *mask,
                    Plan *P) {
  if (q == 0) return fps_fail(FPS_E_ARG, "q must be >= 1");
  if (!k) return fps_fail(FPS_E_ARG, "NULL k");
  P->q = q;
  P->rsets.clear();
  P->qinfo.assign(q, QueryInfo{});
  std::map<uint32_t, uint32_t> seen;
  P->total_cand = 0;
  P->total_out = 0;
  P->max_sample = 0;
  P->total_ctr = 0;
  std::vector<uint32_t> rs_of(q);
  for (uint32_t i = 0; i < q; ++i) {
    const uint32_t m = mask ? mask[i] : FPS_MASK_ALL;
    auto it = seen.find(m);
    uint32_t id;
    if (it == seen.end()) {
      RangeSet rs;
      fps_status rc = fps_make_rangeset(lib, m, &rs);
      if (rc) return rc;
      id = (uint32_t)P->rsets.size();
      P->rsets.push_back(rs);
      seen[m] = id;
    } else {
      id = it->second;
    }
    rs_of[i] = id;
  }
  uint64_t max_neff = 0, max_keff = 0;
  for (uint32_t i = 0; i < q; ++i) {
    const uint64_t neff = P->rsets[rs_of[i]].neff;
    const uint64_t keff = std::min<uint64_t>(k[i], neff);
    if (keff) max_neff = std::max(max_neff, neff);
    max_keff = std::max(max_keff, keff);
  }
  const uint64_t s1 = lib->sample;
  P->bounds = phase_bounds(lib, max_neff, max_keff, s1, q);
  for (uint32_t i = 0; i < q; ++i) {
    const RangeSet &rs = P->rsets[rs_of[i]];
    QueryInfo &qi = P->qinfo[i];
    qi.rset = rs_of[i];
    qi.keff = (uint32_t)std::min<uint64_t>(k[i], rs.neff);
    qi.sample = std::min<uint64_t>(s1, rs.neff);
    const uint32_t base_cap = capacity(lib, P->bounds, qi.keff, rs.neff, qi.sample);
    // Small batches: kSegments segments sharing base_cap, plus a spill area of
    // base_cap (appends are spread over the segments' counters).
    qi.nseg = (q <= kSegQueries && qi.keff > 0) ? kSegments : 1u;
    if (qi.nseg > 1) {
      qi.segcap = (base_cap + kSegments - 1) / kSegments;
      qi.spillcap = base_cap;
      qi.cap = qi.nseg * qi.segcap + qi.spillcap;
    } else {
      qi.segcap = base_cap;
      qi.spillcap = 0;
      qi.cap = base_cap;
    }
    qi.ctr_off = (uint32_t)P->total_ctr;
    P->total_ctr += qi.nseg > 1 ? (uint64_t)(qi.nseg + 1) * kCtrStride : 1u;
    qi.cand_off = P->total_cand;
    qi.out_off = P->total_out;
    P->total_cand += qi.cap;
    P->total_out += qi.keff;
    if (qi.keff) P->max_sample = std::max(P->max_sample, qi.sample);
  }
  // sizes: parameter region (uploaded), then device-computed state
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  // the parameter region is packed (16-byte fields) so that a small plan fits
  // a kernel argument
  auto take16 = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 16);
    return o;
  };
  const size_t maxqb = (size_t)q + P->rsets.size() + 1;
  P->off_rsets = take16(P->rsets.size() * sizeof(RangeSet));
  P->off_qinfo = take16((size_t)q * sizeof(QueryInfo));
  P->off_perm = take16((size_t)q * sizeof(uint32_t));
  P->off_qblocks = take16(maxqb * sizeof(QBlock));
  P->off_qbitem = take16((size_t)kMaxPhases * (maxqb + 1) * sizeof(uint64_t));
  P->off_bblocks = take16(maxqb * sizeof(QBlock));
  P->params_bytes = off;
  off = align_up(off, 256);
  P->off_bdone = take(maxqb * 4);
  P->off_T = take((size_t)q * 4);
  P->off_ctr = take(P->total_ctr * 4);
  P->off_hist = take((size_t)q * kHistCopies * kBins * 4);
  P->off_cand = take(P->total_cand * sizeof(uint64_t));
  // count, flags and the hits are contiguous: one copy brings them back
  P->off_count = take((size_t)q * 4);
  P->off_flags = take((size_t)q * 4);
  P->off_out = take(P->total_out * sizeof(fps_hit));
  P->off_fbh = take((size_t)kFbWaves * kBins * 4);
  P->off_fbo = take((size_t)kFbWaves * kBins * 4);
  P->off_fbt = take((size_t)kBins * 4);
  P->total_bytes = off;
  return FPS_OK;
}

extern "C" fps_status fps_workspace_bytes(const fps_library *lib, uint32_t q, const uint32_t *k,
                                          const uint32_t *mask, size_t *bytes) {
  fps_clear_error();
  if (!lib || !bytes) return fps_fail(FPS_E_ARG, "NULL argument");
  Plan P;
  fps_status rc = fps_plan(lib, q, k, mask, &P);
  if (rc) return rc;
  *bytes = P.total_bytes;
  return FPS_OK;
}

// Groups queries by RangeSet into blocks of at most `qbs` queries; fills perm,
// the blocks, and for every scan phase the prefix of work items (batch tiles of
// the phase) over the blocks: items[p * (nblocks + 1) + b].  group_k: the rows
// of a RangeSet in order of k (for a kernel whose blocks take the work items
// round robin, so that blocks of candidate-heavy large-k rows do not set the
// grid's tail).
static void fps_make_blocks(Plan *P, uint32_t qbs, const std::vector<uint64_t> &tile_bounds,
                            bool group_k, std::vector<QBlock> *blocks,
                            std::vector<uint64_t> *items) {
  P->perm.clear();
  blocks->clear();
  for (uint32_t r = 0; r < P->rsets.size(); ++r) {
    const uint32_t first = (uint32_t)P->perm.size();
    for (uint32_t i = 0; i < P->q; ++i)
      if (P->qinfo[i].rset == r && P->qinfo[i].keff > 0) P->perm.push_back(i);
    // Every run of 32 rows samples the whole range of k: sorted by k, then laid
    // out with stride W = ceil(n / 32) (sorted elements g, g + W, g + 2W, ...
    // for g = 0, 1, ...).  A matrix-core wave decodes a result tile whenever
    // any of its rows has a candidate, and a block's work items take as long
    // as its busiest wave; queries arriving in runs of one k (a batch of
    // concatenated requests) would otherwise gather the candidate-heavy
    // large-k rows in a few blocks, whose items then set the grid's tail.
    {
      std::vector<uint32_t> sorted(P->perm.begin() + first, P->perm.end());
      std::stable_sort(sorted.begin(), sorted.end(), [&](uint32_t x, uint32_t y) {
        return P->qinfo[x].keff < P->qinfo[y].keff;
      });
      const size_t n = sorted.size(), W = group_k ? 1 : (n + 31) / 32;
      size_t o = first;
      for (size_t g = 0; g < W; ++g)
        for (size_t j = g; j < n; j += W) P->perm[o++] = sorted[j];
    }
    const uint32_t cnt = (uint32_t)P->perm.size() - first;
    const RangeSet &rs = P->rsets[r];
    for (uint32_t f = 0; f < cnt; f += qbs) {
      QBlock b{};
      b.first = first + f;
      b.count = std::min(qbs, cnt - f);
      b.rset = r;
      b.tiles = (uint32_t)rs.tboff[rs.nranges];
      blocks->push_back(b);
    }
  }
  // queries with keff = 0 go last (never scanned)
  for (uint32_t i = 0; i < P->q; ++i)
    if (P->qinfo[i].keff == 0) P->perm.push_back(i);
  const size_t nb = blocks->size(), np = tile_bounds.size() - 1;
  items->assign(np * (nb + 1), 0);
  for (size_t p = 0; p < np; ++p) {
    uint64_t acc = 0;
    for (size_t b = 0; b < nb; ++b) {
      (*items)[p * (nb + 1) + b] = acc;
      const uint64_t t = (*blocks)[b].tiles;
      acc += std::min(tile_bounds[p + 1], t) - std::min(tile_bounds[p], t);
    }
    (*items)[p * (nb + 1) + nb] = acc;
  }
}

// ---------------------------------------------------------------------------
// search
// ---------------------------------------------------------------------------
static Workspace ws_view(const Plan &P, uint8_t *base) {
  Workspace w{};
  w.rsets = (RangeSet *)(base + P.off_rsets);
  w.qinfo = (QueryInfo *)(base + P.off_qinfo);
  w.perm = (uint32_t *)(base + P.off_perm);
  w.qblocks = (QBlock *)(base + P.off_qblocks);
  w.qb_item = (uint64_t *)(base + P.off_qbitem);
  w.bblocks = (QBlock *)(base + P.off_bblocks);
  w.bdone = (uint32_t *)(base + P.off_bdone);
  w.T = (uint32_t *)(base + P.off_T);
  w.ctr = (uint32_t *)(base + P.off_ctr);
  w.count = (uint32_t *)(base + P.off_count);
  w.flags = (uint32_t *)(base + P.off_flags);
  w.hist = (uint32_t *)(base + P.off_hist);
  w.cand = (uint64_t *)(base + P.off_cand);
  w.out = (fps_hit *)(base + P.off_out);
  w.fb_wave_hist = (uint32_t *)(base + P.off_fbh);
  w.fb_wave_off = (uint32_t *)(base + P.off_fbo);
  w.fb_bin_total = (uint32_t *)(base + P.off_fbt);
  return w;
}

static fps_status launch_search(fps_library *lib, SearchCtx *ctx, Plan &P, fps_path path,
                                int variant, uint8_t *wsbase, hipStream_t s, bool timed,
                                bool capturing = false, bool d2h = false, bool host_only = false);
static fps_status resolve_path(fps_library *lib, SearchCtx *ctx, Plan &P, fps_path requested,
                               uint8_t *wsb, hipStream_t s, bool may_tune, fps_path *path,
                               int *variant);

// Timing events.  Inside a stream capture an event-record node is added after
// the current capture frontier and the capture continues from it, so replays of
// the graph record the events like an eager launch does.
static fps_status record(hipEvent_t e, hipStream_t s, bool capturing) {
  if (!capturing) {
    HIP_TRY(hipEventRecord(e, s));
    return FPS_OK;
  }
  hipStreamCaptureStatus st;
  unsigned long long id = 0;
  hipGraph_t g = nullptr;
  const hipGraphNode_t *deps = nullptr;
  size_t ndeps = 0;
  HIP_TRY(hipStreamGetCaptureInfo_v2(s, &st, &id, &g, &deps, &ndeps));
  if (st != hipStreamCaptureStatusActive || !g)
    return fps_fail(FPS_E_DEVICE, "stream is not capturing");
  hipGraphNode_t node = nullptr;
  HIP_TRY(hipGraphAddEventRecordNode(&node, g, deps, ndeps, e));
  HIP_TRY(hipStreamUpdateCaptureDependencies(s, &node, 1, hipStreamSetCaptureDependencies));
  return FPS_OK;
}

// Bytes brought back after a search: per-query counts and flags, then the hits.
static size_t back_bytes(const Plan &P) {
  return P.off_out + P.total_out * sizeof(fps_hit) - P.off_count;
}

// Enqueues the whole search of a planned batch on stream s (no host sync):
// parameter upload, prep, bound, the scan phases with refines, select, and
// with d2h the copy of counts, flags and hits into the pinned staging.  Also
// used under stream capture (capturing = true) to record a graph.
static fps_status launch_search(fps_library *lib, SearchCtx *ctx, Plan &P, fps_path path,
                                int variant, uint8_t *wsbase, hipStream_t s, bool timed,
                                bool capturing, bool d2h, bool host_only) {
  const Workspace ws = ws_view(P, wsbase);
  const Lib L = lib_view(lib);
  // scan phases in tiles of the single-query kernel and of the batched kernels
  const size_t nphases = P.bounds.size() - 1;
  std::vector<uint64_t> t1b(nphases + 1), tbb(nphases + 1);
  for (size_t i = 0; i <= nphases; ++i) {
    const uint64_t b = P.bounds[i];
    t1b[i] = b == UINT64_MAX ? UINT64_MAX : (b + kScanTile - 1) / kScanTile;
    tbb[i] = b == UINT64_MAX ? UINT64_MAX : (b + kBatchTile - 1) / kBatchTile;
  }
  // blocks for the bound kernel and for the batched scan
  std::vector<QBlock> bblocks, qblocks;
  std::vector<uint64_t> bitems, qitems;
  // the fp4 kernel takes its work items round robin and its rows grouped by k
  const bool group_k = path == FPS_PATH_MFMA_F4;
  fps_make_blocks(&P, kBoundQBlock, tbb, group_k, &bblocks, &bitems);
  const uint32_t qbs = path == FPS_PATH_MFMA_I8   ? mfma_qblock(variant)
                       : path == FPS_PATH_MFMA_F4 ? mfma_f4_qblock(variant)
                                                  : (uint32_t)kPopQBlock;
  fps_make_blocks(&P, qbs, tbb, group_k, &qblocks, &qitems);
  const uint32_t nqb = (uint32_t)qblocks.size();
  // parameter upload
  fps_status rc = ensure_pinned(&ctx->h_params, &ctx->h_params_bytes, P.params_bytes);
  if (rc) return rc;
  uint8_t *h = (uint8_t *)ctx->h_params;
  std::memcpy(h + P.off_rsets, P.rsets.data(), P.rsets.size() * sizeof(RangeSet));
  std::memcpy(h + P.off_qinfo, P.qinfo.data(), P.q * sizeof(QueryInfo));
  std::memcpy(h + P.off_perm, P.perm.data(), P.q * sizeof(uint32_t));
  std::memcpy(h + P.off_qblocks, qblocks.data(), qblocks.size() * sizeof(QBlock));
  std::memcpy(h + P.off_qbitem, qitems.data(), qitems.size() * sizeof(uint64_t));
  std::memcpy(h + P.off_bblocks, bblocks.data(), bblocks.size() * sizeof(QBlock));
  // Scan launches of every phase: the single path launches once per query whose
  // range reaches into the phase, the batched paths once per nonempty phase.
  std::vector<std::vector<uint32_t>> phase_q(nphases);
  ctx->last_phases = (uint32_t)nphases;
  ctx->last_launches = 0;
  ctx->last_timed = 0;
  for (size_t p = 0; p < nphases; ++p) {
    uint32_t n = 0;
    if (path == FPS_PATH_SINGLE) {
      for (uint32_t i = 0; i < P.q; ++i) {
        const QueryInfo &qi = P.qinfo[i];
        const RangeSet &rs = P.rsets[qi.rset];
        const uint64_t tiles = rs.t1off[rs.nranges];
        if (qi.keff && std::min(t1b[p + 1], tiles) > std::min(t1b[p], tiles))
          phase_q[p].push_back(i);
      }
      n = (uint32_t)phase_q[p].size();
    } else {
      n = qitems[p * (nqb + 1) + nqb] > 0 ? 1u : 0u;
    }
    ctx->last_launches += n;
    // eager launches stamp the events of a phase only if it launches; a graph
    // holds event nodes for every phase
    if (timed && (n > 0 || capturing || host_only)) ctx->last_timed |= 1u << p;
  }
  ctx->last_total_timed = timed;
  if (host_only) return FPS_OK;
  // Direct mode (eager launches of a small plan): the parameter block travels
  // as an argument of the prep kernel and select writes counts, flags and hits
  // straight into the pinned staging buffer -- no copy commands on the stream.
  // Graph replays need the copies (their kernel arguments are frozen).
  const bool direct = !capturing && d2h && P.params_bytes <= kInlineParams &&
                      back_bytes(P) <= ctx->h_out_bytes && ctx->h_out_dev;
  HostBack hb{nullptr, nullptr, nullptr};
  // Eager launches carry their timing events (stamped by the dispatches, no
  // marker packets); under capture the events are graph nodes.
  const LaunchEv none{};
  const bool mark = timed && capturing;  // event nodes of a graph
  const bool stamp = timed && !capturing;  // events carried by eager launches
  if (mark && (rc = record(ctx->ev[0], s, true))) return rc;
  const LaunchEv ev_first = stamp ? LaunchEv{ctx->ev[0], nullptr} : none;
  if (direct) {
    InlineParams ip;
    ip.bytes = align_up(P.params_bytes, 8);
    std::memcpy(ip.w, h, ip.bytes);
    launch_prep_inline(ws, P.q, (uint32_t)bblocks.size(), (uint32_t)P.total_ctr, wsbase, ip, s,
                       ev_first);
    uint8_t *hd = (uint8_t *)ctx->h_out_dev;
    hb.count = (uint32_t *)hd;
    hb.flags = (uint32_t *)(hd + (P.off_flags - P.off_count));
    hb.hits = (fps_hit *)(hd + (P.off_out - P.off_count));
  } else {
    HIP_TRY(hipMemcpyAsync(wsbase, h, P.params_bytes, hipMemcpyHostToDevice, s));
    launch_prep(ws, P.q, (uint32_t)bblocks.size(), (uint32_t)P.total_ctr, s, ev_first);
  }
  launch_bound(L, ws, (uint32_t)bblocks.size(), P.max_sample, s);
  for (size_t p = 0; p < nphases; ++p) {
    if (p > 0) launch_refine(ws, P.q, s);
    hipEvent_t e0 = ctx->ev[2 + 2 * p], e1 = ctx->ev[3 + 2 * p];
    if (mark && (rc = record(e0, s, true))) return rc;
    if (path == FPS_PATH_SINGLE) {
      const std::vector<uint32_t> &qs = phase_q[p];
      for (size_t j = 0; j < qs.size(); ++j) {
        const QueryInfo &qi = P.qinfo[qs[j]];
        const RangeSet &rs = P.rsets[qi.rset];
        const uint64_t tiles = rs.t1off[rs.nranges];
        LaunchEv e{};
        if (stamp) {
          if (j == 0) e.start = e0;
          if (j + 1 == qs.size()) e.stop = e1;
        }
        launch_scan_single(L, ws, qs[j], std::min(t1b[p], tiles), std::min(t1b[p + 1], tiles),
                           lib->cus, s, e);
      }
    } else {
      const uint64_t *item_off = ws.qb_item + p * (nqb + 1);
      const uint64_t items = qitems[p * (nqb + 1) + nqb];
      const LaunchEv e = stamp ? LaunchEv{e0, e1} : none;
      if (path == FPS_PATH_POPCOUNT)
        launch_scan_popcount(L, ws, nqb, item_off, tbb[p], items, lib->cus, s, e);
      else if (path == FPS_PATH_MFMA_F4)
        launch_scan_mfma_f4(L, ws, nqb, item_off, tbb[p], items, lib->cus, variant, s, e);
      else
        launch_scan_mfma_i8(L, ws, nqb, item_off, tbb[p], items, lib->cus, variant, s, e);
    }
    if (mark && (rc = record(e1, s, true))) return rc;
  }
  HIP_TRY(hipGetLastError());
  launch_select(ws, P.q, hb, s, stamp ? LaunchEv{nullptr, ctx->ev[1]} : none);
  HIP_TRY(hipGetLastError());
  if (mark && (rc = record(ctx->ev[1], s, true))) return rc;
  if (d2h && !direct) {
    if ((rc = ensure_pinned(&ctx->h_out, &ctx->h_out_bytes, back_bytes(P)))) return rc;
    HIP_TRY(hipMemcpyAsync(ctx->h_out, wsbase + P.off_count, back_bytes(P), hipMemcpyDeviceToHost,
                           s));
  }
  return FPS_OK;
}

// Everything a captured launch sequence depends on besides the parameter
// block's contents: if two calls have equal keys, the same graph serves both.
static std::vector<uint64_t> graph_key(const fps_library *lib, const SearchCtx *ctx,
                                       const Plan &P, fps_path path, int variant,
                                       const uint8_t *wsb) {
  std::vector<uint64_t> k = {(uint64_t)lib->timing, (uint64_t)(uintptr_t)wsb,
                             (uint64_t)(uintptr_t)lib->dev,
                             (uint64_t)(uintptr_t)ctx->h_params, (uint64_t)(uintptr_t)ctx->h_out,
                             (uint64_t)path, (uint64_t)variant, P.q, P.params_bytes,
                             P.total_bytes, P.max_sample, (uint64_t)lib->cus};
  k.insert(k.end(), P.bounds.begin(), P.bounds.end());
  for (const auto &rs : P.rsets) {
    k.push_back(rs.mask);
    k.push_back(rs.neff);
  }
  for (const auto &qi : P.qinfo) {
    k.push_back(qi.keff);
    k.push_back(qi.rset);
    k.push_back(qi.cap);
    k.push_back(qi.sample);
  }
  return k;
}

// Runs the launch sequence on stream s: replays a captured graph when the
// launch shape matches one (up to kGraphs per context, least recently used
// evicted), captures a graph when the shape was seen among the last kSeen
// calls, and otherwise launches eagerly.
static fps_status run_search(fps_library *lib, SearchCtx *ctx, Plan &P, fps_path path,
                             int variant, uint8_t *wsb, hipStream_t s) {
  fps_status rc;
  if ((rc = ensure_pinned(&ctx->h_params, &ctx->h_params_bytes, P.params_bytes))) return rc;
  if ((rc = ensure_pinned(&ctx->h_out, &ctx->h_out_bytes, back_bytes(P)))) return rc;
  if (ctx->h_out_dev_of != ctx->h_out) {
    void *d = nullptr;
    ctx->h_out_dev = hipHostGetDevicePointer(&d, ctx->h_out, 0) == hipSuccess ? d : nullptr;
    (void)hipGetLastError();
    ctx->h_out_dev_of = ctx->h_out;
  }
  ctx->last.graph = 0;
  // Graph replay serves the batched paths; for the single-query scan (a few
  // launches around one long kernel) direct launches measured faster.
  if (!lib->graphs || path == FPS_PATH_SINGLE)
    return launch_search(lib, ctx, P, path, variant, wsb, s, lib->timing, false, true);
  std::vector<uint64_t> key = graph_key(lib, ctx, P, path, variant, wsb);
  for (size_t i = 0; i < ctx->graphs.size(); ++i) {
    if (ctx->graphs[i].first != key) continue;
    // same shape: refresh the parameter block on the host, replay the graph
    if ((rc = launch_search(lib, ctx, P, path, variant, wsb, nullptr, lib->timing, false, false,
                            true)))
      return rc;
    std::rotate(ctx->graphs.begin() + i, ctx->graphs.begin() + i + 1, ctx->graphs.end());
    HIP_TRY(hipGraphLaunch(ctx->graphs.back().second, s));
    ctx->last.graph = 1;
    return FPS_OK;
  }
  if (std::find(ctx->seen.begin(), ctx->seen.end(), key) == ctx->seen.end()) {
    ctx->seen.push_back(std::move(key));
    if (ctx->seen.size() > SearchCtx::kSeen) ctx->seen.erase(ctx->seen.begin());
    return launch_search(lib, ctx, P, path, variant, wsb, s, lib->timing, false, true);
  }
  // a recent shape again: capture it (on any capture failure, launch eagerly)
  HIP_TRY(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
  rc = launch_search(lib, ctx, P, path, variant, wsb, ctx->cap, lib->timing, true, true);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(ctx->cap, &g);
  hipGraphExec_t ex = nullptr;
  hipError_t e2 = hipErrorUnknown;
  if (!rc && e == hipSuccess && g) e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (rc || e != hipSuccess || e2 != hipSuccess) {
    (void)hipGetLastError();
    fps_clear_error();
    ctx->graph_failures++;
    return launch_search(lib, ctx, P, path, variant, wsb, s, lib->timing, false, true);
  }
  if (ctx->graphs.size() >= SearchCtx::kGraphs) {
    (void)hipGraphExecDestroy(ctx->graphs.front().second);
    ctx->graphs.erase(ctx->graphs.begin());
  }
  ctx->graphs.push_back({std::move(key), ex});
  HIP_TRY(hipGraphLaunch(ex, s));
  ctx->last.graph = 1;
  return FPS_OK;
}

// Validates the queries and plans a search of them: per-query parameters,
// the query words in the library layout and their key counts.
static fps_status plan_queries(fps_library *lib, const uint64_t *queries, uint32_t q,
                               const uint32_t *k, const uint32_t *mask, Plan *P) {
  for (uint32_t i = 0; i < q; ++i)
    if (bad_fingerprint(queries + 3 * (size_t)i))
      return fps_fail(FPS_E_FINGERPRINT, "query %u has bit 0 or a bit above key 166 set", i);
  fps_status rc = fps_plan(lib, q, k, mask, P);
  if (rc) return rc;
  for (uint32_t i = 0; i < q; ++i) {
    QueryInfo &qi = P->qinfo[i];
    relabel(queries + 3 * (size_t)i, &qi.qa, &qi.qb, &qi.qc, &qi.qd);
    qi.popc = (uint32_t)(__builtin_popcountll(qi.qa) + __builtin_popcountll(qi.qb) +
                         __builtin_popcount(qi.qc) + __builtin_popcount(qi.qd));
  }
  return FPS_OK;
}

fps_status fps_search_impl(fps_library *lib, SearchCtx *ctx, const uint64_t *queries, uint32_t q,
                           const uint32_t *k, const uint32_t *mask, void *workspace,
                           size_t ws_bytes, fps_hit *out, uint64_t out_capacity,
                           uint64_t *out_offset, hipStream_t s, fps_path forced,
                           bool may_tune) {
  if (!lib || !ctx || !queries || !k || !workspace || !out_offset)
    return fps_fail(FPS_E_ARG, "NULL argument");
  Plan P;
  fps_status rc = plan_queries(lib, queries, q, k, mask, &P);
  if (rc) return rc;
  if (P.total_out > 0 && !out) return fps_fail(FPS_E_ARG, "NULL out");
  if (out_capacity < P.total_out)
    return fps_fail(FPS_E_ARG, "out holds %llu hits, %llu needed",
                    (unsigned long long)out_capacity, (unsigned long long)P.total_out);
  if (ws_bytes < P.total_bytes)
    return fps_fail(FPS_E_NOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, P.total_bytes);
  if (((uintptr_t)workspace & 255) != 0)
    return fps_fail(FPS_E_ARG, "workspace must be 256-byte aligned");
  out_offset[0] = 0;
  for (uint32_t i = 0; i < q; ++i) out_offset[i + 1] = out_offset[i] + P.qinfo[i].keff;
  ctx->last = fps_search_stats{};
  ctx->last.queries = q;
  ctx->last_untuned = false;
  if (P.total_out == 0) return FPS_OK;
  uint8_t *wsb = (uint8_t *)workspace;
  fps_path path;
  int variant;
  rc = resolve_path(lib, ctx, P, forced, wsb, s, may_tune, &path, &variant);
  if (rc) return rc;
  ctx->last.path = (uint32_t)path;
  ctx->last.variant =
      path == FPS_PATH_MFMA_I8 || path == FPS_PATH_MFMA_F4 ? (uint32_t)variant : 0u;
  rc = run_search(lib, ctx, P, path, variant, wsb, s);
  if (rc) return rc;
  // per-query counts and flags and the hits came back in one copy
  const size_t out_bytes = P.total_out * sizeof(fps_hit);
  uint8_t *ho = (uint8_t *)ctx->h_out;
  uint32_t *h_count = (uint32_t *)ho;
  uint32_t *h_flags = (uint32_t *)(ho + (P.off_flags - P.off_count));
  fps_hit *h_hits = (fps_hit *)(ho + (P.off_out - P.off_count));
  HIP_TRY(hipStreamSynchronize(s));
  float ms = 0;
  for (uint32_t p = 0; p < ctx->last_phases; ++p)
    if ((ctx->last_timed >> p & 1u) &&
        hipEventElapsedTime(&ms, ctx->ev[2 + 2 * p], ctx->ev[3 + 2 * p]) == hipSuccess)
      ctx->last.scan_ms += ms;
  if (ctx->last_total_timed && hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]) == hipSuccess)
    ctx->last.total_ms = ms;
  ctx->last.scan_launches = ctx->last_launches;
  ctx->sum_scan_ms += ctx->last.scan_ms;
  ctx->sum_total_ms += ctx->last.total_ms;
  ctx->sum_calls += 1;
  ctx->sum_launches += ctx->last.scan_launches;
  ctx->last.scan_ms_sum = ctx->sum_scan_ms;
  ctx->last.total_ms_sum = ctx->sum_total_ms;
  ctx->last.calls = ctx->sum_calls;
  ctx->last.scan_launches_sum = ctx->sum_launches;
  const Workspace ws = ws_view(P, wsb);
  const Lib L = lib_view(lib);
  for (uint32_t i = 0; i < q; ++i) {
    ctx->last.candidates += h_count[i];
    const QueryInfo &qi = P.qinfo[i];
    if (qi.keff == 0) continue;
    if (h_flags[i] == 0 && !lib->force_fb) continue;
    ctx->last.fallbacks++;
    launch_fallback(L, ws, i, P.rsets[qi.rset].neff, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(h_hits + qi.out_off, wsb + P.off_out + qi.out_off * sizeof(fps_hit),
                           qi.keff * sizeof(fps_hit), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  std::memcpy(out, h_hits, out_bytes);
  return FPS_OK;
}

extern "C" fps_status fps_search(fps_library *lib, const uint64_t query[3], uint32_t k,
                                 uint32_t mask, void *workspace, size_t ws_bytes, fps_hit *out,
                                 uint32_t *n_out, void *stream) {
  fps_clear_error();
  if (!n_out) return fps_fail(FPS_E_ARG, "NULL n_out");
  uint64_t off[2] = {0, 0};
  if (!lib) return fps_fail(FPS_E_ARG, "NULL library");
  fps_status rc = fps_search_impl(lib, &lib->ctx, query, 1, &k, &mask, workspace, ws_bytes, out,
                                  out ? (uint64_t)k : 0, off, (hipStream_t)stream,
                                  FPS_PATH_SINGLE, true);
  if (rc) return rc;
  *n_out = (uint32_t)off[1];
  return FPS_OK;
}

extern "C" fps_status fps_search_batch(fps_library *lib, const uint64_t *queries, uint32_t q,
                                       const uint32_t *k, const uint32_t *mask, void *workspace,
                                       size_t ws_bytes, fps_hit *out, uint64_t out_capacity,
                                       uint64_t *out_offset, void *stream) {
  fps_clear_error();
  if (!lib) return fps_fail(FPS_E_ARG, "NULL library");
  return fps_search_impl(lib, &lib->ctx, queries, q, k, mask, workspace, ws_bytes, out, out_capacity,
                         out_offset, (hipStream_t)stream, FPS_PATH_AUTO, true);
}

// ---------------------------------------------------------------------------
// autotuner: the batch scan kernel (path and matrix-core tile shape) for a
// batch shape is chosen by timing every applicable candidate on the first
// batch of that shape (device time between the first and the last kernel);
// the winner is cached per (live queries, largest k, library size), each
// rounded up to a power of two, and optionally persisted as JSON lines in the
// file named by FPS_TUNE_CACHE.  Every candidate returns identical results.
// ---------------------------------------------------------------------------
static uint32_t pow2_ceil(uint64_t x) {
  uint32_t p = 0;
  while (p < 63 && (1ull << p) < x) ++p;
  return p;
}

static TuneKey tune_key(const Plan &P) {
  uint64_t live = 0, kmax = 0, nmax = 0;
  for (const auto &qi : P.qinfo)
    if (qi.keff) {
      ++live;
      kmax = std::max<uint64_t>(kmax, qi.keff);
      nmax = std::max<uint64_t>(nmax, P.rsets[qi.rset].neff);
    }
  return TuneKey{pow2_ceil(live), pow2_ceil(kmax), pow2_ceil(nmax)};
}

static void tune_load(fps_library *lib) {
  const char *path = std::getenv("FPS_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "r");
  if (!f) return;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    int cus = 0, q = 0, k = 0, n = 0, p = 0, v = 0;
    if (std::sscanf(line, "{\"cus\": %d, \"q_log2\": %d, \"k_log2\": %d, \"n_log2\": %d, \"path\": %d, "
                    "\"variant\": %d",
                    &cus, &q, &k, &n, &p, &v) == 6 &&
        cus == lib->cus && p >= FPS_PATH_SINGLE && p <= FPS_PATH_MFMA_F4)
      lib->tuned[TuneKey{(uint32_t)q, (uint32_t)k, (uint32_t)n}] = {(fps_path)p, v};
  }
  std::fclose(f);
}

static void tune_save(const fps_library *lib, const TuneKey &key, fps_path p, int v, double ms) {
  const char *path = std::getenv("FPS_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f,
               "{\"cus\": %d, \"q_log2\": %u, \"k_log2\": %u, \"n_log2\": %u, \"path\": %d, "
               "\"variant\": %d, \"ms\": %.4f}\n",
               lib->cus, key.q, key.k, key.n, (int)p, v, ms);
  std::fclose(f);
}

static std::vector<std::pair<fps_path, int>> tune_candidates(const Plan &P) {
  uint64_t live = 0;
  for (const auto &qi : P.qinfo) live += qi.keff > 0;
  std::vector<std::pair<fps_path, int>> c;
  if (live <= 16) c.push_back({FPS_PATH_SINGLE, 0});
  c.push_back({FPS_PATH_POPCOUNT, 0});
  if (live >= 8) {
    for (int v = 0; v < mfma_variants(); ++v) c.push_back({FPS_PATH_MFMA_I8, v});
    for (int v = 0; v < mfma_f4_variants(); ++v) c.push_back({FPS_PATH_MFMA_F4, v});
  }
  return c;
}

// Kernel choice for a shape the autotuner has not timed, when timing is not
// allowed (a server's request path): the single-query scan for one or two
// live queries, the fp4 matrix-core kernel otherwise -- its shape of 64
// queries shared by a block's four waves up to 64 queries, 64 queries per
// wave beyond, and eight such waves per block from 512 queries.
static uint64_t live_queries(const Plan &P) {
  uint64_t live = 0;
  for (const auto &qi : P.qinfo) live += qi.keff > 0;
  return live;
}

static int default_f4_variant(uint64_t live) { return live <= 64 ? 2 : live >= 512 ? 4 : 0; }

static void default_path(const Plan &P, fps_path *path, int *variant) {
  const uint64_t live = live_queries(P);
  if (live <= 2) {
    *path = FPS_PATH_SINGLE;
    *variant = 0;
  } else {
    *path = FPS_PATH_MFMA_F4;
    *variant = default_f4_variant(live);
  }
}

static fps_status resolve_path(fps_library *lib, SearchCtx *ctx, Plan &P, fps_path requested,
                               uint8_t *wsb, hipStream_t s, bool may_tune, fps_path *path,
                               int *variant) {
  if (requested != FPS_PATH_AUTO || lib->path != FPS_PATH_AUTO) {
    *path = requested != FPS_PATH_AUTO ? requested : lib->path;
    // default tile shapes: 64 queries per wave, two waves per SIMD
    const int nv = *path == FPS_PATH_MFMA_F4 ? mfma_f4_variants() : mfma_variants();
    *variant = lib->variant >= 0 ? lib->variant % nv
               : *path == FPS_PATH_MFMA_F4 ? (default_f4_variant(live_queries(P)) == 4 ? 4 : 0)
                                           : 1;
    return FPS_OK;
  }
  *variant = 0;
  const TuneKey key = tune_key(P);
  {
    std::lock_guard<std::mutex> lk(lib->tune_mu);
    auto it = lib->tuned.find(key);
    if (it != lib->tuned.end()) {
      *path = it->second.first;
      *variant = it->second.second;
      return FPS_OK;
    }
  }
  if (!may_tune) {
    default_path(P, path, variant);
    ctx->last_untuned = true;
    return FPS_OK;
  }
  double best = 1e30;
  fps_path bp = FPS_PATH_POPCOUNT;
  int bv = 0;
  for (const auto &cand : tune_candidates(P)) {
    fps_status rc = launch_search(lib, ctx, P, cand.first, cand.second, wsb, s, true);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(s));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
    if (ms < best) {
      best = ms;
      bp = cand.first;
      bv = cand.second;
    }
  }
  {
    std::lock_guard<std::mutex> lk(lib->tune_mu);
    lib->tuned[key] = {bp, bv};
  }
  tune_save(lib, key, bp, bv, best);
  *path = bp;
  *variant = bv;
  return FPS_OK;
}

// Synthetic query i of the tuner: every key set with probability 1/4, from a
// multiply-xorshift hash of (i, word).
static void tune_query(uint32_t i, uint64_t w[3]) {
  for (int j = 0; j < 3; ++j) {
    uint64_t a = 0x9E3779B97F4A7C15ull * (4ull * i + (uint64_t)j + 1ull), b;
    a ^= a >> 31;
    a *= 0xD6E8FEB86659FD93ull;
    a ^= a >> 29;
    b = a * 0xBF58476D1CE4E5B9ull;
    b ^= b >> 32;
    w[j] = a & b;
  }
  w[0] &= ~1ull;                  // bit 0 is not a key
  w[2] &= (1ull << 39) - 1ull;    // nor are the bits above key 166
}

fps_status fps_tune_impl(fps_library *lib, SearchCtx *ctx, uint32_t q, const uint32_t *k,
                         const uint32_t *mask, void *workspace, size_t ws_bytes, hipStream_t s) {
  if (!lib || !ctx || !k || !workspace) return fps_fail(FPS_E_ARG, "NULL argument");
  std::vector<uint64_t> qs((size_t)q * 3);
  for (uint32_t i = 0; i < q; ++i) tune_query(i, &qs[3 * (size_t)i]);
  Plan P;
  fps_status rc = plan_queries(lib, qs.data(), q, k, mask, &P);
  if (rc) return rc;
  if (ws_bytes < P.total_bytes)
    return fps_fail(FPS_E_NOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, P.total_bytes);
  if (((uintptr_t)workspace & 255) != 0)
    return fps_fail(FPS_E_ARG, "workspace must be 256-byte aligned");
  if (P.total_out == 0) return FPS_OK;
  fps_path path;
  int variant;
  rc = resolve_path(lib, ctx, P, FPS_PATH_AUTO, (uint8_t *)workspace, s, true, &path, &variant);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  return FPS_OK;
}

extern "C" fps_status fps_tune(fps_library *lib, uint32_t q, const uint32_t *k,
                               const uint32_t *mask, void *workspace, size_t ws_bytes,
                               void *stream) {
  fps_clear_error();
  if (!lib) return fps_fail(FPS_E_ARG, "NULL library");
  if (lib->path != FPS_PATH_AUTO) return FPS_OK;  // a forced path is never tuned
  return fps_tune_impl(lib, &lib->ctx, q, k, mask, workspace, ws_bytes, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// allocation-free single-query search: the workspace of fps_search lives in a
// static device array, one copy per GPU, whose address is taken once per
// device when a library is loaded there.  Kernels get that address as their
// workspace argument; host code never uses the array's name.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[FPS_NOALLOC_SCRATCH_BYTES];
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch[kMaxDevices];

static fps_status scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices)
    return fps_fail(FPS_E_DEVICE, "device %d beyond the %d the scratch table holds", device,
                    kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return FPS_OK;
  void *p = nullptr;
  HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) return fps_fail(FPS_E_DEVICE, "hipGetSymbolAddress returned a null scratch address");
  g_scratch[device] = p;
  return FPS_OK;
}

extern "C" fps_status fps_search_noalloc(fps_library *lib, const uint64_t query[3], uint32_t k,
                                         uint32_t mask, fps_hit *out, uint32_t *n_out,
                                         void *stream) {
  fps_clear_error();
  if (!lib || !n_out) return fps_fail(FPS_E_ARG, "NULL argument");
  void *ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (lib->device >= 0 && lib->device < kMaxDevices) ws = g_scratch[lib->device];
  }
  if (!ws) return fps_fail(FPS_E_STATE, "no scratch address for device %d", lib->device);
  Plan P;
  fps_status rc = fps_plan(lib, 1, &k, &mask, &P);
  if (rc) return rc;
  if (P.total_bytes > (size_t)FPS_NOALLOC_SCRATCH_BYTES)
    return fps_fail(FPS_E_NOMEM,
                    "this search needs %zu bytes of workspace; the static scratch holds %zu "
                    "(use fps_search with a workspace)",
                    P.total_bytes, (size_t)FPS_NOALLOC_SCRATCH_BYTES);
  if (P.params_bytes > lib->ctx.h_params_bytes || back_bytes(P) > lib->ctx.h_out_bytes)
    return fps_fail(FPS_E_NOMEM,
                    "this search needs %zu + %zu bytes of host staging; %zu + %zu are allocated",
                    P.params_bytes, back_bytes(P), lib->ctx.h_params_bytes,
                    lib->ctx.h_out_bytes);
  uint64_t off[2] = {0, 0};
  rc = fps_search_impl(lib, &lib->ctx, query, 1, &k, &mask, ws, FPS_NOALLOC_SCRATCH_BYTES, out,
                       out ? (uint64_t)k : 0, off, (hipStream_t)stream, FPS_PATH_SINGLE, true);
  if (rc) return rc;
  *n_out = (uint32_t)off[1];
  return FPS_OK;
}
