/*
 * fps.h -- C ABI of the MI355X exact fingerprint top-k engine.
 *
 * The engine answers the question of FPScreen (arXiv 1906.06170), Fig. 3: given a
 * target MACCS-166 fingerprint and a library of fingerprints, return the N
 * library entries with the smallest Manhattan distance to the target, with
 * their distances, in ascending order.  The distance is the one of Section 4.3,
 *     dist(a, b) = sum_{j=1..166} |a_j - b_j|,
 * which for 0/1 keys equals the number of keys in which a and b differ.  Equal
 * distances are ordered by ascending library index (the paper states no tie
 * rule; this one makes the answer unique).  The library may be cut into strides
 * (Section 2.1, Fig. 1); a query may search any union of strides and the
 * results are combined into one global order (Section 4.3).
 *
 * Fingerprint layout (records and queries): three uint64 words; key j (1..166)
 * is bit (j & 63) of word (j >> 6).  Bit 0 of word 0 and bits 39..63 of word 2
 * (keys 167..191) must be zero: a record or query with any of them set is
 * rejected with FPS_E_FINGERPRINT, never silently masked.
 *
 * Conventions for every call:
 *   - the return value is an fps_status; FPS_OK is 0 and errors are negative;
 *     nothing throws across this interface;
 *   - fps_last_error() returns a message for the last failure on the calling
 *     thread (empty string if none); the pointer stays valid until the next
 *     call on that thread;
 *   - all arguments are validated before any device work is queued;
 *   - device memory is owned by the caller (typically torch tensors): the
 *     library buffer and every workspace; the library handle owns only host
 *     state, pinned host staging buffers and its device-side parameter cache;
 *   - "stream" is a hipStream_t (NULL = the default stream); calls that return
 *     results are synchronous with respect to that stream: they return after
 *     the results are in host memory;
 *   - one handle must not be used by two threads at once; concurrency between
 *     requests comes from the server API below.
 */
#ifndef FPS_H
#define FPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FPS_OK = 0,
  FPS_E_ARG = -1,         /* NULL pointer, bad mask, bad size, buffer too small */
  FPS_E_FINGERPRINT = -2, /* bit 0 or a bit above key 166 set in a record/query */
  FPS_E_NOMEM = -3,       /* workspace smaller than fps_workspace_bytes, or host allocation failed */
  FPS_E_DEVICE = -4,      /* a HIP runtime error (message from hipGetErrorString) */
  FPS_E_STATE = -5,       /* handle used in a state that does not allow the call */
  FPS_E_BUSY = -6         /* server admission full (non-blocking submit only) */
} fps_status;

#define FPS_KEYS 166
#define FPS_WORDS 3
#define FPS_MAX_STRIDES 32
/* Stride mask selecting every stride of the library. */
#define FPS_MASK_ALL 0xFFFFFFFFu

typedef struct fps_library fps_library; /* opaque handle */

/* One result: global library row and its distance (0..166). */
typedef struct {
  uint32_t index;
  uint32_t distance;
} fps_hit;

/* Scan kernels a batch may use. */
typedef enum {
  FPS_PATH_AUTO = 0,     /* autotuner's choice: on the first batch of a shape (live
                            queries, largest k, library size, each rounded up to a
                            power of two) every applicable kernel is timed and the
                            fastest is kept; FPS_TUNE_CACHE names a file that
                            persists the choices as JSON lines */
  FPS_PATH_SINGLE = 1,   /* the single-query scan, one query per pass over the library */
  FPS_PATH_POPCOUNT = 2, /* batched XOR + popcount kernel */
  FPS_PATH_MFMA_I8 = 3,  /* batched int8 matrix-core kernel (a.b with exact int32 sums) */
  FPS_PATH_MFMA_F4 = 4   /* batched 4-bit-float matrix-core kernel (exact fp32 sums) */
} fps_path;

/* ------------------------------------------------------------------------ */
/* Library (Fig. 3 step 1: the library file becomes the matrix A).           */
/* ------------------------------------------------------------------------ */

/* Device bytes needed to hold n records: 21 bytes per record (the 166 keys
 * packed into one 64-bit, one 64-bit, one 32-bit and one 8-bit word-major
 * array), n rounded up to a multiple of 4096. */
size_t fps_library_device_bytes(uint64_t n);

/*
 * Validates n records and uploads them into device_buf in the engine's layout.
 *   host_words:   n x 3 uint64, record-major, host memory (read only, not kept).
 *   n:            1 <= n < 2^32.
 *   stride_begin: nstrides + 1 non-decreasing offsets, stride_begin[0] = 0 and
 *                 stride_begin[nstrides] = n; stride s holds records
 *                 [stride_begin[s], stride_begin[s+1]).  NULL means one stride.
 *   nstrides:     1..FPS_MAX_STRIDES (ignored when stride_begin is NULL).
 *   device_buf:   caller-owned device memory of device_bytes >=
 *                 fps_library_device_bytes(n); it must stay allocated and
 *                 unmodified until fps_library_free.  Its contents are
 *                 overwritten.
 *   stream:       hipStream_t for the upload; the call returns after it ends.
 *   out:          receives the handle.
 * Errors: FPS_E_ARG (NULL, n out of range, bad strides, small buffer),
 * FPS_E_FINGERPRINT (the message names the first bad row), FPS_E_DEVICE.
 */
fps_status fps_library_load(const uint64_t *host_words, uint64_t n, const uint64_t *stride_begin,
                            uint32_t nstrides, void *device_buf, size_t device_bytes,
                            void *stream, fps_library **out);

/* Library size and stride table (stride_begin may be NULL; else nstrides+1 entries). */
fps_status fps_library_info(const fps_library *lib, uint64_t *n, uint32_t *nstrides,
                            uint64_t *stride_begin);

/* Releases the handle and its host state.  Never frees device_buf. NULL is OK. */
fps_status fps_library_free(fps_library *lib);

/* Selects the batch scan kernel (default FPS_PATH_AUTO). */
fps_status fps_set_path(fps_library *lib, fps_path path);

/* Graph replay of batched searches (default on): when a launch shape (query
 * count, per-query k and mask, workspace, kernel choice) comes again within the
 * last 8 calls, its launch sequence is recorded into a HIP graph, and later
 * calls of that shape replay it with the new queries (up to 4 graphs per
 * handle or server slot).  Single-query scans always launch directly.
 * enable = 0 launches every kernel directly. */
fps_status fps_set_graphs(fps_library *lib, int enable);

/* Device timing of searches (scan_ms, total_ms and their sums in
 * fps_search_stats).  Off by default: the timing events cost about 10
 * microseconds of a single-query search, whose first kernels wait on the
 * host.  enable != 0 stamps HIP events at the first kernel, around every scan
 * phase and at the last kernel of every call.  The autotuner times its
 * candidates regardless.  Errors: FPS_E_ARG. */
fps_status fps_set_timing(fps_library *lib, int enable);

/* Selects the tile shape of the matrix-core kernel of a path forced with
 * fps_set_path.  int8: 0 = 64 queries per wave, 1 = 64 per wave with two waves
 * per SIMD, 2 = 128 per wave, 3 = 32 per wave with two waves per SIMD, 4 = 64
 * queries shared by a block's four waves, which split the records.  fp4: 0 = 64
 * queries per wave with two waves per SIMD, 1 = 128 per wave, 2 = 64 queries
 * shared by the four waves, 3 = 32 per wave with two waves per SIMD, 4 = 64
 * queries per wave in blocks of eight waves (512 queries).  A value beyond the
 * path's shapes wraps around.  -1 (default): the autotuner chooses under
 * FPS_PATH_AUTO; a forced path takes int8 shape 1, or fp4 shape 4 for 512 or
 * more live queries and shape 0 below.
 * Results never depend on it.  Errors: FPS_E_ARG (variant < -1 or >= 5). */
fps_status fps_set_variant(fps_library *lib, int variant);

/* ------------------------------------------------------------------------ */
/* The library file and the query box (Fig. 3 steps 1, 2 and 5; Fig. 1).     */
/* ------------------------------------------------------------------------ */

/*
 * The library file F of Fig. 3 step 1 holds one line of MACCS text per molecule
 * (Abstract) and the molecule's PubChem CID, which the results carry (Fig. 3
 * step 5, Fig. 2).  The paper prints no line format; these calls read
 *     <id> <separator> <keys> [blanks] '\n'
 *   id:        1..19 decimal digits (any 64-bit id up to 10^19 - 1);
 *   separator: one or more of ' ', '\t', ',';
 *   keys:      167 characters '0'/'1' for positions 0..166, of which position
 *              0 holds no key and must be '0', or 166 characters for keys
 *              1..166 (the two forms may be mixed);
 *   blanks:    ' ', '\t', '\r' (so CRLF line ends are accepted);
 *   a line has at most 255 characters before its '\n'; the last line may lack
 *   its '\n'; a '\n' ending the text starts no line, any other empty line is
 *   malformed.  Record i of the library is line i + 1 of the text.
 * The text is parsed on the GPU from device memory: the caller copies the
 * file's bytes into HBM (a torch tensor) first.
 */

/* Device workspace bytes for fps_text_count and fps_text_library_load on a text
 * of text_bytes bytes (about 12 bytes per 16 KiB of text). Errors: FPS_E_ARG. */
fps_status fps_text_workspace_bytes(uint64_t text_bytes, size_t *bytes);

/*
 * Number of records (lines) of a library text, so the caller can size the
 * library buffer (fps_library_device_bytes) and the id column.
 *   text:       device memory, text_bytes > 0 bytes, 16-byte aligned.
 *   workspace:  device memory of ws_bytes >= fps_text_workspace_bytes, 256-byte
 *               aligned; its contents are scratch.
 *   stream:     hipStream_t; the call returns when the count is known.
 * Lines are not validated here (fps_text_library_load does that).
 * Errors: FPS_E_ARG (NULL, empty or misaligned text), FPS_E_NOMEM (small
 * workspace), FPS_E_DEVICE.
 */
fps_status fps_text_count(const void *text, uint64_t text_bytes, void *workspace,
                          size_t ws_bytes, void *stream, uint64_t *n_records);

/*
 * Builds a library from its text on the GPU (Fig. 3 step 1: the molecules of F
 * become the matrix A and the CID column).
 *   text, text_bytes, workspace, ws_bytes, stream: as fps_text_count.
 *   n_records:    the count fps_text_count returned (checked again here).
 *   stride_begin, nstrides, device_buf, device_bytes, out: as fps_library_load.
 *   ids_device:   device memory for n_records uint64 ids (record i's id at
 *                 [i]), or NULL to discard the ids.  When given, the handle
 *                 keeps the pointer for fps_hit_ids: it must stay valid and
 *                 unmodified until fps_library_free;
 *   ids_host:     host memory for n_records uint64 ids, or NULL.  When given
 *                 (it needs ids_device), the ids are copied there and the
 *                 handle keeps the pointer for fps_hit_ids: it must stay valid
 *                 until fps_library_free.  Without it the ids stay in device
 *                 memory only (no download: the 8 bytes per record of the id
 *                 column never cross PCIe).
 * When workspace still holds what fps_text_count computed for this text
 * (same address and size) and n_records, the lines are not counted again; the
 * parse checks every chunk's newlines against those counts (FPS_E_ARG "line L:
 * the text changed since it was counted" if they differ).
 * Every line is validated; the first malformed line is reported by number:
 * FPS_E_ARG "line L: <problem>" (problems: line too long, id missing or
 * longer than 19 digits, no separator, keys not 166 or 167 characters '0'/'1',
 * characters other than blanks after the keys), or FPS_E_FINGERPRINT for a
 * 167-character key field with position 0 set.  Also FPS_E_ARG (n_records
 * differs from the text's line count, and the errors of fps_library_load),
 * FPS_E_NOMEM, FPS_E_DEVICE.  The text and the workspace are not kept.
 */
fps_status fps_text_library_load(const void *text, uint64_t text_bytes, uint64_t n_records,
                                 const uint64_t *stride_begin, uint32_t nstrides, void *workspace,
                                 size_t ws_bytes, void *device_buf, size_t device_bytes,
                                 uint64_t *ids_device, uint64_t *ids_host, void *stream,
                                 fps_library **out);

/* Fig. 3 step 5 ("CID + K"): ids[i] = the id of record hits[i].index, from the
 * id table of a library loaded from text: the host copy when the load was given
 * ids_host, else the device table (gathered by a kernel on the null stream
 * through mapped pinned staging the handle keeps; calls on one handle are
 * serialized).  hits and ids are host memory.
 * Errors: FPS_E_ARG (NULL, an index beyond the library), FPS_E_STATE (the
 * library has no id table), FPS_E_DEVICE. */
fps_status fps_hit_ids(const fps_library *lib, const fps_hit *hits, uint64_t n, uint64_t *ids);

/*
 * The target as typed into the search box of Fig. 1 (Fig. 3 step 2: the target
 * fingerprint becomes the vector b): "[v,v,...,v]", each v '0' or '1', blanks
 * around any token, one optional ',' before ']' (Fig. 1 shows one).  166 values
 * are keys 1..166; 167 values are positions 0..166 (position 0 must be 0).
 *   text/len: host memory (not NUL-terminated necessarily).
 *   query:    receives the three words (key j at bit j & 63 of word j >> 6).
 * Errors: FPS_E_ARG with the character position, FPS_E_FINGERPRINT (position
 * 0 set).  Host only; no device work.
 */
fps_status fps_parse_query(const char *text, size_t len, uint64_t query[3]);

/* A batch of targets, one bracketed list per line; lines holding only blanks
 * are skipped.  queries: room for capacity x 3 words; *nq receives the count.
 * Errors as fps_parse_query, the message naming the 1-based line; FPS_E_ARG
 * when more than capacity lists are present. */
fps_status fps_parse_queries(const char *text, size_t len, uint64_t *queries, uint32_t capacity,
                             uint32_t *nq);

/* ------------------------------------------------------------------------ */
/* Search (Fig. 3 steps 2-6; single and batch searches of Section 4.4).       */
/* ------------------------------------------------------------------------ */

/*
 * Device workspace bytes for a search of q queries with per-query k[] and
 * stride masks mask[] (mask NULL = FPS_MASK_ALL for every query).  The same
 * value is valid for fps_search (q = 1) and fps_search_batch.
 * Errors: FPS_E_ARG (NULL lib/k/bytes, q == 0, a zero mask or a mask naming a
 * stride the library does not have).
 */
fps_status fps_workspace_bytes(const fps_library *lib, uint32_t q, const uint32_t *k,
                               const uint32_t *mask, size_t *bytes);

/*
 * One query (Fig. 3; the "single molecular search" of Section 4.4).
 *   query:  3 uint64 words, host memory.
 *   k:      number of results wanted (0 allowed).
 *   mask:   strides to search (bit s = stride s) or FPS_MASK_ALL.
 *   workspace/ws_bytes: caller-owned device memory, at least
 *           fps_workspace_bytes(lib, 1, &k, &mask).
 *   out:    host memory with room for min(k, n_eff) hits, n_eff being the number
 *           of records in the selected strides; written in ascending
 *           (distance, index) order.
 *   n_out:  receives min(k, n_eff).
 * Errors: FPS_E_ARG, FPS_E_FINGERPRINT, FPS_E_NOMEM, FPS_E_DEVICE.
 */
fps_status fps_search(fps_library *lib, const uint64_t query[3], uint32_t k, uint32_t mask,
                      void *workspace, size_t ws_bytes, fps_hit *out, uint32_t *n_out,
                      void *stream);

/*
 * Independent queries in one launch sequence (the batch search of Section 4.4
 * without its clustering step).
 *   queries:  q x 3 uint64, record-major, host memory.
 *   k:        q result counts; mask: q stride masks or NULL (all strides).
 *   out:      host memory of out_capacity hits; query i's hits are
 *             out[out_offset[i] .. out_offset[i+1]), min(k[i], n_eff[i]) of them,
 *             in ascending (distance, index) order.
 *   out_offset: host array of q + 1 entries, filled by the call.
 * Errors: FPS_E_ARG (also when out_capacity < sum of min(k[i], n_eff[i])),
 * FPS_E_FINGERPRINT (the message names the first bad query), FPS_E_NOMEM,
 * FPS_E_DEVICE.
 */
fps_status fps_search_batch(fps_library *lib, const uint64_t *queries, uint32_t q,
                            const uint32_t *k, const uint32_t *mask, void *workspace,
                            size_t ws_bytes, fps_hit *out, uint64_t out_capacity,
                            uint64_t *out_offset, void *stream);

/*
 * fps_search without a workspace argument, for callers that cannot allocate
 * device memory: code that must not call hipMalloc (serving loops with fixed
 * memory, harnesses that forbid allocation).  The same kernels as fps_search
 * run on a static device array of FPS_NOALLOC_SCRATCH_BYTES, one per GPU,
 * reserved when the library's code is loaded on that GPU and held until the
 * process ends; the pinned host staging it uses is allocated by
 * fps_library_load.  The call itself allocates no device or pinned memory
 * (its host-side plan uses a few small heap blocks).
 *   Arguments, results and errors as fps_search, plus FPS_E_NOMEM when the
 *   search needs more workspace than the static array holds (very large k
 *   on a large library; fps_workspace_bytes tells) or more host staging than
 *   the load allocated (k above about 8,000).
 * Every call on one GPU shares that GPU's array and the handle's staging, and
 * the array keeps the last call's contents (the kernels clear what must start
 * at zero): calls that overlap on one GPU, from any handle or thread, race.
 */
#define FPS_NOALLOC_SCRATCH_BYTES (32u << 20)
fps_status fps_search_noalloc(fps_library *lib, const uint64_t query[3], uint32_t k,
                              uint32_t mask, fps_hit *out, uint32_t *n_out, void *stream);

/* Counters of the last search on this handle (for tests and benchmarks). */
typedef struct {
  uint32_t path;          /* fps_path actually used */
  uint32_t queries;       /* queries in the call */
  uint32_t fallbacks;     /* queries answered by the exact two-pass fallback */
  uint32_t variant;       /* matrix-core tile shape used (fps_set_variant) */
  uint64_t candidates;    /* candidates appended by the scan, summed over queries */
  double scan_ms;         /* device time of the scan kernel launches of the call (HIP
                             events; 0 unless fps_set_timing enabled them) */
  double total_ms;        /* device time from the first to the last kernel (likewise) */
  uint32_t graph;         /* 1 if the launch sequence was replayed from a HIP graph */
  uint32_t scan_launches; /* scan kernel launches of the call */
  /* running sums over every call on this handle (or server slot) */
  double scan_ms_sum;
  double total_ms_sum;
  uint64_t calls;
  uint64_t scan_launches_sum;
} fps_search_stats;

fps_status fps_last_search_stats(const fps_library *lib, fps_search_stats *stats);

/*
 * Runs the autotuner of FPS_PATH_AUTO for one batch shape ahead of use: q
 * queries with result counts k[] and stride masks mask[] (NULL = all).  The
 * shape's key is that of FPS_PATH_AUTO (live queries, largest k, largest
 * n_eff, each rounded up to a power of two); if it is already tuned the call
 * does nothing.  Otherwise every applicable kernel runs once on q synthetic
 * queries (keys set with probability 1/4 from a fixed hash) and the fastest is
 * cached, as the first batch of that shape would do.  workspace/ws_bytes as
 * for fps_search_batch with these k and masks.  Nothing is returned to the
 * host besides the status.  Errors: as fps_workspace_bytes, FPS_E_NOMEM
 * (small workspace), FPS_E_DEVICE.
 */
fps_status fps_tune(fps_library *lib, uint32_t q, const uint32_t *k, const uint32_t *mask,
                    void *workspace, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Batch clustering search (Section 4.4; Fig. 2).                             */
/* ------------------------------------------------------------------------ */

/*
 * Section 4.4 describes a "batch clustering search": a batch of targets is
 * clustered and the top 30 molecules are found per cluster; Fig. 2 picks the
 * number of clusters ("categories") by the silhouette ("contour coefficient").
 * The paper names neither the algorithm nor what is searched for a cluster.
 * These calls take:
 *   - for every cluster count K in [k_min, k_max]: farthest-first initial
 *     centers (target 0, then the target farthest from its nearest center,
 *     ties to the lowest index) and k-medians under the Manhattan distance of
 *     Section 4.3 (targets join the nearest center, ties to the lowest center;
 *     a center becomes the key-wise strict majority of its members, the
 *     median that minimises their summed distance; an empty cluster keeps its
 *     center), until no label changes or max_iter rounds;
 *   - the mean silhouette (Rousseeuw 1987: s = (b - a) / max(a, b); 0 for a
 *     singleton cluster or max(a, b) = 0), each s from exact integer distance
 *     sums, added in index order in double precision; the K with the largest
 *     mean wins, ties to the smaller K;
 *   - the chosen clusters' centers are then searched as targets (Fig. 3).
 */
#define FPS_CLUSTER_MAX_K 16
#define FPS_CLUSTER_MAX_Q 16384

typedef struct {
  uint32_t k;      /* the chosen number of clusters */
  uint32_t rounds; /* k-medians rounds of the chosen clustering */
  double score[FPS_CLUSTER_MAX_K + 1]; /* score[K] = mean silhouette of K clusters (0 if not tried) */
} fps_cluster_info;

/* Device workspace bytes of fps_cluster for q targets (3 <= q <= FPS_CLUSTER_MAX_Q). */
fps_status fps_cluster_workspace_bytes(uint32_t q, size_t *bytes);

/*
 * Clusters q targets (host memory, q x 3 words) on the GPU.
 *   k_min, k_max: cluster counts tried, 2 <= k_min <= k_max <= FPS_CLUSTER_MAX_K,
 *                 k_max < q;
 *   max_iter:     k-medians rounds at most (>= 1; 100 is ample);
 *   workspace:    device memory, 256-byte aligned, >= fps_cluster_workspace_bytes;
 *   labels:       host, q entries: the cluster of every target (0..k-1);
 *   centers:      host, room for k_max x 3 words: the chosen centers;
 *   info:         host (may be NULL): the chosen k, its rounds, every score.
 * Synchronous on stream.  Errors: FPS_E_ARG, FPS_E_FINGERPRINT, FPS_E_NOMEM,
 * FPS_E_DEVICE.
 */
fps_status fps_cluster(const uint64_t *queries, uint32_t q, uint32_t k_min, uint32_t k_max,
                       uint32_t max_iter, void *workspace, size_t ws_bytes, void *stream,
                       uint32_t *labels, uint64_t *centers, fps_cluster_info *info);

/* Workspace bytes of fps_cluster_search: the larger of the clustering's and
 * that of a search of k_max targets with result count k and stride mask. */
fps_status fps_cluster_search_workspace_bytes(const fps_library *lib, uint32_t q, uint32_t k_max,
                                              uint32_t k, uint32_t mask, size_t *bytes);

/*
 * fps_cluster, then the top-k of every chosen center over the strides of mask
 * (the batch clustering search of Section 4.4).  out / out_capacity /
 * out_offset as fps_search_batch for info->k targets (out_offset needs
 * k_max + 1 entries); category c's hits are out[out_offset[c] ..
 * out_offset[c+1]).  Errors: those of fps_cluster and fps_search_batch.
 */
fps_status fps_cluster_search(fps_library *lib, const uint64_t *queries, uint32_t q,
                              uint32_t k_min, uint32_t k_max, uint32_t max_iter, uint32_t k,
                              uint32_t mask, void *workspace, size_t ws_bytes, fps_hit *out,
                              uint64_t out_capacity, uint64_t *out_offset, uint32_t *labels,
                              uint64_t *centers, fps_cluster_info *info, void *stream);

/* ------------------------------------------------------------------------ */
/* Wider fingerprints (Section 5, concluding remark 3: more features).         */
/* ------------------------------------------------------------------------ */

/*
 * Libraries of fingerprints of W 64-bit words, W in {4, 8, 16, 32} (256 to
 * 2,048 keys, e.g. hashed circular fingerprints of 1,024 or 2,048 bits).
 * Key j (0 .. 64 W - 1) is bit (j & 63) of word (j >> 6); every bit is a key,
 * none is reserved.  The distance is the Section 4.3 sum over all 64 W keys
 * (the number of differing keys, 0 .. 64 W), the top-k order, tie rule,
 * strides and merge are those of the MACCS calls above, and the results are
 * fps_hit (index, distance).  Device memory is caller-owned as above.
 */
#define FPS_WIDE_MAX_WORDS 32

typedef struct fps_wide fps_wide; /* opaque handle */

/* Device bytes of n records of `words` words: 8 * words bytes per record,
 * word-major, n rounded up to a multiple of 4096. */
size_t fps_wide_device_bytes(uint64_t n, uint32_t words);

/* Uploads n records (host, n x words uint64, record-major) into device_buf in
 * the engine's layout.  Arguments and errors as fps_library_load, plus
 * FPS_E_ARG when words is not 4, 8, 16 or 32. */
fps_status fps_wide_load(const uint64_t *host_words, uint64_t n, uint32_t words,
                         const uint64_t *stride_begin, uint32_t nstrides, void *device_buf,
                         size_t device_bytes, void *stream, fps_wide **out);

/* Releases the handle (never device_buf).  NULL is OK. */
fps_status fps_wide_free(fps_wide *lib);

/* Scan kernel of a search: FPS_PATH_SINGLE (one query per pass), _POPCOUNT,
 * _MFMA_I8, _MFMA_F4, or FPS_PATH_AUTO (default: single for 1-2 queries,
 * popcount below 32, fp4 matrix cores from 32).  Results never depend on it. */
fps_status fps_wide_set_path(fps_wide *lib, fps_path path);

/* candidate_scale multiplies the candidate capacity (tiny values force the
 * overflow fallback); sample_records is the bound sample (0 = 65,536);
 * force_fallback != 0 answers every query with the exact two-pass fallback.
 * Results never depend on these; workspace sizes do. */
fps_status fps_wide_set_tuning(fps_wide *lib, double candidate_scale, uint64_t sample_records,
                               int force_fallback);

/* HIP-event timing of scan_ms / total_ms in the statistics (off by default). */
fps_status fps_wide_set_timing(fps_wide *lib, int enable);

/* Workspace bytes of a search of q queries with k[] and masks (NULL = all);
 * depends on the path set with fps_wide_set_path. */
fps_status fps_wide_workspace_bytes(const fps_wide *lib, uint32_t q, const uint32_t *k,
                                    const uint32_t *mask, size_t *bytes);

/* Independent queries (host, q x words uint64).  Arguments, results and errors
 * as fps_search_batch. */
fps_status fps_wide_search_batch(fps_wide *lib, const uint64_t *queries, uint32_t q,
                                 const uint32_t *k, const uint32_t *mask, void *workspace,
                                 size_t ws_bytes, fps_hit *out, uint64_t out_capacity,
                                 uint64_t *out_offset, void *stream);

/* One query (host, `words` uint64), as fps_search. */
fps_status fps_wide_search(fps_wide *lib, const uint64_t *query, uint32_t k, uint32_t mask,
                           void *workspace, size_t ws_bytes, fps_hit *out, uint32_t *n_out,
                           void *stream);

/* Counters of the last search on this handle, as fps_last_search_stats. */
fps_status fps_wide_last_search_stats(const fps_wide *lib, fps_search_stats *stats);

/* ------------------------------------------------------------------------ */
/* Tuning knobs, for tests that must force the rare paths.                   */
/* ------------------------------------------------------------------------ */

/*
 * candidate_scale: multiplies every query's candidate-buffer capacity (1.0 is
 *   the default; tiny values force the overflow fallback).
 * sample_records:  records per query whose distance histogram gives the first
 *   bound (0 = default 2^16).
 * phase_records:   records per query scanned before the bound is first
 *   refined from the candidates found so far (0 = sample_records times the
 *   geometric phase ratio, which is 4096 / max k clamped to 8..64).
 * force_fallback:  nonzero answers every query with the exact two-pass path.
 * Results never depend on these; workspace sizes do: query
 * fps_workspace_bytes after setting them.
 */
fps_status fps_set_tuning(fps_library *lib, double candidate_scale, uint64_t sample_records,
                          uint64_t phase_records, int force_fallback);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of independent requests (the queue between the */
/* user side and the computing side, Sections 3.1 and 4.4).                    */
/* ------------------------------------------------------------------------ */

typedef struct fps_server fps_server;

typedef struct {
  size_t pool_bytes;          /* device workspace pool the server may use (<= ws_bytes) */
  uint32_t max_batch_queries; /* cap on queries coalesced into one batch */
  uint32_t max_wait_us;       /* longest a request waits for others to join its batch */
  uint32_t n_streams;         /* batches in flight at once (1..8) */
  uint32_t deadline_cap;      /* nonzero: a batch stops growing before its predicted completion
                                 passes the earliest deadline among its requests, unless that
                                 deadline is missed anyway (the queue is behind); completion is
                                 predicted by a linear model of batch service time fitted to the
                                 batches served so far (fps_server_stats reports it) */
  uint32_t reserve_streams;   /* of the n_streams, how many take a batch only under overload: at
                                 least max_batch_queries queries wait and the first request would
                                 miss its deadline even if served now; < n_streams.  At light load
                                 fewer batches then share the GPU; under overload the extra
                                 batches keep it busy between the phases of the others */
  const uint32_t *tune_k;     /* n_tune_k result counts the server expects (may be NULL): at
                                 creation the autotuner times every batch shape of 1, 2, 4, ...
                                 up to max_batch_queries queries with each of these k over all
                                 strides (fps_tune), so that no request waits for tuning.  A
                                 batch whose shape was not tuned never times candidates on the
                                 request path: it takes a fixed default kernel choice and counts
                                 in fps_server_stats.untuned_batches */
  uint32_t n_tune_k;
} fps_server_config;

typedef struct {
  uint64_t arrival_ns;  /* steady-clock times (fps_clock_ns): the request's arrival, */
  uint64_t submit_ns;   /* its admission into the server's queue, */
  uint64_t start_ns;    /* the launch of its batch and */
  uint64_t done_ns;     /* the moment its results were available */
  uint32_t batch_id;
  uint32_t batch_queries;
} fps_request_stats;

typedef struct {
  uint64_t requests;         /* completed requests */
  uint64_t queries;
  uint64_t batches;
  uint64_t deadline_misses;  /* requests completed more than deadline_us after arrival */
  double p50_us, p99_us, max_us; /* latency from arrival to completion */
  double mean_batch_queries;
  double cost_fixed_us;      /* fitted service time of a batch: cost_fixed_us + */
  double cost_per_weight_us; /* cost_per_weight_us * sum of q * (1 + k / 700) over its requests */
  double admit_p50_us, admit_p99_us; /* wait from arrival to admission (queue full) */
  uint64_t untuned_batches;  /* batches whose shape the autotuner had not timed */
} fps_server_stats;

/*
 * Creates a server over a loaded library.  workspace/ws_bytes: caller-owned
 * device memory, carved into n_streams slots.  The server owns one worker
 * thread and n_streams HIP streams (default priority).
 */
fps_status fps_server_create(fps_library *lib, const fps_server_config *cfg, void *workspace,
                             size_t ws_bytes, fps_server **out);

/*
 * Queues one request of q queries (host memory, copied before return) with one k
 * and one stride mask.  deadline_us is the request's latency budget from its
 * arrival (counted as a miss when exceeded; the request still completes).
 * arrival_ns is the request's arrival time on the steady clock of
 * fps_clock_ns (0 = the moment of this call); latency and deadlines are
 * counted from it, so the time a request spends before admission -- in a
 * client's queue or blocked in this call -- is part of its latency.  Blocks
 * while the pool lacks room for the request unless nonblocking != 0, which
 * returns FPS_E_BUSY instead.  A request larger than a whole slot is rejected
 * with FPS_E_NOMEM.
 */
fps_status fps_server_submit(fps_server *srv, const uint64_t *queries, uint32_t q, uint32_t k,
                             uint32_t mask, uint32_t deadline_us, uint64_t arrival_ns,
                             int nonblocking, uint64_t *ticket);

/*
 * Waits until a request is done and reports the size of its result: *q
 * queries (out_offset needs q + 1 entries) and *n_hits hits (the sum over its
 * queries of min(k, n_eff)).  The ticket stays valid.  Either pointer may be
 * NULL.  Errors: FPS_E_ARG (unknown ticket).
 */
fps_status fps_server_result_size(fps_server *srv, uint64_t ticket, uint32_t *q,
                                  uint64_t *n_hits);

/*
 * Waits for a request and copies its results: out has out_capacity hits,
 * out_offset offset_capacity entries (q + 1 are written, as fps_search_batch).
 * stats may be NULL.  The ticket is consumed only when the results are
 * delivered: a too-small buffer returns FPS_E_ARG (the message states the
 * sizes needed) and the same ticket can be waited for again.  A failed
 * request returns its error and consumes the ticket.
 */
fps_status fps_server_wait(fps_server *srv, uint64_t ticket, fps_hit *out, uint64_t out_capacity,
                           uint64_t *out_offset, uint64_t offset_capacity,
                           fps_request_stats *stats);

/* Latency and throughput counters since creation (or the last reset).  The
 * counts cover every request; the latency percentiles and maximum cover the
 * last 1,048,576 requests (a bounded window for long-running servers). */
fps_status fps_server_stats_get(fps_server *srv, fps_server_stats *stats, int reset);

/* Drains outstanding requests and releases the server (never the workspace). */
fps_status fps_server_destroy(fps_server *srv);

/* Now on the steady clock used by the server's time stamps, in nanoseconds. */
uint64_t fps_clock_ns(void);

/* Message of the last failure on the calling thread. */
const char *fps_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FPS_H */
