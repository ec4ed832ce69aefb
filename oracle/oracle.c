/*
 * CPU ORACLE -- test infrastructure, not part of the product.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this file's library.  It shares no code, header, table or helper with the GPU
 * path, and it is deliberately plain and slow.
 *
 * What it computes (FPScreen, Section 4.3 and Fig. 3):
 *   - the Manhattan distance between two 166-key fingerprints,
 *       dist(a, b) = sum over j = 1..166 of |a_j - b_j|          (Section 4.3 equation)
 *     evaluated literally, key by key, with an integer subtraction and an
 *     absolute value -- Fig. 3 steps 3 and 4 (C = A - b, K = SUM(ABS(C))) for
 *     one row of A at a time;
 *   - pairing each record's index with its distance (Fig. 3 step 5) and keeping
 *     the first N in ascending order (Fig. 3 step 6), N being the caller's k.
 *     The paper states no tie rule; equal distances are ordered by ascending
 *     library index, so the answer is unique;
 *   - a library split into strides: the answer over a set of strides is the
 *     answer over the union of their records, indices staying global; the
 *     threaded form searches contiguous chunks separately and then combines and
 *     sorts their results (Section 2.1 strides; the combine rule of Section 4.3).
 *
 * Fingerprint layout: key j (1..166) is bit (j & 63) of 64-bit word (j >> 6) of a
 * record of three words; records are stored record-major.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_KEYS 166

typedef struct {
  uint32_t index;
  uint32_t distance;
} oracle_hit;

/* Value (0 or 1) of key j of a record. */
static int key_value(const uint64_t *rec, int j) {
  return (int)((rec[j >> 6] >> (j & 63)) & 1u);
}

/* Section 4.3 equation: sum over j = 1..n of |a_j - b_j|, n = 166. */
uint32_t oracle_distance(const uint64_t *a, const uint64_t *b) {
  int sum = 0;
  for (int j = 1; j <= ORACLE_KEYS; ++j) {
    int c = key_value(a, j) - key_value(b, j); /* Fig. 3 step 3 */
    sum += (c < 0) ? -c : c;                   /* Fig. 3 step 4 */
  }
  return (uint32_t)sum;
}

/* Distances of records [begin, end) to the query, written to out[i - begin]. */
void oracle_distances(const uint64_t *lib, uint64_t begin, uint64_t end, const uint64_t *query,
                      uint32_t *out) {
  for (uint64_t i = begin; i < end; ++i) out[i - begin] = oracle_distance(lib + 3 * i, query);
}

/* (d, index) order: ascending distance, then ascending index. */
static int hit_less(uint32_t d0, uint32_t i0, uint32_t d1, uint32_t i1) {
  return d0 < d1 || (d0 == d1 && i0 < i1);
}

/* A list holding the `cap` smallest hits seen so far, sorted ascending. */
typedef struct {
  oracle_hit *h;
  uint64_t len, cap;
} topk_list;

static void topk_offer(topk_list *t, uint32_t idx, uint32_t d) {
  if (t->cap == 0) return;
  if (t->len == t->cap && !hit_less(d, idx, t->h[t->len - 1].distance, t->h[t->len - 1].index))
    return; /* not smaller than the current N-th */
  /* position: first entry that is larger than the new hit */
  uint64_t lo = 0, hi = t->len;
  while (lo < hi) {
    uint64_t mid = (lo + hi) / 2;
    if (hit_less(t->h[mid].distance, t->h[mid].index, d, idx)) lo = mid + 1;
    else hi = mid;
  }
  uint64_t keep = (t->len == t->cap) ? t->len - 1 : t->len;
  memmove(t->h + lo + 1, t->h + lo, (keep - lo) * sizeof(oracle_hit));
  t->h[lo].index = idx;
  t->h[lo].distance = d;
  if (t->len < t->cap) t->len++;
}

/* Serial search of record ranges [begin[r], end[r]) in ascending index order. */
static void search_ranges(const uint64_t *lib, const uint64_t *begin, const uint64_t *end,
                          uint32_t nranges, const uint64_t *query, topk_list *t) {
  for (uint32_t r = 0; r < nranges; ++r)
    for (uint64_t i = begin[r]; i < end[r]; ++i)
      topk_offer(t, (uint32_t)i, oracle_distance(lib + 3 * i, query));
}

typedef struct {
  const uint64_t *lib;
  const uint64_t *query;
  uint64_t begin, end;
  topk_list list;
} chunk_job;

static void *chunk_worker(void *arg) {
  chunk_job *c = (chunk_job *)arg;
  search_ranges(c->lib, &c->begin, &c->end, 1, c->query, &c->list);
  return NULL;
}

/*
 * Top-k of one query over the union of record ranges.
 *   lib:      n x 3 uint64, record-major (host memory).
 *   begin/end: nranges disjoint ranges of global record indices.
 *   k:        number of results wanted; min(k, records in the ranges) are returned.
 *   out:      room for that many hits, written in (distance, index) order.
 *   nthreads: 1 for the serial form; > 1 splits every range into contiguous chunks
 *             searched in parallel and then combined and sorted.
 * Returns the number of hits, or -1 if memory runs out.
 */
int64_t oracle_search(const uint64_t *lib, const uint64_t *begin, const uint64_t *end,
                      uint32_t nranges, const uint64_t *query, uint64_t k, oracle_hit *out,
                      int nthreads) {
  uint64_t total = 0;
  for (uint32_t r = 0; r < nranges; ++r) total += end[r] - begin[r];
  uint64_t want = k < total ? k : total;
  topk_list t = {out, 0, want};
  if (nthreads <= 1 || total < 4096) {
    search_ranges(lib, begin, end, nranges, query, &t);
    return (int64_t)t.len;
  }
  if (nthreads > 256) nthreads = 256;
  /* contiguous chunks of the concatenated ranges, one per thread */
  chunk_job *jobs = (chunk_job *)calloc((size_t)nthreads * nranges, sizeof(chunk_job));
  pthread_t *th = (pthread_t *)calloc((size_t)nthreads * nranges, sizeof(pthread_t));
  if (!jobs || !th) {
    free(jobs);
    free(th);
    return -1;
  }
  int njobs = 0, failed = 0;
  for (uint32_t r = 0; r < nranges; ++r) {
    uint64_t len = end[r] - begin[r];
    int parts = (int)((len * (uint64_t)nthreads + total - 1) / total);
    if (parts < 1) parts = 1;
    for (int p = 0; p < parts; ++p) {
      chunk_job *c = &jobs[njobs++];
      c->lib = lib;
      c->query = query;
      c->begin = begin[r] + len * (uint64_t)p / (uint64_t)parts;
      c->end = begin[r] + len * (uint64_t)(p + 1) / (uint64_t)parts;
      c->list.cap = want;
      c->list.len = 0;
      c->list.h = (oracle_hit *)malloc((want ? want : 1) * sizeof(oracle_hit));
      if (!c->list.h) failed = 1;
    }
  }
  if (!failed) {
    for (int j = 1; j < njobs; ++j) pthread_create(&th[j], NULL, chunk_worker, &jobs[j]);
    chunk_worker(&jobs[0]);
    for (int j = 1; j < njobs; ++j) pthread_join(th[j], NULL);
    /* combine and sort (Section 4.3): offer every chunk's hits to one list */
    for (int j = 0; j < njobs; ++j)
      for (uint64_t i = 0; i < jobs[j].list.len; ++i)
        topk_offer(&t, jobs[j].list.h[i].index, jobs[j].list.h[i].distance);
  }
  for (int j = 0; j < njobs; ++j) free(jobs[j].list.h);
  free(jobs);
  free(th);
  return failed ? -1 : (int64_t)t.len;
}

/*
 * Batch form: query q (queries + 3q) with its own k[q] and ranges
 * [begin[q*nranges_max + r], end[...]) for r < nranges[q]; its hits start at
 * out + offset[q], and offset[q + 1] - offset[q] hits are written.
 * offset has nq + 1 entries and is filled by this call.  Returns 0 or -1.
 */
int oracle_search_batch(const uint64_t *lib, const uint64_t *begin, const uint64_t *end,
                        const uint32_t *nranges, uint32_t nranges_max, const uint64_t *queries,
                        uint64_t nq, const uint64_t *k, oracle_hit *out, uint64_t *offset,
                        int nthreads) {
  offset[0] = 0;
  for (uint64_t q = 0; q < nq; ++q) {
    int64_t got = oracle_search(lib, begin + q * nranges_max, end + q * nranges_max, nranges[q],
                                queries + 3 * q, k[q], out + offset[q], nthreads);
    if (got < 0) return -1;
    offset[q + 1] = offset[q] + (uint64_t)got;
  }
  return 0;
}

/*
 * The library file F of Fig. 3 step 1 ("obtain all the molecules from F,
 * construct CID, matrix A"), read line by line as the paper's engine does
 * (Abstract: one line of MACCS text per molecule).  The paper does not print
 * the line format; the reading taken is
 *     <id> <separator> <keys> [trailing blanks] <end of line>
 *   id:        1..19 decimal digits (the PubChem CID);
 *   separator: one or more of ' ', '\t', ',';
 *   keys:      167 characters '0'/'1' for positions 0..166 (position 0 holds
 *              no key and must be '0'), or 166 characters for keys 1..166;
 *   blanks:    ' ', '\t', '\r' only;
 *   a line has at most 255 characters before its '\n'; the last line may
 *   lack the '\n'; a '\n' that ends the text starts no further line.
 * Checks, in this order, name the first problem of a line:
 *   1 line too long, 2 id missing or longer than 19 digits, 3 no separator,
 *   4 keys not 166 or 167 characters '0'/'1', 5 position 0 set, 6 other
 *   characters after the keys.
 * Returns the number of records (lines) read, or -1 when a line is malformed
 * (*err_line = its 1-based number, *err_kind = the problem) or more than cap
 * records are present (*err_kind = 0).
 */
#define ORACLE_LINE_MAX 255

static int is_digit(char c) { return c >= '0' && c <= '9'; }
static int is_sep(char c) { return c == ' ' || c == '\t' || c == ','; }
static int is_blank(char c) { return c == ' ' || c == '\t' || c == '\r'; }

static int read_line(const char *s, uint64_t len, uint64_t rec[3], uint64_t *id) {
  if (len > ORACLE_LINE_MAX) return 1;
  uint64_t p = 0;
  uint64_t v = 0;
  while (p < len && is_digit(s[p])) {
    if (p < 19) v = v * 10 + (uint64_t)(s[p] - '0');
    ++p;
  }
  if (p == 0 || p > 19) return 2;
  uint64_t q = p;
  while (q < len && is_sep(s[q])) ++q;
  if (q == p) return 3;
  uint64_t r = q;
  while (r < len && (s[r] == '0' || s[r] == '1')) ++r;
  uint64_t width = r - q;
  if (width != 166 && width != 167) return 4;
  /* character c of the key field is key c (167 wide) or key c + 1 (166 wide) */
  uint64_t first_key = (width == 167) ? 0 : 1;
  rec[0] = rec[1] = rec[2] = 0;
  for (uint64_t c = 0; c < width; ++c) {
    uint64_t j = first_key + c;
    if (s[q + c] == '1') {
      if (j == 0) return 5;
      rec[j >> 6] |= 1ull << (j & 63);
    }
  }
  for (uint64_t t = r; t < len; ++t)
    if (!is_blank(s[t])) return 6;
  *id = v;
  return 0;
}

int64_t oracle_read_text(const char *text, uint64_t len, uint64_t *words, uint64_t *ids,
                         uint64_t cap, uint64_t *err_line, int *err_kind) {
  uint64_t n = 0, pos = 0;
  *err_line = 0;
  *err_kind = 0;
  while (pos < len) {
    uint64_t end = pos;
    while (end < len && text[end] != '\n') ++end;
    if (n == cap) {
      *err_line = n + 1;
      return -1;
    }
    int kind = read_line(text + pos, end - pos, words + 3 * n, ids + n);
    if (kind) {
      *err_line = n + 1;
      *err_kind = kind;
      return -1;
    }
    ++n;
    pos = end + 1; /* past the '\n' (or past the end of the text) */
  }
  return (int64_t)n;
}

/*
 * Wider fingerprints (Section 5, concluding remark 3: more features): records
 * of `words` 64-bit words, keys 0 .. 64 * words - 1, key j at bit (j & 63) of
 * word (j >> 6); every bit is a key.  The distance is again the Section 4.3
 * sum, now over all 64 * words keys, and the top-k, tie rule, strides and the
 * threaded combine-and-sort are those above.
 */
static int key_value_w(const uint64_t *rec, uint32_t j) {
  return (int)((rec[j >> 6] >> (j & 63)) & 1u);
}

uint32_t oracle_distance_w(const uint64_t *a, const uint64_t *b, uint32_t words) {
  int sum = 0;
  for (uint32_t j = 0; j < 64 * words; ++j) {
    int c = key_value_w(a, j) - key_value_w(b, j); /* Fig. 3 step 3 */
    sum += (c < 0) ? -c : c;                       /* Fig. 3 step 4 */
  }
  return (uint32_t)sum;
}

void oracle_distances_w(const uint64_t *lib, uint32_t words, uint64_t begin, uint64_t end,
                        const uint64_t *query, uint32_t *out) {
  for (uint64_t i = begin; i < end; ++i)
    out[i - begin] = oracle_distance_w(lib + (uint64_t)words * i, query, words);
}

static void search_ranges_w(const uint64_t *lib, uint32_t words, const uint64_t *begin,
                            const uint64_t *end, uint32_t nranges, const uint64_t *query,
                            topk_list *t) {
  for (uint32_t r = 0; r < nranges; ++r)
    for (uint64_t i = begin[r]; i < end[r]; ++i)
      topk_offer(t, (uint32_t)i, oracle_distance_w(lib + (uint64_t)words * i, query, words));
}

typedef struct {
  const uint64_t *lib;
  const uint64_t *query;
  uint32_t words;
  uint64_t begin, end;
  topk_list list;
} chunk_job_w;

static void *chunk_worker_w(void *arg) {
  chunk_job_w *c = (chunk_job_w *)arg;
  search_ranges_w(c->lib, c->words, &c->begin, &c->end, 1, c->query, &c->list);
  return NULL;
}

/* oracle_search for records of `words` words (arguments as oracle_search). */
int64_t oracle_search_w(const uint64_t *lib, uint32_t words, const uint64_t *begin,
                        const uint64_t *end, uint32_t nranges, const uint64_t *query, uint64_t k,
                        oracle_hit *out, int nthreads) {
  uint64_t total = 0;
  for (uint32_t r = 0; r < nranges; ++r) total += end[r] - begin[r];
  uint64_t want = k < total ? k : total;
  topk_list t = {out, 0, want};
  if (nthreads <= 1 || total < 4096) {
    search_ranges_w(lib, words, begin, end, nranges, query, &t);
    return (int64_t)t.len;
  }
  if (nthreads > 256) nthreads = 256;
  chunk_job_w *jobs = (chunk_job_w *)calloc((size_t)nthreads * nranges, sizeof(chunk_job_w));
  pthread_t *th = (pthread_t *)calloc((size_t)nthreads * nranges, sizeof(pthread_t));
  if (!jobs || !th) {
    free(jobs);
    free(th);
    return -1;
  }
  int njobs = 0, failed = 0;
  for (uint32_t r = 0; r < nranges; ++r) {
    uint64_t len = end[r] - begin[r];
    int parts = (int)((len * (uint64_t)nthreads + total - 1) / total);
    if (parts < 1) parts = 1;
    for (int p = 0; p < parts; ++p) {
      chunk_job_w *c = &jobs[njobs++];
      c->lib = lib;
      c->query = query;
      c->words = words;
      c->begin = begin[r] + len * (uint64_t)p / (uint64_t)parts;
      c->end = begin[r] + len * (uint64_t)(p + 1) / (uint64_t)parts;
      c->list.cap = want;
      c->list.len = 0;
      c->list.h = (oracle_hit *)malloc((want ? want : 1) * sizeof(oracle_hit));
      if (!c->list.h) failed = 1;
    }
  }
  if (!failed) {
    for (int j = 1; j < njobs; ++j) pthread_create(&th[j], NULL, chunk_worker_w, &jobs[j]);
    chunk_worker_w(&jobs[0]);
    for (int j = 1; j < njobs; ++j) pthread_join(th[j], NULL);
    for (int j = 0; j < njobs; ++j) /* combine and sort (Section 4.3) */
      for (uint64_t i = 0; i < jobs[j].list.len; ++i)
        topk_offer(&t, jobs[j].list.h[i].index, jobs[j].list.h[i].distance);
  }
  for (int j = 0; j < njobs; ++j) free(jobs[j].list.h);
  free(jobs);
  free(th);
  return failed ? -1 : (int64_t)t.len;
}
