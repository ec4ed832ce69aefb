/*
 * Seeded synthetic MACCS-166-shaped fingerprints: the input generator shared by
 * the CPU oracle's tests and the GPU path's tests and benchmark.
 *
 * This file holds no part of the search method (no distance, no ranking): it
 * only draws bits.  A fingerprint has 166 binary keys numbered 1..166 (the key
 * table of Section 4.2 starts at key 1 and the distance formula of Section 4.3
 * sums j = 1..166); key j lives in 64-bit word j >> 6 at bit j & 63, so bit 0
 * and bits 167..191 of the three words are always zero.
 *
 * Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used as a counter-based
 * generator: every draw is the hash of (seed, purpose tag, record, counter), so
 * generation is reproducible whatever the thread count.
 *
 * Library model (stand-in for the PubChem MACCS library, which is not shipped):
 *   - per-key set probabilities p_j (drawn by the caller, Beta(0.6, 2.0));
 *   - a record is "fresh" (key j set with probability p_j, independently) or,
 *     with probability dup_frac and only for record index > 0, a copy of a
 *     uniformly chosen earlier record with F distinct keys flipped, F uniform in
 *     [flip_lo, flip_hi].  Section 3.3 shows distinct molecules at distance 0;
 *     copies with zero flips reproduce that.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NKEYS 166
#define TAG_BITS 0x62697473ULL  /* "bits" */
#define TAG_DUP 0x64757073ULL   /* "dups" */
#define TAG_QRY 0x71727973ULL   /* "qrys" */

static inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

/* Key of an independent stream for (seed, tag, item). */
static inline uint64_t stream_key(uint64_t seed, uint64_t tag, uint64_t item) {
  return splitmix64(splitmix64(splitmix64(seed) ^ tag) + item);
}

/* Uniform integer in [0, m) from a 64-bit draw (Lemire's multiply-shift; the
 * bias is below 2^-32 for m < 2^32). */
static inline uint64_t below(uint64_t r, uint64_t m) {
  return (uint64_t)(((unsigned __int128)r * m) >> 64);
}

/* Fresh record: key j set iff a 32-bit uniform is below thr[j]. */
static void fresh_bits(uint64_t key, const uint32_t *thr, uint64_t out[3]) {
  out[0] = out[1] = out[2] = 0;
  for (int t = 0; t < NKEYS / 2; ++t) {
    uint64_t r = splitmix64(key + (uint64_t)t);
    int j0 = 2 * t + 1, j1 = 2 * t + 2;
    if ((uint32_t)r < thr[j0]) out[j0 >> 6] |= 1ULL << (j0 & 63);
    if ((uint32_t)(r >> 32) < thr[j1]) out[j1 >> 6] |= 1ULL << (j1 & 63);
  }
}

/* Flip `nflips` distinct keys drawn from the stream `key`; positions written
 * to pos[] (sorted is not required). */
static void flip_distinct(uint64_t key, int nflips, uint64_t rec[3], uint8_t *pos) {
  int got = 0;
  uint64_t ctr = 0;
  while (got < nflips) {
    int j = 1 + (int)below(splitmix64(key + 1000 + ctr++), NKEYS);
    int dup = 0;
    for (int a = 0; a < got; ++a) dup |= (pos[a] == j);
    if (dup) continue;
    pos[got++] = (uint8_t)j;
    rec[j >> 6] ^= 1ULL << (j & 63);
  }
}

typedef struct {
  uint64_t seed, begin, end;
  const uint32_t *thr;
  uint64_t *words;
} fresh_job;

static void *fresh_worker(void *arg) {
  fresh_job *jb = (fresh_job *)arg;
  for (uint64_t i = jb->begin; i < jb->end; ++i)
    fresh_bits(stream_key(jb->seed, TAG_BITS, i), jb->thr, jb->words + 3 * i);
  return NULL;
}

static void run_fresh(uint64_t seed, uint64_t n, const uint32_t *thr, uint64_t *words,
                      int nthreads) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  pthread_t th[256];
  fresh_job jobs[256];
  for (int t = 0; t < nthreads; ++t) {
    jobs[t].seed = seed;
    jobs[t].begin = n * (uint64_t)t / (uint64_t)nthreads;
    jobs[t].end = n * (uint64_t)(t + 1) / (uint64_t)nthreads;
    jobs[t].thr = thr;
    jobs[t].words = words;
  }
  for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, fresh_worker, &jobs[t]);
  fresh_worker(&jobs[0]);
  for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/*
 * Library of n records, record-major (record i = words[3i .. 3i+2]).
 * thr[192]: per-bit 32-bit thresholds (thr[0] and thr[167..191] must be 0).
 * dup_src[i]: source record of a near-duplicate, or -1 for a fresh record.
 * dup_flips[i]: number of keys flipped relative to the source (0 if fresh).
 * Any of dup_src / dup_flips may be NULL.  Returns 0, or -1 on bad arguments.
 */
int fpsynth_library(uint64_t seed, uint64_t n, const uint32_t *thr, double dup_frac,
                    int flip_lo, int flip_hi, uint64_t *words, int32_t *dup_src,
                    uint8_t *dup_flips, int nthreads) {
  if (!thr || !words || flip_lo < 0 || flip_hi < flip_lo || flip_hi > NKEYS) return -1;
  if (thr[0] != 0) return -1;
  for (int j = NKEYS + 1; j < 192; ++j)
    if (thr[j] != 0) return -1;
  run_fresh(seed, n, thr, words, nthreads);
  const double scale = 9007199254740992.0; /* 2^53 */
  const uint64_t cut = (uint64_t)(dup_frac * scale);
  for (uint64_t i = 0; i < n; ++i) {
    int32_t src = -1;
    int nf = 0;
    if (i > 0) {
      uint64_t key = stream_key(seed, TAG_DUP, i);
      if ((splitmix64(key) >> 11) < cut) {
        src = (int32_t)below(splitmix64(key + 1), i);
        nf = flip_lo + (int)below(splitmix64(key + 2), (uint64_t)(flip_hi - flip_lo + 1));
        uint64_t *rec = words + 3 * i;
        memcpy(rec, words + 3 * (uint64_t)src, 3 * sizeof(uint64_t));
        uint8_t pos[NKEYS];
        flip_distinct(key, nf, rec, pos);
      }
    }
    if (dup_src) dup_src[i] = src;
    if (dup_flips) dup_flips[i] = (uint8_t)nf;
  }
  return 0;
}

/*
 * nq queries, record-major.  Query q is fresh (drawn from the same per-key model
 * as the library, from its own stream) when fresh[q] != 0; otherwise it is a
 * copy of a uniformly drawn library record with F distinct keys flipped, F
 * uniform in [flip_lo, flip_hi].  src[q] is that record (-1 for fresh) and
 * flips[q] the number of flipped keys.  Returns 0, or -1 on bad arguments.
 */
int fpsynth_queries(uint64_t seed, uint64_t nq, const uint64_t *lib, uint64_t n,
                    const uint32_t *thr, const uint8_t *fresh, int flip_lo, int flip_hi,
                    uint64_t *out, int64_t *src, uint8_t *flips) {
  if (!thr || !out || !fresh || flip_lo < 0 || flip_hi < flip_lo || flip_hi > NKEYS) return -1;
  for (uint64_t q = 0; q < nq; ++q) {
    uint64_t key = stream_key(seed, TAG_QRY, q);
    uint64_t *rec = out + 3 * q;
    if (fresh[q]) {
      fresh_bits(splitmix64(key + 7), thr, rec);
      if (src) src[q] = -1;
      if (flips) flips[q] = 0;
      continue;
    }
    if (!lib || n == 0) return -1;
    uint64_t s = below(splitmix64(key), n);
    int nf = flip_lo + (int)below(splitmix64(key + 1), (uint64_t)(flip_hi - flip_lo + 1));
    memcpy(rec, lib + 3 * s, 3 * sizeof(uint64_t));
    uint8_t pos[NKEYS];
    flip_distinct(key, nf, rec, pos);
    if (src) src[q] = (int64_t)s;
    if (flips) flips[q] = (uint8_t)nf;
  }
  return 0;
}

/*
 * Text form of a library: one line per record, "<id><sep><keys><eol>", the
 * shape of the paper's library file (Abstract: one line of MACCS text per
 * molecule; Fig. 3 step 1 reads molecules and their CIDs from it).
 *   width 167: the key characters are positions 0..166 ('0' at position 0,
 *              which holds no key), width 166: keys 1..166 only;
 *   ids[i]:    decimal, no leading zeros;
 *   sep:       any separator string (e.g. " ", "\t", ",");
 *   eol:       "\n", or "\r\n" when crlf != 0; final_eol = 0 leaves the last
 *              line unterminated.
 * This only formats the bits and ids it is given.
 */
static int dec_len(uint64_t v) {
  int l = 1;
  while (v >= 10) {
    v /= 10;
    ++l;
  }
  return l;
}

static uint64_t line_len(uint64_t id, int width, size_t seplen, int crlf) {
  return (uint64_t)dec_len(id) + seplen + (uint64_t)width + (crlf ? 2u : 1u);
}

uint64_t fpsynth_text_size(const uint64_t *ids, uint64_t n, int width, uint64_t seplen,
                           int crlf, int final_eol) {
  uint64_t total = 0;
  for (uint64_t i = 0; i < n; ++i) total += line_len(ids[i], width, (size_t)seplen, crlf);
  if (n && !final_eol) total -= crlf ? 2u : 1u;
  return total;
}

typedef struct {
  const uint64_t *words, *ids;
  uint64_t begin, end, offset;
  int width, crlf, final_eol;
  const char *sep;
  size_t seplen;
  uint64_t n;
  char *out;
} text_job;

static void *text_worker(void *arg) {
  text_job *jb = (text_job *)arg;
  char *p = jb->out + jb->offset;
  const int first = jb->width == 167 ? 0 : 1;
  for (uint64_t i = jb->begin; i < jb->end; ++i) {
    char digits[24];
    int nd = 0;
    uint64_t v = jb->ids[i];
    do {
      digits[nd++] = (char)('0' + v % 10);
      v /= 10;
    } while (v);
    while (nd) *p++ = digits[--nd];
    memcpy(p, jb->sep, jb->seplen);
    p += jb->seplen;
    const uint64_t *rec = jb->words + 3 * i;
    for (int j = first; j <= NKEYS; ++j) *p++ = (char)('0' + ((rec[j >> 6] >> (j & 63)) & 1u));
    if (i + 1 < jb->n || jb->final_eol) {
      if (jb->crlf) *p++ = '\r';
      *p++ = '\n';
    }
  }
  return NULL;
}

/* Writes the text of records [0, n) into out (fpsynth_text_size bytes).  Returns
 * 0, or -1 on bad arguments. */
int fpsynth_text_write(const uint64_t *words, const uint64_t *ids, uint64_t n, int width,
                       const char *sep, uint64_t seplen, int crlf, int final_eol, char *out,
                       int nthreads) {
  if (!words || !ids || !sep || !out || (width != 166 && width != 167)) return -1;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  pthread_t th[256];
  text_job jobs[256];
  uint64_t off = 0;
  for (int t = 0; t < nthreads; ++t) {
    text_job *jb = &jobs[t];
    jb->words = words;
    jb->ids = ids;
    jb->begin = n * (uint64_t)t / (uint64_t)nthreads;
    jb->end = n * (uint64_t)(t + 1) / (uint64_t)nthreads;
    jb->offset = off;
    jb->width = width;
    jb->crlf = crlf;
    jb->final_eol = final_eol;
    jb->sep = sep;
    jb->seplen = (size_t)seplen;
    jb->n = n;
    jb->out = out;
    for (uint64_t i = jb->begin; i < jb->end; ++i) off += line_len(ids[i], width, seplen, crlf);
  }
  for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, text_worker, &jobs[t]);
  text_worker(&jobs[0]);
  for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
  return 0;
}

/*
 * Wider fingerprints (records of `words` 64-bit words, every bit a key): key j
 * is set iff an 8-bit uniform draw is below thr8[j] (probability thr8[j] / 256;
 * eight draws per SplitMix64 output).  Near-duplicates as above: with
 * probability dup_frac a record (index > 0) copies a uniformly chosen earlier
 * record and flips F distinct keys, F uniform in [flip_lo, flip_hi].
 */
#define TAG_WIDE 0x77696465ULL  /* "wide" */

/* Bit b (0..7) of the result: byte b of r below byte b of t.  Even and odd
 * bytes are compared in 16-bit lanes (the borrow of (r_b | 0x100) - t_b
 * clears bit 8 iff r_b < t_b), then the eight flags are gathered. */
static inline uint32_t bytes_below(uint64_t r, uint64_t t) {
  const uint64_t M = 0x00FF00FF00FF00FFULL, H = 0x0100010001000100ULL;
  const uint64_t lt_e = ~(((r & M) | H) - (t & M)) & H;
  const uint64_t lt_o = ~((((r >> 8) & M) | H) - ((t >> 8) & M)) & H;
  const uint64_t x = (lt_e >> 8) | (lt_o >> 7);
  return (uint32_t)((x | (x >> 14) | (x >> 28) | (x >> 42)) & 0xFFu);
}

static void wide_fresh(uint64_t key, const uint8_t *thr8, uint32_t words, uint64_t *out) {
  for (uint32_t w = 0; w < words; ++w) {
    uint64_t v = 0;
    for (uint32_t g = 0; g < 8; ++g) {
      uint64_t r = splitmix64(key + 8 * (uint64_t)w + g);
      uint64_t t;
      memcpy(&t, thr8 + 64 * w + 8 * g, 8);
      v |= (uint64_t)bytes_below(r, t) << (8 * g);
    }
    out[w] = v;
  }
}

static void wide_flip(uint64_t key, int nflips, uint32_t words, uint64_t *rec) {
  uint32_t pos[64];
  int got = 0;
  uint64_t ctr = 0;
  while (got < nflips) {
    uint32_t j = (uint32_t)below(splitmix64(key + 1000 + ctr++), 64ULL * words);
    int dup = 0;
    for (int a = 0; a < got; ++a) dup |= (pos[a] == j);
    if (dup) continue;
    pos[got++] = j;
    rec[j >> 6] ^= 1ULL << (j & 63);
  }
}

typedef struct {
  uint64_t seed, begin, end;
  const uint8_t *thr8;
  uint32_t words;
  uint64_t *out;
} wide_job;

static void *wide_worker(void *arg) {
  wide_job *jb = (wide_job *)arg;
  for (uint64_t i = jb->begin; i < jb->end; ++i)
    wide_fresh(stream_key(jb->seed, TAG_WIDE, i), jb->thr8, jb->words,
               jb->out + (uint64_t)jb->words * i);
  return NULL;
}

int fpsynth_wide_library(uint64_t seed, uint64_t n, uint32_t words, const uint8_t *thr8,
                         double dup_frac, int flip_lo, int flip_hi, uint64_t *out,
                         int32_t *dup_src, uint8_t *dup_flips, int nthreads) {
  if (!thr8 || !out || words < 1 || words > 32 || flip_lo < 0 || flip_hi < flip_lo ||
      flip_hi > 64)
    return -1;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  pthread_t th[256];
  wide_job jobs[256];
  for (int t = 0; t < nthreads; ++t) {
    jobs[t].seed = seed;
    jobs[t].begin = n * (uint64_t)t / (uint64_t)nthreads;
    jobs[t].end = n * (uint64_t)(t + 1) / (uint64_t)nthreads;
    jobs[t].thr8 = thr8;
    jobs[t].words = words;
    jobs[t].out = out;
  }
  for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, wide_worker, &jobs[t]);
  wide_worker(&jobs[0]);
  for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
  const uint64_t cut = (uint64_t)(dup_frac * 9007199254740992.0);
  for (uint64_t i = 0; i < n; ++i) {
    int32_t src = -1;
    int nf = 0;
    if (i > 0) {
      uint64_t key = stream_key(seed, TAG_DUP ^ TAG_WIDE, i);
      if ((splitmix64(key) >> 11) < cut) {
        src = (int32_t)below(splitmix64(key + 1), i);
        nf = flip_lo + (int)below(splitmix64(key + 2), (uint64_t)(flip_hi - flip_lo + 1));
        memcpy(out + (uint64_t)words * i, out + (uint64_t)words * (uint64_t)src,
               words * sizeof(uint64_t));
        wide_flip(key, nf, words, out + (uint64_t)words * i);
      }
    }
    if (dup_src) dup_src[i] = src;
    if (dup_flips) dup_flips[i] = (uint8_t)nf;
  }
  return 0;
}

int fpsynth_wide_queries(uint64_t seed, uint64_t nq, const uint64_t *lib, uint64_t n,
                         uint32_t words, const uint8_t *thr8, const uint8_t *fresh, int flip_lo,
                         int flip_hi, uint64_t *out, int64_t *src, uint8_t *flips) {
  if (!thr8 || !out || !fresh || words < 1 || words > 32 || flip_lo < 0 || flip_hi < flip_lo ||
      flip_hi > 64)
    return -1;
  for (uint64_t q = 0; q < nq; ++q) {
    uint64_t key = stream_key(seed, TAG_QRY ^ TAG_WIDE, q);
    uint64_t *rec = out + (uint64_t)words * q;
    if (fresh[q]) {
      wide_fresh(splitmix64(key + 7), thr8, words, rec);
      if (src) src[q] = -1;
      if (flips) flips[q] = 0;
      continue;
    }
    if (!lib || n == 0) return -1;
    uint64_t s = below(splitmix64(key), n);
    int nf = flip_lo + (int)below(splitmix64(key + 1), (uint64_t)(flip_hi - flip_lo + 1));
    memcpy(rec, lib + (uint64_t)words * s, words * sizeof(uint64_t));
    wide_flip(key, nf, words, rec);
    if (src) src[q] = (int64_t)s;
    if (flips) flips[q] = (uint8_t)nf;
  }
  return 0;
}
