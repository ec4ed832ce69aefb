/*
 * Host-only check of the CPU oracle and the input generator, built with the
 * address / undefined-behaviour sanitizers and, separately, the thread
 * sanitizer (tests/test_sanitizers_cpu.py).  It generates a small library with
 * near-duplicates, and for several queries, k values and stride sets compares
 * the oracle's serial, threaded and batch forms with a brute force written
 * here: every distance from oracle_distance, then a plain sort by
 * (distance, index).  Prints "ok" and exits 0 when everything agrees.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  uint32_t index;
  uint32_t distance;
} hit;

/* oracle/oracle.c */
uint32_t oracle_distance(const uint64_t *a, const uint64_t *b);
int64_t oracle_search(const uint64_t *lib, const uint64_t *begin, const uint64_t *end,
                      uint32_t nranges, const uint64_t *query, uint64_t k, hit *out,
                      int nthreads);
int oracle_search_batch(const uint64_t *lib, const uint64_t *begin, const uint64_t *end,
                        const uint32_t *nranges, uint32_t nranges_max, const uint64_t *queries,
                        uint64_t nq, const uint64_t *k, hit *out, uint64_t *offset, int nthreads);
/* fpsynth/gen.c */
int fpsynth_library(uint64_t seed, uint64_t n, const uint32_t *thr, double dup_frac, int flip_lo,
                    int flip_hi, uint64_t *words, int32_t *dup_src, uint8_t *dup_flips,
                    int nthreads);
int fpsynth_queries(uint64_t seed, uint64_t nq, const uint64_t *lib, uint64_t n,
                    const uint32_t *thr, const uint8_t *fresh, int flip_lo, int flip_hi,
                    uint64_t *out, int64_t *src, uint8_t *flips);

static int by_key(const void *x, const void *y) {
  const hit *a = (const hit *)x, *b = (const hit *)y;
  if (a->distance != b->distance) return a->distance < b->distance ? -1 : 1;
  return a->index < b->index ? -1 : (a->index > b->index);
}

/* Brute force over the ranges: all distances, sorted, first min(k, total). */
static uint64_t brute(const uint64_t *lib, const uint64_t *begin, const uint64_t *end,
                      uint32_t nr, const uint64_t *q, uint64_t k, hit *out) {
  uint64_t total = 0;
  for (uint32_t r = 0; r < nr; ++r) total += end[r] - begin[r];
  hit *all = (hit *)malloc((total ? total : 1) * sizeof(hit));
  uint64_t m = 0;
  for (uint32_t r = 0; r < nr; ++r)
    for (uint64_t i = begin[r]; i < end[r]; ++i) {
      all[m].index = (uint32_t)i;
      all[m].distance = oracle_distance(lib + 3 * i, q);
      ++m;
    }
  qsort(all, m, sizeof(hit), by_key);
  const uint64_t want = k < m ? k : m;
  memcpy(out, all, want * sizeof(hit));
  free(all);
  return want;
}

int main(void) {
  enum { N = 9000, NQ = 8 };
  uint32_t thr[192] = {0};
  for (int j = 1; j <= 166; ++j)
    thr[j] = (uint32_t)((0.05 + 0.4 * (double)((j * 37) % 100) / 100.0) * 4294967296.0);
  uint64_t *lib = (uint64_t *)calloc(3 * (size_t)N, sizeof(uint64_t));
  uint64_t *qs = (uint64_t *)calloc(3 * (size_t)NQ, sizeof(uint64_t));
  uint8_t fresh[NQ];
  for (int i = 0; i < NQ; ++i) fresh[i] = (uint8_t)(i & 1);
  if (fpsynth_library(7, N, thr, 0.05, 0, 3, lib, NULL, NULL, 3) != 0) return 10;
  if (fpsynth_queries(8, NQ, lib, N, thr, fresh, 0, 5, qs, NULL, NULL) != 0) return 11;

  const uint64_t b_all[1] = {0}, e_all[1] = {N};
  const uint64_t b_two[2] = {0, 6000}, e_two[2] = {2500, N};
  const uint64_t ks[4] = {1, 7, 30, N + 5};
  hit *want = (hit *)malloc(((size_t)N + 5) * sizeof(hit));
  hit *got = (hit *)malloc(((size_t)N + 5) * sizeof(hit));
  int bad = 0;
  for (int q = 0; q < NQ; ++q)
    for (int kk = 0; kk < 4; ++kk)
      for (int rs = 0; rs < 2; ++rs) {
        const uint64_t *b = rs ? b_two : b_all, *e = rs ? e_two : e_all;
        const uint32_t nr = rs ? 2 : 1;
        const uint64_t nw = brute(lib, b, e, nr, qs + 3 * q, ks[kk], want);
        for (int th = 1; th <= 4; th += 3) {
          const int64_t ng = oracle_search(lib, b, e, nr, qs + 3 * q, ks[kk], got, th);
          if (ng != (int64_t)nw || memcmp(got, want, nw * sizeof(hit)) != 0) {
            fprintf(stderr, "mismatch q=%d k=%llu ranges=%u threads=%d\n", q,
                    (unsigned long long)ks[kk], nr, th);
            bad = 1;
          }
        }
      }
  /* batch form: per-query k and ranges (one or two), threaded */
  {
    uint64_t bb[2 * NQ], ee[2 * NQ], k[NQ], off[NQ + 1], total = 0;
    uint32_t nr[NQ];
    for (int q = 0; q < NQ; ++q) {
      nr[q] = (q % 3 == 0) ? 2 : 1;
      bb[2 * q] = nr[q] == 2 ? b_two[0] : 0;
      ee[2 * q] = nr[q] == 2 ? e_two[0] : N;
      bb[2 * q + 1] = b_two[1];
      ee[2 * q + 1] = e_two[1];
      k[q] = ks[q % 4];
      total += k[q] < N ? k[q] : N;
    }
    hit *out = (hit *)malloc(total * sizeof(hit));
    if (oracle_search_batch(lib, bb, ee, nr, 2, qs, NQ, k, out, off, 4) != 0) bad = 1;
    for (int q = 0; q < NQ && !bad; ++q) {
      const uint64_t nw = brute(lib, bb + 2 * q, ee + 2 * q, nr[q], qs + 3 * q, k[q], want);
      if (off[q + 1] - off[q] != nw || memcmp(out + off[q], want, nw * sizeof(hit)) != 0) {
        fprintf(stderr, "batch mismatch q=%d\n", q);
        bad = 1;
      }
    }
    free(out);
  }
  free(want);
  free(got);
  free(lib);
  free(qs);
  if (bad) return 1;
  printf("ok\n");
  return 0;
}
