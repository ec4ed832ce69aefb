// Host-side check of the fp4 digit arithmetic of the matrix-core scan
// (csrc/f4_digits.h), with an e2m1 decoder written here from the format's
// definition (sign bit 3, exponent bits 2..1 with bias 1, mantissa bit 0).
//
// Part 1 (exhaustive): the |r| digits of every count 0..167, the sentinel of
// every invalid count, and the bias digits of every B in -167..167.
// Part 2 (one tile): reads query rows (three key words, T, valid flag) and
// records (three key words, valid flag) from stdin, lays their digits out as
// the kernel's operand fragments do (keys relabeled into the library words,
// 2-bit groups through a byte permutation of the digit tables, spare digits
// in the d fragment), and prints u = the fragments' dot product for every
// pair.  The caller compares u with d - T - 1 from the oracle's distance.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "f4_digits.h"

using namespace fps;

static double e2m1(uint32_t nib) {
  const uint32_t s = (nib >> 3) & 1u, e = (nib >> 1) & 3u, m = nib & 1u;
  const double v = e == 0 ? 0.5 * m : std::ldexp(1.0 + 0.5 * m, (int)e - 1);
  return s ? -v : v;
}

static uint32_t nibble(uint32_t x, int i) { return (x >> (4 * i)) & 0xFu; }

// Value of seven digits in nibbles 0..6 weighted 6,6,6,6,6,6,1.
static double six_one_value(uint32_t pat) {
  double v = 0;
  for (int i = 0; i < 6; ++i) v += 6.0 * e2m1(nibble(pat, i));
  return v + e2m1(nibble(pat, 6));
}

// v_perm_b32 with both sources equal to t: result byte i is byte (sel_i & 3)
// of t for selector bytes 0..3 (the only ones used).
static uint32_t perm_same(uint32_t t, uint32_t sel) {
  uint32_t r = 0;
  for (int i = 0; i < 4; ++i) {
    const uint32_t s = (sel >> (8 * i)) & 0xFFu;
    r |= ((t >> (8 * (s & 3u))) & 0xFFu) << (8 * i);
  }
  return r;
}

static void spread(uint32_t c, uint32_t table, uint32_t *o) {
  for (int j = 0; j < 4; ++j) o[j] = perm_same(table, (c >> (2 * j)) & 0x03030303u);
}

// Library words of a fingerprint (key j at bit j & 63 of word j >> 6): keys
// 1..63 and key 160 (bit 0) in a, 64..127 in b, 128..159 in c, 161..166 in d.
static void relabel(const uint64_t w[3], uint32_t ch[6]) {
  const uint64_t a = w[0] | ((w[2] >> 32) & 1ull), b = w[1];
  ch[0] = (uint32_t)a;
  ch[1] = (uint32_t)(a >> 32);
  ch[2] = (uint32_t)b;
  ch[3] = (uint32_t)(b >> 32);
  ch[4] = (uint32_t)w[2];
  ch[5] = (uint32_t)((w[2] >> 33) & 0x3Full);
}

static int popc(const uint32_t ch[6]) {
  int p = 0;
  for (int i = 0; i < 6; ++i) p += __builtin_popcount(ch[i]);
  return p;
}

int main() {
  // ---- part 1 ----
  int bad = 0;
  for (uint32_t p = 0; p <= 167; ++p) {
    const uint32_t pat = six_one_digits(p);
    if (six_one_value(pat) != (double)p || nibble(pat, 7) != 0) ++bad;
    for (int i = 0; i < 7; ++i)
      if (nibble(pat, i) & 8u) ++bad;  // no negative digit
  }
  std::printf("six_one_bad %d\n", bad);
  bad = 0;
  for (uint32_t p = 0; p < 256; ++p) {
    const double want = p <= kF4MaxCount ? (double)p : 216.0;
    if (six_one_value(pop_digits(p)) != want) ++bad;
  }
  std::printf("pop_bad %d\n", bad);
  bad = 0;
  for (int b = -167; b <= 167; ++b)
    if (six_one_value(bias_digits(b)) != (double)b) ++bad;
  std::printf("bias_bad %d\n", bad);
  // ---- part 2 ----
  int nq = 0, nr = 0;
  if (std::scanf("%d %d", &nq, &nr) != 2) return 0;
  std::vector<uint32_t> A((size_t)nq * 24), B((size_t)nr * 24);
  for (int q = 0; q < nq; ++q) {
    unsigned long long w[3];
    long long T;
    int valid;
    if (std::scanf("%llu %llu %llu %lld %d", &w[0], &w[1], &w[2], &T, &valid) != 5) return 2;
    const uint64_t ww[3] = {w[0], w[1], w[2]};
    uint32_t ch[6] = {0, 0, 0, 0, 0, 0};
    if (valid) relabel(ww, ch);
    const int32_t bias = valid ? popc(ch) - (int32_t)T - 1 : kInvalidRowBias;
    uint32_t *o = &A[(size_t)q * 24];
    for (int f = 0; f < 6; ++f) spread(ch[f], kDigitsQuery, o + 4 * f);
    const uint32_t bd = bias_digits(bias);
    o[20] |= (bd & 0xFFFFFFu) << 8;
    o[21] |= ((bd >> 24) & 0xFu) << 8;
    o[23] = valid ? kQueryPopDigits : 0u;
  }
  for (int r = 0; r < nr; ++r) {
    unsigned long long w[3];
    int valid;
    if (std::scanf("%llu %llu %llu %d", &w[0], &w[1], &w[2], &valid) != 4) return 2;
    const uint64_t ww[3] = {w[0], w[1], w[2]};
    uint32_t ch[6] = {0, 0, 0, 0, 0, 0};
    if (valid) relabel(ww, ch);
    uint32_t *o = &B[(size_t)r * 24];
    for (int f = 0; f < 6; ++f) spread(ch[f], kDigitsRecord, o + 4 * f);
    o[23] = pop_digits(valid ? (uint32_t)popc(ch) : 255u);
    o[20] |= kRecordBiasDw0;
    o[21] |= kRecordBiasDw1;
  }
  for (int q = 0; q < nq; ++q)
    for (int r = 0; r < nr; ++r) {
      double u = 0;
      for (int x = 0; x < 24; ++x)
        for (int i = 0; i < 8; ++i)
          u += e2m1(nibble(A[(size_t)q * 24 + x], i)) * e2m1(nibble(B[(size_t)r * 24 + x], i));
      std::printf("u %d %d %.1f\n", q, r, u);
    }
  return 0;
}
