// Digits of the fp4 (e2m1) matrix-core form of the distance, shared by the
// device code (mfma_f4.hip) and host-side checks.
//
// For 0/1 keys the Manhattan distance of Section 4.3 is d = |q| + |r| - 2 q.r.
// The fp4 kernel computes, per (query, record) pair, u = d - T - 1 as one dot
// product over K = 192 digits (a candidate iff u < 0):
//   key digits  : query -2.0 per set key, record 1.0 per set key  -> -2 q.r
//   |r| digits  : seven spare digits; query 6,6,6,6,6,6,1 against the record's
//                 digits v_0..v_5, w with |r| = 6 (v_0 + .. + v_5) + w
//   bias digits : seven more spare digits; record 6,6,6,6,6,6,1 against the
//                 query's digits of B = |q| - T - 1 in the same form (every
//                 digit negated when B < 0)
// An invalid record carries |r| digits worth 216 and an invalid query row the
// bias 166, so neither ever gives u < 0.
//
// e2m1 nibbles: bit 3 sign, bits 2..1 exponent (bias 1), bit 0 mantissa; the
// eight magnitudes are 0, 0.5, 1, 1.5, 2, 3, 4, 6.  Every product of two such
// digits here is an integer or a multiple of 0.5 whose sums stay integers
// below 2^9, so fp32 accumulation is exact.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fps {

constexpr uint32_t kF4MaxCount = 166;            // keys of a fingerprint
constexpr uint32_t kDigitsRecord = 0x22200200u;  // 2-bit index -> two digits of 1.0
constexpr uint32_t kDigitsQuery = 0xCCC00C00u;   // 2-bit index -> two digits of -2.0
constexpr uint32_t kQueryPopDigits = 0x02777777u;  // 6.0 x 6, 1.0
constexpr uint32_t kInvalidPopDigits = 0x00777777u;  // worth 6 * 36 = 216
constexpr uint32_t kRecordBiasDw0 = 0x77777700u;  // six 6.0 digits in bytes 1..3
constexpr uint32_t kRecordBiasDw1 = 0x00000200u;  // one 1.0 digit in byte 1
constexpr int32_t kInvalidRowBias = 166;

// p = 6 * (v_0 + ... + v_5) + w as fp4 digits in nibbles 0..5 (v_i in {0, .5,
// 1, 1.5, 2, 3, 4, 6}) and nibble 6 (w in {0, 1, 2}); 2 v_i is taken greedily
// from {12, 8, 6, 4, 3, 2, 1}, which covers every p = 3 m + w <= 167 within
// six digits (6 * 12 >= 55).
__host__ __device__ inline uint32_t six_one_digits(uint32_t p) {
  uint32_t m = p / 3, w = p % 3, pat = 0;
  const uint32_t two_v[7] = {12, 8, 6, 4, 3, 2, 1};
  const uint32_t code[7] = {0x7, 0x6, 0x5, 0x4, 0x3, 0x2, 0x1};
  for (int i = 0; i < 6; ++i) {
    for (int c = 0; c < 7; ++c) {
      if (two_v[c] <= m) {
        pat |= code[c] << (4 * i);
        m -= two_v[c];
        break;
      }
    }
  }
  pat |= (w == 0 ? 0u : (w == 1 ? 0x2u : 0x4u)) << 24;
  return pat;
}

// Record-side |r| digits; counts above 166 (an invalid record) get the sentinel.
__host__ __device__ inline uint32_t pop_digits(uint32_t p) {
  return p > kF4MaxCount ? kInvalidPopDigits : six_one_digits(p);
}

// The bias B (|B| <= 167) as the same seven digits, each negated for B < 0.
__host__ __device__ inline uint32_t bias_digits(int32_t b) {
  const uint32_t pat = six_one_digits((uint32_t)(b < 0 ? -b : b));
  // the sign bit of every nonzero digit (e2m1: bit 3 of the nibble)
  uint32_t neg = 0;
  for (int i = 0; i < 7; ++i) neg |= ((pat >> (4 * i)) & 0x7u) ? 0x8u << (4 * i) : 0u;
  return b < 0 ? pat | neg : pat;
}

}  // namespace fps
