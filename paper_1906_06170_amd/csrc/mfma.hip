// Batched scan on the gfx950 matrix cores, int8 operands, exact int32 sums.
//
// For 0/1 keys the distance of Section 4.3 is d(q, r) = |q| + |r| - 2 q.r, so a
// batch of queries against a tile of records is a dense contraction Q x K x R
// (the matrix form of Section 4.3, where the library is the matrix A).  The
// kernel computes, for every (query, record) pair,
//     u = d - T_q - 1,
// whose sign says whether the record is a candidate (d <= T_q).  Everything is
// folded into one int8 product of K = 192 slots (6 MFMA K-steps of 32):
//   slot j in 1..166 : query byte -2 * q_j,  record byte r_j        -> -2 q.r
//   slots 0 and 167  : query bytes c1, c2,   record bytes 1, 1       -> c1 + c2 = |q| - T_q - 1
//   slots 168, 169   : query bytes 1, 1,     record bytes p1, p2     -> p1 + p2 = |r|
// (slots 0 and 167..191 carry no key: bit 0 and keys above 166 are always 0).
// So the epilogue is an OR over the accumulators and one sign test; only tiles
// holding a candidate take the slow path that decodes (query, record).
//
// Invalid rows (past the end of a query block) get c1 = c2 = 127 and no |r|
// term, invalid records (past the end of a tile) get p1 = p2 = 127 and no keys:
// both make u >= 87, so they can never pass.
//
// Layout: 4 waves per block, each holding 2 query tiles of 32 rows (A operands
// stay in registers, 48 VGPRs); records are expanded from bits to bytes into
// LDS in stages of 128 (208-byte padded rows, so the 16-byte fragment reads of
// a wave hit distinct banks) and shared by the 4 waves.
#include "fps_internal.h"

namespace fps {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kMQ = 2;            // 32-row query tiles per wave
constexpr int kSub = 128;         // records per LDS stage
constexpr int kRecStride = 208;   // bytes per expanded record (192 + 16 pad)

// Four key bits -> four bytes of value 0 or 1 (shifted copies do not overlap).
__device__ __forceinline__ uint32_t spread4(uint32_t nib) {
  return (nib * 0x00204081u) & 0x01010101u;
}

__device__ __forceinline__ uint32_t chunk32(uint64_t w0, uint64_t w1, uint64_t w2, int c) {
  const uint64_t w = c < 2 ? w0 : (c < 4 ? w1 : w2);
  return (c & 1) ? (uint32_t)(w >> 32) : (uint32_t)w;
}

__global__ __launch_bounds__(256) void k_scan_mfma_i8(Lib lib, Workspace ws, uint32_t nqb,
                                                      uint64_t items, uint64_t per_block) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[kSub * kRecStride];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint64_t it0 = (uint64_t)blockIdx.x * per_block;
  const uint64_t it1 = min(it0 + per_block, items);
  v4i A[kMQ][6];
  uint32_t cur_qb = 0xFFFFFFFFu;
  QBlock qb{};
  bool wave_live = false;
  for (uint64_t item = it0; item < it1; ++item) {
    uint32_t b = 0;
    while (b + 1 < nqb && item >= ws.qb_item_off[b + 1]) ++b;
    if (b != cur_qb) {
      cur_qb = b;
      qb = ws.qblocks[b];
      wave_live = qb.count > wv * (kMQ * 32);
      // A operands of this wave: row i = lane & 31 of tile mq; K slice 16 * (lane >> 5).
#pragma unroll
      for (int mq = 0; mq < kMQ; ++mq) {
        const uint32_t row = wv * (kMQ * 32) + mq * 32 + (lane & 31);
        uint64_t q0 = 0, q1 = 0, q2 = 0;
        int32_t qc = 254;
        const bool valid = row < qb.count;
        if (valid) {
          const uint32_t q = ws.perm[qb.first + row];
          q0 = ws.qinfo[q].w[0];
          q1 = ws.qinfo[q].w[1];
          q2 = ws.qinfo[q].w[2];
          qc = (int32_t)ws.qinfo[q].popc - (int32_t)ws.T[q] - 1;
        }
        const int32_t c1 = qc > 127 ? 127 : (qc < -127 ? -127 : qc);
        const int32_t c2 = qc - c1;
#pragma unroll
        for (int s = 0; s < 6; ++s) {
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const int k0 = 32 * s + 16 * (int)(lane >> 5) + 4 * m;
            uint32_t x = spread4((chunk32(q0, q1, q2, k0 >> 5) >> (k0 & 31)) & 15u) * 0xFEu;
            if (k0 == 0) x = (x & 0xFFFFFF00u) | ((uint32_t)c1 & 0xFFu);
            if (k0 == 164) x = (x & 0x00FFFFFFu) | (((uint32_t)c2 & 0xFFu) << 24);
            if (k0 == 168 && valid) x = (x & 0xFFFF0000u) | 0x0101u;
            A[mq][s][m] = (int)x;
          }
        }
      }
    }
    const RangeSet *rs = ws.rsets + qb.rset;
    const uint64_t tile = item - ws.qb_item_off[b];
    uint32_t r = 0;
    while (tile >= rs->tboff[r + 1]) ++r;
    const uint64_t g0 = rs->begin[r] + (tile - rs->tboff[r]) * kBatchTile;
    const uint64_t g1 = min(g0 + (uint64_t)kBatchTile, rs->end[r]);
    for (uint64_t sub = g0; sub < g1; sub += kSub) {
      // ---- expand 128 records into LDS: thread = (record tid>>1, half tid&1)
      {
        const uint32_t rr = tid >> 1, h = tid & 1;
        const uint64_t g = sub + rr;
        const bool ok = g < g1;
        const uint64_t w0 = ok ? lib.w0[g] : 0, w1 = ok ? lib.w1[g] : 0, w2 = ok ? lib.w2[g] : 0;
        const uint32_t pr = (uint32_t)(__popcll(w0) + __popcll(w1) + __popcll(w2));
        const uint32_t p1 = ok ? (pr > 127 ? 127 : pr) : 127;
        const uint32_t p2 = ok ? pr - p1 : 127;
        uint32_t dw[24];
#pragma unroll
        for (int e = 0; e < 24; ++e) {
          const uint32_t ch = chunk32(w0, w1, w2, 3 * (int)h + e / 8);
          dw[e] = spread4((ch >> (4 * (e % 8))) & 15u);
        }
        if (h == 0) {
          dw[0] |= 1u;                 // slot 0
        } else {
          dw[17] |= 1u << 24;          // slot 167
          dw[18] |= p1 | (p2 << 8);    // slots 168, 169
        }
        v4i *dst = reinterpret_cast<v4i *>(lds + rr * kRecStride + 96 * h);
#pragma unroll
        for (int e = 0; e < 6; ++e) {
          v4i v = {(int)dw[4 * e], (int)dw[4 * e + 1], (int)dw[4 * e + 2], (int)dw[4 * e + 3]};
          dst[e] = v;
        }
      }
      __syncthreads();
      if (wave_live) {
#pragma unroll 1
        for (int c = 0; c < kSub / 32; ++c) {
          v4i B[6];
          const uint8_t *src = lds + (32 * c + (lane & 31)) * kRecStride + 16 * (lane >> 5);
#pragma unroll
          for (int s = 0; s < 6; ++s) B[s] = *reinterpret_cast<const v4i *>(src + 32 * s);
          v16i acc[kMQ];
#pragma unroll
          for (int mq = 0; mq < kMQ; ++mq) {
            v16i zero = {};
            acc[mq] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[mq][0], B[0], zero, 0, 0, 0);
#pragma unroll
            for (int s = 1; s < 6; ++s)
              acc[mq] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[mq][s], B[s], acc[mq], 0, 0, 0);
          }
          int32_t any = 0;
#pragma unroll
          for (int mq = 0; mq < kMQ; ++mq)
#pragma unroll
            for (int e = 0; e < 16; ++e) any |= acc[mq][e];
          if (__ballot(any < 0) == 0) continue;
          // slow path: decode (query row, record) of every negative entry.
          // Output layout of a 32x32 tile: lane holds column lane & 31 and rows
          // 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3), e = 0..15.
          const uint64_t g = sub + 32 * c + (lane & 31);
#pragma unroll
          for (int mq = 0; mq < kMQ; ++mq) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
              const int32_t u = acc[mq][e];
              const uint32_t row =
                  wv * (kMQ * 32) + mq * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
              if (u < 0 && row < qb.count && g < g1) {
                const uint32_t q = ws.perm[qb.first + row];
                const uint32_t d = (uint32_t)(u + (int32_t)ws.T[q] + 1);
                const QueryInfo *qi = ws.qinfo + q;
                const uint32_t pos = atomicAdd(ws.count + q, 1u);
                if (pos < qi->cap) ws.cand[qi->cand_off + pos] = ((uint64_t)d << 32) | g;
              }
            }
          }
        }
      }
      __syncthreads();
    }
  }
}

void launch_scan_mfma_i8(const Lib &lib, const Workspace &ws, uint32_t nqb, uint64_t items,
                         int cus, hipStream_t s) {
  if (items == 0) return;
  uint64_t blocks = (uint64_t)cus * 2;
  if (blocks > items) blocks = items;
  const uint64_t per = (items + blocks - 1) / blocks;
  blocks = (items + per - 1) / per;
  hipLaunchKernelGGL(k_scan_mfma_i8, dim3((uint32_t)blocks), dim3(256), 0, s, lib, ws, nqb,
                     items, per);
}

}  // namespace fps
