// Batched scan on the gfx950 matrix cores, int8 operands, exact int32 sums.
//
// For 0/1 keys the distance of Section 4.3 is d(q, r) = |q| + |r| - 2 q.r, so a
// batch of queries against a tile of records is a dense contraction Q x K x R
// (the matrix form of Section 4.3, where the library is the matrix A).  The
// kernel computes, for every (query, record) pair,
//     u = d - T_q - 1,
// whose sign says whether the record is a candidate (d <= T_q).  Everything is
// folded into one int8 product of K = 192 slots (6 MFMA K-steps of 32):
//   slots 0..165     : query byte -2 * q_s,  record byte r_s         -> -2 q.r
//   slots 166, 167   : query bytes c1, c2,   record bytes 1, 1       -> c1 + c2 = |q| - T_q - 1
//   slots 168, 169   : query bytes 1, 1,     record bytes p1, p2     -> p1 + p2 = |r|
// Slot s holds bit s of the record in the library layout (a: slots 0..63,
// b: 64..127, c: 128..159, d: 160..165); slots 166..191 carry no key.
// So the epilogue is an OR over the accumulators and one sign test; only tiles
// holding a candidate take the slow path that decodes (query, record).
//
// Invalid rows (past the end of a query block) get c1 = c2 = 127 and no |r|
// term, invalid records (past the end of a tile) get p1 = p2 = 127 and no keys:
// both make u >= 87, so they can never pass.
//
// Layout: 4 waves per block, each holding MQ query tiles of 32 rows (A operands
// stay in registers); records are expanded from bits to bytes into LDS in
// stages of 128 (208-byte padded rows, so the 16-byte fragment reads of a wave
// hit distinct banks) and shared by the 4 waves.  A block walks its work items
// as one stream of stages: the records of stage s+2 are loaded into registers
// while stage s is multiplied, and stage s+1 is expanded into the other LDS
// buffer, so each stage costs one barrier and HBM latency stays hidden.  The
// four 32-record columns of a stage are multiplied back to back (fragments of
// column c+1 are read while column c is in the matrix core) and all results
// are OR-ed into one flag; only a stage that holds a candidate is multiplied
// again, column by column, to decode its hits.  In a 32x32 result tile the 32
// lanes of a half-wave share one query row per accumulator element, so hits
// are appended with one atomic per half-wave.
#include "mfma_common.h"

namespace fps {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kRecStride = 208;  // bytes per expanded record (192 + 16 pad)

// Four key bits -> four bytes of value 0 or 1 (shifted copies do not overlap).
__device__ __forceinline__ uint32_t spread4(uint32_t nib) {
  return (nib * 0x00204081u) & 0x01010101u;
}

// 32-bit chunk i (0..5) of a record: lo a, hi a, lo b, hi b, c, d.
__device__ __forceinline__ uint32_t chunk32(uint64_t a, uint64_t b, uint32_t c, uint32_t d,
                                            int i) {
  switch (i) {
    case 0: return (uint32_t)a;
    case 1: return (uint32_t)(a >> 32);
    case 2: return (uint32_t)b;
    case 3: return (uint32_t)(b >> 32);
    case 4: return c;
    default: return d;
  }
}

// Thread (record tid >> 1, half tid & 1) writes the 96 slots 96h .. 96h + 95.
__device__ __forceinline__ void expand(const Regs &R, uint8_t *buf, uint32_t tid) {
  const uint32_t rr = tid >> 1, h = tid & 1;
  const uint64_t ra = R.ok ? R.a : 0, rb = R.ok ? R.b : 0;
  const uint32_t rc = R.ok ? R.c : 0, rd = R.ok ? R.d : 0;
  const uint32_t pr = (uint32_t)(__popcll(ra) + __popcll(rb) + __popc(rc) + __popc(rd));
  const uint32_t p1 = R.ok ? (pr > 127 ? 127 : pr) : 127;
  const uint32_t p2 = R.ok ? pr - p1 : 127;
  const uint32_t ch[3] = {h ? (uint32_t)(rb >> 32) : (uint32_t)ra, h ? rc : (uint32_t)(ra >> 32),
                          h ? rd : (uint32_t)rb};
  uint32_t dw[24];
#pragma unroll
  for (int e = 0; e < 24; ++e) dw[e] = spread4((ch[e / 8] >> (4 * (e % 8))) & 15u);
  if (h == 1) {
    dw[17] |= (1u << 16) | (1u << 24);  // slots 166, 167
    dw[18] |= p1 | (p2 << 8);           // slots 168, 169
  }
  v4i *dst = reinterpret_cast<v4i *>(buf + rr * kRecStride + 96 * h);
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    v4i v = {(int)dw[4 * e], (int)dw[4 * e + 1], (int)dw[4 * e + 2], (int)dw[4 * e + 3]};
    dst[e] = v;
  }
}

// A operands of wave wv: row i = lane & 31 of tile mq; K slice 16 * (lane >> 5).
template <int MQ>
__device__ __forceinline__ void build_a(const Workspace &ws, const QBlock &qb, uint32_t row0,
                                        uint32_t lane, v4i (&A)[MQ][6]) {
#pragma unroll
  for (int mq = 0; mq < MQ; ++mq) {
    const uint32_t row = row0 + mq * 32 + (lane & 31);
    uint64_t qa = 0, qbw = 0;
    uint32_t qcw = 0, qdw = 0;
    int32_t qc = 254;
    const bool valid = row < qb.count;
    if (valid) {
      const uint32_t q = ws.perm[qb.first + row];
      qa = ws.qinfo[q].qa;
      qbw = ws.qinfo[q].qb;
      qcw = ws.qinfo[q].qc;
      qdw = ws.qinfo[q].qd;
      qc = (int32_t)ws.qinfo[q].popc - (int32_t)ws.T[q] - 1;
    }
    const int32_t c1 = qc > 127 ? 127 : (qc < -127 ? -127 : qc);
    const int32_t c2 = qc - c1;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int k0 = 32 * s + 16 * (int)(lane >> 5) + 4 * m;
        uint32_t x = spread4((chunk32(qa, qbw, qcw, qdw, s) >> (k0 & 31)) & 15u) * 0xFEu;
        if (k0 == 164)
          x = (x & 0x0000FFFFu) | (((uint32_t)c1 & 0xFFu) << 16) | (((uint32_t)c2 & 0xFFu) << 24);
        if (k0 == 168 && valid) x = (x & 0xFFFF0000u) | 0x0101u;
        A[mq][s][m] = (int)x;
      }
    }
  }
}

template <int MQ>
__device__ __forceinline__ void load_b(const uint8_t *buf, int c, uint32_t lane, v4i (&B)[6]) {
  const uint8_t *src = buf + (32 * c + (lane & 31)) * kRecStride + 16 * (lane >> 5);
#pragma unroll
  for (int k = 0; k < 6; ++k) B[k] = *reinterpret_cast<const v4i *>(src + 32 * k);
}

template <int MQ>
__device__ __forceinline__ void multiply(const v4i (&A)[MQ][6], const v4i (&B)[6],
                                         v16i (&acc)[MQ]) {
#pragma unroll
  for (int mq = 0; mq < MQ; ++mq) {
    v16i zero = {};
    acc[mq] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[mq][0], B[0], zero, 0, 0, 0);
#pragma unroll
    for (int k = 1; k < 6; ++k)
      acc[mq] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[mq][k], B[k], acc[mq], 0, 0, 0);
  }
}

// Appends the hits of one 32x32 result tile (column block c of stage st).
template <int MQ>
__device__ __forceinline__ void decode(const Workspace &ws, const QBlock &qb, const Stage &st,
                                       int c, uint32_t row0, uint32_t lane,
                                       const v16i (&acc)[MQ]) {
  // lane holds column lane & 31 and rows 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3)
  const uint64_t g = st.g0 + 32 * c + (lane & 31);
  const uint32_t half = lane >> 5;
  const uint32_t below = (uint32_t)((1ull << (lane & 31)) - 1ull);
#pragma unroll
  for (int mq = 0; mq < MQ; ++mq) {
#pragma unroll 1
    for (int e = 0; e < 16; ++e) {
      const int32_t u = acc[mq][e];
      const uint32_t row = row0 + mq * 32 + 8 * (e >> 2) + 4 * half + (e & 3);
      const bool hit = u < 0 && row < qb.count && g < st.g1;
      const uint64_t bal = __ballot(hit);
      if (bal == 0) continue;
      const uint32_t mine = (uint32_t)(bal >> (32 * half));
      Resv rv{0, 0};
      uint32_t q = 0;
      if (mine) q = ws.perm[qb.first + row];
      const QueryInfo *qi = ws.qinfo + q;
      const uint32_t seg = blockIdx.x % (mine ? qi->nseg : 1u);
      if (mine && (lane & 31) == (uint32_t)(__ffs(mine) - 1))
        rv = cand_reserve(ws, qi, seg, (uint32_t)__popc(mine));
      // leader of each half: its lowest hit lane
      const uint32_t lead = mine ? 32 * half + (uint32_t)(__ffs(mine) - 1) : lane;
      rv.base = __shfl(rv.base, (int)lead);
      rv.sbase = __shfl(rv.sbase, (int)lead);
      if (hit) {
        const uint32_t d = (uint32_t)(u + (int32_t)ws.T[q] + 1);
        cand_put(ws, qi, seg, rv, (uint32_t)__popc(mine & below), ((uint64_t)d << 32) | g);
      }
    }
  }
}

// COLS = false: the 4 waves hold different queries (128 * MQ per block) and
// each multiplies every column of a stage.  COLS = true: the 4 waves hold the
// same 32 * MQ queries and wave w multiplies column w of every stage (for
// small batches, so that no wave idles).
template <int MQ, int WPE, bool COLS>
__global__ __launch_bounds__(256, WPE) void k_scan_mfma_i8(Lib lib, Workspace ws, uint32_t nqb,
                                                           const uint64_t *item_off,
                                                           uint64_t tile_lo, uint64_t items,
                                                           uint64_t per_block) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[2][kSub * kRecStride];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint64_t it0 = (uint64_t)blockIdx.x * per_block;
  const uint64_t it1 = min(it0 + per_block, items);
  if (it0 >= it1) return;
  const uint64_t nst = (it1 - it0) * kSubPerTile;
  const uint32_t row0 = COLS ? 0u : wv * (MQ * 32);
  v4i A[MQ][6];
  uint32_t a_qb = 0xFFFFFFFFu;
  QBlock qb{};
  bool wave_live = false;

  // item descriptions are computed half an item ahead of the stage prefetch
  Item pinfo = describe(ws, item_off, nqb, tile_lo, it0);
  Item ninfo = pinfo;
  Stage cur = stage_of(pinfo, 0);
  Stage nxt = stage_of(pinfo, 1);
  const Regs R0 = load_stage(lib, cur, tid);
  Regs R1 = load_stage(lib, nxt, tid);
  expand(R0, lds[0], tid);
  __syncthreads();
  for (uint64_t s = 0; s < nst; ++s) {
    // prefetch stage s + 2
    Stage nn = nxt;
    Regs R2 = R1;
    const uint64_t s2 = s + 2;
    if (s2 < nst) {
      const uint32_t sub = (uint32_t)(s2 % kSubPerTile);
      if (sub == 0) pinfo = ninfo;
      nn = stage_of(pinfo, sub);
      R2 = load_stage(lib, nn, tid);
      if (sub == kSubPerTile / 2 && it0 + s2 / kSubPerTile + 1 < it1)
        ninfo = describe(ws, item_off, nqb, tile_lo, it0 + s2 / kSubPerTile + 1);
    }
    // multiply stage s
    if (cur.b != a_qb) {
      a_qb = cur.b;
      qb = ws.qblocks[cur.b];
      wave_live = qb.count > row0;
      build_a<MQ>(ws, qb, row0, lane, A);
    }
    if (COLS && wave_live && cur.g0 + 32 * wv < cur.g1) {
      const uint8_t *buf = lds[s & 1];
      v4i B0[6];
      v16i acc[MQ];
      load_b<MQ>(buf, (int)wv, lane, B0);
      multiply<MQ>(A, B0, acc);
      int32_t any = 0;
#pragma unroll
      for (int mq = 0; mq < MQ; ++mq)
#pragma unroll
        for (int e = 0; e < 16; ++e) any |= acc[mq][e];
      if (__ballot(any < 0) != 0) decode<MQ>(ws, qb, cur, (int)wv, row0, lane, acc);
    }
    if (!COLS && wave_live && cur.g1 > cur.g0) {
      const uint8_t *buf = lds[s & 1];
      int32_t any = 0;
      v4i B0[6], B1[6];
      load_b<MQ>(buf, 0, lane, B0);
#pragma unroll
      for (int c = 0; c < kSub / 32; c += 2) {
        v16i acc[MQ];
        load_b<MQ>(buf, c + 1, lane, B1);
        multiply<MQ>(A, B0, acc);
#pragma unroll
        for (int mq = 0; mq < MQ; ++mq)
#pragma unroll
          for (int e = 0; e < 16; ++e) any |= acc[mq][e];
        if (c + 2 < kSub / 32) load_b<MQ>(buf, c + 2, lane, B0);
        multiply<MQ>(A, B1, acc);
#pragma unroll
        for (int mq = 0; mq < MQ; ++mq)
#pragma unroll
          for (int e = 0; e < 16; ++e) any |= acc[mq][e];
      }
      if (__ballot(any < 0) != 0) {
        // rare: multiply again column by column and append the hits
#pragma unroll 1
        for (int c = 0; c < kSub / 32; ++c) {
          v16i acc[MQ];
          load_b<MQ>(buf, c, lane, B0);
          multiply<MQ>(A, B0, acc);
          int32_t a2 = 0;
#pragma unroll
          for (int mq = 0; mq < MQ; ++mq)
#pragma unroll
            for (int e = 0; e < 16; ++e) a2 |= acc[mq][e];
          if (__ballot(a2 < 0) != 0) decode<MQ>(ws, qb, cur, c, row0, lane, acc);
        }
      }
    }
    // expand stage s + 1 into the other buffer
    if (s + 1 < nst) expand(R1, lds[(s + 1) & 1], tid);
    lds_barrier();
    cur = nxt;
    nxt = nn;
    R1 = R2;
  }
}

// Tile-shape variants.
//   0: 64 queries per wave, 256 per block, one wave per SIMD
//   1: 64 queries per wave, 256 per block, two waves per SIMD
//   2: 128 queries per wave, 512 per block
//   3: 32 queries per wave, 128 per block, two waves per SIMD
//   4: 64 queries shared by the 4 waves, which split the columns (small batches)
int mfma_variants() { return 5; }

uint32_t mfma_qblock(int variant) {
  switch (variant) {
    case 2: return 4 * 4 * 32;
    case 3: return 4 * 1 * 32;
    case 4: return 2 * 32;
    default: return 4 * 2 * 32;
  }
}

void launch_scan_mfma_i8(const Lib &lib, const Workspace &ws, uint32_t nqb,
                         const uint64_t *item_off, uint64_t tile_lo, uint64_t items, int cus,
                         int variant, hipStream_t s, const LaunchEv &ev) {
  if (items == 0) return;
  const int per_cu = variant == 1 || variant == 3 || variant == 4 ? 2 : 1;
  uint64_t blocks = (uint64_t)cus * per_cu;
  if (blocks > items) blocks = items;
  const uint64_t per = (items + blocks - 1) / blocks;
  blocks = (items + per - 1) / per;
  const dim3 g((uint32_t)blocks), b(256);
#define FPS_MFMA_LAUNCH(MQ, WPE, COLS)                                                     \
  launch_k((k_scan_mfma_i8<MQ, WPE, COLS>), g, b, s, ev, lib, ws, nqb, item_off, tile_lo, items, \
           per)
  switch (variant) {
    case 1: FPS_MFMA_LAUNCH(2, 2, false); break;
    case 2: FPS_MFMA_LAUNCH(4, 1, false); break;
    case 3: FPS_MFMA_LAUNCH(1, 2, false); break;
    case 4: FPS_MFMA_LAUNCH(2, 2, true); break;
    default: FPS_MFMA_LAUNCH(2, 1, false); break;
  }
#undef FPS_MFMA_LAUNCH
}

}  // namespace fps
