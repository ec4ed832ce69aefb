// Batched scan on the gfx950 matrix cores with 4-bit float operands.
//
// The same contraction as the int8 kernel (d = |q| + |r| - 2 q.r, the matrix
// form of Section 4.3), on v_mfma_scale_f32_32x32x64_f8f6f4 with both operands
// in fp4 (e2m1) and unit block scales: twice the K of the int8 instruction per
// issue.  Every operand value is one of {0, 1, -2, 6, 0.5 .. 6} and every
// partial sum is an integer below 2^9, so the fp32 accumulation is exact.
//
// Per (query, record) pair the product is u = d - T_q - 1 (a candidate iff
// u < 0), accumulated from zero (the MFMA's C input is the inline constant 0,
// so no accumulator-input registers are needed):
//   key digits  : query -2 * q_s, record r_s      -> -2 q.r
//   |r| digits  : 7 spare digits; query 6,6,6,6,6,6,1, record the digits
//                 v_0..v_5, w of |r| = 6 (v_0 + .. + v_5) + w (a per-|r|
//                 table in LDS)
//   bias digits : 7 more spare digits; record 6,6,6,6,6,6,1, query the digits
//                 of B = |q| - T_q - 1 in the same form (negated digits for
//                 B < 0)
// Invalid rows carry B = 166 and invalid records |r| digits worth 216, so
// neither can pass.
//
// Bit -> digit expansion: a 32-bit chunk of keys becomes 32 digits (16 bytes)
// with four byte permutations (v_perm_b32) of a 4-entry table: output dword j,
// byte b holds the digits of key bits 8b + 2j (low nibble) and 8b + 2j + 1.
// Queries and records use the same order, which is all a dot product needs.
// The six chunks of a record (lo a, hi a, lo b, hi b, c, d) are the six 16-byte
// K fragments of its three MFMA K-steps; the |r| digits sit in dword 3 of the
// d fragment, which holds bits 6, 7, 14, 15, ... of d (always zero), and the
// bias digits in bytes 1..3 of dword 0 and byte 1 of dword 1 (bits 8..29 of d,
// also zero).
#include <type_traits>

#include "f4_digits.h"
#include "mfma_common.h"

namespace fps {

typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef int v4i_ __attribute__((ext_vector_type(4)));

constexpr int kF4Stride = 112;  // bytes per expanded record (96 + 16 pad)

__device__ __forceinline__ void spread_f4(uint32_t c, uint32_t table, uint32_t *o) {
#pragma unroll
  for (int j = 0; j < 4; ++j)
    o[j] = __builtin_amdgcn_perm(table, table, (c >> (2 * j)) & 0x03030303u);
}

// Thread tid expands record tid of a 256-record stage: six 16-byte fragments
// (keys of a lo, a hi, b lo, b hi, c, d), the |r| digits in dword 3 of the
// last one and the record side of the bias digits in its dwords 0 and 1.
__device__ __forceinline__ void expand_f4(const Rec1 &R, bool ok, uint8_t *buf,
                                          const uint32_t *poptab, uint32_t tid) {
  const uint64_t ra = ok ? R.a : 0, rb = ok ? R.b : 0;
  const uint32_t rc = ok ? R.c : 0, rd = ok ? R.d : 0;
  const uint32_t ch[6] = {(uint32_t)ra, (uint32_t)(ra >> 32), (uint32_t)rb,
                          (uint32_t)(rb >> 32), rc, rd};
  uint32_t dw[24];
#pragma unroll
  for (int f = 0; f < 6; ++f) spread_f4(ch[f], kDigitsRecord, dw + 4 * f);
  const uint32_t pr = (uint32_t)(__popcll(ra) + __popcll(rb) + __popc(rc) + __popc(rd));
  dw[23] = poptab[ok ? pr : 255u];
  dw[20] |= kRecordBiasDw0;
  dw[21] |= kRecordBiasDw1;
  v4i_ *dst = reinterpret_cast<v4i_ *>(buf + tid * kF4Stride);
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    v4i_ v = {(int)dw[4 * f], (int)dw[4 * f + 1], (int)dw[4 * f + 2], (int)dw[4 * f + 3]};
    dst[f] = v;
  }
}

// Half of expand_f4 for blocks of 512 threads: thread tid takes record
// tid & 255 and the fragments 3h .. 3h + 2 of it (h = tid >> 8); the |r| and
// bias digits live in the last fragment.
__device__ __forceinline__ void expand_half_f4(const Rec1 &R, bool ok, uint8_t *buf,
                                               const uint32_t *poptab, uint32_t tid) {
  const uint32_t rec = tid & 255u, h = tid >> 8;
  const uint64_t ra = ok ? R.a : 0, rb = ok ? R.b : 0;
  const uint32_t rc = ok ? R.c : 0, rd = ok ? R.d : 0;
  const uint32_t ch[3] = {h ? (uint32_t)(rb >> 32) : (uint32_t)ra,
                          h ? rc : (uint32_t)(ra >> 32), h ? rd : (uint32_t)rb};
  uint32_t dw[12];
#pragma unroll
  for (int f = 0; f < 3; ++f) spread_f4(ch[f], kDigitsRecord, dw + 4 * f);
  if (h) {
    const uint32_t pr = (uint32_t)(__popcll(ra) + __popcll(rb) + __popc(rc) + __popc(rd));
    dw[11] = poptab[ok ? pr : 255u];
    dw[8] |= kRecordBiasDw0;
    dw[9] |= kRecordBiasDw1;
  }
  v4i_ *dst = reinterpret_cast<v4i_ *>(buf + rec * kF4Stride + 48 * h);
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    v4i_ v = {(int)dw[4 * f], (int)dw[4 * f + 1], (int)dw[4 * f + 2], (int)dw[4 * f + 3]};
    dst[f] = v;
  }
}

// A operands of a wave: lane holds query row row0 + mq * 32 + (lane & 31)
// (K half lane >> 5), including the row's bias digits B = |q| - T - 1.
template <int MQ>
__device__ __forceinline__ void build_a_f4(const Workspace &ws, const QBlock &qb, uint32_t row0,
                                           uint32_t lane, v8i (&A)[MQ][3]) {
  const uint32_t h = lane >> 5;
#pragma unroll
  for (int mq = 0; mq < MQ; ++mq) {
    const uint32_t row = row0 + mq * 32 + (lane & 31);
    uint64_t qa = 0, qbw = 0;
    uint32_t qcw = 0, qdw = 0;
    int32_t bias = kInvalidRowBias;
    const bool valid = row < qb.count;
    if (valid) {
      const uint32_t q = ws.perm[qb.first + row];
      qa = ws.qinfo[q].qa;
      qbw = ws.qinfo[q].qb;
      qcw = ws.qinfo[q].qc;
      qdw = ws.qinfo[q].qd;
      bias = (int32_t)ws.qinfo[q].popc - (int32_t)ws.T[q] - 1;
    }
    const uint32_t ch[3] = {h ? (uint32_t)(qa >> 32) : (uint32_t)qa,
                            h ? (uint32_t)(qbw >> 32) : (uint32_t)qbw, h ? qdw : qcw};
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      uint32_t o[4];
      spread_f4(ch[s], kDigitsQuery, o);
      if (s == 2 && h == 1) {
        const uint32_t bd = bias_digits(bias);
        o[0] |= (bd & 0xFFFFFFu) << 8;  // against the record's six 6.0 digits
        o[1] |= ((bd >> 24) & 0xFu) << 8;  // against its 1.0 digit
        o[3] = valid ? kQueryPopDigits : 0u;
      }
      v8i v = {(int)o[0], (int)o[1], (int)o[2], (int)o[3], 0, 0, 0, 0};
      A[mq][s] = v;
    }
  }
}

template <int MQ>
__device__ __forceinline__ void load_b_f4(const uint8_t *buf, int c, uint32_t lane,
                                          v8i (&B)[3]) {
  const uint8_t *src = buf + (32 * c + (lane & 31)) * kF4Stride + 16 * (lane >> 5);
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const v4i_ x = *reinterpret_cast<const v4i_ *>(src + 32 * s);
    v8i v = {x[0], x[1], x[2], x[3], 0, 0, 0, 0};
    B[s] = v;
  }
}

template <int MQ>
__device__ __forceinline__ void multiply_f4(const v8i (&A)[MQ][3], const v8i (&B)[3],
                                            v16f (&acc)[MQ]) {
  const v16f zero = {};  // the inline constant 0 as the C input
#pragma unroll
  for (int mq = 0; mq < MQ; ++mq) {
    acc[mq] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[mq][0], B[0], zero, 4, 4, 0, 127,
                                                              0, 127);
    acc[mq] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[mq][1], B[1], acc[mq], 4, 4, 0,
                                                              127, 0, 127);
    acc[mq] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[mq][2], B[2], acc[mq], 4, 4, 0,
                                                              127, 0, 127);
  }
}

template <int MQ>
__device__ __forceinline__ int32_t or_bits(const v16f (&acc)[MQ]) {
  int32_t any = 0;
#pragma unroll
  for (int mq = 0; mq < MQ; ++mq)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const float x = acc[mq][e];
      any |= __float_as_int(x);
    }
  return any;
}

// Adds the hits of one 32x32 result tile (column block c of stage st) to the
// wave's hit list.  Lane layout of the result: column lane & 31, rows
// 8 (e >> 2) + 4 (lane >> 5) + (e & 3) of element e.  Each lane folds the
// signs of its elements into a mask; every round then takes the lowest set bit
// of each lane that has one (its element picked by a select tree over the
// bits of its position) and appends those lanes with one ballot.  Rows past
// the block's queries and records past the stage never pass (their products
// start positive), so no further check is needed.
template <int MQ>
__device__ __forceinline__ void decode_f4(const Workspace &ws, const Stage &st, int c,
                                          uint32_t lane, const v16f (&acc)[MQ], HitBuf &hb) {
  constexpr int kE = MQ * 16;
  static_assert(kE <= 64, "one bit per result element");
  const uint32_t g = (uint32_t)(st.g0 + 32 * c + (lane & 31));
  const uint32_t rowh = 4 * (lane >> 5);
  // the sign bits of the elements (every sum starts from +0, so an exact
  // zero is +0: a set sign bit is a negative product)
  typedef std::conditional_t<(kE <= 32), uint32_t, uint64_t> Mask;
  Mask m = 0;
#pragma unroll
  for (int mq = 0; mq < MQ; ++mq)
#pragma unroll
    for (int e = 0; e < 16; ++e)
      m |= (Mask)(__float_as_uint(acc[mq][e]) >> 31) << (16 * mq + e);
  for (;;) {
    const bool has = m != 0;
    const uint64_t bal = __ballot(has);
    if (bal == 0) break;
    if (hb.n + 64 > kHitCap) hits_flush<MQ * 32>(ws, lane, hb);
    if (has) {
      const uint32_t b = (uint32_t)__builtin_ctzll(m);
      m &= m - 1;
      float v[kE];
#pragma unroll
      for (int i = 0; i < kE; ++i) v[i] = acc[i >> 4][i & 15];
#pragma unroll
      for (int l = 0, w = kE; w > 1; ++l, w >>= 1)
#pragma unroll
        for (int i = 0; i < w / 2; ++i) v[i] = ((b >> l) & 1u) ? v[2 * i + 1] : v[2 * i];
      const uint32_t e = b & 15u;
      const uint32_t lr = 32 * (b >> 4) + 8 * (e >> 2) + rowh + (e & 3u);
      hb.list[hb.n + rank_below(bal)] = hit_entry(lr, (int32_t)v[0], g);
    }
    hb.n += (uint32_t)__popcll(bal);
  }
}

// Stages of 256 records (8 per work item); each thread holds the raw words of
// one record for RING stages ahead, in registers named statically (the stage
// loop is unrolled by RING), so the loads of stage s + RING + 1 are issued at
// stage s and first waited for at stage s + RING.
constexpr int kSubF4 = 256;
constexpr int kStagesF4 = kBatchTile / kSubF4;
static_assert(kStagesF4 % 4 == 0, "the stage loop is unrolled by up to 4");

// Multiplies one stage (LDS buffer buf, stage st) for this wave's queries and
// decodes the hits.  COLS = false: every column block; COLS = true: the blocks
// of this wave (wv, wv + 4).
template <int MQ, bool COLS>
__device__ __forceinline__ void stage_f4(const Workspace &ws, const QBlock &qb, const Stage &st,
                                         const uint8_t *buf, uint32_t row0, uint32_t lane,
                                         uint32_t wv, const v8i (&A)[MQ][3],
                                         HitBuf &hb) {
  constexpr int kCols = kSubF4 / 32;
  if (COLS) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = (int)wv + 4 * h;
      if (st.g0 + 32 * c >= st.g1) break;
      v8i B[3];
      v16f acc[MQ];
      load_b_f4<MQ>(buf, c, lane, B);
      multiply_f4<MQ>(A, B, acc);
      if (__builtin_expect(__ballot(or_bits<MQ>(acc) < 0) != 0, 0)) decode_f4<MQ>(ws, st, c, lane, acc, hb);
    }
    return;
  }
  // Every column block, software-pipelined: the products of block c + 1 are
  // issued before the sign test of block c, so the test and the next fragment
  // reads overlap matrix-core work.  A block with a negative result is decoded
  // from the accumulators at hand (the branch is wave-uniform and rare).
  v8i B0[3], B1[3];
  v16f acc0[MQ], acc1[MQ];
  load_b_f4<MQ>(buf, 0, lane, B0);
  multiply_f4<MQ>(A, B0, acc0);
  load_b_f4<MQ>(buf, 1, lane, B1);
#pragma unroll 1
  for (int c = 0; c < kCols; c += 2) {
    multiply_f4<MQ>(A, B1, acc1);  // block c + 1
    if (c + 2 < kCols) load_b_f4<MQ>(buf, c + 2, lane, B0);
    if (__builtin_expect(__ballot(or_bits<MQ>(acc0) < 0) != 0, 0)) decode_f4<MQ>(ws, st, c, lane, acc0, hb);
    if (c + 2 < kCols) {
      multiply_f4<MQ>(A, B0, acc0);  // block c + 2
      load_b_f4<MQ>(buf, c + 3, lane, B1);
    }
    if (__builtin_expect(__ballot(or_bits<MQ>(acc1) < 0) != 0, 0)) decode_f4<MQ>(ws, st, c + 1, lane, acc1, hb);
  }
}

// COLS = false: the 4 waves hold different queries (128 * MQ per block).
// COLS = true: the 4 waves share 32 * MQ queries and split the column blocks.
// NW = 8: blocks of 8 waves (two per SIMD) share each stage's expansion,
// each thread expanding half a record.
template <int MQ, int WPE, bool COLS, int RING, int NW>
__global__ __launch_bounds__(64 * NW, WPE) void k_scan_mfma_f4(Lib lib, Workspace ws, uint32_t nqb,
                                                           const uint64_t *item_off,
                                                           uint64_t tile_lo, uint64_t items) {
  constexpr int kRows = MQ * 32;  // query rows of a wave
  __shared__ __attribute__((aligned(16))) uint8_t lds[2][kSubF4 * kF4Stride];
  __shared__ uint32_t poptab[256];
  __shared__ RowInfo h_row[NW][kRows];
  __shared__ uint32_t h_cnt[NW][kRows], h_base[NW][kRows], h_sbase[NW][kRows];
  __shared__ uint64_t h_list[NW][kHitCap];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // work items blockIdx.x, blockIdx.x + gridDim.x, ... (round robin: every
  // block samples every query block, whatever its rows' k)
  const uint64_t nit =
      items > blockIdx.x ? (items - blockIdx.x + gridDim.x - 1) / gridDim.x : 0;
  if (nit == 0) return;
  auto item_of = [&](uint64_t j) { return (uint64_t)blockIdx.x + j * gridDim.x; };
  HitBuf hb{h_row[wv], h_cnt[wv], h_base[wv], h_sbase[wv], h_list[wv], 0};
  hits_init<kRows>(lane, h_cnt[wv]);
  if (tid < 256) poptab[tid] = pop_digits(tid);
  const uint32_t rtid = NW == 4 ? tid : (tid & 255u);  // the record this thread loads
  auto expand = [&](const Rec1 &R, bool ok, uint8_t *buf) {
    if constexpr (NW == 4) expand_f4(R, ok, buf, poptab, tid);
    else expand_half_f4(R, ok, buf, poptab, tid);
  };
  const uint64_t nst = nit * kStagesF4;
  const uint32_t row0 = COLS ? 0u : wv * (MQ * 32);
  v8i A[MQ][3];
  uint32_t a_qb = 0xFFFFFFFFu;
  QBlock qb{};
  bool wave_live = false;

  // loader: the next stage to load is tload, of work item litem
  uint64_t tload = 0;
  Item litem = describe(ws, item_off, nqb, tile_lo, item_of(0));
  // Past the last stage the loader yields empty stages (record 0 is read and
  // expanded as invalid), so that every stage issues the same loads: the
  // compiler can then count the loads in flight exactly and waits for each
  // stage's records only when they are expanded.
  auto next_stage = [&]() {
    Stage st{litem.b, 0, 0};
    if (tload < nst) {
      const uint32_t sub = (uint32_t)(tload % kStagesF4);
      if (sub == 0 && tload > 0)
        litem = describe(ws, item_off, nqb, tile_lo, item_of(tload / kStagesF4));
      st = stage_of<kSubF4>(litem, sub);
    }
    ++tload;
    return st;
  };
  Stage cs = next_stage();
  const Rec1 first = load_rec1(lib, cs, rtid);
  Stage S[RING];
  Rec1 R[RING];
#pragma unroll
  for (int j = 1; j <= RING; ++j) {
    S[j % RING] = next_stage();
    R[j % RING] = load_rec1(lib, S[j % RING], rtid);
  }
  __syncthreads();  // poptab
  expand(first, cs.g0 + rtid < cs.g1, lds[0]);
  __syncthreads();
  // nst is a multiple of kStagesF4, hence of RING
  for (uint64_t s0 = 0; s0 < nst; s0 += RING) {
#pragma unroll
    for (int j = 0; j < RING; ++j) {
      {
        if (cs.b != a_qb) {
          hits_flush<kRows>(ws, lane, hb);  // the rows change with the query block
          a_qb = cs.b;
          const cptr<QBlock> q = as_const(ws.qblocks) + cs.b;
          qb.first = q->first;
          qb.count = q->count;
          qb.rset = q->rset;
          qb.tiles = q->tiles;
          wave_live = qb.count > row0;
          build_a_f4<MQ>(ws, qb, row0, lane, A);
          hits_rows<kRows>(ws, qb, row0, lane, hb);
        }
        if (wave_live && cs.g1 > cs.g0)
          stage_f4<MQ, COLS>(ws, qb, cs, lds[j & 1], row0, lane, wv, A, hb);
        const int nx = (j + 1) % RING;  // a constant after unrolling
        const Stage cn = S[nx];
        // the expansion gates the block's barrier: it goes ahead of the
        // products of the other waves on the SIMD
        __builtin_amdgcn_s_setprio(2);
        expand(R[nx], cn.g0 + rtid < cn.g1, lds[(j + 1) & 1]);
        S[nx] = next_stage();
        R[nx] = load_rec1(lib, S[nx], rtid);
        lds_barrier();
        __builtin_amdgcn_s_setprio(0);
        cs = cn;
      }
    }
  }
  hits_flush<kRows>(ws, lane, hb);
}

// Tile-shape variants of the fp4 kernel.
//   0: 64 queries per wave, 256 per block, two waves per SIMD
//   1: 128 queries per wave, 512 per block
//   2: 64 queries shared by the 4 waves, which split the columns (small batches)
//   3: 32 queries per wave, 128 per block, two waves per SIMD
//   4: 64 queries per wave, 8 waves (512 queries) per block, one block per CU
int mfma_f4_variants() { return 5; }

uint32_t mfma_f4_qblock(int variant) {
  switch (variant) {
    case 1: return 4 * 4 * 32;
    case 2: return 2 * 32;
    case 3: return 4 * 1 * 32;
    case 4: return 8 * 2 * 32;
    default: return 4 * 2 * 32;
  }
}

void launch_scan_mfma_f4(const Lib &lib, const Workspace &ws, uint32_t nqb,
                         const uint64_t *item_off, uint64_t tile_lo, uint64_t items, int cus,
                         int variant, hipStream_t s, const LaunchEv &ev) {
  if (items == 0) return;
  const int per_cu = variant == 1 || variant == 4 ? 1 : 2;
  uint64_t blocks = (uint64_t)cus * per_cu;
  if (blocks > items) blocks = items;
  const dim3 g((uint32_t)blocks), b(256), b8(512);
#define FPS_F4_LAUNCH(MQ, WPE, COLS, RING, NW)                                          \
  launch_k((k_scan_mfma_f4<MQ, WPE, COLS, RING, NW>), g, NW == 8 ? b8 : b, s, ev, lib, ws, nqb, \
           item_off, tile_lo, items)
  switch (variant) {
    case 1: FPS_F4_LAUNCH(4, 1, false, 2, 4); break;
    case 2: FPS_F4_LAUNCH(2, 2, true, 4, 4); break;
    case 3: FPS_F4_LAUNCH(1, 2, false, 4, 4); break;
    case 4: FPS_F4_LAUNCH(2, 1, false, 4, 8); break;
    default: FPS_F4_LAUNCH(2, 2, false, 4, 4); break;
  }
#undef FPS_F4_LAUNCH
}

}  // namespace fps
