// Wider fingerprints (Section 5, concluding remark 3: more features): the
// same exact top-k search for records of W 64-bit words (W in {4, 8, 16, 32}:
// 256 to 2,048 keys), every bit a key.  The distance is the Section 4.3
// sum over all 64 W keys = the popcount of the XOR, in [0, 64 W].
//
// Library layout: W word-major arrays, word k of record i at w[k * np + i], np
// = n rounded up to 4096 (the tail is zero and never reported).  A single
// query streams 8 W bytes per record from HBM, every load instruction of a
// wave reading one contiguous 1 KiB segment.
//
// The search follows the MACCS engine's plan with histograms of 64 W + 1 bins:
//   bound  : the keff-th smallest distance of the first 65,536 records of each
//            query's strides (a histogram in LDS per block, merged in memory;
//            the last block of a query takes the k-th smallest);
//   phases : the strides are scanned in phases of 16x growing length; every
//            record with d <= T is appended to the query's candidate buffer,
//            and between phases T becomes the keff-th smallest candidate (the
//            buffer holds every record of the prefix with d <= T);
//   select : histogram of the candidates -> D_k; the candidates with
//            d <= D_k are sorted by (d, index) in LDS and the first keff kept;
//   fallback (buffer overflow, or more than 4,096 candidates with d <= D_k):
//            exact ordered two-pass over the strides, as for MACCS.
// Scan kernels:
//   single  : one query, one wave per 128-record tile (2 records per lane);
//   popcount: up to 64 queries in LDS, one record per thread in registers,
//             XOR + popcount per pair (4 W VALU operations);
//   matrix cores, int8 or fp4 operands: d = |q| + |r| - 2 q.r with K = 64 W;
//             blocks of 128 queries x 128 records, K in chunks of 256 keys:
//             the records' bits are expanded into LDS (bytes of 0/1, or fp4
//             digits 0 / 1.0), the queries' were expanded once per call into
//             memory (read from L2), each wave accumulating 32 queries x 128
//             records in four 32 x 32 tiles; products are exact (int32, or
//             fp32 sums of integers below 2^12).
#include <string.h>

#include <algorithm>
#include <vector>

#include "cand.h"
#include "fps_internal.h"
#include "runtime.h"

namespace fps {

constexpr uint32_t kWMaxBins = 64 * FPS_WIDE_MAX_WORDS + 1;
constexpr uint32_t kWTile = 128;          // records per wave tile of the single scan
constexpr uint64_t kWSample = 1u << 16;   // records of the bound sample
constexpr uint64_t kWGrowth = 16;         // phase length ratio
constexpr uint32_t kWSortCap = 4096;      // candidates with d <= D_k sorted in LDS
constexpr uint32_t kWFbBlocks = 256;      // fallback grid (4 waves each)
constexpr uint32_t kWFbWaves = kWFbBlocks * 4;
constexpr uint32_t kWPopQB = 64;          // queries per block of the popcount kernel
constexpr uint32_t kWMmaQB = 128;         // queries per block of the matrix-core kernel
constexpr uint32_t kWMmaRT = 128;         // records per matrix-core work item
constexpr uint32_t kWChunk = 4;           // words (256 keys) per matrix-core K chunk

struct WRange {
  uint32_t nranges, pad;
  uint64_t neff;
  uint64_t begin[FPS_MAX_STRIDES], end[FPS_MAX_STRIDES], voff[FPS_MAX_STRIDES + 1];
};

static_assert(sizeof(WRange) % 8 == 0, "copied into LDS as 64-bit words");

struct WQuery {
  uint64_t cand_off, out_off, sample;
  uint32_t keff, cap, rset, popc;
};

struct WBlock {
  uint32_t first, count, rset, pad;
};

struct WWs {
  const WRange *rs;
  const WQuery *qi;
  const uint32_t *perm;
  const WBlock *qb;
  const uint64_t *item_off;  // per phase: nqb + 1 prefix of items
  const uint64_t *qw;        // q x W query words
  uint8_t *qx;               // q x 64 W bytes: queries expanded for the int8 matrix cores
  uint32_t *T, *ctr, *flags, *count, *hist, *bdone;
  uint64_t *cand;
  fps_hit *out;
  uint32_t *fbh, *fbo, *fbt;
  uint32_t bins, nqb;
};

struct WLib {
  const uint64_t *w;
  uint64_t np, n;
};

__device__ __forceinline__ uint64_t wv2g(const WRange *rs, uint64_t v) {
  uint32_t r = 0;
  const uint32_t nr = rs->nranges;
  while (r + 1 < nr && v >= rs->voff[r + 1]) ++r;
  return rs->begin[r] + (v - rs->voff[r]);
}

template <int W>
__device__ __forceinline__ uint32_t wdist(const WLib &L, uint64_t g, const uint64_t *q) {
  uint32_t d = 0;
#pragma unroll
  for (int k = 0; k < W; ++k) d += (uint32_t)__popcll(L.w[(uint64_t)k * L.np + g] ^ q[k]);
  return d;
}

// Appends key at slot atomicAdd(ctr) of the query's buffer for every lane with
// hit (one reservation per wave).
__device__ __forceinline__ void wappend(bool hit, uint64_t key, const WWs &ws, uint32_t q) {
  const uint64_t bal = __ballot(hit);
  if (bal == 0) return;
  const uint32_t leader = (uint32_t)__ffsll((unsigned long long)bal) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(ws.ctr + q, (uint32_t)__popcll(bal));
  base = __shfl(base, (int)leader);
  const uint32_t pos = base + rank_below(bal);
  if (hit && pos < ws.qi[q].cap) ws.cand[ws.qi[q].cand_off + pos] = key;
}

// Smallest t <= tmax whose cumulative count reaches keff (0xFFFFFFFF if none)
// and that count; h has `bins` entries; every thread of the block calls it
// (256 threads, `part` 256 words of LDS).
__device__ __forceinline__ uint32_t block_kth(const uint32_t *h, uint32_t bins, uint32_t tmax,
                                              uint32_t keff, uint32_t *part, uint32_t *cum) {
  __shared__ uint32_t s_t, s_c;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const uint32_t per = (bins + nt - 1) / nt, t0 = tid * per;
  uint32_t own = 0;
  for (uint32_t t = t0; t < t0 + per && t < bins; ++t) own += t <= tmax ? h[t] : 0u;
  part[tid] = own;
  if (tid == 0) {
    s_t = 0xFFFFFFFFu;
    s_c = 0;
  }
  __syncthreads();
  for (uint32_t off = 1; off < nt; off <<= 1) {
    const uint32_t y = tid >= off ? part[tid - off] : 0u;
    __syncthreads();
    part[tid] += y;
    __syncthreads();
  }
  const uint32_t incl = part[tid], excl = incl - own;
  if (excl < keff && incl >= keff) {  // exactly one thread crosses keff
    uint32_t c = excl;
    for (uint32_t t = t0; t < t0 + per && t < bins; ++t) {
      c += t <= tmax ? h[t] : 0u;
      if (c >= keff) {
        s_t = t;
        s_c = c;
        break;
      }
    }
  }
  if (tid == nt - 1 && incl < keff) s_c = incl;
  __syncthreads();
  *cum = s_c;
  const uint32_t t = s_t;
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------------------
__global__ void k_wprep(WWs ws, uint32_t q) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < q; i += stride) {
    ws.ctr[i] = 0;
    ws.flags[i] = 0;
    ws.count[i] = 0;
    ws.bdone[i] = 0;
    ws.T[i] = 0xFFFFFFFFu;
  }
  for (uint64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < (uint64_t)q * ws.bins; i += stride)
    ws.hist[i] = 0;
}

// Bound: grid (chunk, group of kWBoundQ consecutive queries).  A thread takes
// a record of the chunk, loads its words once for the queries of the group
// that share a stride set (again only when a query's set maps the virtual
// index elsewhere) and adds its distance to each query's LDS histogram: the
// sample is read once per group instead of once per query.
constexpr uint32_t kWBoundQ = 8;

template <int W>
__global__ __launch_bounds__(256) void k_wbound(WLib L, WWs ws, uint32_t chunk, uint32_t q) {
  constexpr uint32_t kB = 64 * W + 1;  // bins of this width
  __shared__ uint32_t h[kWBoundQ * kB];
  __shared__ uint64_t qws[kWBoundQ][W];
  __shared__ uint32_t part[256];
  __shared__ uint32_t s_last;
  const uint32_t q0 = blockIdx.y * kWBoundQ, tid = threadIdx.x, bins = ws.bins;
  const uint32_t nq = min(kWBoundQ, q - q0);
  for (uint32_t i = tid; i < nq * bins; i += blockDim.x) h[i] = 0;
  for (uint32_t i = tid; i < nq * W; i += blockDim.x)
    qws[i / W][i % W] = ws.qw[(uint64_t)(q0 + i / W) * W + i % W];
  __syncthreads();
  const uint64_t v0 = (uint64_t)blockIdx.x * chunk;
  for (uint64_t v = v0 + tid; v < v0 + chunk; v += blockDim.x) {
    uint64_t gw = ~0ull;
    uint64_t rw[W];
    for (uint32_t j = 0; j < nq; ++j) {
      const WQuery &qi = ws.qi[q0 + j];
      if (qi.keff == 0 || v >= qi.sample) continue;
      const uint64_t g = wv2g(ws.rs + qi.rset, v);
      if (g != gw) {
#pragma unroll
        for (int k = 0; k < W; ++k) rw[k] = L.w[(uint64_t)k * L.np + g];
        gw = g;
      }
      uint32_t d = 0;
#pragma unroll
      for (int k = 0; k < W; ++k) d += (uint32_t)__popcll(rw[k] ^ qws[j][k]);
      atomicAdd(&h[j * bins + d], 1u);
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < nq * bins; i += blockDim.x)
    if (h[i]) atomicAdd(ws.hist + (uint64_t)(q0 + i / bins) * bins + i % bins, h[i]);
  // as in k_bound: the adds are device-scope atomics, waited for per block; a
  // partial histogram only loosens the bound
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0) s_last = atomicAdd(ws.bdone + blockIdx.y, 1u) == gridDim.x - 1 ? 1u : 0u;
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  for (uint32_t j = 0; j < nq; ++j) {
    const WQuery &qi = ws.qi[q0 + j];
    if (qi.keff == 0) continue;  // uniform over the block
    for (uint32_t i = tid; i < bins; i += blockDim.x)
      h[i] = __hip_atomic_load(ws.hist + (uint64_t)(q0 + j) * bins + i, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    uint32_t cum;
    uint32_t t = block_kth(h, bins, bins - 1, qi.keff, part, &cum);
    if (t == 0xFFFFFFFFu) t = bins - 1;  // the sample holds fewer than keff records
    if (tid == 0) ws.T[q0 + j] = t;
    __syncthreads();
  }
}

// Single-query scan of the virtual records [vb, ve) of query qidx.
typedef unsigned long long wu64x2 __attribute__((ext_vector_type(2)));

template <int W>
__global__ __launch_bounds__(256) void k_wscan1(WLib L, WWs ws, uint32_t qidx, uint64_t vb,
                                                uint64_t ve) {
  const WQuery &qi = ws.qi[qidx];
  const WRange *rs = ws.rs + qi.rset;
  const int32_t T = (int32_t)ws.T[qidx];
  uint64_t qw[W];
#pragma unroll
  for (int k = 0; k < W; ++k) qw[k] = ws.qw[(uint64_t)qidx * W + k];
  const uint32_t lane = lane_id();
  const uint64_t wave = (uint64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t nwaves = (uint64_t)gridDim.x * 4;
  for (uint32_t r = 0; r < rs->nranges; ++r) {
    const uint64_t a = max(vb, rs->voff[r]), b = min(ve, rs->voff[r + 1]);
    if (a >= b) continue;
    const uint64_t glo = rs->begin[r] + (a - rs->voff[r]), ghi = rs->begin[r] + (b - rs->voff[r]);
    const uint64_t base0 = glo & ~(uint64_t)(kWTile - 1);
    const uint64_t ntiles = (ghi - base0 + kWTile - 1) / kWTile;
    for (uint64_t t = wave; t < ntiles; t += nwaves) {
      const uint64_t i0 = base0 + t * kWTile + 2 * lane;
      uint32_t d0 = 0, d1 = 0;
#pragma unroll
      for (int k = 0; k < W; ++k) {
        const wu64x2 x = __builtin_nontemporal_load(
            reinterpret_cast<const wu64x2 *>(L.w + (uint64_t)k * L.np + i0));
        d0 += (uint32_t)__popcll(x.x ^ qw[k]);
        d1 += (uint32_t)__popcll(x.y ^ qw[k]);
      }
      const bool h0 = (int32_t)d0 <= T && i0 >= glo && i0 < ghi;
      const bool h1 = (int32_t)d1 <= T && i0 + 1 >= glo && i0 + 1 < ghi;
      const uint64_t b0 = __ballot(h0), b1 = __ballot(h1);
      if ((b0 | b1) == 0) continue;
      uint32_t base = 0;
      if (lane == 0) base = atomicAdd(ws.ctr + qidx, (uint32_t)(__popcll(b0) + __popcll(b1)));
      base = __shfl(base, 0);
      uint64_t *cand = ws.cand + qi.cand_off;
      const uint32_t cap = qi.cap;
      if (h0) {
        const uint32_t p = base + rank_below(b0);
        if (p < cap) cand[p] = ((uint64_t)d0 << 32) | i0;
      }
      if (h1) {
        const uint32_t p = base + (uint32_t)__popcll(b0) + rank_below(b1);
        if (p < cap) cand[p] = ((uint64_t)d1 << 32) | (i0 + 1);
      }
    }
  }
}

// Batched popcount scan: item = (query block, 256 RPT virtual records).
template <int W, int RPT>
__global__ __launch_bounds__(256) void k_wscan_pop(WLib L, WWs ws, const uint64_t *item_off,
                                                   uint64_t vb, uint64_t ve, uint64_t items) {
  __shared__ uint64_t qs[kWPopQB][W];
  __shared__ int32_t qt[kWPopQB];
  __shared__ uint32_t qid[kWPopQB];
  const uint32_t tid = threadIdx.x;
  uint32_t cur = 0xFFFFFFFFu;
  WBlock qb{};
  for (uint64_t item = blockIdx.x; item < items; item += gridDim.x) {
    uint32_t b = 0;
    while (b + 1 < ws.nqb && item >= item_off[b + 1]) ++b;
    if (b != cur) {
      __syncthreads();
      cur = b;
      qb = ws.qb[b];
      for (uint32_t j = tid; j < qb.count * W; j += blockDim.x) {
        const uint32_t q = ws.perm[qb.first + j / W];
        qs[j / W][j % W] = ws.qw[(uint64_t)q * W + j % W];
      }
      for (uint32_t j = tid; j < qb.count; j += blockDim.x) {
        const uint32_t q = ws.perm[qb.first + j];
        qid[j] = q;
        qt[j] = (int32_t)ws.T[q];
      }
      __syncthreads();
    }
    const WRange *rs = ws.rs + qb.rset;
    const uint64_t vend = min(ve, rs->neff);
    const uint64_t v0 = vb + (item - item_off[b]) * (256ull * RPT);
    uint64_t x[RPT][W];
    uint64_t g[RPT];
    bool ok[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const uint64_t v = v0 + 256 * u + tid;
      ok[u] = v < vend;
      g[u] = ok[u] ? wv2g(rs, v) : 0;
#pragma unroll
      for (int k = 0; k < W; ++k) x[u][k] = ok[u] ? L.w[(uint64_t)k * L.np + g[u]] : 0ull;
    }
    for (uint32_t j = 0; j < qb.count; ++j) {
      const int32_t T = qt[j];
      uint32_t d[RPT];
      bool any = false;
#pragma unroll
      for (int u = 0; u < RPT; ++u) {
        d[u] = 0;
#pragma unroll
        for (int k = 0; k < W; ++k) d[u] += (uint32_t)__popcll(x[u][k] ^ qs[j][k]);
        any |= ok[u] && (int32_t)d[u] <= T;
      }
      if (__ballot(any) == 0) continue;
#pragma unroll
      for (int u = 0; u < RPT; ++u)
        wappend(ok[u] && (int32_t)d[u] <= T, ((uint64_t)d[u] << 32) | g[u], ws, qid[j]);
    }
  }
}

// ---------------------------------------------------------------------------
// Matrix cores.  FMT 0: int8 bytes 0/1, v_mfma_i32_32x32x32_i8 (K = 32 per
// step, 8 steps per 256-key chunk).  FMT 1: fp4 digits 0 / 1.0 (e2m1 0x2),
// v_mfma_scale_f32_32x32x64_f8f6f4 with unit scales (K = 64 per step, 4 steps).
// Expanded row layout per 256-key chunk: int8, byte i = key i of the chunk;
// fp4, 16 bytes per 32-bit part m of the chunk (v_perm of a 4-entry table:
// dword j, byte b holds keys 8b + 2j and 8b + 2j + 1), the same for queries
// and records, which is all a dot product needs.
// ---------------------------------------------------------------------------
typedef int wv4i __attribute__((ext_vector_type(4)));
typedef int wv8i __attribute__((ext_vector_type(8)));
typedef int wv16i __attribute__((ext_vector_type(16)));
typedef float wv16f __attribute__((ext_vector_type(16)));

template <int FMT>
struct MmaFmt;

template <>
struct MmaFmt<0> {
  static constexpr uint32_t kChunkBytes = 256;  // bytes per row per chunk
  static constexpr uint32_t kSteps = 8;
  static constexpr uint32_t kRowStride = 272;   // LDS bytes per record row (+16 pad)
  typedef wv16i Acc;
  // 32 keys -> 32 bytes of 0/1 (8 dwords)
  __device__ static void expand32(uint32_t c, uint32_t *o) {
#pragma unroll
    for (int e = 0; e < 8; ++e) o[e] = (((c >> (4 * e)) & 15u) * 0x00204081u) & 0x01010101u;
  }
  __device__ static Acc mma(const wv4i &a, const wv4i &b, const Acc &c) {
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
  }
  __device__ static int32_t val(const Acc &acc, int e) { return acc[e]; }
};

template <>
struct MmaFmt<1> {
  static constexpr uint32_t kChunkBytes = 128;
  static constexpr uint32_t kSteps = 4;
  static constexpr uint32_t kRowStride = 144;
  typedef wv16f Acc;
  // 32 keys -> 32 fp4 digits (16 bytes, 4 dwords)
  __device__ static void expand32(uint32_t c, uint32_t *o) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      o[j] = __builtin_amdgcn_perm(0x22200200u, 0x22200200u, (c >> (2 * j)) & 0x03030303u);
  }
  __device__ static Acc mma(const wv4i &a, const wv4i &b, const Acc &c) {
    const wv8i a8 = {a[0], a[1], a[2], a[3], 0, 0, 0, 0};
    const wv8i b8 = {b[0], b[1], b[2], b[3], 0, 0, 0, 0};
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, b8, c, 4, 4, 0, 127, 0, 127);
  }
  __device__ static int32_t val(const Acc &acc, int e) { return (int32_t)acc[e]; }
};

// Expands every query's words into qx (row q: 64 W / 8 bytes per chunk ...).
template <int W, int FMT>
__global__ __launch_bounds__(256) void k_wexpand(WWs ws, uint32_t q) {
  typedef MmaFmt<FMT> F;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;  // one 32-key part
  const uint64_t parts = 2ull * W;
  if (i >= (uint64_t)q * parts) return;
  const uint64_t qq = i / parts, m = i % parts;
  const uint64_t w = ws.qw[qq * W + m / 2];
  const uint32_t c = (uint32_t)(w >> (32 * (m & 1)));
  uint32_t o[8];
  F::expand32(c, o);
  const uint32_t nb = F::kChunkBytes / 8;  // bytes per 32-key part
  uint32_t *dst = reinterpret_cast<uint32_t *>(ws.qx + qq * (uint64_t)(F::kChunkBytes * W / kWChunk) +
                                               m * nb);
#pragma unroll
  for (uint32_t e = 0; e < nb / 4; ++e) dst[e] = o[e];
}

template <int W, int FMT>
__global__ __launch_bounds__(256, 2) void k_wscan_mma(WLib L, WWs ws, const uint64_t *item_off,
                                                   uint64_t vb, uint64_t ve, uint64_t items) {
  typedef MmaFmt<FMT> F;
  constexpr uint32_t RS = F::kRowStride;
  constexpr uint32_t QROW = F::kChunkBytes * (W / kWChunk);  // bytes per expanded query
  constexpr uint32_t NCH = W / kWChunk;
  // A wave multiplies QT query tiles by CT record tiles of 32 x 32: 1 x 4.
  // (2 x 2 halves the LDS reads per product but doubles every wave's query
  // fragments; measured 1.5x slower with expanded query rows from L2, and
  // still 16 % slower with raw query words expanded in registers.)
  constexpr int QT = 1, CT = 4 / QT;
  __shared__ __attribute__((aligned(16))) uint8_t bt[2][kWMmaRT * RS];
  __shared__ int32_t cq[kWMmaQB];   // |q| - T - 1 (large for rows past the block)
  __shared__ int32_t tq[kWMmaQB];   // T
  __shared__ uint32_t qid[kWMmaQB];
  __shared__ uint32_t pr[kWMmaRT];  // |r|
  __shared__ WRange srs;            // the range set of the current query block
  const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // The query block of an item, its first item and the range set are looked
  // up when the block's items (in increasing order) enter a new query block:
  // looked up per item, their chain of dependent global loads delayed every
  // item's record loads by several microseconds.
  uint32_t cur = 0xFFFFFFFFu, b = 0;
  uint64_t bfirst = 0, bnext = ws.nqb > 1 ? item_off[1] : ~0ull;
  WBlock qb{};
  for (uint64_t item = blockIdx.x; item < items; item += gridDim.x) {
    while (item >= bnext) {
      ++b;
      bfirst = bnext;
      bnext = b + 1 < ws.nqb ? item_off[b + 1] : ~0ull;
    }
    __syncthreads();
    if (b != cur) {
      cur = b;
      qb = ws.qb[b];
      {
        const uint64_t *src = reinterpret_cast<const uint64_t *>(ws.rs + qb.rset);
        uint64_t *dst = reinterpret_cast<uint64_t *>(&srs);
        for (uint32_t j = tid; j < sizeof(WRange) / 8; j += blockDim.x) dst[j] = src[j];
      }
      for (uint32_t j = tid; j < kWMmaQB; j += blockDim.x) {
        if (j < qb.count) {
          const uint32_t q = ws.perm[qb.first + j];
          qid[j] = q;
          tq[j] = (int32_t)ws.T[q];
          cq[j] = (int32_t)ws.qi[q].popc - (int32_t)ws.T[q] - 1;
        } else {
          qid[j] = 0;
          tq[j] = 0;
          cq[j] = 1 << 20;
        }
      }
    }
    if (tid < kWMmaRT) pr[tid] = 0;
    __syncthreads();
    const WRange *rs = &srs;
    const uint64_t vend = min(ve, rs->neff);
    const uint64_t v0 = vb + (item - bfirst) * kWMmaRT;
    // thread: record rr, half h of every chunk (words 2h, 2h + 1 of it)
    const uint32_t rr = tid & (kWMmaRT - 1), h = tid >> 7;
    const uint64_t vr = v0 + rr;
    const bool rok = vr < vend;
    const uint64_t g = rok ? wv2g(rs, vr) : 0;
    // the wave's tiles: query tiles QT qg + mq, record tiles CT rg + ct
    const uint32_t qg = wv / (4 / CT), rg = wv % (4 / CT);
    const bool live = 32 * QT * qg < qb.count;
    typename F::Acc acc[QT][CT];
#pragma unroll
    for (int mq = 0; mq < QT; ++mq)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[mq][ct] = typename F::Acc{};
    uint32_t mypop = 0;
    // this thread's words of every chunk, requested at once: one memory
    // latency per item (requested a chunk ahead, the loads left two blocks
    // per CU with 16 bytes in flight per thread, about 1 TB/s at the chip's
    // latency)
    // (loaded unconditionally, from record 0 past the range, and then
    // cleared: sixteen branches around the loads also left the compiler's
    // wait counts at their worst case)
    uint64_t wr[NCH][2];
#pragma unroll
    for (uint32_t ch = 0; ch < NCH; ++ch) {
      const uint64_t k0 = (uint64_t)kWChunk * ch + 2 * h;
      const uint64_t x0 = L.w[k0 * L.np + g], x1 = L.w[(k0 + 1) * L.np + g];
      wr[ch][0] = rok ? x0 : 0ull;
      wr[ch][1] = rok ? x1 : 0ull;
    }
    // The wave's query fragments of a chunk are read one chunk ahead (they
    // come from L2: read when needed they stalled every chunk's products).
    // int8 reads the expanded rows of qx; fp4 reads the raw query words and
    // each lane expands its half of a word per K step (a quarter of the bytes
    // read from L2: measured 2 % faster).
    const uint8_t *abase[QT];
    const uint64_t *qraw[QT];
#pragma unroll
    for (int mq = 0; mq < QT; ++mq) {
      const uint32_t qq = qid[32 * (QT * qg + mq) + (lane & 31)];
      abase[mq] = ws.qx + (uint64_t)qq * QROW + 16 * (lane >> 5);
      qraw[mq] = ws.qw + (uint64_t)qq * W;
    }
    // Two register sets named statically (the chunk loop is unrolled): chunk
    // ch multiplies with set ch & 1 while set (ch + 1) & 1 is being loaded (a
    // copy from one set into the other made every chunk wait for the loads it
    // had just issued).  Every wave loads them, unconditionally: rows past the
    // block read query 0, and loads under a branch made the compiler's wait
    // counts assume the worst.
    wv4i Ab[2][QT][F::kSteps];
    uint64_t Aw[2][QT][F::kSteps];  // fp4: the raw words in flight
#pragma unroll
    for (int mq = 0; mq < QT; ++mq)
#pragma unroll
      for (uint32_t st = 0; st < F::kSteps; ++st) {
        if constexpr (FMT == 1) Aw[0][mq][st] = qraw[mq][st];
        else Ab[0][mq][st] = *reinterpret_cast<const wv4i *>(abase[mq] + 32 * st);
      }
    // Chunk ch is expanded into bt[ch & 1] while the other buffer may still be
    // read by the products of chunk ch - 1: one barrier per chunk.
#pragma unroll
    for (uint32_t ch = 0; ch < NCH; ++ch) {
      // the next chunk's query fragments, requested before this chunk's
      // barrier so that a whole chunk of work covers their latency
      if (ch + 1 < NCH) {
#pragma unroll
        for (int mq = 0; mq < QT; ++mq)
#pragma unroll
          for (uint32_t st = 0; st < F::kSteps; ++st) {
            if constexpr (FMT == 1) Aw[(ch + 1) & 1][mq][st] = qraw[mq][kWChunk * (ch + 1) + st];
            else
              Ab[(ch + 1) & 1][mq][st] = *reinterpret_cast<const wv4i *>(
                  abase[mq] + (ch + 1) * F::kChunkBytes + 32 * st);
          }
      }
      if constexpr (FMT == 1) {
#pragma unroll
        for (int mq = 0; mq < QT; ++mq)
#pragma unroll
          for (uint32_t st = 0; st < F::kSteps; ++st) {
            uint32_t o[8];
            F::expand32((uint32_t)(Aw[ch & 1][mq][st] >> (32 * (lane >> 5))), o);
            Ab[ch & 1][mq][st] = wv4i{(int)o[0], (int)o[1], (int)o[2], (int)o[3]};
          }
      }
      const uint64_t wa = wr[ch][0], wb = wr[ch][1];
      mypop += (uint32_t)(__popcll(wa) + __popcll(wb));
      // expand this thread's 128 keys of the chunk into the record's row
      {
        const uint32_t parts[4] = {(uint32_t)wa, (uint32_t)(wa >> 32), (uint32_t)wb,
                                   (uint32_t)(wb >> 32)};
        uint8_t *dst = bt[ch & 1] + rr * RS + h * (F::kChunkBytes / 2);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          uint32_t o[8];
          F::expand32(parts[m], o);
          constexpr uint32_t nb = F::kChunkBytes / 8;
#pragma unroll
          for (uint32_t e = 0; e < nb / 16; ++e) {
            const wv4i v = {(int)o[4 * e], (int)o[4 * e + 1], (int)o[4 * e + 2], (int)o[4 * e + 3]};
            *reinterpret_cast<wv4i *>(dst + m * nb + 16 * e) = v;
          }
        }
      }
      __syncthreads();
      // the wave's record rows 32 (CT rg + ct) + (lane & 31) of this chunk
      const uint8_t *bbuf =
          bt[ch & 1] + (32 * CT * rg + (lane & 31)) * RS + 16 * (lane >> 5);
      if (live && FMT == 0) {
#pragma unroll
        for (uint32_t st = 0; st < F::kSteps; ++st) {
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            const wv4i bb = *reinterpret_cast<const wv4i *>(bbuf + 32 * ct * RS + 32 * st);
#pragma unroll
            for (int mq = 0; mq < QT; ++mq)
              acc[mq][ct] = F::mma(Ab[ch & 1][mq][st], bb, acc[mq][ct]);
          }
        }
      } else if (live) {
        // fp4: the record fragments of step st + 1 are read from LDS while
        // step st multiplies (two register sets; the scheduling barriers keep
        // the compiler from sinking the reads next to their products, which
        // left every product waiting for its read)
        wv4i bq[2][CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
          bq[0][ct] = *reinterpret_cast<const wv4i *>(bbuf + 32 * ct * RS);
#pragma unroll
        for (uint32_t st = 0; st < F::kSteps; ++st) {
          if (st + 1 < F::kSteps) {
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
              bq[(st + 1) & 1][ct] =
                  *reinterpret_cast<const wv4i *>(bbuf + 32 * ct * RS + 32 * (st + 1));
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int mq = 0; mq < QT; ++mq)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
              acc[mq][ct] = F::mma(Ab[ch & 1][mq][st], bq[st & 1][ct], acc[mq][ct]);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    atomicAdd(&pr[rr], mypop);
    __syncthreads();
    if (!live) continue;
    // u = |q| - T - 1 + |r| - 2 q.r < 0 marks a candidate
    int32_t any = 0;
#pragma unroll
    for (int mq = 0; mq < QT; ++mq)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const uint32_t rw = 32 * (QT * qg + mq) + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
          const uint32_t col = 32 * (CT * rg + ct) + (lane & 31);
          any |= cq[rw] + (int32_t)pr[col] - 2 * F::val(acc[mq][ct], e);
        }
    if (__ballot(any < 0) == 0) continue;
#pragma unroll
    for (int mq = 0; mq < QT; ++mq)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const uint32_t col = 32 * (CT * rg + ct) + (lane & 31);
      const bool cok = v0 + col < vend;
      const uint64_t gc = cok ? wv2g(rs, v0 + col) : 0;
#pragma unroll 1
      for (int e = 0; e < 16; ++e) {
        const uint32_t rw = 32 * (QT * qg + mq) + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        const int32_t dot = F::val(acc[mq][ct], e);
        const int32_t u = cq[rw] + (int32_t)pr[col] - 2 * dot;
        const bool hit = u < 0 && cok && rw < qb.count;
        const uint64_t bal = __ballot(hit);
        if (bal == 0) continue;
        // the 32 lanes of a half share the row rw
        const uint32_t half = lane >> 5;
        const uint32_t mine = (uint32_t)(bal >> (32 * half));
        const uint32_t q = qid[rw];
        uint32_t base = 0;
        const uint32_t lead = mine ? 32 * half + (uint32_t)(__ffs(mine) - 1) : lane;
        if (mine && lane == lead) base = atomicAdd(ws.ctr + q, (uint32_t)__popc(mine));
        base = __shfl(base, (int)lead);
        if (hit) {
          const uint32_t pos = base + (uint32_t)__popc(mine & ((1u << (lane & 31)) - 1u));
          const uint32_t d = (uint32_t)(u + tq[rw] + 1);
          if (pos < ws.qi[q].cap) ws.cand[ws.qi[q].cand_off + pos] = ((uint64_t)d << 32) | gc;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Refine (between phases) and select: one block per query.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_wrefine(WWs ws) {
  __shared__ uint32_t h[kWMaxBins];
  __shared__ uint32_t part[256];
  const uint32_t q = blockIdx.x, tid = threadIdx.x, bins = ws.bins;
  const WQuery qi = ws.qi[q];
  if (qi.keff == 0) return;
  const uint32_t c = ws.ctr[q];
  if (c > qi.cap) return;  // overflowed: answered by the fallback
  for (uint32_t i = tid; i < bins; i += blockDim.x) h[i] = 0;
  __syncthreads();
  for (uint32_t i = tid; i < c; i += blockDim.x)
    atomicAdd(&h[(uint32_t)(ws.cand[qi.cand_off + i] >> 32)], 1u);
  __syncthreads();
  const int32_t T1 = (int32_t)ws.T[q];
  if (T1 <= 0) return;
  uint32_t cum;
  const uint32_t t = block_kth(h, bins, (uint32_t)(T1 - 1), qi.keff, part, &cum);
  if (t != 0xFFFFFFFFu && tid == 0) ws.T[q] = t;
}

__device__ __forceinline__ uint32_t wslot(uint32_t *ctr) {
  const uint64_t act = __ballot(1);
  const uint32_t leader = (uint32_t)__ffsll((unsigned long long)act) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(ctr, (uint32_t)__popcll(act));
  base = __shfl(base, (int)leader);
  return base + rank_below(act);
}

__global__ __launch_bounds__(256) void k_wselect(WWs ws) {
  __shared__ uint32_t h[kWMaxBins];
  __shared__ uint32_t part[256];
  __shared__ uint64_t keys[kWSortCap];
  __shared__ uint32_t s_n;
  const uint32_t q = blockIdx.x, tid = threadIdx.x, bins = ws.bins;
  const WQuery qi = ws.qi[q];
  if (qi.keff == 0) return;
  const uint32_t c = ws.ctr[q];
  if (tid == 0) ws.count[q] = c;
  if (c > qi.cap) {
    if (tid == 0) ws.flags[q] |= 1u;
    return;
  }
  for (uint32_t i = tid; i < bins; i += blockDim.x) h[i] = 0;
  if (tid == 0) s_n = 0;
  __syncthreads();
  const uint64_t *cand = ws.cand + qi.cand_off;
  for (uint32_t i = tid; i < c; i += blockDim.x) atomicAdd(&h[(uint32_t)(cand[i] >> 32)], 1u);
  __syncthreads();
  uint32_t m;
  const uint32_t dk = block_kth(h, bins, bins - 1, qi.keff, part, &m);
  if (dk == 0xFFFFFFFFu || m > kWSortCap) {
    if (tid == 0) ws.flags[q] |= dk == 0xFFFFFFFFu ? 4u : 2u;
    return;
  }
  for (uint32_t i = tid; i < c; i += blockDim.x) {
    const uint64_t key = cand[i];
    if ((uint32_t)(key >> 32) <= dk) keys[wslot(&s_n)] = key;
  }
  __syncthreads();
  uint32_t P = 1;
  while (P < m) P <<= 1;
  for (uint32_t i = m + tid; i < P; i += blockDim.x) keys[i] = ~0ull;
  __syncthreads();
  for (uint32_t k = 2; k <= P; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = tid; i < P; i += blockDim.x) {
        const uint32_t ixj = i ^ j;
        if (ixj > i) {
          const uint64_t a = keys[i], b2 = keys[ixj];
          if ((a > b2) == ((i & k) == 0)) {
            keys[i] = b2;
            keys[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t i = tid; i < qi.keff; i += blockDim.x) {
    fps_hit hh;
    hh.index = (uint32_t)keys[i];
    hh.distance = (uint32_t)(keys[i] >> 32);
    ws.out[qi.out_off + i] = hh;
  }
}

// ---------------------------------------------------------------------------
// Exact ordered fallback for one query (as the MACCS engine's): per-wave
// histograms, their prefix over waves, then every record with d <= D_k goes to
// its rank in (distance, index) order.
// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(256) void k_wfb_hist(WLib L, WWs ws, uint32_t qidx, uint64_t chunk) {
  __shared__ uint32_t h[4][kWMaxBins];
  const WQuery qi = ws.qi[qidx];
  const WRange *rs = ws.rs + qi.rset;
  const uint32_t wl = threadIdx.x >> 6, lane = lane_id(), bins = ws.bins;
  const uint64_t w = (uint64_t)blockIdx.x * 4 + wl;
  uint64_t qw[W];
#pragma unroll
  for (int k = 0; k < W; ++k) qw[k] = ws.qw[(uint64_t)qidx * W + k];
  for (uint32_t i = threadIdx.x; i < 4 * kWMaxBins; i += blockDim.x) (&h[0][0])[i] = 0;
  __syncthreads();
  const uint64_t v0 = w * chunk, v1 = min(v0 + chunk, rs->neff);
  for (uint64_t v = v0 + lane; v < v1; v += 64) atomicAdd(&h[wl][wdist<W>(L, wv2g(rs, v), qw)], 1u);
  __syncthreads();
  for (uint32_t b = lane; b < bins; b += 64) ws.fbh[w * bins + b] = h[wl][b];
}

__global__ __launch_bounds__(256) void k_wfb_scan(WWs ws) {
  __shared__ uint32_t part[256];
  const uint32_t bin = blockIdx.x, tid = threadIdx.x, bins = ws.bins;
  uint32_t carry = 0;
  for (uint32_t w0 = 0; w0 < kWFbWaves; w0 += 256) {
    const uint32_t x = ws.fbh[(uint64_t)(w0 + tid) * bins + bin];
    part[tid] = x;
    __syncthreads();
    for (uint32_t off = 1; off < 256; off <<= 1) {
      const uint32_t y = tid >= off ? part[tid - off] : 0;
      __syncthreads();
      part[tid] += y;
      __syncthreads();
    }
    ws.fbo[(uint64_t)(w0 + tid) * bins + bin] = carry + part[tid] - x;
    carry += part[255];
    __syncthreads();
  }
  if (tid == 0) ws.fbt[bin] = carry;
}

template <int W>
__global__ __launch_bounds__(256) void k_wfb_emit(WLib L, WWs ws, uint32_t qidx, uint64_t chunk) {
  __shared__ uint32_t cumex[kWMaxBins];
  __shared__ uint32_t run[4][kWMaxBins];
  __shared__ uint32_t s_dk;
  const WQuery qi = ws.qi[qidx];
  const WRange *rs = ws.rs + qi.rset;
  const uint32_t bins = ws.bins, keff = qi.keff;
  fps_hit *out = ws.out + qi.out_off;
  const uint32_t wl = threadIdx.x >> 6, lane = lane_id();
  const uint64_t w = (uint64_t)blockIdx.x * 4 + wl;
  uint64_t qw[W];
#pragma unroll
  for (int k = 0; k < W; ++k) qw[k] = ws.qw[(uint64_t)qidx * W + k];
  for (uint32_t i = threadIdx.x; i < 4 * kWMaxBins; i += blockDim.x) (&run[0][0])[i] = 0;
  if (threadIdx.x == 0) {
    uint32_t cum = 0, dk = bins - 1;
    bool found = false;
    for (uint32_t t = 0; t < bins; ++t) {
      cumex[t] = cum;
      cum += ws.fbt[t];
      if (!found && cum >= keff) {
        dk = t;
        found = true;
      }
    }
    s_dk = dk;
  }
  __syncthreads();
  const uint32_t dk = s_dk;
  const uint64_t v0 = w * chunk, v1 = min(v0 + chunk, rs->neff);
  const uint32_t *woff = ws.fbo + w * bins;
  const uint64_t lt = (1ull << lane) - 1ull;
  for (uint64_t step = 0; step < chunk; step += 64) {
    const uint64_t v = v0 + step + lane;
    uint32_t d = 0;
    uint64_t g = 0;
    bool act = false;
    if (v < v1) {
      g = wv2g(rs, v);
      d = wdist<W>(L, g, qw);
      act = d <= dk;
    }
    uint64_t eq = __ballot(act);
#pragma unroll
    for (int bit = 0; bit < 12; ++bit) {
      const bool set = (d >> bit) & 1u;
      const uint64_t bb = __ballot(act && set);
      eq &= set ? bb : ~bb;
    }
    if (act) {
      const uint32_t pos = cumex[d] + woff[d] + run[wl][d] + (uint32_t)__popcll(eq & lt);
      if (pos < keff) {
        out[pos].index = (uint32_t)g;
        out[pos].distance = d;
      }
    }
    __syncthreads();
    if (act && (eq & ~(lt | (1ull << lane))) == 0) run[wl][d] += (uint32_t)__popcll(eq);
    __syncthreads();
  }
}

}  // namespace fps

// ===========================================================================
// Host side.
// ===========================================================================
using namespace fps;

#define WHIP(x)                                                                              \
  do {                                                                                       \
    hipError_t e_ = (x);                                                                     \
    if (e_ != hipSuccess) return fps_fail(FPS_E_DEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

struct fps_wide {
  uint64_t n = 0, np = 0;
  uint32_t W = 0, nstrides = 0;
  uint64_t strides[FPS_MAX_STRIDES + 1] = {};
  uint64_t *dev = nullptr;
  int device = 0, cus = 256;
  fps_path path = FPS_PATH_AUTO;
  double cand_scale = 1.0;
  uint64_t sample = kWSample;
  int force_fb = 0;
  bool timing = false;
  hipEvent_t ev[4] = {};
  fps_search_stats last{};
  ~fps_wide() {
    for (auto &e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

static bool w_supported(uint32_t W) { return W == 4 || W == 8 || W == 16 || W == 32; }

extern "C" size_t fps_wide_device_bytes(uint64_t n, uint32_t words) {
  const uint64_t np = (n + kRowAlign - 1) / kRowAlign * kRowAlign;
  return (size_t)(np * 8 * words);
}

extern "C" fps_status fps_wide_load(const uint64_t *host_words, uint64_t n, uint32_t words,
                                    const uint64_t *stride_begin, uint32_t nstrides,
                                    void *device_buf, size_t device_bytes, void *stream,
                                    fps_wide **out) {
  fps_clear_error();
  if (!host_words || !device_buf || !out) return fps_fail(FPS_E_ARG, "NULL argument");
  if (!w_supported(words))
    return fps_fail(FPS_E_ARG, "words = %u: 4, 8, 16 or 32 supported", words);
  if (n == 0 || n >= (1ull << 32)) return fps_fail(FPS_E_ARG, "n = %llu out of range", (unsigned long long)n);
  if (device_bytes < fps_wide_device_bytes(n, words))
    return fps_fail(FPS_E_ARG, "device buffer of %zu bytes < %zu needed", device_bytes,
                    fps_wide_device_bytes(n, words));
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
  auto *L = new (std::nothrow) fps_wide();
  if (!L) return fps_fail(FPS_E_NOMEM, "host allocation failed");
  L->n = n;
  L->np = (n + kRowAlign - 1) / kRowAlign * kRowAlign;
  L->W = words;
  L->nstrides = (uint32_t)st.size() - 1;
  std::copy(st.begin(), st.end(), L->strides);
  L->dev = (uint64_t *)device_buf;
  hipStream_t s = (hipStream_t)stream;
  fps_status rc = FPS_OK;
  do {
    if (hipGetDevice(&L->device) != hipSuccess ||
        hipDeviceGetAttribute(&L->cus, hipDeviceAttributeMultiprocessorCount, L->device) !=
            hipSuccess) {
      rc = fps_fail(FPS_E_DEVICE, "cannot query the current device");
      break;
    }
    for (auto &e : L->ev)
      if (hipEventCreate(&e) != hipSuccess) rc = fps_fail(FPS_E_DEVICE, "hipEventCreate failed");
    if (rc) break;
    // transpose record-major host words into the W word-major arrays
    const uint64_t CH = 1u << 18;
    std::vector<uint64_t> tmp;
    tmp.resize(CH);
    for (uint64_t c0 = 0; c0 < n && !rc; c0 += CH) {
      const uint64_t m = std::min(n, c0 + CH) - c0;
      for (uint32_t k = 0; k < words && !rc; ++k) {
        for (uint64_t i = 0; i < m; ++i) tmp[i] = host_words[(c0 + i) * words + k];
        if (hipMemcpyAsync(L->dev + (uint64_t)k * L->np + c0, tmp.data(), 8 * m,
                           hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          rc = fps_fail(FPS_E_DEVICE, "upload failed");
      }
    }
    for (uint32_t k = 0; k < words && !rc; ++k)
      if (L->np > n && hipMemsetAsync(L->dev + (uint64_t)k * L->np + n, 0, 8 * (L->np - n), s) !=
                           hipSuccess)
        rc = fps_fail(FPS_E_DEVICE, "hipMemsetAsync failed");
    if (!rc && hipStreamSynchronize(s) != hipSuccess)
      rc = fps_fail(FPS_E_DEVICE, "stream synchronize failed");
  } while (0);
  if (rc) {
    delete L;
    return rc;
  }
  *out = L;
  return FPS_OK;
}

extern "C" fps_status fps_wide_free(fps_wide *lib) {
  fps_clear_error();
  delete lib;
  return FPS_OK;
}

extern "C" fps_status fps_wide_set_path(fps_wide *lib, fps_path path) {
  fps_clear_error();
  if (!lib || path < FPS_PATH_AUTO || path > FPS_PATH_MFMA_F4)
    return fps_fail(FPS_E_ARG, "bad argument");
  lib->path = path;
  return FPS_OK;
}

extern "C" fps_status fps_wide_set_tuning(fps_wide *lib, double candidate_scale,
                                          uint64_t sample_records, int force_fallback) {
  fps_clear_error();
  if (!lib || !(candidate_scale > 0)) return fps_fail(FPS_E_ARG, "bad argument");
  lib->cand_scale = candidate_scale;
  lib->sample = sample_records ? sample_records : kWSample;
  lib->force_fb = force_fallback;
  return FPS_OK;
}

extern "C" fps_status fps_wide_set_timing(fps_wide *lib, int enable) {
  fps_clear_error();
  if (!lib) return fps_fail(FPS_E_ARG, "NULL argument");
  lib->timing = enable != 0;
  return FPS_OK;
}

extern "C" fps_status fps_wide_last_search_stats(const fps_wide *lib, fps_search_stats *stats) {
  fps_clear_error();
  if (!lib || !stats) return fps_fail(FPS_E_ARG, "NULL argument");
  *stats = lib->last;
  return FPS_OK;
}

// ---- plan ----
struct WPlan {
  uint32_t q = 0, W = 0, bins = 0, qbs = 1;
  fps_path path = FPS_PATH_SINGLE;
  std::vector<WRange> rs;
  std::vector<WQuery> qi;
  std::vector<uint32_t> perm;
  std::vector<WBlock> qb;
  std::vector<uint64_t> bounds;  // phase boundaries in virtual records: 0, P1, ..., max neff
  std::vector<uint64_t> items;   // per phase: nqb + 1 prefix
  uint64_t max_neff = 0, total_cand = 0, total_out = 0, max_sample = 0;
  size_t off_rs = 0, off_qi = 0, off_perm = 0, off_qb = 0, off_items = 0, off_qw = 0,
         params = 0;
  size_t off_qx = 0, off_T = 0, off_ctr = 0, off_flags = 0, off_count = 0, off_hist = 0,
         off_bdone = 0, off_cand = 0, off_out = 0, off_fbh = 0, off_fbo = 0, off_fbt = 0,
         total = 0;
};

static inline size_t wal(size_t x) { return (x + 255) & ~(size_t)255; }

static fps_status w_rangeset(const fps_wide *lib, uint32_t mask, WRange *r) {
  memset(r, 0, sizeof(*r));
  uint32_t ns = lib->nstrides;
  if (mask == 0) return fps_fail(FPS_E_ARG, "stride mask 0 selects nothing");
  if (mask != FPS_MASK_ALL && ns < 32 && (mask >> ns) != 0)
    return fps_fail(FPS_E_ARG, "mask 0x%x names a stride the library does not have", mask);
  uint64_t v = 0;
  for (uint32_t s = 0; s < ns; ++s) {
    if (!((mask >> s) & 1u)) continue;
    const uint64_t b = lib->strides[s], e = lib->strides[s + 1];
    if (b == e) continue;
    if (r->nranges && r->end[r->nranges - 1] == b) {
      r->end[r->nranges - 1] = e;
    } else {
      r->begin[r->nranges] = b;
      r->end[r->nranges] = e;
      r->voff[r->nranges] = v;
      r->nranges++;
    }
    v += e - b;
  }
  r->voff[r->nranges] = v;
  r->neff = v;
  return FPS_OK;
}

static fps_path w_default_path(uint32_t q) {
  if (q <= 2) return FPS_PATH_SINGLE;
  if (q < 32) return FPS_PATH_POPCOUNT;
  return FPS_PATH_MFMA_F4;
}

static fps_status w_plan(const fps_wide *lib, uint32_t q, const uint32_t *k, const uint32_t *mask,
                         WPlan *P) {
  if (!lib || !k || q == 0) return fps_fail(FPS_E_ARG, "NULL argument or q = 0");
  if (q > 65535) return fps_fail(FPS_E_ARG, "q = %u: at most 65,535 queries per call", q);
  P->q = q;
  P->W = lib->W;
  P->bins = 64 * lib->W + 1;
  P->path = lib->path == FPS_PATH_AUTO ? w_default_path(q) : lib->path;
  P->qbs = P->path == FPS_PATH_MFMA_I8 || P->path == FPS_PATH_MFMA_F4
               ? kWMmaQB
               : (P->path == FPS_PATH_POPCOUNT ? kWPopQB : 1u);
  std::vector<uint32_t> masks;
  std::vector<uint32_t> rset(q);
  for (uint32_t i = 0; i < q; ++i) {
    const uint32_t m = mask ? mask[i] : FPS_MASK_ALL;
    uint32_t j = 0;
    while (j < masks.size() && masks[j] != m) ++j;
    if (j == masks.size()) {
      WRange r;
      fps_status rc = w_rangeset(lib, m, &r);
      if (rc) return rc;
      masks.push_back(m);
      P->rs.push_back(r);
    }
    rset[i] = j;
  }
  P->qi.resize(q);
  for (uint32_t i = 0; i < q; ++i) {
    const WRange &r = P->rs[rset[i]];
    WQuery &w = P->qi[i];
    w.keff = (uint32_t)std::min<uint64_t>(k[i], r.neff);
    w.rset = rset[i];
    w.sample = std::min<uint64_t>(lib->sample, r.neff);
    P->max_neff = std::max(P->max_neff, r.neff);
    P->max_sample = std::max(P->max_sample, w.sample);
  }
  // phases: 0, sample * G, sample * G^2, ... up to the largest range
  P->bounds = {0};
  uint64_t b = std::max<uint64_t>(lib->sample, 1) * kWGrowth;
  while (b < P->max_neff) {
    P->bounds.push_back(b);
    b *= kWGrowth;
  }
  P->bounds.push_back(std::max<uint64_t>(P->max_neff, 1));
  const uint64_t nph = P->bounds.size() - 1;
  for (uint32_t i = 0; i < q; ++i) {
    WQuery &w = P->qi[i];
    double cap = (64.0 * w.keff + 4096.0) * lib->cand_scale;
    if (cap > 4e9) cap = 4e9;
    w.cap = w.keff ? std::max<uint32_t>(1, (uint32_t)cap) : 0u;
    w.cand_off = P->total_cand;
    P->total_cand += w.cap;
    w.out_off = P->total_out;
    P->total_out += w.keff;
    w.popc = 0;
  }
  // query blocks: queries of one range set, in query order, at most qbs each
  P->perm.clear();
  for (uint32_t r = 0; r < P->rs.size(); ++r) {
    uint32_t first = (uint32_t)P->perm.size(), cnt = 0;
    for (uint32_t i = 0; i < q; ++i) {
      if (rset[i] != r) continue;
      P->perm.push_back(i);
      if (++cnt == P->qbs) {
        P->qb.push_back(WBlock{first, cnt, r, 0});
        first += cnt;
        cnt = 0;
      }
    }
    if (cnt) P->qb.push_back(WBlock{first, cnt, r, 0});
  }
  const uint64_t per_item = P->path == FPS_PATH_POPCOUNT
                                ? 256ull * (P->W >= 16 ? 1 : (P->W == 8 ? 2 : 4))
                                : (uint64_t)kWMmaRT;
  const uint32_t nqb = (uint32_t)P->qb.size();
  P->items.assign(nph * (nqb + 1), 0);
  for (uint64_t p = 0; p < nph; ++p)
    for (uint32_t j = 0; j < nqb; ++j) {
      const uint64_t ne = P->rs[P->qb[j].rset].neff;
      const uint64_t lo = P->bounds[p], hi = std::min(P->bounds[p + 1], ne);
      const uint64_t cnt = hi > lo ? (hi - lo + per_item - 1) / per_item : 0;
      P->items[p * (nqb + 1) + j + 1] = P->items[p * (nqb + 1) + j] + cnt;
    }
  // workspace layout: parameter block, then the device-side arrays
  size_t o = 0;
  P->off_rs = o;
  o = wal(o + sizeof(WRange) * P->rs.size());
  P->off_qi = o;
  o = wal(o + sizeof(WQuery) * q);
  P->off_perm = o;
  o = wal(o + 4ull * q);
  P->off_qb = o;
  o = wal(o + sizeof(WBlock) * nqb);
  P->off_items = o;
  o = wal(o + 8 * P->items.size());
  P->off_qw = o;
  o = wal(o + 8ull * q * P->W);
  P->params = o;
  P->off_qx = o;
  if (P->path == FPS_PATH_MFMA_I8) o = wal(o + 8ull * P->W * 8 * q);
  P->off_T = o;
  o = wal(o + 4ull * q);
  P->off_ctr = o;
  o = wal(o + 4ull * q);
  P->off_flags = o;
  o = wal(o + 4ull * q);
  P->off_count = o;
  o = wal(o + 4ull * q);
  P->off_bdone = o;
  o = wal(o + 4ull * q);
  P->off_hist = o;
  o = wal(o + 4ull * q * P->bins);
  P->off_cand = o;
  o = wal(o + 8 * P->total_cand);
  P->off_out = o;
  o = wal(o + sizeof(fps_hit) * std::max<uint64_t>(P->total_out, 1));
  P->off_fbh = o;
  o = wal(o + 4ull * kWFbWaves * P->bins);
  P->off_fbo = o;
  o = wal(o + 4ull * kWFbWaves * P->bins);
  P->off_fbt = o;
  o = wal(o + 4ull * P->bins);
  P->total = o;
  return FPS_OK;
}

extern "C" fps_status fps_wide_workspace_bytes(const fps_wide *lib, uint32_t q, const uint32_t *k,
                                               const uint32_t *mask, size_t *bytes) {
  fps_clear_error();
  if (!bytes) return fps_fail(FPS_E_ARG, "NULL argument");
  WPlan P;
  fps_status rc = w_plan(lib, q, k, mask, &P);
  if (rc) return rc;
  *bytes = P.total;
  return FPS_OK;
}

template <int W>
static void w_launch_scan(const WLib &L, const WWs &ws, const WPlan &P, uint64_t p, int cus,
                          hipStream_t s) {
  const uint64_t vb = P.bounds[p], ve = P.bounds[p + 1];
  const uint32_t nqb = (uint32_t)P.qb.size();
  const uint64_t *item_dev = ws.item_off + p * (nqb + 1);
  const uint64_t items = P.items[p * (nqb + 1) + nqb];
  switch (P.path) {
    case FPS_PATH_POPCOUNT: {
      if (!items) return;
      const uint32_t blocks = (uint32_t)std::min<uint64_t>(items, (uint64_t)cus * 8);
      constexpr int RPT = W >= 16 ? 1 : (W == 8 ? 2 : 4);  // records per thread
      hipLaunchKernelGGL((k_wscan_pop<W, RPT>), dim3(blocks), dim3(256), 0, s, L, ws, item_dev,
                         vb, ve, items);
      return;
    }
    case FPS_PATH_MFMA_I8:
    case FPS_PATH_MFMA_F4: {
      if (!items) return;
      const uint32_t blocks = (uint32_t)std::min<uint64_t>(items, (uint64_t)cus * 4);
      if (P.path == FPS_PATH_MFMA_I8)
        hipLaunchKernelGGL((k_wscan_mma<W, 0>), dim3(blocks), dim3(256), 0, s, L, ws, item_dev,
                           vb, ve, items);
      else
        hipLaunchKernelGGL((k_wscan_mma<W, 1>), dim3(blocks), dim3(256), 0, s, L, ws, item_dev,
                           vb, ve, items);
      return;
    }
    default: {
      for (uint32_t i = 0; i < P.q; ++i) {
        const uint64_t ne = P.rs[P.qi[i].rset].neff;
        if (P.qi[i].keff == 0 || vb >= ne) continue;
        const uint64_t tiles = (std::min(ve, ne) - vb) / kWTile + 2 * FPS_MAX_STRIDES;
        // up to 128 blocks per CU: 2 % less scan time than 16 over 24 M records
        const uint32_t blocks = (uint32_t)std::min<uint64_t>((tiles + 3) / 4, (uint64_t)cus * 128);
        hipLaunchKernelGGL((k_wscan1<W>), dim3(blocks), dim3(256), 0, s, L, ws, i, vb, ve);
      }
    }
  }
}

template <int W>
static void w_launch_front(const WLib &L, const WWs &ws, const WPlan &P, hipStream_t s) {
  uint64_t chunk = (P.max_sample + 63) / 64;
  chunk = std::max<uint64_t>(1024, (chunk + 1023) / 1024 * 1024);
  const uint32_t chunks = (uint32_t)std::max<uint64_t>(1, (P.max_sample + chunk - 1) / chunk);
  hipLaunchKernelGGL((k_wbound<W>), dim3(chunks, (P.q + kWBoundQ - 1) / kWBoundQ), dim3(256), 0,
                     s, L, ws, (uint32_t)chunk, P.q);
  if (P.path == FPS_PATH_MFMA_I8) {  // (the fp4 kernel expands raw query words itself)
    const uint64_t parts = 2ull * W * P.q;
    hipLaunchKernelGGL((k_wexpand<W, 0>), dim3((uint32_t)((parts + 255) / 256)), dim3(256), 0, s,
                       ws, P.q);
  }
}

template <int W>
static void w_launch_fallback(const WLib &L, const WWs &ws, uint32_t qidx, uint64_t neff,
                              hipStream_t s) {
  uint64_t chunk = (neff + kWFbWaves - 1) / kWFbWaves;
  chunk = (chunk + 63) & ~(uint64_t)63;
  if (chunk == 0) chunk = 64;
  hipLaunchKernelGGL((k_wfb_hist<W>), dim3(kWFbBlocks), dim3(256), 0, s, L, ws, qidx, chunk);
  hipLaunchKernelGGL(k_wfb_scan, dim3(ws.bins), dim3(256), 0, s, ws);
  hipLaunchKernelGGL((k_wfb_emit<W>), dim3(kWFbBlocks), dim3(256), 0, s, L, ws, qidx, chunk);
}

#define W_DISPATCH(W, F, ...)                  \
  switch (W) {                                 \
    case 4: F<4>(__VA_ARGS__); break;          \
    case 8: F<8>(__VA_ARGS__); break;          \
    case 16: F<16>(__VA_ARGS__); break;        \
    default: F<32>(__VA_ARGS__); break;        \
  }

extern "C" fps_status fps_wide_search_batch(fps_wide *lib, const uint64_t *queries, uint32_t q,
                                            const uint32_t *k, const uint32_t *mask,
                                            void *workspace, size_t ws_bytes, fps_hit *out,
                                            uint64_t out_capacity, uint64_t *out_offset,
                                            void *stream) {
  fps_clear_error();
  if (!lib || !queries || !k || !workspace || !out_offset || (!out && out_capacity))
    return fps_fail(FPS_E_ARG, "NULL argument");
  if (((uintptr_t)workspace & 255) != 0)
    return fps_fail(FPS_E_ARG, "workspace must be 256-byte aligned");
  WPlan P;
  fps_status rc = w_plan(lib, q, k, mask, &P);
  if (rc) return rc;
  if (ws_bytes < P.total)
    return fps_fail(FPS_E_NOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, P.total);
  if (out_capacity < P.total_out)
    return fps_fail(FPS_E_ARG, "out_capacity %llu < %llu hits", (unsigned long long)out_capacity,
                    (unsigned long long)P.total_out);
  const uint32_t W = lib->W;
  for (uint32_t i = 0; i < q; ++i) {
    uint32_t pc = 0;
    for (uint32_t w = 0; w < W; ++w) pc += (uint32_t)__builtin_popcountll(queries[(size_t)i * W + w]);
    P.qi[i].popc = pc;
  }
  // parameter block
  std::vector<uint8_t> blk(P.params, 0);
  memcpy(blk.data() + P.off_rs, P.rs.data(), sizeof(WRange) * P.rs.size());
  memcpy(blk.data() + P.off_qi, P.qi.data(), sizeof(WQuery) * q);
  memcpy(blk.data() + P.off_perm, P.perm.data(), 4ull * q);
  memcpy(blk.data() + P.off_qb, P.qb.data(), sizeof(WBlock) * P.qb.size());
  memcpy(blk.data() + P.off_items, P.items.data(), 8 * P.items.size());
  memcpy(blk.data() + P.off_qw, queries, 8ull * q * W);
  uint8_t *b = (uint8_t *)workspace;
  WWs ws;
  ws.rs = (const WRange *)(b + P.off_rs);
  ws.qi = (const WQuery *)(b + P.off_qi);
  ws.perm = (const uint32_t *)(b + P.off_perm);
  ws.qb = (const WBlock *)(b + P.off_qb);
  ws.item_off = (const uint64_t *)(b + P.off_items);
  ws.qw = (const uint64_t *)(b + P.off_qw);
  ws.qx = b + P.off_qx;
  ws.T = (uint32_t *)(b + P.off_T);
  ws.ctr = (uint32_t *)(b + P.off_ctr);
  ws.flags = (uint32_t *)(b + P.off_flags);
  ws.count = (uint32_t *)(b + P.off_count);
  ws.bdone = (uint32_t *)(b + P.off_bdone);
  ws.hist = (uint32_t *)(b + P.off_hist);
  ws.cand = (uint64_t *)(b + P.off_cand);
  ws.out = (fps_hit *)(b + P.off_out);
  ws.fbh = (uint32_t *)(b + P.off_fbh);
  ws.fbo = (uint32_t *)(b + P.off_fbo);
  ws.fbt = (uint32_t *)(b + P.off_fbt);
  ws.bins = P.bins;
  ws.nqb = (uint32_t)P.qb.size();
  WLib L{lib->dev, lib->np, lib->n};
  hipStream_t s = (hipStream_t)stream;
  WHIP(hipMemcpyAsync(b, blk.data(), P.params, hipMemcpyHostToDevice, s));
  const uint32_t pblocks = (uint32_t)std::min<uint64_t>(1024, ((uint64_t)q * P.bins + 255) / 256 + 1);
  if (lib->timing) WHIP(hipEventRecord(lib->ev[0], s));
  hipLaunchKernelGGL(k_wprep, dim3(pblocks), dim3(256), 0, s, ws, q);
  W_DISPATCH(W, w_launch_front, L, ws, P, s);
  if (lib->timing) WHIP(hipEventRecord(lib->ev[2], s));
  const uint64_t nph = P.bounds.size() - 1;
  uint32_t launches = 0;
  for (uint64_t p = 0; p < nph; ++p) {
    W_DISPATCH(W, w_launch_scan, L, ws, P, p, lib->cus, s);
    launches += P.path == FPS_PATH_SINGLE ? q : 1;
    if (p + 1 < nph) hipLaunchKernelGGL(k_wrefine, dim3(q), dim3(256), 0, s, ws);
  }
  if (lib->timing) WHIP(hipEventRecord(lib->ev[3], s));
  hipLaunchKernelGGL(k_wselect, dim3(q), dim3(256), 0, s, ws);
  WHIP(hipGetLastError());
  std::vector<uint32_t> flags(q), count(q);
  WHIP(hipMemcpyAsync(flags.data(), ws.flags, 4ull * q, hipMemcpyDeviceToHost, s));
  WHIP(hipMemcpyAsync(count.data(), ws.count, 4ull * q, hipMemcpyDeviceToHost, s));
  WHIP(hipStreamSynchronize(s));
  uint32_t fallbacks = 0;
  for (uint32_t i = 0; i < q; ++i) {
    if (P.qi[i].keff == 0 || (!flags[i] && !lib->force_fb)) continue;
    W_DISPATCH(W, w_launch_fallback, L, ws, i, P.rs[P.qi[i].rset].neff, s);
    ++fallbacks;
  }
  if (lib->timing) WHIP(hipEventRecord(lib->ev[1], s));
  WHIP(hipGetLastError());
  if (P.total_out)
    WHIP(hipMemcpyAsync(out, ws.out, sizeof(fps_hit) * P.total_out, hipMemcpyDeviceToHost, s));
  WHIP(hipStreamSynchronize(s));
  out_offset[0] = 0;
  for (uint32_t i = 0; i < q; ++i) out_offset[i + 1] = out_offset[i] + P.qi[i].keff;
  fps_search_stats &st = lib->last;
  const double sum_scan = st.scan_ms_sum, sum_total = st.total_ms_sum;
  const uint64_t calls = st.calls, sl = st.scan_launches_sum;
  st = fps_search_stats{};
  st.path = (uint32_t)P.path;
  st.queries = q;
  st.fallbacks = fallbacks;
  for (uint32_t i = 0; i < q; ++i) st.candidates += count[i];
  st.scan_launches = launches;
  if (lib->timing) {
    float a = 0, t = 0;
    if (hipEventElapsedTime(&a, lib->ev[2], lib->ev[3]) == hipSuccess) st.scan_ms = a;
    if (hipEventElapsedTime(&t, lib->ev[0], lib->ev[1]) == hipSuccess) st.total_ms = t;
  }
  st.scan_ms_sum = sum_scan + st.scan_ms;
  st.total_ms_sum = sum_total + st.total_ms;
  st.calls = calls + 1;
  st.scan_launches_sum = sl + launches;
  return FPS_OK;
}

extern "C" fps_status fps_wide_search(fps_wide *lib, const uint64_t *query, uint32_t k,
                                      uint32_t mask, void *workspace, size_t ws_bytes,
                                      fps_hit *out, uint32_t *n_out, void *stream) {
  fps_clear_error();
  if (!n_out) return fps_fail(FPS_E_ARG, "NULL argument");
  uint64_t off[2];
  fps_status rc = fps_wide_search_batch(lib, query, 1, &k, &mask, workspace, ws_bytes, out, k,
                                        off, stream);
  if (rc) return rc;
  *n_out = (uint32_t)off[1];
  return FPS_OK;
}
