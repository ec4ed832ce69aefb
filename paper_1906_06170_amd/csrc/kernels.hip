// Scan, bound, select and fallback kernels for gfx950 (wave64).
//
// The search of FPScreen (Fig. 3) computes, for every library row, the
// Manhattan distance of Section 4.3 to the query and keeps the N smallest.  On
// 0/1 keys that distance is the number of differing keys, so one record costs
// six XORs and six 32-bit popcounts over its four words.  Top-N is exact and
// reads the library once:
//   1. bound:  a histogram of the distances of the first S1 records of each
//      query's range gives T1 = the k-th smallest of them; any k records bound
//      the k-th smallest distance of the whole range from above;
//   2. scan, in phases of geometrically growing length: every record with
//      d <= T is appended to the query's candidate buffer (wave-aggregated:
//      one atomic per wave that has hits);
//   3. refine, between phases: the candidates hold every record of the prefix
//      scanned so far with d <= T, so their histogram gives the k-th smallest
//      distance of that prefix, a tighter bound for the next phase;
//   4. select: a 167-bin histogram of the candidates gives D_k; the candidates
//      with d <= D_k are sorted by (d, index) in LDS and the first k are kept.
// A query whose candidates overflow their buffer, or whose ties at D_k exceed
// the LDS sort, is answered by an exact two-pass ordered fallback.
#include "cand.h"
#include "fps_internal.h"

namespace fps {

// Global record index of virtual index v of a RangeSet.
__device__ __forceinline__ uint64_t v2g(const RangeSet *rs, uint64_t v) {
  uint32_t r = 0;
  const uint32_t nr = rs->nranges;
  while (r + 1 < nr && v >= rs->voff[r + 1]) ++r;
  return rs->begin[r] + (v - rs->voff[r]);
}

// One record in the library layout (see fps_internal.h).
struct Rec {
  uint64_t a, b;
  uint32_t c, d;
};

__device__ __forceinline__ Rec load_rec(const Lib &L, uint64_t g) {
  return Rec{L.a[g], L.b[g], L.c[g], (uint32_t)L.d[g]};
}

// Number of differing keys: popcount of the XOR of the four words.
__device__ __forceinline__ uint32_t dist4(uint64_t a, uint64_t b, uint32_t c, uint32_t d,
                                          uint64_t qa, uint64_t qb, uint32_t qc, uint32_t qd) {
  return (uint32_t)(__popcll(a ^ qa) + __popcll(b ^ qb) + __popc(c ^ qc) + __popc(d ^ qd));
}

__device__ __forceinline__ uint32_t dist_rec(const Rec &r, const QueryInfo *q) {
  return dist4(r.a, r.b, r.c, r.d, q->qa, q->qb, q->qc, q->qd);
}

// ---------------------------------------------------------------------------
// Clears the per-query counters and histograms (a fill kernel, so the sequence
// can be captured into a graph).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void prep_body(const Workspace &ws, uint32_t q, uint32_t nbblocks,
                                          uint32_t nctr) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nctr; i += stride) ws.ctr[i] = 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < q; i += stride) {
    ws.count[i] = 0;
    ws.flags[i] = 0;
    ws.T[i] = 0xFFFFFFFFu;
  }
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nbblocks; i += stride)
    ws.bdone[i] = 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < q * kHistCopies * kBins;
       i += stride)
    ws.hist[i] = 0;
}

__global__ void k_prep(Workspace ws, uint32_t q, uint32_t nbblocks, uint32_t nctr) {
  prep_body(ws, q, nbblocks, nctr);
}

__global__ void k_prep_inline(Workspace ws, uint32_t q, uint32_t nbblocks, uint32_t nctr,
                              uint64_t *dst, InlineParams p) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < p.bytes / 8; i += stride)
    dst[i] = p.w[i];
  prep_body(ws, q, nbblocks, nctr);
}

static uint32_t prep_blocks(uint32_t q) {
  uint32_t blocks = (q * kHistCopies * kBins + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks == 0) blocks = 1;
  return blocks;
}

void launch_prep(const Workspace &ws, uint32_t q, uint32_t nbblocks, uint32_t nctr,
                 hipStream_t s, const LaunchEv &ev) {
  launch_k(k_prep, dim3(prep_blocks(q)), dim3(256), s, ev, ws, q, nbblocks, nctr);
}

void launch_prep_inline(const Workspace &ws, uint32_t q, uint32_t nbblocks, uint32_t nctr,
                        uint8_t *dst, const InlineParams &p, hipStream_t s,
                        const LaunchEv &ev) {
  launch_k(k_prep_inline, dim3(prep_blocks(q)), dim3(256), s, ev, ws, q, nbblocks, nctr,
           (uint64_t *)dst, p);
}

// ---------------------------------------------------------------------------
// Bound: distance histogram of the first `sample` records of each query's
// range.  Grid: x = chunk of `chunk` records, y = block of <= 32 queries
// sharing a range.  Blocks add their histograms into one of 8 copies per query
// (spreading the atomics); the last chunk block of a query block to finish sums
// the copies and sets T1 = smallest t whose cumulative sample count reaches
// keff (166 when the sample holds fewer than keff records, so every record
// passes).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bound(Lib lib, Workspace ws, uint32_t chunk) {
  __shared__ uint32_t h[kBoundQBlock * kBins];
  __shared__ QueryInfo qs[kBoundQBlock];
  __shared__ uint32_t s_last;
  const QBlock bb = ws.bblocks[blockIdx.y];
  const RangeSet *rs = ws.rsets + bb.rset;
  const uint64_t sample = ws.qinfo[ws.perm[bb.first]].sample;
  const uint64_t v0 = (uint64_t)blockIdx.x * chunk;
  const uint32_t tid = threadIdx.x;
  const uint32_t copy = blockIdx.x % kHistCopies;
  if (v0 < sample) {
    const uint64_t v1 = min(v0 + (uint64_t)chunk, sample);
    for (uint32_t i = tid; i < bb.count * kBins; i += blockDim.x) h[i] = 0;
    for (uint32_t i = tid; i < bb.count; i += blockDim.x) qs[i] = ws.qinfo[ws.perm[bb.first + i]];
    __syncthreads();
    // the chunk [v0, v1) of virtual indices, range by range; 8 records per
    // thread in flight
    const uint32_t nr = rs->nranges;
    for (uint32_t r = 0; r < nr; ++r) {
      const uint64_t a = max(v0, rs->voff[r]), b = min(v1, rs->voff[r + 1]);
      if (a >= b) continue;
      const uint64_t gofs = rs->begin[r] - rs->voff[r];  // global index = v + gofs
      for (uint64_t vb = a; vb < b; vb += 256 * 8) {
        Rec rec[8];
        bool ok[8];
        // loads without branches (a lane past the range reads record a of
        // it): under a branch each, the compiler waited between them
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const uint64_t v = vb + 256 * u + tid;
          ok[u] = v < b;
          rec[u] = load_rec(lib, (ok[u] ? v : a) + gofs);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (ok[u])
            for (uint32_t j = 0; j < bb.count; ++j)
              atomicAdd(&h[j * kBins + dist_rec(rec[u], &qs[j])], 1u);
      }
    }
    __syncthreads();
    for (uint32_t i = tid; i < bb.count * kBins; i += blockDim.x) {
      const uint32_t x = h[i];
      if (x)
        atomicAdd(&ws.hist[((uint64_t)ws.perm[bb.first + i / kBins] * kHistCopies + copy) * kBins +
                           i % kBins],
                  x);
    }
  }
  // The histogram adds are device-scope atomics; a block waits for its own to
  // complete before it counts itself done (no L2 write-back per block: a
  // device-scope fence here cost 3 us of a 95.4 M-record query).  Whatever the
  // last block then reads is a count of real sample records, every bin at most
  // its final value, and the keff-th smallest distance of any subset of the
  // sample still bounds D_k from above: the bound can only be looser, never
  // wrong.
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0) s_last = atomicAdd(&ws.bdone[blockIdx.y], 1u) == gridDim.x - 1 ? 1u : 0u;
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  for (uint32_t i = tid; i < bb.count * kBins; i += blockDim.x) {
    const uint32_t *src = ws.hist + (uint64_t)ws.perm[bb.first + i / kBins] * kHistCopies * kBins;
    uint32_t x = 0;
#pragma unroll
    for (int c = 0; c < kHistCopies; ++c)
      x += __hip_atomic_load(src + c * kBins + i % kBins, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    h[i] = x;
  }
  __syncthreads();
  // one wave per query (wave-uniform loop)
  for (uint32_t j = tid >> 6; j < bb.count; j += blockDim.x >> 6) {
    const uint32_t q = ws.perm[bb.first + j];
    const uint32_t keff = ws.qinfo[q].keff;
    uint32_t cum;
    uint32_t T = wave_kth(h + j * kBins, (uint32_t)kKeys, keff, &cum);
    if (T == 0xFFFFFFFFu) T = (uint32_t)kKeys;
    if (lane_id() == 0) ws.T[q] = T;
  }
}

void launch_bound(const Lib &lib, const Workspace &ws, uint32_t nbblocks, uint64_t max_sample,
                  hipStream_t s) {
  if (nbblocks == 0) return;
  // Up to kBoundBlocks chunks of at least kBoundChunk records, and fewer once
  // the query blocks alone fill the GPU: every block adds its histograms into
  // device memory with one atomic per nonzero bin, so more chunks than needed
  // only multiply those atomics.
  const uint64_t per_qb = std::max<uint64_t>(
      1, std::min<uint64_t>(kBoundBlocks, (uint64_t)kBoundGrid / nbblocks));
  uint64_t chunk = (max_sample + per_qb - 1) / per_qb;
  chunk = (chunk + kBoundChunk - 1) / kBoundChunk * kBoundChunk;
  uint32_t chunks = (uint32_t)((max_sample + chunk - 1) / chunk);
  if (chunks == 0) chunks = 1;
  hipLaunchKernelGGL(k_bound, dim3(chunks, nbblocks), dim3(256), 0, s, lib, ws, (uint32_t)chunk);
}

// ---------------------------------------------------------------------------
// Refine: after a scan phase the candidate buffer holds every record of the
// prefix scanned so far with d <= T (each phase appended d <= the bound of its
// time, and bounds only shrink); the keff-th smallest of them is a tighter
// bound.  One block per query.  A query whose buffer overflowed keeps its bound
// (it is answered by the fallback anyway).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_refine(Workspace ws) {
  __shared__ uint32_t hist[kBins];
  __shared__ uint32_t m[kSegments + 1];
  __shared__ uint32_t s_total, s_over;
  const uint32_t q = blockIdx.x, tid = threadIdx.x;
  const QueryInfo *qi = ws.qinfo + q;
  const uint32_t keff = qi->keff;
  if (keff == 0) return;
  for (uint32_t i = tid; i < kBins; i += blockDim.x) hist[i] = 0;
  cand_counts(ws, qi, m, &s_total, &s_over);
  if (s_over) return;
  cand_for_each<true>(ws, qi, m,
                      [&](uint64_t key) { atomicAdd(&hist[(uint32_t)(key >> 32)], 1u); });
  __syncthreads();
  if (tid < 64) {
    const int32_t T1 = (int32_t)ws.T[q];
    if (T1 > 0) {
      uint32_t cum;
      const uint32_t t = wave_kth(hist, (uint32_t)(T1 - 1), keff, &cum);
      if (t != 0xFFFFFFFFu && tid == 0) ws.T[q] = t;
    }
  }
}

void launch_refine(const Workspace &ws, uint32_t q, hipStream_t s) {
  if (q == 0) return;
  hipLaunchKernelGGL(k_refine, dim3(q), dim3(1024), 0, s, ws);
}

// ---------------------------------------------------------------------------
// Single-query scan: HBM-bound stream over the query's ranges.  A wave covers a
// 512-record tile per iteration in four groups of 128 records; in each group a
// lane takes two consecutive records, so every load instruction of the wave
// reads one contiguous segment (16-byte loads of a and b, 8-byte of c, 2-byte
// of d): 16 loads, 168 bytes per lane in flight.  The library is streamed once
// per query, so the loads are nontemporal (they bypass cache retention).
// ---------------------------------------------------------------------------
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void k_scan_single(Lib lib, Workspace ws, uint32_t qidx,
                                                     uint64_t t_begin, uint64_t t_end) {
  const QueryInfo *qi = ws.qinfo + qidx;
  const uint64_t qa = qi->qa, qb = qi->qb;
  const uint32_t qc = qi->qc, qd = qi->qd;
  const int32_t T = (int32_t)ws.T[qidx];
  const RangeSet *rs = ws.rsets + qi->rset;
  const uint32_t lane = lane_id();
  // wave-uniform (scalar) tile loop: the range bookkeeping stays in SGPRs
  const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wib;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const uint32_t seg = (uint32_t)(wave % qi->nseg);
  const uint32_t nranges = rs->nranges;
  // Tiles t = t_begin + wave + j * nwaves, walked range by range so that the
  // range table is read once per range, not per tile.
  for (uint32_t r = 0; r < nranges; ++r) {
  const uint64_t r0 = rs->t1off[r], r1 = rs->t1off[r + 1];
  const uint64_t lo = r0 > t_begin ? r0 : t_begin, hi = r1 < t_end ? r1 : t_end;
  if (lo >= hi) continue;
  const uint64_t rb = rs->begin[r], re = rs->end[r];
  const uint64_t tile0 = (rb & ~(uint64_t)(kScanTile - 1)) - r0 * kScanTile;
  const uint64_t skip = (lo - t_begin) % nwaves;  // first t >= lo of this wave's sequence
  for (uint64_t t = lo + (wave >= skip ? wave - skip : wave + nwaves - skip); t < hi;
       t += nwaves) {
    const uint64_t base = tile0 + t * kScanTile;
    u64x2 A[4], B[4];
    uint64_t C[4];
    uint32_t D[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint64_t i = base + 128 * u + 2 * lane;
      A[u] = __builtin_nontemporal_load(reinterpret_cast<const u64x2 *>(lib.a + i));
      B[u] = __builtin_nontemporal_load(reinterpret_cast<const u64x2 *>(lib.b + i));
      C[u] = __builtin_nontemporal_load(reinterpret_cast<const uint64_t *>(lib.c + i));
      D[u] = __builtin_nontemporal_load(reinterpret_cast<const uint16_t *>(lib.d + i));
    }
    // Distances of the lane's 8 records; the tile's hits take one reservation.
    uint32_t dist[8];
    bool hit[8];
    uint64_t bal[8];
    uint32_t tot = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint64_t i = base + 128 * u + 2 * lane;
      dist[2 * u] = dist4(A[u].x, B[u].x, (uint32_t)C[u], D[u] & 0xFFu, qa, qb, qc, qd);
      dist[2 * u + 1] =
          dist4(A[u].y, B[u].y, (uint32_t)(C[u] >> 32), D[u] >> 8, qa, qb, qc, qd);
      hit[2 * u] = (int32_t)dist[2 * u] <= T && i >= rb && i < re;
      hit[2 * u + 1] = (int32_t)dist[2 * u + 1] <= T && i + 1 >= rb && i + 1 < re;
      bal[2 * u] = __ballot(hit[2 * u]);
      bal[2 * u + 1] = __ballot(hit[2 * u + 1]);
      tot += (uint32_t)(__popcll(bal[2 * u]) + __popcll(bal[2 * u + 1]));
    }
    if (tot == 0) continue;
    Resv rv{0, 0};
    if (lane == 0) rv = cand_reserve(ws, qi, seg, tot);
    rv.base = __shfl(rv.base, 0);
    rv.sbase = __shfl(rv.sbase, 0);
    uint32_t p = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint64_t i = base + 128 * (j >> 1) + 2 * lane + (j & 1);
      if (hit[j]) cand_put(ws, qi, seg, rv, p + rank_below(bal[j]), ((uint64_t)dist[j] << 32) | i);
      p += (uint32_t)__popcll(bal[j]);
    }
  }
  }
}

void launch_scan_single(const Lib &lib, const Workspace &ws, uint32_t qidx, uint64_t t_begin,
                        uint64_t t_end, int cus, hipStream_t s, const LaunchEv &ev) {
  if (t_end <= t_begin) return;
  // A wave per tile up to 256 blocks per CU (then grid-stride): the finer the
  // grid, the shorter the tail; measured 2 % faster over 95.4 M records than
  // 32 blocks per CU, and a resident grid (7 per CU) 5 % slower.
  uint64_t blocks = (t_end - t_begin + 3) / 4;  // 4 waves per block
  const uint64_t maxb = (uint64_t)cus * 256;
  if (blocks > maxb) blocks = maxb;
  launch_k(k_scan_single, dim3((uint32_t)blocks), dim3(256), s, ev, lib, ws, qidx, t_begin, t_end);
}

// ---------------------------------------------------------------------------
// Batched popcount scan: a block takes a 2048-record tile of a query block's
// range, holds 4 records per lane in registers and walks the block's queries
// (staged in LDS).  Per pair: 3 XOR + 6 popcount-accumulate, seeded with
// -(T+1) so that a candidate is exactly a negative sum.
// ---------------------------------------------------------------------------
constexpr int kPopRL = 4;

__global__ __launch_bounds__(256) void k_scan_popcount(Lib lib, Workspace ws, uint32_t nqb,
                                                       const uint64_t *item_off,
                                                       uint64_t tile_lo, uint64_t items) {
  __shared__ uint64_t qw[kPopQBlock][3];  // a, b, c | d << 32
  __shared__ int32_t qseed[kPopQBlock];   // -(T+1)
  __shared__ uint32_t qid[kPopQBlock];
  uint32_t cur_qb = 0xFFFFFFFFu;
  QBlock qb{};
  const uint32_t tid = threadIdx.x;
  for (uint64_t item = blockIdx.x; item < items; item += gridDim.x) {
    uint32_t b = 0;
    while (b + 1 < nqb && item >= item_off[b + 1]) ++b;
    if (b != cur_qb) {
      __syncthreads();
      cur_qb = b;
      qb = ws.qblocks[b];
      for (uint32_t j = tid; j < qb.count; j += blockDim.x) {
        const uint32_t q = ws.perm[qb.first + j];
        qid[j] = q;
        qw[j][0] = ws.qinfo[q].qa;
        qw[j][1] = ws.qinfo[q].qb;
        qw[j][2] = (uint64_t)ws.qinfo[q].qc | ((uint64_t)ws.qinfo[q].qd << 32);
        qseed[j] = -((int32_t)ws.T[q] + 1);
      }
      __syncthreads();
    }
    const RangeSet *rs = ws.rsets + qb.rset;
    const uint64_t tile = item - item_off[b] + min(tile_lo, (uint64_t)qb.tiles);
    uint32_t r = 0;
    while (tile >= rs->tboff[r + 1]) ++r;
    const uint64_t g0 = rs->begin[r] + (tile - rs->tboff[r]) * kBatchTile;
    const uint64_t g1 = min(g0 + (uint64_t)kBatchTile, rs->end[r]);
    for (uint64_t sub = g0; sub < g1; sub += 256 * kPopRL) {
      Rec x[kPopRL];
      bool ok[kPopRL];
#pragma unroll
      for (int u = 0; u < kPopRL; ++u) {
        const uint64_t g = sub + 256 * u + tid;
        ok[u] = g < g1;
        x[u] = load_rec(lib, ok[u] ? g : g0);
      }
      for (uint32_t j = 0; j < qb.count; ++j) {
        const uint64_t qa = qw[j][0], qb2 = qw[j][1], qcd = qw[j][2];
        const int32_t seed = qseed[j];
        int32_t v[kPopRL];
        int32_t any = 0;
#pragma unroll
        for (int u = 0; u < kPopRL; ++u) {
          v[u] = seed + (int32_t)dist4(x[u].a, x[u].b, x[u].c, x[u].d, qa, qb2, (uint32_t)qcd,
                                       (uint32_t)(qcd >> 32));
          any |= v[u];
        }
        if (__ballot(any < 0) == 0) continue;
        const uint32_t q = qid[j];
        const QueryInfo *qi = ws.qinfo + q;
        const uint32_t seg = blockIdx.x % qi->nseg;
        const int32_t T1 = -seed;  // T + 1
#pragma unroll
        for (int u = 0; u < kPopRL; ++u) {
          const uint64_t g = sub + 256 * u + tid;
          const bool hit = ok[u] && v[u] < 0;
          wave_append(hit, ((uint64_t)(uint32_t)(v[u] + T1) << 32) | g, ws, qi, seg);
        }
      }
    }
  }
}

void launch_scan_popcount(const Lib &lib, const Workspace &ws, uint32_t nqb,
                          const uint64_t *item_off, uint64_t tile_lo, uint64_t items, int cus,
                          hipStream_t s, const LaunchEv &ev) {
  if (items == 0) return;
  uint64_t blocks = items;
  const uint64_t maxb = (uint64_t)cus * 8;
  if (blocks > maxb) blocks = maxb;
  launch_k(k_scan_popcount, dim3((uint32_t)blocks), dim3(256), s, ev, lib, ws, nqb, item_off,
           tile_lo, items);
}

// ---------------------------------------------------------------------------
// Select: one block of 1024 threads per query.  A 167-bin histogram of the
// candidates gives D_k and the number m of candidates with d <= D_k.  Up to
// kSortCap candidates are staged in LDS during the histogram pass, so the
// buffer is read from memory once.  m <= kRankCap: each of the m keys is
// ranked directly by counting the smaller ones (the keys (d << 32) | index are
// unique); larger m: a bitonic sort in LDS.
// ---------------------------------------------------------------------------
constexpr uint32_t kRankCap = 1024;

// A slot for every active lane from an LDS counter: one atomic per wave.
__device__ __forceinline__ uint32_t wave_slot(uint32_t *ctr) {
  const uint64_t act = __ballot(1);
  const uint32_t leader = (uint32_t)__ffsll((unsigned long long)act) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(ctr, (uint32_t)__popcll(act));
  base = __shfl(base, (int)leader);
  return base + rank_below(act);
}

__device__ __forceinline__ fps_hit hit_of(uint64_t key) {
  fps_hit h;
  h.index = (uint32_t)key;
  h.distance = (uint32_t)(key >> 32);
  return h;
}

__global__ __launch_bounds__(1024) void k_select(Workspace ws, HostBack hb) {
  __shared__ uint32_t hist[kBins];
  __shared__ uint64_t keys[kSortCap];
  __shared__ uint64_t rk[kRankCap];
  __shared__ uint32_t s_dk, s_fail, s_m, s_ncoll, s_nstage;
  __shared__ uint32_t segn[kSegments + 1];
  __shared__ uint32_t s_total, s_over;
  const uint32_t q = blockIdx.x;
  const QueryInfo *qi = ws.qinfo + q;
  const uint32_t keff = qi->keff;
  const uint32_t tid = threadIdx.x;
  if (keff == 0) {
    if (tid == 0 && hb.count) {
      hb.count[q] = 0;
      hb.flags[q] = 0;
    }
    return;
  }
  for (uint32_t i = tid; i < kBins; i += blockDim.x) hist[i] = 0;
  if (tid == 0) {
    s_ncoll = 0;
    s_nstage = 0;
  }
  const uint32_t n = cand_counts(ws, qi, segn, &s_total, &s_over);
  if (tid == 0) {
    ws.count[q] = n;
    if (hb.count) hb.count[q] = n;
  }
  if (s_over) {
    if (tid == 0) {
      ws.flags[q] |= 1u;
      if (hb.flags) hb.flags[q] = ws.flags[q];
    }
    return;
  }
  const bool staged = n <= kSortCap;
  cand_for_each(ws, qi, segn, [&](uint64_t key) {
    atomicAdd(&hist[(uint32_t)(key >> 32)], 1u);
    if (staged) keys[wave_slot(&s_nstage)] = key;
  });
  __syncthreads();
  if (tid < 64) {
    uint32_t cum;
    const uint32_t dk = wave_kth(hist, (uint32_t)kKeys, keff, &cum);
    if (tid == 0) {
      s_fail = dk == 0xFFFFFFFFu ? 4u : (cum > kSortCap ? 2u : 0u);
      s_dk = dk;
      s_m = cum;
    }
  }
  __syncthreads();
  if (s_fail) {
    if (tid == 0) {
      ws.flags[q] |= s_fail;
      if (hb.flags) hb.flags[q] = ws.flags[q];
    }
    return;
  }
  if (tid == 0 && hb.flags) hb.flags[q] = ws.flags[q];
  const uint32_t dk = s_dk, m = s_m;
  fps_hit *out = (hb.hits ? hb.hits : ws.out) + qi->out_off;
  if (m <= kRankCap) {
    if (staged) {
      for (uint32_t i = tid; i < n; i += blockDim.x) {
        const uint64_t key = keys[i];
        if ((uint32_t)(key >> 32) <= dk) rk[wave_slot(&s_ncoll)] = key;
      }
    } else {
      cand_for_each(ws, qi, segn, [&](uint64_t key) {
        if ((uint32_t)(key >> 32) <= dk) rk[wave_slot(&s_ncoll)] = key;
      });
    }
    __syncthreads();
    if (tid < m) {
      const uint64_t key = rk[tid];
      uint32_t r = 0;
      for (uint32_t j = 0; j < m; ++j) r += rk[j] < key ? 1u : 0u;
      if (r < keff) out[r] = hit_of(key);
    }
    return;
  }
  // m > kRankCap: gather the keys with d <= D_k into keys[] (in place when
  // staged: every thread first takes its share into registers) and sort
  if (staged) {
    constexpr int kPer = kSortCap / 1024;
    uint64_t mine[kPer];
#pragma unroll
    for (int c = 0; c < kPer; ++c) {
      const uint32_t i = tid + 1024u * c;
      mine[c] = i < n ? keys[i] : ~0ull;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kPer; ++c)
      if (tid + 1024u * c < n && (uint32_t)(mine[c] >> 32) <= dk) keys[wave_slot(&s_ncoll)] = mine[c];
  } else {
    cand_for_each(ws, qi, segn, [&](uint64_t key) {
      if ((uint32_t)(key >> 32) <= dk) keys[wave_slot(&s_ncoll)] = key;
    });
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
          const uint64_t a = keys[i], b = keys[ixj];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            keys[i] = b;
            keys[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t i = tid; i < keff; i += blockDim.x) out[i] = hit_of(keys[i]);
}

void launch_select(const Workspace &ws, uint32_t q, const HostBack &hb, hipStream_t s,
                   const LaunchEv &ev) {
  if (q == 0) return;
  launch_k(k_select, dim3(q), dim3(1024), s, ev, ws, hb);
}

// ---------------------------------------------------------------------------
// Exact ordered fallback for one query.  Every wave owns a contiguous chunk of
// the query's virtual range.
//   pass 1: per-wave distance histograms;
//   scan:   per-bin exclusive prefix over waves, and bin totals;
//   pass 2: every record with d <= D_k goes to position
//           cum(d-1) + (records with the same d in earlier waves)
//                    + (records with the same d earlier in this wave),
//           i.e. its rank in (distance, index) order; positions < keff are
//           written.  No sort is needed.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fb_hist(Lib lib, Workspace ws, uint32_t qidx,
                                                 uint64_t neff, uint64_t chunk) {
  __shared__ uint32_t h[4][kBins];
  const QueryInfo *qi = ws.qinfo + qidx;
  const RangeSet *rs = ws.rsets + qi->rset;
  const uint32_t wl = threadIdx.x >> 6, lane = lane_id();
  const uint64_t w = (uint64_t)blockIdx.x * 4 + wl;
  for (uint32_t i = threadIdx.x; i < 4 * kBins; i += blockDim.x) (&h[0][0])[i] = 0;
  __syncthreads();
  const uint64_t v0 = w * chunk, v1 = min(v0 + chunk, neff);
  for (uint64_t v = v0 + lane; v < v1; v += 64) {
    const uint64_t g = v2g(rs, v);
    atomicAdd(&h[wl][dist_rec(load_rec(lib, g), qi)], 1u);
  }
  __syncthreads();
  for (uint32_t b = lane; b < (uint32_t)kBins; b += 64) ws.fb_wave_hist[w * kBins + b] = h[wl][b];
}

__global__ __launch_bounds__(256) void k_fb_scan(Workspace ws) {
  __shared__ uint32_t part[256];
  const uint32_t bin = blockIdx.x, tid = threadIdx.x;
  uint32_t carry = 0;
  for (uint32_t w0 = 0; w0 < (uint32_t)kFbWaves; w0 += 256) {
    const uint32_t x = ws.fb_wave_hist[(uint64_t)(w0 + tid) * kBins + bin];
    part[tid] = x;
    __syncthreads();
    for (uint32_t off = 1; off < 256; off <<= 1) {
      const uint32_t y = tid >= off ? part[tid - off] : 0;
      __syncthreads();
      part[tid] += y;
      __syncthreads();
    }
    ws.fb_wave_off[(uint64_t)(w0 + tid) * kBins + bin] = carry + part[tid] - x;
    carry += part[255];
    __syncthreads();
  }
  if (tid == 0) ws.fb_bin_total[bin] = carry;
}

__global__ __launch_bounds__(256) void k_fb_emit(Lib lib, Workspace ws, uint32_t qidx,
                                                 uint64_t neff, uint64_t chunk) {
  __shared__ uint32_t cumex[kBins];
  __shared__ uint32_t run[4][kBins];
  __shared__ uint32_t s_dk;
  const QueryInfo *qi = ws.qinfo + qidx;
  const RangeSet *rs = ws.rsets + qi->rset;
  const uint32_t keff = qi->keff;
  fps_hit *out = ws.out + qi->out_off;
  const uint32_t wl = threadIdx.x >> 6, lane = lane_id();
  const uint64_t w = (uint64_t)blockIdx.x * 4 + wl;
  for (uint32_t i = threadIdx.x; i < 4 * kBins; i += blockDim.x) (&run[0][0])[i] = 0;
  if (threadIdx.x == 0) {
    uint32_t cum = 0, dk = (uint32_t)kKeys;
    bool found = false;
    for (uint32_t t = 0; t < (uint32_t)kBins; ++t) {
      cumex[t] = cum;
      cum += (t <= (uint32_t)kKeys) ? ws.fb_bin_total[t] : 0;
      if (!found && cum >= keff) {
        dk = t;
        found = true;
      }
    }
    s_dk = dk;
  }
  __syncthreads();
  const uint32_t dk = s_dk;
  const uint64_t v0 = w * chunk, v1 = min(v0 + chunk, neff);
  const uint32_t *woff = ws.fb_wave_off + w * kBins;
  const uint64_t lt = (1ull << lane) - 1ull;
  for (uint64_t step = 0; step < chunk; step += 64) {
    const uint64_t v = v0 + step + lane;
    uint32_t d = 0;
    uint64_t g = 0;
    bool act = false;
    if (v < v1) {
      g = v2g(rs, v);
      d = dist_rec(load_rec(lib, g), qi);
      act = d <= dk;
    }
    uint64_t eq = __ballot(act);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool set = (d >> bit) & 1u;
      const uint64_t bb = __ballot(act && set);
      eq &= set ? bb : ~bb;
    }
    uint32_t pos = 0xFFFFFFFFu;
    if (act) {
      pos = cumex[d] + woff[d] + run[wl][d] + (uint32_t)__popcll(eq & lt);
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

void launch_fallback(const Lib &lib, const Workspace &ws, uint32_t qidx, uint64_t neff,
                     hipStream_t s) {
  uint64_t chunk = (neff + kFbWaves - 1) / kFbWaves;
  chunk = (chunk + 63) & ~(uint64_t)63;
  if (chunk == 0) chunk = 64;
  hipLaunchKernelGGL(k_fb_hist, dim3(kFbBlocks), dim3(256), 0, s, lib, ws, qidx, neff, chunk);
  hipLaunchKernelGGL(k_fb_scan, dim3(kBins), dim3(256), 0, s, ws);
  hipLaunchKernelGGL(k_fb_emit, dim3(kFbBlocks), dim3(256), 0, s, lib, ws, qidx, neff, chunk);
}

}  // namespace fps
