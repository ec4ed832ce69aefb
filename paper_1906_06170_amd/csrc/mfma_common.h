// Work-item and stage bookkeeping shared by the matrix-core kernels.
//
// A block of a matrix-core kernel walks a contiguous run of work items (one
// query block x one batch tile of kBatchTile records) as a stream of stages;
// the records of a stage are held in registers before they are expanded into
// LDS.  The int8 kernel uses stages of kSub records (one record per two
// threads, Regs); the fp4 kernel stages of 256 (one record per thread, Rec1).
// Also here: the scalar-load view of the parameter tables, the LDS hit lists
// and the LDS-only barrier.
#pragma once
#include "cand.h"
#include "fps_internal.h"

namespace fps {

constexpr int kSub = 128;                       // records per LDS stage (int8 kernel)
constexpr int kSubPerTile = kBatchTile / kSub;  // stages per work item (int8 kernel)

// A work item: query block b and the records [t0, t1) of one batch tile.
struct Item {
  uint32_t b;
  uint64_t t0, t1;
};

// A stage: query block b and the records [g0, g1) (at most kSub, maybe none).
struct Stage {
  uint32_t b;
  uint64_t g0, g1;
};

// Read-only parameter tables seen through the constant address space: uniform
// reads of them become scalar loads, which do not wait on (and so do not drain)
// the vector loads of records in flight.
template <class T>
using cptr = const __attribute__((address_space(4))) T *;

template <class T>
__device__ __forceinline__ cptr<T> as_const(const T *p) {
  return (cptr<T>)p;
}

__device__ __forceinline__ Item describe(const Workspace &ws, const uint64_t *item_off,
                                         uint32_t nqb, uint64_t tile_lo, uint64_t item) {
  const cptr<uint64_t> io = as_const(item_off);
  uint32_t b = 0;
  while (b + 1 < nqb && item >= io[b + 1]) ++b;
  const cptr<QBlock> qb = as_const(ws.qblocks) + b;
  const cptr<RangeSet> rs = as_const(ws.rsets) + qb->rset;
  const uint64_t tile = item - io[b] + min(tile_lo, (uint64_t)qb->tiles);
  uint32_t r = 0;
  while (tile >= rs->tboff[r + 1]) ++r;
  Item it;
  it.b = b;
  it.t0 = rs->begin[r] + (tile - rs->tboff[r]) * kBatchTile;
  it.t1 = min(it.t0 + (uint64_t)kBatchTile, rs->end[r]);
  return it;
}

template <int SUB = kSub>
__device__ __forceinline__ Stage stage_of(const Item &it, uint32_t sub) {
  Stage st;
  st.b = it.b;
  st.g0 = min(it.t0 + (uint64_t)sub * SUB, it.t1);
  st.g1 = min(st.g0 + (uint64_t)SUB, it.t1);
  return st;
}

// Records of a stage held in registers: thread tid loads record tid >> 1.
struct Regs {
  uint64_t a, b;
  uint32_t c, d;
  uint32_t ok, pad;
};

// One record per thread (stages of 256 records): the raw words, 6 registers.
struct Rec1 {
  uint64_t a, b;
  uint32_t c, d;
};

__device__ __forceinline__ Rec1 load_rec1(const Lib &lib, const Stage &st, uint32_t tid) {
  const uint64_t g = st.g0 + tid;
  const uint64_t gs = g < st.g1 ? g : 0;
  Rec1 R;
  R.a = lib.a[gs];
  R.b = lib.b[gs];
  R.c = lib.c[gs];
  R.d = (uint32_t)lib.d[gs];
  return R;
}

// ---------------------------------------------------------------------------
// Hits of the matrix-core kernels, gathered per wave in LDS and written out in
// batches.  Decoding a result tile then touches LDS only; a flush (list nearly
// full, a new query block, the end of the kernel) reserves each row's hits
// with one device atomic -- one per row, all in flight together -- and stores
// the keys.  Global loads and returning atomics wait on the same counter as
// the record loads in flight, so doing them per tile would stall the record
// prefetch at every hit.
// ---------------------------------------------------------------------------
struct RowInfo {  // a query row's candidate-buffer fields (see QueryInfo)
  uint64_t cand_off;
  uint32_t ctr_off, nseg, segcap, spillcap;
  uint32_t T1;  // T + 1: the distance of a pair is its product u plus T1
  uint32_t pad;
};

constexpr uint32_t kHitCap = 256;  // list entries per wave

// Zeroes the per-row counts of a wave (before its first flush).
template <int ROWS>
__device__ __forceinline__ void hits_init(uint32_t lane, uint32_t *cnt) {
  for (uint32_t lr = lane; lr < (uint32_t)ROWS; lr += 64) cnt[lr] = 0;
}

struct HitBuf {
  RowInfo *row;    // the wave's rows
  uint32_t *cnt;   // per row: entries of the list being flushed
  uint32_t *base;  // per row: reservation of the flush
  uint32_t *sbase;
  uint64_t *list;  // (row << 40) | ((T + 1 - d) << 32) | record index
  uint32_t n;      // entries (wave-uniform)
};

// A list entry: local row lr, product u = d - T - 1 (negative), record g.
__device__ __forceinline__ uint64_t hit_entry(uint32_t lr, int32_t u, uint32_t g) {
  return ((uint64_t)lr << 40) | ((uint64_t)(uint32_t)(-u) << 32) | g;
}

// Waits for this wave's LDS operations; the clobber keeps the compiler from
// moving memory accesses across.  The lanes of a wave run in lockstep, so the
// wave's later LDS reads see what its earlier LDS writes and atomics left.
__device__ __forceinline__ void lds_wave_fence() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// Loads the RowInfo of rows row0 .. row0 + ROWS - 1 of query block qb.
template <int ROWS>
__device__ __forceinline__ void hits_rows(const Workspace &ws, const QBlock &qb, uint32_t row0,
                                          uint32_t lane, HitBuf &hb) {
#pragma unroll
  for (int k = 0; k < (ROWS + 63) / 64; ++k) {
    const uint32_t lr = lane + 64u * k;
    if (lr < (uint32_t)ROWS) {
      RowInfo ri{0, 0, 1, 0, 0, 0, 0};
      const uint32_t row = row0 + lr;
      if (row < qb.count) {
        const uint32_t q = ws.perm[qb.first + row];
        const QueryInfo *qi = ws.qinfo + q;
        ri.cand_off = qi->cand_off;
        ri.ctr_off = qi->ctr_off;
        ri.nseg = qi->nseg;
        ri.segcap = qi->segcap;
        ri.spillcap = qi->spillcap;
        ri.T1 = ws.T[q] + 1u;
      }
      hb.row[lr] = ri;
      hb.cnt[lr] = 0;
    }
  }
}

// Moves the list to the candidate buffers: ranks within each row from LDS
// atomics on the row counts, one reservation per row with entries (all in
// flight together), then the stores.  Only rows with entries have their
// RowInfo read (a hit needs a row of the current query block), so an empty
// list reads no RowInfo at all.
template <int ROWS>
__device__ __forceinline__ void hits_flush(const Workspace &ws, uint32_t lane, HitBuf &hb) {
  if (hb.n == 0) return;
  constexpr int kPer = (int)kHitCap / 64;
  uint64_t e[kPer];
  uint32_t rank[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const uint32_t i = lane + 64u * j;
    e[j] = 0;
    rank[j] = 0;
    if (i < hb.n) {
      e[j] = hb.list[i];
      rank[j] = atomicAdd(hb.cnt + (uint32_t)(e[j] >> 40), 1u);
    }
  }
  lds_wave_fence();
#pragma unroll
  for (int k = 0; k < (ROWS + 63) / 64; ++k) {
    const uint32_t lr = lane + 64u * k;
    if (lr < (uint32_t)ROWS) {
      const uint32_t c = hb.cnt[lr];
      if (c) {
        const RowInfo *ri = hb.row + lr;
        const Resv rv = cand_reserve(ws, ri, blockIdx.x % ri->nseg, c);
        hb.base[lr] = rv.base;
        hb.sbase[lr] = rv.sbase;
        hb.cnt[lr] = 0;
      }
    }
  }
  lds_wave_fence();
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const uint32_t i = lane + 64u * j;
    if (i < hb.n) {
      const uint32_t lr = (uint32_t)(e[j] >> 40);
      const uint32_t d = hb.row[lr].T1 - ((uint32_t)(e[j] >> 32) & 0xFFu);
      const RowInfo *ri = hb.row + lr;
      const Resv rv{hb.base[lr], hb.sbase[lr]};
      cand_put(ws, ri, blockIdx.x % ri->nseg, rv, rank[j], ((uint64_t)d << 32) | (uint32_t)e[j]);
    }
  }
  hb.n = 0;
}

// Block barrier for LDS traffic: this wave's LDS operations complete, then the
// barrier.  __syncthreads() would also wait for every outstanding global load
// (the workgroup fence waits on the one counter that loads and stores share),
// which drains the record prefetch of the stage stream at every stage.  The
// stage loop exchanges data through LDS only; the clobber keeps the compiler
// from moving memory accesses across the barrier.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ Regs load_stage(const Lib &lib, const Stage &st, uint32_t tid) {
  Regs R;
  const uint64_t g = st.g0 + (tid >> 1);
  R.ok = g < st.g1 ? 1u : 0u;
  R.pad = 0;
  const uint64_t gs = R.ok ? g : 0;
  R.a = lib.a[gs];
  R.b = lib.b[gs];
  R.c = lib.c[gs];
  R.d = (uint32_t)lib.d[gs];
  return R;
}

}  // namespace fps
