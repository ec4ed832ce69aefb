// Work-item and stage bookkeeping shared by the matrix-core kernels.
//
// A block of a matrix-core kernel walks a contiguous run of work items (one
// query block x one batch tile of kBatchTile records) as a stream of stages of
// kSub records; the records of a stage are held in registers (one record per
// two threads) before they are expanded into LDS.
#pragma once
#include "cand.h"
#include "fps_internal.h"

namespace fps {

constexpr int kSub = 128;                       // records per LDS stage
constexpr int kSubPerTile = kBatchTile / kSub;  // stages per work item

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

__device__ __forceinline__ Item describe(const Workspace &ws, const uint64_t *item_off,
                                         uint32_t nqb, uint64_t tile_lo, uint64_t item) {
  uint32_t b = 0;
  while (b + 1 < nqb && item >= item_off[b + 1]) ++b;
  const QBlock qb = ws.qblocks[b];
  const RangeSet *rs = ws.rsets + qb.rset;
  const uint64_t tile = item - item_off[b] + min(tile_lo, (uint64_t)qb.tiles);
  uint32_t r = 0;
  while (tile >= rs->tboff[r + 1]) ++r;
  Item it;
  it.b = b;
  it.t0 = rs->begin[r] + (tile - rs->tboff[r]) * kBatchTile;
  it.t1 = min(it.t0 + (uint64_t)kBatchTile, rs->end[r]);
  return it;
}

__device__ __forceinline__ Stage stage_of(const Item &it, uint32_t sub) {
  Stage st;
  st.b = it.b;
  st.g0 = min(it.t0 + (uint64_t)sub * kSub, it.t1);
  st.g1 = min(st.g0 + (uint64_t)kSub, it.t1);
  return st;
}

// Records of a stage held in registers: thread tid loads record tid >> 1.
struct Regs {
  uint64_t a, b;
  uint32_t c, d;
  uint32_t ok, pad;
};

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
