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
