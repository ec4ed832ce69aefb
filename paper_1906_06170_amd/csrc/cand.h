// Candidate buffers: appending (scan kernels) and reading (refine, select).
//
// A query's buffer is nseg segments of segcap slots, each with its own
// counter on its own 128-byte line, followed -- when nseg > 1 -- by a spill
// area of spillcap slots with one more counter.  A scan wave appends to one
// segment (chosen from its wave or block index); appends that do not fit go to
// the spill area.  Device-wide atomics on one address are serialized, so a
// single-query scan over ~10^8 records with one counter pays for every append;
// with 64 counters they proceed in parallel.  Queries of large batches use one
// segment (their appends are already spread over the batch's counters).
//
// Counters count every append, also past capacity.  A buffer has overflowed
// when nseg == 1 and its counter exceeds segcap, or nseg > 1 and the spill
// counter exceeds spillcap; the query is then answered by the exact fallback.
#pragma once

#include "fps_internal.h"

namespace fps {

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63; }

// Number of set bits of mask below this lane.
__device__ __forceinline__ uint32_t rank_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

struct Resv {
  uint32_t base;   // first position in the segment
  uint32_t sbase;  // first position in the spill area (for the part past segcap)
};

// The candidate-buffer fields of a query: QueryInfo, or a copy of those fields
// (any type with cand_off, ctr_off, nseg, segcap, spillcap).
template <class QI>
__device__ __forceinline__ uint32_t *seg_counter(const Workspace &ws, const QI *qi, uint32_t s) {
  return ws.ctr + qi->ctr_off + s * kCtrStride;
}

// Reserves n slots in segment seg (one lane calls this for its group).
template <class QI>
__device__ __forceinline__ Resv cand_reserve(const Workspace &ws, const QI *qi, uint32_t seg,
                                             uint32_t n) {
  Resv r;
  r.base = atomicAdd(seg_counter(ws, qi, seg), n);
  r.sbase = 0;
  const uint32_t segcap = qi->segcap;
  if (qi->nseg > 1 && r.base + n > segcap) {
    const uint32_t fit = r.base < segcap ? segcap - r.base : 0u;
    r.sbase = atomicAdd(seg_counter(ws, qi, qi->nseg), n - fit);
  }
  return r;
}

// Stores the p-th key of a reservation.
template <class QI>
__device__ __forceinline__ void cand_put(const Workspace &ws, const QI *qi, uint32_t seg,
                                         const Resv &r, uint32_t p, uint64_t key) {
  const uint32_t segcap = qi->segcap;
  const uint32_t pos = r.base + p;
  if (pos < segcap) {
    ws.cand[qi->cand_off + (uint64_t)seg * segcap + pos] = key;
    return;
  }
  if (qi->nseg > 1) {
    const uint32_t fit = r.base < segcap ? segcap - r.base : 0u;
    const uint32_t sp = r.sbase + (p - fit);
    if (sp < qi->spillcap) ws.cand[qi->cand_off + (uint64_t)qi->nseg * segcap + sp] = key;
  }
}

// Appends key for every lane of the wave with hit set: one reservation.
__device__ __forceinline__ void wave_append(bool hit, uint64_t key, const Workspace &ws,
                                            const QueryInfo *qi, uint32_t seg) {
  const uint64_t bal = __ballot(hit);
  if (bal == 0) return;
  const uint32_t lane = lane_id();
  const uint32_t leader = (uint32_t)__ffsll((unsigned long long)bal) - 1;
  Resv r{0, 0};
  if (lane == leader) r = cand_reserve(ws, qi, seg, (uint32_t)__popcll(bal));
  r.base = __shfl(r.base, (int)leader);
  r.sbase = __shfl(r.sbase, (int)leader);
  if (hit) cand_put(ws, qi, seg, r, rank_below(bal), key);
}

// Valid slots per segment (m[s], s < nseg) and of the spill area (m[nseg]),
// staged in LDS by the whole block.  Returns the number of valid candidates;
// *s_over (LDS) becomes nonzero when the buffer overflowed.  Both barriers are
// block-wide: every thread of the block calls this.
__device__ __forceinline__ uint32_t cand_counts(const Workspace &ws, const QueryInfo *qi,
                                                uint32_t *m, uint32_t *s_total,
                                                uint32_t *s_over) {
  const uint32_t nseg = qi->nseg, tid = threadIdx.x;
  if (tid == 0) {
    *s_total = 0;
    *s_over = 0;
  }
  __syncthreads();
  const uint32_t nc = nseg > 1 ? nseg + 1 : 1u;
  for (uint32_t s = tid; s < nc; s += blockDim.x) {
    const uint32_t c = *seg_counter(ws, qi, s);
    const uint32_t cap = nseg == 1 ? qi->segcap : (s < nseg ? qi->segcap : qi->spillcap);
    const bool over = (nseg == 1 || s == nseg) && c > cap;
    m[s] = c < cap ? c : cap;
    if (over) atomicOr(s_over, 1u);
    atomicAdd(s_total, c < cap ? c : cap);
  }
  __syncthreads();
  return *s_total;
}

// Calls f(key) for every valid candidate; the block's threads share the work.
// One segment: all threads stride over it, four keys per thread at a time.
// Several: wave w takes segments w, w + waves, ... (the spill area is segment
// nseg), four at a time.  The four loads are issued without branches (a lane
// with nothing to read reads slot 0, which every buffer of a query with
// keff > 0 has), so that they are in flight together: under a branch each, the
// compiler waited for every load before issuing the next.  Callers handle
// keff == 0 before calling this.  DIST: only the distance (the key's high
// word) is read and f gets it as (d << 32) -- half the bytes, and no load
// whose unused low half the register allocator reuses (which made it wait for
// the load).
template <bool DIST = false, class F>
__device__ __forceinline__ void cand_for_each(const Workspace &ws, const QueryInfo *qi,
                                              const uint32_t *m, F f) {
  const uint32_t nseg = qi->nseg, tid = threadIdx.x;
  const uint64_t *cand = ws.cand + qi->cand_off;
  // slot i of the buffer: the whole key, or (DIST) its distance word
  auto get = [&](uint64_t i) -> uint64_t {
    if constexpr (DIST)
      return (uint64_t)reinterpret_cast<const uint32_t *>(cand)[2 * i + 1] << 32;
    else
      return cand[i];
  };
  if (nseg == 1) {
    const uint32_t n = m[0], nt = blockDim.x;
    for (uint32_t i0 = tid; i0 < n; i0 += 4 * nt) {
      uint64_t key[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t i = i0 + j * nt;
        key[j] = get(i < n ? i : 0u);
      }
      __builtin_amdgcn_sched_barrier(0);  // all four loads go out first
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (i0 + j * nt < n) f(key[j]);
    }
    return;
  }
  const uint32_t wv = tid >> 6, nw = blockDim.x >> 6, lane = tid & 63u;
  const uint32_t segcap = qi->segcap;
  for (uint32_t s0 = wv; s0 <= nseg; s0 += 4 * nw) {
    uint32_t c[4];
    uint64_t key[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t s = s0 + j * nw;
      c[j] = s <= nseg ? m[s] : 0u;
      key[j] = get(lane < c[j] ? (uint64_t)s * segcap + lane : 0ull);
    }
    __builtin_amdgcn_sched_barrier(0);  // all four loads go out first
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (lane < c[j]) f(key[j]);
#pragma unroll 1
    for (int j = 0; j < 4; ++j) {
      const uint64_t p = (uint64_t)(s0 + j * nw) * segcap;
      for (uint32_t i = lane + 64; i < c[j]; i += 64) f(get(p + i));
    }
  }
}

// k-th smallest from a distance histogram: the smallest t <= tmax whose
// cumulative count reaches keff (0xFFFFFFFF if none), and that cumulative
// count in *cum.  Called by all 64 lanes of one wave; h has kBins entries.
// Lane l sums bins 3l .. 3l+2; a prefix sum over the lanes finds the lane
// whose bins cross keff.
__device__ __forceinline__ uint32_t wave_kth(const uint32_t *h, uint32_t tmax, uint32_t keff,
                                             uint32_t *cum) {
  const uint32_t lane = lane_id(), t0 = 3 * lane;
  const uint32_t v0 = t0 <= tmax && t0 < (uint32_t)kBins ? h[t0] : 0u;
  const uint32_t v1 = t0 + 1 <= tmax && t0 + 1 < (uint32_t)kBins ? h[t0 + 1] : 0u;
  const uint32_t v2 = t0 + 2 <= tmax && t0 + 2 < (uint32_t)kBins ? h[t0 + 2] : 0u;
  const uint32_t own = v0 + v1 + v2;
  uint32_t incl = own;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t x = __shfl_up(incl, o);
    if (lane >= (uint32_t)o) incl += x;
  }
  const uint64_t bal = __ballot(incl >= keff);
  if (bal == 0) {
    *cum = __shfl(incl, 63);
    return 0xFFFFFFFFu;
  }
  const uint32_t L = (uint32_t)__ffsll((unsigned long long)bal) - 1;
  const uint32_t excl = incl - own;
  uint32_t t = t0 + 2, c = incl;
  if (excl + v0 >= keff) {
    t = t0;
    c = excl + v0;
  } else if (excl + v0 + v1 >= keff) {
    t = t0 + 1;
    c = excl + v0 + v1;
  }
  *cum = __shfl(c, (int)L);
  return __shfl(t, (int)L);
}

}  // namespace fps
