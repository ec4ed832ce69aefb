// Internal declarations of the MI355X fingerprint top-k engine: device-side
// parameter blocks and the host launchers of the kernels.
//
// Library layout in HBM: four word-major arrays, 21 bytes per record (the 166
// keys need 20.75), Np = n rounded up to a multiple of 4096:
//   a[Np] uint64: keys 1..63 at bits 1..63, key 160 at bit 0
//   b[Np] uint64: keys 64..127 at bits 0..63
//   c[Np] uint32: keys 128..159 at bits 0..31
//   d[Np] uint8 : keys 161..166 at bits 0..5
// This only relabels key positions, so the number of differing keys (the
// distance) is the popcount of a^a' + b^b' + c^c' + d^d'.  Queries are relabeled
// the same way on the host.  Records [n, Np) are zero and never reported.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/fps.h"

namespace fps {

constexpr int kKeys = 166;
constexpr int kBins = 168;          // distances 0..166, padded
constexpr uint64_t kRowAlign = 4096;
constexpr uint64_t kBytesPerRecord = 21;
constexpr uint32_t kSortCap = 8192; // candidates with d <= D_k sorted in LDS by one block
constexpr int kFbBlocks = 2048;     // fallback grid (blocks of 256 threads)
constexpr int kFbWaves = kFbBlocks * 4;

constexpr int kScanTile = 512;      // records per wave iteration of the single-query scan
constexpr int kBatchTile = 2048;    // records per work item of the batched kernels
constexpr int kBoundChunk = 1024;   // least records per block of the bound kernel
constexpr int kBoundBlocks = 128;   // most blocks per query block of the bound kernel
constexpr int kBoundGrid = 1024;    // bound blocks aimed at once query blocks fill the GPU
constexpr int kHistCopies = 8;      // bound histograms are spread over 8 copies per query
constexpr uint64_t kDefaultBoundSample = 1ull << 16;  // records of the bound sample
// One scan phase when the first bound is expected to admit at most this many
// records per query (keff * neff / sample); more phases otherwise.
constexpr uint64_t kSinglePhaseAppends = 8192;
constexpr uint64_t kDefaultPhaseA = 0;  // first phase length in records (0 = from the schedule)
constexpr int kMaxPhases = 12;          // scan phases (the bound is refined between phases)
constexpr uint32_t kSegments = 64;      // candidate segments of a query in a small batch
constexpr uint32_t kSegQueries = 16;    // batches up to this size use kSegments segments
constexpr uint32_t kCtrStride = 32;     // counters of a segmented query, 128 bytes apart

// A union of record ranges (the strides one mask selects), in ascending order,
// adjacent strides merged.  Virtual index v in [0, neff) enumerates its records
// in ascending global order.
struct RangeSet {
  uint32_t nranges;
  uint32_t mask;
  uint64_t neff;
  uint64_t begin[FPS_MAX_STRIDES];
  uint64_t end[FPS_MAX_STRIDES];
  uint64_t voff[FPS_MAX_STRIDES + 1];  // virtual index of begin[r]
  uint64_t t1off[FPS_MAX_STRIDES + 1]; // first single-scan tile of range r (512-record tiles)
  uint64_t tboff[FPS_MAX_STRIDES + 1]; // first batch tile of range r (kBatchTile records)
};

// Per-query parameters, uploaded with every call (query in the library layout).
struct QueryInfo {
  uint64_t qa, qb;
  uint32_t qc, qd;
  uint32_t keff;      // min(k, neff)
  uint32_t rset;      // RangeSet index
  uint64_t cand_off;  // first candidate slot
  uint32_t cap;       // candidate slots: nseg * segcap (+ spillcap when nseg > 1)
  uint32_t popc;      // keys set in the query
  uint64_t out_off;   // first output hit
  uint64_t sample;    // records used for the bound: min(sample_records, neff)
  uint32_t nseg;      // candidate segments (1 or kSegments)
  uint32_t segcap;    // slots per segment
  uint32_t spillcap;  // slots of the spill area (nseg > 1)
  uint32_t ctr_off;   // first counter in Workspace::ctr (segment s at + s * kCtrStride)
};

// A block of queries sharing one RangeSet (indices into the permutation).
struct QBlock {
  uint32_t first;  // position in perm[]
  uint32_t count;  // queries in the block
  uint32_t rset;
  uint32_t tiles;  // batch tiles of the block's range
};

struct Workspace {
  RangeSet *rsets;
  QueryInfo *qinfo;
  uint32_t *perm;
  QBlock *qblocks;      // for the batched kernels
  uint64_t *qb_item;    // per phase: nqb + 1 prefix of work items (tiles of the phase)
  QBlock *bblocks;      // for the bound kernel (<= kBoundQBlock queries each)
  uint32_t *bdone;      // per bound block: finished chunk blocks
  uint32_t *T;          // per-query distance bound (int32; -1 = no candidate wanted)
  uint32_t *ctr;        // candidate counters (see QueryInfo::ctr_off)
  uint32_t *count;      // per-query valid candidates, written by select (statistics)
  uint32_t *flags;      // per-query: 1 overflow, 2 too many ties for LDS sort, 4 bound failed
  uint32_t *hist;       // per query: kHistCopies x kBins histogram of the bound sample
  uint64_t *cand;       // candidates: (distance << 32) | index
  fps_hit *out;         // results, query q at qinfo[q].out_off
  uint32_t *fb_wave_hist; // fallback: kFbWaves x kBins
  uint32_t *fb_wave_off;  // fallback: kFbWaves x kBins
  uint32_t *fb_bin_total; // fallback: kBins
};

// Library-layout words of a fingerprint given as three words with key j at bit
// (j & 63) of word (j >> 6): key 160 moves into the always-zero bit 0 of a, keys
// 161..166 go to d.
__host__ __device__ inline void relabel3(uint64_t w0, uint64_t w1, uint64_t w2, uint64_t *a,
                                         uint64_t *b, uint32_t *c, uint32_t *d) {
  *a = w0 | ((w2 >> 32) & 1ull);
  *b = w1;
  *c = (uint32_t)w2;
  *d = (uint32_t)((w2 >> 33) & 0x3Full);
}

inline void relabel(const uint64_t *w, uint64_t *a, uint64_t *b, uint32_t *c, uint32_t *d) {
  relabel3(w[0], w[1], w[2], a, b, c, d);
}

struct Lib {
  const uint64_t *a, *b;
  const uint32_t *c;
  const uint8_t *d;
  uint64_t n, np;
};

// Timing events of a launch.  They are stamped by the kernel dispatch itself
// (no marker packets between kernels); both null: an untimed launch.
struct LaunchEv {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};

template <typename F, typename... Args>
inline void launch_k(F kernel, dim3 grid, dim3 block, hipStream_t s, const LaunchEv &ev,
                     Args... args) {
  hipExtLaunchKernelGGL(kernel, grid, block, 0u, s, ev.start, ev.stop, 0u, args...);
}

// ---- launchers (kernels.hip) ----
void launch_prep(const Workspace &ws, uint32_t q, uint32_t nbblocks, uint32_t nctr,
                 hipStream_t s, const LaunchEv &ev);
// A parameter block small enough to travel as a kernel argument: the prep
// kernel copies it to dst (the workspace), which saves a host-to-device copy.
constexpr size_t kInlineParams = 3072;
struct InlineParams {
  uint64_t bytes;
  uint64_t w[kInlineParams / 8];
};
void launch_prep_inline(const Workspace &ws, uint32_t q, uint32_t nbblocks, uint32_t nctr,
                        uint8_t *dst, const InlineParams &p, hipStream_t s,
                        const LaunchEv &ev);
void launch_bound(const Lib &lib, const Workspace &ws, uint32_t nbblocks, uint64_t max_sample,
                  hipStream_t s);
void launch_refine(const Workspace &ws, uint32_t q, hipStream_t s);
void launch_scan_single(const Lib &lib, const Workspace &ws, uint32_t qidx, uint64_t t_begin,
                        uint64_t t_end, int cus, hipStream_t s, const LaunchEv &ev);
// Batched scans: work items are the tiles [tile_lo, tile_hi) of every query
// block's range (clamped to its tile count); item_off is the phase's nqb + 1
// prefix of items per query block.
void launch_scan_popcount(const Lib &lib, const Workspace &ws, uint32_t nqb,
                          const uint64_t *item_off, uint64_t tile_lo, uint64_t items, int cus,
                          hipStream_t s, const LaunchEv &ev);
// Where select also writes the per-query counts and flags and the hits: the
// device addresses of pinned host buffers (all null: the workspace only).
struct HostBack {
  uint32_t *count;
  uint32_t *flags;
  fps_hit *hits;
};
void launch_select(const Workspace &ws, uint32_t q, const HostBack &hb, hipStream_t s,
                   const LaunchEv &ev);
void launch_fallback(const Lib &lib, const Workspace &ws, uint32_t qidx, uint64_t neff,
                     hipStream_t s);
// ---- launchers (mfma.hip) ----
void launch_scan_mfma_i8(const Lib &lib, const Workspace &ws, uint32_t nqb,
                         const uint64_t *item_off, uint64_t tile_lo, uint64_t items, int cus,
                         int variant, hipStream_t s, const LaunchEv &ev);
int mfma_variants();
uint32_t mfma_qblock(int variant);
// ---- launchers (mfma_f4.hip) ----
void launch_scan_mfma_f4(const Lib &lib, const Workspace &ws, uint32_t nqb,
                         const uint64_t *item_off, uint64_t tile_lo, uint64_t items, int cus,
                         int variant, hipStream_t s, const LaunchEv &ev);
int mfma_f4_variants();
uint32_t mfma_f4_qblock(int variant);

constexpr int kPopQBlock = 128;   // queries per block of the popcount kernel
constexpr int kBoundQBlock = 32;  // queries per block of the bound kernel

}  // namespace fps
