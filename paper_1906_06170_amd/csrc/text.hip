// The library file and the query box on the GPU side of the C ABI.
//
// Fig. 3 step 1 builds the matrix A and the CID column from the library file F,
// which holds one line of MACCS text per molecule (Abstract).  The text is
// parsed where it will be searched: the caller places the file's bytes in HBM,
// and four kernels turn them into the packed library arrays and a column of
// ids:
//   1. count: one wave per 16 KiB chunk counts its '\n' bytes (a carry-free
//      byte compare on 32-bit words);
//   2. tiles, scan: a two-level prefix of those counts gives the number of the
//      first line starting in each chunk, and the record count;
//   3. parse: one block per chunk stages the chunk and the 256 bytes after it
//      in LDS, with the positions of its newlines.  Lane j parses the j-th
//      line starting in the chunk: the id digits, the separator run, then the
//      key characters four at a time (one 32-bit LDS read and a byte funnel
//      shift each): a carry-free byte test finds the end of the field and a
//      multiply gathers the four low bits into a nibble of the fingerprint.
//      Consecutive lanes hold consecutive records, so the stores coalesce.
// A malformed line does not stop the kernel: the smallest (line, problem)
// pair is kept with an atomic minimum and reported by the host.
//
// Line format (the paper prints none; this is the reading taken):
//   <id> <separator> <keys> [blanks] '\n'
//   id: 1..19 decimal digits; separator: one or more of ' ' '\t' ',';
//   keys: 167 characters '0'/'1' for positions 0..166 (position 0 holds no
//   key and must be '0') or 166 characters for keys 1..166; blanks: ' ' '\t'
//   '\r'; at most 255 characters before the '\n'; the last line may lack its
//   '\n'.  Problems, checked in this order: 1 line too long, 2 id missing or
//   longer than 19 digits, 3 no separator, 4 keys not 166 or 167 characters,
//   5 position 0 set, 6 other characters after the keys.
//
// The query box of Fig. 1 (Fig. 3 step 2) is parsed on the host: a query is a
// few hundred bytes.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "cand.h"
#include "fps_internal.h"
#include "runtime.h"

namespace fps {

constexpr uint32_t kTextChunk = 16384;  // bytes per wave of the count kernel, per block of parse
constexpr uint32_t kOverhang = 256;     // bytes past its chunk a line starting in it may use
constexpr uint32_t kLineMax = 255;      // characters of a line before its '\n'
constexpr uint32_t kIdDigits = 19;      // every 19-digit id fits in 64 bits

__constant__ uint64_t kPow10u[10] = {1ull, 10ull, 100ull, 1000ull, 10000ull, 100000ull,
                                     1000000ull, 10000000ull, 100000000ull, 1000000000ull};
constexpr uint32_t kPrefixTile = 4096;    // chunk counts per block of the prefix kernels

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Bytes of a 32-bit word equal to '\n', as a mask of their top bits.  t has a
// zero byte exactly where x has '\n'; adding 0x7F to the low seven bits of a
// byte carries into its top bit iff those bits are not all zero, and the
// byte's own top bit is ORed in, so the top bit of a byte of nz is set iff
// that byte of t is nonzero.  No carry crosses a byte boundary: exact.
__device__ __forceinline__ uint32_t nl_bytes(uint32_t x) {
  const uint32_t t = x ^ 0x0A0A0A0Au;
  const uint32_t nz = ((t & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | t;
  return ~nz & 0x80808080u;
}

__device__ __forceinline__ uint32_t nl_count(uint32_t x) { return (uint32_t)__popc(nl_bytes(x)); }

// 16 bytes of the text at p (p a multiple of 16); bytes past the end are 0.
__device__ __forceinline__ u32x4 load16(const uint8_t *text, uint64_t bytes, uint64_t p) {
  if (p + 16 <= bytes) return __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(text + p));
  u32x4 v = {0u, 0u, 0u, 0u};
  for (int b = 0; b < 16; ++b)
    if (p + b < bytes) v[b >> 2] |= (uint32_t)text[p + b] << (8 * (b & 3));
  return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Newlines per 16 KiB chunk: one wave per chunk, every load instruction of the
// wave reading 1 KiB of contiguous text.
__global__ __launch_bounds__(256) void k_text_count(const uint8_t *text, uint64_t bytes,
                                                    uint32_t nchunks, uint32_t *counts) {
  const uint32_t chunk = blockIdx.x * 4 + (threadIdx.x >> 6), lane = lane_id();
  if (chunk >= nchunks) return;
  const uint64_t base = (uint64_t)chunk * kTextChunk;
  uint32_t c = 0;
#pragma unroll 4
  for (uint32_t i = 0; i < kTextChunk / 1024; ++i) {
    const u32x4 v = load16(text, bytes, base + 1024u * i + 16u * lane);
    c += nl_count(v.x) + nl_count(v.y) + nl_count(v.z) + nl_count(v.w);
  }
  c = wave_sum(c);
  if (lane == 0) counts[chunk] = c;
}

// Prefix of the chunk counts in two levels: sums of tiles of 4096 chunks,
// then every tile scans its chunks from the sum of the tiles before it.
__global__ __launch_bounds__(256) void k_text_tiles(const uint32_t *counts, uint32_t nchunks,
                                                    uint64_t *tile_sum) {
  __shared__ uint32_t part[4];
  const uint32_t tid = threadIdx.x;
  const uint64_t c0 = (uint64_t)blockIdx.x * kPrefixTile + 16u * tid;
  uint32_t s = 0;
  for (uint32_t i = 0; i < 16; ++i)
    if (c0 + i < nchunks) s += counts[c0 + i];
  s = wave_sum(s);
  if (lane_id() == 0) part[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) tile_sum[blockIdx.x] = (uint64_t)part[0] + part[1] + part[2] + part[3];
}

// out[c] = newlines before chunk c; out[nchunks] = newlines of the text;
// out[nchunks + 1] = records (a text not ending in '\n' has one more line).
__global__ __launch_bounds__(256) void k_text_scan(const uint8_t *text, uint64_t bytes,
                                                   const uint32_t *counts, uint32_t nchunks,
                                                   const uint64_t *tile_sum, uint32_t ntiles,
                                                   uint64_t *out) {
  __shared__ uint64_t part[4];
  __shared__ uint32_t wtot[4];
  const uint32_t tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
  // sum of the tiles before this one
  uint64_t before = 0;
  for (uint32_t t = tid; t < blockIdx.x; t += 256) before += tile_sum[t];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) before += __shfl_xor(before, o);
  if (lane == 0) part[wv] = before;
  // this thread's 16 chunks, then an exclusive prefix over the block
  const uint64_t c0 = (uint64_t)blockIdx.x * kPrefixTile + 16u * tid;
  uint32_t v[16];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    v[i] = c0 + i < nchunks ? counts[c0 + i] : 0u;
    s += v[i];
  }
  uint32_t incl = s;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off);
    if ((int)lane >= off) incl += y;
  }
  if (lane == 63) wtot[wv] = incl;
  __syncthreads();
  uint64_t run = part[0] + part[1] + part[2] + part[3] + (incl - s);
  for (uint32_t w = 0; w < wv; ++w) run += wtot[w];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (c0 + i < nchunks) out[c0 + i] = run;
    run += v[i];
  }
  if (blockIdx.x == ntiles - 1 && tid == 255) {
    out[nchunks] = run;
    out[nchunks + 1] = run + ((bytes > 0 && text[bytes - 1] != '\n') ? 1u : 0u);
  }
}

struct TextOut {
  uint64_t *a, *b;
  uint32_t *c;
  uint8_t *d;
  uint64_t *ids;  // may be null
  uint64_t n;
  unsigned long long *err;  // (line << 8 | problem) minimum; ~0 when every line is well formed
};

constexpr uint32_t kParseThreads = 128;  // one lane per line, two waves per chunk
// Lines parsed per chunk.  A well-formed line and its '\n' take at least 169
// bytes, so at most 97 well-formed lines start in a 16 KiB chunk (98 in the
// first, whose first line starts at byte 0): a chunk in which more than 128
// lines start has a malformed line among its first 128, and that is the first
// malformed line of the chunk.  Only the first 128 lines are parsed; the load
// fails anyway.
constexpr uint32_t kChunkLines = 128;

__device__ __forceinline__ bool is_sep(uint32_t c) { return c == ' ' || c == '\t' || c == ','; }
__device__ __forceinline__ bool is_blank(uint32_t c) {
  return c == ' ' || c == '\t' || c == '\r';
}

// Four bytes of LDS starting at any byte offset p (aligned reads and a byte
// funnel shift).
__device__ __forceinline__ uint32_t lds_u32(const uint8_t *buf, uint32_t p) {
  const uint32_t *w = reinterpret_cast<const uint32_t *>(buf) + (p >> 2);
  return __builtin_amdgcn_alignbyte(w[1], w[0], p & 3);
}

// Bytes of x that are not '0' or '1', as a mask of their top bits (carry-free
// zero-byte test of (x ^ "0000") with the low bit cleared).
__device__ __forceinline__ uint32_t not01_bytes(uint32_t x) {
  const uint32_t t = (x ^ 0x30303030u) & 0xFEFEFEFEu;
  return (((t & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | t) & 0x80808080u;
}

// The low bits of four '0'/'1' bytes as a 4-bit number, byte 0 in bit 0: the
// multiply moves byte k's bit (at 8k) to bit 24 + k, with no two partial
// products meeting.
__device__ __forceinline__ uint32_t nibble(uint32_t x) {
  return ((x & 0x01010101u) * 0x01020408u) >> 24 & 0xFu;
}

// One block of 128 threads per 16 KiB chunk.  The chunk and the 256 bytes
// after it are staged in LDS with the positions of its first 129 newlines;
// lane j parses the j-th line starting in the chunk (after a newline of the
// chunk, or at byte 0 of the text in chunk 0) on its own, and the lanes store
// their records with coalesced writes (consecutive lanes, consecutive lines).
__global__ __launch_bounds__(kParseThreads) void k_text_parse(const uint8_t *text, uint64_t bytes,
                                                              const uint64_t *nl_before,
                                                              TextOut o) {
  __shared__ __attribute__((aligned(16))) uint8_t buf[kTextChunk + kOverhang + 16];
  __shared__ uint16_t nl[kChunkLines + 1];
  __shared__ uint32_t wsum[2];
  __shared__ uint32_t s_ovl;
  const uint32_t tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
  const uint64_t base = (uint64_t)blockIdx.x * kTextChunk;
  if (tid == 0) s_ovl = kTextChunk + kOverhang;
  // stage: thread t holds bytes [128 t, 128 t + 128) of the chunk (zero past the text)
  uint32_t w[32];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const u32x4 v = load16(text, bytes, base + 128u * tid + 16u * i);
    w[4 * i] = v.x;
    w[4 * i + 1] = v.y;
    w[4 * i + 2] = v.z;
    w[4 * i + 3] = v.w;
    *reinterpret_cast<u32x4 *>(buf + 128u * tid + 16u * i) = v;
  }
  __syncthreads();  // s_ovl initialised
  if (tid < (kOverhang + 16) / 16) {
    const u32x4 v = load16(text, bytes, base + kTextChunk + 16u * tid);
    *reinterpret_cast<u32x4 *>(buf + kTextChunk + 16u * tid) = v;
    uint32_t f = 0xFFFFFFFFu;
    for (int k = 3; k >= 0; --k) {
      const uint32_t m = nl_bytes(v[k]);
      if (m) f = 4u * k + ((uint32_t)__builtin_ctz(m) >> 3);
    }
    if (f != 0xFFFFFFFFu && tid < kOverhang / 16) atomicMin(&s_ovl, kTextChunk + 16u * tid + f);
  }
  // newline positions (the first 129) in order: prefix of the per-thread counts
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < 32; ++i) c += (uint32_t)__popc(nl_bytes(w[i]));
  uint32_t incl = c;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off);
    if ((int)lane >= off) incl += y;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  uint32_t rank = incl - c + (wv ? wsum[0] : 0u);
  const uint32_t total = wsum[0] + wsum[1];
  if (c && rank <= kChunkLines) {
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      uint32_t m = nl_bytes(w[i]);
      while (m && rank <= kChunkLines) {
        nl[rank++] = (uint16_t)(128u * tid + 4u * i + ((uint32_t)__builtin_ctz(m) >> 3));
        m &= m - 1;
      }
    }
  }
  __syncthreads();
  // the chunk's newlines must be the ones counted (a text changed between its
  // count and this parse would otherwise place lines silently wrong)
  if (tid == 0 && nl_before[blockIdx.x + 1] - nl_before[blockIdx.x] != total)
    atomicMin(o.err, (unsigned long long)(((blockIdx.x ? nl_before[blockIdx.x] + 1 : 0) << 8) | 7u));
  // the lines of this chunk
  const bool first = blockIdx.x == 0;
  const uint64_t text_end = bytes - base;  // chunk-relative end of the text
  const uint32_t ovl_end = (uint32_t)min((uint64_t)s_ovl, text_end);
  uint32_t nlines = total;
  if (total && total <= kChunkLines + 1 && base + nl[min(total, kChunkLines + 1) - 1] + 1 >= bytes)
    --nlines;
  if (first) ++nlines;
  const uint32_t j = tid;
  if (j >= min(nlines, kChunkLines)) return;
  const uint32_t s = first ? (j == 0 ? 0u : nl[j - 1] + 1u) : nl[j] + 1u;
  const uint32_t ei = first ? j : j + 1;  // index of the newline ending the line
  const uint32_t E = ei < total ? nl[ei] : ovl_end;
  const uint64_t line = (first ? 0 : nl_before[blockIdx.x] + 1) + j;
  uint32_t kind = 0;
  uint64_t id = 0, w0 = 0, w1 = 0, w2 = 0;
  if (E - s > kLineMax) {
    kind = 1;
  } else {
    // id: the run of digits at the start of the line (at most 20 looked at),
    // accumulated nine digits at a time in 32-bit parts a, b, c
    uint32_t e = 0, pa = 0, pb = 0, pc = 0;
    bool run = true;
#pragma unroll
    for (uint32_t k = 0; k < 20; k += 4) {
      const uint32_t x = lds_u32(buf, s + k);
#pragma unroll
      for (uint32_t b = 0; b < 4; ++b) {
        const uint32_t d = ((x >> (8 * b)) & 0xFFu) - '0';
        run = run && s + k + b < E && d < 10u;
        if (run) {
          if (k + b < 9) pa = pa * 10u + d;
          else if (k + b < 18) pb = pb * 10u + d;
          else pc = pc * 10u + d;
          ++e;
        }
      }
    }
    if (e <= 9) id = pa;
    else if (e <= 18) id = (uint64_t)pa * kPow10u[e - 9] + pb;
    else id = ((uint64_t)pa * 1000000000ull + pb) * kPow10u[e - 18] + pc;
    uint32_t p = s + e;
    while (p < E && is_sep(buf[p])) ++p;
    const uint32_t k0 = p;
    if (e == 0 || e > kIdDigits) {
      kind = 2;
    } else if (k0 == s + e) {
      kind = 3;
    } else if (E - k0 < 166) {
      kind = 4;
    } else {
      // 168 characters from k0: characters 0..163 (words 0..40) must all be
      // '0'/'1'; word 41 (characters 164..167) sets the width.  Two words at a
      // time become a byte of keys: the low bits of word i to bits 0..3, of
      // word i + 1 to bits 4..7, gathered by one multiply (no two partial
      // products meet, so nothing carries into the top byte).
      bool all01 = true;
      uint32_t width = 168;
#pragma unroll
      for (uint32_t i = 0; i < 42; i += 2) {
        const uint32_t x0 = lds_u32(buf, k0 + 4 * i), x1 = lds_u32(buf, k0 + 4 * i + 4);
        all01 = all01 && (x0 & 0xFEFEFEFEu) == 0x30303030u;
        if (i + 1 < 41) {
          all01 = all01 && (x1 & 0xFEFEFEFEu) == 0x30303030u;
        } else {
          const uint32_t bad = not01_bytes(x1);
          width = 164 + (bad ? ((uint32_t)__builtin_ctz(bad) >> 3) : 4u);
        }
        const uint32_t y = (x0 & 0x01010101u) | ((x1 & 0x01010101u) << 4);
        const uint64_t byte = (uint64_t)((y * 0x01020408u) >> 24);
        const uint32_t j = i / 2;  // byte j of the 168-bit field
        if (j < 8) w0 |= byte << (8 * j);
        else if (j < 16) w1 |= byte << (8 * (j - 8));
        else w2 |= byte << (8 * (j - 16));
      }
      if (!all01 || (width != 166 && width != 167)) {
        kind = 4;
      } else {
        w2 &= (1ull << (width - 128)) - 1ull;  // characters past the field
        if (width == 167 && (w0 & 1ull)) {
          kind = 5;
        } else {
          for (uint32_t q = k0 + width; q < E; ++q)
            if (!is_blank(buf[q])) {
              kind = 6;
              break;
            }
          if (width == 166) {  // character c is key c + 1
            w2 = (w2 << 1) | (w1 >> 63);
            w1 = (w1 << 1) | (w0 >> 63);
            w0 <<= 1;
          }
        }
      }
    }
  }
  if (kind) {
    if (line < o.n) atomicMin(o.err, (unsigned long long)((line << 8) | kind));
    return;
  }
  if (line < o.n) {
    uint64_t ra, rb;
    uint32_t rc, rd;
    relabel3(w0, w1, w2, &ra, &rb, &rc, &rd);
    o.a[line] = ra;
    o.b[line] = rb;
    o.c[line] = rc;
    o.d[line] = (uint8_t)rd;
    if (o.ids) o.ids[line] = id;
  }
}

}  // namespace fps

using namespace fps;

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static uint64_t text_chunks(uint64_t bytes) { return (bytes + kTextChunk - 1) / kTextChunk; }

static uint64_t text_tiles(uint64_t nc) { return (nc + kPrefixTile - 1) / kPrefixTile; }

extern "C" fps_status fps_text_workspace_bytes(uint64_t text_bytes, size_t *bytes) {
  fps_clear_error();
  if (!bytes) return fps_fail(FPS_E_ARG, "NULL argument");
  const uint64_t nc = text_chunks(text_bytes);
  if (nc >= (1ull << 31)) return fps_fail(FPS_E_ARG, "text of %llu bytes is too large",
                                          (unsigned long long)text_bytes);
  *bytes = align256(4 * nc) + align256(8 * (nc + 2)) + align256(8 * text_tiles(nc)) + 256;
  return FPS_OK;
}

struct TextWs {
  uint32_t *counts;
  uint64_t *before;  // nchunks prefix entries, then newlines, then records
  uint64_t *tiles;
  unsigned long long *err;
  uint64_t *tag;     // text address, text bytes, records of the last count
};

static fps_status text_validate(const void *text, uint64_t text_bytes, void *workspace,
                                size_t ws_bytes, TextWs *t) {
  if (!text || !workspace) return fps_fail(FPS_E_ARG, "NULL argument");
  if (text_bytes == 0) return fps_fail(FPS_E_ARG, "empty text");
  if (((uintptr_t)text & 15) != 0) return fps_fail(FPS_E_ARG, "text must be 16-byte aligned");
  if (((uintptr_t)workspace & 255) != 0)
    return fps_fail(FPS_E_ARG, "workspace must be 256-byte aligned");
  size_t need = 0;
  fps_status rc = fps_text_workspace_bytes(text_bytes, &need);
  if (rc) return rc;
  if (ws_bytes < need)
    return fps_fail(FPS_E_NOMEM, "text workspace of %zu bytes < %zu needed", ws_bytes, need);
  const uint64_t nc = text_chunks(text_bytes);
  uint8_t *p = (uint8_t *)workspace;
  t->counts = (uint32_t *)p;
  t->before = (uint64_t *)(p + align256(4 * nc));
  t->tiles = (uint64_t *)(p + align256(4 * nc) + align256(8 * (nc + 2)));
  t->err = (unsigned long long *)((uint8_t *)t->tiles + align256(8 * text_tiles(nc)));
  t->tag = (uint64_t *)(t->err + 1);
  return FPS_OK;
}

// Count and prefix kernels; *records receives the number of lines.
static fps_status text_lines(const uint8_t *text, uint64_t bytes, const TextWs &t,
                             hipStream_t s, uint64_t *records) {
  const uint32_t nc = (uint32_t)text_chunks(bytes);
  const uint32_t nt = (uint32_t)text_tiles(nc);
  hipLaunchKernelGGL(k_text_count, dim3((nc + 3) / 4), dim3(256), 0, s, text, bytes, nc,
                     t.counts);
  hipLaunchKernelGGL(k_text_tiles, dim3(nt), dim3(256), 0, s, (const uint32_t *)t.counts, nc,
                     t.tiles);
  hipLaunchKernelGGL(k_text_scan, dim3(nt), dim3(256), 0, s, text, bytes,
                     (const uint32_t *)t.counts, nc, (const uint64_t *)t.tiles, nt, t.before);
  uint64_t r = 0;
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&r, t.before + nc + 1, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fps_fail(FPS_E_DEVICE, "text line count failed");
  *records = r;
  return FPS_OK;
}

extern "C" fps_status fps_text_count(const void *text, uint64_t text_bytes, void *workspace,
                                     size_t ws_bytes, void *stream, uint64_t *n_records) {
  fps_clear_error();
  if (!n_records) return fps_fail(FPS_E_ARG, "NULL argument");
  TextWs t;
  fps_status rc = text_validate(text, text_bytes, workspace, ws_bytes, &t);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = text_lines((const uint8_t *)text, text_bytes, t, s, n_records))) return rc;
  // remember which text these counts belong to: a load of the same text with
  // this workspace need not count again
  const uint64_t tag[3] = {(uint64_t)(uintptr_t)text, text_bytes, *n_records};
  if (hipMemcpyAsync(t.tag, tag, sizeof tag, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fps_fail(FPS_E_DEVICE, "text count tag failed");
  return FPS_OK;
}

static const char *const kTextProblems[] = {
    "", "line longer than 255 characters", "id missing or longer than 19 digits",
    "no separator after the id", "keys not 166 or 167 characters 0/1",
    "position 0 set (it holds no key)", "characters other than blanks after the keys",
    "the text changed since it was counted"};

extern "C" fps_status fps_text_library_load(const void *text, uint64_t text_bytes,
                                            uint64_t n_records, const uint64_t *stride_begin,
                                            uint32_t nstrides, void *workspace, size_t ws_bytes,
                                            void *device_buf, size_t device_bytes,
                                            uint64_t *ids_device, uint64_t *ids_host,
                                            void *stream, fps_library **out) {
  fps_clear_error();
  if (!out) return fps_fail(FPS_E_ARG, "NULL argument");
  if (ids_host && !ids_device)
    return fps_fail(FPS_E_ARG, "ids_host needs ids_device (the ids are copied from it)");
  TextWs t;
  fps_status rc = text_validate(text, text_bytes, workspace, ws_bytes, &t);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const uint8_t *tx = (const uint8_t *)text;
  uint64_t lines = 0;
  uint64_t tag[3] = {0, 0, 0};
  if (hipMemcpyAsync(tag, t.tag, sizeof tag, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fps_fail(FPS_E_DEVICE, "text count tag read failed");
  if (tag[0] == (uint64_t)(uintptr_t)text && tag[1] == text_bytes && tag[2] == n_records) {
    lines = n_records;  // counted by fps_text_count on this text; the parse checks every chunk
  } else if ((rc = text_lines(tx, text_bytes, t, s, &lines))) {
    return rc;
  }
  if (lines != n_records)
    return fps_fail(FPS_E_ARG, "the text holds %llu lines, n_records = %llu",
                    (unsigned long long)lines, (unsigned long long)n_records);
  fps_library *L = nullptr;
  if ((rc = fps_library_new(n_records, stride_begin, nstrides, device_buf, device_bytes, &L)))
    return rc;
  do {
    uint8_t *da = (uint8_t *)L->dev, *db = da + 8 * L->np, *dc = db + 8 * L->np,
            *dd = dc + 4 * L->np;
    TextOut o{(uint64_t *)da, (uint64_t *)db, (uint32_t *)dc, dd, ids_device, n_records, t.err};
    if (hipMemsetAsync(t.err, 0xFF, 8, s) != hipSuccess) {
      rc = fps_fail(FPS_E_DEVICE, "hipMemsetAsync failed");
      break;
    }
    if ((rc = fps_library_zero_tail(L, s))) break;
    const uint32_t nc = (uint32_t)text_chunks(text_bytes);
    hipLaunchKernelGGL(k_text_parse, dim3(nc), dim3(kParseThreads), 0, s, tx, text_bytes,
                       (const uint64_t *)t.before, o);
    unsigned long long err = 0;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&err, t.err, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = fps_fail(FPS_E_DEVICE, "text parse failed");
      break;
    }
    if (err != ~0ull) {
      const uint32_t kind = (uint32_t)(err & 0xFF);
      rc = fps_fail(kind == 5 ? FPS_E_FINGERPRINT : FPS_E_ARG, "line %llu: %s",
                    (unsigned long long)((err >> 8) + 1), kTextProblems[kind < 8 ? kind : 0]);
      break;
    }
    L->ids_dev = ids_device;
    if (ids_host) {
      if (hipMemcpyAsync(ids_host, ids_device, 8 * n_records, hipMemcpyDeviceToHost, s) !=
              hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        rc = fps_fail(FPS_E_DEVICE, "id download failed");
        break;
      }
      L->ids = ids_host;
    }
  } while (0);
  if (rc) {
    delete L;  // (fps_library_free would clear the error message)
    return rc;
  }
  *out = L;
  return FPS_OK;
}

// ids[i] = table[hits[i].index] on the device; hits and ids are the device
// addresses of mapped pinned staging.
__global__ __launch_bounds__(256) void k_gather_ids(const uint64_t *table, const fps_hit *hits,
                                                    uint64_t n, uint64_t *ids) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ids[i] = table[hits[i].index];
}

extern "C" fps_status fps_hit_ids(const fps_library *lib, const fps_hit *hits, uint64_t n,
                                  uint64_t *ids) {
  fps_clear_error();
  if (!lib || (n && (!hits || !ids))) return fps_fail(FPS_E_ARG, "NULL argument");
  if (!lib->ids && !lib->ids_dev)
    return fps_fail(FPS_E_STATE, "the library has no id table (not loaded from text)");
  for (uint64_t i = 0; i < n; ++i)
    if (hits[i].index >= lib->n)
      return fps_fail(FPS_E_ARG, "hit %llu: index %u beyond the library", (unsigned long long)i,
                      hits[i].index);
  if (lib->ids) {
    for (uint64_t i = 0; i < n; ++i) ids[i] = lib->ids[hits[i].index];
    return FPS_OK;
  }
  if (n == 0) return FPS_OK;
  // the ids stay in device memory: gather them there
  fps_library *L = const_cast<fps_library *>(lib);
  std::lock_guard<std::mutex> lk(L->id_mu);
  const size_t need = (size_t)n * (sizeof(fps_hit) + sizeof(uint64_t));
  if (L->id_stage_bytes < need) {
    if (L->id_stage) (void)hipHostFree(L->id_stage);
    L->id_stage = nullptr;
    L->id_stage_bytes = 0;
    HIP_TRY(hipHostMalloc(&L->id_stage, need, hipHostMallocMapped));
    L->id_stage_bytes = need;
  }
  void *dev = nullptr;
  HIP_TRY(hipHostGetDevicePointer(&dev, L->id_stage, 0));
  memcpy(L->id_stage, hits, (size_t)n * sizeof(fps_hit));
  const fps_hit *dh = (const fps_hit *)dev;
  uint64_t *dids = (uint64_t *)((uint8_t *)dev + (size_t)n * sizeof(fps_hit));
  hipLaunchKernelGGL(k_gather_ids, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, nullptr,
                     lib->ids_dev, dh, n, dids);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(nullptr));
  memcpy(ids, (const uint8_t *)L->id_stage + (size_t)n * sizeof(fps_hit),
              (size_t)n * sizeof(uint64_t));
  return FPS_OK;
}

// ---------------------------------------------------------------------------
// The query box (Fig. 1): "[v, v, ..., v]" with blanks around tokens and one
// optional comma before ']'; 166 values are keys 1..166, 167 values positions
// 0..166 (position 0 must be 0).
// ---------------------------------------------------------------------------
static bool qblank(char c) { return c == ' ' || c == '\t' || c == '\r' || c == '\n'; }

static fps_status parse_list(const char *s, size_t len, uint64_t w[3], const char *where) {
  size_t i = 0;
  auto skip = [&]() {
    while (i < len && qblank(s[i])) ++i;
  };
  uint8_t vals[168];
  uint32_t nv = 0;
  skip();
  if (i >= len || s[i] != '[')
    return fps_fail(FPS_E_ARG, "%sposition %zu: expected '['", where, i);
  ++i;
  for (;;) {
    skip();
    if (i < len && s[i] == ']') break;
    if (i < len && (s[i] == '0' || s[i] == '1')) {
      if (nv == 167) return fps_fail(FPS_E_ARG, "%smore than 167 values", where);
      vals[nv++] = (uint8_t)(s[i] - '0');
      ++i;
    } else {
      return fps_fail(FPS_E_ARG, "%sposition %zu: expected 0 or 1", where, i);
    }
    skip();
    if (i < len && s[i] == ',') {
      ++i;
    } else if (i < len && s[i] == ']') {
      break;
    } else {
      return fps_fail(FPS_E_ARG, "%sposition %zu: expected ',' or ']'", where, i);
    }
  }
  ++i;
  skip();
  if (i != len) return fps_fail(FPS_E_ARG, "%sposition %zu: characters after ']'", where, i);
  if (nv != 166 && nv != 167)
    return fps_fail(FPS_E_ARG, "%s%u values; 166 or 167 expected", where, nv);
  const uint32_t first = nv == 167 ? 0 : 1;
  if (first == 0 && vals[0])
    return fps_fail(FPS_E_FINGERPRINT, "%sposition 0 holds no key and must be 0", where);
  w[0] = w[1] = w[2] = 0;
  for (uint32_t c = 0; c < nv; ++c)
    if (vals[c]) {
      const uint32_t j = first + c;
      w[j >> 6] |= 1ull << (j & 63);
    }
  return FPS_OK;
}

extern "C" fps_status fps_parse_query(const char *text, size_t len, uint64_t query[3]) {
  fps_clear_error();
  if (!text || !query) return fps_fail(FPS_E_ARG, "NULL argument");
  return parse_list(text, len, query, "");
}

extern "C" fps_status fps_parse_queries(const char *text, size_t len, uint64_t *queries,
                                        uint32_t capacity, uint32_t *nq) {
  fps_clear_error();
  if (!text || !nq || (capacity && !queries)) return fps_fail(FPS_E_ARG, "NULL argument");
  uint32_t got = 0;
  size_t pos = 0;
  uint64_t line = 0;
  while (pos < len) {
    size_t end = pos;
    while (end < len && text[end] != '\n') ++end;
    ++line;
    bool blank = true;
    for (size_t i = pos; i < end; ++i) blank = blank && qblank(text[i]);
    if (!blank) {
      if (got == capacity)
        return fps_fail(FPS_E_ARG, "more than %u queries (line %llu)", capacity,
                        (unsigned long long)line);
      char where[48];
      snprintf(where, sizeof where, "line %llu: ", (unsigned long long)line);
      fps_status rc = parse_list(text + pos, end - pos, queries + 3 * (size_t)got, where);
      if (rc) return rc;
      ++got;
    }
    pos = end + 1;
  }
  *nq = got;
  return FPS_OK;
}
