// Batch clustering search (Section 4.4): a batch of target fingerprints is
// grouped into clusters and the top-k library records of every cluster are
// searched; the number of clusters is the one with the best silhouette
// ("contour coefficient", Fig. 2).  The paper names neither the algorithm nor
// what is searched for a cluster; the reading taken:
//   - for every cluster count K in [k_min, k_max]: farthest-first initial
//     centers (center 0 = target 0, then the target farthest from its nearest
//     center, ties to the lowest index), then k-medians under the Manhattan
//     distance of Section 4.3: targets join the nearest center (ties to the
//     lowest center), centers become the key-wise strict majority of their
//     members (an empty cluster keeps its center), until no label changes;
//   - the silhouette of Rousseeuw (1987) of every target, s = (b - a) /
//     max(a, b) with a the mean distance to the other members of its cluster
//     and b the smallest mean distance to another cluster (0 for singletons
//     and when max(a, b) = 0), averaged in index order in float64; the K with
//     the largest average wins (ties to the smaller K);
//   - every center of the chosen clustering is searched like a target (Fig. 3).
//
// On the GPU: one block per K runs the whole k-medians loop with the centers,
// per-key member counts and the farthest-first distances in LDS (the batch is
// read from L2); the silhouette takes one wave per target, which recomputes
// the target's distances to the batch (XOR and popcount over three words)
// and keeps K per-cluster sums in registers; one wave adds the values in index
// order.  Every step is integer except the silhouette, whose float64 values
// come from four IEEE operations on exact integer sums.
#include <stdio.h>

#include <algorithm>
#include <vector>

#include "cand.h"
#include "fps_internal.h"
#include "runtime.h"

namespace fps {

constexpr uint32_t kClThreads = 1024;
constexpr uint32_t kClMaxK = FPS_CLUSTER_MAX_K;

__device__ __forceinline__ uint32_t dist3(const uint64_t *x, uint64_t a, uint64_t b,
                                          uint64_t c) {
  return (uint32_t)(__popcll(x[0] ^ a) + __popcll(x[1] ^ b) + __popcll(x[2] ^ c));
}

struct ClOut {
  uint8_t *labels;    // [K - k_min][q]
  uint64_t *centers;  // [K - k_min][kClMaxK][3]
  uint32_t *sizes;    // [K - k_min][kClMaxK]
  uint32_t *rounds;   // [K - k_min]
};

// Largest value with the lowest index over the block (value < 2^16).
__device__ __forceinline__ uint32_t block_argmax(uint32_t key, uint32_t *red) {
  // key = value << 16 | (0xFFFF - index): the maximum key has the largest
  // value and, among equal values, the lowest index
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) key = max(key, (uint32_t)__shfl_xor((int)key, o));
  if (lane_id() == 0) red[threadIdx.x >> 6] = key;
  __syncthreads();
  uint32_t m = 0;
  for (uint32_t w = 0; w < blockDim.x / 64; ++w) m = max(m, red[w]);
  __syncthreads();
  return m;
}

// One block per cluster count K = k_min + blockIdx.x.
__global__ __launch_bounds__(kClThreads) void k_cl_kmedians(const uint64_t *X, uint32_t q,
                                                            uint32_t k_min, uint32_t max_iter,
                                                            ClOut o) {
  __shared__ uint64_t cen[kClMaxK][3];
  __shared__ uint32_t cnt[kClMaxK][168];
  __shared__ uint32_t size[kClMaxK];
  __shared__ uint8_t near[FPS_CLUSTER_MAX_Q];
  __shared__ uint32_t red[kClThreads / 64];
  __shared__ uint32_t s_changed;
  const uint32_t K = k_min + blockIdx.x, tid = threadIdx.x;
  uint8_t *labels = o.labels + (size_t)blockIdx.x * q;
  // farthest-first initial centers
  if (tid < 3) cen[0][tid] = X[tid];
  __syncthreads();
  for (uint32_t i = tid; i < q; i += kClThreads)
    near[i] = (uint8_t)dist3(X + 3 * (size_t)i, cen[0][0], cen[0][1], cen[0][2]);
  __syncthreads();
  for (uint32_t c = 1; c < K; ++c) {
    uint32_t key = 0;
    for (uint32_t i = tid; i < q; i += kClThreads)
      key = max(key, ((uint32_t)near[i] << 16) | (0xFFFFu - i));
    const uint32_t far = 0xFFFFu - (block_argmax(key, red) & 0xFFFFu);
    if (tid < 3) cen[c][tid] = X[3 * (size_t)far + tid];
    __syncthreads();
    for (uint32_t i = tid; i < q; i += kClThreads)
      near[i] = (uint8_t)min((uint32_t)near[i],
                             dist3(X + 3 * (size_t)i, cen[c][0], cen[c][1], cen[c][2]));
    __syncthreads();
  }
  // Lloyd rounds
  uint32_t rounds = 0;
  for (uint32_t r = 1; r <= max_iter; ++r) {
    rounds = r;
    if (tid == 0) s_changed = r == 1 ? 1u : 0u;
    for (uint32_t i = tid; i < kClMaxK * 168; i += kClThreads) (&cnt[0][0])[i] = 0;
    if (tid < kClMaxK) size[tid] = 0;
    __syncthreads();
    bool changed = false;
    for (uint32_t i = tid; i < q; i += kClThreads) {
      const uint64_t *x = X + 3 * (size_t)i;
      uint32_t best = 0, bd = 0xFFFFFFFFu;
      for (uint32_t c = 0; c < K; ++c) {
        const uint32_t dd = dist3(x, cen[c][0], cen[c][1], cen[c][2]);
        if (dd < bd) {
          bd = dd;
          best = c;
        }
      }
      if (r > 1 && labels[i] != best) changed = true;
      labels[i] = (uint8_t)best;
      // member counts per key (keys 1..166 sit at bits 1..63, 0..63, 0..38)
      atomicAdd(&size[best], 1u);
      for (int w = 0; w < 3; ++w) {
        uint64_t m = x[w];
        while (m) {
          const uint32_t bit = (uint32_t)__builtin_ctzll(m);
          atomicAdd(&cnt[best][64 * w + bit], 1u);
          m &= m - 1;
        }
      }
    }
    if (changed) s_changed = 1;
    __syncthreads();
    const bool any = s_changed != 0;
    // centers: strict majority of the members (an empty cluster keeps its center)
    if (any) {
      for (uint32_t e = tid; e < K * 3; e += kClThreads) {
        const uint32_t c = e / 3, w = e % 3;
        if (size[c] == 0) continue;
        uint64_t v = 0;
        const uint32_t nb = w == 2 ? 39u : 64u;  // word 2 holds keys 128..166
        for (uint32_t b = 0; b < nb; ++b)
          if (2 * cnt[c][64 * w + b] > size[c]) v |= 1ull << b;
        cen[c][w] = v;
      }
    }
    __syncthreads();
    if (!any) break;
  }
  for (uint32_t e = tid; e < kClMaxK * 3; e += kClThreads)
    o.centers[(size_t)blockIdx.x * kClMaxK * 3 + e] = e / 3 < K ? (&cen[0][0])[e] : 0ull;
  if (tid < kClMaxK) o.sizes[blockIdx.x * kClMaxK + tid] = tid < K ? size[tid] : 0u;
  if (tid == 0) o.rounds[blockIdx.x] = rounds;
}

// One wave per (target i, K = k_min + blockIdx.y): the silhouette of i.
__global__ __launch_bounds__(256) void k_cl_silhouette(const uint64_t *X, uint32_t q,
                                                       uint32_t k_min, ClOut o, double *s) {
  const uint32_t i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = lane_id();
  const uint32_t kb = blockIdx.y, K = k_min + kb;
  if (i >= q) return;
  const uint8_t *labels = o.labels + (size_t)kb * q;
  const uint32_t *size = o.sizes + kb * kClMaxK;
  const uint64_t x0 = X[3 * (size_t)i], x1 = X[3 * (size_t)i + 1], x2 = X[3 * (size_t)i + 2];
  uint32_t sum[kClMaxK];
#pragma unroll
  for (uint32_t c = 0; c < kClMaxK; ++c) sum[c] = 0;
  for (uint32_t j = lane; j < q; j += 64) {
    const uint32_t d = dist3(X + 3 * (size_t)j, x0, x1, x2);
    const uint32_t l = labels[j];
#pragma unroll
    for (uint32_t c = 0; c < kClMaxK; ++c) sum[c] += (l == c) ? d : 0u;
  }
#pragma unroll
  for (uint32_t c = 0; c < kClMaxK; ++c)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum[c] += (uint32_t)__shfl_xor((int)sum[c], off);
  if (lane != 0) return;
  const uint32_t own = labels[i];
  double v = 0.0;
  if (size[own] > 1) {
    uint32_t sown = 0;
#pragma unroll
    for (uint32_t c = 0; c < kClMaxK; ++c)
      if (c == own) sown = sum[c];
    const double a = (double)sown / (double)(size[own] - 1);
    bool have_b = false;
    double b = 0.0;
#pragma unroll
    for (uint32_t c = 0; c < kClMaxK; ++c) {
      if (c < K && c != own && size[c] > 0) {
        const double m = (double)sum[c] / (double)size[c];
        if (!have_b || m < b) b = m;
        have_b = true;
      }
    }
    if (have_b) {
      const double top = a > b ? a : b;
      if (top > 0.0) v = (b - a) / top;
    }
  }
  s[(size_t)kb * q + i] = v;
}

// Mean silhouette of every K: one wave per K adds the q values in index order
// (lane 0 adds what the wave loaded, 64 values at a time).
__global__ __launch_bounds__(64) void k_cl_score(const double *s, uint32_t q, double *score) {
  const double *v = s + (size_t)blockIdx.x * q;
  double tot = 0.0;
  for (uint32_t j0 = 0; j0 < q; j0 += 64) {
    const double x = j0 + lane_id() < q ? v[j0 + lane_id()] : 0.0;
    const uint32_t m = min(64u, q - j0);
    for (uint32_t l = 0; l < m; ++l) {
      const double y = __shfl(x, (int)l);
      tot = tot + y;
    }
  }
  if (lane_id() == 0) score[blockIdx.x] = tot / (double)q;
}

}  // namespace fps

using namespace fps;

static inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace: the batch, then per K: labels, centers, sizes, rounds; the
// silhouette values; the scores.
struct ClLayout {
  size_t x, labels, centers, sizes, rounds, s, score, total;
};

static ClLayout cl_layout(uint32_t q) {
  const size_t nk = kClMaxK;  // K slots (at most k_max - k_min + 1 <= 15 used)
  ClLayout L;
  L.x = 0;
  L.labels = L.x + al256(24 * (size_t)q);
  L.centers = L.labels + al256(nk * q);
  L.sizes = L.centers + al256(nk * kClMaxK * 24);
  L.rounds = L.sizes + al256(nk * kClMaxK * 4);
  L.s = L.rounds + al256(nk * 4);
  L.score = L.s + al256(nk * 8 * (size_t)q);
  L.total = L.score + al256(nk * 8);
  return L;
}

extern "C" fps_status fps_cluster_workspace_bytes(uint32_t q, size_t *bytes) {
  fps_clear_error();
  if (!bytes) return fps_fail(FPS_E_ARG, "NULL argument");
  if (q < 3 || q > FPS_CLUSTER_MAX_Q)
    return fps_fail(FPS_E_ARG, "q = %u outside 3..%u", q, (unsigned)FPS_CLUSTER_MAX_Q);
  *bytes = cl_layout(q).total;
  return FPS_OK;
}

static fps_status cl_check(const uint64_t *queries, uint32_t q, uint32_t k_min, uint32_t k_max,
                           uint32_t max_iter) {
  if (!queries) return fps_fail(FPS_E_ARG, "NULL argument");
  if (q < 3 || q > FPS_CLUSTER_MAX_Q)
    return fps_fail(FPS_E_ARG, "q = %u outside 3..%u", q, (unsigned)FPS_CLUSTER_MAX_Q);
  if (k_min < 2 || k_max < k_min || k_max > kClMaxK || k_max >= q)
    return fps_fail(FPS_E_ARG, "cluster counts %u..%u must satisfy 2 <= k_min <= k_max <= %u, "
                    "k_max < q", k_min, k_max, (unsigned)kClMaxK);
  if (max_iter == 0) return fps_fail(FPS_E_ARG, "max_iter must be at least 1");
  for (uint32_t i = 0; i < q; ++i) {
    const uint64_t *w = queries + 3 * (size_t)i;
    if ((w[0] & 1ull) || (w[2] >> 39))
      return fps_fail(FPS_E_FINGERPRINT, "query %u has bit 0 or a bit above key 166 set", i);
  }
  return FPS_OK;
}

static fps_status cl_run(const uint64_t *queries, uint32_t q, uint32_t k_min, uint32_t k_max,
                         uint32_t max_iter, void *workspace, size_t ws_bytes, hipStream_t s,
                         uint32_t *labels, uint64_t *centers, fps_cluster_info *info) {
  fps_status rc = cl_check(queries, q, k_min, k_max, max_iter);
  if (rc) return rc;
  if (!workspace || ((uintptr_t)workspace & 255))
    return fps_fail(FPS_E_ARG, "workspace must be non-NULL and 256-byte aligned");
  const ClLayout L = cl_layout(q);
  if (ws_bytes < L.total)
    return fps_fail(FPS_E_NOMEM, "cluster workspace of %zu bytes < %zu needed", ws_bytes, L.total);
  uint8_t *w = (uint8_t *)workspace;
  uint64_t *X = (uint64_t *)(w + L.x);
  ClOut o{w + L.labels, (uint64_t *)(w + L.centers), (uint32_t *)(w + L.sizes),
          (uint32_t *)(w + L.rounds)};
  double *sv = (double *)(w + L.s), *score = (double *)(w + L.score);
  const uint32_t nk = k_max - k_min + 1;
  if (hipMemcpyAsync(X, queries, 24 * (size_t)q, hipMemcpyHostToDevice, s) != hipSuccess)
    return fps_fail(FPS_E_DEVICE, "query upload failed");
  hipLaunchKernelGGL(k_cl_kmedians, dim3(nk), dim3(kClThreads), 0, s, (const uint64_t *)X, q,
                     k_min, max_iter, o);
  hipLaunchKernelGGL(k_cl_silhouette, dim3((q + 3) / 4, nk), dim3(256), 0, s,
                     (const uint64_t *)X, q, k_min, o, sv);
  hipLaunchKernelGGL(k_cl_score, dim3(nk), dim3(64), 0, s, (const double *)sv, q, score);
  std::vector<double> sc(nk);
  std::vector<uint32_t> rounds(nk);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(sc.data(), score, 8 * nk, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(rounds.data(), o.rounds, 4 * nk, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fps_fail(FPS_E_DEVICE, "clustering kernels failed");
  uint32_t best = 0;
  for (uint32_t kb = 1; kb < nk; ++kb)
    if (sc[kb] > sc[best]) best = kb;
  const uint32_t K = k_min + best;
  std::vector<uint8_t> lab(q);
  if (hipMemcpyAsync(lab.data(), o.labels + (size_t)best * q, q, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipMemcpyAsync(centers, o.centers + (size_t)best * kClMaxK * 3, 24 * (size_t)K,
                     hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fps_fail(FPS_E_DEVICE, "cluster download failed");
  for (uint32_t i = 0; i < q; ++i) labels[i] = lab[i];
  if (info) {
    *info = fps_cluster_info{};
    info->k = K;
    info->rounds = rounds[best];
    for (uint32_t kb = 0; kb < nk; ++kb) info->score[k_min + kb] = sc[kb];
  }
  return FPS_OK;
}

extern "C" fps_status fps_cluster(const uint64_t *queries, uint32_t q, uint32_t k_min,
                                  uint32_t k_max, uint32_t max_iter, void *workspace,
                                  size_t ws_bytes, void *stream, uint32_t *labels,
                                  uint64_t *centers, fps_cluster_info *info) {
  fps_clear_error();
  if (!labels || !centers) return fps_fail(FPS_E_ARG, "NULL argument");
  return cl_run(queries, q, k_min, k_max, max_iter, workspace, ws_bytes, (hipStream_t)stream,
                labels, centers, info);
}

extern "C" fps_status fps_cluster_search_workspace_bytes(const fps_library *lib, uint32_t q,
                                                         uint32_t k_max, uint32_t k,
                                                         uint32_t mask, size_t *bytes) {
  fps_clear_error();
  if (!lib || !bytes) return fps_fail(FPS_E_ARG, "NULL argument");
  size_t cb = 0;
  fps_status rc = fps_cluster_workspace_bytes(q, &cb);
  if (rc) return rc;
  if (k_max < 1 || k_max > kClMaxK) return fps_fail(FPS_E_ARG, "k_max = %u out of range", k_max);
  std::vector<uint32_t> kk(k_max, k), mm(k_max, mask);
  size_t sb = 0;
  if ((rc = fps_workspace_bytes(lib, k_max, kk.data(), mm.data(), &sb))) return rc;
  *bytes = std::max(cb, sb);
  return FPS_OK;
}

extern "C" fps_status fps_cluster_search(fps_library *lib, const uint64_t *queries, uint32_t q,
                                         uint32_t k_min, uint32_t k_max, uint32_t max_iter,
                                         uint32_t k, uint32_t mask, void *workspace,
                                         size_t ws_bytes, fps_hit *out, uint64_t out_capacity,
                                         uint64_t *out_offset, uint32_t *labels,
                                         uint64_t *centers, fps_cluster_info *info,
                                         void *stream) {
  fps_clear_error();
  if (!lib || !out || !out_offset || !labels || !centers)
    return fps_fail(FPS_E_ARG, "NULL argument");
  size_t need = 0;
  fps_status rc = fps_cluster_search_workspace_bytes(lib, q, k_max, k, mask, &need);
  if (rc) return rc;
  if (ws_bytes < need)
    return fps_fail(FPS_E_NOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, need);
  fps_cluster_info local{};
  if (!info) info = &local;
  if ((rc = cl_run(queries, q, k_min, k_max, max_iter, workspace, ws_bytes, (hipStream_t)stream,
                   labels, centers, info)))
    return rc;
  // the chosen clustering's centers are searched like targets (Fig. 3)
  std::vector<uint32_t> kk(info->k, k), mm(info->k, mask);
  return fps_search_batch(lib, centers, info->k, kk.data(), mm.data(), workspace, ws_bytes, out,
                          out_capacity, out_offset, stream);
}
