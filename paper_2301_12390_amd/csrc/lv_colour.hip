// gfx950 kernels of colour classes: the graph-colouring route to partial asynchrony that
// section 3.2 of Sahu, arXiv 2301.12390, cites for parallel Louvain. The vertex classes of a
// pass become the colour classes of a distance-1 colouring, so that the vertices of one
// synchronous class step (except the leftover class) have no arc between them.
//
// The colouring is first-fit in descending priority order, the priority of a vertex being its
// 64-bit SplitMix64 draw of the pass (ties cannot occur; they would go to the smaller id),
// colours 0..K-2, and class K-1 for a vertex that finds all K-1 taken. It is computed the
// Jones-Plassmann way, in rounds: a vertex is coloured in the round after its last
// higher-priority neighbour, from the colours of those neighbours. Every higher neighbour is
// coloured before it and no lower neighbour is, so the result equals the sequential first-fit
// in priority order, whatever the schedule.
//
// Per vertex a counter of uncoloured higher-priority neighbours; each round lists the vertices
// whose counter is zero (a flag scan and compaction, no contended appends), colours them, and
// decrements the counters of their lower-priority neighbours. Rows of up to kColShortRow arcs
// take a group of 16 lanes, longer ones a 1024-thread workgroup.
#include <hip/hip_runtime.h>

#include "lv_device.h"
#include "lv_internal.h"

namespace lv {

namespace {

#define LV_LAUNCH(kernel, grid, block, shm, stream, ...)                          \
  do {                                                                            \
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shm, stream, __VA_ARGS__); \
  } while (0)

constexpr int64_t kColShortRow = 256;
constexpr int kColGroup = 16;
constexpr int kColBlock = 1024;
constexpr uint8_t kUncoloured = 0xFF;

inline unsigned blocks_for(int64_t items, int64_t per_block) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (unsigned)b;
}

__device__ __forceinline__ int64_t local_id(int64_t v, const int32_t* gid, const int64_t* gbase) {
  return gid ? v - gbase[gid[v]] : v;
}

// u is coloured before v: larger draw, ties to the smaller id
__device__ __forceinline__ bool precedes(uint64_t pu, int64_t u, uint64_t pv, int64_t v) {
  return pu > pv || (pu == pv && u < v);
}

struct ColArgs {
  const int64_t* rs;
  const int64_t* re;
  const int32_t* idx;
  int64_t n;
  int pass;
  int K;
  const int32_t* gid;
  const int64_t* gbase;
  int32_t* cnt;      // uncoloured higher-priority neighbours
  uint8_t* colour;   // class, kUncoloured before
};

// Counters of every vertex (groups of kColGroup lanes); rows longer than kColShortRow are
// counted by k_col_count_long, their ids appended to `longs`.
__global__ __launch_bounds__(kBlock) void k_col_count(ColArgs a, int32_t* longs, ull* nlong) {
  const int lane = threadIdx.x & (kColGroup - 1);
  const int64_t groups = (int64_t)gridDim.x * (kBlock / kColGroup);
  for (int64_t v = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / kColGroup; v < a.n;
       v += groups) {
    const int64_t b = a.rs[v], e = a.re[v];
    if (e - b > kColShortRow) {
      if (lane == 0) {
        a.colour[v] = kUncoloured;
        longs[atomicAdd(nlong, 1ull)] = (int32_t)v;
      }
      continue;
    }
    const uint64_t pv = vertex_draw(a.pass, local_id(v, a.gid, a.gbase));
    int c = 0;
    for (int64_t x = b + lane; x < e; x += kColGroup) {
      const int64_t u = a.idx[x];
      if (u != v && precedes(vertex_draw(a.pass, local_id(u, a.gid, a.gbase)), u, pv, v)) c++;
    }
    for (int m = kColGroup / 2; m >= 1; m >>= 1) c += __shfl_xor(c, m, kColGroup);
    if (lane == 0) {
      a.cnt[v] = c;
      a.colour[v] = kUncoloured;
    }
  }
}

__global__ __launch_bounds__(kColBlock) void k_col_count_long(ColArgs a, const int32_t* longs) {
  __shared__ int red[kColBlock / 64];
  const int64_t v = longs[blockIdx.x];
  const uint64_t pv = vertex_draw(a.pass, local_id(v, a.gid, a.gbase));
  int c = 0;
  for (int64_t x = a.rs[v] + threadIdx.x; x < a.re[v]; x += kColBlock) {
    const int64_t u = a.idx[x];
    if (u != v && precedes(vertex_draw(a.pass, local_id(u, a.gid, a.gbase)), u, pv, v)) c++;
  }
  for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int i = 0; i < kColBlock / 64; i++) t += red[i];
    a.cnt[v] = t;
  }
}

// Ready vertices of the round: uncoloured with no uncoloured higher neighbour. flag[v] counts
// them for the short list (low 32 bits) or the long list (high 32 bits).
__global__ void k_col_ready(ColArgs a, int64_t* flag) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < a.n;
       v += (int64_t)gridDim.x * blockDim.x) {
    int64_t f = 0;
    if (a.colour[v] == kUncoloured && a.cnt[v] == 0)
      f = a.re[v] - a.rs[v] > kColShortRow ? ((int64_t)1 << 32) : 1;
    flag[v] = f;
  }
}

__global__ void k_col_compact(int64_t n, const int64_t* flag, const int64_t* pos,
                              int32_t* shorts, int32_t* longs) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int64_t f = flag[v];
    if (f == 1) shorts[pos[v] & 0xffffffffll] = (int32_t)v;
    if (f > 1) longs[pos[v] >> 32] = (int32_t)v;
  }
}

// First fit over the colours `used` (bit k: colour k held by a higher neighbour): the smallest
// free colour below K-1, else the leftover class K-1.
__device__ __forceinline__ uint8_t first_fit(uint32_t used, int K) {
  const uint32_t avail = ~used & (K - 1 >= 32 ? 0xffffffffu : ((1u << (K - 1)) - 1u));
  return avail ? (uint8_t)__ffs(avail) - 1 : (uint8_t)(K - 1);
}

// Colour the listed vertices: their higher neighbours are all coloured (earlier rounds); lower
// neighbours lose one uncoloured higher neighbour each, to be listed in a later round.
__global__ __launch_bounds__(kBlock) void k_col_colour(ColArgs a, const int32_t* list,
                                                      int64_t count) {
  const int lane = threadIdx.x & (kColGroup - 1);
  const int64_t groups = (int64_t)gridDim.x * (kBlock / kColGroup);
  for (int64_t t = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / kColGroup; t < count;
       t += groups) {
    const int64_t v = list[t];
    const uint64_t pv = vertex_draw(a.pass, local_id(v, a.gid, a.gbase));
    uint32_t used = 0;
    for (int64_t x = a.rs[v] + lane; x < a.re[v]; x += kColGroup) {
      const int64_t u = a.idx[x];
      if (u == v) continue;
      if (precedes(vertex_draw(a.pass, local_id(u, a.gid, a.gbase)), u, pv, v)) {
        const uint8_t cu = a.colour[u];
        if (cu < a.K - 1) used |= 1u << cu;
      } else {
        atomicSub(&a.cnt[u], 1);
      }
    }
    for (int m = kColGroup / 2; m >= 1; m >>= 1) used |= __shfl_xor(used, m, kColGroup);
    if (lane == 0) a.colour[v] = first_fit(used, a.K);
  }
}

__global__ __launch_bounds__(kColBlock) void k_col_colour_long(ColArgs a, const int32_t* list) {
  __shared__ uint32_t red[kColBlock / 64];
  const int64_t v = list[blockIdx.x];
  const uint64_t pv = vertex_draw(a.pass, local_id(v, a.gid, a.gbase));
  uint32_t used = 0;
  for (int64_t x = a.rs[v] + threadIdx.x; x < a.re[v]; x += kColBlock) {
    const int64_t u = a.idx[x];
    if (u == v) continue;
    if (precedes(vertex_draw(a.pass, local_id(u, a.gid, a.gbase)), u, pv, v)) {
      const uint8_t cu = a.colour[u];
      if (cu < a.K - 1) used |= 1u << cu;
    } else {
      atomicSub(&a.cnt[u], 1);
    }
  }
  for (int m = 32; m >= 1; m >>= 1) used |= __shfl_xor(used, m, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = used;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t u = 0;
    for (int i = 0; i < kColBlock / 64; i++) u |= red[i];
    a.colour[v] = first_fit(u, a.K);
  }
}

}  // namespace

hipError_t colour_classes(const DevGraph& g, int K, int pass, const int32_t* gid,
                          const int64_t* gbase, const ColourBuffers& cb, ull* host_words,
                          uint8_t* colour, int* rounds, hipStream_t s) {
  *rounds = 0;
  const int64_t n = g.n;
  if (n <= 0) return hipSuccess;
  ColArgs a{g.rs, g.re, g.idx, n, pass, K, gid, gbase, cb.cnt, colour};
  hipError_t e;
  if ((e = zero_words(cb.nlong, 1, s)) != hipSuccess) return e;
  LV_LAUNCH(k_col_count, blocks_for(n, kBlock / kColGroup), kBlock, 0, s, a, cb.longs,
            cb.nlong);
  if ((e = hipMemcpyAsync(host_words, cb.nlong, sizeof(ull), hipMemcpyDeviceToHost, s)) !=
      hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  if (host_words[0] > 0)
    LV_LAUNCH(k_col_count_long, (unsigned)host_words[0], kColBlock, 0, s, a, cb.longs);
  int64_t left = n;
  while (left > 0) {
    LV_LAUNCH(k_col_ready, blocks_for(n, kBlock), kBlock, 0, s, a, cb.flag);
    if ((e = scan_i64(cb.flag, n, cb.pos, cb.partial, s)) != hipSuccess) return e;
    LV_LAUNCH(k_col_compact, blocks_for(n, kBlock), kBlock, 0, s, n, cb.flag, cb.pos,
              cb.shorts, cb.longs);
    if ((e = hipMemcpyAsync(host_words, cb.pos + n, sizeof(int64_t), hipMemcpyDeviceToHost,
                            s)) != hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    const int64_t ns = (int64_t)(host_words[0] & 0xffffffffull);
    const int64_t nl = (int64_t)(host_words[0] >> 32);
    if (ns + nl == 0) return hipErrorUnknown;  // cannot happen: the priority order has no cycle
    if (ns > 0)
      LV_LAUNCH(k_col_colour, blocks_for(ns, kBlock / kColGroup), kBlock, 0, s, a, cb.shorts,
                ns);
    if (nl > 0) LV_LAUNCH(k_col_colour_long, (unsigned)nl, kColBlock, 0, s, a, cb.longs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    left -= ns + nl;
    (*rounds)++;
  }
  return hipSuccess;
}

}  // namespace lv
