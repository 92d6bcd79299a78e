// gfx950 kernels of colour classes: the graph-colouring route to partial asynchrony that
// section 3.2 of Sahu, arXiv 2301.12390, cites for parallel Louvain. The vertex classes of a
// pass become the colour classes of a distance-1 colouring, so that the vertices of one
// synchronous class step (except the leftover class) have no arc between them.
//
// The colouring is first-fit in descending priority order, the priority of a vertex being its
// 64-bit SplitMix64 draw of the pass (ties cannot occur; they would go to the smaller id),
// colours 0..K-2, and class K-1 for a vertex that finds all K-1 taken. It is computed in
// rounds, the Jones-Plassmann way with one shortcut: a vertex is coloured in the round after
// its colour became fixed, which is when its last higher-priority neighbour was coloured, or
// earlier, when the higher neighbours coloured so far already hold all of 0..K-2. A colour
// depends on the higher neighbours' colours only, so the result equals the sequential first
// fit in priority order, whatever the schedule.
//
// Per vertex an 8-byte slot: a counter of uncoloured higher-priority neighbours and a mask of
// the colours those already coloured hold. Colouring a vertex pushes to each lower-priority
// neighbour: it ORs its colour into the mask (not the leftover class, which first fit never
// takes) and decrements the counter. A vertex is ready, and joins the next round's frontier,
// on whichever comes first of two events: its counter reaches zero (every higher neighbour is
// coloured, and the mask holds all their colours), or its mask fills up with colours 0..K-2
// (first fit can only give it the leftover class K-1, whatever the uncoloured higher
// neighbours take later). The event's thread claims the vertex with bit 31 of the mask, so the
// later event of a vertex appends nothing. The mask event breaks the long priority chains
// through high-degree vertices: on R-MAT graphs most of those end in the leftover class, and
// the rounds drop from thousands to about a hundred. The colour of a frontier vertex is the
// first fit of its mask: no gather of the neighbours' colours.
//
// Frontier appends are staged per workgroup. Rounds are enqueued in batches with no host
// synchronisation inside a batch: each kernel reads its frontier's size from device memory.
// Rows of up to kColShortRow arcs take a group of 16 lanes, rows of up to kColMidRow a
// wavefront, longer ones a 1024-thread workgroup.
#include <hip/hip_runtime.h>

#include <algorithm>

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
constexpr int kColBatch = 32;          // rounds enqueued between two looks from the host
constexpr unsigned kColRoundBlocks = 512;   // largest short-row part of a round (grid-stride)
constexpr unsigned kColMinBlocks = 8;       // smallest
constexpr unsigned kColLongBlocks = 256;    // largest grid of a long-row round
// Smallest mid- and long-row parts of a round: a batch sizes its grids from its first round,
// and the hubs' rows become ready in bulk later (one workgroup left to them took 196 ms on
// R-MAT s25's hub round); idle workgroups exit after one read.
constexpr unsigned kColMidMin = 128;
constexpr unsigned kColLongMin = 128;

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
  int32_t* slot;     // [2v]: uncoloured higher-priority neighbours; [2v + 1]: their colours
  uint8_t* colour;   // class, kUncoloured before
};

constexpr uint32_t kClaimed = 0x80000000u;  // mask bit of a vertex appended to a frontier

// Colours 0..K-2 (the mask of a vertex that can only take the leftover class)
__device__ __forceinline__ uint32_t all_colours(int K) {
  return K - 1 >= 32 ? 0xffffffffu : (1u << (K - 1)) - 1u;
}

__device__ __forceinline__ void set_slot(const ColArgs& a, int64_t v, int32_t count) {
  *reinterpret_cast<int2*>(a.slot + 2 * v) = make_int2(count, 0);
}

// Row kinds: short rows (up to kColShortRow arcs) take a group of kColGroup lanes, mid rows (up
// to kColMidRow arcs) a wavefront, long rows a kColBlock-thread workgroup.
constexpr int64_t kColMidRow = 4096;
enum { kShort = 0, kMid = 1, kLong = 2, kKinds = 3 };
__device__ __forceinline__ int row_kind(int64_t len) {
  return len <= kColShortRow ? kShort : len <= kColMidRow ? kMid : kLong;
}

// The frontiers: two alternating lists of each kind and three rotating counters of each kind
// (round r reads counter r % 3, appends to (r + 1) % 3 and clears (r + 2) % 3 for the round
// after).
struct Frontier {
  int32_t* list[kKinds][2];
  ull* counts;  // [9]: the counter of kind k for round r at 3k + r % 3
  __device__ __forceinline__ int32_t* at(int k, int r) const { return list[k][r & 1]; }
  __device__ __forceinline__ ull* counter(int k, int r) const { return counts + 3 * k + r % 3; }
};

// Appends u (where `want`) to the list, one atomic per wavefront.
__device__ __forceinline__ void append(bool want, int32_t u, int32_t* list, ull* counter) {
  const uint64_t bal = __ballot(want);
  if (!bal) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((unsigned long long)bal) - 1;
  ull base = 0;
  if (lane == leader) base = atomicAdd(counter, (ull)__popcll(bal));
  base = __shfl(base, leader, 64);
  if (want) list[base + __popcll(bal & ((1ull << lane) - 1))] = u;
}

// Appends staged in LDS per workgroup and flushed at its end with one atomic per list: a
// round's frontier holds ~10^5 vertices, and an atomic per wavefront on the one global counter
// of a list (serialised at ~10^8 per second) cost ~1 ms a round. Entries past a stage's
// capacity go straight to the global list (a testing mode shrinks the capacities to
// kSmallStage so that this path runs on small graphs).
constexpr int kStageShort = 4096;
constexpr int kStageMid = 1024;
constexpr int kStageLong = 512;
constexpr int kSmallStage = 4;

struct Stage {
  int32_t* list;   // LDS entries
  int* count;      // LDS count (may pass cap: the excess went to the global list)
  int cap;
};

__device__ __forceinline__ void stage_append(bool want, int32_t u, const Stage& st,
                                             int32_t* list, ull* counter) {
  const uint64_t bal = __ballot(want);
  if (!bal) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((unsigned long long)bal) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(st.count, __popcll(bal));
  base = __shfl(base, leader, 64);
  const int pos = base + __popcll(bal & ((1ull << lane) - 1));
  if (want && pos < st.cap) st.list[pos] = u;
  append(want && pos >= st.cap, u, list, counter);
}

// Copies a workgroup's staged entries to the global list (after a barrier).
__device__ __forceinline__ void stage_flush(const Stage& st, int32_t* list, ull* counter,
                                            ull* base) {
  const int cnt = min(*st.count, st.cap);
  if (threadIdx.x == 0) *base = cnt ? atomicAdd(counter, (ull)cnt) : 0;
  __syncthreads();
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) list[*base + i] = st.list[i];
}

// Counters of every vertex with a short row (groups of kColGroup lanes); mid and long rows are
// counted by k_col_count_mid and k_col_count_long, their ids appended to `mids` and `longs`
// (staged per workgroup; nrows[0], nrows[1] count them). ready[v] = 1 marks the short-row
// vertices of round 0's frontier (gathered by k_col_compact: one atomic per wavefront on the
// frontier counter, for ~10^7 vertices, serialised on that word for ~0.1 s).
constexpr int kCountStage = 1024;
constexpr unsigned kCountBlocks = 8192;
__global__ __launch_bounds__(kBlock) void k_col_count(ColArgs a, int32_t* mids, int32_t* longs,
                                                     ull* nrows, int32_t* ready, int cap_mid,
                                                     int cap_long) {
  __shared__ int32_t st_mid[kCountStage], st_long[kCountStage / 4];
  __shared__ int n_mid, n_long;
  __shared__ ull base;
  if (threadIdx.x == 0) n_mid = n_long = 0;
  __syncthreads();
  const Stage sm{st_mid, &n_mid, cap_mid}, sl{st_long, &n_long, cap_long};
  const int lane = threadIdx.x & (kColGroup - 1);
  const int64_t groups = (int64_t)gridDim.x * (kBlock / kColGroup);
  for (int64_t v = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / kColGroup; v < a.n;
       v += groups) {
    const int64_t b = a.rs[v], e = a.re[v];
    const int kind = row_kind(e - b);
    stage_append(lane == 0 && kind == kMid, (int32_t)v, sm, mids, nrows);
    stage_append(lane == 0 && kind == kLong, (int32_t)v, sl, longs, nrows + 1);
    if (kind != kShort) {
      if (lane == 0) {
        a.colour[v] = kUncoloured;
        set_slot(a, v, 0);  // counted by k_col_count_mid or k_col_count_long
        ready[v] = 0;
      }
      continue;
    }
    const uint64_t pv = vertex_draw(a.pass, local_id(v, a.gid, a.gbase));
    int c = 0;  // higher neighbours + 2^16 * all neighbours (a row here has at most 256 arcs)
    for (int64_t x = b + lane; x < e; x += kColGroup) {
      const int64_t u = a.idx[x];
      if (u != v)
        c += precedes(vertex_draw(a.pass, local_id(u, a.gid, a.gbase)), u, pv, v) ? 0x10001
                                                                                  : 0x10000;
    }
    for (int m = kColGroup / 2; m >= 1; m >>= 1) c += __shfl_xor(c, m, kColGroup);
    if (lane == 0) {
      // no neighbour: first fit over nothing is colour 0, with no push to make, so such a
      // vertex stays out of the frontier (on R-MAT s25 half the vertices)
      const bool alone = c == 0;
      set_slot(a, v, c & 0xffff);
      a.colour[v] = alone ? 0 : kUncoloured;
      ready[v] = !alone && (c & 0xffff) == 0;
    }
  }
  __syncthreads();
  stage_flush(sm, mids, nrows, &base);
  __syncthreads();
  stage_flush(sl, longs, nrows + 1, &base);
}

// Round 0's short frontier from the ready flags: each workgroup takes kCompactTile vertices,
// ranks its ready ones (wavefront prefix counts) and claims their list range with one atomic.
constexpr int kCompactPer = 16;
constexpr int64_t kCompactTile = (int64_t)kBlock * kCompactPer;
__global__ __launch_bounds__(kBlock) void k_col_compact(const int32_t* ready, int64_t n,
                                                       int32_t* list, ull* counter) {
  __shared__ int wsum[kBlock / 64];
  __shared__ ull base;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t t0 = blockIdx.x * kCompactTile; t0 < n; t0 += (int64_t)gridDim.x * kCompactTile) {
    const int64_t v0 = t0 + (int64_t)threadIdx.x * kCompactPer;
    int mine = 0;
#pragma unroll
    for (int k = 0; k < kCompactPer; k++) mine += v0 + k < n && ready[v0 + k] ? 1 : 0;
    int incl = mine;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(incl, d, 64);
      if (lane >= d) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int w = 0; w < kBlock / 64; w++) {
        const int x = wsum[w];
        wsum[w] = tot;
        tot += x;
      }
      base = tot ? atomicAdd(counter, (ull)tot) : 0;
    }
    __syncthreads();
    ull pos = base + wsum[wave] + incl - mine;
#pragma unroll
    for (int k = 0; k < kCompactPer; k++)
      if (v0 + k < n && ready[v0 + k]) list[pos++] = (int32_t)(v0 + k);
    __syncthreads();
  }
}

// Counters of the mid rows, a wavefront each (grid-stride over the list); those with no higher
// neighbour form round 0's mid frontier (staged per workgroup).
constexpr unsigned kColMidBlocks = 512;  // largest grid of a mid-row kernel
__global__ __launch_bounds__(kColBlock) void k_col_count_mid(ColArgs a, const int32_t* mids,
                                                             int64_t count, Frontier f,
                                                             int cap) {
  __shared__ int32_t st[kStageMid];
  __shared__ int nst;
  __shared__ ull base;
  if (threadIdx.x == 0) nst = 0;
  __syncthreads();
  const Stage sm{st, &nst, cap};
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (kColBlock / 64);
  for (int64_t t = (blockIdx.x * (int64_t)kColBlock + threadIdx.x) / 64; t < count;
       t += waves) {  // uniform over the wavefront
    const int64_t v = mids[t];
    const uint64_t pv = vertex_draw(a.pass, local_id(v, a.gid, a.gbase));
    const int64_t e = a.re[v];
    int c = 0;
    for (int64_t x = a.rs[v] + lane; x < e; x += 64) {
      const int64_t u = a.idx[x];
      if (u != v && precedes(vertex_draw(a.pass, local_id(u, a.gid, a.gbase)), u, pv, v)) c++;
    }
    for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m, 64);
    if (lane == 0) a.slot[2 * v] = c;
    stage_append(lane == 0 && c == 0, (int32_t)v, sm, f.at(kMid, 0), f.counter(kMid, 0));
  }
  __syncthreads();
  stage_flush(sm, f.at(kMid, 0), f.counter(kMid, 0), &base);
}

__global__ __launch_bounds__(kColBlock) void k_col_count_long(ColArgs a, const int32_t* longs,
                                                              Frontier f) {
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
    a.slot[2 * v] = t;
    if (t == 0) f.at(kLong, 0)[atomicAdd(f.counter(kLong, 0), 1ull)] = (int32_t)v;
  }
}

// First fit over the colours `used` (bit k: colour k held by a higher neighbour): the smallest
// free colour below K-1, else the leftover class K-1.
__device__ __forceinline__ uint8_t first_fit(uint32_t used, int K) {
  const uint32_t avail = ~used & all_colours(K);
  return avail ? (uint8_t)__ffs(avail) - 1 : (uint8_t)(K - 1);
}

// Appends a ready vertex (`want`) to the frontier of its kind for round `next`.
__device__ __forceinline__ void append_ready(const ColArgs& a, bool want, int64_t u,
                                             const Frontier& f, int next, const Stage* st) {
  const int kind = want ? row_kind(a.re[u] - a.rs[u]) : -1;
#pragma unroll
  for (int k = 0; k < kKinds; k++)
    stage_append(kind == k, (int32_t)u, st[k], f.at(k, next), f.counter(k, next));
}

// Colours frontier vertex v and pushes to its lower neighbours, with `lanes` threads from
// `lane` (appends staged in `stages`, one per row kind). U arcs per thread per trip, their
// loads and atomics issued together. U = 4 for every kind of row: 16 for long rows measured
// slower (more registers for the whole round kernel, whose short-row part then holds fewer
// wavefronts).
template <int U>
__device__ __forceinline__ void colour_push(const ColArgs& a, int64_t v, int lane, int lanes,
                                            const Frontier& f, int next, const Stage* stages) {
  const uint8_t c = first_fit(a.slot[2 * v + 1], a.K);
  if (lane == 0) a.colour[v] = c;
  const uint32_t bit = c < a.K - 1 ? 1u << c : 0u;
  const uint32_t full = all_colours(a.K);
  const uint64_t pv = vertex_draw(a.pass, local_id(v, a.gid, a.gbase));
  const int64_t b = a.rs[v], e = a.re[v];
  for (int64_t x0 = b; x0 < e; x0 += (int64_t)lanes * U) {
    int64_t u[U];
#pragma unroll
    for (int k = 0; k < U; k++) {
      const int64_t x = x0 + (int64_t)k * lanes + lane;
      u[k] = x < e ? a.idx[x] : v;
    }
    bool lower[U];
#pragma unroll
    for (int k = 0; k < U; k++)
      lower[k] = u[k] != v &&
                 precedes(pv, v, vertex_draw(a.pass, local_id(u[k], a.gid, a.gbase)), u[k]);
    // A plain read of the slot first: a push to a claimed vertex changes nothing (its colour
    // is fixed), and neither does an OR of a colour the mask holds. Bits are only ever set while
    // the colouring runs, so a stale read just skips less.
    int2 st[U];
#pragma unroll
    for (int k = 0; k < U; k++)
      st[k] = lower[k] ? *reinterpret_cast<const int2*>(a.slot + 2 * u[k]) : make_int2(0, kClaimed);
    uint32_t was[U];
    int32_t left[U];
#pragma unroll
    for (int k = 0; k < U; k++) {
      const uint32_t m = (uint32_t)st[k].y;
      const bool live = !(m & kClaimed);
      was[k] = live && (bit & ~m) ? atomicOr((uint32_t*)a.slot + 2 * u[k] + 1, bit) : full;
      left[k] = live ? atomicSub(a.slot + 2 * u[k], 1) : 0;
    }
#pragma unroll
    for (int k = 0; k < U; k++) {
      // the counter's last decrement, or the colour that completes the mask
      bool ready = left[k] == 1 || ((was[k] & full) != full && ((was[k] | bit) & full) == full);
      if (ready)
        ready = !(atomicOr((uint32_t*)a.slot + 2 * u[k] + 1, kClaimed) & kClaimed);
      append_ready(a, ready, u[k], f, next, stages);
    }
  }
}

// Round r in one launch of kColBlock-thread workgroups: the first gs take the short frontier
// (groups of kColGroup lanes), the next gm the mid frontier (a wavefront per vertex), the others
// the long frontier (a workgroup per vertex). Block 0 clears the counters of round r + 2.
__global__ __launch_bounds__(kColBlock) void k_col_round(ColArgs a, Frontier f, int r,
                                                         unsigned gs, unsigned gm, int cap_short,
                                                         int cap_mid, int cap_long) {
  __shared__ int32_t st_short[kStageShort], st_mid[kStageMid], st_long[kStageLong];
  __shared__ int nst[kKinds];
  __shared__ ull base;
  if (threadIdx.x < kKinds) nst[threadIdx.x] = 0;
  __syncthreads();
  const Stage st[kKinds] = {{st_short, &nst[kShort], cap_short},
                            {st_mid, &nst[kMid], cap_mid},
                            {st_long, &nst[kLong], cap_long}};
  const int next = r + 1;
  if (blockIdx.x < gs) {  // workgroup-uniform
    if (blockIdx.x == 0 && threadIdx.x < kKinds) f.counts[3 * threadIdx.x + (r + 2) % 3] = 0;
    const int64_t count = (int64_t)*f.counter(kShort, r);
    const int32_t* list = f.at(kShort, r);
    const int lane = threadIdx.x & (kColGroup - 1);
    const int64_t groups = (int64_t)gs * (kColBlock / kColGroup);
    for (int64_t t = (blockIdx.x * (int64_t)kColBlock + threadIdx.x) / kColGroup; t < count;
         t += groups)
      colour_push<4>(a, list[t], lane, kColGroup, f, next, st);
  } else if (blockIdx.x < gs + gm) {
    const int64_t count = (int64_t)*f.counter(kMid, r);
    const int32_t* list = f.at(kMid, r);
    const int64_t waves = (int64_t)gm * (kColBlock / 64);
    for (int64_t t = ((blockIdx.x - gs) * (int64_t)kColBlock + threadIdx.x) / 64; t < count;
         t += waves)
      colour_push<4>(a, list[t], threadIdx.x & 63, 64, f, next, st);
  } else {
    const int64_t count = (int64_t)*f.counter(kLong, r);
    const int32_t* list = f.at(kLong, r);
    const unsigned gl = gridDim.x - gs - gm;
    for (int64_t t = blockIdx.x - gs - gm; t < count; t += gl)
      colour_push<4>(a, list[t], threadIdx.x, kColBlock, f, next, st);
  }
  for (int k = 0; k < kKinds; k++) {
    __syncthreads();
    stage_flush(st[k], f.at(k, next), f.counter(k, next), &base);
  }
}

}  // namespace

hipError_t colour_classes(const DevGraph& g, int K, int pass, const int32_t* gid,
                          const int64_t* gbase, const ColourBuffers& cb, ull* host_words,
                          uint8_t* colour, int* rounds, bool small_stages, hipStream_t s) {
  *rounds = 0;
  const int64_t n = g.n;
  if (K < 2 || K > 32) return hipErrorInvalidValue;  // K = 1 is one class, no colouring
  if (n <= 0) return hipSuccess;
  ColArgs a{g.rs, g.re, g.idx, n, pass, K, gid, gbase, cb.slot, colour};
  Frontier f{{{cb.shorts, cb.shorts + n}, {cb.mids, cb.mids + n}, {cb.longs, cb.longs + n}},
             cb.counts};
  hipError_t e;
  if ((e = zero_words(cb.counts, 11, s)) != hipSuccess) return e;  // 9 counters + 2 row counts
  ull* nrows = cb.counts + 9;
  int32_t* ready = cb.shorts + n;  // round 0 appends to shorts[1] only after this is read
  const int cap = small_stages ? kSmallStage : 0;  // 0: each stage's full size
  LV_LAUNCH(k_col_count, std::min(blocks_for(n, kBlock / kColGroup), kCountBlocks), kBlock, 0, s,
            a, cb.all_long, cb.all_long + n, nrows, ready, cap ? cap : kCountStage,
            cap ? cap : kCountStage / 4);
  LV_LAUNCH(k_col_compact, blocks_for(n, kCompactTile), kBlock, 0, s, ready, n, f.list[kShort][0],
            cb.counts);
  if ((e = hipMemcpyAsync(host_words, nrows, 2 * sizeof(ull), hipMemcpyDeviceToHost, s)) !=
      hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  const ull nmid = host_words[0], nlong = host_words[1];
  if (nmid > 0)
    LV_LAUNCH(k_col_count_mid, (unsigned)std::min<ull>((nmid + 15) / 16, kColMidBlocks),
              kColBlock, 0, s, a, cb.all_long, (int64_t)nmid, f, cap ? cap : kStageMid);
  if (nlong > 0)
    LV_LAUNCH(k_col_count_long, (unsigned)nlong, kColBlock, 0, s, a, cb.all_long + n, f);
  // rounds in batches; a batch ends with a look at the next round's frontier sizes, which also
  // sizes the next batch's grids (any grid is correct: the kernels stride over their frontier)
  int r = 0;
  while (true) {
    if ((e = hipMemcpyAsync(host_words, cb.counts, 9 * sizeof(ull), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    const ull ns = host_words[r % 3], nm = host_words[3 + r % 3], nl = host_words[6 + r % 3];
    if (ns == 0 && nm == 0 && nl == 0) break;
    if (r > n + kColBatch) return hipErrorUnknown;  // cannot happen: each round colours a vertex
    const ull want_s = (ns + kColBlock / kColGroup - 1) / (kColBlock / kColGroup);
    const unsigned gs = (unsigned)std::min<ull>(std::max<ull>(want_s, kColMinBlocks),
                                                kColRoundBlocks);
    const unsigned gm = (unsigned)std::min<ull>(std::max<ull>((nm + 15) / 16, kColMidMin),
                                                kColMidBlocks);
    const unsigned gl = (unsigned)std::min<ull>(std::max<ull>(nl, kColLongMin), kColLongBlocks);
    for (int k = 0; k < kColBatch; k++, r++)
      LV_LAUNCH(k_col_round, gs + gm + gl, kColBlock, 0, s, a, f, r, gs, gm,
                cap ? cap : kStageShort, cap ? cap : kStageMid, cap ? cap : kStageLong);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  *rounds = r;
  return hipSuccess;
}

}  // namespace lv
