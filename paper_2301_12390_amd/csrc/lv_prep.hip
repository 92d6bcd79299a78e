// gfx950 kernels of graph preparation: an edge list becomes the undirected weighted CSR the
// method runs on (section 3.1.2 and Table 1: every edge also taken in reverse, unit weights, a
// self-loop on every vertex; repeated arcs combine into one).
//
// Design: every arc becomes a 64-bit key (source << b | neighbour) with a 32-bit weight. A
// stable LSD radix sort over the 2b significant key bits (8-bit digits, one histogram pass and
// one scatter pass per digit) orders the arcs by row, then by neighbour. Without input weights
// only the keys are sorted: every arc weighs 1 except the second copy of a self-loop edge,
// which weighs 0 and is marked by key bit 63 (outside the sorted bits, masked in comparisons). One last pass marks
// the first arc of every run of equal keys, combines each run's weights in LDS and writes the
// CSR: indices, weights and the row offsets (from the rows where the source changes). All of it
// streams the arc arrays through HBM; none of it is a contraction.
#include <hip/hip_runtime.h>

#include "lv_device.h"
#include "lv_internal.h"

namespace lv {

namespace {

#define LV_LAUNCH(kernel, grid, block, shm, stream, ...)                          \
  do {                                                                            \
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shm, stream, __VA_ARGS__); \
  } while (0)

constexpr int kItems = (int)(kPrepTile / kBlock);  // items per thread (16)
constexpr int kWaves = kBlock / 64;
constexpr int kWaveItems = (int)(kPrepTile / kWaves);  // consecutive items per wavefront (1024)
constexpr int kBins = 1 << kRadixBits;
static_assert(kItems * kBlock == kPrepTile, "tile = threads * items");
static_assert(kWaveItems == 64 * kItems, "a wavefront covers kItems rounds of 64 lanes");
// threads of the scatter (256 measured faster than 512 on the same tile)
constexpr int kScatterBlock = 256;
constexpr int kScatterWaves = kScatterBlock / 64;
constexpr int kScatterItems = (int)(kPrepTile / kScatterBlock);       // 8
constexpr int kScatterWaveItems = (int)(kPrepTile / kScatterWaves);  // 512
static_assert(kScatterWaveItems == 64 * kScatterItems, "scatter wavefront = rounds of 64");
static_assert(kBins <= kScatterBlock, "one digit per scatter thread");

inline unsigned grid_stride_blocks(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (unsigned)b;
}

inline int64_t tiles_of(int64_t N) { return (N + kPrepTile - 1) / kPrepTile; }

__global__ void k_fill_ull(ull* a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0;
}

constexpr uint64_t kZeroWeight = 1ull << 63;  // keys-only arcs: this copy weighs 0

// Weight of arc i (key k) of the sorted or unsorted arrays.
__device__ __forceinline__ ull arc_weight(const uint32_t* vals, int64_t i, uint64_t k) {
  return vals ? (ull)vals[i] : ((k & kZeroWeight) ? 0ull : 1ull);
}

// Arcs of the edge list: with kPrepSym, edge e gives arcs 2e (u -> v) and 2e+1 (v -> u; for a
// self-loop the second copy has weight 0, so it adds nothing to the one arc a loop stands for);
// with kPrepLoops, arcs base + v are the added loops of weight 1. vals == nullptr (no input
// weights): keys only, the zero-weight copy marked by kZeroWeight. Bad endpoints set bit 0 of
// *bad and bad weights bit 1; their arcs are written with endpoint 0 so that every later index
// stays in range (the caller stops before using them).
__global__ __launch_bounds__(kBlock) void k_prep_expand(int64_t n, int64_t m, const int32_t* src,
                                                       const int32_t* dst, const uint32_t* w,
                                                       uint32_t flags, int b, uint64_t* keys,
                                                       uint32_t* vals, unsigned int* bad) {
  const bool sym = (flags & kPrepSym) != 0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < m; e += stride) {
    const int32_t u = src[e], v = dst[e];
    const uint32_t x = w ? w[e] : 1u;
    unsigned int err = 0;
    if (u < 0 || u >= n || v < 0 || v >= n) err |= 1u;
    if (x == 0) err |= 2u;
    if (err) atomicOr(bad, err);
    const uint64_t uu = (err & 1u) ? 0 : (uint64_t)u, vv = (err & 1u) ? 0 : (uint64_t)v;
    if (sym) {
      keys[2 * e] = (uu << b) | vv;
      keys[2 * e + 1] = ((vv << b) | uu) | (!vals && u == v ? kZeroWeight : 0);
      if (vals) {
        vals[2 * e] = x;
        vals[2 * e + 1] = u == v ? 0u : x;
      }
    } else {
      keys[e] = (uu << b) | vv;
      if (vals) vals[e] = x;
    }
  }
  if (flags & kPrepLoops) {
    const int64_t base = sym ? 2 * m : m;
    for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += stride) {
      keys[base + v] = ((uint64_t)v << b) | (uint64_t)v;
      if (vals) vals[base + v] = 1u;
    }
  }
}

__device__ __forceinline__ ull wave_max_u64(ull x) {
  for (int m = 32; m >= 1; m >>= 1) {
    const ull y = __shfl_xor(x, m, 64);
    x = y > x ? y : x;
  }
  return x;
}

// Lanes among `valid` whose digit equals this lane's (d < 2^bits), from one ballot per bit.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, int bits, uint64_t valid) {
  uint64_t peers = valid;
  for (int i = 0; i < bits; i++) {
    const uint32_t bit = (d >> i) & 1u;
    const uint64_t bal = __ballot(bit);
    peers &= bit ? bal : ~bal;
  }
  return peers;
}

// Per-tile digit histogram, digit-major: hist[d * ntiles + tile]. Each wavefront counts runs of
// equal digits once (its leader lane adds the run length), so skewed digits cost no LDS
// atomic contention.
__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint64_t* keys, int64_t N, int shift,
                                                      int bits, int32_t* hist, int64_t ntiles) {
  __shared__ int32_t h[kBins];
  const int bins = 1 << bits;
  for (int i = threadIdx.x; i < bins; i += kBlock) h[i] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t lt = (1ull << lane) - 1;
  const int64_t base = blockIdx.x * kPrepTile + (int64_t)wave * kWaveItems;
  for (int r = 0; r < kItems; r++) {
    const int64_t i = base + r * 64 + lane;
    const bool ok = i < N;
    const uint32_t d = ok ? (uint32_t)(keys[i] >> shift) & (uint32_t)(bins - 1) : 0u;
    const uint64_t peers = match_digit(d, bits, __ballot(ok));
    if (ok && (peers & lt) == 0) atomicAdd(&h[d], (int32_t)__popcll(peers));
  }
  __syncthreads();
  for (int d = threadIdx.x; d < bins; d += kBlock) hist[(int64_t)d * ntiles + blockIdx.x] = h[d];
}

// Inclusive scan of x over the WAVES wavefronts of the workgroup (wsum: WAVES ints of LDS; the
// call contains __syncthreads()).
template <int WAVES>
__device__ __forceinline__ int32_t block_inclusive_scan(int32_t x, int32_t* wsum) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  for (int wv = 0; wv < wave; wv++) x += wsum[wv];
  __syncthreads();
  return x;
}

// Stable scatter of one digit. Tile items are ordered (wavefront, round, lane); a lane's rank
// among the equal digits of its wavefront is the wavefront's running count for the digit plus
// the equal lanes below it in the round. The tile is first ordered by digit in LDS (the
// position of an item: the tile's start for its digit, plus the counts of earlier wavefronts,
// plus its rank), then written out in LDS order, so that consecutive threads write consecutive
// addresses of a digit's run. offs (exclusive scan of the histogram, digit-major) gives every
// (digit, tile) its output start.
template <bool VALS>
__global__ __launch_bounds__(kScatterBlock) void k_radix_scatter(
    const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout, int64_t N,
    int shift, int bits, const int64_t* offs, int64_t ntiles) {
  __shared__ uint64_t skey[kPrepTile];
  __shared__ uint32_t sval[VALS ? kPrepTile : 1];
  __shared__ int32_t cnt[kScatterWaves][kBins];
  __shared__ int64_t gstart[kBins];
  __shared__ int32_t wsum[kScatterWaves];
  const int bins = 1 << bits;
  for (int i = threadIdx.x; i < kScatterWaves * kBins; i += kScatterBlock)
    cnt[i / kBins][i % kBins] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t lt = (1ull << lane) - 1;
  const int64_t tbase = blockIdx.x * kPrepTile;
  const int64_t base = tbase + (int64_t)wave * kScatterWaveItems;
  uint64_t key[kScatterItems];
  uint32_t val[kScatterItems];
  int32_t rank[kScatterItems];
#pragma unroll
  for (int r = 0; r < kScatterItems; r++) {
    const int64_t i = base + r * 64 + lane;
    const bool ok = i < N;
    key[r] = ok ? kin[i] : 0;
    val[r] = VALS && ok ? vin[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kScatterItems; r++) {
    const int64_t i = base + r * 64 + lane;
    const bool ok = i < N;
    const uint32_t d = (uint32_t)(key[r] >> shift) & (uint32_t)(bins - 1);
    const uint64_t peers = match_digit(d, bits, __ballot(ok));
    // all lanes of the digit read the running count before its leader lane advances it (LDS
    // operations of one wavefront complete in program order)
    const int32_t before = ok ? cnt[wave][d] : 0;
    rank[r] = before + (int32_t)__popcll(peers & lt);
    if (ok && (peers & lt) == 0) cnt[wave][d] = before + (int32_t)__popcll(peers);
  }
  __syncthreads();
  // tile-local start of every (wavefront, digit); global start minus tile-local start per digit
  {
    const int t = threadIdx.x;  // one digit per thread
    int32_t c[kScatterWaves];
    int32_t tot = 0;
#pragma unroll
    for (int wv = 0; wv < kScatterWaves; wv++) {
      c[wv] = t < bins ? cnt[wv][t] : 0;
      tot += c[wv];
    }
    const int32_t excl = block_inclusive_scan<kScatterWaves>(tot, wsum) - tot;
    if (t < bins) {
      int32_t run = excl;
#pragma unroll
      for (int wv = 0; wv < kScatterWaves; wv++) {
        cnt[wv][t] = run;
        run += c[wv];
      }
      gstart[t] = offs[(int64_t)t * ntiles + blockIdx.x] - excl;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kScatterItems; r++) {
    const int64_t i = base + r * 64 + lane;
    if (i < N) {
      const uint32_t d = (uint32_t)(key[r] >> shift) & (uint32_t)(bins - 1);
      const int32_t lp = cnt[wave][d] + rank[r];
      skey[lp] = key[r];
      if (VALS) sval[lp] = val[r];
    }
  }
  __syncthreads();
  const int64_t tn = N - tbase < kPrepTile ? N - tbase : kPrepTile;
  for (int j = threadIdx.x; j < tn; j += kScatterBlock) {
    const uint64_t k = skey[j];
    const uint32_t d = (uint32_t)(k >> shift) & (uint32_t)(bins - 1);
    const int64_t pos = gstart[d] + j;
    kout[pos] = k;
    if (VALS) vout[pos] = sval[j];
  }
}

// ---- one-sweep variant: global digit counts up front, tile offsets by decoupled look-back

// Counts of every digit of every pass over all keys (ghist[p * kBins + d], zeroed by the
// caller): grid-stride with per-workgroup LDS counts, added to ghist once per workgroup.
__global__ __launch_bounds__(kBlock) void k_radix_counts(const uint64_t* keys, int64_t N,
                                                        SortPlan plan, ull* ghist) {
  __shared__ int32_t h[kMaxSortPasses][kBins];
  for (int i = threadIdx.x; i < kMaxSortPasses * kBins; i += kBlock) h[i / kBins][i % kBins] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < N; i += stride) {
    const uint64_t k = keys[i];
    for (int p = 0; p < plan.passes; p++)
      atomicAdd(&h[p][(uint32_t)(k >> plan.shift[p]) & ((1u << plan.bits[p]) - 1)], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < plan.passes * kBins; i += kBlock) {
    const int32_t c = h[i / kBins][i % kBins];
    if (c) atomicAdd(&ghist[i], (ull)c);
  }
}

// Exclusive scan of every pass's digit counts into the passes' output starts (one thread).
__global__ void k_radix_bases(const ull* ghist, int passes, int64_t* gbase) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int p = 0; p < passes; p++) {
    int64_t run = 0;
    for (int d = 0; d < kBins; d++) {
      gbase[p * kBins + d] = run;
      run += (int64_t)ghist[p * kBins + d];
    }
  }
}

// Look-back status words: flag in the top two bits (0 not ready, 1 the tile's own count, 2 the
// count of the tile and all tiles before it), the count below.
constexpr ull kStAgg = 1ull << 62, kStIncl = 2ull << 62, kStMask = (1ull << 62) - 1;
// Waits on one predecessor's status before giving up (bit 3 of *bad): predecessors are
// workgroups already running, so in practice the wait is a few microseconds.
constexpr int kLookbackSpinCap = 1 << 22;
constexpr int kLookbackWindow = 16;  // predecessors read at once

// One stable scatter pass without a histogram pass of its own. Workgroups take tiles in order
// from *counter, so every earlier tile belongs to a running or finished workgroup. Ranks within
// the tile are as in k_radix_scatter; the tile's start for digit d is gbase[d] plus the counts
// of d in earlier tiles, summed by walking back over their status words until one holds an
// inclusive count (decoupled look-back, Merrill and Garland's single-pass scan), after which
// the tile publishes its own inclusive count.
template <bool VALS>
__global__ __launch_bounds__(kScatterBlock) void k_radix_onesweep(
    const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout, int64_t N,
    int shift, int bits, const int64_t* gbase, ull* status, ull* counter, unsigned int* bad) {
  __shared__ uint64_t skey[kPrepTile];
  __shared__ uint32_t sval[VALS ? kPrepTile : 1];
  __shared__ int32_t cnt[kScatterWaves][kBins];
  __shared__ int32_t lstart[kBins];  // tile-local start of every digit
  __shared__ int64_t gstart[kBins];
  __shared__ int32_t wsum[kScatterWaves];
  __shared__ int64_t tile_sh;
  const int bins = 1 << bits;
  for (int i = threadIdx.x; i < kScatterWaves * kBins; i += kScatterBlock)
    cnt[i / kBins][i % kBins] = 0;
  if (threadIdx.x == 0) tile_sh = (int64_t)atomicAdd(counter, 1ull);
  __syncthreads();
  const int64_t tile = tile_sh;
  const int t = threadIdx.x;  // one digit per thread in the per-digit steps
  int32_t tot = 0;
  {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lt = (1ull << lane) - 1;
    const int64_t base = tile * kPrepTile + (int64_t)wave * kScatterWaveItems;
    uint64_t key[kScatterItems];
    uint32_t val[kScatterItems];
    int32_t rank[kScatterItems];
#pragma unroll
    for (int r = 0; r < kScatterItems; r++) {
      const int64_t i = base + r * 64 + lane;
      const bool ok = i < N;
      key[r] = ok ? kin[i] : 0;
      val[r] = VALS && ok ? vin[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kScatterItems; r++) {
      const int64_t i = base + r * 64 + lane;
      const bool ok = i < N;
      const uint32_t d = (uint32_t)(key[r] >> shift) & (uint32_t)(bins - 1);
      const uint64_t peers = match_digit(d, bits, __ballot(ok));
      const int32_t before = ok ? cnt[wave][d] : 0;
      rank[r] = before + (int32_t)__popcll(peers & lt);
      if (ok && (peers & lt) == 0) cnt[wave][d] = before + (int32_t)__popcll(peers);
    }
    __syncthreads();
    // the tile's count of every digit, published at once for the tiles after it; tile-local
    // starts of every (wavefront, digit)
    int32_t c[kScatterWaves];
#pragma unroll
    for (int wv = 0; wv < kScatterWaves; wv++) {
      c[wv] = t < bins ? cnt[wv][t] : 0;
      tot += c[wv];
    }
    if (t < bins)
      __hip_atomic_store(status + tile * kBins + t, (tile == 0 ? kStIncl : kStAgg) | (ull)tot,
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t excl = block_inclusive_scan<kScatterWaves>(tot, wsum) - tot;
    if (t < bins) {
      lstart[t] = excl;
      int32_t run = excl;
#pragma unroll
      for (int wv = 0; wv < kScatterWaves; wv++) {
        cnt[wv][t] = run;
        run += c[wv];
      }
    }
    __syncthreads();
    // the tile ordered by digit in LDS
#pragma unroll
    for (int r = 0; r < kScatterItems; r++) {
      const int64_t i = base + r * 64 + lane;
      if (i < N) {
        const uint32_t d = (uint32_t)(key[r] >> shift) & (uint32_t)(bins - 1);
        const int32_t lp = cnt[wave][d] + rank[r];
        skey[lp] = key[r];
        if (VALS) sval[lp] = val[r];
      }
    }
  }
  // counts of every digit in the earlier tiles: look back over windows of kLookbackWindow
  // predecessors loaded together, nearest first, until an inclusive count
  if (t < bins) {
    int64_t earlier = 0;
    if (tile > 0) {
      int64_t p = tile - 1;
      int spins = 0;
      bool done = false;
      while (!done) {
        const int wn = p + 1 < kLookbackWindow ? (int)(p + 1) : kLookbackWindow;
        ull v[kLookbackWindow];
#pragma unroll
        for (int j = 0; j < kLookbackWindow; j++)
          v[j] = j < wn ? __hip_atomic_load(status + (p - j) * kBins + t, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT)
                        : 0ull;
        for (int j = 0; j < wn && !done; j++) {
          ull x = v[j];
          while ((x >> 62) == 0) {
            if (++spins > kLookbackSpinCap) break;
            __builtin_amdgcn_s_sleep(1);
            x = __hip_atomic_load(status + (p - j) * kBins + t, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
          }
          if ((x >> 62) == 0) {  // gave up: the result is marked bad
            atomicOr(bad, 8u);
            done = true;
            break;
          }
          earlier += (int64_t)(x & kStMask);
          if ((x >> 62) == 2) done = true;
        }
        p -= wn;
        if (p < 0) done = true;  // tile 0 always publishes an inclusive count
      }
      __hip_atomic_store(status + tile * kBins + t, kStIncl | (ull)(earlier + tot),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    gstart[t] = gbase[t] + earlier - lstart[t];
  }
  __syncthreads();
  const int64_t tbase = tile * kPrepTile;
  const int64_t tn = N - tbase < kPrepTile ? N - tbase : kPrepTile;
  for (int j = threadIdx.x; j < tn; j += kScatterBlock) {
    const uint64_t k = skey[j];
    const uint32_t d = (uint32_t)(k >> shift) & (uint32_t)(bins - 1);
    const int64_t pos = gstart[d] + j;
    kout[pos] = k;
    if (VALS) vout[pos] = sval[j];
  }
}

// Per tile: the heads (first arc of a run of equal keys) and the combined weight of the arcs
// before the tile's first head (all its arcs if it has none): the part of a run that began in
// an earlier tile.
template <bool MAXC>
__global__ __launch_bounds__(kBlock) void k_prep_heads(const uint64_t* keys, const uint32_t* vals,
                                                      int64_t N, uint64_t kmask,
                                                      int32_t* tile_heads, ull* tile_first) {
  __shared__ ull red[kBlock / 64];
  const int64_t base = blockIdx.x * kPrepTile;
  ull c = 0;
  int64_t mine = kPrepTile;  // this thread's first head (tile offset); its items ascend with r
  for (int r = 0; r < kItems; r++) {
    const int64_t i = base + r * kBlock + threadIdx.x;
    if (i < N && (i == 0 || ((keys[i] ^ keys[i - 1]) & kmask) != 0)) {
      c++;
      if (mine == kPrepTile) mine = i - base;
    }
  }
  // the tile's first head: minimum over the block
  for (int m = 32; m >= 1; m >>= 1) {
    const int64_t y = __shfl_xor(mine, m, 64);
    mine = y < mine ? y : mine;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = (ull)mine;
  __syncthreads();
  int64_t first = kPrepTile;
  for (int wv = 0; wv < kWaves; wv++) first = (int64_t)red[wv] < first ? (int64_t)red[wv] : first;
  __syncthreads();
  const int64_t fh = base + first;
  ull part = 0;
  for (int r = 0; r < kItems; r++) {
    const int64_t i = base + r * kBlock + threadIdx.x;
    if (i < N && i < fh) {
      const ull x = arc_weight(vals, i, keys[i]);
      part = MAXC ? (x > part ? x : part) : part + x;
    }
  }
  c = block_sum_u64(c, red);
  if (MAXC) {
    part = wave_max_u64(part);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0)
      for (int wv = 0; wv < kWaves; wv++) part = red[wv] > part ? red[wv] : part;
  } else {
    part = block_sum_u64(part, red);
  }
  if (threadIdx.x == 0) {
    tile_heads[blockIdx.x] = (int32_t)c;
    tile_first[blockIdx.x] = part;
  }
}

// The CSR from the sorted arcs. tile_slot: exclusive scan of the heads per tile ([ntiles+1],
// the last entry the arc count). A head's slot is tile_slot[tile] + (heads of the tile up to and
// including it) - 1; the arcs before a tile's first head continue the previous tile's last run
// (local slot 0, left to the tile that holds that run's head). Weights combine per local slot in
// LDS. A tile whose last run continues past its end adds the leading parts (tile_first) of the
// following tiles, through those without heads, and stores the total: every slot is written
// once, with no atomics. Offsets: the head that starts row r (after rows prow+1..r-1 without
// arcs) writes off[prow+1..r]; the last arc writes the rows after its own. W32: weights are
// written as uint32 and a total above 2^32-1 sets bit 2 of *bad.
template <bool MAXC, bool W32>
__global__ __launch_bounds__(kBlock) void k_prep_emit(const uint64_t* keys, const uint32_t* vals,
                                                     int64_t N, int64_t n, int b, uint64_t kmask,
                                                     const int64_t* tile_slot,
                                                     const int32_t* tile_heads,
                                                     const ull* tile_first, int64_t ntiles,
                                                     int64_t* off, int32_t* idx, void* wout,
                                                     unsigned int* bad) {
  __shared__ ull acc[kPrepTile + 1];
  __shared__ int32_t wsum[kWaves];
  const int64_t tile = blockIdx.x, base = tile * kPrepTile;
  const int64_t end = base + kPrepTile < N ? base + kPrepTile : N;
  const int64_t sbase = tile_slot[tile];
  const int64_t nheads = tile_slot[tile + 1] - sbase;
  const int64_t total = tile_slot[ntiles];
  const uint64_t vmask = (1ull << b) - 1;
  for (int i = threadIdx.x; i <= kPrepTile; i += kBlock) acc[i] = 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t le = lane == 63 ? ~0ull : (2ull << lane) - 1;
  int64_t running = 0;
  __syncthreads();
  for (int r = 0; r < kItems; r++) {
    const int64_t i = base + r * kBlock + threadIdx.x;
    const bool ok = i < N;
    uint64_t kr = 0, k = 0, kp = 0;
    if (ok) {
      kr = keys[i];
      k = kr & kmask;
      kp = i > 0 ? keys[i - 1] & kmask : 0;
    }
    const bool head = ok && (i == 0 || k != kp);
    const uint64_t bal = __ballot(head);
    if (lane == 0) wsum[wave] = (int32_t)__popcll(bal);
    __syncthreads();
    int64_t pre = running, round_total = 0;
    for (int wv = 0; wv < kWaves; wv++) {
      if (wv < wave) pre += wsum[wv];
      round_total += wsum[wv];
    }
    __syncthreads();
    running += round_total;
    if (ok) {
      const int64_t upto = pre + __popcll(bal & le);  // heads of the tile up to this arc
      if (upto > 0) {
        const ull x = arc_weight(vals, i, kr);
        if (MAXC)
          atomicMax(&acc[upto], x);
        else
          atomicAdd(&acc[upto], x);
      }
      if (head) {
        const int64_t slot = sbase + upto - 1;
        idx[slot] = (int32_t)(k & vmask);
        const int64_t row = (int64_t)(k >> b);
        const int64_t prow = i == 0 ? -1 : (int64_t)(kp >> b);
        for (int64_t rr = prow + 1; rr <= row; rr++) off[rr] = slot;
      }
      if (i == N - 1)
        for (int64_t rr = (int64_t)(k >> b) + 1; rr <= n; rr++) off[rr] = total;
    }
  }
  __syncthreads();
  const bool last_continues = end < N && ((keys[end] ^ keys[end - 1]) & kmask) == 0;
  for (int64_t l = 1 + threadIdx.x; l <= nheads; l += kBlock) {
    ull x = acc[l];
    if (l == nheads && last_continues) {
      for (int64_t t = tile + 1; t < ntiles; t++) {
        const ull y = tile_first[t];
        x = MAXC ? (y > x ? y : x) : x + y;
        if (tile_heads[t] > 0) break;  // the run ends before this tile's first head
      }
    }
    const int64_t slot = sbase + l - 1;
    if (W32) {
      if (x > 0xffffffffull) atomicOr(bad, 4u);
      ((uint32_t*)wout)[slot] = (uint32_t)x;
    } else {
      ((ull*)wout)[slot] = x;
    }
  }
}

}  // namespace

int prep_key_bits(int64_t n) {
  int b = 1;
  while (b < 62 && ((int64_t)1 << b) < n) b++;
  return b;  // every id in [0, n) is below 2^b
}

hipError_t prep_expand(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                       const uint32_t* w, uint32_t flags, int b, uint64_t* keys, uint32_t* vals,
                       unsigned int* bad, hipStream_t s) {
  const int64_t items = m > n ? m : n;
  LV_LAUNCH(k_prep_expand, grid_stride_blocks(items), kBlock, 0, s, n, m, src, dst, w, flags, b,
            keys, vals, bad);
  return hipGetLastError();
}

hipError_t radix_hist(const uint64_t* keys, int64_t N, int shift, int bits, int32_t* hist,
                      hipStream_t s) {
  const int64_t nt = tiles_of(N);
  LV_LAUNCH(k_radix_hist, (unsigned)nt, kBlock, 0, s, keys, N, shift, bits, hist, nt);
  return hipGetLastError();
}

hipError_t radix_scatter(const uint64_t* kin, const uint32_t* vin, uint64_t* kout,
                         uint32_t* vout, int64_t N, int shift, int bits, const int64_t* offs,
                         hipStream_t s) {
  const int64_t nt = tiles_of(N);
  if (vin)
    LV_LAUNCH(k_radix_scatter<true>, (unsigned)nt, kScatterBlock, 0, s, kin, vin, kout, vout, N,
              shift, bits, offs, nt);
  else
    LV_LAUNCH(k_radix_scatter<false>, (unsigned)nt, kScatterBlock, 0, s, kin, vin, kout, vout, N,
              shift, bits, offs, nt);
  return hipGetLastError();
}

hipError_t radix_counts(const uint64_t* keys, int64_t N, const SortPlan& plan,
                        unsigned long long* ghist, int64_t* gbase, hipStream_t s) {
  LV_LAUNCH(k_fill_ull, 1, kBlock, 0, s, ghist, (int64_t)kMaxSortPasses * kBins);
  LV_LAUNCH(k_radix_counts, grid_stride_blocks(N / 4), kBlock, 0, s, keys, N, plan, ghist);
  LV_LAUNCH(k_radix_bases, 1, 64, 0, s, ghist, plan.passes, gbase);
  return hipGetLastError();
}

hipError_t radix_onesweep(const uint64_t* kin, const uint32_t* vin, uint64_t* kout,
                          uint32_t* vout, int64_t N, int shift, int bits, const int64_t* gbase,
                          unsigned long long* status, unsigned int* bad, hipStream_t s) {
  const int64_t nt = tiles_of(N);
  ull* counter = status + nt * kBins;
  LV_LAUNCH(k_fill_ull, grid_stride_blocks(nt * kBins + 1), kBlock, 0, s, status,
            nt * kBins + 1);
  if (vin)
    LV_LAUNCH(k_radix_onesweep<true>, (unsigned)nt, kScatterBlock, 0, s, kin, vin, kout, vout, N,
              shift, bits, gbase, status, counter, bad);
  else
    LV_LAUNCH(k_radix_onesweep<false>, (unsigned)nt, kScatterBlock, 0, s, kin, vin, kout, vout,
              N, shift, bits, gbase, status, counter, bad);
  return hipGetLastError();
}

hipError_t prep_heads(const uint64_t* keys, const uint32_t* vals, int64_t N, int b,
                      bool combine_max, int32_t* tile_heads, unsigned long long* tile_first,
                      hipStream_t s) {
  const unsigned nt = (unsigned)tiles_of(N);
  const uint64_t kmask = (1ull << (2 * b)) - 1;
  if (combine_max)
    LV_LAUNCH(k_prep_heads<true>, nt, kBlock, 0, s, keys, vals, N, kmask, tile_heads, tile_first);
  else
    LV_LAUNCH(k_prep_heads<false>, nt, kBlock, 0, s, keys, vals, N, kmask, tile_heads,
              tile_first);
  return hipGetLastError();
}

hipError_t prep_emit(const uint64_t* keys, const uint32_t* vals, int64_t N, int64_t n, int b,
                     bool combine_max, bool w32, const int64_t* tile_slot,
                     const int32_t* tile_heads, const unsigned long long* tile_first,
                     int64_t* off, int32_t* idx, void* w, unsigned int* bad, hipStream_t s) {
  const int64_t nt = tiles_of(N);
  const uint64_t kmask = (1ull << (2 * b)) - 1;
#define LV_EMIT(M, W)                                                                        \
  LV_LAUNCH((k_prep_emit<M, W>), (unsigned)nt, kBlock, 0, s, keys, vals, N, n, b, kmask,     \
            tile_slot, tile_heads, tile_first, nt, off, idx, w, bad)
  if (combine_max && w32)
    LV_EMIT(true, true);
  else if (combine_max)
    LV_EMIT(true, false);
  else if (w32)
    LV_EMIT(false, true);
  else
    LV_EMIT(false, false);
#undef LV_EMIT
  return hipGetLastError();
}

}  // namespace lv
