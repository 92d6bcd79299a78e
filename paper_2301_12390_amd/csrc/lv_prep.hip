// gfx950 kernels of graph preparation: an edge list becomes the undirected weighted CSR the
// method runs on (section 3.1.2 and Table 1: every edge also taken in reverse, unit weights, a
// self-loop on every vertex; repeated arcs combine into one).
//
// Design: every arc becomes a 64-bit key (source << b | neighbour) with a 32-bit weight. A
// stable LSD radix sort over the 2b significant key bits (8-bit digits, one histogram pass and
// one scatter pass per digit) orders the arcs by row, then by neighbour. One last pass marks
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

inline unsigned grid_stride_blocks(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (unsigned)b;
}

inline int64_t tiles_of(int64_t N) { return (N + kPrepTile - 1) / kPrepTile; }

// Arcs of the edge list: with kPrepSym, edge e gives arcs 2e (u -> v) and 2e+1 (v -> u; for a
// self-loop the second copy has weight 0, so it adds nothing to the one arc a loop stands for);
// with kPrepLoops, arcs base + v are the added loops of weight 1. Bad endpoints set bit 0 of
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
      vals[2 * e] = x;
      keys[2 * e + 1] = (vv << b) | uu;
      vals[2 * e + 1] = u == v ? 0u : x;
    } else {
      keys[e] = (uu << b) | vv;
      vals[e] = x;
    }
  }
  if (flags & kPrepLoops) {
    const int64_t base = sym ? 2 * m : m;
    for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += stride) {
      keys[base + v] = ((uint64_t)v << b) | (uint64_t)v;
      vals[base + v] = 1u;
    }
  }
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

// Stable scatter of one digit. Tile items are ordered (wavefront, round, lane); a lane's rank
// among the equal digits of its wavefront is the wavefront's running count for the digit plus
// the equal lanes below it in the round. offs (exclusive scan of the histogram, digit-major)
// gives every (digit, tile) its output start; earlier wavefronts of the tile come first.
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint64_t* kin, const uint32_t* vin,
                                                         uint64_t* kout, uint32_t* vout,
                                                         int64_t N, int shift, int bits,
                                                         const int64_t* offs, int64_t ntiles) {
  __shared__ int64_t cnt[kWaves][kBins];
  const int bins = 1 << bits;
  for (int i = threadIdx.x; i < kWaves * kBins; i += kBlock) cnt[i / kBins][i % kBins] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t lt = (1ull << lane) - 1;
  const int64_t base = blockIdx.x * kPrepTile + (int64_t)wave * kWaveItems;
  uint64_t key[kItems];
  uint32_t val[kItems];
  int32_t rank[kItems];
#pragma unroll
  for (int r = 0; r < kItems; r++) {
    const int64_t i = base + r * 64 + lane;
    const bool ok = i < N;
    key[r] = ok ? kin[i] : 0;
    val[r] = ok ? vin[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kItems; r++) {
    const int64_t i = base + r * 64 + lane;
    const bool ok = i < N;
    const uint32_t d = (uint32_t)(key[r] >> shift) & (uint32_t)(bins - 1);
    const uint64_t peers = match_digit(d, bits, __ballot(ok));
    // all lanes of the digit read the running count before its leader lane advances it (LDS
    // operations of one wavefront complete in program order)
    const int64_t before = ok ? cnt[wave][d] : 0;
    rank[r] = (int32_t)(before + __popcll(peers & lt));
    if (ok && (peers & lt) == 0) cnt[wave][d] = before + __popcll(peers);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < bins; d += kBlock) {
    int64_t run = offs[(int64_t)d * ntiles + blockIdx.x];
    for (int wv = 0; wv < kWaves; wv++) {
      const int64_t c = cnt[wv][d];
      cnt[wv][d] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kItems; r++) {
    const int64_t i = base + r * 64 + lane;
    if (i < N) {
      const uint32_t d = (uint32_t)(key[r] >> shift) & (uint32_t)(bins - 1);
      const int64_t pos = cnt[wave][d] + rank[r];
      kout[pos] = key[r];
      vout[pos] = val[r];
    }
  }
}

// Heads (first arc of a run of equal keys) per tile.
__global__ __launch_bounds__(kBlock) void k_prep_heads(const uint64_t* keys, int64_t N,
                                                      int32_t* tile_heads) {
  __shared__ ull red[kBlock / 64];
  const int64_t base = blockIdx.x * kPrepTile;
  ull c = 0;
  for (int r = 0; r < kItems; r++) {
    const int64_t i = base + r * kBlock + threadIdx.x;
    if (i < N && (i == 0 || keys[i] != keys[i - 1])) c++;
  }
  c = block_sum_u64(c, red);
  if (threadIdx.x == 0) tile_heads[blockIdx.x] = (int32_t)c;
}

// The CSR from the sorted arcs. tile_slot: exclusive scan of the heads per tile ([ntiles+1],
// the last entry the arc count). A head's slot is tile_slot[tile] + (heads of the tile up to and
// including it) - 1; the arcs before a tile's first head continue the previous tile's last run
// (local slot 0). Weights combine per local slot in LDS; a run crossing a tile edge is combined
// across tiles with global atomics (w must be zero there), the others are stored. Offsets: the
// head that starts row r (after rows prow+1..r-1 without arcs) writes off[prow+1..r]; the last
// arc writes the rows after its own.
template <bool MAXC>
__global__ __launch_bounds__(kBlock) void k_prep_emit(const uint64_t* keys, const uint32_t* vals,
                                                     int64_t N, int64_t n, int b,
                                                     const int64_t* tile_slot, int64_t ntiles,
                                                     int64_t* off, int32_t* idx, ull* w) {
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
    uint64_t k = 0, kp = 0;
    if (ok) {
      k = keys[i];
      kp = i > 0 ? keys[i - 1] : 0;
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
      if (MAXC)
        atomicMax(&acc[upto], (ull)vals[i]);
      else
        atomicAdd(&acc[upto], (ull)vals[i]);
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
  const bool first_is_head = base == 0 || keys[base] != keys[base - 1];
  const bool last_continues = end < N && keys[end] == keys[end - 1];
  for (int64_t l = threadIdx.x; l <= nheads; l += kBlock) {
    if (l == 0 && first_is_head) continue;  // no run continues into this tile
    const int64_t slot = sbase + l - 1;
    const bool shared = l == 0 || (l == nheads && last_continues);
    if (!shared)
      w[slot] = acc[l];
    else if (MAXC)
      atomicMax(&w[slot], acc[l]);
    else
      atomicAdd(&w[slot], acc[l]);
  }
}

__global__ void k_prep_narrow_w(const ull* w, uint32_t* out, int64_t nnz, unsigned int* bad) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nnz;
       i += (int64_t)gridDim.x * blockDim.x) {
    const ull x = w[i];
    if (x > 0xffffffffull) atomicOr(bad, 4u);
    out[i] = (uint32_t)x;
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
  LV_LAUNCH(k_radix_scatter, (unsigned)nt, kBlock, 0, s, kin, vin, kout, vout, N, shift, bits,
            offs, nt);
  return hipGetLastError();
}

hipError_t prep_heads(const uint64_t* keys, int64_t N, int32_t* tile_heads, hipStream_t s) {
  LV_LAUNCH(k_prep_heads, (unsigned)tiles_of(N), kBlock, 0, s, keys, N, tile_heads);
  return hipGetLastError();
}

hipError_t prep_emit(const uint64_t* keys, const uint32_t* vals, int64_t N, int64_t n, int b,
                     bool combine_max, const int64_t* tile_slot, int64_t* off, int32_t* idx,
                     unsigned long long* w, hipStream_t s) {
  const int64_t nt = tiles_of(N);
  if (combine_max)
    LV_LAUNCH(k_prep_emit<true>, (unsigned)nt, kBlock, 0, s, keys, vals, N, n, b, tile_slot, nt,
              off, idx, w);
  else
    LV_LAUNCH(k_prep_emit<false>, (unsigned)nt, kBlock, 0, s, keys, vals, N, n, b, tile_slot, nt,
              off, idx, w);
  return hipGetLastError();
}

hipError_t prep_narrow_weights(const unsigned long long* w, uint32_t* out, int64_t nnz,
                               unsigned int* bad, hipStream_t s) {
  LV_LAUNCH(k_prep_narrow_w, grid_stride_blocks(nnz), kBlock, 0, s, w, out, nnz, bad);
  return hipGetLastError();
}

}  // namespace lv
