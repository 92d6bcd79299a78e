// gfx950 kernels of the Louvain library: pass set-up, degree classes, the synchronous
// local-moving iteration, community updates, modularity pieces and aggregation.
//
// Method: section 3.2 of Sahu, arXiv 2301.12390 (local-moving phase, aggregation phase,
// synchronous vs asynchronous variants, per-worker hashtables of community -> weight).
#include <hip/hip_runtime.h>

#include "lv_device.h"
#include "lv_internal.h"

namespace lv {

static inline unsigned grid_for(int64_t n, int64_t per_block = kBlock, int64_t cap = 16384) {
  int64_t b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

#define LV_LAUNCH(kernel, grid, block, shm, stream, ...)                          \
  do {                                                                            \
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shm, stream, __VA_ARGS__); \
  } while (0)

// =============================================================================================
// Elementwise

__global__ void k_fill_u64(uint64_t* a, uint64_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}
__global__ void k_fill_i32(int32_t* a, int32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}
__global__ void k_fill_i64(int64_t* a, int64_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}
__global__ void k_iota_i32(int32_t* a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = (int32_t)i;
}
__global__ void k_copy_i64(int64_t* d, const int64_t* s, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}
__global__ void k_widen_offsets(const int32_t* in, int64_t* out, int64_t m) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (int64_t)in[i];
}
__global__ void k_narrow_offsets(const int64_t* in, int32_t* out, int64_t m) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (int32_t)in[i];
}
__global__ void k_widen_weights(const uint32_t* in, uint64_t* out, int64_t m) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (uint64_t)in[i];
}

hipError_t fill_u64(uint64_t* a, uint64_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_fill_u64, grid_for(n), kBlock, 0, s, a, v, n);
  return hipGetLastError();
}
hipError_t fill_i32(int32_t* a, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_fill_i32, grid_for(n), kBlock, 0, s, a, v, n);
  return hipGetLastError();
}
hipError_t fill_i64(int64_t* a, int64_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_fill_i64, grid_for(n), kBlock, 0, s, a, v, n);
  return hipGetLastError();
}
hipError_t iota_i32(int32_t* a, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_iota_i32, grid_for(n), kBlock, 0, s, a, n);
  return hipGetLastError();
}
hipError_t copy_i64(int64_t* d, const int64_t* src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_copy_i64, grid_for(n), kBlock, 0, s, d, src, n);
  return hipGetLastError();
}
hipError_t widen_offsets(const int32_t* in, int64_t* out, int64_t m, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  LV_LAUNCH(k_widen_offsets, grid_for(m), kBlock, 0, s, in, out, m);
  return hipGetLastError();
}
hipError_t narrow_offsets(const int64_t* in, int32_t* out, int64_t m, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  LV_LAUNCH(k_narrow_offsets, grid_for(m), kBlock, 0, s, in, out, m);
  return hipGetLastError();
}
hipError_t widen_weights(const uint32_t* in, uint64_t* out, int64_t m, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  LV_LAUNCH(k_widen_weights, grid_for(m), kBlock, 0, s, in, out, m);
  return hipGetLastError();
}

__global__ void k_zero_words(ull* a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0;
}
hipError_t zero_words(ull* a, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_zero_words, grid_for(n), kBlock, 0, s, a, n);
  return hipGetLastError();
}

// =============================================================================================
// Reductions over vertex arrays

// One atomic of each kind per block: per-wave atomics on the two words contend at the memory
// side once there are thousands of blocks.
__global__ __launch_bounds__(kBlock) void k_sum_max(const uint64_t* a, int64_t n, ull* out) {
  __shared__ ull red[kBlock / 64];
  __shared__ ull wmax[kBlock / 64];
  ull sum = 0, mx = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    ull v = a[i];
    sum += v;
    mx = v > mx ? v : mx;
  }
  ull bs = block_sum_u64(sum, red);
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    ull o = __shfl_xor(mx, m, 64);
    mx = o > mx ? o : mx;
  }
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; w++) mx = wmax[w] > mx ? wmax[w] : mx;
    if (mx) atomicMax(&out[1], mx);
    if (bs) atomicAdd(&out[0], bs);
  }
}
hipError_t sum_max_u64(const uint64_t* a, int64_t n, ull* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_sum_max, grid_for(n, kBlock, 1024), kBlock, 0, s, a, n, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_sum_squares(const uint64_t* a, int64_t n, ull* out) {
  __shared__ u128 red[kBlock / 64];
  u128 sum = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    u128 v = a[i];
    sum += v * v;
  }
  u128 bs = block_sum_u128(sum, red);
  if (threadIdx.x == 0 && bs) atomic_add_u128(out, bs);
}
hipError_t sum_squares_u64(const uint64_t* a, int64_t n, ull* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_sum_squares, grid_for(n, kBlock, 1024), kBlock, 0, s, a, n, out);
  return hipGetLastError();
}

// out[0..1] += the 128-bit sum of all arc weights. Row sums and W are 64-bit words; this exact
// total tells the host whether any of them could have wrapped (they cannot when it is <= 2^62).
template <typename WT>
__global__ __launch_bounds__(kBlock) void k_total_weight(const WT* w, int64_t nnz, ull* out) {
  __shared__ u128 red[kBlock / 64];
  u128 acc = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x)
    acc += (u128)ld_stream(w + e);
  acc = block_sum_u128(acc, red);
  if (threadIdx.x == 0 && acc) atomic_add_u128(out, acc);
}
hipError_t total_weight_u128(const DevGraph& g, ull* out, hipStream_t s) {
  if (g.nnz <= 0) return hipSuccess;
  if (g.w64)
    LV_LAUNCH(k_total_weight<uint64_t>, grid_for(g.nnz, kBlock, 4096), kBlock, 0, s,
              (const uint64_t*)g.w, g.nnz, out);
  else
    LV_LAUNCH(k_total_weight<uint32_t>, grid_for(g.nnz, kBlock, 4096), kBlock, 0, s,
              (const uint32_t*)g.w, g.nnz, out);
  return hipGetLastError();
}

template <typename WT>
__global__ void k_validate(const int64_t* off, int64_t n, int64_t nnz, const int32_t* idx,
                           const WT* w, unsigned int* bad) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (off[i + 1] < off[i]) atomicOr(bad, 1u);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    int32_t j = idx[e];
    if (j < 0 || (int64_t)j >= n) atomicOr(bad, 2u);
    if (w[e] == 0) atomicOr(bad, 4u);
  }
}
hipError_t validate_graph(const DevGraph& g, unsigned int* bad, hipStream_t s) {
  int64_t m = g.n > g.nnz ? g.n : g.nnz;
  if (m <= 0) return hipSuccess;
  if (g.w64)
    LV_LAUNCH(k_validate<uint64_t>, grid_for(m), kBlock, 0, s, g.off, g.n, g.nnz, g.idx,
              (const uint64_t*)g.w, bad);
  else
    LV_LAUNCH(k_validate<uint32_t>, grid_for(m), kBlock, 0, s, g.off, g.n, g.nnz, g.idx,
              (const uint32_t*)g.w, bad);
  return hipGetLastError();
}

// =============================================================================================
// Exclusive scan (reduce, scan the block partials, rescan with offsets). Each block covers
// kScanTile consecutive elements, kScanItems per thread.

constexpr int kScanItems = 8;
constexpr int64_t kScanTile = (int64_t)kBlock * kScanItems;

int64_t scan_partial_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

struct ReadI64 {
  const int64_t* a;
  __device__ int64_t operator()(int64_t i) const { return a[i]; }
};
struct ReadPos {
  const int32_t* a;
  __device__ int64_t operator()(int64_t i) const { return a[i] > 0 ? 1 : 0; }
};
struct ReadI32 {
  const int32_t* a;
  __device__ int64_t operator()(int64_t i) const { return (int64_t)a[i]; }
};
// Degree of the member in slot p, 0 past the last member (*count slots are filled).
struct ReadMemberDegGuard {
  const int32_t* members;
  const int64_t* rs;
  const int64_t* re;
  const int64_t* count;
  __device__ int64_t operator()(int64_t p) const {
    if (p >= *count) return 0;
    const int32_t v = members[p];
    return re[v] - rs[v];
  }
};

template <typename F>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(F f, int64_t n, int64_t* partial) {
  __shared__ ull red[kBlock / 64];
  const int64_t base = blockIdx.x * kScanTile;
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; k++) {
    int64_t i = base + k * kBlock + threadIdx.x;
    if (i < n) s += f(i);
  }
  ull t = block_sum_u64((ull)s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = (int64_t)t;
}

// Inclusive scan of one value per thread across the block; returns the exclusive prefix and
// the block total.
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t x, int64_t* total, int64_t* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t inc = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int64_t y = __shfl_up(inc, d, 64);
    if (lane >= d) inc += y;
  }
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  int64_t wbase = 0, tot = 0;
  for (int i = 0; i < kBlock / 64; i++) {
    if (i < wave) wbase += sh[i];
    tot += sh[i];
  }
  __syncthreads();
  *total = tot;
  return wbase + inc - x;
}

// Single block: exclusive scan of partial[0..nb) in place, partial[nb] = total.
__global__ __launch_bounds__(kBlock) void k_scan_partials(int64_t* partial, int64_t nb) {
  __shared__ int64_t sh[kBlock / 64];
  int64_t carry = 0;
  for (int64_t base = 0; base < nb; base += kBlock) {
    int64_t i = base + threadIdx.x;
    int64_t x = i < nb ? partial[i] : 0;
    int64_t tot;
    int64_t ex = block_exclusive_scan(x, &tot, sh);
    if (i < nb) partial[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) partial[nb] = carry;
}

template <typename F>
__global__ __launch_bounds__(kBlock) void k_scan_apply(F f, int64_t n, const int64_t* partial,
                                                       int64_t* out) {
  __shared__ int64_t sh[kBlock / 64];
  const int64_t base = blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; k++) {
    int64_t i = base + k;
    v[k] = i < n ? f(i) : 0;
    s += v[k];
  }
  int64_t tot;
  int64_t ex = block_exclusive_scan(s, &tot, sh) + partial[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; k++) {
    int64_t i = base + k;
    if (i < n) out[i] = ex;
    ex += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = partial[gridDim.x];
}

template <typename F>
static hipError_t scan_impl(F f, int64_t n, int64_t* out, int64_t* partial, hipStream_t s) {
  if (n <= 0) {
    LV_LAUNCH(k_fill_i64, 1, 1, 0, s, out, (int64_t)0, (int64_t)1);
    return hipGetLastError();
  }
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  LV_LAUNCH(k_scan_reduce<F>, (unsigned)nb, kBlock, 0, s, f, n, partial);
  LV_LAUNCH(k_scan_partials, 1, kBlock, 0, s, partial, nb);
  LV_LAUNCH(k_scan_apply<F>, (unsigned)nb, kBlock, 0, s, f, n, partial, out);
  return hipGetLastError();
}

hipError_t scan_i64(const int64_t* x, int64_t n, int64_t* out, int64_t* partial, hipStream_t s) {
  return scan_impl(ReadI64{x}, n, out, partial, s);
}
hipError_t scan_i32(const int32_t* x, int64_t n, int64_t* out, int64_t* partial, hipStream_t s) {
  return scan_impl(ReadI32{x}, n, out, partial, s);
}
hipError_t scan_flags_pos(const int32_t* x, int64_t n, int64_t* out, int64_t* partial,
                          hipStream_t s) {
  return scan_impl(ReadPos{x}, n, out, partial, s);
}

// =============================================================================================
// Largest member index i in [0, mc) with start[i] <= t (start[0] = 0 <= t).
template <typename T>
__device__ __forceinline__ int member_at(const T* start, int mc, int64_t t) {
  int lo = 0, hi = mc;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)start[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

// Largest member index i in [lo, hi) with start[i] <= t, given start[lo] <= t.
template <typename T>
__device__ __forceinline__ int member_in(const T* start, int lo, int hi, int64_t t) {
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)start[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

// Arc-segment kernels: thread t covers arcs [t*kSeg, (t+1)*kSeg), finds the row of its first
// arc by binary search over the offsets and walks forward. Work is balanced by arcs, so hub
// rows do not serialise on one thread.

constexpr int64_t kSeg = 16;

// Row sums: workgroup b sums the arcs of its range [lo, hi) of kRowTile arcs, attributing them
// to the rows they belong to: up to kShortRow arcs of a row one per thread, longer stretches one
// per wavefront (coalesced). A row lying wholly inside the range is stored; the (at most two)
// rows crossing its ends are added atomically. K must be zero (rows of no arcs keep 0).
constexpr int64_t kRowTile = 4096;
constexpr int64_t kShortRow = 32;

// tile_rows[t] = the row holding arc t * kRowTile, for every tile t (each arc lies in exactly
// one non-empty row, so every tile gets one writer); tile_rows[tiles] = n - 1.
__global__ __launch_bounds__(kBlock) void k_tile_rows(const int64_t* off, int64_t n,
                                                     int64_t tiles, int64_t* tile_rows) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b0 = off[r], b1 = off[r + 1];
    if (b1 <= b0) continue;
    const int64_t t1 = (b1 + kRowTile - 1) / kRowTile;
    for (int64_t t = (b0 + kRowTile - 1) / kRowTile; t < t1; t++) tile_rows[t] = r;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) tile_rows[tiles] = n - 1;
}

// The rows a tile touches run from tile_rows[b] to tile_rows[b + 1] (that last one may start
// at the next tile and then contributes nothing here). With SELF, selfw[r] receives the weight
// of row r's self-loops the same way (one more coalesced read, of the indices).
template <typename WT, bool SELF>
__global__ __launch_bounds__(kBlock) void k_row_sums(const int64_t* off, int64_t nnz,
                                                    const int64_t* tile_rows, const WT* w,
                                                    const int32_t* idx, uint64_t* K,
                                                    uint64_t* selfw) {
  __shared__ int64_t span[2];
  __shared__ int64_t longs[kRowTile / kShortRow + 2];
  __shared__ int nlong;
  const int64_t lo = (int64_t)blockIdx.x * kRowTile;
  const int64_t hi = lo + kRowTile < nnz ? lo + kRowTile : nnz;
  if (threadIdx.x < 2) span[threadIdx.x] = tile_rows[blockIdx.x + threadIdx.x];
  if (threadIdx.x == 0) nlong = 0;
  __syncthreads();
  for (int64_t r = span[0] + threadIdx.x; r <= span[1]; r += kBlock) {
    const int64_t b0 = off[r], b1 = off[r + 1];
    const int64_t e0 = b0 > lo ? b0 : lo, e1 = b1 < hi ? b1 : hi;
    if (e1 <= e0) continue;
    if (e1 - e0 > kShortRow) {
      longs[atomicAdd(&nlong, 1)] = r;
      continue;
    }
    // up to kSumBatch loads in flight per thread (a row's arcs are read in turn, not by
    // neighbouring lanes, so each thread hides its own latency)
    constexpr int kSumBatch = 8;
    ull acc = 0, sl = 0;
    for (int64_t e = e0; e < e1; e += kSumBatch) {
      ull x[kSumBatch];
      int32_t j[kSumBatch];
#pragma unroll
      for (int q = 0; q < kSumBatch; q++) {
        x[q] = e + q < e1 ? (ull)w[e + q] : 0;
        if (SELF) j[q] = e + q < e1 ? idx[e + q] : -1;
      }
#pragma unroll
      for (int q = 0; q < kSumBatch; q++) {
        acc += x[q];
        if (SELF && j[q] == (int32_t)r) sl += x[q];
      }
    }
    if (b0 >= lo && b1 <= hi) {
      K[r] = acc;
      if (SELF) selfw[r] = sl;
    } else {
      atomicAdd((ull*)&K[r], acc);
      if (SELF && sl) atomicAdd((ull*)&selfw[r], sl);
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = wave; i < nlong; i += kBlock / 64) {
    const int64_t r = longs[i];
    const int64_t b0 = off[r], b1 = off[r + 1];
    const int64_t e0 = b0 > lo ? b0 : lo, e1 = b1 < hi ? b1 : hi;
    constexpr int kWaveBatch = 8;  // loads in flight per lane
    ull acc = 0, sl = 0;
    for (int64_t e = e0 + lane; e < e1; e += 64 * kWaveBatch) {
      ull x[kWaveBatch];
      int32_t j[kWaveBatch];
#pragma unroll
      for (int q = 0; q < kWaveBatch; q++) {
        const int64_t eq = e + 64 * q;
        x[q] = eq < e1 ? (ull)ld_stream(w + eq) : 0;
        if (SELF) j[q] = eq < e1 ? ld_stream(idx + eq) : -1;
      }
#pragma unroll
      for (int q = 0; q < kWaveBatch; q++) {
        acc += x[q];
        if (SELF && j[q] == (int32_t)r) sl += x[q];
      }
    }
    acc = group_sum_u64<64>(acc);
    if (SELF) sl = group_sum_u64<64>(sl);
    if (lane == 0) {
      if (b0 >= lo && b1 <= hi) {
        K[r] = acc;
        if (SELF) selfw[r] = sl;
      } else {
        atomicAdd((ull*)&K[r], acc);
        if (SELF && sl) atomicAdd((ull*)&selfw[r], sl);
      }
    }
  }
}

int64_t row_sum_tiles(int64_t nnz) { return (nnz + kRowTile - 1) / kRowTile; }

hipError_t row_sums(const DevGraph& g, uint64_t* K, int64_t* tile_rows, hipStream_t s,
                    uint64_t* selfw) {
  if (g.nnz <= 0) return hipSuccess;
  const int64_t tiles = row_sum_tiles(g.nnz);
  LV_LAUNCH(k_tile_rows, grid_for(g.n), kBlock, 0, s, g.off, g.n, tiles, tile_rows);
  const unsigned grid = (unsigned)tiles;
  if (g.w64) {
    if (selfw)
      LV_LAUNCH((k_row_sums<uint64_t, true>), grid, kBlock, 0, s, g.off, g.nnz, tile_rows,
                (const uint64_t*)g.w, g.idx, K, selfw);
    else
      LV_LAUNCH((k_row_sums<uint64_t, false>), grid, kBlock, 0, s, g.off, g.nnz, tile_rows,
                (const uint64_t*)g.w, g.idx, K, selfw);
  } else {
    if (selfw)
      LV_LAUNCH((k_row_sums<uint32_t, true>), grid, kBlock, 0, s, g.off, g.nnz, tile_rows,
                (const uint32_t*)g.w, g.idx, K, selfw);
    else
      LV_LAUNCH((k_row_sums<uint32_t, false>), grid, kBlock, 0, s, g.off, g.nnz, tile_rows,
                (const uint32_t*)g.w, g.idx, K, selfw);
  }
  return hipGetLastError();
}

// Weight of the arcs whose endpoints share a label (C == nullptr: self-loops).
template <typename WT>
__global__ __launch_bounds__(kBlock) void k_intra_weight(const int64_t* off, int64_t n,
                                                        int64_t nnz, const int32_t* idx,
                                                        const WT* w, const int32_t* C,
                                                        ull* out) {
  __shared__ ull red[kBlock / 64];
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t e0 = t * kSeg;
  ull acc = 0;
  if (e0 < nnz) {
    const int64_t e1 = e0 + kSeg < nnz ? e0 + kSeg : nnz;
    int64_t r = row_of_arc(off, n, e0);
    int64_t rend = off[r + 1];
    int32_t cr = C ? C[r] : (int32_t)r;
    for (int64_t e = e0; e < e1; e++) {
      if (e >= rend) {
        r = advance_row(off, n, r + 1, e);
        rend = off[r + 1];
        cr = C ? C[r] : (int32_t)r;
      }
      const int32_t j = idx[e];
      const int32_t cj = C ? C[j] : j;
      if (cj == cr) acc += (ull)w[e];
    }
  }
  ull b = block_sum_u64(acc, red);
  if (threadIdx.x == 0 && b) atomicAdd(out, b);
}

hipError_t intra_weight(const DevGraph& g, const int32_t* C, ull* out, hipStream_t s) {
  if (g.nnz <= 0) return hipSuccess;
  const int64_t threads = (g.nnz + kSeg - 1) / kSeg;
  const unsigned grid = (unsigned)((threads + kBlock - 1) / kBlock);
  if (g.w64)
    LV_LAUNCH(k_intra_weight<uint64_t>, grid, kBlock, 0, s, g.off, g.n, g.nnz, g.idx,
              (const uint64_t*)g.w, C, out);
  else
    LV_LAUNCH(k_intra_weight<uint32_t>, grid, kBlock, 0, s, g.off, g.n, g.nnz, g.idx,
              (const uint32_t*)g.w, C, out);
  return hipGetLastError();
}

__global__ void k_sigma_by_label(const uint64_t* K, const int32_t* C, int64_t n, uint64_t* Sig) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (K[i]) atomicAdd((ull*)&Sig[C[i]], (ull)K[i]);
}
hipError_t sigma_by_label(const uint64_t* K, const int32_t* C, int64_t n, uint64_t* Sig,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_sigma_by_label, grid_for(n), kBlock, 0, s, K, C, n, Sig);
  return hipGetLastError();
}

__global__ void k_count_labels(const int32_t* C, int64_t n, int32_t* csize) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&csize[C[i]], 1);
}
hipError_t count_labels(const int32_t* C, int64_t n, int32_t* csize, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_count_labels, grid_for(n), kBlock, 0, s, C, n, csize);
  return hipGetLastError();
}

// =============================================================================================
// Pass set-up: every vertex its own community (section 3.2).

__global__ void k_init_state(int64_t n, const uint64_t* K, VRec* rec, int32_t* lab) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    VRec r;
    r.c = (int32_t)i;
    r.size = 1;
    r.sig = K[i];
    rec[i] = r;
    if (lab) lab[i] = (int32_t)i;
  }
}
hipError_t init_state(int64_t n, const uint64_t* K, void* rec, int32_t* lab, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_init_state, grid_for(n), kBlock, 0, s, n, K, (VRec*)rec, lab);
  return hipGetLastError();
}

__global__ void k_pack_state(int64_t n, const int32_t* C, const uint64_t* Sig,
                             const int32_t* csize, VRec* rec) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    VRec r;
    r.c = C[i];
    r.size = csize[i];
    r.sig = Sig[i];
    rec[i] = r;
  }
}
__global__ void k_unpack_state(int64_t n, const VRec* rec, int32_t* C, uint64_t* Sig,
                               int32_t* csize) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const VRec r = rec[i];
    C[i] = r.c;
    csize[i] = r.size;
    Sig[i] = r.sig;
  }
}
hipError_t pack_state(int64_t n, const int32_t* C, const uint64_t* Sig, const int32_t* csize,
                      void* rec, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_pack_state, grid_for(n), kBlock, 0, s, n, C, Sig, csize, (VRec*)rec);
  return hipGetLastError();
}
hipError_t unpack_state(int64_t n, const void* rec, int32_t* C, uint64_t* Sig, int32_t* csize,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_unpack_state, grid_for(n), kBlock, 0, s, n, (const VRec*)rec, C, Sig, csize);
  return hipGetLastError();
}

// =============================================================================================
// Degree classes. Items with length 0 (isolated vertices, empty communities) are skipped: an
// isolated vertex has no neighbour community to move to.

__device__ __forceinline__ int64_t item_len(const int64_t* rs, const int64_t* re,
                                            const int64_t* len, int64_t i) {
  return len ? len[i] : re[i] - rs[i];
}

// Segment of item i: kDegClasses * (vertex class) + degree class.
constexpr int kMaxSeg = kDegClasses * kMaxClasses;

// Vertex classes hash the id of a vertex within its own graph: i - gbase[gid[i]] in a batch of
// graphs packed with consecutive ids (gid null: one graph). In a batch, rows of graphs that are
// not iterating (act[gid[i]] == 0) are left out of the lists.
// vclass (may be null): the class of every vertex given (colour classes), instead of the hash.
__device__ __forceinline__ int segment_of(int64_t L, int K, int pass, int64_t i,
                                          const int32_t* gid, const int64_t* gbase,
                                          const uint8_t* vclass) {
  int k = 0;
  if (vclass) {
    k = vclass[i];
  } else if (K > 1) {
    const int64_t loc = gid ? i - gbase[gid[i]] : i;
    k = vertex_class(pass, K, loc);
  }
  return kDegClasses * k + bucket_of(L);
}

// counts[0 .. nseg): items per segment, counts[kMaxSeg .. kMaxSeg + nseg): total length.
__device__ __forceinline__ bool listed(int64_t L, int64_t i, const int32_t* gid,
                                       const uint8_t* act) {
  return L > 0 && (!act || act[gid[i]]);
}

__global__ __launch_bounds__(kBlock) void k_bucket_count(const int64_t* rs, const int64_t* re,
                                                        const int64_t* len, int64_t m, int K,
                                                        int pass, const int32_t* gid,
                                                        const int64_t* gbase, const uint8_t* act,
                                                        const uint8_t* vclass, ull* counts) {
  __shared__ ull c[2 * kMaxSeg];
  const int nseg = kDegClasses * K;
  for (int t = threadIdx.x; t < 2 * kMaxSeg; t += blockDim.x) c[t] = 0;
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t L = item_len(rs, re, len, i);
    if (listed(L, i, gid, act)) {
      const int sg = segment_of(L, K, pass, i, gid, gbase, vclass);
      atomicAdd(&c[sg], 1ull);
      atomicAdd(&c[kMaxSeg + sg], (ull)L);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nseg; t += blockDim.x) {
    if (c[t]) atomicAdd(&counts[t], c[t]);
    if (c[kMaxSeg + t]) atomicAdd(&counts[kMaxSeg + t], c[kMaxSeg + t]);
  }
}

// starts: first list position per segment; cursor: per-segment fill counters (zero). A block
// ranks a chunk of kFillItems items per thread in LDS and then claims each segment's share of
// the chunk with one global atomic, so that the few segment cursors are not hit once per tile
// of every block.
constexpr int kFillItems = 16;
__global__ __launch_bounds__(kBlock) void k_bucket_fill(const int64_t* rs, const int64_t* re,
                                                       const int64_t* len, int64_t m, int K,
                                                       int pass, const int32_t* gid,
                                                       const int64_t* gbase, const uint8_t* act,
                                                       const uint8_t* vclass, const ull* starts,
                                                       ull* cursor, int32_t* list) {
  __shared__ int cnt[kMaxSeg];
  __shared__ ull base[kMaxSeg];
  const int nseg = kDegClasses * K;
  constexpr int64_t kChunk = (int64_t)kBlock * kFillItems;
  for (int64_t c0 = (int64_t)blockIdx.x * kChunk; c0 < m; c0 += (int64_t)gridDim.x * kChunk) {
    for (int t = threadIdx.x; t < nseg; t += blockDim.x) cnt[t] = 0;
    __syncthreads();
    int sg[kFillItems], rank[kFillItems];
#pragma unroll
    for (int u = 0; u < kFillItems; u++) {
      const int64_t i = c0 + (int64_t)u * kBlock + threadIdx.x;
      sg[u] = -1;
      rank[u] = 0;
      if (i < m) {
        const int64_t L = item_len(rs, re, len, i);
        if (listed(L, i, gid, act)) {
          sg[u] = segment_of(L, K, pass, i, gid, gbase, vclass);
          rank[u] = atomicAdd(&cnt[sg[u]], 1);
        }
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nseg; t += blockDim.x)
      if (cnt[t]) base[t] = atomicAdd(&cursor[t], (ull)cnt[t]);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kFillItems; u++)
      if (sg[u] >= 0)
        list[(int64_t)starts[sg[u]] + (int64_t)base[sg[u]] + rank[u]] =
            (int32_t)(c0 + (int64_t)u * kBlock + threadIdx.x);
    __syncthreads();
  }
}

hipError_t bucket_rows(const int64_t* rs, const int64_t* re, const int64_t* len, int64_t m,
                       int K, int pass, const int32_t* gid, const int64_t* gbase,
                       const uint8_t* act, const uint8_t* vclass, int32_t* list, ull* counts,
                       ull* host_counts, Buckets& b, hipStream_t s) {
  b = Buckets();
  b.classes = K;
  if (m <= 0) return hipSuccess;
  const int nseg = kDegClasses * K;
  // counts layout (kMaxSeg words each): items, lengths, fill cursors, segment starts
  LV_LAUNCH(k_zero_words, 8, kBlock, 0, s, counts, (int64_t)(3 * kMaxSeg));
  LV_LAUNCH(k_bucket_count, grid_for(m, kBlock, 4096), kBlock, 0, s, rs, re, len, m, K, pass,
            gid, gbase, act, vclass, counts);
  hipError_t e = hipMemcpyAsync(host_counts, counts, 2 * kMaxSeg * sizeof(ull),
                                hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  int64_t acc = 0;
  ull* hstarts = host_counts + 3 * kMaxSeg;
  for (int sg = 0; sg < nseg; sg++) {
    b.count[sg] = (int64_t)host_counts[sg];
    b.arcs[sg] = (int64_t)host_counts[kMaxSeg + sg];
    b.lstart[sg] = acc;
    hstarts[sg] = (ull)acc;
    acc += b.count[sg];
  }
  b.lstart[nseg] = acc;
  if (acc == 0) return hipSuccess;
  e = hipMemcpyAsync(counts + 3 * kMaxSeg, hstarts, nseg * sizeof(ull), hipMemcpyHostToDevice,
                     s);
  if (e != hipSuccess) return e;
  LV_LAUNCH(k_bucket_fill, grid_for(m, (int64_t)kBlock * kFillItems, 8192), kBlock, 0, s, rs,
            re, len, m, K, pass,
            gid, gbase, act, vclass, counts + 3 * kMaxSeg, counts + 2 * kMaxSeg, list);
  return hipGetLastError();
}

// Two-phase decomposition of long items (see part_chunk). Per item of length L whose keys take
// at most min(L, cap) distinct values: nck = ceil(L / Q) chunks, walked by phase-1 workgroups of
// R consecutive chunks each (R grows with nck so that an item has at most kPartBlocksPerItem of
// them); P partitions (a power of two, at most kMaxParts, sized for (table / 2) >> shift keys
// each; 1 if the item is one chunk); nck * (P + 1) segment bounds (one row per chunk, of which
// a workgroup uses one per table flush); and the phase-2 workgroups (none for a one-chunk item
// of the aggregation, which phase 1 finishes by itself).
constexpr int64_t kPartBlocksPerItem = 256;

struct PartSizes {
  int64_t c, R, nblk, P, hsz, p2;
};

__device__ __forceinline__ PartSizes part_sizes_of(int64_t L, int64_t cap, int vb, int merge,
                                                   int shift) {
  const int64_t Q = part_chunk(vb);
  const int64_t T = (((int64_t)1 << part_log2h(vb)) / 2) >> shift;
  PartSizes z;
  z.c = (L + Q - 1) / Q;
  const int64_t per = shift ? 4 : kPartBlocksPerItem;  // testing: several chunks per walker
  z.R = (z.c + per - 1) / per;
  const int64_t D = L < cap ? L : cap;
  z.P = 1;
  if (z.c > 1)
    while (z.P * T < D && z.P < kMaxParts) z.P <<= 1;
  z.nblk = (z.c + z.R - 1) / z.R;
  z.hsz = z.c * (z.P + 1);
  z.p2 = (merge && z.c == 1) ? 0 : z.P;
  return z;
}

// The plans of up to kPlanBatch item lists in one launch, one 1024-thread workgroup per list:
// the sizes of k_part_sizes and the four exclusive scans of plan_parts (chunk, walker,
// partition and bound-row starts), in tiles of 1024 items with a running carry. The four totals
// of list k go to totals[4k .. 4k + 4).
constexpr int kPlanBatch = 32;
constexpr int kPlanBlock = 1024;
struct PlanBatchArgs {
  const int64_t* rs;
  const int64_t* re;
  const int64_t* len;
  const int32_t* items[kPlanBatch];
  int64_t nh[kPlanBatch];
  int64_t* arrays[kPlanBatch];
  int64_t* totals;
  int64_t cap;
  int vb, merge, shift;
};
static_assert(sizeof(PlanBatchArgs) <= 1024, "kernel arguments");

__global__ __launch_bounds__(kPlanBlock) void k_plan_batch(PlanBatchArgs a) {
  constexpr int NW = kPlanBlock / 64;
  __shared__ int64_t wtot[4][NW + 1];
  __shared__ int64_t carry[4];
  const int k = blockIdx.x;
  const int64_t nh = a.nh[k];
  int64_t* arr = a.arrays[k];
  int64_t* nck = arr;
  int64_t* nblk = arr + nh;
  int64_t* hsz = arr + 2 * nh;
  int64_t* p2 = arr + 3 * nh;
  int64_t* rper = arr + 4 * nh;
  int64_t* nparts = arr + 5 * nh;
  int64_t* st[4] = {arr + 6 * nh, arr + 7 * nh + 1, arr + 8 * nh + 2, arr + 9 * nh + 3};
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x < 4) carry[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t base = 0; base < nh; base += kPlanBlock) {  // block-uniform trip count
    const int64_t h = base + threadIdx.x;
    int64_t v[4] = {0, 0, 0, 0};
    if (h < nh) {
      const PartSizes z = part_sizes_of(item_len(a.rs, a.re, a.len, a.items[k][h]), a.cap, a.vb,
                                        a.merge, a.shift);
      nck[h] = z.c;
      rper[h] = z.R;
      nblk[h] = z.nblk;
      nparts[h] = z.P;
      hsz[h] = z.hsz;
      p2[h] = z.p2;
      v[0] = z.c;
      v[1] = z.nblk;
      v[2] = z.p2;
      v[3] = z.hsz;
    }
    int64_t inc[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      int64_t x = v[q];
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int64_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
      }
      inc[q] = x;
      if (lane == 63) wtot[q][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
      int64_t t = 0;
      for (int w = 0; w < NW; w++) {
        const int64_t x = wtot[threadIdx.x][w];
        wtot[threadIdx.x][w] = t;
        t += x;
      }
      wtot[threadIdx.x][NW] = t;
    }
    __syncthreads();
    if (h < nh)
#pragma unroll
      for (int q = 0; q < 4; q++) st[q][h] = carry[q] + wtot[q][wave] + inc[q] - v[q];
    __syncthreads();
    if (threadIdx.x < 4) carry[threadIdx.x] += wtot[threadIdx.x][NW];
    __syncthreads();
  }
  if (threadIdx.x < 4) {
    st[threadIdx.x][nh] = carry[threadIdx.x];
    a.totals[4 * k + threadIdx.x] = carry[threadIdx.x];
  }
}

hipError_t plan_parts_batch(const int64_t* rs, const int64_t* re, const int64_t* len,
                            const int32_t* const* items, const int64_t* nh, int K, int64_t cap,
                            int vb, bool merge, int shift, int64_t* const* arrays,
                            int64_t* totals, ull* host_buf, PartPlan* pp, hipStream_t s) {
  if (K <= 0 || K > kPlanBatch) return hipErrorInvalidValue;
  PlanBatchArgs a;
  a.rs = rs;
  a.re = re;
  a.len = len;
  for (int k = 0; k < kPlanBatch; k++) {
    a.items[k] = k < K ? items[k] : nullptr;
    a.nh[k] = k < K ? nh[k] : 0;
    a.arrays[k] = k < K ? arrays[k] : nullptr;
  }
  a.totals = totals;
  a.cap = cap;
  a.vb = vb;
  a.merge = merge ? 1 : 0;
  a.shift = shift;
  LV_LAUNCH(k_plan_batch, (unsigned)K, kPlanBlock, 0, s, a);
  hipError_t e = hipMemcpyAsync(host_buf, totals, 4 * K * sizeof(int64_t),
                                hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  for (int k = 0; k < K; k++) {
    PartPlan& p = pp[k];
    p = PartPlan();
    p.nh = nh[k];
    p.vb = vb;
    p.shift = shift;
    if (nh[k] <= 0) continue;
    int64_t* arr = arrays[k];
    const int64_t n = nh[k];
    p.rper = arr + 4 * n;
    p.nparts = arr + 5 * n;
    p.chunk_start = arr + 6 * n;
    p.block_start = p.chunk_start + (n + 1);
    p.part_start = p.block_start + (n + 1);
    p.hoff_start = p.part_start + (n + 1);
    p.chunks = (int64_t)host_buf[4 * k];
    p.blocks = (int64_t)host_buf[4 * k + 1];
    p.parts = (int64_t)host_buf[4 * k + 2];
    p.hoff_entries = (int64_t)host_buf[4 * k + 3];
  }
  return hipSuccess;
}


// =============================================================================================
// Synchronous local-moving iteration, LDS-table path (rows of up to 1024 arcs).
//
// One group of G lanes decides one vertex v (every class of the fused kernel has its own G and
// table size). The group accumulates k_{v->c} for the communities of v's non-self neighbours
// into an LDS open-addressing table (the per-worker hashtable of section 3.2, one per group),
// then every lane scans its share of slots computing the exact gain
// g(c) = W*k_{v->c} - K_v*Sigma_c, and the group reduces (gain, -c) to the best candidate.
// All reads are of the previous iteration's C, Sigma and csize; every vertex writes its decision,
// and the decisions are applied after the kernel, so the outcome does not depend on scheduling.

// Adds arcs e0 + lane, e0 + lane + S, ... (< e1) of vertex v's row to an LDS table keyed by the
// neighbour's community, self-loops skipped. Each lane first issues U independent index loads and
// U independent record gathers, then makes its U table updates, so that U gathers per lane are
// in flight instead of one. With lab (a 4-byte copy of every record's community, kept for
// graphs of up to kLabMaxVertices vertices), the community comes from lab instead of the
// 16-byte record: the gathers then fall in a table a quarter the size, which the caches hold
// (R-MAT s25's pass 1, 1.85M vertices: its iterations 17.3 -> 15.6 ms), and Sigma comes from
// the candidate evaluation's own gather. Returns the number of slots this lane claimed.
template <typename V, typename WT, int U>
__device__ __forceinline__ int accumulate_row(const int32_t* idx, const WT* w, const VRec* rec,
                                              const int32_t* lab, int32_t v, int64_t e0,
                                              int64_t e1, int lane, int S, int32_t* keys,
                                              V* vals, int log2h) {
  int fresh = 0;
  for (int64_t e = e0 + lane; e < e1; e += (int64_t)U * S) {
    int32_t j[U];
    V wv[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t eu = e + (int64_t)u * S;
      j[u] = eu < e1 ? ld_stream(idx + eu) : v;
      wv[u] = eu < e1 ? (V)ld_stream(w + eu) : (V)0;
    }
    int32_t c[U];
#pragma unroll
    for (int u = 0; u < U; u++)
      c[u] = j[u] == v ? kEmpty : lab ? lab[j[u]] : rec[j[u]].c;
#pragma unroll
    for (int u = 0; u < U; u++) {
      if (j[u] == v) continue;
      fresh += table_add<V>(keys, vals, log2h, c[u], wv[u]);
    }
  }
  return fresh;
}

// Batches of graphs (GraphSet): W and graph of vertex v, false if its graph is not iterating in
// this phase; and the per-graph gain sums of the iteration.
__device__ __forceinline__ bool gs_vertex(const GraphSet& gs, int32_t v, uint64_t* W,
                                          int32_t* g) {
  if (!gs.gid) return true;
  const int32_t x = gs.gid[v];
  *g = x;
  *W = gs.Wg[x];
  return gs.act[x] != 0;
}
// The gain sums are kept in kGainSlices copies, a workgroup adding to the copy of its index
// modulo kGainSlices, so that the workgroups of one large graph do not all meet on one word;
// fold_gain_slices sums the copies into the first before the host reads them.
__device__ __forceinline__ ull* gs_slot(const GraphSet& gs, int32_t g) {
  return gs.gS + 2 * ((int64_t)(blockIdx.x & (kGainSlices - 1)) * gs.G + g);
}
__device__ __forceinline__ void gs_add_gain(const GraphSet& gs, int32_t g, u128 gain) {
  if (gs.gS) atomic_add_u128(gs_slot(gs, g), gain);
}

// Per-graph gain sums of a workgroup of the fused kernel (all threads call it): one atomic for
// the block total when every mover of the block belongs to one graph (always, for graphs much
// larger than a block), else one per mover.
template <typename SH>
__device__ __forceinline__ void gs_add_block(const GraphSet& gs, int32_t gr, u128 gain, u128 bsum,
                                             SH& sh) {
  if (!gs.gS) return;
  const bool mover = gain != 0;
  int32_t lo = mover ? gr : INT32_MAX, hi = mover ? gr : -1;
  for (int m = 32; m >= 1; m >>= 1) {
    const int32_t a = __shfl_xor(lo, m, 64), b = __shfl_xor(hi, m, 64);
    lo = a < lo ? a : lo;
    hi = b > hi ? b : hi;
  }
  if ((threadIdx.x & 63) == 0) {
    sh.gmin[threadIdx.x >> 6] = lo;
    sh.gmax[threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  for (int i = 0; i < kBlock / 64; i++) {
    lo = sh.gmin[i] < lo ? sh.gmin[i] : lo;
    hi = sh.gmax[i] > hi ? sh.gmax[i] : hi;
  }
  __syncthreads();
  if (hi < 0) return;  // no mover
  if (lo == hi) {
    if (threadIdx.x == 0) atomic_add_u128(gs_slot(gs, lo), bsum);
  } else if (mover) {
    atomic_add_u128(gs_slot(gs, gr), gain);
  }
}

// A class step's decision for a vertex that keeps its community.
constexpr int32_t kStay = -1;

template <typename WT>
struct MoveArgs {
  const int64_t* rs;
  const int64_t* re;
  const int32_t* idx;
  const WT* w;
  const uint64_t* K;
  const VRec* rec;
  const int32_t* lab;  // every vertex's community (rec[x].c), or null: read from rec
  uint64_t W;
  const int32_t* list;
  int64_t bstart[8];  // first block of class k; bstart[7] = total blocks
  int64_t lstart[8];  // first list position of class k; lstart[7] = end of class 6
  int32_t* tgt;       // decisions by list position: the new community of a mover, else kStay
  ull* partial;       // per block: gain sum (2 words), moves, candidate pairs
  GraphSet gs;        // batch of graphs (gs.gid null: one graph, W above)
};

struct BlockShared {
  u128 red128[kBlock / 64];
  ull red64[kBlock / 64];
  int32_t gmin[kBlock / 64], gmax[kBlock / 64];
  typename Gain<true>::T bg[kBlock / 64];
  int32_t bc[kBlock / 64];
  ull kd[kBlock / 64];
};

template <bool WIDE, typename WT, int G, int LOG2H>
__device__ __forceinline__ void move_group(const MoveArgs<WT>& a, int64_t lb, int64_t lbase,
                                           int64_t lcount, unsigned char* smem,
                                           BlockShared& sh) {
  typedef Gain<WIDE> Ar;
  typedef typename Ar::T T;
  typedef typename Ar::V V;
  constexpr int H = 1 << LOG2H;
  constexpr int NG = kBlock / G;
  int32_t* keys = (int32_t*)smem;
  V* vals = (V*)(smem + (size_t)NG * H * sizeof(int32_t));
  const int gid = threadIdx.x / G, lane = threadIdx.x % G;
  const int64_t li = lb * NG + gid;
  const bool valid = li < lcount;
  const int32_t v = valid ? a.list[lbase + li] : 0;
  int32_t* gk = keys + gid * H;
  V* gv = vals + gid * H;
  for (int s = lane; s < H; s += G) {
    gk[s] = kEmpty;
    gv[s] = 0;
  }
  __syncthreads();
  uint64_t W = a.W;
  int32_t gr = 0;
  const bool on = valid && gs_vertex(a.gs, v, &W, &gr);
  int64_t e0 = 0, e1 = 0;
  if (on) {
    e0 = a.rs[v];
    e1 = a.re[v];
  }
  // lanes per row cover a class's longest row in one round for classes 0..4; rows of classes 5
  // and up take several arcs per lane, gathered together
  constexpr int U = (1 << LOG2H) / 2 > G ? 4 : 1;
  accumulate_row<V, WT, U>(a.idx, a.w, a.rec, a.lab, v, e0, e1, lane, G, gk, gv, LOG2H);
  __syncthreads();
  T bg = Ar::lowest();
  int32_t bc = INT32_MAX;
  ull kd = 0;
  ull nc = 0;
  int32_t d = 0;
  uint64_t Ki = 0;
  if (valid) {
    d = a.rec[v].c;
    Ki = a.K[v];
    for (int s = lane; s < H; s += G) {
      const int32_t c = gk[s];
      if (c == kEmpty) continue;
      const ull kv = (ull)gv[s];
      if (c == d) {
        kd = kv;
        continue;
      }
      nc++;
      const T g = Ar::of(W, kv, Ki, a.rec[c].sig);
      if (better(g, c, bg, bc)) {
        bg = g;
        bc = c;
      }
    }
  }
  // group argmax of (gain, -community) and the own-community weight
  constexpr int WG = G < 64 ? G : 64;
#pragma unroll
  for (int m = WG / 2; m >= 1; m >>= 1) {
    const T og = Ar::shfl_xor(bg, m, WG);
    const int32_t oc = __shfl_xor(bc, m, WG);
    const ull ok = __shfl_xor(kd, m, WG);
    if (better(og, oc, bg, bc)) {
      bg = og;
      bc = oc;
    }
    kd += ok;
  }
  if (G > 64) {
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
      sh.bg[wave] = (typename Gain<true>::T)bg;
      sh.bc[wave] = bc;
      sh.kd[wave] = kd;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int i = 1; i < kBlock / 64; i++) {
        const T og = (T)sh.bg[i];
        if (better(og, sh.bc[i], bg, bc)) {
          bg = og;
          bc = sh.bc[i];
        }
        kd += sh.kd[i];
      }
    }
  }
  u128 gain = 0;
  ull moved = 0;
  if (valid && lane == 0) {
    int32_t target = d;
    if (bc != INT32_MAX) {
      const VRec rd = a.rec[d];
      const T stay = Ar::of(W, kd, Ki, rd.sig - Ki);
      if (bg > stay && !(rd.size == 1 && a.rec[bc].size == 1 && bc > d)) {
        target = bc;
        moved = 1;
        gain = Ar::diff(bg, stay);
      }
    }
    a.tgt[lbase + li] = moved ? target : kStay;
  }
  // block totals go to this block's own record: no contended atomics in the hot kernel
  const u128 bsum = block_sum_u128(gain, sh.red128);
  gs_add_block(a.gs, gr, gain, bsum, sh);
  const ull bm = block_sum_u64(moved, sh.red64);
  const ull bn = block_sum_u64(nc, sh.red64);
  if (threadIdx.x == 0) {
    ull* o = a.partial + 4 * (int64_t)blockIdx.x;
    o[0] = (ull)bsum;
    o[1] = (ull)(bsum >> 64);
    o[2] = bm;
    o[3] = bn;
  }
}

template <bool WIDE, typename WT>
__global__ __launch_bounds__(kBlock) void k_move_lds(MoveArgs<WT> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ BlockShared sh;
  const int64_t b = blockIdx.x;
  int k = 0;
  while (k < 6 && b >= a.bstart[k + 1]) k++;
  const int64_t lb = b - a.bstart[k];
  const int64_t lbase = a.lstart[k], lcount = a.lstart[k + 1] - a.lstart[k];
  switch (k) {
    case 0: move_group<WIDE, WT, bucket_group(0), bucket_log2h(0)>(a, lb, lbase, lcount, smem, sh); break;
    case 1: move_group<WIDE, WT, bucket_group(1), bucket_log2h(1)>(a, lb, lbase, lcount, smem, sh); break;
    case 2: move_group<WIDE, WT, bucket_group(2), bucket_log2h(2)>(a, lb, lbase, lcount, smem, sh); break;
    case 3: move_group<WIDE, WT, bucket_group(3), bucket_log2h(3)>(a, lb, lbase, lcount, smem, sh); break;
    case 4: move_group<WIDE, WT, bucket_group(4), bucket_log2h(4)>(a, lb, lbase, lcount, smem, sh); break;
    case 5: move_group<WIDE, WT, bucket_group(5), bucket_log2h(5)>(a, lb, lbase, lcount, smem, sh); break;
    default: move_group<WIDE, WT, bucket_group(6), bucket_log2h(6)>(a, lb, lbase, lcount, smem, sh); break;
  }
}


// Workgroup-per-row tier (degree classes 7..9): one 1024-thread workgroup decides one vertex
// with an LDS table of 2^LOG2H slots (twice the longest row of the class). The table has no
// Sigma cache: with one (8 more bytes per slot, which cost the class-8 kernel half its
// occupancy), this tier took 32.3 and 13.6 ms per s25 iteration of passes 0 and 1, without it
// 29.0 and 10.4 ms.
constexpr int kWgBlock = 1024;

template <typename WT>
struct WgArgs {
  const int64_t* rs;
  const int64_t* re;
  const int32_t* idx;
  const WT* w;
  const uint64_t* K;
  const VRec* rec;
  const int32_t* lab;
  uint64_t W;
  const int32_t* rows;  // the class's rows
  int32_t* tgt;         // their decisions, by row (as MoveArgs)
  ull* partial;         // this launch's block records
  GraphSet gs;
};

template <bool WIDE, typename WT, int LOG2H>
__global__ __launch_bounds__(kWgBlock) void k_move_wg(WgArgs<WT> a) {
  typedef Gain<WIDE> Ar;
  typedef typename Ar::T T;
  typedef typename Ar::V V;
  constexpr int H = 1 << LOG2H;
  constexpr int NW = kWgBlock / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ typename Gain<true>::T sbg[NW];
  __shared__ int32_t sbc[NW];
  __shared__ ull skd[NW];
  __shared__ ull snc[NW];
  int32_t* keys = (int32_t*)smem;
  V* vals = (V*)(smem + (size_t)H * sizeof(int32_t));
  const int32_t v = a.rows[blockIdx.x];
  for (int s = threadIdx.x; s < H; s += kWgBlock) {
    keys[s] = kEmpty;
    vals[s] = 0;
  }
  __syncthreads();
  uint64_t W = a.W;
  int32_t gr = 0;
  const bool on = gs_vertex(a.gs, v, &W, &gr);
  const int64_t e0 = a.rs[v], e1 = on ? a.re[v] : e0;
  accumulate_row<V, WT, 4>(a.idx, a.w, a.rec, a.lab, v, e0, e1, threadIdx.x, kWgBlock, keys,
                           vals, LOG2H);
  __syncthreads();
  const int32_t d = a.rec[v].c;
  const uint64_t Ki = a.K[v];
  T bg = Ar::lowest();
  int32_t bc = INT32_MAX;
  ull kd = 0, nc = 0;
  for (int s = threadIdx.x; s < H; s += kWgBlock) {
    const int32_t c = keys[s];
    if (c == kEmpty) continue;
    const ull kv = (ull)vals[s];
    if (c == d) {
      kd = kv;
      continue;
    }
    nc++;
    const T g = Ar::of(W, kv, Ki, a.rec[c].sig);
    if (better(g, c, bg, bc)) {
      bg = g;
      bc = c;
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const T og = Ar::shfl_xor(bg, m, 64);
    const int32_t oc = __shfl_xor(bc, m, 64);
    if (better(og, oc, bg, bc)) {
      bg = og;
      bc = oc;
    }
    kd += __shfl_xor(kd, m, 64);
    nc += __shfl_xor(nc, m, 64);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sbg[wave] = (typename Gain<true>::T)bg;
    sbc[wave] = bc;
    skd[wave] = kd;
    snc[wave] = nc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < NW; i++) {
      const T og = (T)sbg[i];
      if (better(og, sbc[i], bg, bc)) {
        bg = og;
        bc = sbc[i];
      }
      kd += skd[i];
      nc += snc[i];
    }
    int32_t target = d;
    u128 gain = 0;
    ull moved = 0;
    if (bc != INT32_MAX) {
      const VRec rd = a.rec[d];
      const T stay = Ar::of(W, kd, Ki, rd.sig - Ki);
      if (bg > stay && !(rd.size == 1 && a.rec[bc].size == 1 && bc > d)) {
        target = bc;
        moved = 1;
        gain = Ar::diff(bg, stay);
        gs_add_gain(a.gs, gr, gain);
      }
    }
    a.tgt[blockIdx.x] = moved ? target : kStay;
    ull* o = a.partial + 4 * (int64_t)blockIdx.x;
    o[0] = (ull)gain;
    o[1] = (ull)(gain >> 64);
    o[2] = moved;
    o[3] = nc;
  }
}

// Degree class 7 (rows of 1025..2048 arcs): one 256-thread group per row with a table of
// 2^kGrp7Log2H slots, in a launch of its own (in the fused launch its table would raise the LDS
// of every block).
constexpr int kGrp7Log2H = 12;

template <bool WIDE, typename WT>
__global__ __launch_bounds__(kBlock) void k_move_grp7(MoveArgs<WT> a, int64_t lbase,
                                                     int64_t lcount) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ BlockShared sh;
  move_group<WIDE, WT, kBlock, kGrp7Log2H>(a, blockIdx.x, lbase, lcount, smem, sh);
}

static size_t wg_table_bytes(int k, size_t vbytes) { return ((size_t)1 << wg_log2h(k)) * (4 + vbytes); }

int hub_first_class(size_t max_lds, bool wide) {
  const size_t vb = wide ? 8 : 4;
  int k = kFusedClasses;
  while (k < kHubClass && wg_table_bytes(k, vb) + 2048 <= max_lds) k++;
  return k;
}

template <bool WIDE, typename WT, int LOG2H>
static hipError_t launch_wg(const WgArgs<WT>& a, int64_t rows, hipStream_t s) {
  constexpr size_t vb = sizeof(typename Gain<WIDE>::V);
  constexpr size_t shm = ((size_t)1 << LOG2H) * (4 + vb);
  // once per instantiation; a function-local static initialiser is thread-safe, and contexts
  // on different host threads launch these kernels concurrently
  static const bool attr = [] {
    (void)hipFuncSetAttribute((const void*)k_move_wg<WIDE, WT, LOG2H>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    return true;
  }();
  (void)attr;
  LV_LAUNCH((k_move_wg<WIDE, WT, LOG2H>), (unsigned)rows, kWgBlock, shm, s, a);
  return hipGetLastError();
}

static int64_t fused_blocks(const Buckets& b, int cls) {
  int64_t blocks = 0;
  for (int k = 0; k < kFusedClasses; k++) {
    const int64_t rpb = move_rows_per_block(k);
    blocks += (b.count[kDegClasses * cls + k] + rpb - 1) / rpb;
  }
  return blocks;
}

static size_t lds_table_bytes(int k, size_t vbytes) {
  return (size_t)move_rows_per_block(k) * ((size_t)1 << bucket_log2h(k)) * (4 + vbytes);
}

template <typename WT>
static MoveArgs<WT> move_args(const DevGraph& g, const MoveBuffers& m) {
  MoveArgs<WT> a;
  a.rs = g.rs;
  a.re = g.re;
  a.idx = g.idx;
  a.w = (const WT*)g.w;
  a.K = m.K;
  a.rec = (const VRec*)m.rec;
  a.lab = m.lab;
  a.W = m.W;
  a.list = m.list;
  a.tgt = m.tgt;
  a.partial = m.block_partial;
  a.gs = m.gs;
  return a;
}

template <bool WIDE, typename WT>
static hipError_t move_fused_t(const DevGraph& g, const Buckets& b, int cls, const MoveBuffers& m,
                               hipStream_t s) {
  MoveArgs<WT> a = move_args<WT>(g, m);
  int64_t blocks = 0;
  size_t shm = 0;
  const int base = kDegClasses * cls;
  for (int k = 0; k < kFusedClasses; k++) {
    a.bstart[k] = blocks;
    a.lstart[k] = b.lstart[base + k];
    const int64_t rpb = move_rows_per_block(k);
    blocks += (b.count[base + k] + rpb - 1) / rpb;
    if (b.count[base + k]) {
      size_t t = lds_table_bytes(k, sizeof(typename Gain<WIDE>::V));
      shm = t > shm ? t : shm;
    }
  }
  a.bstart[7] = blocks;
  a.lstart[7] = b.lstart[base + kFusedClasses];
  if (blocks > 0) LV_LAUNCH((k_move_lds<WIDE, WT>), (unsigned)blocks, kBlock, shm, s, a);
  return hipGetLastError();
}

template <bool WIDE, typename WT>
static hipError_t move_wg_t(const DevGraph& g, const Buckets& b, int cls, const MoveBuffers& m,
                            hipStream_t s) {
  const int base = kDegClasses * cls;
  const int64_t fused = fused_blocks(b, cls);
  int64_t records = fused;
  WgArgs<WT> wa;
  wa.rs = g.rs;
  wa.re = g.re;
  wa.idx = g.idx;
  wa.w = (const WT*)g.w;
  wa.K = m.K;
  wa.rec = (const VRec*)m.rec;
  wa.lab = m.lab;
  wa.W = m.W;
  wa.tgt = m.tgt;
  wa.gs = m.gs;
  for (int k = kFusedClasses; k < m.hub_first; k++) {
    const int64_t rows = b.count[base + k];
    if (rows == 0) continue;
    wa.rows = m.list + b.lstart[base + k];
    wa.tgt = m.tgt + b.lstart[base + k];
    wa.partial = m.block_partial + 4 * records;
    hipError_t e = hipSuccess;
    if (k == 7) {
      MoveArgs<WT> a = move_args<WT>(g, m);
      a.partial = wa.partial;
      const size_t shm = ((size_t)1 << kGrp7Log2H) * (4 + sizeof(typename Gain<WIDE>::V));
      LV_LAUNCH((k_move_grp7<WIDE, WT>), (unsigned)rows, kBlock, shm, s, a, b.lstart[base + k],
                rows);
      e = hipGetLastError();
    } else if (k == 8) e = launch_wg<WIDE, WT, wg_log2h(8)>(wa, rows, s);
    else e = launch_wg<WIDE, WT, wg_log2h(9)>(wa, rows, s);
    if (e != hipSuccess) return e;
    records += rows;
  }
  return hipSuccess;
}

int64_t move_lds_blocks(const Buckets& b, int cls, int hub_first) {
  int64_t blocks = fused_blocks(b, cls);
  for (int k = kFusedClasses; k < hub_first; k++) blocks += b.count[kDegClasses * cls + k];
  return blocks;
}

hipError_t move_fused(const DevGraph& g, const Buckets& b, int cls, const MoveBuffers& m,
                      bool wide, hipStream_t s) {
  if (wide)
    return g.w64 ? move_fused_t<true, uint64_t>(g, b, cls, m, s)
                 : move_fused_t<true, uint32_t>(g, b, cls, m, s);
  return g.w64 ? move_fused_t<false, uint64_t>(g, b, cls, m, s)
               : move_fused_t<false, uint32_t>(g, b, cls, m, s);
}

hipError_t move_wg(const DevGraph& g, const Buckets& b, int cls, const MoveBuffers& m, bool wide,
                   hipStream_t s) {
  if (wide)
    return g.w64 ? move_wg_t<true, uint64_t>(g, b, cls, m, s)
                 : move_wg_t<true, uint32_t>(g, b, cls, m, s);
  return g.w64 ? move_wg_t<false, uint64_t>(g, b, cls, m, s)
               : move_wg_t<false, uint32_t>(g, b, cls, m, s);
}

// =============================================================================================
// Two-phase path for long items (hub rows here, large communities in the aggregation): the
// per-worker hashtable of section 3.2 split by a hash partition of the keys so that every piece
// fits in LDS (see part_chunk). No global hash table and no global atomics on keys.

__device__ __forceinline__ int64_t find_segment(const int64_t* start, int64_t cnt, int64_t x) {
  int64_t lo = 0, hi = cnt;  // start[lo] <= x < start[hi]
  while (hi - lo > 1) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (start[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int ilog2_i64(int64_t x) { return 63 - __clzll((long long)x); }

// Exclusive scan in place of a[0 .. n), n <= 4 * kPartBlock, by a kPartBlock-thread workgroup.
// Returns the total in every thread. wsum: kPartBlock / 64 + 1 shared ints.
__device__ int block_scan_excl(int* a, int n, int* wsum) {
  constexpr int NW = kPartBlock / 64;
  const int per = (n + kPartBlock - 1) / kPartBlock;
  const int i0 = threadIdx.x * per;
  int loc[4];
  int sum = 0;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    loc[i] = (i < per && i0 + i < n) ? a[i0 + i] : 0;
    sum += loc[i];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = sum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < NW; w++) {
      const int x = wsum[w];
      wsum[w] = t;
      t += x;
    }
    wsum[NW] = t;
  }
  __syncthreads();
  int run = wsum[wave] + incl - sum;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    if (i < per && i0 + i < n) a[i0 + i] = run;
    run += loc[i];
  }
  const int total = wsum[NW];
  __syncthreads();
  return total;
}

template <typename V>
__device__ __forceinline__ void part_table_clear(int32_t* keys, V* vals, int H) {
  for (int s = threadIdx.x; s < H; s += kPartBlock) {
    keys[s] = kEmpty;
    vals[s] = 0;
  }
}

// Phase-1 table flush: the table's keys written to pk/pv + base grouped by partition, with the
// partition bounds (offsets from pk/pv) in hoff_row[0 .. P]. Returns the number of keys.
template <typename V>
__device__ int part_emit(const int32_t* keys, const V* vals, int H, int P, int* cnt, int* wsum,
                         int32_t* hoff_row, int base, int32_t* pk, V* pv) {
  const int lp = ilog2_i64(P);
  for (int p = threadIdx.x; p < P; p += kPartBlock) cnt[p] = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < H; s += kPartBlock)
    if (keys[s] != kEmpty) atomicAdd(&cnt[part_of(keys[s], lp)], 1);
  __syncthreads();
  const int total = block_scan_excl(cnt, P, wsum);
  for (int p = threadIdx.x; p < P; p += kPartBlock) hoff_row[p] = base + cnt[p];
  if (threadIdx.x == 0) hoff_row[P] = base + total;
  __syncthreads();
  for (int s = threadIdx.x; s < H; s += kPartBlock) {
    const int32_t key = keys[s];
    if (key == kEmpty) continue;
    const int pos = base + atomicAdd(&cnt[part_of(key, lp)], 1);
    pk[pos] = key;
    pv[pos] = vals[s];
  }
  return total;
}

// Phase-1 walk of chunks [k0, k1) of an item: acc(k, keys, vals, flags) adds chunk k to the LDS
// table, counting newly claimed slots in flags[0]; the table is flushed (part_emit) into the
// next bound row (hoff_rows, P + 1 entries each) whenever the next chunk might push it past 3/4
// full, and at the end. The pairs go to the workgroup's region pk/pv (room for k1 - k0 chunks,
// which the flushed keys cannot exceed). Returns the number of flushes.
template <typename V, int LOG2H, typename Acc>
__device__ int part_walk(Acc& acc, int64_t k0, int64_t k1, int P, int32_t* keys, V* vals,
                         int* cnt, int* wsum, int* flags, int32_t* hoff_rows, int32_t* pk,
                         V* pv) {
  constexpr int H = 1 << LOG2H;
  constexpr int Q = part_chunk((int)sizeof(V));
  static_assert(2 * Q == H, "phase-1 table holds two chunks");
  int flushes = 0, written = 0;
  part_table_clear<V>(keys, vals, H);
  if (threadIdx.x == 0) flags[0] = 0;
  __syncthreads();
  for (int64_t k = k0; k < k1; k++) {
    if (flags[0] > Q / 2) {
      written += part_emit<V>(keys, vals, H, P, cnt, wsum, hoff_rows + flushes * (P + 1),
                              written, pk, pv);
      flushes++;
      __syncthreads();
      part_table_clear<V>(keys, vals, H);
      if (threadIdx.x == 0) flags[0] = 0;
      __syncthreads();
    }
    acc(k, keys, vals, flags);
    __syncthreads();
  }
  if (flags[0] > 0) {
    part_emit<V>(keys, vals, H, P, cnt, wsum, hoff_rows + flushes * (P + 1), written, pk, pv);
    flushes++;
  }
  return flushes;
}

// Phase 2: combine partition p of an item into the LDS table, in rounds over sub-ranges of the
// key hash when the partition holds more distinct keys than a round may claim (cap); fin(keys,
// vals, H) consumes each completed round. The item's bound rows (one per chunk, nck of them,
// from hrow) belong to its phase-1 workgroups, R consecutive rows each, of which workgroup i
// used the first nflush[i]; its pairs are at pk/pv + (i * R) * Q. cap <= part_cap(LOG2H), so
// the claims made before every thread sees the overflow still find free slots. flags: 4 shared
// ints (claimed slots, overflow, and two for fin). With FIT > 0, when the item's rows fit one
// tile, the table is sized to the partition: the smallest power of two (at least 256 slots)
// holding 2^FIT times its pairs, so all its keys fit one round, and a partition of few keys
// clears and scans few slots (partitions are sized by the item's length, as if every key were
// distinct, and once communities have formed they hold far fewer).
template <typename V, int LOG2H, int FIT, typename Fin>
__device__ void part_reduce(const int32_t* pk, const V* pv, const int32_t* hrow,
                            const int32_t* nflush, int64_t nck, int64_t R, int P, int p, int cap,
                            int32_t* keys, V* vals, unsigned char* aux, int* wsum, int* flags,
                            Fin& fin) {
  constexpr int H = 1 << LOG2H;
  constexpr int Q = part_chunk((int)sizeof(V));
  static_assert(part_cap(LOG2H) + kPartBlock <= H, "claims past the cap must find free slots");
  int64_t* sbeg = (int64_t*)aux;                             // first pair of each row's segment
  int* sstart = (int*)(aux + kPartTile * sizeof(int64_t));  // exclusive scan of their lengths
  const int lp = ilog2_i64(P);
  const uint64_t pbeg = (uint64_t)p << (32 - lp);
  const uint64_t pend = (uint64_t)(p + 1) << (32 - lp);
  // the segment bounds of the rows of tile t0 into sbeg / sstart (exclusive scan); returns the
  // tile's pairs of partition p
  auto load_tile = [&](int64_t t0, int nt) -> int {
    for (int i = threadIdx.x; i < nt; i += kPartBlock) {
      const int64_t r = t0 + i;
      const int64_t blk = r / R;
      int len = 0;
      if (r - blk * R < nflush[blk]) {
        const int32_t* row = hrow + r * (int64_t)(P + 1);
        const int32_t s0 = row[p];
        sbeg[i] = blk * R * Q + s0;
        len = row[p + 1] - s0;
      }
      sstart[i] = len;
    }
    __syncthreads();
    return block_scan_excl(sstart, nt, wsum);
  };
  int log2h = LOG2H;
  if (FIT > 0 && nck <= kPartTile) {
    const int total = load_tile(0, (int)nck);
    int l = 8;
    while (l < LOG2H && (1 << l) < ((int64_t)total << FIT)) l++;
    log2h = l;
    __syncthreads();
  }
  const int Hs = 1 << log2h;
  const int capr = cap < part_cap(log2h) ? cap : part_cap(log2h);
  uint64_t lo = pbeg, width = pend - pbeg;
  while (lo < pend) {
    const uint64_t hi = lo + width < pend ? lo + width : pend;
    part_table_clear<V>(keys, vals, Hs);
    if (threadIdx.x == 0) {
      flags[0] = 0;
      flags[1] = 0;
    }
    __syncthreads();
    for (int64_t t0 = 0; t0 < nck; t0 += kPartTile) {
      const int nt = (int)(nck - t0 < kPartTile ? nck - t0 : kPartTile);
      const int total = load_tile(t0, nt);
      for (int f = threadIdx.x; f < total; f += kPartBlock) {
        if (*(volatile int*)&flags[1]) break;
        int a = 0, b = nt;  // sstart[a] <= f < sstart[b] (segment a is the non-empty one)
        while (b - a > 1) {
          const int mid = (a + b) >> 1;
          if (sstart[mid] <= f) a = mid; else b = mid;
        }
        const int64_t pos = sbeg[a] + (f - sstart[a]);
        const int32_t key = pk[pos];
        const uint64_t hk = fmix32((uint32_t)key);
        if (hk >= lo && hk < hi)
          table_add_capped<V>(keys, vals, log2h, key, pv[pos], &flags[0], capr, &flags[1]);
      }
      __syncthreads();
    }
    const int over = flags[1];
    __syncthreads();
    if (over) {
      width = (hi - lo) / 2 > 0 ? (hi - lo) / 2 : 1;
      continue;
    }
    fin(keys, vals, Hs);
    __syncthreads();
    lo = hi;
  }
}

template <typename WT, typename V>
struct HubArgs {
  const int64_t* rs;
  const int64_t* re;
  const int32_t* idx;
  const WT* w;
  const uint64_t* K;
  const VRec* rec;
  const int32_t* lab;
  uint64_t W;
  const int32_t* hubs;
  int64_t nh;
  const int64_t* chunk_start;
  const int64_t* block_start;
  const int64_t* part_start;
  const int64_t* hoff_start;
  const int64_t* rper;
  const int64_t* nparts;
  int32_t* pk;       // phase-1 pairs, part_chunk(sizeof(V)) per chunk
  V* pv;
  int32_t* hoff;     // segment bounds
  int32_t* nflush;   // flushes of every phase-1 workgroup
  int cap;           // phase-2 claim cap per round
  ull* partial;      // 5 words per phase-2 workgroup: gain lo, gain hi, community, kd, candidates
  int32_t* tgt;      // decisions of the hubs, by hub (as MoveArgs)
  ull* stats;
  GraphSet gs;
};

// Phase 1 of the hub rows: workgroup i of hub h walks chunks [i R, (i + 1) R) of its row.
template <typename WT, typename V>
struct HubChunk {
  const HubArgs<WT, V>* a;
  int32_t v;
  int64_t e0, e1;  // the row
  template <int LOG2H>
  __device__ void add(int64_t k, int32_t* keys, V* vals, int* flags) {
    constexpr int Q = part_chunk((int)sizeof(V));
    const int64_t c0 = e0 + k * Q;
    const int64_t c1 = c0 + Q < e1 ? c0 + Q : e1;
    const int fresh = accumulate_row<V, WT, 4>(a->idx, a->w, a->rec, a->lab, v, c0, c1,
                                               threadIdx.x, kPartBlock, keys, vals, LOG2H);
    if (fresh) atomicAdd(&flags[0], fresh);
  }
  __device__ void operator()(int64_t k, int32_t* keys, V* vals, int* flags) {
    add<part_log2h((int)sizeof(V))>(k, keys, vals, flags);
  }
};

template <typename WT, typename V>
__global__ __launch_bounds__(kPartBlock) void k_hub_part(HubArgs<WT, V> a) {
  constexpr int LOG2H = part_log2h((int)sizeof(V));
  constexpr int H = 1 << LOG2H;
  constexpr int Q = part_chunk((int)sizeof(V));
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int wsum[kPartBlock / 64 + 1];
  __shared__ int flags[4];
  int32_t* keys = (int32_t*)smem;
  V* vals = (V*)(smem + (size_t)H * 4);
  int* cnt = (int*)(smem + (size_t)H * (4 + sizeof(V)));
  const int64_t b = blockIdx.x;
  const int64_t h = find_segment(a.block_start, a.nh, b);
  const int64_t i = b - a.block_start[h];
  const int64_t R = a.rper[h];
  const int64_t row0 = a.chunk_start[h], nck = a.chunk_start[h + 1] - row0;
  const int64_t k0 = i * R, k1 = k0 + R < nck ? k0 + R : nck;
  const int P = (int)a.nparts[h];
  HubChunk<WT, V> acc;
  acc.a = &a;
  acc.v = a.hubs[h];
  acc.e0 = a.rs[acc.v];
  acc.e1 = a.re[acc.v];
  uint64_t W;
  int32_t gr;
  // a hub of a graph that is not iterating walks nothing (no rows: phase 2 finds no key)
  const int64_t k1w = gs_vertex(a.gs, acc.v, &W, &gr) ? k1 : k0;
  const int nf = part_walk<V, LOG2H>(acc, k0, k1w, P, keys, vals, cnt, wsum, flags,
                                     a.hoff + a.hoff_start[h] + k0 * (P + 1),
                                     a.pk + (row0 + k0) * Q, a.pv + (row0 + k0) * Q);
  if (threadIdx.x == 0) a.nflush[b] = nf;
}

// Per-thread best candidate over completed phase-2 rounds of one hub.
template <bool WIDE>
struct HubFin {
  typedef Gain<WIDE> Ar;
  typedef typename Ar::T T;
  const VRec* rec;
  uint64_t W, Ki;
  int32_t d;
  T bg;
  int32_t bc;
  ull kd, nc;
  template <typename V>
  __device__ void operator()(const int32_t* keys, const V* vals, int H) {
    for (int s = threadIdx.x; s < H; s += kPartBlock) {
      const int32_t c = keys[s];
      if (c == kEmpty) continue;
      const ull kv = (ull)vals[s];
      if (c == d) {
        kd += kv;
        continue;
      }
      nc++;
      const T g = Ar::of(W, kv, Ki, rec[c].sig);
      if (better(g, c, bg, bc)) {
        bg = g;
        bc = c;
      }
    }
  }
};

// Phase 2 of the hub rows: partition p of hub h -> its best (gain, community), the weight to
// the hub's own community and the candidate count, as a partial record.
template <bool WIDE, typename WT>
__global__ __launch_bounds__(kPartBlock) void k_hub_reduce(
    HubArgs<WT, typename Gain<WIDE>::V> a) {
  typedef Gain<WIDE> Ar;
  typedef typename Ar::T T;
  typedef typename Ar::V V;
  constexpr int LOG2H = part_log2h((int)sizeof(V));
  constexpr int H = 1 << LOG2H;
  constexpr int Q = part_chunk((int)sizeof(V));
  constexpr int NW = kPartBlock / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int wsum[NW + 1];
  __shared__ int flags[4];
  __shared__ typename Gain<true>::T sbg[NW];
  __shared__ int32_t sbc[NW];
  __shared__ ull skd[NW];
  __shared__ ull snc[NW];
  int32_t* keys = (int32_t*)smem;
  V* vals = (V*)(smem + (size_t)H * 4);
  unsigned char* aux = smem + (size_t)H * (4 + sizeof(V));
  const int64_t b = blockIdx.x;
  const int64_t h = find_segment(a.part_start, a.nh, b);
  const int p = (int)(b - a.part_start[h]);
  const int P = (int)a.nparts[h];
  const int64_t c0 = a.chunk_start[h], nck = a.chunk_start[h + 1] - c0;
  const int32_t v = a.hubs[h];
  HubFin<WIDE> fin;
  fin.rec = a.rec;
  fin.W = a.W;
  int32_t gr = 0;
  gs_vertex(a.gs, v, &fin.W, &gr);
  fin.Ki = a.K[v];
  fin.d = a.rec[v].c;
  fin.bg = Ar::lowest();
  fin.bc = INT32_MAX;
  fin.kd = 0;
  fin.nc = 0;
  part_reduce<V, LOG2H, 1>(a.pk + c0 * Q, a.pv + c0 * Q, a.hoff + a.hoff_start[h],
                           a.nflush + a.block_start[h], nck, a.rper[h], P, p, a.cap, keys, vals,
                           aux, wsum, flags, fin);
  T bg = fin.bg;
  int32_t bc = fin.bc;
  ull kd = fin.kd, nc = fin.nc;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const T og = Ar::shfl_xor(bg, m, 64);
    const int32_t oc = __shfl_xor(bc, m, 64);
    if (better(og, oc, bg, bc)) {
      bg = og;
      bc = oc;
    }
    kd += __shfl_xor(kd, m, 64);
    nc += __shfl_xor(nc, m, 64);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sbg[wave] = (typename Gain<true>::T)bg;
    sbc[wave] = bc;
    skd[wave] = kd;
    snc[wave] = nc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < NW; i++) {
      const T og = (T)sbg[i];
      if (better(og, sbc[i], bg, bc)) {
        bg = og;
        bc = sbc[i];
      }
      kd += skd[i];
      nc += snc[i];
    }
    const i128 wideg = (i128)bg;
    ull* out = a.partial + 5 * b;
    out[0] = (ull)(u128)wideg;
    out[1] = (ull)((u128)wideg >> 64);
    out[2] = (ull)(uint32_t)bc;
    out[3] = kd;
    out[4] = nc;
  }
}

template <bool WIDE, typename WT>
__global__ __launch_bounds__(kBlock) void k_hub_decide(HubArgs<WT, typename Gain<WIDE>::V> a) {
  typedef Gain<WIDE> Ar;
  typedef typename Ar::T T;
  __shared__ u128 red[kBlock / 64];
  __shared__ ull red64[kBlock / 64];
  const int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  u128 gain = 0;
  ull nc = 0, moved = 0;
  if (h < a.nh) {
    const int32_t v = a.hubs[h];
    T bg = Ar::lowest();
    int32_t bc = INT32_MAX;
    ull kd = 0;
    for (int64_t p = a.part_start[h]; p < a.part_start[h + 1]; p++) {
      const ull* in = a.partial + 5 * p;
      const T og = (T)(i128)(((u128)in[1] << 64) | in[0]);
      const int32_t oc = (int32_t)(uint32_t)in[2];
      if (better(og, oc, bg, bc)) {
        bg = og;
        bc = oc;
      }
      kd += in[3];
      nc += in[4];
    }
    const int32_t d = a.rec[v].c;
    int32_t target = d;
    uint64_t W = a.W;
    int32_t gr = 0;
    gs_vertex(a.gs, v, &W, &gr);  // an inactive graph's hub has no candidate (bc unset)
    if (bc != INT32_MAX) {
      const uint64_t Ki = a.K[v];
      const VRec rd = a.rec[d];
      const T stay = Ar::of(W, kd, Ki, rd.sig - Ki);
      if (bg > stay && !(rd.size == 1 && a.rec[bc].size == 1 && bc > d)) {
        gain = Ar::diff(bg, stay);
        target = bc;
        moved = 1;
        gs_add_gain(a.gs, gr, gain);
      }
    }
    a.tgt[h] = moved ? target : kStay;
  }
  const u128 bs = block_sum_u128(gain, red);
  const ull ns = block_sum_u64(nc, red64);
  const ull ms = block_sum_u64(moved, red64);
  if (threadIdx.x == 0) {
    if (bs) atomic_add_u128(&a.stats[0], bs);
    if (ms) atomicAdd(&a.stats[2], ms);
    if (ns) atomicAdd(&a.stats[3], ns);
  }
}

template <typename K>
static void allow_part_lds(K kernel, int vb) {
  (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)part_lds_bytes(vb));
}

template <bool WIDE, typename WT>
static hipError_t move_hubs_t(const DevGraph& g, const Buckets& b, int cls, const PartPlan& pp,
                              const MoveBuffers& m, hipStream_t s) {
  typedef typename Gain<WIDE>::V V;
  constexpr int vb = (int)sizeof(V);
  HubArgs<WT, V> a;
  a.rs = g.rs;
  a.re = g.re;
  a.idx = g.idx;
  a.w = (const WT*)g.w;
  a.K = m.K;
  a.rec = (const VRec*)m.rec;
  a.lab = m.lab;
  a.W = m.W;
  a.hubs = m.list + b.lstart[kDegClasses * cls + m.hub_first];
  a.nh = pp.nh;
  a.chunk_start = pp.chunk_start;
  a.block_start = pp.block_start;
  a.part_start = pp.part_start;
  a.hoff_start = pp.hoff_start;
  a.rper = pp.rper;
  a.nparts = pp.nparts;
  a.pk = m.pk;
  a.pv = (V*)m.pv;
  a.hoff = m.hoff;
  a.nflush = m.nflush;
  a.cap = part_round_cap(part_log2h(vb), pp.shift);
  a.partial = m.partial;
  a.tgt = m.tgt + b.lstart[kDegClasses * cls + m.hub_first];
  a.stats = m.stats;
  a.gs = m.gs;
  static const bool attr = [] {  // once, thread-safe (see launch_wg)
    allow_part_lds(k_hub_part<WT, V>, vb);
    allow_part_lds(k_hub_reduce<WIDE, WT>, vb);
    return true;
  }();
  (void)attr;
  const size_t shm = part_lds_bytes(vb);
  LV_LAUNCH((k_hub_part<WT, V>), (unsigned)pp.blocks, kPartBlock, shm, s, a);
  LV_LAUNCH((k_hub_reduce<WIDE, WT>), (unsigned)pp.parts, kPartBlock, shm, s, a);
  LV_LAUNCH((k_hub_decide<WIDE, WT>), grid_for(pp.nh, kBlock, 1 << 30), kBlock, 0, s, a);
  return hipGetLastError();
}

hipError_t move_hubs(const DevGraph& g, const Buckets& b, int cls, const PartPlan& pp,
                     const MoveBuffers& m, bool wide, hipStream_t s) {
  if (pp.nh <= 0) return hipSuccess;
  if (wide)
    return g.w64 ? move_hubs_t<true, uint64_t>(g, b, cls, pp, m, s)
                 : move_hubs_t<true, uint32_t>(g, b, cls, pp, m, s);
  return g.w64 ? move_hubs_t<false, uint64_t>(g, b, cls, pp, m, s)
               : move_hubs_t<false, uint32_t>(g, b, cls, pp, m, s);
}

// Slot of label x in a workgroup's LDS combining table of 2^LOG2 slots (open addressing; the
// table has room for every label the workgroup inserts before it is flushed).
template <int LOG2>
__device__ __forceinline__ int comb_slot(int32_t* keys, int32_t x) {
  uint32_t s = slot_of(x, LOG2);
  while (true) {
    const int32_t prev = atomicCAS(&keys[s], kEmpty, x);
    if (prev == kEmpty || prev == x) return (int)s;
    s = (s + 1u) & ((1u << LOG2) - 1u);
  }
}

// Apply a class step's decisions: C, Sigma and csize after the step. Each workgroup combines
// its movers' changes per community in LDS (a mover adds K to its new community and takes it
// from its old one) and then makes one atomic per community it touched: the movers of a step
// often join the same few large communities, whose words would otherwise take one atomic per
// mover. Integer sums commute, so the result is independent of the order of the movers.
// The same launch also sums the move kernels' per-block records into the class step's
// statistics, in its first kApplyReduceBlocks workgroups: [0..1] gain sum, [2] moves, [3]
// candidate pairs, [4] those of the fused kernel (records < nfused), [5] those of the
// workgroup kernel. Decisions come by list position (tgt[i] for verts[i]), so they are read
// in order, and only a mover's record is gathered.
constexpr int kApplyLog2 = 10;  // 1024 slots for the 2 * kBlock communities of a tile
constexpr int kApplyReduceBlocks = 256;
__global__ __launch_bounds__(kBlock) void k_apply_moves(const int32_t* verts, int64_t count,
                                                       const int32_t* tgt, const uint64_t* K,
                                                       VRec* rec, int32_t* lab, const ull* part,
                                                       int64_t nb, int64_t nfused, ull* stats) {
  constexpr int S = 1 << kApplyLog2;
  __shared__ int32_t ckey[S];
  __shared__ ull csig[S];
  __shared__ int32_t ccnt[S];
  __shared__ u128 red[kBlock / 64];
  __shared__ ull red64[kBlock / 64];
  const int64_t rblocks = gridDim.x < kApplyReduceBlocks ? gridDim.x : kApplyReduceBlocks;
  if (nb > 0 && blockIdx.x < rblocks) {  // block-uniform
    u128 sg = 0;
    ull sm = 0, sf = 0, sw = 0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < nb; i += rblocks * kBlock) {
      const ull* p = part + 4 * i;
      sg += ((u128)p[1] << 64) | p[0];
      sm += p[2];
      if (i < nfused) sf += p[3]; else sw += p[3];
    }
    sg = block_sum_u128(sg, red);
    sm = block_sum_u64(sm, red64);
    sf = block_sum_u64(sf, red64);
    sw = block_sum_u64(sw, red64);
    if (threadIdx.x == 0) {
      if (sg) atomic_add_u128(stats, sg);
      if (sm) atomicAdd(&stats[2], sm);
      if (sf + sw) atomicAdd(&stats[3], sf + sw);
      if (sf) atomicAdd(&stats[4], sf);
      if (sw) atomicAdd(&stats[5], sw);
    }
  }
  // The table is cleared once; each tile's flush empties the slots it used. A tile without
  // movers (most of them once the step's class has settled) touches no slot and is skipped
  // after one vote. Whole workgroups iterate together (the table is shared).
  for (int t = threadIdx.x; t < S; t += kBlock) {
    ckey[t] = kEmpty;
    csig[t] = 0;
    ccnt[t] = 0;
  }
  __syncthreads();
  for (int64_t base = blockIdx.x * (int64_t)kBlock; base < count;
       base += (int64_t)gridDim.x * kBlock) {
    const int64_t i = base + threadIdx.x;
    int32_t v = 0, c = kStay, d = kStay;
    if (i < count) {
      c = tgt[i];
      if (c != kStay) {
        v = verts[i];
        d = rec[v].c;
      }
    }
    if (!__syncthreads_or(c != d)) continue;
    if (c != d) {
      const ull k = (ull)K[v];
      rec[v].c = c;
      if (lab) lab[v] = c;
      const int sc = comb_slot<kApplyLog2>(ckey, c);
      atomicAdd(&csig[sc], k);
      atomicAdd(&ccnt[sc], 1);
      const int sd = comb_slot<kApplyLog2>(ckey, d);
      atomicAdd(&csig[sd], 0ull - k);
      atomicAdd(&ccnt[sd], -1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < S; t += kBlock) {
      const int32_t x = ckey[t];
      if (x == kEmpty) continue;
      if (csig[t]) atomicAdd((ull*)&rec[x].sig, csig[t]);
      if (ccnt[t]) atomicAdd(&rec[x].size, ccnt[t]);
      ckey[t] = kEmpty;
      csig[t] = 0;
      ccnt[t] = 0;
    }
    __syncthreads();
  }
}

hipError_t apply_moves(const Buckets& b, int cls, const MoveBuffers& m, hipStream_t s) {
  const int64_t first = b.lstart[kDegClasses * cls];
  const int64_t count = b.lstart[kDegClasses * cls + kDegClasses] - first;
  const int64_t fused = fused_blocks(b, cls);
  const int64_t records = move_lds_blocks(b, cls, m.hub_first);
  if (count <= 0 && records == 0) return hipSuccess;
  const unsigned grid = count > 0 ? grid_for(count, kBlock, 8192)
                                  : grid_for(records, kBlock, kApplyReduceBlocks);
  LV_LAUNCH(k_apply_moves, grid, kBlock, 0, s, m.list + first, count, m.tgt + first, m.K,
            (VRec*)m.rec, m.lab, m.block_partial, records, fused, m.stats);
  return hipGetLastError();
}

// =============================================================================================
// Aggregation (section 3.2): communities -> super-vertices.
//
// Used labels are renumbered by rank (scan of csize > 0). The vertices of each community that
// have arcs are listed contiguously (counting sort by label), and an exclusive scan of their
// degrees in that order gives every community a flat arc range [astart[c], astart[c] + A[c]) and
// every member the flat index of its first arc. A group (or, for communities of more than 1024
// arcs, a set of blocks) walks the community's flat range, reads each arc from its member's row,
// and combines the arcs by target super-vertex in an open-addressing table. The distinct
// (target, summed weight) pairs are written to the front of the community's range in the
// output arrays: the super-vertex graph keeps the rows where they were produced (row a spans
// [rs[a], re[a]) of those arrays), so no compaction pass is needed between passes.

// Both member kernels combine per label within a workgroup first (LDS table, one global
// atomic per label per workgroup): after the first pass the members of a level mostly belong
// to a few large communities, whose counters would otherwise take one atomic per member.
constexpr int kMemberLog2 = 9;  // 512 slots for the kBlock labels of a tile

// Vertices with arcs per label.
__global__ __launch_bounds__(kBlock) void k_count_members(const int64_t* rs, const int64_t* re,
                                                         const int32_t* C, int64_t n,
                                                         int32_t* mcount) {
  constexpr int S = 1 << kMemberLog2;
  __shared__ int32_t ckey[S];
  __shared__ int32_t ccnt[S];
  for (int64_t b = blockIdx.x * (int64_t)kBlock; b < n; b += (int64_t)gridDim.x * kBlock) {
    for (int t = threadIdx.x; t < S; t += kBlock) {
      ckey[t] = kEmpty;
      ccnt[t] = 0;
    }
    __syncthreads();
    const int64_t i = b + threadIdx.x;
    if (i < n && re[i] > rs[i]) atomicAdd(&ccnt[comb_slot<kMemberLog2>(ckey, C[i])], 1);
    __syncthreads();
    for (int t = threadIdx.x; t < S; t += kBlock)
      if (ckey[t] != kEmpty) atomicAdd(&mcount[ckey[t]], ccnt[t]);
    __syncthreads();
  }
}

// map[v] = new id of v's community (-1 if the community gets none); members with arcs placed in
// their community's slot range (a workgroup claims each label's share with one atomic; its
// members take consecutive slots).
__global__ __launch_bounds__(kBlock) void k_fill_members(const int64_t* rs, const int64_t* re,
                                                        const int32_t* C, int64_t n,
                                                        const int64_t* newid,
                                                        const int64_t* mstart, int32_t* mcur,
                                                        int32_t* map, int32_t* members) {
  constexpr int S = 1 << kMemberLog2;
  __shared__ int32_t ckey[S];
  __shared__ int32_t ccnt[S];
  __shared__ int32_t cbase[S];
  for (int64_t b = blockIdx.x * (int64_t)kBlock; b < n; b += (int64_t)gridDim.x * kBlock) {
    for (int t = threadIdx.x; t < S; t += kBlock) {
      ckey[t] = kEmpty;
      ccnt[t] = 0;
    }
    __syncthreads();
    const int64_t i = b + threadIdx.x;
    int32_t c = -1;
    int slot = 0, rank = 0;
    if (i < n) {
      c = C[i];
      map[i] = newid[c + 1] > newid[c] ? (int32_t)newid[c] : -1;
      if (re[i] > rs[i]) {
        slot = comb_slot<kMemberLog2>(ckey, c);
        rank = atomicAdd(&ccnt[slot], 1);
      } else {
        c = -1;
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < S; t += kBlock)
      if (ckey[t] != kEmpty) cbase[t] = atomicAdd(&mcur[ckey[t]], ccnt[t]);
    __syncthreads();
    if (c >= 0) members[mstart[c] + cbase[slot] + rank] = (int32_t)i;
    __syncthreads();
  }
}

// Per label: its flat arc range and arc count; per label with a new id, that id's tables.
__global__ void k_label_ranges(int64_t n, const int64_t* newid, const int64_t* mstart,
                               const int64_t* gscan, const uint64_t* Sig, int32_t* oldlabel,
                               uint64_t* Kp, int64_t* astart, int64_t* A) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a0 = gscan[mstart[c]];
    astart[c] = a0;
    A[c] = gscan[mstart[c + 1]] - a0;
    if (newid[c + 1] > newid[c]) {
      const int64_t a = newid[c];
      oldlabel[a] = (int32_t)c;
      if (Kp) Kp[a] = Sig[c];
    }
  }
}

hipError_t aggregate_prepare(const DevGraph& g, const int32_t* C, const int32_t* csize,
                             const uint64_t* Sig, uint64_t* Kp, int32_t* map,
                             const AggBuffers& a, bool live_only, hipStream_t s) {
  const int64_t n = g.n;
  if (n <= 0) return hipSuccess;
  hipError_t e;
  LV_LAUNCH(k_fill_i32, grid_for(n), kBlock, 0, s, a.mcount, 0, n);
  LV_LAUNCH(k_count_members, grid_for(n), kBlock, 0, s, g.rs, g.re, C, n, a.mcount);
  // new ids: rank of the used labels, or (live_only) of the labels whose members have arcs
  if ((e = scan_flags_pos(live_only ? a.mcount : csize, n, a.newid, a.partial, s)) != hipSuccess)
    return e;
  if ((e = scan_impl(ReadI32{a.mcount}, n, a.mstart, a.partial, s)) != hipSuccess) return e;
  LV_LAUNCH(k_fill_i32, grid_for(n), kBlock, 0, s, a.mcount, 0, n);  // reused as cursors
  LV_LAUNCH(k_fill_members, grid_for(n), kBlock, 0, s, g.rs, g.re, C, n, a.newid, a.mstart,
            a.mcount, map, a.members);
  // members occupy mstart[n] slots; gscan over them (mstart[n] + 1 entries)
  // the number of members is only known on the device: scan over n slots, the tail past
  // mstart[n] reads members left from before and is never used
  if ((e = scan_impl(ReadMemberDegGuard{a.members, g.rs, g.re, a.mstart + n}, n, a.gscan,
                     a.partial, s)) != hipSuccess)
    return e;
  LV_LAUNCH(k_label_ranges, grid_for(n), kBlock, 0, s, n, a.newid, a.mstart, a.gscan, Sig,
            a.oldlabel, Kp, a.astart, a.A);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Live numbering. A vertex without arcs never moves and is never a candidate, so a run may give
// new ids only to communities with arcs (aggregate_prepare with live_only), in the order of
// their labels. That keeps every comparison of labels, and so every decision, as in the
// numbering of the method (new id = rank of every used label), which is recovered where it is
// needed from rep[x], the original vertex that labels super-vertex x's line of communities: the
// numbering's order of super-vertices is the order of their representatives, and its id of x
// is x plus the number of vertices without arcs (one singleton community each, at every level)
// whose id is below rep[x].

// rep of the next level: that of each new id's old label (rep null: the old label itself).
__global__ void k_next_rep(int64_t np, const int32_t* oldlabel, const int32_t* rep,
                           int32_t* rep_next) {
  for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < np;
       a += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = oldlabel[a];
    rep_next[a] = rep ? rep[c] : c;
  }
}

// flag[v] = 1 for the vertices of g without arcs.
__global__ void k_no_arc_flags(const int64_t* rs, const int64_t* re, int64_t n, int32_t* flag) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    flag[v] = re[v] > rs[v] ? 0 : 1;
}

// flag[rep[x]] = 1 for every super-vertex x (flag zero before).
__global__ void k_mark_reps(int64_t nl, const int32_t* rep, int32_t* flag) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < nl;
       x += (int64_t)gridDim.x * blockDim.x)
    flag[rep[x]] = 1;
}

// Hashed class of every super-vertex by its id in the method's numbering.
__global__ void k_live_classes(int64_t nl, int32_t pass, int32_t K, const int32_t* rep,
                               const int64_t* noarc_before, uint8_t* vclass) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < nl;
       x += (int64_t)gridDim.x * blockDim.x)
    vclass[x] = (uint8_t)vertex_class(pass, K, x + noarc_before[rep[x]]);
}

// Membership in the method's numbering from the live one (top[v] < 0: v has no arcs).
// live_before[y]: super-vertices whose representative is below y.
__global__ void k_canon_membership(int64_t n0, const int32_t* top, const int32_t* rep,
                                   const int64_t* noarc_before, const int64_t* live_before,
                                   int32_t* out) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n0;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = top[v];
    out[v] = x >= 0 ? (int32_t)(x + noarc_before[rep[x]])
                    : (int32_t)(live_before[v] + noarc_before[v]);
  }
}

hipError_t next_rep(int64_t np, const int32_t* oldlabel, const int32_t* rep, int32_t* rep_next,
                    hipStream_t s) {
  if (np <= 0) return hipSuccess;
  LV_LAUNCH(k_next_rep, grid_for(np), kBlock, 0, s, np, oldlabel, rep, rep_next);
  return hipGetLastError();
}

hipError_t no_arc_prefix(const DevGraph& g, int32_t* flag, int64_t* noarc_before,
                         int64_t* partial, hipStream_t s) {
  LV_LAUNCH(k_no_arc_flags, grid_for(g.n), kBlock, 0, s, g.rs, g.re, g.n, flag);
  return scan_flags_pos(flag, g.n, noarc_before, partial, s);
}

hipError_t live_classes(int64_t nl, int32_t pass, int32_t K, const int32_t* rep,
                        const int64_t* noarc_before, uint8_t* vclass, hipStream_t s) {
  if (nl <= 0) return hipSuccess;
  LV_LAUNCH(k_live_classes, grid_for(nl), kBlock, 0, s, nl, pass, K, rep, noarc_before, vclass);
  return hipGetLastError();
}

hipError_t canon_membership(int64_t n0, const int32_t* top, int64_t nl, const int32_t* rep,
                            const int64_t* noarc_before, int32_t* flag, int64_t* live_before,
                            int64_t* partial, int32_t* out, hipStream_t s) {
  if (n0 <= 0) return hipSuccess;
  LV_LAUNCH(k_fill_i32, grid_for(n0), kBlock, 0, s, flag, 0, n0);
  if (nl > 0) LV_LAUNCH(k_mark_reps, grid_for(nl), kBlock, 0, s, nl, rep, flag);
  hipError_t e = scan_flags_pos(flag, n0, live_before, partial, s);
  if (e != hipSuccess) return e;
  LV_LAUNCH(k_canon_membership, grid_for(n0), kBlock, 0, s, n0, top, rep, noarc_before,
            live_before, out);
  return hipGetLastError();
}

// Super-arc weights: 32-bit when every community's Sigma (which bounds the weight of each of
// its super-arcs) is below 2^32, else 64-bit.
struct WOut {
  uint64_t* w64;
  uint32_t* w32;
  __device__ __forceinline__ void put(int64_t i, ull v) const {
    if (w32) w32[i] = (uint32_t)v;
    else w64[i] = v;
  }
  __device__ __forceinline__ WOut at(int64_t off) const {
    WOut o;
    o.w64 = w32 ? nullptr : w64 + off;
    o.w32 = w32 ? w32 + off : nullptr;
    return o;
  }
};

// The map in 16 bits, for aggregations into fewer than 0xFFFF super-vertices: the merge kernels
// gather a neighbour's new id per arc, at random, and the narrower copy of a graph of ~2·10⁶
// vertices fits an XCD's L2 (R-MAT s25's aggregation after pass 1: 7.4 -> 3.7 MB).
__global__ void k_narrow_map(const int32_t* map, int64_t n, uint16_t* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = map[i] < 0 ? (uint16_t)0xFFFF : (uint16_t)map[i];
}
hipError_t narrow_map(const int32_t* map, int64_t n, uint16_t* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_narrow_map, grid_for(n), kBlock, 0, s, map, n, out);
  return hipGetLastError();
}

// A neighbour's new id from the 16-bit map when there is one (see narrow_map), else the 32-bit
constexpr uint16_t kNoMap16 = 0xFFFF;
__device__ __forceinline__ int32_t map_of(const int32_t* map, const uint16_t* map16, int32_t j) {
  if (map16) {
    const uint16_t x = map16[j];
    return x == kNoMap16 ? -1 : (int32_t)x;
  }
  return map[j];
}

template <typename WT>
struct MergeArgs {
  const int64_t* rs;
  const int32_t* idx;
  const WT* w;
  const int32_t* map;
  const uint16_t* map16;  // the same in 16 bits (kNoMap16: no arcs), or null
  const int32_t* members;
  const int64_t* mstart;
  const int64_t* gscan;
  const int64_t* astart;
  const int64_t* A;
  const int64_t* newid;
  int32_t* okey;     // output arrays: row of community c at astart[c]
  WOut ow;
  int64_t* dcount;   // distinct targets per new id
  ull* partial;      // per block: weight of its self super-arcs
  ull* stats;        // [0] weight of self super-arcs (added to directly by the mid merge)
  const int32_t* list;
  int64_t bstart[8];
  int64_t lstart[8];
  const int32_t* gid;  // batches: graph of every label, and per-graph self super-arc weights
  ull* gself;
};

template <typename WT, int G, int LOG2H>
__device__ __forceinline__ void merge_group(const MergeArgs<WT>& a, int64_t lb, int64_t lbase,
                                            int64_t lcount, unsigned char* smem, int* gcount,
                                            ull* red) {
  constexpr int H = 1 << LOG2H;
  constexpr int M = H / 2;  // members <= arcs <= H/2
  constexpr int NG = kBlock / G;
  int32_t* keys = (int32_t*)smem;
  ull* vals = (ull*)(smem + (size_t)NG * H * sizeof(int32_t));
  int32_t* mvert = (int32_t*)(smem + (size_t)NG * H * (sizeof(int32_t) + sizeof(ull)));
  int32_t* mfirst = mvert + NG * M;
  const int gid = threadIdx.x / G, lane = threadIdx.x % G;
  const int64_t li = lb * NG + gid;
  const bool valid = li < lcount;
  const int32_t c = valid ? a.list[lbase + li] : 0;
  int32_t* gk = keys + gid * H;
  ull* gv = vals + gid * H;
  int32_t* gm = mvert + gid * M;
  int32_t* gf = mfirst + gid * M;
  for (int s = lane; s < H; s += G) {
    gk[s] = kEmpty;
    gv[s] = 0;
  }
  int64_t a0 = 0, L = 0;
  int mc = 0;
  if (valid) {
    const int64_t m0 = a.mstart[c];
    mc = (int)(a.mstart[c + 1] - m0);
    a0 = a.astart[c];
    L = a.A[c];
    for (int i = lane; i < mc; i += G) {
      gm[i] = a.members[m0 + i];
      gf[i] = (int32_t)(a.gscan[m0 + i] - a0);
    }
  }
  if (lane == 0) gcount[gid] = 0;
  __syncthreads();
  constexpr int U = (1 << LOG2H) / 2 > G ? 4 : 1;  // arcs per lane gathered together
  for (int64_t t = lane; t < L; t += (int64_t)U * G) {
    int64_t e[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t tu = t + (int64_t)u * G;
      e[u] = -1;
      if (tu < L) {
        const int i = member_at(gf, mc, tu);
        e[u] = a.rs[gm[i]] + (tu - gf[i]);
      }
    }
    int32_t j[U];
    ull wv[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      j[u] = e[u] >= 0 ? a.idx[e[u]] : 0;
      wv[u] = e[u] >= 0 ? (ull)a.w[e[u]] : 0;
    }
    int32_t key[U];
#pragma unroll
    for (int u = 0; u < U; u++) key[u] = e[u] >= 0 ? map_of(a.map, a.map16, j[u]) : kEmpty;
#pragma unroll
    for (int u = 0; u < U; u++)
      if (key[u] != kEmpty) table_add<ull>(gk, gv, LOG2H, key[u], wv[u]);
  }
  __syncthreads();
  ull self = 0;
  if (valid) {
    const int32_t me = (int32_t)a.newid[c];
    for (int s = lane; s < H; s += G) {
      const int32_t key = gk[s];
      if (key == kEmpty) continue;
      const int p = atomicAdd(&gcount[gid], 1);
      a.okey[a0 + p] = key;
      a.ow.put(a0 + p, gv[s]);
      if (key == me) {
        self = gv[s];
        if (a.gself) atomicAdd(&a.gself[a.gid[c]], self);
      }
    }
  }
  __syncthreads();
  if (valid && lane == 0) a.dcount[a.newid[c]] = gcount[gid];
  const ull bs = block_sum_u64(self, red);
  if (threadIdx.x == 0) a.partial[blockIdx.x] = bs;
}

__global__ __launch_bounds__(kBlock) void k_reduce_sum(const ull* part, int64_t nb, ull* out) {
  __shared__ ull red[kBlock / 64];
  ull t = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nb;
       i += (int64_t)gridDim.x * blockDim.x)
    t += part[i];
  t = block_sum_u64(t, red);
  if (threadIdx.x == 0 && t) atomicAdd(out, t);
}

int64_t merge_lds_blocks(const Buckets& b) {
  int64_t blocks = 0;
  for (int k = 0; k < kFusedClasses; k++) {
    const int64_t rpb = bucket_rows_per_block(k);
    blocks += (b.count[k] + rpb - 1) / rpb;
  }
  return blocks;
}

template <typename WT>
__global__ __launch_bounds__(kBlock) void k_merge_lds(MergeArgs<WT> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int gcount[kBlock / 4];
  __shared__ ull red[kBlock / 64];
  const int64_t b = blockIdx.x;
  int k = 0;
  while (k < 6 && b >= a.bstart[k + 1]) k++;
  const int64_t lb = b - a.bstart[k];
  const int64_t lbase = a.lstart[k], lcount = a.lstart[k + 1] - a.lstart[k];
  switch (k) {
    case 0: merge_group<WT, bucket_group(0), bucket_log2h(0)>(a, lb, lbase, lcount, smem, gcount, red); break;
    case 1: merge_group<WT, bucket_group(1), bucket_log2h(1)>(a, lb, lbase, lcount, smem, gcount, red); break;
    case 2: merge_group<WT, bucket_group(2), bucket_log2h(2)>(a, lb, lbase, lcount, smem, gcount, red); break;
    case 3: merge_group<WT, bucket_group(3), bucket_log2h(3)>(a, lb, lbase, lcount, smem, gcount, red); break;
    case 4: merge_group<WT, bucket_group(4), bucket_log2h(4)>(a, lb, lbase, lcount, smem, gcount, red); break;
    case 5: merge_group<WT, bucket_group(5), bucket_log2h(5)>(a, lb, lbase, lcount, smem, gcount, red); break;
    default: merge_group<WT, bucket_group(6), bucket_log2h(6)>(a, lb, lbase, lcount, smem, gcount, red); break;
  }
}

static size_t merge_table_bytes(int k) {
  // table (key + 8-byte value) and the member arrays (vertex + first flat arc)
  const size_t H = (size_t)1 << bucket_log2h(k);
  return (size_t)bucket_rows_per_block(k) * (H * 12 + (H / 2) * 8);
}

template <typename WT>
static hipError_t merge_lds_t(const DevGraph& g, const Buckets& b, const AggBuffers& ag,
                              hipStream_t s) {
  MergeArgs<WT> a;
  a.rs = g.rs;
  a.idx = g.idx;
  a.w = (const WT*)g.w;
  a.map = ag.map;
  a.map16 = ag.map16;
  a.members = ag.members;
  a.mstart = ag.mstart;
  a.gscan = ag.gscan;
  a.astart = ag.astart;
  a.A = ag.A;
  a.newid = ag.newid;
  a.okey = ag.okey;
  a.ow.w64 = ag.ow;
  a.ow.w32 = ag.w32 ? (uint32_t*)ag.ow : nullptr;
  a.dcount = ag.dcount;
  a.partial = ag.block_partial;
  a.list = ag.list;
  a.gid = ag.gs.gid;
  a.gself = ag.gs.gself;
  int64_t blocks = 0;
  size_t shm = 0;
  for (int k = 0; k < kFusedClasses; k++) {
    a.bstart[k] = blocks;
    a.lstart[k] = b.lstart[k];
    const int64_t rpb = bucket_rows_per_block(k);
    blocks += (b.count[k] + rpb - 1) / rpb;
    if (b.count[k]) shm = std::max(shm, merge_table_bytes(k));
  }
  a.bstart[7] = blocks;
  a.lstart[7] = b.lstart[kFusedClasses];
  if (blocks == 0) return hipSuccess;
  LV_LAUNCH(k_merge_lds<WT>, (unsigned)blocks, kBlock, shm, s, a);
  LV_LAUNCH(k_reduce_sum, grid_for(blocks, kBlock, 256), kBlock, 0, s, a.partial, blocks,
            ag.stats);
  return hipGetLastError();
}

hipError_t merge_lds(const DevGraph& g, const Buckets& b, const AggBuffers& ag, hipStream_t s) {
  return g.w64 ? merge_lds_t<uint64_t>(g, b, ag, s) : merge_lds_t<uint32_t>(g, b, ag, s);
}

// Communities of bucket classes 7 to 9 (1025 to 8192 arcs): one workgroup per community,
// listed directly, with the whole community in one LDS table of twice its arc bound. Its
// members' first flat arcs are staged in LDS (16-bit offsets), so locating the member of an arc
// is an LDS search; class 7 also stages each member's displacement from flat arc to row
// position, while classes 8 and 9 ("lean", to fit two or one workgroups per CU) read the
// member's vertex and row start per arc from global memory (cached: a wave's lanes mostly share
// one member). A workgroup's chain of dependent global loads is the community's bounds, its
// member list, and per arc the arc itself and its target's new id. Lanes take consecutive flat
// arcs, U of them per round.
template <int K>
struct MidShape {
  static_assert(K >= 7 && K <= 9, "mid merge classes");
  static constexpr int kLog2H = K == 7 ? 12 : K == 8 ? 13 : 14;  // twice the arc bound
  static constexpr int kBlock = K == 7 ? 256 : 1024;
  static constexpr bool kLean = K >= 8;
  static constexpr int kMembers = 1 << (kLog2H - 1);  // members <= arcs <= H / 2
};

template <int K>
__host__ __device__ constexpr size_t mid_lds_bytes(int vb) {
  return (size_t)MidShape<K>::kMembers * ((MidShape<K>::kLean ? 0 : 8) + 2) +
         ((size_t)1 << MidShape<K>::kLog2H) * (4 + (size_t)vb);
}

template <typename WT, typename V, int K>
__global__ __launch_bounds__(MidShape<K>::kBlock) void k_merge_mid(MergeArgs<WT> a,
                                                                   int64_t lbase) {
  constexpr int LOG2H = MidShape<K>::kLog2H;
  constexpr int H = 1 << LOG2H;
  constexpr int M = MidShape<K>::kMembers;
  constexpr int B = MidShape<K>::kBlock;
  constexpr bool LEAN = MidShape<K>::kLean;
  constexpr int U = 4;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int cnt;
  __shared__ ull red[B / 64];
  int64_t* disp = (int64_t*)smem;                      // [M] (not lean) flat arc t of member
  int32_t* keys = (int32_t*)(disp + (LEAN ? 0 : M));   // [H]  i sits at row position disp[i] + t
  V* vals = (V*)(keys + H);                            // [H]
  int16_t* mfirst = (int16_t*)(vals + H);              // [M] first flat arc of each member
  const int32_t c = a.list[lbase + blockIdx.x];
  const int64_t m0 = a.mstart[c];
  const int mc = (int)(a.mstart[c + 1] - m0);
  const int64_t a0 = a.astart[c];
  const int L = (int)a.A[c];
  const int32_t me = (int32_t)a.newid[c];
  for (int s = threadIdx.x; s < H; s += B) {
    keys[s] = kEmpty;
    vals[s] = 0;
  }
  for (int i = threadIdx.x; i < mc; i += B) {
    const int64_t first = a.gscan[m0 + i] - a0;
    mfirst[i] = (int16_t)first;
    if (!LEAN) disp[i] = a.rs[a.members[m0 + i]] - first;
  }
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int t = threadIdx.x; t < L; t += U * B) {
    int64_t e[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int tu = t + u * B;
      e[u] = -1;
      if (tu < L) {
        const int i = member_at(mfirst, mc, tu);
        e[u] = LEAN ? a.rs[a.members[m0 + i]] + (tu - mfirst[i]) : disp[i] + tu;
      }
    }
    int32_t j[U];
    V wv[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      j[u] = e[u] >= 0 ? a.idx[e[u]] : 0;
      wv[u] = e[u] >= 0 ? (V)a.w[e[u]] : 0;
    }
    int32_t key[U];
#pragma unroll
    for (int u = 0; u < U; u++) key[u] = e[u] >= 0 ? map_of(a.map, a.map16, j[u]) : kEmpty;
#pragma unroll
    for (int u = 0; u < U; u++)
      if (key[u] != kEmpty) table_add<V>(keys, vals, LOG2H, key[u], wv[u]);
  }
  __syncthreads();
  ull self = 0;
  for (int s = threadIdx.x; s < H; s += B) {
    const int32_t key = keys[s];
    if (key == kEmpty) continue;
    const int p = atomicAdd(&cnt, 1);
    a.okey[a0 + p] = key;
    a.ow.put(a0 + p, (ull)vals[s]);
    if (key == me) {
      self = (ull)vals[s];
      if (a.gself) atomicAdd(&a.gself[a.gid[c]], self);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) a.dcount[me] = cnt;
  self = group_sum_u64<64>(self);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = self;
  __syncthreads();
  if (threadIdx.x == 0) {
    ull t = 0;
    for (int i = 0; i < B / 64; i++) t += red[i];
    if (t) atomicAdd(&a.stats[0], t);
  }
}

int merge_part_first_class(size_t max_lds, bool w32) {
  const int vb = w32 ? 4 : 8;
  if (mid_lds_bytes<7>(vb) + 2048 > max_lds) return 7;
  if (mid_lds_bytes<8>(vb) + 2048 > max_lds) return 8;
  if (mid_lds_bytes<9>(vb) + 2048 > max_lds) return 9;
  return 10;
}

template <typename WT, typename V, int K>
static hipError_t launch_mid(const MergeArgs<WT>& a, const Buckets& b, hipStream_t s) {
  const int64_t rows = b.count[K];
  if (rows <= 0) return hipSuccess;
  constexpr size_t shm = mid_lds_bytes<K>((int)sizeof(V));
  static const bool attr = [] {  // once, thread-safe (see launch_wg)
    (void)hipFuncSetAttribute((const void*)k_merge_mid<WT, V, K>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    return true;
  }();
  (void)attr;
  LV_LAUNCH((k_merge_mid<WT, V, K>), (unsigned)rows, MidShape<K>::kBlock, shm, s, a,
            b.lstart[K]);
  return hipGetLastError();
}

template <typename WT, typename V>
static hipError_t merge_mid_t(const DevGraph& g, const Buckets& b, const AggBuffers& ag,
                              int part_first, hipStream_t s) {
  MergeArgs<WT> a;
  a.rs = g.rs;
  a.idx = g.idx;
  a.w = (const WT*)g.w;
  a.map = ag.map;
  a.map16 = ag.map16;
  a.members = ag.members;
  a.mstart = ag.mstart;
  a.gscan = ag.gscan;
  a.astart = ag.astart;
  a.A = ag.A;
  a.newid = ag.newid;
  a.okey = ag.okey;
  a.ow.w64 = ag.ow;
  a.ow.w32 = ag.w32 ? (uint32_t*)ag.ow : nullptr;
  a.dcount = ag.dcount;
  a.stats = ag.stats;
  a.list = ag.list;
  a.gid = ag.gs.gid;
  a.gself = ag.gs.gself;
  hipError_t e = hipSuccess;
  if (part_first > 7 && (e = launch_mid<WT, V, 7>(a, b, s)) != hipSuccess) return e;
  if (part_first > 8 && (e = launch_mid<WT, V, 8>(a, b, s)) != hipSuccess) return e;
  if (part_first > 9 && (e = launch_mid<WT, V, 9>(a, b, s)) != hipSuccess) return e;
  return hipSuccess;
}

hipError_t merge_mid(const DevGraph& g, const Buckets& b, const AggBuffers& ag, int part_first,
                     hipStream_t s) {
  if (ag.w32)
    return g.w64 ? merge_mid_t<uint64_t, uint32_t>(g, b, ag, part_first, s)
                 : merge_mid_t<uint32_t, uint32_t>(g, b, ag, part_first, s);
  return g.w64 ? merge_mid_t<uint64_t, ull>(g, b, ag, part_first, s)
               : merge_mid_t<uint32_t, ull>(g, b, ag, part_first, s);
}

// Communities of more than 1024 arcs: the two-phase path over their flat arc ranges. Values are
// weight sums of V (4 bytes when every community's Sigma, which bounds them, is below 2^32,
// else 8): phase 1 covers part_chunk(sizeof(V)) flat arcs per workgroup (8192 or 4096), each
// thread a run of consecutive flat arcs (one member search, then a forward walk); a community of
// one chunk is finished there, others are finished by one phase-2 workgroup per partition.
template <typename WT, typename V>
struct MergeHubArgs {
  const int64_t* rs;
  const int32_t* idx;
  const WT* w;
  const int32_t* map;
  const uint16_t* map16;
  const int32_t* members;
  const int64_t* mstart;
  const int64_t* gscan;
  const int64_t* astart;
  const int64_t* A;
  const int64_t* newid;
  int32_t* okey;
  WOut ow;
  int64_t* dcount;   // distinct targets per new id (zero before the merge)
  ull* stats;        // [0] weight of self super-arcs
  const int32_t* hubs;
  int64_t nh;
  const int64_t* chunk_start;
  const int64_t* block_start;
  const int64_t* part_start;
  const int64_t* hoff_start;
  const int64_t* rper;
  const int64_t* nparts;
  int32_t* pk;
  V* pv;
  int32_t* hoff;
  int32_t* nflush;
  int32_t* cfm;      // per chunk row: its first member (index among its community's members)
  int cap;
  const int32_t* gid;  // batches: graph of every label, and per-graph self super-arc weights
  ull* gself;
};

template <typename V>
struct MergeShape {
  static constexpr int kChunk = part_chunk((int)sizeof(V));
  static constexpr int kLog2H = part_log2h((int)sizeof(V));
  static constexpr int kPerThread = kChunk / kPartBlock;
};

// Write the LDS table's entries to the community's output row at row + base + (claimed
// position), base = atomicAdd(dcount, entries) when `shared_row`, else 0 with *dcount = entries.
// Returns the weight of the entry keyed `me` (this thread's share). flags[2..3]: shared ints.
template <typename V>
__device__ ull merge_emit_table(const int32_t* keys, const V* vals, int H, int32_t me,
                                int32_t* okey, WOut ow, int64_t* dcount, bool shared_row,
                                int* flags, int64_t* base_sh, ull* gself) {
  int mine = 0;
  for (int s = threadIdx.x; s < H; s += kPartBlock) mine += keys[s] != kEmpty;
  if (threadIdx.x == 0) {
    flags[2] = 0;
    flags[3] = 0;
  }
  __syncthreads();
  if (mine) atomicAdd(&flags[2], mine);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int tot = flags[2];
    if (shared_row) {
      *base_sh = tot ? (int64_t)atomicAdd((ull*)dcount, (ull)tot) : 0;
    } else {
      *base_sh = 0;
      *dcount = tot;
    }
  }
  __syncthreads();
  const int64_t base = *base_sh;
  ull self = 0;
  for (int s = threadIdx.x; s < H; s += kPartBlock) {
    const int32_t key = keys[s];
    if (key == kEmpty) continue;
    const int64_t pos = base + atomicAdd(&flags[3], 1);
    okey[pos] = key;
    ow.put(pos, (ull)vals[s]);
    if (key == me) {
      self = (ull)vals[s];
      if (gself) atomicAdd(gself, self);
    }
  }
  return self;
}

__device__ __forceinline__ ull part_block_sum(ull x, ull* red) {
  x = group_sum_u64<64>(x);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  ull t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kPartBlock / 64; i++) t += red[i];
  __syncthreads();
  return t;
}

// Chunk k of community c's flat arc range. The members covering the chunk (from the chunk's
// first member, found beforehand by k_chunk_members) have their first flat arcs staged in LDS
// as 16-bit offsets from the chunk start (the first member's clamped to 0; its true first arc
// kept apart), in the aux region that table flushes use between chunks. Lanes then take
// consecutive flat arcs, U per round: the member of an arc is an LDS search, its row start a
// load shared by the lanes of that member, and the arc loads of a wave are contiguous within a
// row.
template <typename WT, typename V>
struct MergeChunk {
  static constexpr int kMergeChunk = MergeShape<V>::kChunk;
  static constexpr int kMergeLog2H = MergeShape<V>::kLog2H;
  const MergeHubArgs<WT, V>* a;
  int64_t m0, a0, L, row0;
  int mc;
  int16_t* mf;  // aux LDS, kMergeChunk + 1 entries
  static_assert(kAuxInts * 4 >= (kMergeChunk + 1) * 2, "chunk members fit the aux LDS");
  static_assert(kMergeChunk < 32768, "16-bit offsets within a chunk");
  __device__ void operator()(int64_t k, int32_t* keys, V* vals, int* flags) {
    constexpr int U = 4;
    __shared__ int span[2];
    __shared__ int64_t f0;
    const int64_t c0 = k * kMergeChunk;
    const int n = (int)(c0 + kMergeChunk < L ? kMergeChunk : L - c0);
    if (threadIdx.x == 0) {
      const int i0 = a->cfm[row0 + k];
      span[0] = i0;
      // members up to the one holding the next chunk's first arc (or the last member)
      span[1] = c0 + kMergeChunk < L ? a->cfm[row0 + k + 1] : mc - 1;
      f0 = a->gscan[m0 + i0] - a0;
    }
    __syncthreads();
    const int s0 = span[0];
    const int nm = span[1] - s0 + 1;
    for (int i = threadIdx.x; i < nm; i += kPartBlock) {
      const int64_t f = a->gscan[m0 + s0 + i] - a0 - c0;
      mf[i] = (int16_t)(f > 0 ? f : 0);
    }
    __syncthreads();
    const int64_t first0 = f0;
    int fresh = 0;
    for (int t = threadIdx.x; t < n; t += U * kPartBlock) {
      int64_t e[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int tu = t + u * kPartBlock;
        e[u] = -1;
        if (tu < n) {
          const int i = member_at(mf, nm, tu);
          const int64_t f = i == 0 ? first0 : c0 + mf[i];
          e[u] = a->rs[a->members[m0 + s0 + i]] + (c0 + tu - f);
        }
      }
      int32_t j[U];
      V wv[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        j[u] = e[u] >= 0 ? a->idx[e[u]] : 0;
        wv[u] = e[u] >= 0 ? (V)a->w[e[u]] : 0;
      }
      int32_t key[U];
#pragma unroll
      for (int u = 0; u < U; u++) key[u] = e[u] >= 0 ? map_of(a->map, a->map16, j[u]) : kEmpty;
#pragma unroll
      for (int u = 0; u < U; u++)
        if (key[u] != kEmpty) fresh += table_add<V>(keys, vals, kMergeLog2H, key[u], wv[u]);
    }
    if (fresh) atomicAdd(&flags[0], fresh);
  }
};

// First member of every chunk row of the two-phase merge (one thread per row).
template <typename WT, typename V>
__global__ void k_chunk_members(MergeHubArgs<WT, V> a, int64_t rows) {
  constexpr int Q = MergeShape<V>::kChunk;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t h = find_segment(a.chunk_start, a.nh, r);
    const int32_t c = a.hubs[h];
    const int64_t m0 = a.mstart[c];
    const int mc = (int)(a.mstart[c + 1] - m0);
    const int64_t t = a.astart[c] + (r - a.chunk_start[h]) * Q;
    a.cfm[r] = member_at(a.gscan + m0, mc, t);
  }
}

template <typename WT, typename V>
__global__ __launch_bounds__(kPartBlock) void k_merge_part(MergeHubArgs<WT, V> a) {
  constexpr int kMergeChunk = MergeShape<V>::kChunk;
  constexpr int kMergeLog2H = MergeShape<V>::kLog2H;
  constexpr int H = 1 << kMergeLog2H;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int wsum[kPartBlock / 64 + 1];
  __shared__ int flags[4];
  __shared__ int64_t base_sh;
  __shared__ ull red[kPartBlock / 64];
  int32_t* keys = (int32_t*)smem;
  V* vals = (V*)(smem + (size_t)H * 4);
  int* cnt = (int*)(smem + (size_t)H * (4 + sizeof(V)));
  const int64_t b = blockIdx.x;
  const int64_t h = find_segment(a.block_start, a.nh, b);
  const int64_t i = b - a.block_start[h];
  const int64_t R = a.rper[h];
  const int64_t row0 = a.chunk_start[h], nck = a.chunk_start[h + 1] - row0;
  const int64_t k0 = i * R, k1 = k0 + R < nck ? k0 + R : nck;
  const int32_t c = a.hubs[h];
  MergeChunk<WT, V> acc;
  acc.a = &a;
  acc.m0 = a.mstart[c];
  acc.mc = (int)(a.mstart[c + 1] - acc.m0);
  acc.a0 = a.astart[c];
  acc.L = a.A[c];
  acc.row0 = row0;
  acc.mf = (int16_t*)cnt;
  if (nck == 1) {
    // the whole community in one table: write its row directly
    part_table_clear<V>(keys, vals, H);
    __syncthreads();
    acc(0, keys, vals, flags);
    __syncthreads();
    const int32_t me = (int32_t)a.newid[c];
    const ull self = merge_emit_table(keys, vals, H, me, a.okey + acc.a0, a.ow.at(acc.a0),
                                      a.dcount + me, false, flags, &base_sh,
                                      a.gself ? a.gself + a.gid[c] : nullptr);
    const ull bs = part_block_sum(self, red);
    if (threadIdx.x == 0 && bs) atomicAdd(&a.stats[0], bs);
    return;
  }
  const int P = (int)a.nparts[h];
  const int nf = part_walk<V, kMergeLog2H>(acc, k0, k1, P, keys, vals, cnt, wsum, flags,
                                             a.hoff + a.hoff_start[h] + k0 * (P + 1),
                                             a.pk + (row0 + k0) * kMergeChunk,
                                             a.pv + (row0 + k0) * kMergeChunk);
  if (threadIdx.x == 0) a.nflush[b] = nf;
}

template <typename V>
struct MergeFin {
  int32_t me;
  int32_t* okey;
  WOut ow;
  int64_t* dcount;
  int* flags;
  int64_t* base_sh;
  ull* gself;
  ull self;
  __device__ void operator()(const int32_t* keys, const V* vals, int H) {
    self += merge_emit_table(keys, vals, H, me, okey, ow, dcount, true, flags, base_sh, gself);
  }
};

template <typename WT, typename V>
__global__ __launch_bounds__(kPartBlock) void k_merge_reduce(MergeHubArgs<WT, V> a) {
  constexpr int kMergeChunk = MergeShape<V>::kChunk;
  constexpr int kMergeLog2H = MergeShape<V>::kLog2H;
  constexpr int H = 1 << kMergeLog2H;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int wsum[kPartBlock / 64 + 1];
  __shared__ int flags[4];
  __shared__ int64_t base_sh;
  __shared__ ull red[kPartBlock / 64];
  int32_t* keys = (int32_t*)smem;
  V* vals = (V*)(smem + (size_t)H * 4);
  unsigned char* aux = smem + (size_t)H * (4 + sizeof(V));
  const int64_t b = blockIdx.x;
  const int64_t h = find_segment(a.part_start, a.nh, b);
  const int p = (int)(b - a.part_start[h]);
  const int P = (int)a.nparts[h];
  const int64_t c0 = a.chunk_start[h], nck = a.chunk_start[h + 1] - c0;
  const int32_t c = a.hubs[h];
  const int64_t a0 = a.astart[c];
  MergeFin<V> fin;
  fin.me = (int32_t)a.newid[c];
  fin.okey = a.okey + a0;
  fin.ow = a.ow.at(a0);
  fin.dcount = a.dcount + fin.me;
  fin.flags = flags;
  fin.base_sh = &base_sh;
  fin.gself = a.gself ? a.gself + a.gid[c] : nullptr;
  fin.self = 0;
  part_reduce<V, kMergeLog2H, 0>(a.pk + c0 * kMergeChunk, a.pv + c0 * kMergeChunk,
                                   a.hoff + a.hoff_start[h], a.nflush + a.block_start[h], nck,
                                   a.rper[h], P, p, a.cap, keys, vals, aux, wsum, flags, fin);
  const ull bs = part_block_sum(fin.self, red);
  if (threadIdx.x == 0 && bs) atomicAdd(&a.stats[0], bs);
}

template <typename WT, typename V>
static hipError_t merge_hubs_t(const DevGraph& g, const Buckets& b, const PartPlan& pp,
                               const AggBuffers& ag, int part_first, hipStream_t s) {
  constexpr int vb = (int)sizeof(V);
  MergeHubArgs<WT, V> a;
  a.rs = g.rs;
  a.idx = g.idx;
  a.w = (const WT*)g.w;
  a.map = ag.map;
  a.map16 = ag.map16;
  a.members = ag.members;
  a.mstart = ag.mstart;
  a.gscan = ag.gscan;
  a.astart = ag.astart;
  a.A = ag.A;
  a.newid = ag.newid;
  a.okey = ag.okey;
  a.ow.w64 = ag.ow;
  a.ow.w32 = ag.w32 ? (uint32_t*)ag.ow : nullptr;
  a.dcount = ag.dcount;
  a.stats = ag.stats;
  a.hubs = ag.list + b.lstart[part_first];
  a.nh = pp.nh;
  a.chunk_start = pp.chunk_start;
  a.block_start = pp.block_start;
  a.part_start = pp.part_start;
  a.hoff_start = pp.hoff_start;
  a.rper = pp.rper;
  a.nparts = pp.nparts;
  a.pk = ag.pk;
  a.pv = (V*)ag.pv;
  a.hoff = ag.hoff;
  a.nflush = ag.nflush;
  a.gid = ag.gs.gid;
  a.gself = ag.gs.gself;
  a.cfm = ag.cfm;
  a.cap = part_round_cap(MergeShape<V>::kLog2H, pp.shift);
  static const bool attr = [] {  // once, thread-safe (see launch_wg)
    allow_part_lds(k_merge_part<WT, V>, vb);
    allow_part_lds(k_merge_reduce<WT, V>, vb);
    return true;
  }();
  (void)attr;
  const size_t shm = part_lds_bytes(vb);
  LV_LAUNCH((k_chunk_members<WT, V>), grid_for(pp.chunks), kBlock, 0, s, a, pp.chunks);
  LV_LAUNCH((k_merge_part<WT, V>), (unsigned)pp.blocks, kPartBlock, shm, s, a);
  if (pp.parts > 0)
    LV_LAUNCH((k_merge_reduce<WT, V>), (unsigned)pp.parts, kPartBlock, shm, s, a);
  return hipGetLastError();
}

hipError_t merge_hubs(const DevGraph& g, const Buckets& b, const PartPlan& pp,
                      const AggBuffers& ag, int part_first, hipStream_t s) {
  if (pp.nh <= 0) return hipSuccess;
  if (ag.w32)
    return g.w64 ? merge_hubs_t<uint64_t, uint32_t>(g, b, pp, ag, part_first, s)
                 : merge_hubs_t<uint32_t, uint32_t>(g, b, pp, ag, part_first, s);
  return g.w64 ? merge_hubs_t<uint64_t, ull>(g, b, pp, ag, part_first, s)
               : merge_hubs_t<uint32_t, ull>(g, b, pp, ag, part_first, s);
}

// Rows of the super-vertex graph where the merge left them.
__global__ void k_super_rows(int64_t np, const int32_t* oldlabel, const int64_t* astart,
                             const int64_t* dcount, int64_t* rs, int64_t* re) {
  for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < np;
       a += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = astart[oldlabel[a]];
    rs[a] = r;
    re[a] = r + dcount[a];
  }
}
hipError_t super_rows(int64_t np, const AggBuffers& ag, int64_t* rs, int64_t* re, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  LV_LAUNCH(k_super_rows, grid_for(np), kBlock, 0, s, np, ag.oldlabel, ag.astart, ag.dcount, rs,
            re);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_sum_i64(const int64_t* a, int64_t n, ull* out) {
  __shared__ ull red[kBlock / 64];
  ull t = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    t += (ull)a[i];
  t = block_sum_u64(t, red);
  if (threadIdx.x == 0 && t) atomicAdd(out, t);
}
hipError_t sum_i64(const int64_t* a, int64_t n, unsigned long long* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_sum_i64, grid_for(n, kBlock, 1024), kBlock, 0, s, a, n, out);
  return hipGetLastError();
}

// Gather the merged rows into the output CSR (thread per kSeg output arcs).
__global__ __launch_bounds__(kBlock) void k_compact_rows(const int64_t* offp, int64_t np,
                                                        int64_t nnzp, const int32_t* oldlabel,
                                                        const int64_t* astart,
                                                        const int32_t* tkey, const uint64_t* tw,
                                                        int32_t* idx_out, uint64_t* w_out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t e0 = t * kSeg;
  if (e0 >= nnzp) return;
  const int64_t e1 = e0 + kSeg < nnzp ? e0 + kSeg : nnzp;
  int64_t r = row_of_arc(offp, np, e0);
  int64_t rb = offp[r], rend = offp[r + 1];
  int64_t src = astart[oldlabel[r]];
  for (int64_t e = e0; e < e1; e++) {
    if (e >= rend) {
      r = advance_row(offp, np, r + 1, e);
      rb = offp[r];
      rend = offp[r + 1];
      src = astart[oldlabel[r]];
    }
    idx_out[e] = tkey[src + (e - rb)];
    w_out[e] = tw[src + (e - rb)];
  }
}
hipError_t compact_rows(const int64_t* offp, int64_t np, int64_t nnzp, const int32_t* oldlabel,
                        const int64_t* astart, const int32_t* tkey, const uint64_t* tw,
                        int32_t* idx_out, uint64_t* w_out, hipStream_t s) {
  if (nnzp <= 0) return hipSuccess;
  const int64_t threads = (nnzp + kSeg - 1) / kSeg;
  const unsigned grid = (unsigned)((threads + kBlock - 1) / kBlock);
  LV_LAUNCH(k_compact_rows, grid, kBlock, 0, s, offp, np, nnzp, oldlabel, astart, tkey, tw,
            idx_out, w_out);
  return hipGetLastError();
}

// =============================================================================================
// Batches of graphs packed with consecutive vertex ids: graph g owns vertices
// [gbase[g], gbase[g+1]). Communities never span graphs, so the aggregation of the union keeps
// every graph's super-vertices consecutive and in order.

__global__ void k_graph_ids(const int64_t* gbase, int64_t G, int64_t n, int32_t* gid) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = G;  // gbase[lo] <= v < gbase[hi]
    while (hi - lo > 1) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if (gbase[mid] <= v) lo = mid; else hi = mid;
    }
    gid[v] = (int32_t)lo;
  }
}
// gS[0 .. 2G) = sum over the kGainSlices copies (128-bit, per graph).
__global__ void k_fold_gain_slices(ull* gS, int64_t G) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < G;
       g += (int64_t)gridDim.x * blockDim.x) {
    u128 t = 0;
    for (int k = 0; k < kGainSlices; k++) {
      const ull* p = gS + 2 * ((int64_t)k * G + g);
      t += ((u128)p[1] << 64) | p[0];
    }
    gS[2 * g] = (ull)t;
    gS[2 * g + 1] = (ull)(t >> 64);
  }
}
hipError_t fold_gain_slices(ull* gS, int64_t G, hipStream_t s) {
  if (G <= 0) return hipSuccess;
  LV_LAUNCH(k_fold_gain_slices, grid_for(G), kBlock, 0, s, gS, G);
  return hipGetLastError();
}

hipError_t graph_ids(const int64_t* gbase, int64_t G, int64_t n, int32_t* gid, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_graph_ids, grid_for(n), kBlock, 0, s, gbase, G, n, gid);
  return hipGetLastError();
}

// Per-graph sums of x (out[g], 64-bit) or of x^2 (out[2g..2g+1], 128-bit) over the vertices.
// Each thread covers kSeg consecutive vertices and flushes when the graph changes; a block whose
// vertices all belong to one graph (graphs are contiguous ranges) adds its total once instead.
template <bool SQ>
__global__ __launch_bounds__(kBlock) void k_graph_sum(const uint64_t* x, int64_t n,
                                                     const int32_t* gid, ull* out) {
  __shared__ u128 red[kBlock / 64];
  const int64_t b0 = (int64_t)blockIdx.x * kBlock * kSeg;
  const int64_t b1 = b0 + kBlock * kSeg < n ? b0 + kBlock * kSeg : n;
  const int64_t v0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * kSeg;
  const int64_t v1 = v0 + kSeg < n ? v0 + kSeg : n;
  if (gid[b0] == gid[b1 - 1]) {
    u128 acc = 0;
    for (int64_t v = v0; v < v1; v++) acc += SQ ? (u128)x[v] * x[v] : (u128)x[v];
    acc = block_sum_u128(acc, red);
    if (threadIdx.x == 0 && acc) {
      if (SQ) atomic_add_u128(out + 2 * gid[b0], acc);
      else atomicAdd(out + gid[b0], (ull)acc);
    }
    return;
  }
  if (v0 >= n) return;
  int32_t g = gid[v0];
  u128 acc = 0;
  for (int64_t v = v0; v <= v1; v++) {
    const int32_t gv = v < v1 ? gid[v] : -1;
    if (gv != g) {
      if (acc) {
        if (SQ) atomic_add_u128(out + 2 * g, acc);
        else atomicAdd(out + g, (ull)acc);
      }
      acc = 0;
      g = gv;
    }
    if (v < v1) acc += SQ ? (u128)x[v] * x[v] : (u128)x[v];
  }
}
hipError_t graph_sums(const uint64_t* x, int64_t n, const int32_t* gid, bool squares,
                      unsigned long long* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t threads = (n + kSeg - 1) / kSeg;
  const unsigned grid = (unsigned)((threads + kBlock - 1) / kBlock);
  if (squares) LV_LAUNCH(k_graph_sum<true>, grid, kBlock, 0, s, x, n, gid, out);
  else LV_LAUNCH(k_graph_sum<false>, grid, kBlock, 0, s, x, n, gid, out);
  return hipGetLastError();
}

// First super-vertex of every graph after an aggregation: the rank of its first label.
__global__ void k_next_gbase(const int64_t* newid, const int64_t* gbase, int64_t G,
                             int64_t* out) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g <= G;
       g += (int64_t)gridDim.x * blockDim.x)
    out[g] = newid[gbase[g]];
}
hipError_t next_gbase(const int64_t* newid, const int64_t* gbase, int64_t G, int64_t* out,
                      hipStream_t s) {
  LV_LAUNCH(k_next_gbase, grid_for(G + 1), kBlock, 0, s, newid, gbase, G, out);
  return hipGetLastError();
}

// Membership as ids within each graph.
__global__ void k_localize(int32_t* memb, int64_t n, const int32_t* gid0, const int64_t* gfinal) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    memb[v] -= (int32_t)gfinal[gid0[v]];
}
hipError_t localize_membership(int32_t* memb, int64_t n, const int32_t* gid0,
                               const int64_t* gfinal, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_localize, grid_for(n), kBlock, 0, s, memb, n, gid0, gfinal);
  return hipGetLastError();
}

// Batch layout checks: every graph's first arc is at aptr[g] and every arc stays in its graph.
__global__ void k_validate_batch(const int64_t* off, int64_t n, int64_t nnz, const int32_t* idx,
                                 const int32_t* gid, const int64_t* gbase, const int64_t* aptr,
                                 int64_t G, unsigned int* bad) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t <= G && off[gbase[t]] != aptr[t]) atomicOr(bad, 1u);
  const int64_t e0 = t * kSeg;
  if (e0 >= nnz) return;
  const int64_t e1 = e0 + kSeg < nnz ? e0 + kSeg : nnz;
  int64_t r = row_of_arc(off, n, e0);
  for (int64_t e = e0; e < e1; e++) {
    if (e >= off[r + 1]) r = advance_row(off, n, r + 1, e);
    const int32_t g = gid[r];
    const int32_t j = idx[e];
    if (j < gbase[g] || j >= gbase[g + 1]) atomicOr(bad, 2u);
  }
}
hipError_t validate_batch(const DevGraph& g, const int32_t* gid, const int64_t* gbase,
                          const int64_t* aptr, int64_t G, unsigned int* bad, hipStream_t s) {
  const int64_t threads = std::max((g.nnz + kSeg - 1) / kSeg, G + 1);
  LV_LAUNCH(k_validate_batch, grid_for(threads, kBlock, 1 << 30), kBlock, 0, s, g.off, g.n,
            g.nnz, g.idx, gid, gbase, aptr, G, bad);
  return hipGetLastError();
}

__global__ void k_compose(int32_t* top, int64_t n, const int32_t* map) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = top[i];
    top[i] = x >= 0 ? map[x] : -1;  // -1: a vertex without arcs in the live numbering
  }
}
hipError_t compose_membership(int32_t* top, int64_t n, const int32_t* map, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_compose, grid_for(n), kBlock, 0, s, top, n, map);
  return hipGetLastError();
}
// As k_compose, leaving the vertices of graphs with keep[g] != 0 at their current level.
__global__ void k_compose_masked(int32_t* top, int64_t n, const int32_t* map,
                                 const int32_t* gid0, const uint8_t* keep) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (!keep[gid0[i]]) top[i] = map[top[i]];
}
hipError_t compose_membership_masked(int32_t* top, int64_t n, const int32_t* map,
                                     const int32_t* gid0, const uint8_t* keep, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_compose_masked, grid_for(n), kBlock, 0, s, top, n, map, gid0, keep);
  return hipGetLastError();
}

// Kernel-argument structs are passed by value: keep each far inside the 4 KiB kernarg segment.
static_assert(sizeof(MoveArgs<uint64_t>) <= 1024 && sizeof(WgArgs<uint64_t>) <= 1024 &&
                  sizeof(HubArgs<uint64_t, u128>) <= 1024 && sizeof(MergeArgs<uint64_t>) <= 1024 &&
                  sizeof(MergeHubArgs<uint64_t, ull>) <= 1024,
              "kernel arguments must stay small");

}  // namespace lv
