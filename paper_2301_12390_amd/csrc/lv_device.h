// Device-side helpers of the gfx950 Louvain kernels: exact gain arithmetic, LDS/global
// open-addressing tables, wavefront and workgroup reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lv {

typedef unsigned long long ull;
typedef __int128 i128;
typedef unsigned __int128 u128;

constexpr int kBlock = 256;        // threads of every general-purpose kernel
constexpr int32_t kEmpty = -1;     // empty table key (community ids are >= 0)
constexpr int kNumBuckets = 8;     // degree classes, the last one being hubs

// Degree classes of the local-moving and aggregation kernels. Class k < 7 holds rows of length
// in (bucket_max(k-1), bucket_max(k)] and is handled by the fused LDS kernel: each class has a
// fixed group width (lanes per row) and a table with room for twice the row length, so open
// addressing always finds a free slot.
__host__ __device__ constexpr int64_t bucket_max(int k) {
  return k == 0 ? 4 : k == 1 ? 8 : k == 2 ? 16 : k == 3 ? 32 : k == 4 ? 64 : k == 5 ? 256 : 1024;
}
__host__ __device__ constexpr int bucket_group(int k) {
  return k == 0 ? 4 : k == 1 ? 8 : k == 2 ? 16 : k == 3 ? 32 : k == 4 ? 64 : k == 5 ? 64 : 256;
}
__host__ __device__ constexpr int bucket_log2h(int k) {
  return k == 0 ? 3 : k == 1 ? 4 : k == 2 ? 5 : k == 3 ? 6 : k == 4 ? 7 : k == 5 ? 9 : 11;
}
__host__ __device__ constexpr int bucket_rows_per_block(int k) { return kBlock / bucket_group(k); }

// Lanes per row of the move kernel in degree class k.
__host__ __device__ constexpr int move_group_size(int k) { return bucket_group(k); }
__host__ __device__ constexpr int move_rows_per_block(int k) { return kBlock / move_group_size(k); }

// Degree class 7 (rows of up to 2048 arcs) is decided by one 256-thread group per row with a
// 4096-slot LDS table; classes 8 and 9 (up to 4096, 8192 arcs) by one 1024-thread workgroup per
// row with an LDS table of 8192 or 16384 slots when the device allows such a workgroup
// allocation; class 10 (longer rows), and any class whose table does not fit, take the
// two-phase hub path. kDegClasses is the stride of the (vertex class, degree class) segments.
constexpr int kDegClasses = 12;
constexpr int kFusedClasses = 7;
constexpr int kHubClass = 10;
__host__ __device__ constexpr int wg_log2h(int k) { return k == 7 ? 12 : k == 8 ? 13 : 14; }

__host__ __device__ inline int bucket_of(int64_t len) {
  if (len <= 4) return 0;
  if (len <= 8) return 1;
  if (len <= 16) return 2;
  if (len <= 32) return 3;
  if (len <= 64) return 4;
  if (len <= 256) return 5;
  if (len <= 1024) return 6;
  if (len <= 2048) return 7;
  if (len <= 4096) return 8;
  if (len <= 8192) return 9;
  return kHubClass;
}

// Partial asynchrony: at most kMaxClasses vertex classes per iteration. The class of vertex v
// in pass p is floor(hi32(s) * K / 2^32) for s the SplitMix64 output number v+1 of the
// sequence started at state p (Steele, Lea, Flood 2014: s = mix(p + (v+1) * golden gamma)).
constexpr int kMaxClasses = 32;

__host__ __device__ inline uint64_t vertex_draw(int32_t pass, int64_t v) {
  uint64_t z = (uint64_t)(uint32_t)pass + ((uint64_t)v + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ inline int vertex_class(int32_t pass, int32_t K, int64_t v) {
  return (int)(((vertex_draw(pass, v) >> 32) * (uint64_t)(uint32_t)K) >> 32);
}

// Community state of the local-moving phase, one record per index x in [0, n): the community
// of vertex x, and the size and total weight Sigma of the community labelled x. Packing them
// puts Sigma[j] on the cache line that the gather of C[j] fetches, so a candidate community
// whose label is a neighbour of the deciding vertex costs no further memory traffic.
struct __align__(16) VRec {
  int32_t c;
  int32_t size;
  unsigned long long sig;
};

// Items too long for one workgroup's table (hub rows of the local-moving phase, communities with
// many arcs in the aggregation) are combined in two phases of kPartBlock-thread workgroups.
// Phase 1: each chunk of part_chunk(vb) arcs is combined in an LDS table of twice that many
// slots, and its distinct keys are written out grouped by partition (the top bits of a
// bijective hash of the key). Phase 2: one workgroup per (item, partition) combines the
// partition's keys from every chunk in an LDS table of 2^part_log2h(vb) slots. vb is the byte
// width of the summed values (4 or 8). Partitions are sized for half a table on average; a
// partition that holds more distinct keys is processed in several rounds over sub-ranges of the
// hash, which always ends because the hash is a bijection.
constexpr int kPartBlock = 1024;
constexpr int kMaxParts = 4096;
constexpr int kPartTile = 1024;  // bound rows whose segments phase 2 holds in LDS at once
__host__ __device__ constexpr int part_chunk(int vb) { return vb == 4 ? 8192 : 4096; }
__host__ __device__ constexpr int part_log2h(int vb) { return vb == 4 ? 14 : 13; }
// LDS of the phase kernels: keys, values, and kAuxInts ints of partition counters (phase 1) or
// segment bounds (phase 2: an int64 start and an int length per row of a tile).
constexpr int kAuxInts = kMaxParts + 4;
static_assert(kAuxInts * 4 >= kPartTile * 12 + 4, "phase-2 segment tile fits the aux LDS");
__host__ __device__ constexpr size_t part_lds_bytes(int vb) {
  return ((size_t)1 << part_log2h(vb)) * (4 + (size_t)vb) + (size_t)kAuxInts * 4;
}

// Keys a phase-2 round may claim before it is abandoned: 3/4 of the table, or (testing shift)
// a small fraction of the reduced partition size so that most partitions take several rounds.
__host__ __device__ constexpr int part_cap(int log2h) { return 3 * (1 << log2h) / 4; }
__host__ __device__ constexpr int part_round_cap(int log2h, int shift) {
  return shift == 0 ? part_cap(log2h)
                    : (((1 << log2h) >> (shift + 3)) > 8 ? ((1 << log2h) >> (shift + 3)) : 8);
}

// MurmurHash3's 32-bit finaliser (Appleby): a bijection on 32-bit values.
__host__ __device__ inline uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

// Partition of a key among 2^lp partitions.
__device__ __forceinline__ int part_of(int32_t key, int lp) {
  return lp == 0 ? 0 : (int)(fmix32((uint32_t)key) >> (32 - lp));
}

// ---------------------------------------------------------------------------------------------
// Exact gains. Narrow: 64-bit, exact when W * max_i K_i < 2^63 (both products and their
// difference fit). Wide: 128-bit, exact for W <= 2^62.

template <bool WIDE>
struct Gain;

template <>
struct Gain<false> {
  typedef int64_t T;
  typedef uint32_t V;  // table value type: k_{i->c} <= K_i < 2^32 here
  static __device__ __forceinline__ T lowest() { return INT64_MIN; }
  static __device__ __forceinline__ T of(uint64_t W, uint64_t k, uint64_t Ki, uint64_t S) {
    return (int64_t)(W * k) - (int64_t)(Ki * S);
  }
  // g_best - stay, known to lie in [1, 2^64)
  static __device__ __forceinline__ u128 diff(T a, T b) { return (u128)((uint64_t)a - (uint64_t)b); }
  static __device__ __forceinline__ T shfl_xor(T x, int m, int w) {
    return (T)__shfl_xor((long long)x, m, w);
  }
};

template <>
struct Gain<true> {
  typedef i128 T;
  typedef ull V;
  static __device__ __forceinline__ T lowest() { return (i128)((u128)1 << 127); }
  static __device__ __forceinline__ T of(uint64_t W, uint64_t k, uint64_t Ki, uint64_t S) {
    return (i128)((u128)W * k) - (i128)((u128)Ki * S);
  }
  static __device__ __forceinline__ u128 diff(T a, T b) { return (u128)(a - b); }
  static __device__ __forceinline__ T shfl_xor(T x, int m, int w) {
    ull lo = (ull)(u128)x, hi = (ull)((u128)x >> 64);
    lo = __shfl_xor(lo, m, w);
    hi = __shfl_xor(hi, m, w);
    return (i128)(((u128)hi << 64) | lo);
  }
};

// (gain, community) ordering: larger gain first, then smaller community id.
template <typename T>
__device__ __forceinline__ bool better(T g, int32_t c, T bg, int32_t bc) {
  return g > bg || (g == bg && c < bc);
}


// ---------------------------------------------------------------------------------------------
// Open-addressing tables (linear probing, multiplicative hashing on the top bits).

__device__ __forceinline__ uint32_t slot_of(int32_t key, int log2h) {
  return ((uint32_t)key * 0x9E3779B1u) >> (32 - log2h);
}

// Add w to the value of `key`, claiming a slot if the key is new. Returns true if this call
// claimed the slot (the key was not in the table). The table must have a free slot.
template <typename V>
__device__ __forceinline__ bool table_add(int32_t* keys, V* vals, int log2h, int32_t key, V w,
                                          uint32_t* slot_out = nullptr) {
  const uint32_t mask = (1u << log2h) - 1u;
  uint32_t s = slot_of(key, log2h);
  while (true) {
    int32_t prev = atomicCAS(&keys[s], kEmpty, key);
    if (prev == kEmpty || prev == key) {
      atomicAdd(&vals[s], w);
      if (slot_out) *slot_out = s;
      return prev == kEmpty;
    }
    s = (s + 1u) & mask;
  }
}

// As table_add, for a table that may receive more keys than it can hold: once `cap` slots are
// claimed (counted in *fresh), or when no free slot is found, *overflow is set and the table's
// contents are to be discarded by the caller. Keys already present are still combined.
template <typename V>
__device__ __forceinline__ void table_add_capped(int32_t* keys, V* vals, int log2h, int32_t key,
                                                 V w, int* fresh, int cap, int* overflow) {
  const uint32_t mask = (1u << log2h) - 1u;
  uint32_t s = slot_of(key, log2h);
  for (uint32_t probe = 0; probe <= mask; probe++) {
    const int32_t prev = atomicCAS(&keys[s], kEmpty, key);
    if (prev == kEmpty || prev == key) {
      atomicAdd(&vals[s], w);
      if (prev == kEmpty && atomicAdd(fresh, 1) >= cap) atomicExch(overflow, 1);
      return;
    }
    s = (s + 1u) & mask;
  }
  atomicExch(overflow, 1);
}

// ---------------------------------------------------------------------------------------------
// 128-bit accumulation in global memory: two 64-bit words with carry propagation. Additions are
// commutative modulo 2^128, so the final value does not depend on the order of the atomics.

__device__ __forceinline__ void atomic_add_u128(ull* lohi, u128 v) {
  ull lo = (ull)v, hi = (ull)(v >> 64);
  if (lo) {
    ull old = atomicAdd(&lohi[0], lo);
    if (old + lo < old) hi += 1;
  }
  if (hi) atomicAdd(&lohi[1], hi);
}

// ---------------------------------------------------------------------------------------------
// Wavefront (64 lanes) and workgroup reductions.

__device__ __forceinline__ u128 shfl_xor_u128(u128 x, int m, int w) {
  ull lo = (ull)x, hi = (ull)(x >> 64);
  lo = __shfl_xor(lo, m, w);
  hi = __shfl_xor(hi, m, w);
  return ((u128)hi << 64) | lo;
}

template <int W>
__device__ __forceinline__ u128 group_sum_u128(u128 x) {
#pragma unroll
  for (int m = W / 2; m >= 1; m >>= 1) x += shfl_xor_u128(x, m, W);
  return x;
}

template <int W>
__device__ __forceinline__ ull group_sum_u64(ull x) {
#pragma unroll
  for (int m = W / 2; m >= 1; m >>= 1) x += __shfl_xor(x, m, W);
  return x;
}

// Sum over the whole block of kBlock threads; the result is valid in thread 0.
// `red` is shared scratch of kBlock/64 entries; the call contains __syncthreads().
__device__ __forceinline__ u128 block_sum_u128(u128 x, u128* red) {
  x = group_sum_u128<64>(x);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[wave] = x;
  __syncthreads();
  u128 t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / 64; i++) t += red[i];
  __syncthreads();
  return t;
}

__device__ __forceinline__ ull block_sum_u64(ull x, ull* red) {
  x = group_sum_u64<64>(x);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[wave] = x;
  __syncthreads();
  ull t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / 64; i++) t += red[i];
  __syncthreads();
  return t;
}

// Row of arc e: the largest r with off[r] <= e (off has n+1 entries, off[n] = nnz > e).
__device__ __forceinline__ int64_t row_of_arc(const int64_t* off, int64_t n, int64_t e) {
  int64_t lo = 0, hi = n;  // invariant: off[lo] <= e < off[hi]
  while (hi - lo > 1) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (off[mid] <= e) lo = mid; else hi = mid;
  }
  return lo;
}

// Row of arc e given a row r with off[r] <= e (e < off[n]): a few linear steps (the common case
// of short rows), then a binary search, so long runs of empty rows cost O(log n), not O(run).
__device__ __forceinline__ int64_t advance_row(const int64_t* off, int64_t n, int64_t r,
                                               int64_t e) {
#pragma unroll 1
  for (int k = 0; k < 4; k++) {
    if (e < off[r + 1]) return r;
    r++;
  }
  int64_t lo = r, hi = n;  // off[lo] <= e < off[hi]
  while (hi - lo > 1) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (off[mid] <= e) lo = mid; else hi = mid;
  }
  return lo;
}

// Streamed reads of arrays touched once per iteration.
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) { return __builtin_nontemporal_load(p); }

}  // namespace lv
