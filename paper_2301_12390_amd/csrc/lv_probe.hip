// Measurement kernel: the device's rate of random 4-byte gathers. The local-moving and
// aggregation kernels read one record (or one label) of a neighbour per arc, at positions
// with no locality, so this rate, not HBM bandwidth, is the ceiling they run against; it is
// measured here with the same kind of access and nothing else.
#include <hip/hip_runtime.h>

#include "lv_device.h"
#include "lv_internal.h"

namespace lv {

namespace {

constexpr int kProbeGathers = 64;       // gathers per thread
constexpr unsigned kProbeBlocks = 16384;

// MurmurHash3's 32-bit finaliser: spreads consecutive thread/gather numbers over the table
__device__ __forceinline__ uint32_t probe_hash(uint32_t x) {
  x ^= x >> 16;
  x *= 0x85ebca6bu;
  x ^= x >> 13;
  x *= 0xc2b2ae35u;
  x ^= x >> 16;
  return x;
}

// Thread t makes kProbeGathers gathers from the slice of workgroup b (slice b mod slices of
// `per` entries) and writes their sum, so that none of them can be dropped.
__global__ __launch_bounds__(kBlock) void k_gather_probe(const int32_t* __restrict__ table,
                                                        uint64_t per, uint32_t slices,
                                                        int32_t* out) {
  const uint32_t t = blockIdx.x * (uint32_t)kBlock + threadIdx.x;
  const uint64_t base = (uint64_t)(blockIdx.x % slices) * per;
  int32_t acc = 0;
#pragma unroll 16
  for (int q = 0; q < kProbeGathers; q++)
    acc += table[base + probe_hash(t * (uint32_t)kProbeGathers + (uint32_t)q) % per];
  out[t] = acc;
}

}  // namespace

int64_t probe_threads() { return (int64_t)kProbeBlocks * kBlock; }
int64_t probe_gathers() { return probe_threads() * kProbeGathers; }

hipError_t gather_probe(const int32_t* table, uint64_t n, uint32_t slices, int32_t* out,
                        hipStream_t s) {
  if (slices == 0 || n < slices) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gather_probe, dim3(kProbeBlocks), dim3(kBlock), 0, s, table, n / slices,
                     slices, out);
  return hipGetLastError();
}

}  // namespace lv
