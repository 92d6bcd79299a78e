// gfx950 kernels of partition and merge (the remedy section 3.2 and the conclusion of Sahu,
// arXiv 2301.12390, propose for the poor scaling of the shared-memory method: run partitions
// of the graph independently, then combine them). The parts are contiguous vertex ranges, so
// the union of their induced subgraphs keeps the input's vertex ids and is one batch of graphs
// for the batched driver; these kernels cut that union out of the input CSR and handle the
// labels around it.
#include <hip/hip_runtime.h>

#include "lv_device.h"
#include "lv_internal.h"

namespace lv {

namespace {

#define LV_LAUNCH(kernel, grid, block, shm, stream, ...)                          \
  do {                                                                            \
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shm, stream, __VA_ARGS__); \
  } while (0)

constexpr int64_t kPmSeg = 16;  // arcs per thread of the arc-segment kernel

inline unsigned grid_of(int64_t items, int64_t per_block = kBlock) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (unsigned)b;
}

// Part bounds balanced by arcs: bounds[k] is the least v with off[v] >= floor(k * nnz / P)
// (bounds[0] = 0, bounds[P] = n).
__global__ void k_pm_bounds(const int64_t* off, int64_t n, int64_t nnz, int64_t P,
                            int64_t* bounds) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k <= P;
       k += (int64_t)gridDim.x * blockDim.x) {
    if (k == 0 || k == P) {
      bounds[k] = k == 0 ? 0 : n;
      continue;
    }
    const int64_t target = (k * nnz) / P;
    int64_t lo = 0, hi = n;  // off[hi] = nnz >= target; find the least such index
    while (lo < hi) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if (off[mid] >= target) hi = mid; else lo = mid + 1;
    }
    bounds[k] = lo;
  }
}

// flag[e] = 1 when arc e joins two vertices of the same part (gid: part of every vertex).
// Grid-stride over segments of kPmSeg arcs (the grid is capped).
__global__ __launch_bounds__(kBlock) void k_pm_flags(const int64_t* off, int64_t n, int64_t nnz,
                                                    const int32_t* idx, const int32_t* gid,
                                                    const int64_t* vptr, int32_t* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * kPmSeg;
  for (int64_t e0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * kPmSeg; e0 < nnz;
       e0 += stride) {
    const int64_t e1 = e0 + kPmSeg < nnz ? e0 + kPmSeg : nnz;
    int64_t r = row_of_arc(off, n, e0);
    int64_t rend = off[r + 1];
    int32_t k = gid[r];
    int64_t lo = vptr[k], hi = vptr[k + 1];
    for (int64_t e = e0; e < e1; e++) {
      if (e >= rend) {
        r = advance_row(off, n, r + 1, e);
        rend = off[r + 1];
        k = gid[r];
        lo = vptr[k];
        hi = vptr[k + 1];
      }
      const int64_t j = idx[e];
      flag[e] = j >= lo && j < hi ? 1 : 0;
    }
  }
}

// The kept arcs at their scanned positions, and the offsets of the induced union.
template <typename WT>
__global__ void k_pm_compact(const int64_t* off, int64_t n, int64_t nnz, const int32_t* idx,
                             const WT* w, const int32_t* flag, const int64_t* pos,
                             int32_t* nidx, WT* nw, int64_t* noff) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += stride) {
    if (flag[e]) {
      nidx[pos[e]] = idx[e];
      nw[pos[e]] = w[e];
    }
  }
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n; v += stride)
    noff[v] = pos[off[v]];
}

// aptr[k] = noff[vptr[k]]: the arc bounds of every part in the induced union.
__global__ void k_pm_arc_bounds(const int64_t* noff, const int64_t* vptr, int64_t P,
                                int64_t* aptr) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k <= P;
       k += (int64_t)gridDim.x * blockDim.x)
    aptr[k] = noff[vptr[k]];
}

// lab[v] += loff[gid[v]]: part-local community ids made distinct across parts.
__global__ void k_pm_offset_labels(int32_t* lab, int64_t n, const int32_t* gid,
                                   const int64_t* loff) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    lab[v] += (int32_t)loff[gid[v]];
}

}  // namespace

hipError_t part_bounds(const int64_t* off, int64_t n, int64_t nnz, int64_t P, int64_t* bounds,
                       hipStream_t s) {
  LV_LAUNCH(k_pm_bounds, grid_of(P + 1), kBlock, 0, s, off, n, nnz, P, bounds);
  return hipGetLastError();
}

hipError_t part_induced(const DevGraph& g, const int32_t* gid, const int64_t* vptr, int64_t P,
                        int32_t* flag, int64_t* pos, int64_t* partial, int32_t* nidx, void* nw,
                        int64_t* noff, int64_t* aptr, hipStream_t s) {
  hipError_t e;
  if (g.nnz > 0)
    LV_LAUNCH(k_pm_flags, grid_of((g.nnz + kPmSeg - 1) / kPmSeg), kBlock, 0, s, g.off, g.n,
              g.nnz, g.idx, gid, vptr, flag);
  if ((e = scan_flags_pos(flag, g.nnz, pos, partial, s)) != hipSuccess) return e;
  const int64_t items = g.nnz > g.n + 1 ? g.nnz : g.n + 1;
  if (g.w64)
    LV_LAUNCH(k_pm_compact<uint64_t>, grid_of(items), kBlock, 0, s, g.off, g.n, g.nnz, g.idx,
              (const uint64_t*)g.w, flag, pos, nidx, (uint64_t*)nw, noff);
  else
    LV_LAUNCH(k_pm_compact<uint32_t>, grid_of(items), kBlock, 0, s, g.off, g.n, g.nnz, g.idx,
              (const uint32_t*)g.w, flag, pos, nidx, (uint32_t*)nw, noff);
  LV_LAUNCH(k_pm_arc_bounds, grid_of(P + 1), kBlock, 0, s, noff, vptr, P, aptr);
  return hipGetLastError();
}

hipError_t part_offset_labels(int32_t* lab, int64_t n, const int32_t* gid, const int64_t* loff,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LV_LAUNCH(k_pm_offset_labels, grid_of(n), kBlock, 0, s, lab, n, gid, loff);
  return hipGetLastError();
}

}  // namespace lv
