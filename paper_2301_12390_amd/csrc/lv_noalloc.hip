// louvain_modularity_noalloc: the modularity reduction of louvain_modularity with every
// temporary in a fixed device array of the library instead of the context's workspace, for
// callers that must not allocate device memory during the call.
//
// The array lives in this file as `scratch`. Host code never uses the name as an address: each
// device's copy is looked up once with hipGetSymbolAddress (lv::noalloc_setup, called by
// louvain_ctx_create with the context's device current) and that pointer is what the kernels
// receive. Every call on a device shares the device's array, so calls that overlap on one
// device race; the contents left by one call are not relied on by the next (everything the
// reduction accumulates into is cleared with fill kernels first).
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>

#include "../../include/louvain.h"
#include "lv_internal.h"

typedef unsigned long long ull;
typedef __int128 i128;
typedef unsigned __int128 u128;

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // LV_NOALLOC_SCRATCH_BYTES
static_assert(kScratchBytes == LV_NOALLOC_SCRATCH_BYTES, "header and library disagree");
constexpr int kMaxDevices = 64;
constexpr int64_t kStatWords = 32;  // reduction words at the start of the array

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_lock;
void* g_ptr[kMaxDevices] = {};

// Bytes of the array a graph needs: reduction words, K and Sigma (n words each), the widened
// offsets of an int32 CSR (n + 1 words) and the row-sum tile table.
size_t needed_bytes(const lv_graph* g) {
  size_t words = kStatWords + 2 * (size_t)g->n + (g->offsets_64 ? 0 : (size_t)g->n + 1) +
                 (size_t)lv::row_sum_tiles(g->nnz) + 1;
  return words * sizeof(ull);
}

}  // namespace

namespace lv {

// Looks up this device's copy of the array (the device must be current). Idempotent.
hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> guard(g_lock);
  if (g_ptr[device]) return hipSuccess;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_ptr[device] = p;
  return hipSuccess;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> guard(g_lock);
  return g_ptr[device];
}

}  // namespace lv

extern "C" lv_status louvain_modularity_noalloc(lv_ctx* ctx, const lv_graph* g, const int32_t* C,
                                                lv_i128* q_num, uint64_t* W_out, double* q_out,
                                                void* stream) {
  if (!ctx) return LV_EINVAL;
  const int device = lv::ctx_device(ctx);
  auto fail = [&](lv_status st, const std::string& msg) {
    lv::ctx_set_error(ctx, msg.c_str());
    return st;
  };
  if (hipSetDevice(device) != hipSuccess) return fail(LV_EHIP, "hipSetDevice failed");
  if (!g) return fail(LV_EINVAL, "graph is NULL");
  if (g->n < 0 || g->nnz < 0) return fail(LV_EINVAL, "negative n or nnz");
  if (g->n >= ((int64_t)1 << 31)) return fail(LV_EOVERFLOW, "n must be < 2^31");
  if (!g->offsets_64 && g->nnz >= ((int64_t)1 << 31))
    return fail(LV_EOVERFLOW, "nnz >= 2^31 needs int64 offsets");
  if (!g->offsets) return fail(LV_EINVAL, "offsets is NULL");
  if (g->nnz > 0 && (!g->indices || !g->weights))
    return fail(LV_EINVAL, "indices or weights is NULL");
  if (g->n > 0 && !C) return fail(LV_EINVAL, "C is NULL");
  if (((uintptr_t)g->offsets & (g->offsets_64 ? 7 : 3)) || ((uintptr_t)g->indices & 3) ||
      ((uintptr_t)g->weights & (g->weights_64 ? 7 : 3)))
    return fail(LV_EINVAL, "misaligned graph array");
  const size_t need = needed_bytes(g);
  if (need > kScratchBytes)
    return fail(LV_EBUDGET, "the graph needs " + std::to_string(need) +
                                " bytes of the fixed no-allocation scratch of " +
                                std::to_string(kScratchBytes));
  ull* base = (ull*)lv::noalloc_scratch(device);
  if (!base) return fail(LV_EHIP, "no-allocation scratch not set up on this device");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = g->n;
  ull* stats = base;                         // [0..1] 128-bit weight total, [2] W, [3] max K,
                                             // [4] intra weight, [5..6] sum of Sigma^2
  uint64_t* K = (uint64_t*)(base + kStatWords);
  uint64_t* Sig = K + n;
  int64_t* next = (int64_t*)(Sig + n);
  lv::DevGraph dg;
  dg.n = n;
  dg.nnz = g->nnz;
  dg.idx = g->indices;
  dg.w = g->weights;
  dg.w64 = g->weights_64 != 0;
  if (g->offsets_64) {
    dg.off = (const int64_t*)g->offsets;
  } else {
    if (lv::widen_offsets((const int32_t*)g->offsets, next, n + 1, s) != hipSuccess)
      return fail(LV_EHIP, "offset widening failed");
    dg.off = next;
    next += n + 1;
  }
  dg.rs = dg.off;
  dg.re = dg.off + 1;
  int64_t* rtile = next;
  ull* h = lv::ctx_pinned_words(ctx);  // pinned host words allocated with the context
#define NA_CHK(expr, what)                                     \
  do {                                                         \
    if ((expr) != hipSuccess) return fail(LV_EHIP, what);      \
  } while (0)
  NA_CHK(lv::zero_words(stats, 8, s), "clearing the reduction words failed");
  NA_CHK(lv::fill_u64(K, 0, n, s), "clearing K failed");
  NA_CHK(lv::fill_u64(Sig, 0, n, s), "clearing Sigma failed");
  NA_CHK(lv::total_weight_u128(dg, stats, s), "weight total failed");
  NA_CHK(lv::row_sums(dg, K, rtile, s), "row sums failed");
  NA_CHK(lv::sigma_by_label(K, C, n, Sig, s), "Sigma by label failed");
  NA_CHK(lv::sum_max_u64(K, n, stats + 2, s), "W failed");
  NA_CHK(lv::intra_weight(dg, C, stats + 4, s), "intra-community weight failed");
  NA_CHK(lv::sum_squares_u64(Sig, n, stats + 5, s), "sum of Sigma^2 failed");
  NA_CHK(hipMemcpyAsync(h, stats, 8 * sizeof(ull), hipMemcpyDeviceToHost, s), "read-back failed");
  NA_CHK(hipStreamSynchronize(s), "stream synchronisation failed");
#undef NA_CHK
  const u128 total = ((u128)h[1] << 64) | h[0];
  if (total > ((u128)1 << 62)) return fail(LV_EOVERFLOW, "total weight exceeds 2^62");
  const uint64_t W = h[2];
  const u128 sq = ((u128)h[6] << 64) | h[5];
  const i128 qn = (i128)((u128)W * h[4]) - (i128)sq;
  if (q_num) {
    q_num->lo = (uint64_t)(u128)qn;
    q_num->hi = (int64_t)(uint64_t)((u128)qn >> 64);
  }
  if (W_out) *W_out = W;
  if (q_out) *q_out = W ? (double)qn / ((double)W * (double)W) : 0.0;
  lv::ctx_set_error(ctx, "");
  return LV_OK;
}
