// C ABI of liblouvain: context and workspace management, argument checks, and the drivers of
// the local-moving phase, the aggregation phase and whole runs (section 3.2 of Sahu,
// arXiv 2301.12390). Declarations and the contract are in include/louvain.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/louvain.h"
#include "lv_device.h"
#include "lv_internal.h"

typedef unsigned long long ull;
typedef __int128 i128;
typedef unsigned __int128 u128;

namespace {

enum SlotId {
  S_K, S_SIG, S_CSIZE, S_C, S_MAP, S_MOVERS, S_LIST, S_OFF64, S_STATS, S_COUNTS, S_SCANP,
  S_HUBARR, S_PK, S_PV, S_HOFF, S_NFLUSH, S_PARTIAL, S_A, S_ASTART, S_NEWID, S_CURSOR,
  S_OLDLABEL, S_DCOUNT, S_ABASE, S_TKEY, S_TW, S_GOFF0, S_GIDX0, S_GW0, S_GOFF1, S_GIDX1, S_GW1,
  S_BAD, S_AGGOFF, S_BPART, S_MPART, S_MCOUNT, S_MSTART, S_MEMBERS, S_GSCAN, S_GRE0, S_GRE1,
  S_REC, S_GID0, S_GIDA, S_GIDB, S_GBASE, S_GWORDS, S_GACT, S_APTR, S_PKEY0, S_PKEY1, S_PVAL0,
  S_PVAL1, S_PHIST, S_POFFS, S_PTILE, S_PSLOT, S_PFIRST, S_POFF, S_PGHIST, S_PGBASE, S_PSTATUS,
  S_VCLASS, S_CCNT, S_CFLAG, S_CSHORT, S_CLONG, S_CNLONG, S_PM_VPTR, S_PM_GID, S_PM_FLAG,
  S_PM_POS, S_PM_IDX, S_PM_W, S_PM_OFF, S_PM_APTR, S_PM_LAB, S_PM_LOFF, S_PM_MAP, S_PM_SOFF,
  S_PM_SIDX, S_PM_SW, S_PM_M2, S_GSLICE, S_RTILE, S_GKEEP, S_GTOP, S_CFM, S_LFLAG, S_NOARC,
  S_LIVEB, S_REP0, S_REP1, S_PLANTOT, S_LAB, S_PROBE_T, S_PROBE_O, S_MAP16, S_CMID,
  S_COUNT_SLOTS
};

struct Slot {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

const char* lv::params_error(const lv_params* p) {
  if (!p) return "params is NULL";
  if (p->tolerance_exp10 < 0 || p->decline_exp10 < 0)
    return "tolerance and decline exponents must be >= 0";
  if (p->max_iterations < 1) return "max_iterations must be >= 1";
  if (p->max_passes < 1 || p->max_passes > LV_MAX_PASSES) return "max_passes must be in 1..64";
  if (p->substeps < 1 || p->substeps > 32) return "substeps must be in 1..32";
  return nullptr;
}

// Partition size divisor (as a shift) under LV_SMALL_PARTS.
constexpr int kSmallPartShift = 6;

// Word offsets in the device stats slot and in the pinned host buffer.
constexpr int ST_MISC = 256;      // device: [256, 264) scratch sums, 264 aggregation self-loops
constexpr int PIN_COUNTS = 0;     // host: 1536 words of class counts
constexpr int PIN_STATS = 1544;   // host: per-step iteration stats (8 words per class step)
constexpr int PIN_MISC = 1808;    // host: other read-backs
constexpr int PIN_NOALLOC = 2016; // host: 16 words of louvain_modularity_noalloc read-backs
constexpr int PIN_PLANS = 2048;   // host: 4 totals per list of a batched two-phase plan
constexpr int PIN_WORDS = 2048 + 4 * 32;
constexpr int DEG = 12;           // degree classes per vertex class (list segment stride)
constexpr int STATS_WORDS = 512;
constexpr int kEvStep = 5;  // timing events per class step
constexpr int kEvents = kEvStep * 32 + 2;
constexpr int EV_AGG = kEvStep * 32;

struct lv_ctx {
  int device = 0;
  uint64_t budget = 0;
  uint64_t held = 0;
  Slot slots[S_COUNT_SLOTS];
  std::string err;
  size_t max_lds = 65536;  // largest LDS allocation of one workgroup on this device
  int part_shift = 0;      // LV_SMALL_PARTS of the current call
  void* bpin = nullptr;    // pinned host words of batched runs (grow-only)
  size_t bpin_bytes = 0;
  ull* pinned = nullptr;  // host-pinned words for small read-backs
  hipEvent_t ev[kEvents] = {};  // kEvStep per class step, then 2 for aggregation
  bool step_par[32] = {};       // class step k forked its tiers onto the side streams
  // the move tiers of a class step run concurrently: the workgroup tier on side[0], the hub
  // path on side[1], forked from and joined back into the caller's stream
  hipStream_t side[2] = {};
  hipEvent_t fork[32] = {}, join0[32] = {}, join1[32] = {};
  // small phases replay an iteration as a HIP graph on `cap`, after gin and before gout
  hipStream_t cap = nullptr;
  hipEvent_t gin = nullptr, gout = nullptr;
};

int lv::ctx_device(const lv_ctx* ctx) { return ctx->device; }
void lv::ctx_set_error(lv_ctx* ctx, const char* msg) { ctx->err = msg; }
unsigned long long* lv::ctx_pinned_words(lv_ctx* ctx) { return ctx->pinned + PIN_NOALLOC; }

namespace {

lv_status fail(lv_ctx* ctx, lv_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return st;
}

lv_status fail_hip(lv_ctx* ctx, const char* what, hipError_t e) {
  return fail(ctx, LV_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr)                                   \
  do {                                                 \
    hipError_t _e = (expr);                            \
    if (_e != hipSuccess) return fail_hip(ctx, #expr, _e); \
  } while (0)

#define CHK(expr)                  \
  do {                             \
    lv_status _s = (expr);         \
    if (_s != LV_OK) return _s;    \
  } while (0)

// Grow-only workspace slot; contents are not preserved when it grows.
lv_status ws(lv_ctx* ctx, int id, size_t bytes, void** out) {
  Slot& s = ctx->slots[id];
  if (bytes == 0) bytes = 8;
  if (s.bytes >= bytes) {
    *out = s.p;
    return LV_OK;
  }
  size_t want = bytes + bytes / 8;  // headroom against repeated small growth
  want = (want + 4095) & ~(size_t)4095;
  const uint64_t after = ctx->held - s.bytes + want;
  if (ctx->budget && after > ctx->budget) {
    want = (bytes + 4095) & ~(size_t)4095;
    if (ctx->held - s.bytes + want > ctx->budget)
      return fail(ctx, LV_EBUDGET, "workspace of " + std::to_string(ctx->held - s.bytes + want) +
                                       " bytes exceeds the HBM budget of " +
                                       std::to_string(ctx->budget));
  }
  if (s.p) {
    hipError_t e = hipFree(s.p);
    s.p = nullptr;
    ctx->held -= s.bytes;
    s.bytes = 0;
    if (e != hipSuccess) return fail_hip(ctx, "hipFree", e);
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, LV_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
  }
  s.p = p;
  s.bytes = want;
  ctx->held += want;
  *out = p;
  return LV_OK;
}

template <typename T>
lv_status wst(lv_ctx* ctx, int id, int64_t count, T** out) {
  void* p = nullptr;
  lv_status st = ws(ctx, id, (size_t)(count > 0 ? count : 1) * sizeof(T), &p);
  *out = (T*)p;
  return st;
}

lv_i128 to_i128(i128 v) {
  lv_i128 r;
  r.lo = (uint64_t)(u128)v;
  r.hi = (int64_t)(uint64_t)((u128)v >> 64);
  return r;
}

double q_of(i128 qnum, uint64_t W) {
  if (W == 0) return 0.0;
  return (double)qnum / ((double)W * (double)W);
}

// floor(W^2 / (2 * 10^(a + b*p))): S > T exactly when 2S/W^2 exceeds the pass tolerance.
u128 tolerance_threshold(uint64_t W, int a, int b, int p) {
  const u128 W2 = (u128)W * W;
  const int64_t ex = (int64_t)a + (int64_t)b * p;
  u128 div = 2;
  for (int64_t k = 0; k < ex; k++) {
    if (div > W2 / 10) return 0;
    div *= 10;
  }
  return W2 / div;
}

constexpr int lv_max_classes() { return 32; }

lv_status check_params(lv_ctx* ctx, const lv_params* p) {
  const char* e = lv::params_error(p);
  return e ? fail(ctx, LV_EINVAL, e) : LV_OK;
}

// Checks the graph descriptor and produces a device view with int64 offsets.
lv_status import_graph(lv_ctx* ctx, const lv_graph* g, bool validate, hipStream_t s,
                       lv::DevGraph* out) {
  if (!g) return fail(ctx, LV_EINVAL, "graph is NULL");
  if (g->n < 0 || g->nnz < 0) return fail(ctx, LV_EINVAL, "negative n or nnz");
  if (g->n >= ((int64_t)1 << 31)) return fail(ctx, LV_EOVERFLOW, "n must be < 2^31");
  if (!g->offsets_64 && g->nnz >= ((int64_t)1 << 31))
    return fail(ctx, LV_EOVERFLOW, "nnz >= 2^31 needs int64 offsets");
  if (!g->offsets) return fail(ctx, LV_EINVAL, "offsets is NULL");
  if (g->nnz > 0 && (!g->indices || !g->weights))
    return fail(ctx, LV_EINVAL, "indices or weights is NULL");
  if (((uintptr_t)g->offsets & (g->offsets_64 ? 7 : 3)) || ((uintptr_t)g->indices & 3) ||
      ((uintptr_t)g->weights & (g->weights_64 ? 7 : 3)))
    return fail(ctx, LV_EINVAL, "misaligned graph array");
  out->n = g->n;
  out->nnz = g->nnz;
  out->idx = g->indices;
  out->w = g->weights;
  out->w64 = g->weights_64 != 0;
  if (g->offsets_64) {
    out->off = (const int64_t*)g->offsets;
  } else {
    int64_t* o = nullptr;
    CHK(wst(ctx, S_OFF64, g->n + 1, &o));
    HIPCHK(lv::widen_offsets((const int32_t*)g->offsets, o, g->n + 1, s));
    out->off = o;
  }
  out->rs = out->off;
  out->re = out->off + 1;
  if (validate) {
    unsigned int* bad = nullptr;
    CHK(wst(ctx, S_BAD, 1, &bad));
    HIPCHK(hipMemsetAsync(bad, 0, sizeof(unsigned int), s));
    HIPCHK(lv::validate_graph(*out, bad, s));
    int64_t ends[2];
    unsigned int hb = 0;
    HIPCHK(hipMemcpyAsync(&ends[0], out->off, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&ends[1], out->off + g->n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&hb, bad, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (ends[0] != 0 || ends[1] != g->nnz)
      return fail(ctx, LV_EINVAL, "offsets[0] must be 0 and offsets[n] must be nnz");
    if (hb & 1u) return fail(ctx, LV_EINVAL, "offsets decrease");
    if (hb & 2u) return fail(ctx, LV_EINVAL, "an index is out of range");
    if (hb & 4u) return fail(ctx, LV_EINVAL, "a weight is zero");
  }
  return LV_OK;
}

// W and max K from row sums already in K (n entries).
lv_status weight_stats(lv_ctx* ctx, const uint64_t* K, int64_t n, hipStream_t s, uint64_t* W,
                       uint64_t* maxK) {
  ull* st = nullptr;
  CHK(wst(ctx, S_STATS, STATS_WORDS, &st));
  HIPCHK(lv::zero_words(st + ST_MISC, 2, s));
  HIPCHK(lv::sum_max_u64(K, n, st + ST_MISC, s));
  HIPCHK(hipMemcpyAsync(ctx->pinned + PIN_MISC, st + ST_MISC, 2 * sizeof(ull),
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *W = ctx->pinned[PIN_MISC];
  *maxK = ctx->pinned[PIN_MISC + 1];
  return LV_OK;
}

// The exact (128-bit) total of g's arc weights. Row sums and W are 64-bit words; they are exact
// whenever this total is below 2^64. Skipped (*total = 0) when uint32 weights on at most 2^30
// arcs bound it below 2^62 anyway.
lv_status total_weight(lv_ctx* ctx, const lv::DevGraph& g, hipStream_t s, u128* total) {
  *total = 0;
  if (g.nnz <= 0 || (!g.w64 && g.nnz <= ((int64_t)1 << 30))) return LV_OK;
  ull* st = nullptr;
  CHK(wst(ctx, S_STATS, STATS_WORDS, &st));
  HIPCHK(lv::zero_words(st + ST_MISC, 2, s));
  HIPCHK(lv::total_weight_u128(g, st + ST_MISC, s));
  HIPCHK(hipMemcpyAsync(ctx->pinned + PIN_MISC, st + ST_MISC, 2 * sizeof(ull),
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *total = ((u128)ctx->pinned[PIN_MISC + 1] << 64) | ctx->pinned[PIN_MISC];
  return LV_OK;
}

// LV_EOVERFLOW unless the total weight of g is at most 2^62 (C21: every gain, Sigma product and
// iteration sum then fits 128 bits, and no 64-bit row sum or W can have wrapped).
lv_status check_total_weight(lv_ctx* ctx, const lv::DevGraph& g, hipStream_t s) {
  u128 t = 0;
  CHK(total_weight(ctx, g, s, &t));
  if (t > ((u128)1 << 62)) return fail(ctx, LV_EOVERFLOW, "total weight exceeds 2^62");
  return LV_OK;
}

// ---------------------------------------------------------------------------------------------
// Local-moving phase on the state in m (C, Sig, csize by label).

struct Phase {
  lv::DevGraph g;
  lv::Buckets b;
  lv::PartPlan hp[32];  // per vertex class: two-phase plan of its hub rows
  lv::MoveBuffers m;
  bool wide = false;
  int classes = 1;
  int pass = 0;
  bool colour = false;            // colour classes (LV_COLOR_CLASSES) instead of hashed ones
  const uint8_t* vclass = nullptr;  // the colour classes, once computed for this phase
  int colour_rounds = 0;
};

// Colour classes of the phase's graph and pass (computed once per phase).
lv_status colour_phase(lv_ctx* ctx, Phase& ph, hipStream_t s) {
  const int64_t n = ph.g.n;
  uint8_t* vc = nullptr;
  lv::ColourBuffers cb;
  CHK(wst(ctx, S_VCLASS, n, &vc));
  CHK(wst(ctx, S_CCNT, 2 * n, &cb.slot));
  CHK(wst(ctx, S_CFLAG, 2 * n, &cb.all_long));
  CHK(wst(ctx, S_CSHORT, 2 * n, &cb.shorts));
  CHK(wst(ctx, S_CMID, 2 * n, &cb.mids));
  CHK(wst(ctx, S_CLONG, 2 * n, &cb.longs));
  CHK(wst(ctx, S_CNLONG, 11, &cb.counts));
  HIPCHK(lv::colour_classes(ph.g, ph.classes, ph.pass, ph.m.gs.gid, ph.m.gs.gbase, cb,
                            ctx->pinned + PIN_MISC, vc, &ph.colour_rounds, ctx->part_shift != 0,
                            s));
  ph.vclass = vc;
  return LV_OK;
}

// Row lists by (vertex class, degree class) and the hub tables of every class; fills ph.b,
// ph.hp and the buffers of ph.m that depend on them.
lv_status plan_phase(lv_ctx* ctx, Phase& ph, hipStream_t s) {
  const int64_t n = ph.g.n;
  const int K = ph.classes;
  int32_t* list = nullptr;
  ull* counts = nullptr;
  int64_t* hubarr = nullptr;
  CHK(wst(ctx, S_LIST, n, &list));
  CHK(wst(ctx, S_COUNTS, 1536, &counts));
  if (ph.colour && K > 1 && !ph.vclass) CHK(colour_phase(ctx, ph, s));
  HIPCHK(lv::bucket_rows(ph.g.rs, ph.g.re, nullptr, n, K, ph.pass, ph.m.gs.gid, ph.m.gs.gbase,
                         ph.m.gs.act, K > 1 ? ph.vclass : nullptr, list, counts,
                         ctx->pinned + PIN_COUNTS, ph.b, s));
  const int hf = lv::hub_first_class(ctx->max_lds, ph.wide);
  ph.m.hub_first = hf;
  auto hub_rows = [&](int k) {
    return ph.b.lstart[DEG * k + DEG] - ph.b.lstart[DEG * k + hf];
  };
  int64_t nh_total = 0;
  for (int k = 0; k < K; k++) nh_total += hub_rows(k);
  CHK(wst(ctx, S_HUBARR, lv::kPlanWords * (nh_total + K), &hubarr));
  // the pair, bound and partial buffers are shared by the class steps: sized for the largest
  const int vb = ph.wide ? 8 : 4;
  int64_t max_chunks = 0, max_walkers = 0, max_parts = 0, max_hoff = 0, off = 0;
  const int32_t* items[32];
  int64_t nhs[32];
  int64_t* arrs[32];
  for (int k = 0; k < K; k++) {
    items[k] = list + ph.b.lstart[DEG * k + hf];
    nhs[k] = hub_rows(k);
    arrs[k] = hubarr + off;
    off += lv::kPlanWords * (nhs[k] + 1);
  }
  if (nh_total > 0) {  // every class's plan in one launch and one read-back
    int64_t* tot = nullptr;
    CHK(wst(ctx, S_PLANTOT, 4 * 32, &tot));
    HIPCHK(lv::plan_parts_batch(ph.g.rs, ph.g.re, nullptr, items, nhs, K, n, vb, false,
                                ctx->part_shift, arrs, tot, ctx->pinned + PIN_PLANS, ph.hp, s));
  } else {
    for (int k = 0; k < K; k++) ph.hp[k] = lv::PartPlan();
  }
  for (int k = 0; k < K; k++) {
    max_chunks = std::max(max_chunks, ph.hp[k].chunks);
    max_walkers = std::max(max_walkers, ph.hp[k].blocks);
    max_parts = std::max(max_parts, ph.hp[k].parts);
    max_hoff = std::max(max_hoff, ph.hp[k].hoff_entries);
  }
  ph.m.list = list;
  if (max_chunks > 0) {
    const int64_t pairs = max_chunks * lv::part_chunk(vb);
    CHK(wst(ctx, S_PK, pairs, &ph.m.pk));
    uint8_t* pv = nullptr;
    CHK(wst(ctx, S_PV, pairs * vb, &pv));
    ph.m.pv = pv;
    CHK(wst(ctx, S_HOFF, max_hoff, &ph.m.hoff));
    CHK(wst(ctx, S_NFLUSH, max_walkers, &ph.m.nflush));
    CHK(wst(ctx, S_PARTIAL, 5 * max_parts, &ph.m.partial));
  }
  CHK(wst(ctx, S_MOVERS, n, &ph.m.tgt));
  int64_t max_blocks = 1;
  for (int k = 0; k < K; k++)
    max_blocks = std::max(max_blocks, lv::move_lds_blocks(ph.b, k, hf));
  CHK(wst(ctx, S_BPART, 4 * max_blocks, &ph.m.block_partial));
  ull* st = nullptr;
  CHK(wst(ctx, S_STATS, STATS_WORDS, &st));
  ph.m.stats = st;
  return LV_OK;
}

// Per-graph iteration state of a batch (host side; device arrays in the phase's GraphSet).
struct BatchPhase {
  int64_t G = 0;
  std::vector<u128> T;         // tolerance threshold of every graph for this pass
  std::vector<uint8_t> act;    // graphs still iterating
  std::vector<i128> passgain;  // gain sum over the pass
  std::vector<int32_t> iters;  // iterations this pass
  std::vector<uint8_t> capped; // stopped at max_iterations
  ull* hS = nullptr;           // pinned: 2G words of per-graph gain sums
  uint8_t* hact = nullptr;     // pinned: G activity flags
  std::vector<int64_t> size;   // vertices of every graph at this level
  int64_t listed = 0;          // vertices of the graphs in the current lists
};

struct PhaseOut {
  int32_t iterations = 0;
  bool hit_cap = false;
  i128 gain_sum = 0;
  int64_t moved = 0;
  i128 last_gain = 0;
  int64_t last_moved = 0;
  int64_t last_candidates = 0;
};

// One local-moving iteration's kernels, its K synchronous class steps, enqueued on stream s
// (which may be capturing): clears the step statistics (and the batch's gain sums), then per
// class step the three move tiers, the record reduction and the community update.
lv_status issue_iteration(lv_ctx* ctx, Phase& ph, bool trace, hipStream_t s, BatchPhase* bp) {
  const int K = ph.classes;
  const int hf = ph.m.hub_first;
  ull* stats0 = ph.m.stats;
  HIPCHK(lv::zero_words(stats0, 8 * K, s));
  if (bp) HIPCHK(lv::zero_words(ph.m.gs.gS, 2 * (int64_t)lv::kGainSlices * bp->G, s));
  for (int k = 0; k < K; k++) {
    lv::MoveBuffers m = ph.m;
    m.stats = stats0 + 8 * k;
    hipEvent_t* ev = ctx->ev + kEvStep * k;
    // the three tiers decide disjoint vertices from the same state: when at least two of them
    // have real work they run concurrently, forked onto the side streams and joined back
    int64_t ta = 0, tb = 0, tc = 0;
    for (int j = 0; j < DEG; j++) {
      const int64_t arcs = ph.b.arcs[DEG * k + j];
      if (j < 7) ta += arcs;
      else if (j < hf) tb += arcs;
      else tc += arcs;
    }
    const int64_t kBig = (int64_t)1 << 20;
    const bool par = (ta >= kBig) + (tb >= kBig) + (tc >= kBig) >= 2;
    hipStream_t s1 = par ? ctx->side[0] : s, s2 = par ? ctx->side[1] : s;
    if (par) {
      HIPCHK(hipEventRecord(ctx->fork[k], s));
      HIPCHK(hipStreamWaitEvent(s1, ctx->fork[k], 0));
      HIPCHK(hipStreamWaitEvent(s2, ctx->fork[k], 0));
    }
    // timing (trace): one event after each tier on its own stream and one after the update,
    // which is also the next class step's start (class step 0 records its own); a tier starts
    // at the fork when the tiers are concurrent, else where the one before it ended. Few
    // events: each is a marker on its queue, a bubble before the next kernel, and five per
    // class step cost an s25 run ~2 ms of ~200.
    if (trace && k == 0) HIPCHK(hipEventRecord(ev[0], s));
    HIPCHK(lv::move_fused(ph.g, ph.b, k, m, ph.wide, s));
    if (trace) HIPCHK(hipEventRecord(ev[1], s));
    HIPCHK(lv::move_wg(ph.g, ph.b, k, m, ph.wide, s1));
    if (trace) HIPCHK(hipEventRecord(ev[2], s1));
    HIPCHK(lv::move_hubs(ph.g, ph.b, k, ph.hp[k], m, ph.wide, s2));
    if (trace) HIPCHK(hipEventRecord(ev[3], s2));
    if (par) {
      HIPCHK(hipEventRecord(ctx->join0[k], s1));
      HIPCHK(hipEventRecord(ctx->join1[k], s2));
      HIPCHK(hipStreamWaitEvent(s, ctx->join0[k], 0));
      HIPCHK(hipStreamWaitEvent(s, ctx->join1[k], 0));
    }
    HIPCHK(lv::apply_moves(ph.b, k, m, s));  // also sums the step's decision records
    if (trace) HIPCHK(hipEventRecord(ev[4], s));
    ctx->step_par[k] = par;
  }
  return LV_OK;
}

// An instantiated graph of one iteration, destroyed when it goes out of scope or is replaced.
struct IterGraph {
  hipGraphExec_t exec = nullptr;
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
  }
  ~IterGraph() { reset(); }
};

// Captures issue_iteration on the context's capture stream into g->exec. The kernels' arguments
// are fixed for the phase (row lists, plans and buffers), and everything that changes between
// iterations lives in device memory, so one capture serves every iteration of the phase until
// the rows are listed again.
lv_status capture_iteration(lv_ctx* ctx, Phase& ph, BatchPhase* bp, IterGraph* g) {
  g->reset();
  // the capture stream and its events are made on first use only: every stream a context
  // creates takes its turn among the process's hardware queues, and contexts that never replay
  // (the default) keep the streams they had without it
  if (!ctx->cap) {
    HIPCHK(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&ctx->gin, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ctx->gout, hipEventDisableTiming));
  }
  HIPCHK(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
  const lv_status st = issue_iteration(ctx, ph, false, ctx->cap, bp);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(ctx->cap, &graph);
  if (st != LV_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return fail_hip(ctx, "hipStreamEndCapture", e);
  const hipError_t ei = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    g->exec = nullptr;
    return fail_hip(ctx, "hipGraphInstantiate", ei);
  }
  return LV_OK;
}

// Local-moving iterations; each is `classes` synchronous class steps. With LV_GRAPH_REPLAY a
// phase on at most kGraphArcs arcs runs its first iteration directly and replays the later ones
// as a captured HIP graph on the capture stream, ordered after and before the caller's stream
// by events (not under LV_TRACE); otherwise every kernel is launched directly.
constexpr int64_t kGraphArcs = (int64_t)1 << 24;

lv_status run_phase(lv_ctx* ctx, Phase& ph, u128 T, int max_it, uint32_t flags, hipStream_t s,
                    lv_result* res, PhaseOut* out, BatchPhase* bp = nullptr) {
  const bool trace = (flags & LV_TRACE) != 0;
  const bool use_graph = !trace && (flags & LV_GRAPH_REPLAY) && ph.g.nnz <= kGraphArcs;
  const int K = ph.classes;
  const int hf = ph.m.hub_first;
  // the work of each kernel family per iteration (fixed within the phase)
  int64_t fv = 0, fa = 0, wv = 0, wa = 0, hv = 0, ha = 0;
  int fl = 0, wl = 0, hl = 0;
  for (int k = 0; k < K; k++) {
    int64_t rows = 0;
    for (int j = 0; j < DEG; j++) {
      const int64_t c = ph.b.count[DEG * k + j], a = ph.b.arcs[DEG * k + j];
      if (j < 7) {
        fv += c;
        fa += a;
        rows += c;
      } else if (j < hf) {
        wv += c;
        wa += a;
        wl += c > 0;
      } else {
        hv += c;
        ha += a;
      }
    }
    fl += rows > 0;
    hl += ph.hp[k].nh > 0;
  }
  ull* stats0 = ph.m.stats;
  *out = PhaseOut();
  out->hit_cap = true;
  IterGraph graph;
  for (int it = 0; it < max_it; it++) {
    auto t0 = std::chrono::steady_clock::now();
    if (use_graph && it > 0) {
      if (!graph.exec) CHK(capture_iteration(ctx, ph, bp, &graph));
      HIPCHK(hipEventRecord(ctx->gin, s));
      HIPCHK(hipStreamWaitEvent(ctx->cap, ctx->gin, 0));
      HIPCHK(hipGraphLaunch(graph.exec, ctx->cap));
      HIPCHK(hipEventRecord(ctx->gout, ctx->cap));
      HIPCHK(hipStreamWaitEvent(s, ctx->gout, 0));
    } else {
      CHK(issue_iteration(ctx, ph, trace, s, bp));
    }
    ull* h = ctx->pinned + PIN_STATS;
    HIPCHK(hipMemcpyAsync(h, stats0, 8 * K * sizeof(ull), hipMemcpyDeviceToHost, s));
    if (bp) {
      HIPCHK(lv::fold_gain_slices(ph.m.gs.gS, bp->G, s));
      HIPCHK(hipMemcpyAsync(bp->hS, ph.m.gs.gS, 2 * bp->G * sizeof(ull), hipMemcpyDeviceToHost,
                            s));
    }
    HIPCHK(hipStreamSynchronize(s));
    float t_fused = 0, t_wg = 0, t_hub = 0, t_upd = 0;
    if (trace) {
      for (int k = 0; k < K; k++) {
        hipEvent_t* ev = ctx->ev + kEvStep * k;
        hipEvent_t start = k == 0 ? ev[0] : ctx->ev[kEvStep * (k - 1) + 4];
        float f = 0, w = 0, h = 0, e = 0;  // ends of the tiers and of the step, from the start
        HIPCHK(hipEventElapsedTime(&f, start, ev[1]));
        HIPCHK(hipEventElapsedTime(&w, start, ev[2]));
        HIPCHK(hipEventElapsedTime(&h, start, ev[3]));
        HIPCHK(hipEventElapsedTime(&e, start, ev[4]));
        if (ctx->step_par[k]) {  // concurrent: all three start at the fork
          t_fused += f;
          t_wg += w;
          t_hub += h;
          t_upd += e - std::max(f, std::max(w, h));
        } else {                 // one stream: fused, wg, hub, update in turn
          t_fused += f;
          t_wg += w - f;
          t_hub += h - w;
          t_upd += e - h;
        }
      }
    }
    i128 S = 0;
    int64_t moved = 0, cand = 0, fcand = 0, wcand = 0;
    for (int k = 0; k < K; k++) {
      const ull* x = h + 8 * k;
      S += (i128)(((u128)x[1] << 64) | x[0]);
      moved += (int64_t)x[2];
      cand += (int64_t)x[3];
      fcand += (int64_t)x[4];
      wcand += (int64_t)x[5];
    }
    out->iterations++;
    out->gain_sum += S;
    out->moved += moved;
    out->last_gain = S;
    out->last_moved = moved;
    out->last_candidates = cand;
    if (res && res->n_trace < LV_MAX_TRACE) {
      lv_iter_trace& r = res->trace[res->n_trace++];
      memset(&r, 0, sizeof(r));
      r.pass = ph.pass;
      r.iteration = it;
      r.wide = ph.wide ? 1 : 0;
      r.substeps = K;
      r.fused_launches = fl;
      r.wg_launches = wl;
      r.hub_launches = hl;
      r.gain_sum = to_i128(S);
      r.moved = moved;
      r.candidates = cand;
      r.fused_vertices = fv;
      r.fused_arcs = fa;
      r.fused_candidates = fcand;
      r.wg_vertices = wv;
      r.wg_arcs = wa;
      r.wg_candidates = wcand;
      r.hub_vertices = hv;
      r.hub_arcs = ha;
      if (trace) {
        r.fused_ms = t_fused;
        r.wg_ms = t_wg;
        r.hub_ms = t_hub;
        r.update_ms = t_upd;
        r.iter_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0)
                        .count();
      }
    }
    if (bp) {
      // per graph: the same rule on its own S and threshold; the phase ends when none iterates
      bool any = false;
      for (int64_t g = 0; g < bp->G; g++) {
        if (!bp->act[g]) continue;
        const i128 Sg = (i128)(((u128)bp->hS[2 * g + 1] << 64) | bp->hS[2 * g]);
        bp->passgain[g] += Sg;
        bp->iters[g]++;
        if (!((u128)Sg > bp->T[g])) bp->act[g] = 0;
        else if (it + 1 == max_it) bp->capped[g] = 1, bp->act[g] = 0;
        any = any || bp->act[g];
      }
      if (!any) {
        out->hit_cap = false;
        break;
      }
      memcpy(bp->hact, bp->act.data(), (size_t)bp->G);
      HIPCHK(hipMemcpyAsync((void*)ph.m.gs.act, bp->hact, (size_t)bp->G, hipMemcpyHostToDevice,
                            s));
      // once a quarter of the listed vertices belong to graphs that stopped, list only the
      // others again (their rows cost a class step's kernels even with no arcs to read)
      int64_t live = 0;
      for (int64_t g = 0; g < bp->G; g++)
        if (bp->act[g]) live += bp->size[g];
      if (4 * live < 3 * bp->listed) {
        CHK(plan_phase(ctx, ph, s));
        bp->listed = live;
        graph.reset();
      }
      continue;
    }
    if (!((u128)S > T)) {  // the iteration's modularity change is within the tolerance
      out->hit_cap = false;
      break;
    }
  }
  return LV_OK;
}

// ---------------------------------------------------------------------------------------------
// Aggregation of graph g under labels C (csize by label; Sig by label or NULL). Merged rows go
// to okey/ow (g.nnz entries) at their community's flat position. Outputs: map[n], Kp[n'] (if
// Sig), the buffers describing the rows (*out), n', nnz' and the weight of the self super-arcs.
// With allow_w32 and Sig, the super-arc weights are written as uint32 when every Sigma is below
// 2^32 (out->w32 tells which). With live_only, only communities with arcs get new ids (map -1
// for the others; see the live numbering in lv_kernels.hip).
lv_status aggregate(lv_ctx* ctx, const lv::DevGraph& g, const int32_t* C, const int32_t* csize,
                    const uint64_t* Sig, int32_t* map, int32_t* okey, uint64_t* ow, uint64_t* Kp,
                    lv::AggBuffers* out, int64_t* n_out, int64_t* nnz_out, uint64_t* self_out,
                    hipStream_t s, bool allow_w32 = false, bool live_only = false) {
  const int64_t n = g.n;
  lv::AggBuffers a;
  a.gs = out->gs;  // batches: graph of every label and per-graph self super-arc weights
  CHK(wst(ctx, S_NEWID, n + 1, &a.newid));
  CHK(wst(ctx, S_MCOUNT, n, &a.mcount));
  CHK(wst(ctx, S_MSTART, n + 1, &a.mstart));
  CHK(wst(ctx, S_ASTART, n, &a.astart));
  CHK(wst(ctx, S_A, n, &a.A));
  CHK(wst(ctx, S_OLDLABEL, n, &a.oldlabel));
  CHK(wst(ctx, S_DCOUNT, n + 1, &a.dcount));
  CHK(wst(ctx, S_MEMBERS, n, &a.members));
  CHK(wst(ctx, S_GSCAN, n + 1, &a.gscan));
  CHK(wst(ctx, S_LIST, n, &a.list));
  CHK(wst(ctx, S_SCANP, lv::scan_partial_elems(n + 1) + 1, &a.partial));
  CHK(wst(ctx, S_COUNTS, 1536, &a.counts));
  ull* st = nullptr;
  CHK(wst(ctx, S_STATS, STATS_WORDS, &st));
  a.map = map;
  a.okey = okey;
  a.ow = ow;
  a.stats = st + ST_MISC + 8;
  HIPCHK(lv::zero_words(a.stats, 2, s));
  HIPCHK(lv::aggregate_prepare(g, C, csize, Sig, Kp, map, a, live_only, s));
  lv::Buckets b;
  HIPCHK(lv::bucket_rows(nullptr, nullptr, a.A, n, 1, 0, nullptr, nullptr, nullptr, nullptr,
                         a.list,
                         a.counts,
                         ctx->pinned + PIN_COUNTS, b, s));
  // the super-vertex count bounds the distinct targets of any community
  ull* hm = ctx->pinned + PIN_MISC;
  ull* sm = st + ST_MISC + 12;  // sum and max of Sigma
  const bool check32 = allow_w32 && Sig;
  if (check32) {
    HIPCHK(lv::zero_words(sm, 2, s));
    HIPCHK(lv::sum_max_u64(Sig, n, sm, s));
    HIPCHK(hipMemcpyAsync(hm + 1, sm, 2 * sizeof(ull), hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipMemcpyAsync(hm, a.newid + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int64_t np = (int64_t)hm[0];
  a.w32 = check32 && hm[2] < ((ull)1 << 32);
  // few super-vertices: the merges gather new ids from a 16-bit copy of the map (also taken
  // under LV_SMALL_PARTS, so that small test graphs use it)
  if (np < (int64_t)0xFFFF && (n >= ((int64_t)1 << 20) || ctx->part_shift != 0)) {
    CHK(wst(ctx, S_MAP16, n, &a.map16));
    HIPCHK(lv::narrow_map(map, n, a.map16, s));
  }
  HIPCHK(lv::fill_i64(a.dcount, 0, np + 1, s));
  CHK(wst(ctx, S_MPART, lv::merge_lds_blocks(b), &a.block_partial));
  // Communities of up to 1024 arcs: the LDS merge; classes 7 .. pf - 1: one workgroup each
  // (merge_mid); longer ones: the two-phase merge.
  const int pf = lv::merge_part_first_class(ctx->max_lds, a.w32);
  const int64_t nh = b.lstart[DEG] - b.lstart[pf];
  // The three write disjoint rows and counts and add to the self-arc sum atomically. When the
  // two-phase merge and the others both have real work, the others run on a side stream,
  // overlapping its planning and kernels.
  int64_t small_arcs = 0;
  for (int j = 0; j < pf; j++) small_arcs += b.arcs[j];
  const bool fork = nh > 0 && small_arcs >= ((int64_t)1 << 20);
  hipStream_t s_lds = fork ? ctx->side[0] : s;
  if (fork) {
    HIPCHK(hipEventRecord(ctx->fork[0], s));
    HIPCHK(hipStreamWaitEvent(s_lds, ctx->fork[0], 0));
  }
  HIPCHK(lv::merge_lds(g, b, a, s_lds));
  HIPCHK(lv::merge_mid(g, b, a, pf, s_lds));
  if (nh > 0) {
    lv::PartPlan pp;
    CHK(wst(ctx, S_HUBARR, lv::kPlanWords * (nh + 1), &a.hub_arrays));
    // pair values of the weight width the super-vertex graph gets (both bound by Sigma)
    const int vb = a.w32 ? 4 : 8;
    int64_t* tot = nullptr;
    CHK(wst(ctx, S_PLANTOT, 4 * 32, &tot));
    const int32_t* items = a.list + b.lstart[pf];
    int64_t* arrs = a.hub_arrays;
    HIPCHK(lv::plan_parts_batch(nullptr, nullptr, a.A, &items, &nh, 1, np, vb, true,
                                ctx->part_shift, &arrs, tot, ctx->pinned + PIN_PLANS, &pp, s));
    const int64_t pairs = pp.chunks * lv::part_chunk(vb);
    CHK(wst(ctx, S_PK, pairs, &a.pk));
    CHK(ws(ctx, S_PV, (size_t)pairs * vb, &a.pv));
    CHK(wst(ctx, S_HOFF, pp.hoff_entries, &a.hoff));
    CHK(wst(ctx, S_NFLUSH, pp.blocks, &a.nflush));
    CHK(wst(ctx, S_CFM, pp.chunks, &a.cfm));
    HIPCHK(lv::merge_hubs(g, b, pp, a, pf, s));
  }
  if (fork) {
    HIPCHK(hipEventRecord(ctx->join0[0], s_lds));
    HIPCHK(hipStreamWaitEvent(s, ctx->join0[0], 0));
  }
  HIPCHK(lv::sum_i64(a.dcount, np, a.stats + 1, s));
  HIPCHK(hipMemcpyAsync(hm, a.stats, 2 * sizeof(ull), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *n_out = np;
  *nnz_out = (int64_t)hm[1];
  if (self_out) *self_out = hm[0];
  *out = a;
  return LV_OK;
}

// Qnum of singletons on g: W * (self-loop weight) - sum K^2, from the per-row self-loop
// weights selfw that row_sums wrote.
lv_status singleton_qnum(lv_ctx* ctx, const lv::DevGraph& g, const uint64_t* K,
                         const uint64_t* selfw, uint64_t W, hipStream_t s, i128* q) {
  ull* st = nullptr;
  CHK(wst(ctx, S_STATS, STATS_WORDS, &st));
  ull* d = st + ST_MISC;
  ull* h = ctx->pinned + PIN_MISC;
  HIPCHK(lv::zero_words(d, 4, s));
  HIPCHK(lv::sum_squares_u64(K, g.n, d, s));       // d[0..1]
  HIPCHK(lv::sum_max_u64(selfw, g.n, d + 2, s));   // d[2] (d[3]: max, unused)
  HIPCHK(hipMemcpyAsync(h, d, 4 * sizeof(ull), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const u128 sq = ((u128)h[1] << 64) | h[0];
  *q = (i128)((u128)W * h[2]) - (i128)sq;
  return LV_OK;
}

// Pinned host memory of at least `bytes` for batched runs (grow-only, freed with the context).
lv_status batch_pinned(lv_ctx* ctx, size_t bytes, void** out) {
  if (ctx->bpin_bytes < bytes) {
    if (ctx->bpin) (void)hipHostFree(ctx->bpin);
    ctx->bpin = nullptr;
    ctx->bpin_bytes = 0;
    hipError_t e = hipHostMalloc(&ctx->bpin, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
      ctx->bpin = nullptr;
      return fail_hip(ctx, "hipHostMalloc", e);
    }
    ctx->bpin_bytes = bytes;
  }
  *out = ctx->bpin;
  return LV_OK;
}

}  // namespace

// =============================================================================================
// C ABI

extern "C" {

lv_status louvain_ctx_create(int device, uint64_t hbm_budget_bytes, lv_ctx** out) {
  if (!out) return LV_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return LV_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return LV_EHIP;
  lv_ctx* ctx = new lv_ctx();
  ctx->device = device;
  ctx->budget = hbm_budget_bytes;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
          hipSuccess && lds > 0)
    ctx->max_lds = (size_t)lds;
  // the two-phase kernels take part_lds_bytes(4) of dynamic LDS plus their own shared arrays
  if (ctx->max_lds < lv::part_lds_bytes(4) + 4096) {
    delete ctx;
    return LV_EHIP;
  }
  if (hipHostMalloc((void**)&ctx->pinned, PIN_WORDS * sizeof(ull), hipHostMallocDefault) != hipSuccess) {
    delete ctx;
    return LV_EHIP;
  }
  memset(ctx->pinned, 0, PIN_WORDS * sizeof(ull));
  // this device's copy of louvain_modularity_noalloc's fixed array (looked up once per device)
  if (lv::noalloc_setup(device) != hipSuccess) {
    louvain_ctx_destroy(ctx);
    return LV_EHIP;
  }
  // Timing events only: no system-scope fence when they are recorded (with one, every record
  // wrote back the caches, which cost an R-MAT s25 run ~4 ms of its ~200). Nothing reads device
  // data through them; every read-back has its own copy and stream synchronisation.
  for (int i = 0; i < kEvents; i++) {
    if (hipEventCreateWithFlags(&ctx->ev[i], hipEventDisableSystemFence) != hipSuccess) {
      louvain_ctx_destroy(ctx);
      return LV_EHIP;
    }
  }
  for (int i = 0; i < 2; i++) {
    if (hipStreamCreateWithFlags(&ctx->side[i], hipStreamNonBlocking) != hipSuccess) {
      louvain_ctx_destroy(ctx);
      return LV_EHIP;
    }
  }
  for (int i = 0; i < 32; i++) {
    if (hipEventCreateWithFlags(&ctx->fork[i], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->join0[i], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->join1[i], hipEventDisableTiming) != hipSuccess) {
      louvain_ctx_destroy(ctx);
      return LV_EHIP;
    }
  }
  *out = ctx;
  return LV_OK;
}

void louvain_ctx_destroy(lv_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  for (int i = 0; i < S_COUNT_SLOTS; i++)
    if (ctx->slots[i].p) (void)hipFree(ctx->slots[i].p);
  for (int i = 0; i < kEvents; i++)
    if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
  for (int i = 0; i < 32; i++) {
    if (ctx->fork[i]) (void)hipEventDestroy(ctx->fork[i]);
    if (ctx->join0[i]) (void)hipEventDestroy(ctx->join0[i]);
    if (ctx->join1[i]) (void)hipEventDestroy(ctx->join1[i]);
  }
  for (int i = 0; i < 2; i++)
    if (ctx->side[i]) (void)hipStreamDestroy(ctx->side[i]);
  if (ctx->gin) (void)hipEventDestroy(ctx->gin);
  if (ctx->gout) (void)hipEventDestroy(ctx->gout);
  if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->bpin) (void)hipHostFree(ctx->bpin);
  delete ctx;
}

const char* louvain_last_error(const lv_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

uint64_t louvain_workspace_bytes(const lv_ctx* ctx) { return ctx ? ctx->held : 0; }

lv_status louvain_modularity(lv_ctx* ctx, const lv_graph* g, const int32_t* C, lv_i128* q_num,
                             uint64_t* W_out, double* q_out, void* stream) {
  if (!ctx) return LV_EINVAL;
  ctx->err.clear();
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  lv::DevGraph dg;
  CHK(import_graph(ctx, g, false, s, &dg));
  if (dg.n > 0 && !C) return fail(ctx, LV_EINVAL, "C is NULL");
  CHK(check_total_weight(ctx, dg, s));
  uint64_t* K = nullptr;
  uint64_t* Sig = nullptr;
  CHK(wst(ctx, S_K, dg.n, &K));
  CHK(wst(ctx, S_SIG, dg.n, &Sig));
  HIPCHK(lv::fill_u64(K, 0, dg.n, s));
  HIPCHK(lv::fill_u64(Sig, 0, dg.n, s));
  int64_t* rtile = nullptr;
  CHK(wst(ctx, S_RTILE, lv::row_sum_tiles(dg.nnz) + 1, &rtile));
  HIPCHK(lv::row_sums(dg, K, rtile, s));
  HIPCHK(lv::sigma_by_label(K, C, dg.n, Sig, s));
  ull* st = nullptr;
  CHK(wst(ctx, S_STATS, STATS_WORDS, &st));
  ull* d = st + ST_MISC;
  ull* h = ctx->pinned + PIN_MISC;
  HIPCHK(lv::zero_words(d, 5, s));
  HIPCHK(lv::sum_max_u64(K, dg.n, d, s));
  HIPCHK(lv::intra_weight(dg, C, d + 2, s));
  HIPCHK(lv::sum_squares_u64(Sig, dg.n, d + 3, s));
  HIPCHK(hipMemcpyAsync(h, d, 5 * sizeof(ull), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const uint64_t W = h[0];
  if (W > ((uint64_t)1 << 62)) return fail(ctx, LV_EOVERFLOW, "total weight exceeds 2^62");
  const u128 sq = ((u128)h[4] << 64) | h[3];
  const i128 qn = (i128)((u128)W * h[2]) - (i128)sq;
  if (q_num) *q_num = to_i128(qn);
  if (W_out) *W_out = W;
  if (q_out) *q_out = q_of(qn, W);
  return LV_OK;
}

lv_status louvain_move(lv_ctx* ctx, const lv_graph* g, const uint64_t* Kin, uint64_t Win,
                       int32_t pass_index, const lv_params* p, int32_t* C, uint64_t* Sigma,
                       int32_t* csize, lv_move_stats* stats, void* stream) {
  if (!ctx) return LV_EINVAL;
  ctx->err.clear();
  HIPCHK(hipSetDevice(ctx->device));
  CHK(check_params(ctx, p));
  if (pass_index < 0) return fail(ctx, LV_EINVAL, "pass_index must be >= 0");
  ctx->part_shift = (p->flags & LV_SMALL_PARTS) ? kSmallPartShift : 0;
  hipStream_t s = (hipStream_t)stream;
  Phase ph;
  CHK(import_graph(ctx, g, (p->flags & LV_VALIDATE) != 0, s, &ph.g));
  if (ph.g.n > 0 && (!C || !Sigma || !csize))
    return fail(ctx, LV_EINVAL, "C, Sigma or csize is NULL");
  if (stats) memset(stats, 0, sizeof(*stats));
  if (ph.g.n == 0) return LV_OK;
  CHK(check_total_weight(ctx, ph.g, s));
  const uint64_t* K = Kin;
  if (!K) {
    uint64_t* Kw = nullptr;
    CHK(wst(ctx, S_K, ph.g.n, &Kw));
    HIPCHK(lv::fill_u64(Kw, 0, ph.g.n, s));
    int64_t* rtile = nullptr;
    CHK(wst(ctx, S_RTILE, lv::row_sum_tiles(ph.g.nnz) + 1, &rtile));
    HIPCHK(lv::row_sums(ph.g, Kw, rtile, s));
    K = Kw;
  }
  uint64_t W = 0, maxK = 0;
  CHK(weight_stats(ctx, K, ph.g.n, s, &W, &maxK));
  if (Win) W = Win;
  if (W > ((uint64_t)1 << 62)) return fail(ctx, LV_EOVERFLOW, "total weight exceeds 2^62");
  if (W == 0) return LV_OK;
  void* rec = nullptr;
  CHK(ws(ctx, S_REC, (size_t)ph.g.n * lv::kRecBytes, &rec));
  HIPCHK(lv::pack_state(ph.g.n, C, Sigma, csize, rec, s));
  ph.m.K = K;
  ph.m.rec = rec;
  ph.m.W = W;
  ph.wide = (p->flags & LV_FORCE_WIDE) || !((u128)W * maxK < ((u128)1 << 63));
  ph.classes = p->substeps;
  ph.pass = pass_index;
  ph.colour = (p->flags & LV_COLOR_CLASSES) != 0;
  CHK(plan_phase(ctx, ph, s));
  PhaseOut po;
  CHK(run_phase(ctx, ph, tolerance_threshold(W, p->tolerance_exp10, p->decline_exp10, pass_index),
                p->max_iterations, p->flags, s, nullptr, &po));
  HIPCHK(lv::unpack_state(ph.g.n, rec, C, Sigma, csize, s));
  HIPCHK(hipStreamSynchronize(s));
  if (stats) {
    stats->iterations = po.iterations;
    stats->hit_cap = po.hit_cap ? 1 : 0;
    stats->moved = po.moved;
    stats->gain_sum = to_i128(po.gain_sum);
    stats->last_gain = to_i128(po.last_gain);
    stats->last_moved = po.last_moved;
    stats->last_candidates = po.last_candidates;
  }
  return LV_OK;
}

lv_status louvain_aggregate(lv_ctx* ctx, const lv_graph* g, const int32_t* C, int32_t* map,
                            void* offsets_out, int32_t offsets_64_out, int32_t* indices_out,
                            uint64_t* weights_out, int64_t* n_out, int64_t* nnz_out,
                            void* stream) {
  if (!ctx) return LV_EINVAL;
  ctx->err.clear();
  HIPCHK(hipSetDevice(ctx->device));
  ctx->part_shift = 0;
  hipStream_t s = (hipStream_t)stream;
  lv::DevGraph dg;
  CHK(import_graph(ctx, g, false, s, &dg));
  if (!n_out || !nnz_out) return fail(ctx, LV_EINVAL, "n_out or nnz_out is NULL");
  if (!offsets_out || (dg.n > 0 && (!C || !map)) || (dg.nnz > 0 && (!indices_out || !weights_out)))
    return fail(ctx, LV_EINVAL, "an output or C is NULL");
  int32_t* csize = nullptr;
  CHK(wst(ctx, S_CSIZE, dg.n, &csize));
  HIPCHK(lv::fill_i32(csize, 0, dg.n, s));
  HIPCHK(lv::count_labels(C, dg.n, csize, s));
  int32_t* okey = nullptr;
  uint64_t* ow = nullptr;
  CHK(wst(ctx, S_TKEY, dg.nnz, &okey));
  CHK(wst(ctx, S_TW, dg.nnz, &ow));
  int64_t* off64 = nullptr;
  if (offsets_64_out) {
    off64 = (int64_t*)offsets_out;
  } else {
    CHK(wst(ctx, S_AGGOFF, dg.n + 1, &off64));
  }
  lv::AggBuffers a;
  int64_t np = 0, nnzp = 0;
  CHK(aggregate(ctx, dg, C, csize, nullptr, map, okey, ow, nullptr, &a, &np, &nnzp, nullptr, s));
  HIPCHK(lv::scan_i64(a.dcount, np, off64, a.partial, s));
  HIPCHK(lv::compact_rows(off64, np, nnzp, a.oldlabel, a.astart, okey, ow, indices_out,
                          weights_out, s));
  if (!offsets_64_out) HIPCHK(lv::narrow_offsets(off64, (int32_t*)offsets_out, np + 1, s));
  HIPCHK(hipStreamSynchronize(s));
  *n_out = np;
  *nnz_out = nnzp;
  return LV_OK;
}

}  // extern "C"

// The whole method; levels (may be NULL) receives a copy of the membership after every
// aggregation, *n_levels counting them.
static lv_status run_single(lv_ctx* ctx, const lv_graph* g, const lv_params* p,
                            int32_t* membership, int32_t* levels, int32_t max_levels,
                            int32_t* n_levels, lv_result* res, void* stream) {
  if (!ctx) return LV_EINVAL;
  const auto t_start = std::chrono::steady_clock::now();
  ctx->err.clear();
  HIPCHK(hipSetDevice(ctx->device));
  CHK(check_params(ctx, p));
  if (!res) return fail(ctx, LV_EINVAL, "res is NULL");
  int32_t nlev = 0;
  if (n_levels) *n_levels = 0;
  ctx->part_shift = (p->flags & LV_SMALL_PARTS) ? kSmallPartShift : 0;
  memset(res, 0, sizeof(*res));
  hipStream_t s = (hipStream_t)stream;
  lv::DevGraph g0;
  CHK(import_graph(ctx, g, (p->flags & LV_VALIDATE) != 0, s, &g0));
  const int64_t n0 = g0.n;
  if (n0 > 0 && !membership) return fail(ctx, LV_EINVAL, "membership is NULL");
  if (n_levels && n0 > 0 && !levels) return fail(ctx, LV_EINVAL, "levels is NULL");
  res->n_communities = n0;
  if (n0 == 0) return LV_OK;
  const bool trace = (p->flags & LV_TRACE) != 0;

  uint64_t* K = nullptr;
  int32_t* C = nullptr;
  uint64_t* Sig = nullptr;
  int32_t* csize = nullptr;
  int32_t* map = nullptr;
  CHK(wst(ctx, S_K, n0, &K));
  CHK(wst(ctx, S_C, n0, &C));
  CHK(wst(ctx, S_SIG, n0, &Sig));
  CHK(wst(ctx, S_CSIZE, n0, &csize));
  CHK(wst(ctx, S_MAP, n0, &map));
  HIPCHK(lv::fill_u64(K, 0, n0, s));
  HIPCHK(lv::fill_u64(Sig, 0, n0, s));  // self-loop weight of every row until pass 0 starts
  int64_t* rtile = nullptr;
  CHK(wst(ctx, S_RTILE, lv::row_sum_tiles(g0.nnz) + 1, &rtile));
  HIPCHK(lv::row_sums(g0, K, rtile, s, Sig));
  HIPCHK(lv::iota_i32(membership, n0, s));
  CHK(check_total_weight(ctx, g0, s));
  uint64_t W = 0, maxK = 0;
  CHK(weight_stats(ctx, K, n0, s, &W, &maxK));
  res->W = W;
  if (W > ((uint64_t)1 << 62)) return fail(ctx, LV_EOVERFLOW, "total weight exceeds 2^62");
  if (W == 0) {
    HIPCHK(hipStreamSynchronize(s));
    res->total_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() -
                                                             t_start).count();
    return LV_OK;
  }

  lv::DevGraph cur = g0;
  int64_t n_comm = n0;
  // W^2 Q of the current level (before pass 0: every vertex alone)
  i128 qnum = 0;
  CHK(singleton_qnum(ctx, g0, K, Sig, W, s, &qnum));
  int which = 0;  // next super-graph buffer set
  void* rec = nullptr;
  CHK(ws(ctx, S_REC, (size_t)n0 * lv::kRecBytes, &rec));
  // Live numbering from the first aggregation on (see lv_kernels.hip): the vertices without
  // arcs (n_noarc) leave the working graph, which keeps the order of the others. rep: the
  // representatives of the working graph's super-vertices; noarc_before: prefix count of the
  // vertices without arcs. Not with colour classes, whose colouring reads the vertex ids.
  const bool live = (p->flags & LV_COLOR_CLASSES) == 0;
  bool relabelled = false;  // membership holds live ids (-1: no arcs)
  int64_t n_noarc = 0;
  int32_t* rep = nullptr;
  int rep_which = 0;
  int64_t* noarc_before = nullptr;
  int32_t* lflag = nullptr;
  int64_t* live_before = nullptr;
  int64_t* scanp0 = nullptr;
  for (int pass = 0; pass < p->max_passes; pass++) {
    int32_t* lab = nullptr;  // the records' communities, copied where the copy stays in cache
    if (cur.n <= lv::kLabMaxVertices) CHK(wst(ctx, S_LAB, cur.n, &lab));
    HIPCHK(lv::init_state(cur.n, K, rec, lab, s));
    Phase ph;
    ph.g = cur;
    ph.m.K = K;
    ph.m.rec = rec;
    ph.m.lab = lab;
    ph.m.W = W;
    ph.wide = (p->flags & LV_FORCE_WIDE) || !((u128)W * maxK < ((u128)1 << 63));
    ph.classes = p->substeps;
    ph.pass = pass;
    ph.colour = (p->flags & LV_COLOR_CLASSES) != 0;
    const int64_t n_canon = cur.n + (relabelled ? n_noarc : 0);  // vertices in the method's ids
    if (relabelled && n_noarc > 0 && p->substeps > 1) {
      uint8_t* vc = nullptr;  // hashed classes by the method's ids
      CHK(wst(ctx, S_VCLASS, cur.n, &vc));
      HIPCHK(lv::live_classes(cur.n, pass, p->substeps, rep, noarc_before, vc, s));
      ph.vclass = vc;
    }
    CHK(plan_phase(ctx, ph, s));
    PhaseOut po;
    CHK(run_phase(ctx, ph, tolerance_threshold(W, p->tolerance_exp10, p->decline_exp10, pass),
                  p->max_iterations, p->flags, s, res, &po));
    res->passes = pass + 1;
    res->iterations[pass] = po.iterations;
    res->iterations_total += po.iterations;
    res->n_pass[pass] = n_canon;
    res->nnz_pass[pass] = cur.nnz;
    if (po.hit_cap) res->cap_hits++;
    if (po.gain_sum == 0) {
      // no vertex moved: the partition is that of the previous level
      res->qnum_pass[pass] = to_i128(qnum);
      break;
    }
    // aggregation into the other buffer set: rows stay where the merge writes them
    int64_t* nrs = nullptr;
    int64_t* nre = nullptr;
    int32_t* nidx = nullptr;
    uint64_t* nw = nullptr;
    CHK(wst(ctx, which ? S_GOFF1 : S_GOFF0, cur.n, &nrs));
    CHK(wst(ctx, which ? S_GRE1 : S_GRE0, cur.n, &nre));
    CHK(wst(ctx, which ? S_GIDX1 : S_GIDX0, cur.nnz, &nidx));
    CHK(wst(ctx, which ? S_GW1 : S_GW0, cur.nnz, &nw));
    if (trace) HIPCHK(hipEventRecord(ctx->ev[EV_AGG], s));
    int64_t np = 0, nnzp = 0;
    uint64_t self = 0;
    lv::AggBuffers ab;
    HIPCHK(lv::unpack_state(cur.n, rec, C, Sig, csize, s));
    CHK(aggregate(ctx, cur, C, csize, Sig, map, nidx, nw, K, &ab, &np, &nnzp, &self, s,
                  (p->flags & LV_FORCE_WIDE) == 0, live));
    HIPCHK(lv::super_rows(np, ab, nrs, nre, s));
    // W^2 Q reached by this pass = that of singletons on the super-vertex graph
    ull* st = nullptr;
    CHK(wst(ctx, S_STATS, STATS_WORDS, &st));
    ull* d = st + ST_MISC;
    ull* h = ctx->pinned + PIN_MISC;
    HIPCHK(lv::zero_words(d, 4, s));
    HIPCHK(lv::sum_squares_u64(K, np, d, s));
    HIPCHK(lv::sum_max_u64(K, np, d + 2, s));
    HIPCHK(hipMemcpyAsync(h, d, 4 * sizeof(ull), hipMemcpyDeviceToHost, s));
    if (trace) HIPCHK(hipEventRecord(ctx->ev[EV_AGG + 1], s));
    HIPCHK(hipStreamSynchronize(s));
    if (trace)
      HIPCHK(hipEventElapsedTime(&res->aggregate_ms[pass], ctx->ev[EV_AGG], ctx->ev[EV_AGG + 1]));
    const u128 sq = ((u128)h[1] << 64) | h[0];
    const i128 q_pass = (i128)((u128)W * self) - (i128)sq;
    res->qnum_pass[pass] = to_i128(q_pass);
    // pass_tolerance = 0 (section 3.2): a pass whose moves did not raise modularity ends the
    // run, and its partition is not kept (the membership stays at the previous level)
    if (!(q_pass > qnum)) break;
    qnum = q_pass;
    maxK = h[3];
    if (live) {
      if (!relabelled) {
        // the first kept aggregation is pass 0's: its vertices without arcs got no new id
        int32_t* r0 = nullptr;
        int32_t* r1 = nullptr;
        CHK(wst(ctx, S_REP0, n0, &r0));
        CHK(wst(ctx, S_REP1, n0, &r1));
        CHK(wst(ctx, S_LFLAG, n0, &lflag));
        CHK(wst(ctx, S_NOARC, n0 + 1, &noarc_before));
        CHK(wst(ctx, S_LIVEB, n0 + 1, &live_before));
        CHK(wst(ctx, S_SCANP, lv::scan_partial_elems(n0 + 1) + 1, &scanp0));
        HIPCHK(lv::no_arc_prefix(g0, lflag, noarc_before, scanp0, s));
        HIPCHK(hipMemcpyAsync(h, noarc_before + n0, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        n_noarc = (int64_t)h[0];
        relabelled = true;
      }
      int32_t* rnext = nullptr;
      CHK(wst(ctx, rep_which ? S_REP1 : S_REP0, n0, &rnext));
      HIPCHK(lv::next_rep(np, ab.oldlabel, rep, rnext, s));
      rep = rnext;
      rep_which ^= 1;
    }
    HIPCHK(lv::compose_membership(membership, n0, map, s));
    if (levels && nlev < max_levels) {
      int32_t* lev = levels + (size_t)nlev * (size_t)n0;
      if (relabelled && n_noarc > 0) {
        CHK(wst(ctx, S_SCANP, lv::scan_partial_elems(n0 + 1) + 1, &scanp0));
        HIPCHK(lv::canon_membership(n0, membership, np, rep, noarc_before, lflag, live_before,
                                    scanp0, lev, s));
      } else {
        HIPCHK(hipMemcpyAsync(lev, membership, sizeof(int32_t) * (size_t)n0,
                              hipMemcpyDeviceToDevice, s));
      }
      nlev++;
    }
    const bool shrunk = np + (relabelled ? n_noarc : 0) < n_canon;
    lv::DevGraph nxt;
    nxt.n = np;
    nxt.nnz = nnzp;
    nxt.rs = nrs;
    nxt.re = nre;
    nxt.off = nullptr;
    nxt.idx = nidx;
    nxt.w = nw;
    nxt.w64 = !ab.w32;
    cur = nxt;
    n_comm = np + (relabelled ? n_noarc : 0);
    which ^= 1;
    if (!shrunk) break;
  }
  if (relabelled && n_noarc > 0) {  // back to the method's numbering, in place
    CHK(wst(ctx, S_SCANP, lv::scan_partial_elems(n0 + 1) + 1, &scanp0));
    HIPCHK(lv::canon_membership(n0, membership, cur.n, rep, noarc_before, lflag, live_before,
                                scanp0, membership, s));
  }
  res->n_communities = n_comm;
  res->q_num = to_i128(qnum);
  res->q = q_of(qnum, W);
  HIPCHK(hipStreamSynchronize(s));
  if (n_levels) *n_levels = nlev;
  res->total_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() -
                                                           t_start).count();
  return LV_OK;
}

extern "C" {

lv_status louvain_run(lv_ctx* ctx, const lv_graph* g, const lv_params* p, int32_t* membership,
                      lv_result* res, void* stream) {
  return run_single(ctx, g, p, membership, nullptr, 0, nullptr, res, stream);
}

lv_status louvain_run_levels(lv_ctx* ctx, const lv_graph* g, const lv_params* p,
                             int32_t* membership, int32_t* levels, int32_t max_levels,
                             int32_t* n_levels, lv_result* res, void* stream) {
  if (!ctx) return LV_EINVAL;
  ctx->err.clear();
  if (!n_levels) return fail(ctx, LV_EINVAL, "n_levels is NULL");
  *n_levels = 0;
  if (!p) return fail(ctx, LV_EINVAL, "params is NULL");
  if (max_levels < p->max_passes)
    return fail(ctx, LV_EINVAL, "max_levels is below max_passes");
  return run_single(ctx, g, p, membership, levels, max_levels, n_levels, res, stream);
}

// Many graphs in one run: the packed union goes through the same kernels as one graph, with each
// vertex's W, tolerance, iteration state and class hash taken from its own graph, so that every
// graph's result equals that of louvain_run on it alone.
lv_status louvain_run_batched(lv_ctx* ctx, const lv_graph* packed, int32_t G,
                              const int64_t* graph_vptr, const int64_t* graph_aptr,
                              const lv_params* p, int32_t* membership,
                              lv_graph_result* per_graph, void* stream) {
  if (!ctx) return LV_EINVAL;
  ctx->err.clear();
  HIPCHK(hipSetDevice(ctx->device));
  CHK(check_params(ctx, p));
  if (G < 1) return fail(ctx, LV_EINVAL, "G must be >= 1");
  if (!graph_vptr || !graph_aptr || !per_graph)
    return fail(ctx, LV_EINVAL, "graph_vptr, graph_aptr or per_graph is NULL");
  if (!packed) return fail(ctx, LV_EINVAL, "graph is NULL");
  if (graph_vptr[0] != 0 || graph_aptr[0] != 0 || graph_vptr[G] != packed->n ||
      graph_aptr[G] != packed->nnz)
    return fail(ctx, LV_EINVAL, "graph_vptr/graph_aptr must start at 0 and end at n/nnz");
  for (int32_t g = 0; g < G; g++)
    if (graph_vptr[g + 1] < graph_vptr[g] || graph_aptr[g + 1] < graph_aptr[g])
      return fail(ctx, LV_EINVAL, "graph_vptr/graph_aptr must be non-decreasing");
  ctx->part_shift = (p->flags & LV_SMALL_PARTS) ? kSmallPartShift : 0;
  memset(per_graph, 0, sizeof(lv_graph_result) * (size_t)G);
  for (int32_t g = 0; g < G; g++) per_graph[g].n_communities = graph_vptr[g + 1] - graph_vptr[g];
  hipStream_t s = (hipStream_t)stream;
  lv::DevGraph g0;
  CHK(import_graph(ctx, packed, (p->flags & LV_VALIDATE) != 0, s, &g0));
  const int64_t n0 = g0.n;
  if (n0 > 0 && !membership) return fail(ctx, LV_EINVAL, "membership is NULL");
  if (n0 == 0) return LV_OK;

  // per-graph device words: Wg [G], gS [2G], gself [G], gsq [2G]; act [G] bytes; graph bases:
  // three arrays of G + 1 (level 0, then two alternating levels); aptr for validation
  ull* gw = nullptr;
  uint8_t* gact = nullptr;
  int64_t* gbase = nullptr;
  int64_t* aptr_d = nullptr;
  int32_t* gid0 = nullptr;
  CHK(wst(ctx, S_GWORDS, 6 * (int64_t)G, &gw));
  CHK(wst(ctx, S_GACT, G, &gact));
  CHK(wst(ctx, S_GBASE, 3 * ((int64_t)G + 1), &gbase));
  CHK(wst(ctx, S_GID0, n0, &gid0));
  ull* Wg = gw;
  ull* gS = nullptr;  // kGainSlices copies of 2G words
  CHK(wst(ctx, S_GSLICE, 2 * (int64_t)lv::kGainSlices * G, &gS));
  ull* gself = gw + 3 * (int64_t)G;
  ull* gsq = gw + 4 * (int64_t)G;
  void* pin = nullptr;
  CHK(batch_pinned(ctx, (size_t)G * (6 * sizeof(ull) + 2) + 64, &pin));
  ull* hw = (ull*)pin;                       // 4G words of read-backs
  uint8_t* hact = (uint8_t*)(hw + 4 * (int64_t)G);
  uint8_t* hkeep = hact + G;
  HIPCHK(hipMemcpyAsync(gbase, graph_vptr, ((size_t)G + 1) * sizeof(int64_t),
                        hipMemcpyHostToDevice, s));
  HIPCHK(lv::graph_ids(gbase, G, n0, gid0, s));
  if (p->flags & LV_VALIDATE) {
    CHK(wst(ctx, S_APTR, (int64_t)G + 1, &aptr_d));
    unsigned int* bad = nullptr;
    CHK(wst(ctx, S_BAD, 1, &bad));
    HIPCHK(hipMemsetAsync(bad, 0, sizeof(unsigned int), s));
    HIPCHK(hipMemcpyAsync(aptr_d, graph_aptr, ((size_t)G + 1) * sizeof(int64_t),
                          hipMemcpyHostToDevice, s));
    HIPCHK(lv::validate_batch(g0, gid0, gbase, aptr_d, G, bad, s));
    unsigned int hb = 0;
    HIPCHK(hipMemcpyAsync(&hb, bad, sizeof(hb), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hb & 1u) return fail(ctx, LV_EINVAL, "graph_aptr does not match the offsets");
    if (hb & 2u) return fail(ctx, LV_EINVAL, "an arc joins two graphs of the batch");
  }

  uint64_t* K = nullptr;
  int32_t* C = nullptr;
  uint64_t* Sig = nullptr;
  int32_t* csize = nullptr;
  int32_t* map = nullptr;
  CHK(wst(ctx, S_K, n0, &K));
  CHK(wst(ctx, S_C, n0, &C));
  CHK(wst(ctx, S_SIG, n0, &Sig));
  CHK(wst(ctx, S_CSIZE, n0, &csize));
  CHK(wst(ctx, S_MAP, n0, &map));
  HIPCHK(lv::fill_u64(K, 0, n0, s));
  uint64_t* selfw = Sig;  // self-loop weight of every row until the first pass
  HIPCHK(lv::fill_u64(selfw, 0, n0, s));
  int64_t* rtile = nullptr;
  CHK(wst(ctx, S_RTILE, lv::row_sum_tiles(g0.nnz) + 1, &rtile));
  HIPCHK(lv::row_sums(g0, K, rtile, s, selfw));
  {
    // every 64-bit sum below (row sums, per-graph W, their total) is exact when the batch's
    // total weight is below 2^64
    u128 t = 0;
    CHK(total_weight(ctx, g0, s, &t));
    if (t >> 64) return fail(ctx, LV_EOVERFLOW, "the batch's total weight reaches 2^64");
  }
  uint64_t Wtot = 0, maxK = 0;
  CHK(weight_stats(ctx, K, n0, s, &Wtot, &maxK));
  // per graph: W, and W^2 Q of every vertex alone (self-loop weight and sum of K^2)
  HIPCHK(lv::zero_words(Wg, G, s));
  HIPCHK(lv::zero_words(gself, 3 * (int64_t)G, s));
  HIPCHK(lv::graph_sums(K, n0, gid0, false, Wg, s));
  HIPCHK(lv::graph_sums(selfw, n0, gid0, false, gself, s));
  HIPCHK(lv::graph_sums(K, n0, gid0, true, gsq, s));
  HIPCHK(hipMemcpyAsync(hw, Wg, (size_t)G * sizeof(ull), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hw + G, gself, 3 * (size_t)G * sizeof(ull), hipMemcpyDeviceToHost, s));
  HIPCHK(lv::iota_i32(membership, n0, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<uint64_t> W(G);
  std::vector<uint8_t> done(G);
  std::vector<i128> qnum(G, 0);  // W^2 Q of every graph's current level
  uint64_t maxW = 0;
  for (int32_t g = 0; g < G; g++) {
    W[g] = hw[g];
    per_graph[g].W = W[g];
    done[g] = W[g] == 0;  // no arcs: identity membership, Q = 0, no pass
    maxW = std::max(maxW, W[g]);
    const u128 sq = ((u128)hw[2 * G + 2 * (int64_t)g + 1] << 64) | hw[2 * G + 2 * (int64_t)g];
    qnum[g] = (i128)((u128)W[g] * hw[G + g]) - (i128)sq;
  }
  if (maxW > ((uint64_t)1 << 62)) return fail(ctx, LV_EOVERFLOW, "a graph's weight exceeds 2^62");
  // graphs whose last pass was dropped (it did not raise modularity): their membership stays at
  // the level that pass ran on, whose first super-vertex is gtop[g]
  std::vector<uint8_t> kept(G, 0);
  std::vector<int64_t> gtop(graph_vptr, graph_vptr + G);
  uint8_t* keep_d = nullptr;
  bool any_kept = false;

  lv::DevGraph cur = g0;
  const int32_t* gid = gid0;
  int64_t* gb_cur = gbase;
  int which = 0;
  void* rec = nullptr;
  CHK(ws(ctx, S_REC, (size_t)n0 * lv::kRecBytes, &rec));
  BatchPhase bp;
  bp.G = G;
  bp.hS = hw;
  bp.hact = hact;
  bp.size.resize(G);
  for (int32_t g = 0; g < G; g++) bp.size[g] = graph_vptr[g + 1] - graph_vptr[g];
  for (int pass = 0; pass < p->max_passes; pass++) {
    bool any = false;
    for (int32_t g = 0; g < G; g++) any = any || !done[g];
    if (!any) break;
    HIPCHK(lv::init_state(cur.n, K, rec, nullptr, s));
    Phase ph;
    ph.g = cur;
    ph.m.K = K;
    ph.m.rec = rec;
    ph.m.W = Wtot;
    ph.m.gs.G = G;
    ph.m.gs.gid = gid;
    ph.m.gs.gbase = gb_cur;
    ph.m.gs.Wg = (const uint64_t*)Wg;
    ph.m.gs.act = gact;
    ph.m.gs.gS = gS;
    ph.wide = (p->flags & LV_FORCE_WIDE) || !((u128)maxW * maxK < ((u128)1 << 63));
    ph.classes = p->substeps;
    ph.pass = pass;
    ph.colour = (p->flags & LV_COLOR_CLASSES) != 0;
    bp.T.assign(G, 0);
    bp.act.assign(G, 0);
    bp.passgain.assign(G, 0);
    bp.iters.assign(G, 0);
    bp.capped.assign(G, 0);
    for (int32_t g = 0; g < G; g++) {
      bp.act[g] = !done[g];
      bp.T[g] = tolerance_threshold(W[g], p->tolerance_exp10, p->decline_exp10, pass);
    }
    memcpy(hact, bp.act.data(), (size_t)G);
    HIPCHK(hipMemcpyAsync(gact, hact, (size_t)G, hipMemcpyHostToDevice, s));
    bp.listed = 0;
    for (int32_t g = 0; g < G; g++)
      if (bp.act[g]) bp.listed += bp.size[g];
    CHK(plan_phase(ctx, ph, s));
    PhaseOut po;
    CHK(run_phase(ctx, ph, 0, p->max_iterations, p->flags & ~LV_TRACE, s, nullptr, &po, &bp));
    std::vector<uint8_t> ran(G, 0);
    for (int32_t g = 0; g < G; g++) {
      if (done[g]) continue;
      ran[g] = 1;
      lv_graph_result& r = per_graph[g];
      r.passes = pass + 1;
      r.iterations[pass] = bp.iters[g];
      r.iterations_total += bp.iters[g];
      r.cap_hits += bp.capped[g];
      if (bp.passgain[g] == 0) done[g] = 1;  // no move: the partition is that of this level
    }
    // aggregate the whole union (a graph with no move maps to itself); per-graph Qnum of the
    // new level = that of singletons on it
    int64_t* nrs = nullptr;
    int64_t* nre = nullptr;
    int32_t* nidx = nullptr;
    uint64_t* nw = nullptr;
    int32_t* ngid = nullptr;
    CHK(wst(ctx, which ? S_GOFF1 : S_GOFF0, cur.n, &nrs));
    CHK(wst(ctx, which ? S_GRE1 : S_GRE0, cur.n, &nre));
    CHK(wst(ctx, which ? S_GIDX1 : S_GIDX0, cur.nnz, &nidx));
    CHK(wst(ctx, which ? S_GW1 : S_GW0, cur.nnz, &nw));
    CHK(wst(ctx, which ? S_GIDB : S_GIDA, cur.n, &ngid));
    int64_t* gb_next = gbase + ((int64_t)G + 1) * (which ? 2 : 1);
    int64_t np = 0, nnzp = 0;
    uint64_t self = 0;
    lv::AggBuffers ab;
    ab.gs.gid = gid;
    ab.gs.gself = gself;
    HIPCHK(lv::zero_words(gself, G, s));
    HIPCHK(lv::unpack_state(cur.n, rec, C, Sig, csize, s));
    CHK(aggregate(ctx, cur, C, csize, Sig, map, nidx, nw, K, &ab, &np, &nnzp, &self, s,
                  (p->flags & LV_FORCE_WIDE) == 0));
    HIPCHK(lv::super_rows(np, ab, nrs, nre, s));
    HIPCHK(lv::next_gbase(ab.newid, gb_cur, G, gb_next, s));
    HIPCHK(lv::graph_ids(gb_next, G, np, ngid, s));
    HIPCHK(lv::zero_words(gsq, 2 * (int64_t)G, s));
    HIPCHK(lv::graph_sums(K, np, ngid, true, gsq, s));
    ull* d = nullptr;
    {
      ull* st = nullptr;
      CHK(wst(ctx, S_STATS, STATS_WORDS, &st));
      d = st + ST_MISC;
    }
    HIPCHK(lv::zero_words(d, 2, s));
    HIPCHK(lv::sum_max_u64(K, np, d, s));
    HIPCHK(hipMemcpyAsync(hw, gself, 3 * (size_t)G * sizeof(ull), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hw + 3 * (int64_t)G, d, 2 * sizeof(ull), hipMemcpyDeviceToHost, s));
    std::vector<int64_t> nb_old(G + 1), nb_new(G + 1);
    HIPCHK(hipMemcpyAsync(nb_old.data(), gb_cur, ((size_t)G + 1) * sizeof(int64_t),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(nb_new.data(), gb_next, ((size_t)G + 1) * sizeof(int64_t),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    maxK = hw[3 * (int64_t)G + 1];
    bool newly_kept = false;
    for (int32_t g = 0; g < G; g++) {
      bp.size[g] = nb_new[g + 1] - nb_new[g];
      if (kept[g]) continue;
      if (ran[g]) {
        const u128 sq = ((u128)hw[G + 2 * (int64_t)g + 1] << 64) | hw[G + 2 * (int64_t)g];
        const i128 q_pass = (i128)((u128)W[g] * hw[g]) - (i128)sq;
        if (bp.passgain[g] != 0 && !(q_pass > qnum[g])) {
          // pass_tolerance = 0: the pass moved vertices without raising modularity; it is
          // dropped and the graph's membership stays at the level it ran on
          kept[g] = 1;
          done[g] = 1;
          newly_kept = true;
          continue;
        }
        qnum[g] = q_pass;
        if (nb_new[g + 1] - nb_new[g] == nb_old[g + 1] - nb_old[g]) done[g] = 1;  // no shrink
      }
      per_graph[g].n_communities = nb_new[g + 1] - nb_new[g];
      gtop[g] = nb_new[g];
    }
    if (newly_kept) {
      if (!keep_d) CHK(wst(ctx, S_GKEEP, G, &keep_d));
      memcpy(hkeep, kept.data(), (size_t)G);
      HIPCHK(hipMemcpyAsync(keep_d, hkeep, (size_t)G, hipMemcpyHostToDevice, s));
      any_kept = true;
    }
    if (any_kept) HIPCHK(lv::compose_membership_masked(membership, n0, map, gid0, keep_d, s));
    else HIPCHK(lv::compose_membership(membership, n0, map, s));
    lv::DevGraph nxt;
    nxt.n = np;
    nxt.nnz = nnzp;
    nxt.rs = nrs;
    nxt.re = nre;
    nxt.off = nullptr;
    nxt.idx = nidx;
    nxt.w = nw;
    nxt.w64 = !ab.w32;
    cur = nxt;
    gid = ngid;
    gb_cur = gb_next;
    which ^= 1;
  }
  int64_t* gtop_d = nullptr;
  CHK(wst(ctx, S_GTOP, G, &gtop_d));
  HIPCHK(hipMemcpyAsync(gtop_d, gtop.data(), (size_t)G * sizeof(int64_t), hipMemcpyHostToDevice,
                        s));
  HIPCHK(lv::localize_membership(membership, n0, gid0, gtop_d, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int32_t g = 0; g < G; g++) {
    per_graph[g].q_num = to_i128(qnum[g]);
    per_graph[g].q = q_of(qnum[g], W[g]);
  }
  return LV_OK;
}

// Graph preparation: expand the edge list into arcs, radix-sort them by (source, neighbour),
// combine runs of equal arcs and write the CSR.
lv_status louvain_prepare(lv_ctx* ctx, int64_t n, int64_t m, const int32_t* src,
                          const int32_t* dst, const uint32_t* weights, uint32_t flags,
                          void* offsets_out, int32_t offsets_64_out, int32_t* indices_out,
                          void* weights_out, int32_t weights_64_out, int64_t capacity,
                          int64_t* nnz_out, lv_prep_stats* stats, void* stream) {
  if (!ctx) return LV_EINVAL;
  const auto t_start = std::chrono::steady_clock::now();
  ctx->err.clear();
  if (!nnz_out) return fail(ctx, LV_EINVAL, "nnz_out is NULL");
  *nnz_out = 0;
  lv_prep_stats st_local;
  lv_prep_stats& ps = stats ? *stats : st_local;
  memset(&ps, 0, sizeof(ps));
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  if (n < 0 || m < 0 || capacity < 0) return fail(ctx, LV_EINVAL, "negative size");
  if (n >= ((int64_t)1 << 31)) return fail(ctx, LV_EOVERFLOW, "n must be below 2^31");
  if (flags & ~(LV_PREP_SYMMETRIZE | LV_PREP_SELF_LOOPS | LV_PREP_MAX | LV_PREP_TRACE |
                LV_PREP_TILE_SORT))
    return fail(ctx, LV_EINVAL, "unknown preparation flag");
  if (m > 0 && (!src || !dst)) return fail(ctx, LV_EINVAL, "src or dst is NULL");
  const bool query = !indices_out && !weights_out;
  if (!query && (!offsets_out || !indices_out || !weights_out))
    return fail(ctx, LV_EINVAL, "offsets_out, indices_out or weights_out is NULL");
  const bool sym = (flags & LV_PREP_SYMMETRIZE) != 0, loops = (flags & LV_PREP_SELF_LOOPS) != 0;
  if (m > ((int64_t)1 << 60)) return fail(ctx, LV_EOVERFLOW, "too many edges");
  const int64_t N = m * (sym ? 2 : 1) + (loops ? n : 0);
  if (N >= ((int64_t)1 << 40) || N / lv::kPrepTile >= ((int64_t)1 << 31))
    return fail(ctx, LV_EOVERFLOW, "too many arcs");
  ps.arcs = N;
  // LV_PREP_TRACE: events at phase boundaries, phase kind of every interval
  const bool trace = (flags & LV_PREP_TRACE) != 0;
  int nev = 0;
  int kinds[kEvents];
  auto mark = [&](int kind) -> hipError_t {
    if (!trace || nev >= kEvents) return hipSuccess;
    kinds[nev] = kind;
    return hipEventRecord(ctx->ev[nev++], s);
  };
  auto finish = [&]() -> hipError_t {
    ps.total_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() -
                                                           t_start).count();
    if (!trace || nev < 2) return hipSuccess;
    hipError_t e = hipEventSynchronize(ctx->ev[nev - 1]);
    if (e != hipSuccess) return e;
    for (int i = 1; i < nev; i++) {
      if (kinds[i] == 0) continue;  // an interval spent waiting for the host
      float ms = 0;
      if ((e = hipEventElapsedTime(&ms, ctx->ev[i - 1], ctx->ev[i])) != hipSuccess) return e;
      float* dst = kinds[i] == 1 ? &ps.expand_ms : kinds[i] == 2 ? &ps.hist_ms
                   : kinds[i] == 3 ? &ps.scan_ms : kinds[i] == 4 ? &ps.scatter_ms
                   : &ps.emit_ms;
      *dst += ms;
    }
    return hipSuccess;
  };
  if (N == 0) {
    if (!query) {
      if (offsets_64_out)
        HIPCHK(lv::fill_i64((int64_t*)offsets_out, 0, n + 1, s));
      else
        HIPCHK(lv::fill_i32((int32_t*)offsets_out, 0, n + 1, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    return LV_OK;
  }
  const int b = lv::prep_key_bits(n);
  const int64_t ntiles = (N + lv::kPrepTile - 1) / lv::kPrepTile;
  uint64_t* k0 = nullptr;
  uint64_t* k1 = nullptr;
  uint32_t* v0 = nullptr;
  uint32_t* v1 = nullptr;
  unsigned int* bad = nullptr;
  CHK(wst(ctx, S_PKEY0, N, &k0));
  CHK(wst(ctx, S_PKEY1, N, &k1));
  if (weights) {  // without input weights only the keys are sorted
    CHK(wst(ctx, S_PVAL0, N, &v0));
    CHK(wst(ctx, S_PVAL1, N, &v1));
  }
  CHK(wst(ctx, S_BAD, 1, &bad));
  HIPCHK(lv::fill_i32((int32_t*)bad, 0, 1, s));
  ps.key_bits = 2 * b;
  HIPCHK(mark(0));
  HIPCHK(lv::prep_expand(n, m, src, dst, weights, flags, b, k0, v0, bad, s));
  HIPCHK(mark(1));
  unsigned int hb = 0;
  HIPCHK(hipMemcpyAsync(&hb, bad, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hb & 1u) return fail(ctx, LV_EINVAL, "an edge endpoint is out of range");
  if (hb & 2u) return fail(ctx, LV_EINVAL, "a weight is zero");
  HIPCHK(mark(0));
  // LSD passes over the 2b key bits, digits as even as possible
  const int B = 2 * b;
  lv::SortPlan plan;
  plan.passes = (B + lv::kRadixBits - 1) / lv::kRadixBits;
  for (int p = 0, shift = 0; p < plan.passes; p++) {
    plan.shift[p] = shift;
    plan.bits[p] = (B - shift + (plan.passes - p) - 1) / (plan.passes - p);
    shift += plan.bits[p];
  }
  ps.sort_passes = plan.passes;
  int64_t* scanp = nullptr;
  CHK(wst(ctx, S_SCANP, lv::scan_partial_elems(((int64_t)1 << lv::kRadixBits) * ntiles + 1) + 1,
          &scanp));
  if (flags & LV_PREP_TILE_SORT) {
    // per pass: per-tile histograms, their scan, the scatter
    int32_t* hist = nullptr;
    int64_t* offs = nullptr;
    const int64_t hist_n = ((int64_t)1 << lv::kRadixBits) * ntiles;
    CHK(wst(ctx, S_PHIST, hist_n, &hist));
    CHK(wst(ctx, S_POFFS, hist_n + 1, &offs));
    for (int p = 0; p < plan.passes; p++) {
      const int64_t hn = ((int64_t)1 << plan.bits[p]) * ntiles;
      HIPCHK(lv::radix_hist(k0, N, plan.shift[p], plan.bits[p], hist, s));
      HIPCHK(mark(2));
      HIPCHK(lv::scan_i32(hist, hn, offs, scanp, s));
      HIPCHK(mark(3));
      HIPCHK(lv::radix_scatter(k0, v0, k1, v1, N, plan.shift[p], plan.bits[p], offs, s));
      HIPCHK(mark(4));
      std::swap(k0, k1);
      std::swap(v0, v1);
    }
  } else {
    // all passes' digit counts in one read, then one look-back scatter per pass
    ull* ghist = nullptr;
    int64_t* gbase = nullptr;
    ull* status = nullptr;
    CHK(wst(ctx, S_PGHIST, lv::kMaxSortPasses * 256, &ghist));
    CHK(wst(ctx, S_PGBASE, lv::kMaxSortPasses * 256, &gbase));
    CHK(wst(ctx, S_PSTATUS, ntiles * 256 + 1, &status));
    HIPCHK(lv::fill_i32((int32_t*)bad, 0, 1, s));
    HIPCHK(lv::radix_counts(k0, N, plan, ghist, gbase, s));
    HIPCHK(mark(2));
    for (int p = 0; p < plan.passes; p++) {
      HIPCHK(lv::radix_onesweep(k0, v0, k1, v1, N, plan.shift[p], plan.bits[p], gbase + 256 * p,
                                status, bad, s));
      HIPCHK(mark(4));
      std::swap(k0, k1);
      std::swap(v0, v1);
    }
    HIPCHK(hipMemcpyAsync(&hb, bad, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hb & 8u) return fail(ctx, LV_EHIP, "radix sort look-back did not complete");
    HIPCHK(mark(0));
  }
  int32_t* theads = nullptr;
  int64_t* tslot = nullptr;
  ull* tfirst = nullptr;
  const bool cmax = (flags & LV_PREP_MAX) != 0;
  CHK(wst(ctx, S_PTILE, ntiles, &theads));
  CHK(wst(ctx, S_PSLOT, ntiles + 1, &tslot));
  CHK(wst(ctx, S_PFIRST, ntiles, &tfirst));
  HIPCHK(lv::prep_heads(k0, v0, N, b, cmax, theads, tfirst, s));
  HIPCHK(lv::scan_i32(theads, ntiles, tslot, scanp, s));
  HIPCHK(mark(5));
  int64_t nnz = 0;
  HIPCHK(hipMemcpyAsync(&nnz, tslot + ntiles, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *nnz_out = nnz;
  ps.nnz = nnz;
  if (query) {
    HIPCHK(finish());
    return LV_OK;
  }
  if (capacity < nnz)
    return fail(ctx, LV_EINVAL, "capacity " + std::to_string(capacity) + " is below the " +
                                    std::to_string(nnz) + " arcs of the prepared graph");
  if (!offsets_64_out && nnz >= ((int64_t)1 << 31))
    return fail(ctx, LV_EOVERFLOW, "nnz >= 2^31 needs int64 offsets");
  HIPCHK(mark(0));
  int64_t* off64 = nullptr;
  if (offsets_64_out)
    off64 = (int64_t*)offsets_out;
  else
    CHK(wst(ctx, S_POFF, n + 1, &off64));
  HIPCHK(lv::fill_i32((int32_t*)bad, 0, 1, s));
  HIPCHK(lv::prep_emit(k0, v0, N, n, b, cmax, !weights_64_out, tslot, theads, tfirst, off64,
                       indices_out, weights_out, bad, s));
  if (!offsets_64_out) HIPCHK(lv::narrow_offsets(off64, (int32_t*)offsets_out, n + 1, s));
  if (!weights_64_out)
    HIPCHK(hipMemcpyAsync(&hb, bad, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
  HIPCHK(mark(5));
  HIPCHK(hipStreamSynchronize(s));
  if (!weights_64_out && (hb & 4u))
    return fail(ctx, LV_EOVERFLOW, "a combined weight exceeds 32 bits; use 64-bit weights");
  HIPCHK(finish());
  return LV_OK;
}

lv_status louvain_colour_classes(lv_ctx* ctx, const lv_graph* g, int32_t pass, int32_t K,
                                 uint8_t* classes, int32_t* rounds, void* stream) {
  if (!ctx) return LV_EINVAL;
  ctx->err.clear();
  if (rounds) *rounds = 0;
  HIPCHK(hipSetDevice(ctx->device));
  if (pass < 0) return fail(ctx, LV_EINVAL, "pass must be >= 0");
  if (K < 1 || K > lv_max_classes()) return fail(ctx, LV_EINVAL, "K must be in 1..32");
  hipStream_t s = (hipStream_t)stream;
  ctx->part_shift = 0;
  Phase ph;
  CHK(import_graph(ctx, g, false, s, &ph.g));
  if (ph.g.n > 0 && !classes) return fail(ctx, LV_EINVAL, "classes is NULL");
  if (ph.g.n == 0) return LV_OK;
  if (K == 1) {
    HIPCHK(hipMemsetAsync(classes, 0, (size_t)ph.g.n, s));
    HIPCHK(hipStreamSynchronize(s));
    return LV_OK;
  }
  ph.classes = K;
  ph.pass = pass;
  CHK(colour_phase(ctx, ph, s));
  HIPCHK(hipMemcpyAsync(classes, ph.vclass, (size_t)ph.g.n, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  if (rounds) *rounds = ph.colour_rounds;
  return LV_OK;
}

lv_status louvain_probe_gather(lv_ctx* ctx, uint64_t table_bytes, int32_t slices, double* rate,
                               void* stream) {
  if (!ctx) return LV_EINVAL;
  ctx->err.clear();
  HIPCHK(hipSetDevice(ctx->device));
  if (!rate) return fail(ctx, LV_EINVAL, "rate is NULL");
  *rate = 0;
  if (slices < 1 || slices > 64) return fail(ctx, LV_EINVAL, "slices must be in 1..64");
  const uint64_t n = table_bytes / 4 / (uint64_t)slices * (uint64_t)slices;
  if (n < (uint64_t)slices) return fail(ctx, LV_EINVAL, "the table holds fewer than slices ints");
  if (n > ((uint64_t)1 << 40)) return fail(ctx, LV_EINVAL, "table_bytes is too large");
  hipStream_t s = (hipStream_t)stream;
  int32_t* table = nullptr;
  int32_t* out = nullptr;
  CHK(wst(ctx, S_PROBE_T, (int64_t)n, &table));
  CHK(wst(ctx, S_PROBE_O, lv::probe_threads(), &out));
  HIPCHK(hipMemsetAsync(table, 0, n * sizeof(int32_t), s));
  HIPCHK(lv::gather_probe(table, n, (uint32_t)slices, out, s));  // warm-up
  float best = 0;
  for (int r = 0; r < 3; r++) {
    HIPCHK(hipEventRecord(ctx->ev[0], s));
    HIPCHK(lv::gather_probe(table, n, (uint32_t)slices, out, s));
    HIPCHK(hipEventRecord(ctx->ev[1], s));
    HIPCHK(hipEventSynchronize(ctx->ev[1]));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
    if (ms > 0 && (best == 0 || ms < best)) best = ms;
  }
  if (best > 0) *rate = (double)lv::probe_gathers() / (best * 1e-3);
  return LV_OK;
}

// Partition and merge: the parts' induced subgraphs as one batch, their communities combined,
// the whole graph aggregated by them and run once more.
lv_status louvain_run_partitioned(lv_ctx* ctx, const lv_graph* g, int32_t P,
                                  const int64_t* part_vptr, const lv_params* p,
                                  int32_t* membership, lv_graph_result* per_part,
                                  lv_result* merge_res, void* stream) {
  if (!ctx) return LV_EINVAL;
  ctx->err.clear();
  HIPCHK(hipSetDevice(ctx->device));
  CHK(check_params(ctx, p));
  if (!merge_res) return fail(ctx, LV_EINVAL, "merge_res is NULL");
  if (P < 1 || P > (1 << 20)) return fail(ctx, LV_EINVAL, "P must be in 1..2^20");
  memset(merge_res, 0, sizeof(*merge_res));
  if (per_part) memset(per_part, 0, sizeof(lv_graph_result) * (size_t)P);
  hipStream_t s = (hipStream_t)stream;
  lv::DevGraph dg;
  CHK(import_graph(ctx, g, (p->flags & LV_VALIDATE) != 0, s, &dg));
  const int64_t n = dg.n;
  if (n > 0 && !membership) return fail(ctx, LV_EINVAL, "membership is NULL");
  if (n == 0) return LV_OK;
  // part bounds (host and device)
  std::vector<int64_t> vptr((size_t)P + 1), aptr((size_t)P + 1);
  int64_t* vptr_d = nullptr;
  CHK(wst(ctx, S_PM_VPTR, (int64_t)P + 1, &vptr_d));
  if (part_vptr) {
    if (part_vptr[0] != 0 || part_vptr[P] != n)
      return fail(ctx, LV_EINVAL, "part bounds must run from 0 to n");
    for (int32_t k = 0; k < P; k++)
      if (part_vptr[k + 1] < part_vptr[k]) return fail(ctx, LV_EINVAL, "part bounds decrease");
    memcpy(vptr.data(), part_vptr, sizeof(int64_t) * ((size_t)P + 1));
    HIPCHK(hipMemcpyAsync(vptr_d, vptr.data(), sizeof(int64_t) * ((size_t)P + 1),
                          hipMemcpyHostToDevice, s));
  } else {
    HIPCHK(lv::part_bounds(dg.off, n, dg.nnz, P, vptr_d, s));
    HIPCHK(hipMemcpyAsync(vptr.data(), vptr_d, sizeof(int64_t) * ((size_t)P + 1),
                          hipMemcpyDeviceToHost, s));
  }
  // the induced union: arcs whose ends share a part, same vertex ids
  int32_t* gid = nullptr;
  int32_t* flag = nullptr;
  int64_t* pos = nullptr;
  int64_t* partial = nullptr;
  int32_t* nidx = nullptr;
  void* nw = nullptr;
  int64_t* noff = nullptr;
  int64_t* aptr_d = nullptr;
  CHK(wst(ctx, S_PM_GID, n, &gid));
  CHK(wst(ctx, S_PM_FLAG, dg.nnz, &flag));
  CHK(wst(ctx, S_PM_POS, dg.nnz + 1, &pos));
  CHK(wst(ctx, S_SCANP, lv::scan_partial_elems(dg.nnz + 1) + 1, &partial));
  CHK(wst(ctx, S_PM_IDX, dg.nnz, &nidx));
  CHK(ws(ctx, S_PM_W, (size_t)(dg.nnz > 0 ? dg.nnz : 1) * (dg.w64 ? 8 : 4), &nw));
  CHK(wst(ctx, S_PM_OFF, n + 1, &noff));
  CHK(wst(ctx, S_PM_APTR, (int64_t)P + 1, &aptr_d));
  HIPCHK(lv::graph_ids(vptr_d, P, n, gid, s));
  HIPCHK(lv::part_induced(dg, gid, vptr_d, P, flag, pos, partial, nidx, nw, noff, aptr_d, s));
  HIPCHK(hipMemcpyAsync(aptr.data(), aptr_d, sizeof(int64_t) * ((size_t)P + 1),
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  // every part on its own: one batched run
  lv_graph ug;
  ug.n = n;
  ug.nnz = aptr[P];
  ug.offsets = noff;
  ug.indices = nidx;
  ug.weights = nw;
  ug.offsets_64 = 1;
  ug.weights_64 = dg.w64 ? 1 : 0;
  lv_params inner = *p;
  inner.flags &= ~(LV_VALIDATE | LV_TRACE);
  int32_t* lab = nullptr;
  CHK(wst(ctx, S_PM_LAB, n, &lab));
  std::vector<lv_graph_result> pr((size_t)P);
  CHK(louvain_run_batched(ctx, &ug, P, vptr.data(), aptr.data(), &inner, lab, pr.data(),
                          stream));
  if (per_part) memcpy(per_part, pr.data(), sizeof(lv_graph_result) * (size_t)P);
  // part communities numbered part after part
  std::vector<int64_t> loff((size_t)P);
  int64_t acc = 0;
  for (int32_t k = 0; k < P; k++) {
    loff[k] = acc;
    acc += pr[k].n_communities;
  }
  int64_t* loff_d = nullptr;
  CHK(wst(ctx, S_PM_LOFF, P, &loff_d));
  HIPCHK(hipMemcpyAsync(loff_d, loff.data(), sizeof(int64_t) * (size_t)P, hipMemcpyHostToDevice,
                        s));
  HIPCHK(lv::part_offset_labels(lab, n, gid, loff_d, s));
  // the merge: the whole graph aggregated by the combined communities, then the method on it
  int32_t* map = nullptr;
  int64_t* soff = nullptr;
  int32_t* sidx = nullptr;
  uint64_t* sw = nullptr;
  CHK(wst(ctx, S_PM_MAP, n, &map));
  CHK(wst(ctx, S_PM_SOFF, n + 1, &soff));
  CHK(wst(ctx, S_PM_SIDX, dg.nnz, &sidx));
  CHK(wst(ctx, S_PM_SW, dg.nnz, &sw));
  int64_t sn = 0, snnz = 0;
  CHK(louvain_aggregate(ctx, g, lab, map, soff, 1, sidx, sw, &sn, &snnz, stream));
  lv_graph sg;
  sg.n = sn;
  sg.nnz = snnz;
  sg.offsets = soff;
  sg.indices = sidx;
  sg.weights = sw;
  sg.offsets_64 = 1;
  sg.weights_64 = 1;
  int32_t* m2 = nullptr;
  CHK(wst(ctx, S_PM_M2, sn, &m2));
  lv_params mp = *p;
  mp.flags &= ~LV_VALIDATE;
  CHK(louvain_run(ctx, &sg, &mp, m2, merge_res, stream));
  // final membership: the merge community of every vertex's combined part community
  HIPCHK(hipMemcpyAsync(membership, map, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice,
                        s));
  HIPCHK(lv::compose_membership(membership, n, m2, s));
  HIPCHK(hipStreamSynchronize(s));
  return LV_OK;
}

}  // extern "C"
