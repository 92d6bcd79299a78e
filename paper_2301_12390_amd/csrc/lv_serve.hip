// Request server of liblouvain: continuous batching of independent graphs (whole runs of the
// method of section 3.2 of Sahu, arXiv 2301.12390) over one device. Slots, each a host thread
// with its own context and stream, take the head of a shared queue, pack it into one CSR on the
// device and run it with louvain_run_batched; device memory is admitted against a budget.
// The contract is in include/louvain.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/louvain.h"
#include "lv_device.h"
#include "lv_internal.h"

namespace {

constexpr int kMaxSlots = 16;
constexpr int64_t kMaxBatchGraphs = 1 << 16;
constexpr int64_t kMaxPackedVertices = ((int64_t)1 << 31) - 2;

// Upper bound of the device bytes a slot holds after a run whose largest batch so far had N
// vertices, A arcs and G graphs: its packing buffers (exact, page-rounded) and the context's
// workspace. The workspace terms bound what the drivers allocate: the input widened to int64
// offsets, the vertex state and super-vertex graphs (double-buffered), the aggregation's
// sort keys and per-graph words, each grown with 1/8 headroom.
uint64_t slot_bound(int64_t N, int64_t A, int64_t G) {
  const uint64_t n = (uint64_t)N + 1, a = (uint64_t)A + 1, g = (uint64_t)G + 1;
  const uint64_t own = 20 * n + 8 * a + 56 * g + 6 * 4096;
  const uint64_t work = 320 * n + 72 * a + 640 * g + ((uint64_t)48 << 20);
  return own + work;
}

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Largest g in [0, G) with bounds[g] <= x (bounds non-decreasing from 0, x < bounds[G]).
__device__ __forceinline__ int32_t graph_of(const int64_t* bounds, int32_t G, int64_t x) {
  int32_t lo = 0, hi = G - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (bounds[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

struct PackMeta {
  const int64_t* vptr;   // [G+1] first packed vertex of every request
  const int64_t* aptr;   // [G+1] first packed arc
  const int64_t* rawb;   // [G] byte offset of the request's offsets in the staging area
  const int32_t* wide;   // [G] offsets are int64
  int32_t* bad;          // [G] out: 1 bad offsets, 2 bad neighbour or weight
  int32_t G;
};

__device__ __forceinline__ int64_t raw_offset(const unsigned char* raw, const PackMeta& m,
                                              int32_t g, int64_t i) {
  const unsigned char* p = raw + m.rawb[g];
  return m.wide[g] ? ((const int64_t*)p)[i] : (int64_t)((const int32_t*)p)[i];
}

// Packs the requests' CSRs (copied verbatim: offsets into the staging area, neighbours and
// weights at their packed arc positions) into one CSR with consecutive vertex ids: offsets
// shifted by the request's first arc, neighbours by its first vertex. Checks every request on
// the way; a request flagged bad is not run, so its partly shifted arrays do not matter.
__global__ __launch_bounds__(lv::kBlock) void k_srv_pack(const unsigned char* raw, PackMeta m,
                                                        int64_t N, int64_t A, int64_t* off,
                                                        int32_t* idx, const uint32_t* w) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t items = N > A ? N : A;
  for (int64_t x = tid; x < items; x += stride) {
    if (x < N) {
      const int32_t g = graph_of(m.vptr, m.G, x);
      const int64_t local = x - m.vptr[g];
      const int64_t ng = m.vptr[g + 1] - m.vptr[g];
      const int64_t ag = m.aptr[g + 1] - m.aptr[g];
      const int64_t o0 = raw_offset(raw, m, g, local);
      const int64_t o1 = raw_offset(raw, m, g, local + 1);
      const bool ok = o0 >= 0 && o0 <= o1 && o1 <= ag && (local != 0 || o0 == 0) &&
                      (local != ng - 1 || o1 == ag);
      if (!ok) atomicOr(&m.bad[g], 1);
      off[x] = m.aptr[g] + o0;
    }
    if (x < A) {
      const int32_t g = graph_of(m.aptr, m.G, x);
      const int64_t ng = m.vptr[g + 1] - m.vptr[g];
      const int64_t j = idx[x];
      if (j < 0 || j >= ng || w[x] == 0u)
        atomicOr(&m.bad[g], 2);
      else
        idx[x] = (int32_t)(j + m.vptr[g]);
    }
  }
  if (tid == 0) off[N] = A;
}

struct Request {
  uint64_t ticket = 0;
  lv_graph g{};
  int32_t* out = nullptr;
  bool done = false;
  bool waited = false;  // a thread is waiting for it
  lv_request_result res{};
};

void set_error(Request* r, lv_status st, const std::string& msg) {
  r->res.status = st;
  snprintf(r->res.error, sizeof(r->res.error), "%s", msg.c_str());
}

// Grow-only device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Slot {
  int index = 0;
  lv_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  DevBuf raw, off, idx, w, memb, meta;
  void* pin = nullptr;  // pinned host copy of the packing metadata and the bad flags
  size_t pin_bytes = 0;
  lv_result* single = nullptr;  // result of a request run alone
  std::vector<lv_graph_result> per_graph;
  int64_t hwN = 0, hwA = 0, hwG = 0;  // largest batch so far (buffers are grow-only)
  uint64_t reserved = 0;              // bytes this slot is admitted to hold
  uint64_t held = 0;                  // bytes it held after its last run
  std::thread thread;
};

}  // namespace

struct lv_server {
  int device = 0;
  lv_server_config cfg{};
  std::mutex mu;
  std::condition_variable cv;       // slots: work, memory or shutdown
  std::condition_variable cv_done;  // waiters: a request completed
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, Request*> requests;
  uint64_t next_ticket = 1;
  bool stopping = false;
  int mem_waiters = 0;
  int running = 0;
  int64_t run_seq = 0;  // runs admitted so far
  uint64_t committed = 0;
  uint64_t held_total = 0;
  lv_server_stats stats{};
  std::vector<Slot*> slots;
};

namespace {

bool budget_ok(const lv_server* S, uint64_t others, uint64_t need) {
  return S->cfg.hbm_budget_bytes == 0 || others + need <= S->cfg.hbm_budget_bytes;
}

uint64_t slot_need(const Slot* s, int64_t N, int64_t A, int64_t G) {
  return slot_bound(std::max(s->hwN, N), std::max(s->hwA, A), std::max(s->hwG, G));
}

lv_status grow(DevBuf& b, size_t bytes) {
  bytes = (std::max<size_t>(bytes, 8) + 4095) & ~(size_t)4095;
  if (b.bytes >= bytes) return LV_OK;
  if (b.p && hipFree(b.p) != hipSuccess) return LV_EHIP;
  b.p = nullptr;
  b.bytes = 0;
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return LV_ENOMEM;
  }
  b.bytes = bytes;
  return LV_OK;
}

void release(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

uint64_t own_bytes(const Slot* s) {
  return s->raw.bytes + s->off.bytes + s->idx.bytes + s->w.bytes + s->memb.bytes + s->meta.bytes;
}

// Frees the slot's device memory (packing buffers and context workspace). Called with the
// lock held; releases it around the HIP calls.
void trim(lv_server* S, Slot* s, std::unique_lock<std::mutex>& lk) {
  lk.unlock();
  release(s->raw);
  release(s->off);
  release(s->idx);
  release(s->w);
  release(s->memb);
  release(s->meta);
  if (s->ctx) louvain_ctx_destroy(s->ctx);
  s->ctx = nullptr;
  if (louvain_ctx_create(S->device, 0, &s->ctx) != LV_OK) s->ctx = nullptr;
  lk.lock();
  S->committed -= s->reserved;
  S->held_total -= s->held;
  s->reserved = 0;
  s->held = 0;
  s->hwN = s->hwA = s->hwG = 0;
  S->stats.trims++;
  S->cv.notify_all();
}

void finish(lv_server* S, Request* r) {
  r->done = true;
  S->stats.completed++;
  if (r->res.status != LV_OK) S->stats.failed++;
}

// Takes the head of the queue and the requests behind it that fit the run (arcs, vertices and
// memory). Called with the lock held and a non-empty queue. A head that cannot fit the budget
// even alone completes with LV_EBUDGET and the batch comes back empty.
void take_batch(lv_server* S, Slot* s, std::vector<Request*>& batch) {
  Request* h = S->queue.front();
  S->queue.pop_front();
  const uint64_t alone = slot_bound(h->g.n, h->g.nnz, 1);
  if (!budget_ok(S, 0, alone)) {
    set_error(h, LV_EBUDGET, "request needs up to " + std::to_string(alone) +
                                 " bytes of device memory; the budget is " +
                                 std::to_string(S->cfg.hbm_budget_bytes));
    finish(S, h);
    S->cv_done.notify_all();
    return;
  }
  batch.push_back(h);
  int64_t N = h->g.n, A = h->g.nnz;
  const uint64_t others = S->committed - s->reserved;
  while (!S->queue.empty() && S->cfg.batch_arcs > 0 && (int64_t)batch.size() < kMaxBatchGraphs) {
    const Request* r = S->queue.front();
    if (A + r->g.nnz > S->cfg.batch_arcs || N + r->g.n > kMaxPackedVertices) break;
    if (!budget_ok(S, others, slot_need(s, N + r->g.n, A + r->g.nnz, (int64_t)batch.size() + 1)))
      break;
    batch.push_back(S->queue.front());
    S->queue.pop_front();
    N += r->g.n;
    A += r->g.nnz;
  }
}

// One run of a batch on slot s (no lock held); false if nothing ran. Fills the results of the
// requests in `batch` on return. When some requests fail the packing checks, only those stay in
// `batch` (with LV_EINVAL) and the others go to `again`, to be queued again.
bool run_batch(lv_server* S, Slot* s, int64_t seq, std::vector<Request*>& batch,
               std::vector<Request*>& again) {
  const int32_t G = (int32_t)batch.size();
  const int64_t t0 = now_ns();
  std::vector<int64_t> vptr(G + 1, 0), aptr(G + 1, 0), rawb(G, 0);
  for (int32_t k = 0; k < G; k++) {
    const lv_graph& g = batch[k]->g;
    vptr[k + 1] = vptr[k] + g.n;
    aptr[k + 1] = aptr[k] + g.nnz;
  }
  int64_t rawbytes = 0;
  for (int32_t k = 0; k < G; k++) {
    rawb[k] = rawbytes;
    const lv_graph& g = batch[k]->g;
    rawbytes += ((g.n + 1) * (g.offsets_64 ? 8 : 4) + 7) & ~(int64_t)7;
  }
  const int64_t N = vptr[G], A = aptr[G];
  auto fail_all = [&](lv_status st, const std::string& msg) {
    for (Request* r : batch) {
      set_error(r, st, msg);
      r->res.slot = s->index;
      r->res.start_ns = t0;
      r->res.done_ns = now_ns();
    }
    return false;
  };
  if (!s->ctx && louvain_ctx_create(S->device, 0, &s->ctx) != LV_OK) {
    s->ctx = nullptr;  // tried again by the slot's next run
    return fail_all(LV_EHIP, "the slot's context could not be created");
  }
  if (S->cfg.fail_run > 0 && seq == S->cfg.fail_run)
    return fail_all(LV_ENOMEM, "injected failure of run " + std::to_string(seq));
  const size_t meta_bytes = (size_t)(3 * G + 2) * 8 + (size_t)(2 * G) * 4;
  if (grow(s->raw, (size_t)rawbytes) != LV_OK || grow(s->off, (size_t)(N + 1) * 8) != LV_OK ||
      grow(s->idx, (size_t)A * 4) != LV_OK || grow(s->w, (size_t)A * 4) != LV_OK ||
      grow(s->memb, (size_t)std::max<int64_t>(N, 1) * 4) != LV_OK ||
      grow(s->meta, meta_bytes) != LV_OK)
    return fail_all(LV_ENOMEM, "device allocation of the packing buffers failed");
  if (s->pin_bytes < meta_bytes) {
    if (s->pin) (void)hipHostFree(s->pin);
    s->pin = nullptr;
    s->pin_bytes = 0;
    if (hipHostMalloc(&s->pin, meta_bytes, hipHostMallocDefault) != hipSuccess) {
      s->pin = nullptr;
      return fail_all(LV_EHIP, "hipHostMalloc of the packing metadata failed");
    }
    s->pin_bytes = meta_bytes;
  }
  int64_t* hm = (int64_t*)s->pin;
  memcpy(hm, vptr.data(), (G + 1) * 8);
  memcpy(hm + G + 1, aptr.data(), (G + 1) * 8);
  memcpy(hm + 2 * G + 2, rawb.data(), G * 8);
  int32_t* hw = (int32_t*)(hm + 3 * G + 2);
  for (int32_t k = 0; k < G; k++) {
    hw[k] = batch[k]->g.offsets_64 ? 1 : 0;
    hw[G + k] = 0;
  }
  hipStream_t st = s->stream;
  unsigned char* raw = (unsigned char*)s->raw.p;
  int32_t* idx = (int32_t*)s->idx.p;
  uint32_t* w = (uint32_t*)s->w.p;
  int64_t* dm = (int64_t*)s->meta.p;
  bool ok = hipMemcpyAsync(dm, hm, meta_bytes, hipMemcpyHostToDevice, st) == hipSuccess;
  for (int32_t k = 0; k < G && ok; k++) {
    const lv_graph& g = batch[k]->g;
    if (g.n > 0)
      ok = hipMemcpyAsync(raw + rawb[k], g.offsets, (g.n + 1) * (g.offsets_64 ? 8 : 4),
                          hipMemcpyHostToDevice, st) == hipSuccess;
    if (ok && g.nnz > 0)
      ok = hipMemcpyAsync(idx + aptr[k], g.indices, g.nnz * 4, hipMemcpyHostToDevice, st) ==
               hipSuccess &&
           hipMemcpyAsync(w + aptr[k], g.weights, g.nnz * 4, hipMemcpyHostToDevice, st) ==
               hipSuccess;
  }
  if (!ok) return fail_all(LV_EHIP, "copy of the request graphs to the device failed");
  PackMeta m;
  m.vptr = dm;
  m.aptr = dm + G + 1;
  m.rawb = dm + 2 * G + 2;
  m.wide = (const int32_t*)(dm + 3 * G + 2);
  m.bad = (int32_t*)(dm + 3 * G + 2) + G;
  m.G = G;
  int64_t blocks = (std::max(N, A) + lv::kBlock - 1) / lv::kBlock;
  blocks = std::min<int64_t>(std::max<int64_t>(blocks, 1), 16384);
  hipLaunchKernelGGL(k_srv_pack, dim3((unsigned)blocks), dim3(lv::kBlock), 0, st, raw, m, N, A,
                     (int64_t*)s->off.p, idx, w);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(hw + G, m.bad, G * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail_all(LV_EHIP, "packing the request graphs failed");
  bool any_bad = false;
  for (int32_t k = 0; k < G; k++) any_bad |= hw[G + k] != 0;
  if (any_bad) {
    std::vector<Request*> bad;
    for (int32_t k = 0; k < G; k++) {
      Request* r = batch[k];
      if (hw[G + k] == 0) {
        again.push_back(r);
        continue;
      }
      set_error(r, LV_EINVAL, (hw[G + k] & 1) ? "offsets are not a CSR of nnz arcs"
                                             : "a neighbour outside [0, n) or a zero weight");
      r->res.slot = s->index;
      r->res.start_ns = t0;
      r->res.done_ns = now_ns();
      bad.push_back(r);
    }
    batch.swap(bad);
    return false;
  }

  lv_graph pg;
  pg.n = N;
  pg.nnz = A;
  pg.offsets = s->off.p;
  pg.indices = idx;
  pg.weights = w;
  pg.offsets_64 = 1;
  pg.weights_64 = 0;
  lv_params p = S->cfg.params;
  p.flags &= ~LV_TRACE;
  int32_t* memb = (int32_t*)s->memb.p;
  lv_status rs;
  if (G == 1) {
    rs = louvain_run(s->ctx, &pg, &p, memb, s->single, st);
    if (rs == LV_OK) {
      const lv_result& r = *s->single;
      lv_graph_result& gr = s->per_graph[0];
      memset(&gr, 0, sizeof(gr));
      gr.passes = r.passes;
      gr.iterations_total = r.iterations_total;
      for (int i = 0; i < r.passes && i < LV_MAX_PASSES; i++) gr.iterations[i] = r.iterations[i];
      gr.cap_hits = (uint32_t)r.cap_hits;
      gr.n_communities = r.n_communities;
      gr.W = r.W;
      gr.q_num = r.q_num;
      gr.q = r.q;
    }
  } else {
    rs = louvain_run_batched(s->ctx, &pg, G, vptr.data(), aptr.data(), &p, memb,
                             s->per_graph.data(), st);
  }
  if (rs != LV_OK) return fail_all(rs, louvain_last_error(s->ctx));
  ok = true;
  for (int32_t k = 0; k < G && ok; k++)
    if (batch[k]->g.n > 0)
      ok = hipMemcpyAsync(batch[k]->out, memb + vptr[k], batch[k]->g.n * 4,
                          hipMemcpyDeviceToHost, st) == hipSuccess;
  if (!ok || hipStreamSynchronize(st) != hipSuccess)
    return fail_all(LV_EHIP, "copy of the memberships to the host failed");
  const int64_t t1 = now_ns();
  for (int32_t k = 0; k < G; k++) {
    Request* r = batch[k];
    r->res.status = LV_OK;
    r->res.error[0] = 0;
    r->res.slot = s->index;
    r->res.batch_graphs = G;
    r->res.batch_arcs = A;
    r->res.start_ns = t0;
    r->res.done_ns = t1;
    r->res.result = s->per_graph[k];
  }
  return true;
}

void worker(lv_server* S, Slot* s) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    S->cv.wait(lk, [&] {
      return S->stopping || (S->mem_waiters > 0 && s->reserved > 0) ||
             (!S->queue.empty() && S->mem_waiters == 0);
    });
    if (S->stopping) break;
    if (S->mem_waiters > 0 && s->reserved > 0) {
      trim(S, s, lk);
      continue;
    }
    std::vector<Request*> batch;
    take_batch(S, s, batch);
    if (batch.empty()) continue;
    int64_t N = 0, A = 0;
    for (const Request* r : batch) {
      N += r->g.n;
      A += r->g.nnz;
    }
    const int64_t G = (int64_t)batch.size();
    // admission: the slot's bound after this run, against what the other slots hold
    bool cancelled = false;
    for (;;) {
      const uint64_t need = slot_need(s, N, A, G);
      if (budget_ok(S, S->committed - s->reserved, need)) {
        S->committed = S->committed - s->reserved + need;
        s->reserved = need;
        break;
      }
      if (s->reserved > 0) {  // start from an empty slot before waiting for the others
        trim(S, s, lk);
        continue;
      }
      S->mem_waiters++;
      S->cv.notify_all();
      S->cv.wait(lk, [&] {
        return S->stopping || budget_ok(S, S->committed, slot_need(s, N, A, G));
      });
      S->mem_waiters--;
      S->cv.notify_all();  // the other slots may take work again
      if (S->stopping) {
        cancelled = true;
        break;
      }
    }
    if (cancelled) {
      for (Request* r : batch) {
        set_error(r, LV_ECANCELLED, "the server was destroyed");
        finish(S, r);
      }
      S->cv_done.notify_all();
      break;
    }
    s->hwN = std::max(s->hwN, N);
    s->hwA = std::max(s->hwA, A);
    s->hwG = std::max(s->hwG, G);
    if ((int64_t)s->per_graph.size() < G) s->per_graph.resize(G);
    S->stats.peak_committed_bytes = std::max(S->stats.peak_committed_bytes, S->committed);
    S->running++;
    S->stats.peak_running = std::max(S->stats.peak_running, S->running);
    const int64_t seq = ++S->run_seq;
    lk.unlock();
    std::vector<Request*> again;
    const bool ran = run_batch(S, s, seq, batch, again);
    const uint64_t held = own_bytes(s) + (s->ctx ? louvain_workspace_bytes(s->ctx) : 0);
    lk.lock();
    S->running--;
    if (ran) {
      S->stats.runs++;
      if (batch.size() > 1) S->stats.batched_requests += (int64_t)batch.size();
    }
    S->held_total = S->held_total - s->held + held;
    s->held = held;
    S->stats.peak_held_bytes = std::max(S->stats.peak_held_bytes, S->held_total);
    if (held > s->reserved) {  // keep the accounting true if the bound was exceeded
      S->stats.bound_misses++;
      S->committed += held - s->reserved;
      s->reserved = held;
    }
    for (auto it = again.rbegin(); it != again.rend(); ++it) S->queue.push_front(*it);
    for (Request* r : batch) finish(S, r);
    S->cv_done.notify_all();
    S->cv.notify_all();
  }
}

void destroy_slot(Slot* s) {
  release(s->raw);
  release(s->off);
  release(s->idx);
  release(s->w);
  release(s->memb);
  release(s->meta);
  if (s->ctx) louvain_ctx_destroy(s->ctx);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  if (s->pin) (void)hipHostFree(s->pin);
  delete s->single;
  delete s;
}

}  // namespace

extern "C" {

int64_t louvain_server_clock_ns(void) { return now_ns(); }

lv_status louvain_server_create(int device, const lv_server_config* cfg, lv_server** out) {
  if (!out) return LV_EINVAL;
  *out = nullptr;
  if (!cfg || cfg->slots < 1 || cfg->slots > kMaxSlots || cfg->batch_arcs < 0) return LV_EINVAL;
  if (lv::params_error(&cfg->params)) return LV_EINVAL;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return LV_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return LV_EHIP;
  lv_server* S = new lv_server();
  S->device = device;
  S->cfg = *cfg;
  S->stats.slots = cfg->slots;
  for (int i = 0; i < cfg->slots; i++) {
    Slot* s = new Slot();
    s->index = i;
    s->single = new lv_result();
    s->per_graph.resize(1);
    S->slots.push_back(s);
    if (louvain_ctx_create(device, 0, &s->ctx) != LV_OK ||
        hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
      for (Slot* t : S->slots) destroy_slot(t);
      delete S;
      return LV_EHIP;
    }
  }
  for (Slot* s : S->slots) s->thread = std::thread(worker, S, s);
  *out = S;
  return LV_OK;
}

void louvain_server_destroy(lv_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
    for (Request* r : S->queue) {
      set_error(r, LV_ECANCELLED, "the server was destroyed");
      finish(S, r);
    }
    S->queue.clear();
    S->cv.notify_all();
    S->cv_done.notify_all();
  }
  for (Slot* s : S->slots)
    if (s->thread.joinable()) s->thread.join();
  (void)hipSetDevice(S->device);
  for (Slot* s : S->slots) destroy_slot(s);
  for (auto& kv : S->requests) delete kv.second;
  delete S;
}

lv_status louvain_server_submit(lv_server* S, const lv_graph* g, int32_t* membership,
                                uint64_t* ticket) {
  if (!S || !g || !ticket) return LV_EINVAL;
  if (g->n < 0 || g->n >= ((int64_t)1 << 31) || g->nnz < 0) return LV_EINVAL;
  if (g->n == 0 && g->nnz > 0) return LV_EINVAL;
  if (g->weights_64) return LV_EINVAL;
  if (!g->offsets_64 && g->nnz >= ((int64_t)1 << 31)) return LV_EINVAL;
  if (g->n > 0 && (!g->offsets || !membership)) return LV_EINVAL;
  if (g->nnz > 0 && (!g->indices || !g->weights)) return LV_EINVAL;
  Request* r = new Request();
  r->g = *g;
  r->out = membership;
  r->res.slot = -1;
  r->res.submit_ns = now_ns();
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stopping) {
    delete r;
    return LV_ECANCELLED;
  }
  r->ticket = S->next_ticket++;
  S->requests[r->ticket] = r;
  S->queue.push_back(r);
  S->stats.submitted++;
  *ticket = r->ticket;
  S->cv.notify_all();
  return LV_OK;
}

lv_status louvain_server_wait(lv_server* S, uint64_t ticket, int64_t timeout_ms,
                              lv_request_result* out) {
  if (!S || !out) return LV_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->requests.find(ticket);
  if (it == S->requests.end()) return LV_EINVAL;
  Request* r = it->second;
  if (r->waited) return LV_EINVAL;  // one waiter per ticket
  r->waited = true;
  if (timeout_ms < 0) {
    S->cv_done.wait(lk, [&] { return r->done; });
  } else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                                  [&] { return r->done; })) {
    r->waited = false;
    return LV_ETIMEOUT;
  }
  *out = r->res;
  S->requests.erase(ticket);
  delete r;
  return LV_OK;
}

lv_status louvain_server_cancel(lv_server* S, uint64_t ticket, int32_t* cancelled) {
  if (cancelled) *cancelled = 0;
  if (!S) return LV_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->requests.find(ticket);
  if (it == S->requests.end()) return LV_EINVAL;
  Request* r = it->second;
  auto q = std::find(S->queue.begin(), S->queue.end(), r);
  if (q == S->queue.end()) return LV_OK;  // running or done
  S->queue.erase(q);
  set_error(r, LV_ECANCELLED, "cancelled before it ran");
  finish(S, r);
  S->cv_done.notify_all();
  if (cancelled) *cancelled = 1;
  return LV_OK;
}

lv_status louvain_server_stats(lv_server* S, lv_server_stats* out) {
  if (!S || !out) return LV_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->stats;
  out->committed_bytes = S->committed;
  return LV_OK;
}

}  // extern "C"
