// Host-side declarations of the kernel launchers (liblouvain internals).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lv {

// A CSR on the device with int64 offsets (int32 inputs are widened once per call).
struct DevGraph {
  int64_t n = 0, nnz = 0;
  const int64_t* off = nullptr;
  const int32_t* idx = nullptr;
  const void* w = nullptr;
  bool w64 = false;  // weights are uint64 (else uint32)
};

// Rows grouped by (vertex class k, degree class j), list segment 12k + j (12 = kDegClasses).
struct Buckets {
  int classes = 1;
  int64_t count[384] = {0};   // rows per segment
  int64_t arcs[384] = {0};    // arcs per segment
  int64_t lstart[385] = {0};  // first list position per segment (lstart[12K] = total)
};

// Hub (global-table) work decomposition of one pass.
struct HubPlan {
  int64_t nh = 0;             // hub rows
  int64_t chunks = 0;         // accumulation blocks
  int64_t slots = 0;          // table slots (sum of per-row power-of-two sizes)
  int64_t scan_blocks = 0;    // scan blocks
  int64_t* chunk_start = nullptr;  // [nh+1]
  int64_t* tab_start = nullptr;    // [nh+1]
  int64_t* scan_start = nullptr;   // [nh+1]
};

// ---- elementwise / reductions
hipError_t fill_u64(uint64_t* a, uint64_t v, int64_t n, hipStream_t s);
hipError_t fill_i32(int32_t* a, int32_t v, int64_t n, hipStream_t s);
hipError_t fill_i64(int64_t* a, int64_t v, int64_t n, hipStream_t s);
hipError_t iota_i32(int32_t* a, int64_t n, hipStream_t s);
hipError_t copy_i64(int64_t* dst, const int64_t* src, int64_t n, hipStream_t s);
hipError_t widen_offsets(const int32_t* in, int64_t* out, int64_t m, hipStream_t s);
hipError_t narrow_offsets(const int64_t* in, int32_t* out, int64_t m, hipStream_t s);
hipError_t widen_weights(const uint32_t* in, uint64_t* out, int64_t m, hipStream_t s);
// out[0] += sum(a), out[1] = max(out[1], max(a))
hipError_t sum_max_u64(const uint64_t* a, int64_t n, unsigned long long* out, hipStream_t s);
// out[0..1] += sum(a[i]^2) as a 128-bit value
hipError_t sum_squares_u64(const uint64_t* a, int64_t n, unsigned long long* out, hipStream_t s);
// Validation: sets *bad nonzero if an index is out of range, a weight is 0, or offsets
// decrease.
hipError_t validate_graph(const DevGraph& g, unsigned int* bad, hipStream_t s);

// ---- exclusive scans: out[i] = sum_{j<i} x[j], out[n] = total. `partial` needs
// scan_partial_elems(n) int64 entries.
int64_t scan_partial_elems(int64_t n);
hipError_t scan_i64(const int64_t* x, int64_t n, int64_t* out, int64_t* partial, hipStream_t s);
hipError_t scan_flags_pos(const int32_t* x, int64_t n, int64_t* out, int64_t* partial,
                          hipStream_t s);  // counts x[i] > 0

// ---- pass set-up
hipError_t row_sums(const DevGraph& g, uint64_t* K, hipStream_t s);  // K must be zero
hipError_t init_state(int64_t n, const uint64_t* K, int32_t* C, uint64_t* Sig, int32_t* csize,
                      hipStream_t s);
// Classify rows (lengths from offsets, or from `len` if non-null over m items) by vertex
// class (K classes of pass `pass`) and degree class. counts: device scratch of 1536 words;
// host_counts: 1536 pinned words. Host result in `b` (synchronises the stream).
hipError_t bucket_rows(const int64_t* off, const int64_t* len, int64_t m, int K, int pass,
                       int32_t* list, unsigned long long* counts,
                       unsigned long long* host_counts, Buckets& b, hipStream_t s);
// Hub decomposition of the rows hubs[0 .. nh) whose keys take at most `cap` distinct values.
// arrays: 6 * (nh + 1) int64, partial: scan scratch; host_buf: 3 pinned words.
hipError_t plan_hubs(const int64_t* off, const int64_t* len, const int32_t* hubs, int64_t nh,
                     int64_t cap, int64_t* arrays, int64_t* partial,
                     unsigned long long* host_buf, HubPlan& hp, hipStream_t s);

// ---- local-moving iteration
struct MoveBuffers {
  const uint64_t* K = nullptr;
  int32_t* C = nullptr;
  uint64_t* Sig = nullptr;
  int32_t* csize = nullptr;
  uint64_t W = 0;
  const int32_t* list = nullptr;
  int32_t* tgt = nullptr;               // [n] decision of every vertex of the class step
  unsigned long long* block_partial = nullptr;  // 4 words per block of the LDS move kernel
  // per class step, 8 words: [0..1] S, [2] moved, [3] candidates, [4] LDS-kernel candidates,
  // [5] LDS-kernel moves
  unsigned long long* stats = nullptr;
  int32_t* tkeys = nullptr;             // hub tables
  void* tvals = nullptr;
  int32_t* occ = nullptr;
  int32_t* occ_count = nullptr;
  unsigned long long* partial = nullptr;  // hub scan partials: 5 words per scan block
  int hub_first = 10;                     // first degree class on the global-table path
};

// First degree class that takes the global-table path, given the largest LDS allocation a
// workgroup may make and the table value width (wide: 8-byte values).
int hub_first_class(size_t max_lds_per_block, bool wide);
hipError_t zero_words(unsigned long long* a, int64_t n, hipStream_t s);
// LDS-table move kernel over the rows of vertex class `cls`.
hipError_t move_lds(const DevGraph& g, const Buckets& b, int cls, const MoveBuffers& m,
                    bool wide, hipStream_t s);
hipError_t hub_reset_tables(const HubPlan& hp, const MoveBuffers& m, bool wide, hipStream_t s);
// Hub kernels over the hub rows of vertex class `cls` (plan hp made for those rows).
hipError_t move_hubs(const DevGraph& g, const Buckets& b, int cls, const HubPlan& hp,
                     const MoveBuffers& m, bool wide, hipStream_t s);
hipError_t apply_moves(const Buckets& b, int cls, const MoveBuffers& m, hipStream_t s);
// Block records the LDS move kernels of class cls write (sizes block_partial).
int64_t move_lds_blocks(const Buckets& b, int cls, int hub_first);

// ---- modularity pieces
// out[0] += sum of w over arcs (r, j) with C[r] == C[j] (C == nullptr: r == j, i.e. loops)
hipError_t intra_weight(const DevGraph& g, const int32_t* C, unsigned long long* out,
                        hipStream_t s);
hipError_t sigma_by_label(const uint64_t* K, const int32_t* C, int64_t n, uint64_t* Sig,
                          hipStream_t s);  // Sig zeroed; Sig[C[i]] += K[i]
hipError_t count_labels(const int32_t* C, int64_t n, int32_t* csize, hipStream_t s);  // zeroed

// ---- aggregation
struct AggBuffers {
  // per label (n entries unless noted)
  int64_t* A = nullptr;        // arcs per label [n+1] (scanned in place to starts)
  int64_t* astart = nullptr;   // [n+1]
  int64_t* newid = nullptr;    // [n+1] exclusive rank of used labels
  int64_t* cursor = nullptr;   // [n]
  int32_t* oldlabel = nullptr; // [n] label of each new id
  int64_t* dcount = nullptr;   // [n+1] distinct neighbours per new id, scanned to offsets
  int64_t* abase = nullptr;    // [n] per vertex
  int32_t* tkey = nullptr;     // [nnz]
  uint64_t* tw = nullptr;      // [nnz]
  int32_t* list = nullptr;     // [n]
  int64_t* partial = nullptr;  // scan scratch
  unsigned long long* counts = nullptr;  // 32 words
  unsigned long long* stats = nullptr;   // [0] self-loop weight total
  unsigned long long* block_partial = nullptr;  // 1 word per block of the LDS merge kernel
  int64_t* hub_arrays = nullptr;         // 6 * (hubs + 1)
  int32_t* tkeys = nullptr;              // global tables (sized by caller from plan)
  unsigned long long* tvals = nullptr;
  int32_t* occ = nullptr;
  int32_t* occ_count = nullptr;          // [n]
};
hipError_t label_arcs(const int64_t* off, const int32_t* C, int64_t n, int64_t* A,
                      hipStream_t s);
hipError_t label_tables(int64_t n, const int32_t* csize, const int64_t* newid,
                        const uint64_t* Sig, int32_t* oldlabel, uint64_t* Kp, hipStream_t s);
hipError_t vertex_map(const int64_t* off, const int32_t* C, int64_t n, const int64_t* newid,
                      int64_t* cursor, int32_t* map, int64_t* abase, hipStream_t s);
hipError_t scatter_arcs(const DevGraph& g, const int32_t* map, const int64_t* abase,
                        int32_t* tkey, uint64_t* tw, hipStream_t s);
hipError_t merge_lds(const Buckets& b, const AggBuffers& a, hipStream_t s);
int64_t merge_lds_blocks(const Buckets& b);  // sizes block_partial
hipError_t merge_hubs(const Buckets& b, const HubPlan& hp, const AggBuffers& a, hipStream_t s);
hipError_t compact_rows(const int64_t* offp, int64_t np, int64_t nnzp, const int32_t* oldlabel,
                        const int64_t* astart, const int32_t* tkey, const uint64_t* tw,
                        int32_t* idx_out, uint64_t* w_out, hipStream_t s);
hipError_t compose_membership(int32_t* top, int64_t n, const int32_t* map, hipStream_t s);

}  // namespace lv
