// Host-side declarations of the kernel launchers (liblouvain internals).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/louvain.h"

namespace lv {

// Why a parameter set is invalid, or nullptr if it is valid.
const char* params_error(const lv_params* p);

// Context accessors for entry points outside lv_api.hip.
int ctx_device(const lv_ctx* ctx);
void ctx_set_error(lv_ctx* ctx, const char* msg);
unsigned long long* ctx_pinned_words(lv_ctx* ctx);  // 16 pinned host words of the context

// The fixed device array of louvain_modularity_noalloc (lv_noalloc.hip): noalloc_setup looks up
// the current device's copy once (call with `device` current); noalloc_scratch returns it.
hipError_t noalloc_setup(int device);
void* noalloc_scratch(int device);

// A graph on the device: row v spans arcs [rs[v], re[v]) of idx/w. For a CSR, rs = off and
// re = off + 1 (off has n+1 int64 entries; int32 inputs are widened once per call) and `off`
// is set; super-vertex graphs keep rows where the aggregation wrote them (off is null).
struct DevGraph {
  int64_t n = 0, nnz = 0;          // vertices, arcs
  const int64_t* rs = nullptr;
  const int64_t* re = nullptr;
  const int64_t* off = nullptr;    // contiguous CSR offsets, or null
  const int32_t* idx = nullptr;
  const void* w = nullptr;
  bool w64 = false;  // weights are uint64 (else uint32)
};

// A batch of graphs packed with consecutive vertex ids, each with its own W and iteration state
// (gid null: a single graph, whose W is passed separately).
constexpr int kGainSlices = 32;  // copies of the per-graph gain sums (power of two)
struct GraphSet {
  int64_t G = 0;
  const int32_t* gid = nullptr;       // [n] graph of every vertex
  const int64_t* gbase = nullptr;     // [G+1] first vertex of every graph
  const uint64_t* Wg = nullptr;       // [G] total weight
  const uint8_t* act = nullptr;       // [G] graphs iterating in this phase
  unsigned long long* gS = nullptr;   // [kGainSlices][2G] gain sums of the iteration per graph
                                      // (128-bit), folded into the first copy after it
  unsigned long long* gself = nullptr;  // [G] weight of self super-arcs made by an aggregation
};

// Rows grouped by (vertex class k, degree class j), list segment 12k + j (12 = kDegClasses).
struct Buckets {
  int classes = 1;
  int64_t count[384] = {0};   // rows per segment
  int64_t arcs[384] = {0};    // arcs per segment
  int64_t lstart[385] = {0};  // first list position per segment (lstart[12K] = total)
};

// Two-phase decomposition of the long items of one launch (see part_chunk in lv_device.h).
struct PartPlan {
  int64_t nh = 0;             // items
  int vb = 4;                 // value bytes (4 or 8)
  int shift = 0;              // partitions sized for (table / 2) >> shift keys (testing: > 0)
  int64_t chunks = 0;         // chunk rows (one pair region of part_chunk(vb) and bound row each)
  int64_t blocks = 0;         // phase-1 workgroups
  int64_t parts = 0;          // phase-2 workgroups
  int64_t hoff_entries = 0;   // segment bounds
  int64_t* rper = nullptr;         // [nh] chunks per phase-1 workgroup
  int64_t* nparts = nullptr;       // [nh] partitions per item
  int64_t* chunk_start = nullptr;  // [nh+1]
  int64_t* block_start = nullptr;  // [nh+1]
  int64_t* part_start = nullptr;   // [nh+1]
  int64_t* hoff_start = nullptr;   // [nh+1]
};
constexpr int64_t kPlanWords = 10;  // plan arrays: kPlanWords * (nh + 1) int64

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
// out[0..1] += sum of all arc weights of g as a 128-bit value
hipError_t total_weight_u128(const DevGraph& g, unsigned long long* out, hipStream_t s);
// Validation: sets *bad nonzero if an index is out of range, a weight is 0, or offsets
// decrease.
hipError_t validate_graph(const DevGraph& g, unsigned int* bad, hipStream_t s);

// ---- exclusive scans: out[i] = sum_{j<i} x[j], out[n] = total. `partial` needs
// scan_partial_elems(n) int64 entries.
int64_t scan_partial_elems(int64_t n);
hipError_t scan_i64(const int64_t* x, int64_t n, int64_t* out, int64_t* partial, hipStream_t s);
hipError_t scan_i32(const int32_t* x, int64_t n, int64_t* out, int64_t* partial, hipStream_t s);
hipError_t scan_flags_pos(const int32_t* x, int64_t n, int64_t* out, int64_t* partial,
                          hipStream_t s);  // counts x[i] > 0

// ---- pass set-up
// K must be zero; tile_rows: row_sum_tiles(g.nnz) + 1 words of scratch. selfw (zeroed, or
// null): per row, the weight of its self-loops.
hipError_t row_sums(const DevGraph& g, uint64_t* K, int64_t* tile_rows, hipStream_t s,
                    uint64_t* selfw = nullptr);
int64_t row_sum_tiles(int64_t nnz);
// Community state as 16-byte records {C[x], csize[x], Sigma[x]} (see lv_device.h).
constexpr size_t kRecBytes = 16;
hipError_t init_state(int64_t n, const uint64_t* K, void* rec, int32_t* lab, hipStream_t s);
hipError_t pack_state(int64_t n, const int32_t* C, const uint64_t* Sig, const int32_t* csize,
                      void* rec, hipStream_t s);
hipError_t unpack_state(int64_t n, const void* rec, int32_t* C, uint64_t* Sig, int32_t* csize,
                        hipStream_t s);
// Classify rows (lengths from offsets, or from `len` if non-null over m items) by vertex
// class (K classes of pass `pass`, hashing ids local to their graph when gid is given) and
// degree class; with act, rows of graphs g with act[g] == 0 are left out. counts: device scratch of 1536 words;
// host_counts: 1536 pinned words. Host result in `b` (synchronises the stream).
hipError_t bucket_rows(const int64_t* rs, const int64_t* re, const int64_t* len, int64_t m,
                       int K, int pass, const int32_t* gid, const int64_t* gbase,
                       const uint8_t* act, const uint8_t* vclass, int32_t* list,
                       unsigned long long* counts, unsigned long long* host_counts, Buckets& b,
                       hipStream_t s);
// Two-phase plans of K <= 32 item lists in one launch and one read-back. List k holds the items
// items[k][0 .. nh[k]) (lengths from rs/re, or len[item]) whose keys take at most `cap`
// distinct values; vb: value bytes; merge: one-chunk items need no phase 2. arrays[k]:
// kPlanWords * (nh[k] + 1) int64; totals: 4 * K device words; host_buf: 4 * K pinned words.
// Synchronises the stream. shift > 0 (testing) divides the partition size by 2^shift and caps
// the phase-2 tables so that partitions take several rounds.
hipError_t plan_parts_batch(const int64_t* rs, const int64_t* re, const int64_t* len,
                            const int32_t* const* items, const int64_t* nh, int K, int64_t cap,
                            int vb, bool merge, int shift, int64_t* const* arrays,
                            int64_t* totals, unsigned long long* host_buf, PartPlan* pp,
                            hipStream_t s);

// ---- local-moving iteration
struct MoveBuffers {
  const uint64_t* K = nullptr;
  void* rec = nullptr;                  // [n] community state records
  int32_t* lab = nullptr;               // [n] copy of every record's community, or null
                                        //   (graphs of up to kLabMaxVertices vertices)
  uint64_t W = 0;
  const int32_t* list = nullptr;
  int32_t* tgt = nullptr;               // [n] class-step decisions, by list position
  unsigned long long* block_partial = nullptr;  // 4 words per block of the LDS move kernel
  // per class step, 8 words: [0..1] S, [2] moved, [3] candidates, [4] candidates of the fused
  // kernel, [5] candidates of the workgroup kernel
  unsigned long long* stats = nullptr;
  int32_t* pk = nullptr;                // hub phase-1 pairs (keys, values of the gain width)
  void* pv = nullptr;
  int32_t* hoff = nullptr;              // hub segment bounds
  int32_t* nflush = nullptr;            // table flushes of every hub phase-1 workgroup
  unsigned long long* partial = nullptr;  // hub phase-2 partials: 5 words per workgroup
  int hub_first = 10;                     // first degree class on the two-phase hub path
  GraphSet gs;                            // batch of graphs, if any
};

// Largest graph whose move kernels read neighbour communities from a 4-byte copy (8 MiB) instead
// of the 16-byte records: larger copies no longer stay in the caches, and measured slower
// (R-MAT s22's pass 0, 4.2M vertices: 22.8 against 22.6 ms per run; s25's pass 0 slower too).
constexpr int64_t kLabMaxVertices = (int64_t)1 << 21;

// First degree class that takes the two-phase hub path, given the largest LDS allocation a
// workgroup may make and the table value width (wide: 8-byte values).
int hub_first_class(size_t max_lds_per_block, bool wide);
hipError_t zero_words(unsigned long long* a, int64_t n, hipStream_t s);
// Fused LDS-table move kernel (degree classes 0..6) over the rows of vertex class `cls`.
hipError_t move_fused(const DevGraph& g, const Buckets& b, int cls, const MoveBuffers& m,
                      bool wide, hipStream_t s);
// Kernels of degree classes 7 .. hub_first-1 of class `cls` (a 256-thread group per row for
// class 7, a 1024-thread workgroup per row above).
hipError_t move_wg(const DevGraph& g, const Buckets& b, int cls, const MoveBuffers& m, bool wide,
                   hipStream_t s);
// Hub kernels over the hub rows of vertex class `cls` (plan hp made for those rows).
hipError_t move_hubs(const DevGraph& g, const Buckets& b, int cls, const PartPlan& pp,
                     const MoveBuffers& m, bool wide, hipStream_t s);
// The class step's decisions applied to the records, and the block records of move_fused and
// move_wg summed into m.stats (after all three tiers).
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
  // per label (n entries, +1 where noted)
  int64_t* newid = nullptr;    // [n+1] exclusive rank of used labels
  int32_t* mcount = nullptr;   // [n] members with arcs, then fill cursors
  int64_t* mstart = nullptr;   // [n+1] first member slot per label
  int64_t* astart = nullptr;   // [n] first flat arc per label
  int64_t* A = nullptr;        // [n] arcs per label
  int32_t* oldlabel = nullptr; // [n] label of each new id
  int64_t* dcount = nullptr;   // [n+1] distinct targets per new id
  // per member slot / vertex
  int32_t* members = nullptr;  // [n] vertices with arcs, grouped by label
  int64_t* gscan = nullptr;    // [n+1] first flat arc of each member slot
  int32_t* map = nullptr;      // [n] new id of each vertex
  uint16_t* map16 = nullptr;   // [n] the same in 16 bits (0xFFFF: no arcs), or null
  // output rows (at astart[c] for community c) and scratch
  int32_t* okey = nullptr;     // [nnz]
  uint64_t* ow = nullptr;      // [nnz] (read as uint32 [nnz] when w32)
  bool w32 = false;            // super-arc weights written as uint32
  int32_t* list = nullptr;     // [n]
  int64_t* partial = nullptr;  // scan scratch
  unsigned long long* counts = nullptr;  // 1536 words
  unsigned long long* stats = nullptr;   // [0] weight of self super-arcs
  unsigned long long* block_partial = nullptr;  // 1 word per block of the LDS merge kernel
  int64_t* hub_arrays = nullptr;         // kPlanWords * (hubs + 1)
  int32_t* pk = nullptr;                 // phase-1 pairs of the large communities
  void* pv = nullptr;                    // their values: uint32 when w32, else uint64
  int32_t* hoff = nullptr;               // their segment bounds
  int32_t* nflush = nullptr;             // table flushes of every phase-1 workgroup
  int32_t* cfm = nullptr;                // first member of every chunk row
  GraphSet gs;                           // batches: gid (of labels) and gself are used
};
// Renumbering, member lists and flat arc ranges (everything before the merge).
hipError_t aggregate_prepare(const DevGraph& g, const int32_t* C, const int32_t* csize,
                             const uint64_t* Sig, uint64_t* Kp, int32_t* map,
                             const AggBuffers& a, bool live_only, hipStream_t s);
// Live numbering (only communities with arcs get new ids; see lv_kernels.hip): the next level's
// representatives, the prefix count of vertices without arcs, the hashed classes by the
// method's ids, and the membership in the method's numbering.
hipError_t next_rep(int64_t np, const int32_t* oldlabel, const int32_t* rep, int32_t* rep_next,
                    hipStream_t s);
hipError_t no_arc_prefix(const DevGraph& g, int32_t* flag, int64_t* noarc_before,
                         int64_t* partial, hipStream_t s);
hipError_t live_classes(int64_t nl, int32_t pass, int32_t K, const int32_t* rep,
                        const int64_t* noarc_before, uint8_t* vclass, hipStream_t s);
hipError_t canon_membership(int64_t n0, const int32_t* top, int64_t nl, const int32_t* rep,
                            const int64_t* noarc_before, int32_t* flag, int64_t* live_before,
                            int64_t* partial, int32_t* out, hipStream_t s);
hipError_t merge_lds(const DevGraph& g, const Buckets& b, const AggBuffers& a, hipStream_t s);
int64_t merge_lds_blocks(const Buckets& b);  // sizes block_partial
// Communities of classes 7 .. part_first - 1 (one workgroup each, whole table in LDS); the
// two-phase merge takes classes part_first and up (merge_part_first_class: 7 to 10).
int merge_part_first_class(size_t max_lds_per_block, bool w32);
hipError_t merge_mid(const DevGraph& g, const Buckets& b, const AggBuffers& a, int part_first,
                     hipStream_t s);
hipError_t merge_hubs(const DevGraph& g, const Buckets& b, const PartPlan& pp,
                      const AggBuffers& a, int part_first, hipStream_t s);
// rs[a], re[a] of the super-vertex graph's rows in okey/ow
hipError_t super_rows(int64_t np, const AggBuffers& a, int64_t* rs, int64_t* re, hipStream_t s);
hipError_t sum_i64(const int64_t* a, int64_t n, unsigned long long* out, hipStream_t s);
// Gather gapped rows (row a at astart[oldlabel[a]], length offp[a+1]-offp[a]) into a CSR.
hipError_t compact_rows(const int64_t* offp, int64_t np, int64_t nnzp, const int32_t* oldlabel,
                        const int64_t* astart, const int32_t* tkey, const uint64_t* tw,
                        int32_t* idx_out, uint64_t* w_out, hipStream_t s);
hipError_t compose_membership(int32_t* top, int64_t n, const int32_t* map, hipStream_t s);
// top[v] = map[top[v]] except for the vertices v of graphs with keep[gid0[v]] != 0
hipError_t compose_membership_masked(int32_t* top, int64_t n, const int32_t* map,
                                     const int32_t* gid0, const uint8_t* keep, hipStream_t s);

// ---- batches of graphs (consecutive vertex ranges gbase[g] .. gbase[g+1])
hipError_t fold_gain_slices(unsigned long long* gS, int64_t G, hipStream_t s);
hipError_t graph_ids(const int64_t* gbase, int64_t G, int64_t n, int32_t* gid, hipStream_t s);
// out[g] += sum over graph g of x (squares: out[2g..2g+1] += sum of x^2, 128-bit)
hipError_t graph_sums(const uint64_t* x, int64_t n, const int32_t* gid, bool squares,
                      unsigned long long* out, hipStream_t s);
// out[g] = newid[gbase[g]] for g = 0 .. G
hipError_t next_gbase(const int64_t* newid, const int64_t* gbase, int64_t G, int64_t* out,
                      hipStream_t s);
hipError_t localize_membership(int32_t* memb, int64_t n, const int32_t* gid0,
                               const int64_t* gfinal, hipStream_t s);
// *bad |= 1 if a graph's first arc is not at aptr[g], |= 2 if an arc leaves its graph.
hipError_t validate_batch(const DevGraph& g, const int32_t* gid, const int64_t* gbase,
                          const int64_t* aptr, int64_t G, unsigned int* bad, hipStream_t s);

// ---- partition and merge (lv_part.hip)
// bounds[0..P]: contiguous parts balanced by arcs (bounds[k] = least v with
// off[v] >= floor(k * nnz / P))
hipError_t part_bounds(const int64_t* off, int64_t n, int64_t nnz, int64_t P, int64_t* bounds,
                       hipStream_t s);
// The union of the parts' induced subgraphs (same vertex ids): flag [nnz] and pos [nnz+1]
// scratch, nidx/nw [nnz] (weights of g's width), noff [n+1], aptr [P+1] part arc bounds.
hipError_t part_induced(const DevGraph& g, const int32_t* gid, const int64_t* vptr, int64_t P,
                        int32_t* flag, int64_t* pos, int64_t* partial, int32_t* nidx, void* nw,
                        int64_t* noff, int64_t* aptr, hipStream_t s);
// lab[v] += loff[gid[v]]
hipError_t part_offset_labels(int32_t* lab, int64_t n, const int32_t* gid, const int64_t* loff,
                              hipStream_t s);

// The aggregation map in 16 bits (0xFFFF for -1), for fewer than 0xFFFF super-vertices.
hipError_t narrow_map(const int32_t* map, int64_t n, uint16_t* out, hipStream_t s);

// ---- gather-rate probe (lv_probe.hip): measurement, not part of the method
// Threads and gathers of one probe launch (out holds probe_threads() ints).
int64_t probe_threads();
int64_t probe_gathers();
// One launch over table[0, n): slices > 0, n >= slices; workgroup b gathers from slice
// b mod slices of n / slices entries.
hipError_t gather_probe(const int32_t* table, uint64_t n, uint32_t slices, int32_t* out,
                        hipStream_t s);

// ---- colour classes (lv_colour.hip)
struct ColourBuffers {
  int32_t* slot = nullptr;      // [2n] per vertex: uncoloured higher-priority neighbours, and
                                //   the mask of the colours the coloured ones hold
  int32_t* all_long = nullptr;  // [2n] vertices with mid rows, then (from n) with long rows
  int32_t* shorts = nullptr;    // [2n] two alternating frontiers of short-row vertices
  int32_t* mids = nullptr;      // [2n] two alternating frontiers of mid-row vertices
  int32_t* longs = nullptr;     // [2n] two alternating frontiers of long-row vertices
  unsigned long long* counts = nullptr;  // [11] frontier counters, mid and long row counts
};
// Class of every vertex of pass `pass` (K classes): first-fit colouring in descending priority
// order, colours 0..K-2, the rest class K-1 (gid/gbase: ids local to each graph of a batch).
// host_words: pinned host words for read-backs; rounds: Jones-Plassmann rounds taken;
// small_stages (testing): tiny per-workgroup append stages, so that their overflow path runs.
hipError_t colour_classes(const DevGraph& g, int K, int pass, const int32_t* gid,
                          const int64_t* gbase, const ColourBuffers& cb,
                          unsigned long long* host_words, uint8_t* colour, int* rounds,
                          bool small_stages, hipStream_t s);

// ---- graph preparation (lv_prep.hip)
constexpr uint32_t kPrepSym = 0x1u, kPrepLoops = 0x2u, kPrepMax = 0x4u;
constexpr int64_t kPrepTile = 4096;  // items per workgroup of the sort and emit kernels
constexpr int kRadixBits = 8;        // largest digit of one sort pass
int prep_key_bits(int64_t n);        // bits of a vertex id in the sort key
constexpr int kMaxSortPasses = 8;    // 62 key bits at most, digits of at most 8 bits
struct SortPlan {                    // the LSD passes: digit (key >> shift[p]) & (2^bits[p] - 1)
  int passes = 0;
  int shift[kMaxSortPasses] = {0};
  int bits[kMaxSortPasses] = {0};
};
hipError_t prep_expand(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                       const uint32_t* w, uint32_t flags, int b, uint64_t* keys, uint32_t* vals,
                       unsigned int* bad, hipStream_t s);
hipError_t radix_hist(const uint64_t* keys, int64_t N, int shift, int bits, int32_t* hist,
                      hipStream_t s);
hipError_t radix_scatter(const uint64_t* kin, const uint32_t* vin, uint64_t* kout,
                         uint32_t* vout, int64_t N, int shift, int bits, const int64_t* offs,
                         hipStream_t s);
// vals == nullptr: keys-only arcs (no input weights)
// one-sweep sort: counts of every pass (ghist [kMaxSortPasses * 256] scratch, gbase the same
// size, output starts), then one look-back scatter per pass (status: [tiles * 256 + 1] words;
// a look-back that waits too long sets bit 3 of *bad)
hipError_t radix_counts(const uint64_t* keys, int64_t N, const SortPlan& plan,
                        unsigned long long* ghist, int64_t* gbase, hipStream_t s);
hipError_t radix_onesweep(const uint64_t* kin, const uint32_t* vin, uint64_t* kout,
                          uint32_t* vout, int64_t N, int shift, int bits, const int64_t* gbase,
                          unsigned long long* status, unsigned int* bad, hipStream_t s);
hipError_t prep_heads(const uint64_t* keys, const uint32_t* vals, int64_t N, int b,
                      bool combine_max, int32_t* tile_heads, unsigned long long* tile_first,
                      hipStream_t s);
hipError_t prep_emit(const uint64_t* keys, const uint32_t* vals, int64_t N, int64_t n, int b,
                     bool combine_max, bool w32, const int64_t* tile_slot,
                     const int32_t* tile_heads, const unsigned long long* tile_first,
                     int64_t* off, int32_t* idx, void* w, unsigned int* bad, hipStream_t s);

}  // namespace lv
