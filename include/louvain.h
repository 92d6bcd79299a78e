/*
 * louvain.h -- C ABI of the MI355X (gfx950) Louvain library, liblouvain.so.
 *
 * The library runs the static Louvain method of Sahu, "Enhancing Efficiency in Parallel
 * Louvain Algorithm for Community Detection" (arXiv 2301.12390), section 3.2: passes of a
 * local-moving phase (every vertex moves to the neighbour community of greatest modularity
 * increase, repeated while an iteration's total modularity change exceeds a tolerance that
 * shrinks by a decline factor each pass) and an aggregation phase (communities collapse into
 * super-vertices, combined edge weights, intra-community edges become self-loops).
 *
 * The local-moving phase uses the synchronous (Jacobi) rule the paper compares in section 3.2:
 * every decision reads only the previous iteration's memberships. It is exact integer
 * arithmetic throughout, so results are deterministic and independent of scheduling:
 *   W       = sum of all arc weights; K_i = row sum of i (a self-loop counts once);
 *   Sigma_c = sum of K_i over community c; k_{i->x} = weight of i's non-self arcs into x;
 *   gain of placing i into x: g_i(x) = W*k_{i->x} - K_i*(Sigma_x - [x == C_i]*K_i)
 *   (twice the change in W^2*Q of the move, Blondel et al.'s delta-modularity scaled by W^2/2).
 * A vertex moves to the candidate (a non-self neighbour's community) of largest g, ties to
 * the smallest community id, iff that g is strictly larger than g_i(own community) and it is
 * not a singleton about to swap with a singleton of larger id. An iteration's gain sum S
 * continues the phase iff S > floor(W^2 / (2*10^(a+b*p))) in pass p (tolerance 10^-a declining
 * by 10^b per pass; the paper's defaults are a = 2, b = 1).
 *
 * Partial asynchrony (section 3.2 recommends it over a fully synchronous rule): with
 * substeps = K > 1 the vertices of pass p are split into K classes, vertex v going to class
 * floor(hi32(s) * K / 2^32) where s = SplitMix64 output v+1 of the sequence started at state p
 * (s = mix(p + (v+1)*0x9E3779B97F4A7C15), Steele et al. 2014). An iteration is then K
 * synchronous steps, class 0 first, each step reading the memberships left by the steps
 * before it. K = 1 is the fully synchronous rule.
 *
 * Graph format (all functions): a symmetric CSR of arcs. An undirected edge {u,v} is stored as
 * arcs (u,v) and (v,u); a self-loop (u,u) is stored once. Rows need not be sorted; repeated
 * arcs in a row mean their summed weight. Weights are integers >= 1.
 *
 * Pointers are DEVICE pointers unless marked (host). Inputs and outputs are owned by the
 * caller and must stay valid until the work enqueued on `stream` has completed; functions
 * with host outputs synchronise `stream` before returning. The library owns only its context
 * workspace (tables, scan temporaries, super-vertex graphs), charged to the HBM budget given
 * at creation. `stream` is a hipStream_t. The library enqueues nothing on the null stream of
 * its own accord and never synchronises the device: a call's work goes to its `stream` and to
 * non-blocking side streams that it forks from and joins back to `stream` with events, and
 * the server's slots (louvain_server_*) run on non-blocking streams of their own. A caller
 * whose own stream is the default one (torch's default stream) passes NULL, and the work then
 * runs there.
 *
 * Errors: every function returns an lv_status; no exception crosses the boundary. On error
 * the outputs are unspecified and the context stays usable (after a sticky HIP error it
 * should be destroyed). louvain_last_error() describes the last failure. A context is not
 * thread-safe: use one per host thread.
 */
#ifndef LOUVAIN_H
#define LOUVAIN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LV_OK = 0,
  LV_EINVAL = -1,    /* null pointer, negative size, bad parameter, or invalid graph */
  LV_ENOMEM = -2,    /* device allocation failed */
  LV_EHIP = -3,      /* a HIP runtime call or kernel launch failed */
  LV_EOVERFLOW = -4, /* n >= 2^31, nnz >= 2^31 with int32 offsets, or W > 2^62 (W is the
                        exact sum of the weights, so a 64-bit wrap-around is detected too) */
  LV_EBUDGET = -5,   /* the workspace would exceed the context's HBM budget */
  LV_ECANCELLED = -6, /* a server request dropped because the server was destroyed first */
  LV_ETIMEOUT = -7    /* louvain_server_wait: the request had not completed in time */
} lv_status;

/* 128-bit two's-complement integer: value = hi * 2^64 + lo. */
typedef struct {
  uint64_t lo;
  int64_t hi;
} lv_i128;

typedef struct lv_ctx lv_ctx;

/* Symmetric CSR of arcs (see above). */
typedef struct {
  int64_t n;               /* vertices, 0 <= n < 2^31 */
  int64_t nnz;             /* arcs */
  const void* offsets;     /* [n+1], int32 if offsets_64 == 0 else int64; offsets[0] == 0 */
  const int32_t* indices;  /* [nnz], neighbour ids in [0, n) */
  const void* weights;     /* [nnz], uint32 if weights_64 == 0 else uint64; each >= 1 */
  int32_t offsets_64;
  int32_t weights_64;
} lv_graph;

#define LV_VALIDATE 0x1u   /* check indices, weights and offsets on the device (O(nnz)) */
#define LV_TRACE 0x2u      /* time the kernels of every iteration with HIP events */
#define LV_FORCE_WIDE 0x4u /* use 128-bit gains, 64-bit table values and 64-bit super-arc
                              weights even where narrower ones are exact (results are
                              identical; for testing) */
#define LV_SMALL_PARTS 0x8u /* split long rows and large communities into many hash
                               partitions with tiny workgroup tables, so that the partitioned
                               and multi-round code paths run on small graphs (results are
                               identical; slower; for testing) */
#define LV_COLOR_CLASSES 0x10u /* colour classes instead of hashed ones (section 3.2 cites graph
                                  colouring for partial asynchrony): in every pass the K =
                                  substeps classes are a first-fit distance-1 colouring in
                                  descending order of the vertices' SplitMix64 draws, colours
                                  0..K-2 (independent sets), the rest in class K-1; computed in
                                  Jones-Plassmann rounds on the device */
#define LV_GRAPH_REPLAY 0x20u /* a local-moving phase on at most 2^24 arcs runs its first
                                 iteration directly and replays the later ones as a HIP graph
                                 captured once per phase, instead of launching every kernel
                                 directly (results are identical). Off by default: on MI355X the
                                 capture costs more than the launches it saves (SBM-10k 3.4 ms
                                 against 2.4 ms per run) */

typedef struct {
  int32_t tolerance_exp10; /* initial tolerance 10^-a, a >= 0 (paper's best: a = 2) */
  int32_t decline_exp10;   /* tolerance divided by 10^b between passes, b >= 0 (b = 1) */
  int32_t max_iterations;  /* local-moving iterations per pass, >= 1 (default 20) */
  int32_t max_passes;      /* passes, 1..64 (default 10) */
  int32_t substeps;        /* vertex classes per iteration, 1..32 (1 = fully synchronous) */
  uint32_t flags;          /* LV_* flags */
} lv_params;

#define LV_MAX_PASSES 64
#define LV_MAX_TRACE 1024

/* One local-moving iteration (host). The move kernels are: the fused LDS-table kernel
 * (k_move_lds, rows of up to 1024 arcs), the group and workgroup-per-row kernels (k_move_grp7,
 * k_move_wg: rows of up to 8192 arcs when the device allows their LDS tables) and the two-phase
 * hub kernels (longer rows). The tiers of a class step may run concurrently, so their times
 * overlap. */
typedef struct {
  int32_t pass, iteration;
  int32_t wide;            /* 1 if this iteration used 128-bit gains */
  int32_t substeps;        /* class steps of the iteration */
  int32_t fused_launches;  /* launches of k_move_lds */
  int32_t wg_launches;     /* class steps with rows for k_move_grp7 / k_move_wg */
  int32_t hub_launches;    /* class steps that ran the hub kernels */
  int32_t reserved;
  lv_i128 gain_sum;        /* S: sum of the applied gains */
  int64_t moved;           /* vertices that changed community */
  int64_t candidates;      /* distinct (vertex, other community) pairs examined */
  int64_t fused_vertices, fused_arcs, fused_candidates; /* work of k_move_lds */
  int64_t wg_vertices, wg_arcs, wg_candidates;          /* work of k_move_grp7 / k_move_wg */
  int64_t hub_vertices, hub_arcs;                       /* work of the hub kernels */
  float fused_ms;          /* k_move_lds, summed over the class steps (LV_TRACE) */
  float wg_ms;             /* k_move_grp7 and k_move_wg (LV_TRACE) */
  float hub_ms;            /* hub kernels (LV_TRACE) */
  float update_ms;         /* the step's record reduction and community updates (LV_TRACE) */
  float iter_ms;           /* whole iteration including the host read-back (LV_TRACE) */
  float reserved2;
} lv_iter_trace;

/* Result of louvain_run (host). */
typedef struct {
  int32_t passes;                         /* passes that ran a local-moving phase */
  int32_t iterations_total;
  int32_t iterations[LV_MAX_PASSES];
  int64_t n_pass[LV_MAX_PASSES];          /* vertices of the graph pass p ran on */
  int64_t nnz_pass[LV_MAX_PASSES];        /* arcs of that graph */
  lv_i128 qnum_pass[LV_MAX_PASSES];       /* W^2*Q after pass p's local-moving phase (a last
                                             pass whose value is not above the level before it
                                             was dropped: see louvain_run) */
  int32_t cap_hits;                       /* phases stopped by max_iterations */
  int32_t n_trace;                        /* records in trace[] (first LV_MAX_TRACE) */
  int64_t n_communities;                  /* communities of the result */
  uint64_t W;                             /* total arc weight */
  lv_i128 q_num;                          /* W^2 * Q of the result, exact */
  double q;                               /* Q = q_num / W^2 (0 when W == 0) */
  float total_ms;                         /* host wall time of the call */
  float aggregate_ms[LV_MAX_PASSES];      /* aggregation duration per pass (LV_TRACE) */
  lv_iter_trace trace[LV_MAX_TRACE];
} lv_result;

/* Statistics of louvain_move (host). */
typedef struct {
  int32_t iterations;      /* iterations run */
  int32_t hit_cap;         /* 1 if stopped by max_iterations rather than the tolerance */
  int64_t moved;           /* total moves */
  lv_i128 gain_sum;        /* sum of S over the iterations */
  lv_i128 last_gain;       /* S of the last iteration */
  int64_t last_moved;      /* moves of the last iteration */
  int64_t last_candidates; /* candidate pairs of the last iteration */
} lv_move_stats;

/* Result of one graph of a batch (host). */
typedef struct {
  int32_t passes;                      /* passes run on this graph */
  int32_t iterations_total;
  int32_t iterations[LV_MAX_PASSES];   /* local-moving iterations of every pass */
  uint32_t cap_hits;                   /* phases that stopped at max_iterations */
  int32_t reserved;
  int64_t n_communities;               /* communities of the graph's last level */
  uint64_t W;                          /* total arc weight of the graph */
  lv_i128 q_num;                       /* W^2 * Q exactly */
  double q;
} lv_graph_result;

/* Context: binds a device and a workspace limited to hbm_budget_bytes (0 = no limit).
 * Returns LV_EINVAL for a bad device or null out, LV_EHIP if the device cannot be set. */
lv_status louvain_ctx_create(int device, uint64_t hbm_budget_bytes, lv_ctx** out);
void louvain_ctx_destroy(lv_ctx* ctx);
/* Text of the last failure on this context ("" if none). Valid until the next call. */
const char* louvain_last_error(const lv_ctx* ctx);
/* Bytes of device workspace currently held by the context. */
uint64_t louvain_workspace_bytes(const lv_ctx* ctx);

/* Whole method (section 3.2): passes of local-moving + aggregation while every pass raises
 * modularity (pass_tolerance = 0). A pass that does not (nothing moved, or simultaneous moves
 * that together did not raise Q) ends the run and is dropped: the result is the level before
 * it. Aggregation that does not shrink the graph, or max_passes, also ends the run.
 * membership: [n] out, the community of every input vertex in the last level of the
 * dendrogram (dense ids 0..n_communities-1; the identity if no pass aggregated).
 * res (host): passes, iterations, per-iteration trace, W and exact Q. */
lv_status louvain_run(lv_ctx* ctx, const lv_graph* g, const lv_params* p, int32_t* membership,
                      lv_result* res, void* stream);

/* louvain_run that also returns the whole dendrogram. In section 3.2 the communities a pass
 * finds become the vertices of the next pass, so every aggregation yields a coarser partition
 * of the input vertices that nests the previous one.
 * levels: [max_levels * n] out (device, caller-owned): levels[l*n + v] is the community of input
 * vertex v after the l-th aggregation (dense ids, l = 0 the finest); rows at and beyond
 * *n_levels are not written. The last written row equals membership; no row is written when no
 * pass aggregated. max_levels must be >= p->max_passes (else LV_EINVAL, nothing run), which
 * bounds the aggregations. n_levels (host) out: rows written. Other arguments and errors as
 * louvain_run; the dendrogram adds one n-int device copy per aggregation. */
lv_status louvain_run_levels(lv_ctx* ctx, const lv_graph* g, const lv_params* p,
                             int32_t* membership, int32_t* levels, int32_t max_levels,
                             int32_t* n_levels, lv_result* res, void* stream);

/* One local-moving phase (section 3.2) on an arbitrary state, under pass p's tolerance
 * (max_iterations = 1 runs exactly one synchronous iteration: the per-iteration parity entry).
 * K: [n] row sums, or NULL to compute them. W: total arc weight, or 0 to compute it.
 * C: [n] in/out community labels in [0, n). Sigma: [n] in/out, Sigma[c] = sum of K over c.
 * csize: [n] in/out, csize[c] = members of c. Sigma and csize must match C on entry.
 * stats (host, may be NULL). */
lv_status louvain_move(lv_ctx* ctx, const lv_graph* g, const uint64_t* K, uint64_t W,
                       int32_t pass_index, const lv_params* p, int32_t* C, uint64_t* Sigma,
                       int32_t* csize, lv_move_stats* stats, void* stream);

/* Aggregation phase (section 3.2): collapse the communities of C (labels in [0, n)) into
 * super-vertices numbered by ascending rank of their label. Arcs between communities combine
 * into super-arcs; arcs inside a community combine into the super-vertex's self-loop.
 * map: [n] out, super-vertex of every vertex. offsets_out: [n+1] out, int64 when
 * offsets_64_out else int32. indices_out: [nnz] out. weights_out: [nnz] out, uint64 (sums may
 * exceed 32 bits). Output rows hold distinct neighbours in unspecified order.
 * n_out, nnz_out (host): size of the super-vertex graph. */
lv_status louvain_aggregate(lv_ctx* ctx, const lv_graph* g, const int32_t* C, int32_t* map,
                            void* offsets_out, int32_t offsets_64_out, int32_t* indices_out,
                            uint64_t* weights_out, int64_t* n_out, int64_t* nnz_out,
                            void* stream);

/* Batch of independent graphs in one run (section 3.2 applied to every graph at once; the
 * kernels of every step cover all graphs, so many small graphs fill the device together).
 * packed: one CSR of the G graphs with consecutive global vertex ids: graph g owns vertices
 * graph_vptr[g] .. graph_vptr[g+1]-1 and arcs graph_aptr[g] .. graph_aptr[g+1]-1, and no arc
 * joins two graphs. graph_vptr, graph_aptr: (host) [G+1], from 0 to n and nnz, non-decreasing
 * (LV_VALIDATE also checks them against the offsets and indices on the device).
 * Every graph has its own W, tolerance schedule, convergence and stop rules, and its vertex
 * classes hash ids local to the graph, so its result equals louvain_run on that graph alone.
 * membership: [n] out, community of every vertex as a dense id local to its graph.
 * per_graph (host): [G] results. G >= 1; errors as louvain_run (a graph with W > 2^62, or a batch
 * whose total weight reaches 2^64, gives
 * LV_EOVERFLOW for the whole batch). LV_TRACE is ignored. */
lv_status louvain_run_batched(lv_ctx* ctx, const lv_graph* packed, int32_t G,
                              const int64_t* graph_vptr, const int64_t* graph_aptr,
                              const lv_params* p, int32_t* membership,
                              lv_graph_result* per_graph, void* stream);

/* Modularity (section 1: Newman-Girvan) of membership C (labels in [0, n)):
 * q_num = W * sum_c sigma_c - sum_c Sigma_c^2 exactly (sigma_c: weight of arcs inside c),
 * W = total weight, q = q_num / W^2. All outputs host; any may be NULL. */
lv_status louvain_modularity(lv_ctx* ctx, const lv_graph* g, const int32_t* C, lv_i128* q_num,
                             uint64_t* W, double* q, void* stream);

/* Bytes of the fixed device array behind louvain_modularity_noalloc (per device). */
#define LV_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* louvain_modularity without any device allocation, for callers that cannot allocate during
 * the call (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and errors as louvain_modularity, but the temporaries (row sums and
 * Sigma, n words each; widened offsets for int32 CSRs, n + 1 words; a tile table of nnz / 4096
 * words; 32 reduction words) live in a fixed array of LV_NOALLOC_SCRATCH_BYTES that the library
 * holds on every device it has a context on, from louvain_ctx_create until the process ends.
 * A graph needing more returns LV_EBUDGET (about 4M vertices with int64 offsets, 2.7M with
 * int32). The context's workspace is neither used nor grown. Every call on one device shares
 * that device's array: calls that overlap on the same device (other streams, other host
 * threads, other contexts) race and must be serialised by the caller. */
lv_status louvain_modularity_noalloc(lv_ctx* ctx, const lv_graph* g, const int32_t* C,
                                     lv_i128* q_num, uint64_t* W, double* q, void* stream);

/* Partition and merge (the remedy section 3.2 and the conclusion propose for the method's poor
 * shared-memory scaling: run partitions of the graph independently, then combine them). The P
 * parts are contiguous vertex ranges: part_vptr (host) [P+1] from 0 to n, non-decreasing, or
 * NULL for parts balanced by arcs (part k starts at the least v with offsets[v] >=
 * floor(k * nnz / P)). Each part's induced subgraph (arcs with both ends in the part) runs the
 * whole method on its own, with ids local to the part, all parts in one batch (as
 * louvain_run_batched). Their communities, numbered part after part, partition the graph;
 * the whole graph, cross-part arcs included, is aggregated by that partition and the method
 * runs again on the super-vertex graph (the merge).
 * membership: [n] out, the final community of every vertex (dense ids). per_part (host, may be
 * NULL): [P] results of the part runs. merge_res (host): the merge run's result; its q_num and
 * q are the final partition's on the whole graph. P in 1..2^20. Errors as louvain_run. */
lv_status louvain_run_partitioned(lv_ctx* ctx, const lv_graph* g, int32_t P,
                                  const int64_t* part_vptr, const lv_params* p,
                                  int32_t* membership, lv_graph_result* per_part,
                                  lv_result* merge_res, void* stream);

/* Colour classes of a graph (LV_COLOR_CLASSES; section 3.2 cites graph colouring for partial
 * asynchrony): classes[v] in [0, K) for pass `pass` (>= 0) and K in 1..32 classes. Vertices
 * are visited in descending order of their SplitMix64 draws of the pass (the draw behind the
 * hashed classes, all 64 bits); each takes the smallest colour in 0..K-2 that none of its
 * earlier-visited neighbours holds, else class K-1. classes: [n] out (device, uint8). rounds
 * (host, may be NULL): Jones-Plassmann rounds the device took. Errors as louvain_run. */
lv_status louvain_colour_classes(lv_ctx* ctx, const lv_graph* g, int32_t pass, int32_t K,
                                 uint8_t* classes, int32_t* rounds, void* stream);

/* Measurement, not part of the method: the device's rate of random 4-byte gathers, the
 * ceiling the local-moving and aggregation kernels run against (each arc reads a neighbour's
 * record or label at a position with no locality). Every thread of a 4.2M-thread grid makes 64
 * gathers at hashed positions of a table of table_bytes bytes, rounded down to a multiple of
 * 4 * slices. With slices > 1, workgroup b gathers only from slice b mod slices; with
 * slices = 8 each XCD's L2 then holds one eighth of the table. The table (contents
 * irrelevant) is taken from the context's workspace. rate (host): gathers per second, the best
 * of three timed launches after a warm-up. Errors: LV_EINVAL for slices outside 1..64, a table
 * of fewer than 4 * slices bytes or a NULL rate; LV_ENOMEM beyond the budget. */
lv_status louvain_probe_gather(lv_ctx* ctx, uint64_t table_bytes, int32_t slices, double* rate,
                               void* stream);

/* Graph preparation flags of louvain_prepare. */
#define LV_PREP_SYMMETRIZE 0x1u /* add the reverse (v, u, w) of every edge (u, v, w), u != v */
#define LV_PREP_SELF_LOOPS 0x2u /* add a self-loop of weight 1 on every vertex */
#define LV_PREP_MAX 0x4u        /* repeated arcs combine by max (default: by sum) */
#define LV_PREP_TRACE 0x8u      /* time the kernel phases with HIP events (lv_prep_stats) */
#define LV_PREP_TILE_SORT 0x10u /* sort with a histogram pass per digit instead of the one-sweep
                                   look-back sort (results are identical; for testing) */

/* What louvain_prepare did (host). */
typedef struct {
  int64_t arcs;        /* arcs before combining: m (2m with LV_PREP_SYMMETRIZE) (+ n loops) */
  int64_t nnz;         /* arcs after combining */
  int32_t key_bits;    /* significant bits of the (source, neighbour) sort key */
  int32_t sort_passes; /* radix passes over the key, digits of at most 8 bits */
  float expand_ms;     /* LV_PREP_TRACE: edge list -> keyed arcs */
  float hist_ms;       /* LV_PREP_TRACE: digit counts (all passes, or per pass) */
  float scan_ms;       /* LV_PREP_TRACE: per-tile histogram scans (LV_PREP_TILE_SORT) */
  float scatter_ms;    /* LV_PREP_TRACE: stable digit scatters, summed */
  float emit_ms;       /* LV_PREP_TRACE: run heads, their scan, the CSR writes and narrowing */
  float total_ms;      /* whole call (host clock) */
} lv_prep_stats;

/* Graph preparation (section 3.1.2 and Table 1: the inputs of the method are edge lists made
 * undirected by adding every edge's reverse, with unit weights and a self-loop on every
 * vertex): turns an edge list into the symmetric CSR every function above takes.
 * src, dst: [m] int32 endpoints in [0, n). weights: [m] uint32 >= 1, or NULL for all ones.
 * The arcs are the edges, their reverses (LV_PREP_SYMMETRIZE; a self-loop edge stays one arc)
 * and one loop per vertex (LV_PREP_SELF_LOOPS); arcs with equal (source, neighbour) combine
 * into one, by sum or, with LV_PREP_MAX, by max (so LV_PREP_SYMMETRIZE | LV_PREP_SELF_LOOPS |
 * LV_PREP_MAX with NULL weights gives the paper's unit-weight graphs).
 * Outputs: offsets_out [n+1] (int64 if offsets_64_out else int32), indices_out [nnz] and
 * weights_out [nnz] (uint64 if weights_64_out else uint32), rows in ascending neighbour order.
 * capacity: entries available in indices_out and weights_out. nnz_out (host): arcs of the
 * prepared graph. With indices_out and weights_out both NULL the call only counts (*nnz_out).
 * stats (host, may be NULL): sizes, and phase times with LV_PREP_TRACE.
 * Errors: LV_EINVAL for a bad argument or flag, an endpoint outside [0, n), a zero weight, or
 * capacity < nnz (then *nnz_out holds the needed size); LV_EOVERFLOW for n >= 2^31, more than
 * 2^40 arcs, nnz >= 2^31 with int32 offsets, or a combined weight above 2^32-1 with uint32
 * weights. Workspace: about 24 bytes per arc before combining (sort keys and weights, double
 * buffered). */
lv_status louvain_prepare(lv_ctx* ctx, int64_t n, int64_t m, const int32_t* src,
                          const int32_t* dst, const uint32_t* weights, uint32_t flags,
                          void* offsets_out, int32_t offsets_64_out, int32_t* indices_out,
                          void* weights_out, int32_t weights_64_out, int64_t capacity,
                          int64_t* nnz_out, lv_prep_stats* stats, void* stream);

/* ---------------------------------------------------------------------------------------
 * Request server: continuous batching of independent graphs over one device. It is not a step
 * of the paper's method but a serving pattern around it: every request is the whole method
 * of section 3.2 on one graph.
 *
 * Requests are whole runs (louvain_run) on graphs held in host memory. The server keeps
 * `slots` runs in flight at once, each on its own context and HIP stream, so that the work of
 * different requests overlaps on the device. A slot that becomes free takes the requests at
 * the head of the queue (first come, first served) up to batch_arcs arcs and runs them as one
 * louvain_run_batched call (one request alone goes through louvain_run); requests that arrive
 * while others run are admitted as soon as a slot and device memory are free. Every result
 * equals that of louvain_run on the graph alone (louvain_run_batched's guarantee), whatever
 * else shares its batch or the device.
 *
 * Admission is by device memory: a slot holds its packing buffers and its context's workspace
 * (both grow-only) and reserves, before each run, an upper bound of what it will hold after it
 * (its buffers exactly, and for the workspace 320 bytes per vertex, 72 per arc, 640 per graph
 * and 48 MiB, at the largest batch it has run); the reservations of all slots stay within
 * hbm_budget_bytes. A request whose bound alone exceeds the budget fails with LV_EBUDGET;
 * when a request waits for memory, idle slots release theirs and no slot starts other work
 * until it has been admitted.
 *
 * Request graphs: lv_graph with HOST pointers (offsets int32 or int64, weights uint32 only),
 * checked on the device while they are packed (offsets from 0 to nnz and non-decreasing,
 * neighbours in [0, n), weights >= 1); a request that fails the check ends with LV_EINVAL and
 * the rest of its batch runs without it. Symmetry is the caller's contract, as for louvain_run.
 * A failure of the run itself ends every request of that run with its status (LV_EOVERFLOW for
 * a graph whose total weight exceeds 2^62, which takes about 2^30 arcs of weight near 2^32).
 * The graph's host arrays and the membership buffer must stay valid and untouched until
 * louvain_server_wait has returned the request (pinned host memory copies fastest).
 * A server is thread-safe: any thread may submit and wait.
 */
typedef struct lv_server lv_server;

typedef struct {
  int32_t slots;             /* runs in flight at once, 1..16 */
  int32_t fail_run;          /* fault injection for tests: run number fail_run (counting from
                                1; 0 = none) fails with LV_ENOMEM as if its packing buffers
                                could not be allocated, before it touches the device */
  uint64_t hbm_budget_bytes; /* device memory of all slots together; 0 = no limit */
  int64_t batch_arcs;        /* most arcs of one batched run (a larger request runs alone);
                                0 = one request per run */
  lv_params params;          /* of every request (LV_TRACE is ignored) */
} lv_server_config;

/* What became of one request (host). Times are louvain_server_clock_ns() readings. */
typedef struct {
  int32_t status;            /* lv_status of the request */
  int32_t slot;              /* slot that ran it (-1 if it never ran) */
  int32_t batch_graphs;      /* requests of the run it was part of */
  int32_t reserved;
  int64_t batch_arcs;        /* arcs of that run */
  int64_t submit_ns;         /* louvain_server_submit */
  int64_t start_ns;          /* its run began (admitted, packing started) */
  int64_t done_ns;           /* its membership was in host memory */
  lv_graph_result result;    /* as louvain_run_batched's per-graph result */
  char error[160];           /* text of a failure ("" on success) */
} lv_request_result;

typedef struct {
  int64_t submitted, completed, failed; /* requests; completed counts failures too */
  int64_t runs;              /* louvain_run / louvain_run_batched calls */
  int64_t batched_requests;  /* requests that shared their run with others */
  int32_t slots;
  int32_t peak_running;      /* most slots running at the same time */
  int32_t trims;             /* times a slot released its memory for a waiting request */
  int32_t bound_misses;      /* runs after which a slot held more than it had reserved (0) */
  uint64_t committed_bytes;  /* device memory reserved by the slots now */
  uint64_t peak_committed_bytes;
  uint64_t peak_held_bytes;  /* most device memory all slots held together (measured) */
} lv_server_stats;

/* Starts the server's slots on `device` (contexts, streams and one host thread per slot).
 * LV_EINVAL for a bad device, config or parameter set; LV_EHIP if the device fails. */
lv_status louvain_server_create(int device, const lv_server_config* cfg, lv_server** out);
/* Drops the queued requests (LV_ECANCELLED), waits for the runs in flight, frees everything.
 * Tickets not yet waited for become invalid. No other call on the server may be in progress
 * (a thread blocked in louvain_server_wait included). */
void louvain_server_destroy(lv_server* server);
/* Queues a request: g (host pointers, see above) and membership (host, [n] out: dense
 * community ids, as louvain_run). ticket (host) out: the handle for louvain_server_wait.
 * LV_EINVAL for a malformed descriptor (null pointers, n outside [0, 2^31), nnz < 0, n == 0
 * with arcs, uint64 weights); LV_ECANCELLED once the server is being destroyed. */
lv_status louvain_server_submit(lv_server* server, const lv_graph* g, int32_t* membership,
                                uint64_t* ticket);
/* Waits up to timeout_ms (< 0: no limit, 0: poll) for a request; on LV_OK `out` holds its
 * outcome and the ticket is released. LV_ETIMEOUT if it is still queued or running (the ticket
 * stays valid); LV_EINVAL for an unknown or already returned ticket, or one that another
 * thread is waiting for (one waiter per ticket). */
lv_status louvain_server_wait(lv_server* server, uint64_t ticket, int64_t timeout_ms,
                              lv_request_result* out);
/* Drops a request that is still queued: it completes with LV_ECANCELLED (collect it with
 * louvain_server_wait) and *cancelled (host, may be NULL) is 1. A request already running or
 * done is not affected (*cancelled = 0). LV_EINVAL for an unknown ticket. */
lv_status louvain_server_cancel(lv_server* server, uint64_t ticket, int32_t* cancelled);
/* Counters of the server (host). */
lv_status louvain_server_stats(lv_server* server, lv_server_stats* out);
/* The server's clock: monotonic nanoseconds (CLOCK_MONOTONIC). */
int64_t louvain_server_clock_ns(void);

#ifdef __cplusplus
}
#endif

#endif /* LOUVAIN_H */
