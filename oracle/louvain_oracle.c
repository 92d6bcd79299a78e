/*
 * Louvain oracle: a plain, slow, obviously correct CPU implementation of the static Louvain
 * method described in section 3.2 ("Louvain algorithm") of Sahu, "Enhancing Efficiency in
 * Parallel Louvain Algorithm for Community Detection" (arXiv 2301.12390).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load this library. It shares no code, header, table or helper with the GPU
 * library; the two are written independently and compared.
 *
 * Conventions (the paper prints no formula; these are the standard definitions):
 *   A graph is a symmetric CSR of arcs: an edge {u,v}, u != v, is stored as arcs (u,v) and
 *   (v,u); a self-loop is stored once. Weights are positive integers.
 *   W      = sum of all arc weights.
 *   K_i    = sum of the weights of the arcs of row i (a self-loop counts once).
 *   sigma_c = sum of the weights of the arcs (i,j) with C[i] = C[j] = c.
 *   Sigma_c = sum of K_i over the vertices i of community c.
 *   Modularity (Newman-Girvan, section 1): Q = sum_c [ sigma_c/W - (Sigma_c/W)^2 ]
 *             = Qnum / W^2 with Qnum = W * sum_c sigma_c - sum_c Sigma_c^2 (exact integer).
 *   Gain of placing vertex i into community x ("delta-modularity", section 3.2):
 *             g_i(x) = W * k_{i->x} - K_i * (Sigma_x - [x == C[i]] * K_i)
 *   where k_{i->x} is the weight of the non-self arcs from i into x. Moving i from d to c
 *   changes Qnum by exactly 2 * (g_i(c) - g_i(d)).
 *
 * Readings of the paper adopted where it is silent:
 *   - candidates are the communities of the vertex's non-self neighbours (the method moves a
 *     vertex into some neighbour's community);
 *   - a vertex moves only if the best gain is strictly greater than the gain of staying;
 *   - ties between candidates go to the smallest community id;
 *   - synchronous (Jacobi) iterations read only the previous iteration's state, and a vertex
 *     whose own community and best community are both singletons does not move to a larger id
 *     (singleton-swap prevention, from the Grappolo line of work the paper cites);
 *   - the total modularity change of an iteration is 2*S/W^2 with S the sum of the applied
 *     gains; the phase repeats while it exceeds tolerance_p = 10^-(a + b*p) in pass p, i.e.
 *     while S > floor(W^2 / (2 * 10^(a+b*p)));
 *   - pass_tolerance is 0: the passes go on while a pass raises modularity. A pass that does
 *     not (no vertex moved, or simultaneous synchronous moves that together did not raise it)
 *     ends the run and is not kept: the result is the level before it. Aggregation that does
 *     not shrink the graph, or the pass limit, also ends the run;
 *   - aggregation renumbers used community labels by ascending rank.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __int128 i128;
typedef unsigned __int128 u128;

/* 128-bit values cross the C ABI as two 64-bit words, low word first. */
static void put_i128(uint64_t* out, i128 v) {
  out[0] = (uint64_t)(u128)v;
  out[1] = (uint64_t)((u128)v >> 64);
}

/* Vertex classes of the partially asynchronous rule. Section 3.2 of the paper recommends
 * asynchronous or partially asynchronous vertex processing over a fully synchronous one (it
 * cites graph colouring as one way). Here the vertices of pass p are split into K classes by a
 * counter-based SplitMix64 draw (Steele, Lea, Flood 2014): the draw for vertex v is the
 * (v+1)-th output of the sequence started at state p, mix(p + (v+1)*0x9E3779B97F4A7C15), and
 * its upper 32 bits select the class floor(hi32 * K / 2^32). */
static uint64_t splitmix64_finaliser(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int32_t orc_vertex_class(int32_t pass, int32_t K, int64_t v) {
  uint64_t z = (uint64_t)pass + ((uint64_t)v + 1u) * 0x9E3779B97F4A7C15ull;
  uint64_t hi = splitmix64_finaliser(z) >> 32;
  return (int32_t)((hi * (uint64_t)K) >> 32);
}

/* Vertices of each class of pass p, ascending within a class: verts[start[k] .. start[k+1]). */
void orc_class_lists(int64_t n, int32_t pass, int32_t K, int32_t* verts, int64_t* start) {
  int64_t pos = 0;
  for (int32_t k = 0; k < K; k++) {
    start[k] = pos;
    for (int64_t v = 0; v < n; v++)
      if (K == 1 || orc_vertex_class(pass, K, v) == k) verts[pos++] = (int32_t)v;
  }
  start[K] = pos;
}

/* Colour classes: the graph-colouring route to partial asynchrony that section 3.2 cites. A
 * first-fit distance-1 colouring of the current graph visits the vertices by descending
 * priority, the priority of v in pass p being the whole 64-bit draw above (ties cannot occur:
 * the finaliser is a bijection and the counters differ; they would go to the smaller id). Each
 * vertex takes the smallest colour in [0, K-2] that no neighbour coloured before it holds (its
 * higher-priority neighbours); if all K-1 are taken it joins the leftover class K-1, which,
 * unlike the others, need not be an independent set. K = 1: every vertex in class 0. */
uint64_t orc_vertex_priority(int32_t pass, int64_t v) {
  return splitmix64_finaliser((uint64_t)pass + ((uint64_t)v + 1u) * 0x9E3779B97F4A7C15ull);
}

typedef struct {
  uint64_t prio;
  int32_t v;
} prio_vertex;

static int cmp_prio_desc(const void* a, const void* b) {
  const prio_vertex* x = (const prio_vertex*)a;
  const prio_vertex* y = (const prio_vertex*)b;
  if (x->prio != y->prio) return x->prio > y->prio ? -1 : 1;
  return x->v < y->v ? -1 : (x->v > y->v ? 1 : 0);
}

void orc_colour(int64_t n, const int64_t* off, const int32_t* idx, int32_t pass, int32_t K,
                int32_t* colour) {
  if (K <= 1) {
    for (int64_t v = 0; v < n; v++) colour[v] = 0;
    return;
  }
  prio_vertex* order = (prio_vertex*)malloc(sizeof(prio_vertex) * (size_t)(n > 0 ? n : 1));
  for (int64_t v = 0; v < n; v++) {
    order[v].prio = orc_vertex_priority(pass, v);
    order[v].v = (int32_t)v;
    colour[v] = -1;
  }
  qsort(order, (size_t)n, sizeof(prio_vertex), cmp_prio_desc);
  const uint32_t all = K - 1 >= 32 ? 0xffffffffu : ((1u << (K - 1)) - 1u);
  for (int64_t t = 0; t < n; t++) {
    const int32_t v = order[t].v;
    uint32_t used = 0;
    for (int64_t e = off[v]; e < off[v + 1]; e++) {
      const int32_t u = idx[e];
      if (u != v && colour[u] >= 0 && colour[u] < K - 1) used |= 1u << colour[u];
    }
    int32_t c = K - 1;
    for (int32_t k = 0; k < K - 1; k++)
      if (!((used & all) >> k & 1u)) { c = k; break; }
    colour[v] = c;
  }
  free(order);
}

/* ---------------------------------------------------------------------------------------- */
/* Degrees, total weight, modularity                                                          */
/* ---------------------------------------------------------------------------------------- */

/* K_i = row sums; returns W. */
uint64_t orc_degrees(int64_t n, const int64_t* off, const uint64_t* w, uint64_t* K) {
  uint64_t W = 0;
  for (int64_t i = 0; i < n; i++) {
    uint64_t s = 0;
    for (int64_t e = off[i]; e < off[i + 1]; e++) s += w[e];
    K[i] = s;
    W += s;
  }
  return W;
}

/* Qnum = W * sum_c sigma_c - sum_c Sigma_c^2 for labels C[i] in [0, n).
 * Outputs: qnum (two words), W, sigma_total = sum_c sigma_c. */
void orc_modularity(int64_t n, const int64_t* off, const int32_t* idx, const uint64_t* w,
                    const int32_t* C, uint64_t* qnum_out, uint64_t* W_out,
                    uint64_t* sigma_out) {
  uint64_t* Sig = (uint64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
  uint64_t W = 0, sigma = 0;
  for (int64_t i = 0; i < n; i++) {
    for (int64_t e = off[i]; e < off[i + 1]; e++) {
      W += w[e];
      Sig[C[i]] += w[e];
      if (C[idx[e]] == C[i]) sigma += w[e];
    }
  }
  u128 sq = 0;
  for (int64_t c = 0; c < n; c++) sq += (u128)Sig[c] * Sig[c];
  i128 q = (i128)((u128)W * sigma) - (i128)sq;
  put_i128(qnum_out, q);
  *W_out = W;
  if (sigma_out) *sigma_out = sigma;
  free(Sig);
}

/* Integer threshold of the tolerance test in pass p: floor(W^2 / (2 * 10^(a + b*p))).
 * Zero when the divisor exceeds W^2 (then any positive S continues). */
void orc_threshold(uint64_t W, int32_t a, int32_t b, int32_t pass, uint64_t* out) {
  u128 W2 = (u128)W * W;
  int64_t ex = (int64_t)a + (int64_t)b * pass;
  u128 T = 0;
  if (ex <= 38) {
    u128 div = 2;
    int over = 0;
    for (int64_t k = 0; k < ex; k++) {
      if (div > W2) { over = 1; break; }
      div *= 10;
    }
    if (!over && div <= W2) T = W2 / div;
  }
  out[0] = (uint64_t)T;
  out[1] = (uint64_t)(T >> 64);
}

/* ---------------------------------------------------------------------------------------- */
/* One vertex's decision                                                                       */
/* ---------------------------------------------------------------------------------------- */

typedef struct {
  int32_t target;     /* community after the decision */
  int32_t best;       /* best candidate (or -1 when there is none) */
  i128 gain;          /* g(best) - stay if moving, else 0 */
  i128 stay;          /* g_i(own community) */
  i128 best_gain;     /* g_i(best) */
  int64_t ncand;      /* distinct neighbour communities other than the own one */
} decision;

/* acc: dense scratch of n words, all zero on entry and on exit; list: scratch of >= deg ints.
 * swap_rule: apply singleton-swap prevention (synchronous rule only). */
static decision decide(int64_t i, const int64_t* off, const int32_t* idx, const uint64_t* w,
                       const uint64_t* K, uint64_t W, const int32_t* C, const uint64_t* Sig,
                       const int32_t* csize, int swap_rule, uint64_t* acc, int32_t* list) {
  decision r;
  int32_t d = C[i];
  int64_t nl = 0;
  for (int64_t e = off[i]; e < off[i + 1]; e++) {
    int32_t j = idx[e];
    if (j == i) continue; /* self-loop: not a move candidate, not part of k_{i->x} */
    int32_t c = C[j];
    if (acc[c] == 0) list[nl++] = c; /* weights are >= 1, so zero means "not seen yet" */
    acc[c] += w[e];
  }
  i128 Ki = (i128)K[i];
  i128 kd = (i128)acc[d];
  r.stay = (i128)W * kd - Ki * ((i128)Sig[d] - Ki);
  r.best = -1;
  r.best_gain = 0;
  r.ncand = 0;
  for (int64_t t = 0; t < nl; t++) {
    int32_t c = list[t];
    if (c == d) continue;
    r.ncand++;
    i128 g = (i128)W * (i128)acc[c] - Ki * (i128)Sig[c];
    if (r.best < 0 || g > r.best_gain || (g == r.best_gain && c < r.best)) {
      r.best = c;
      r.best_gain = g;
    }
  }
  for (int64_t t = 0; t < nl; t++) acc[list[t]] = 0;
  r.target = d;
  r.gain = 0;
  if (r.best >= 0 && r.best_gain > r.stay) {
    int blocked = swap_rule && csize[d] == 1 && csize[r.best] == 1 && r.best > d;
    if (!blocked) {
      r.target = r.best;
      r.gain = r.best_gain - r.stay;
    }
  }
  return r;
}

static int64_t max_degree(int64_t n, const int64_t* off) {
  int64_t m = 0;
  for (int64_t i = 0; i < n; i++)
    if (off[i + 1] - off[i] > m) m = off[i + 1] - off[i];
  return m;
}

/* Decisions for a list of vertices under the synchronous rule, against a given state.
 * Used to check sampled vertices of large graphs one by one.
 * Outputs per sampled vertex: target, gain (two words each). */
void orc_decide_sample(int64_t n, const int64_t* off, const int32_t* idx, const uint64_t* w,
                       const uint64_t* K, uint64_t W, const int32_t* C, const uint64_t* Sig,
                       const int32_t* csize, int64_t count, const int64_t* verts,
                       int32_t swap_rule, int32_t* target_out, uint64_t* gain_out,
                       int64_t* ncand_out) {
  uint64_t* acc = (uint64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
  int32_t* list = (int32_t*)malloc(sizeof(int32_t) * (size_t)(max_degree(n, off) + 1));
  for (int64_t t = 0; t < count; t++) {
    decision r = decide(verts[t], off, idx, w, K, W, C, Sig, csize, swap_rule, acc, list);
    target_out[t] = r.target;
    put_i128(gain_out + 2 * t, r.gain);
    if (ncand_out) ncand_out[t] = r.ncand;
  }
  free(list);
  free(acc);
}

/* Every candidate's gain for one vertex (for the single-move identity check).
 * Writes up to cap (community, g) pairs, sorted by community, plus the stay value.
 * Returns the number of candidates. */
int64_t orc_vertex_gains(int64_t n, const int64_t* off, const int32_t* idx, const uint64_t* w,
                         const uint64_t* K, uint64_t W, const int32_t* C, const uint64_t* Sig,
                         int64_t i, int64_t cap, int32_t* comm_out, uint64_t* g_out,
                         uint64_t* stay_out) {
  uint64_t* acc = (uint64_t*)calloc((size_t)n, sizeof(uint64_t));
  char* seen = (char*)calloc((size_t)n, 1);
  int32_t d = C[i];
  for (int64_t e = off[i]; e < off[i + 1]; e++) {
    if (idx[e] == i) continue;
    acc[C[idx[e]]] += w[e];
    seen[C[idx[e]]] = 1;
  }
  i128 Ki = (i128)K[i];
  put_i128(stay_out, (i128)W * (i128)acc[d] - Ki * ((i128)Sig[d] - Ki));
  int64_t cnt = 0;
  for (int64_t c = 0; c < n; c++) {
    if (!seen[c] || c == d) continue;
    if (cnt < cap) {
      comm_out[cnt] = (int32_t)c;
      put_i128(g_out + 2 * cnt, (i128)W * (i128)acc[c] - Ki * (i128)Sig[c]);
    }
    cnt++;
  }
  free(seen);
  free(acc);
  return cnt;
}

/* ---------------------------------------------------------------------------------------- */
/* Local-moving iterations                                                                     */
/* ---------------------------------------------------------------------------------------- */

/* Recompute Sigma and csize from a membership (the definitions, from scratch). */
void orc_community_state(int64_t n, const uint64_t* K, const int32_t* C, uint64_t* Sig,
                         int32_t* csize) {
  memset(Sig, 0, sizeof(uint64_t) * (size_t)n);
  memset(csize, 0, sizeof(int32_t) * (size_t)n);
  for (int64_t i = 0; i < n; i++) {
    Sig[C[i]] += K[i];
    csize[C[i]] += 1;
  }
}

/* One synchronous (Jacobi) step over a set of vertices: every listed vertex decides from
 * (C, Sig, csize) as given, then the new memberships are written and Sigma/csize are
 * recomputed. Unlisted vertices keep their community. verts == NULL means all vertices.
 * In/out: C, Sig, csize. Out: S (two words), moved count, candidate-pair count.
 * nthreads <= 0 uses the OpenMP default; the result does not depend on it. */
void orc_sync_step(int64_t n, const int64_t* off, const int32_t* idx, const uint64_t* w,
                   const uint64_t* K, uint64_t W, int32_t* C, uint64_t* Sig, int32_t* csize,
                   const int32_t* verts, int64_t nverts, int32_t nthreads, uint64_t* S_out,
                   int64_t* moved_out, int64_t* ncand_out) {
  int64_t m = verts ? nverts : n;
  int32_t* Cn = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  i128* gain = (i128*)malloc(sizeof(i128) * (size_t)(m > 0 ? m : 1));
  int64_t* nc = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
  int64_t maxdeg = max_degree(n, off);
  memcpy(Cn, C, sizeof(int32_t) * (size_t)n);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel
  {
    uint64_t* acc = (uint64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
    int32_t* list = (int32_t*)malloc(sizeof(int32_t) * (size_t)(maxdeg + 1));
#pragma omp for schedule(dynamic, 1024)
    for (int64_t t = 0; t < m; t++) {
      int64_t i = verts ? verts[t] : t;
      decision r = decide(i, off, idx, w, K, W, C, Sig, csize, 1, acc, list);
      Cn[i] = r.target;
      gain[t] = r.gain;
      nc[t] = r.ncand;
    }
    free(list);
    free(acc);
  }
  i128 S = 0;
  int64_t moved = 0, ncand = 0;
  for (int64_t t = 0; t < m; t++) {
    int64_t i = verts ? verts[t] : t;
    S += gain[t];
    moved += (Cn[i] != C[i]);
    ncand += nc[t];
  }
  memcpy(C, Cn, sizeof(int32_t) * (size_t)n);
  orc_community_state(n, K, C, Sig, csize);
  put_i128(S_out, S);
  *moved_out = moved;
  if (ncand_out) *ncand_out = ncand;
  free(nc);
  free(gain);
  free(Cn);
}

/* One synchronous (Jacobi) iteration: a step over all vertices. */
void orc_sync_iteration(int64_t n, const int64_t* off, const int32_t* idx, const uint64_t* w,
                        const uint64_t* K, uint64_t W, int32_t* C, uint64_t* Sig,
                        int32_t* csize, int32_t nthreads, uint64_t* S_out, int64_t* moved_out,
                        int64_t* ncand_out) {
  orc_sync_step(n, off, idx, w, K, W, C, Sig, csize, NULL, 0, nthreads, S_out, moved_out,
                ncand_out);
}

/* One asynchronous (Gauss-Seidel) iteration: vertices in ascending id, each decision sees
 * every earlier move of the same iteration; no singleton-swap rule. In/out: C, Sig, csize. */
void orc_async_iteration(int64_t n, const int64_t* off, const int32_t* idx, const uint64_t* w,
                         const uint64_t* K, uint64_t W, int32_t* C, uint64_t* Sig,
                         int32_t* csize, uint64_t* S_out, int64_t* moved_out) {
  uint64_t* acc = (uint64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
  int32_t* list = (int32_t*)malloc(sizeof(int32_t) * (size_t)(max_degree(n, off) + 1));
  i128 S = 0;
  int64_t moved = 0;
  for (int64_t i = 0; i < n; i++) {
    decision r = decide(i, off, idx, w, K, W, C, Sig, csize, 0, acc, list);
    if (r.target != C[i]) {
      int32_t d = C[i], c = r.target;
      Sig[d] -= K[i];
      Sig[c] += K[i];
      csize[d] -= 1;
      csize[c] += 1;
      C[i] = c;
      S += r.gain;
      moved++;
    }
  }
  put_i128(S_out, S);
  *moved_out = moved;
  free(list);
  free(acc);
}

/* ---------------------------------------------------------------------------------------- */
/* Aggregation                                                                                 */
/* ---------------------------------------------------------------------------------------- */

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Collapse each community into a super-vertex (section 3.2's aggregation phase): labels are
 * renumbered by ascending rank among used labels; the super-arc (a, b) weighs the sum of the
 * arcs (i, j) with new ids (a, b), so arcs inside a community become the self-loop of its
 * super-vertex. Rows of the output are sorted by neighbour id.
 * Outputs: map[n] (new id of each vertex), off_out[n+1], idx_out[<=nnz], w_out[<=nnz]
 * (caller-sized to the input), n_out, nnz_out. */
void orc_aggregate(int64_t n, const int64_t* off, const int32_t* idx, const uint64_t* w,
                   const int32_t* C, int32_t* map, int64_t* off_out, int32_t* idx_out,
                   uint64_t* w_out, int64_t* n_out, int64_t* nnz_out) {
  int32_t* newid = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  char* used = (char*)calloc((size_t)(n > 0 ? n : 1), 1);
  for (int64_t i = 0; i < n; i++) used[C[i]] = 1;
  int64_t nn = 0;
  for (int64_t c = 0; c < n; c++) newid[c] = used[c] ? (int32_t)nn++ : -1;
  for (int64_t i = 0; i < n; i++) map[i] = newid[C[i]];
  /* members of each super-vertex (counting sort by new id) */
  int64_t* mstart = (int64_t*)calloc((size_t)nn + 1, sizeof(int64_t));
  for (int64_t i = 0; i < n; i++) mstart[map[i] + 1]++;
  for (int64_t a = 0; a < nn; a++) mstart[a + 1] += mstart[a];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nn + 1));
  memcpy(fill, mstart, sizeof(int64_t) * (size_t)(nn + 1));
  int32_t* members = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; i++) members[fill[map[i]]++] = (int32_t)i;
  /* one super row at a time: dense accumulation, then emit neighbours in ascending order */
  uint64_t* acc = (uint64_t*)calloc((size_t)(nn > 0 ? nn : 1), sizeof(uint64_t));
  char* seen = (char*)calloc((size_t)(nn > 0 ? nn : 1), 1);
  int32_t* list = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nn > 0 ? nn : 1));
  int64_t pos = 0;
  off_out[0] = 0;
  for (int64_t a = 0; a < nn; a++) {
    int64_t nl = 0;
    for (int64_t m = mstart[a]; m < mstart[a + 1]; m++) {
      int32_t i = members[m];
      for (int64_t e = off[i]; e < off[i + 1]; e++) {
        int32_t b = map[idx[e]];
        if (!seen[b]) { seen[b] = 1; list[nl++] = b; }
        acc[b] += w[e];
      }
    }
    /* emit the neighbours in ascending order */
    qsort(list, (size_t)nl, sizeof(int32_t), cmp_i32);
    for (int64_t t = 0; t < nl; t++) {
      idx_out[pos] = list[t];
      w_out[pos] = acc[list[t]];
      pos++;
      acc[list[t]] = 0;
      seen[list[t]] = 0;
    }
    off_out[a + 1] = pos;
  }
  *n_out = nn;
  *nnz_out = pos;
  free(list);
  free(seen);
  free(acc);
  free(members);
  free(fill);
  free(mstart);
  free(used);
  free(newid);
}

/* ---------------------------------------------------------------------------------------- */
/* Whole run                                                                                   */
/* ---------------------------------------------------------------------------------------- */

#define ORC_MAX_PASSES 64
#define ORC_MAX_TRACE 4096

typedef struct {
  int32_t passes;            /* passes that ran a local-moving phase */
  int32_t iterations_total;
  int32_t iterations[ORC_MAX_PASSES];
  int64_t n_pass[ORC_MAX_PASSES];   /* vertices of the graph each pass ran on */
  int64_t nnz_pass[ORC_MAX_PASSES];
  int32_t cap_hits;          /* phases stopped by max_iterations */
  int32_t n_trace;           /* iterations recorded below (capped at ORC_MAX_TRACE) */
  int32_t trace_pass[ORC_MAX_TRACE];
  int64_t trace_moved[ORC_MAX_TRACE];
  uint64_t trace_S[2 * ORC_MAX_TRACE];
  int64_t trace_ncand[ORC_MAX_TRACE];
  uint64_t qnum_pass[2 * ORC_MAX_PASSES]; /* Qnum(G_p, C) after each local-moving phase */
  int64_t n_communities;
  uint64_t W;
  uint64_t qnum[2];
} orc_result;

static int64_t* copy64(const int64_t* a, int64_t k) {
  int64_t* r = (int64_t*)malloc(sizeof(int64_t) * (size_t)(k > 0 ? k : 1));
  memcpy(r, a, sizeof(int64_t) * (size_t)k);
  return r;
}

/* The Louvain method of section 3.2, passes of local-moving + aggregation.
 * mode 0: synchronous rule (the GPU's rule); mode 1: sequential asynchronous rule.
 * substeps (mode 0): K vertex classes; an iteration is K synchronous steps, class 0 first,
 * each seeing the moves of the classes before it (K = 1: fully synchronous).
 * a, b: initial tolerance 10^-a, decline factor 10^b (defaults 2 and 1, section 3.2).
 * top[n]: output membership (dense labels of the last level).
 * levels (may be NULL): levels[l*n + v] = community of input vertex v after the l-th
 * aggregation, for l < *n_levels <= max_levels; the hierarchy the passes build (section 3.2:
 * each pass's communities become the vertices of the next). */
static int run_impl(int64_t n, const int64_t* off0, const int32_t* idx0, const uint64_t* w0,
                    int32_t mode, int32_t a, int32_t b, int32_t max_it, int32_t max_pass,
                    int32_t substeps, int32_t nthreads, int32_t colour_classes, int32_t* top,
                    orc_result* res, int32_t* levels, int32_t max_levels, int32_t* n_levels) {
  memset(res, 0, sizeof(*res));
  if (n_levels) *n_levels = 0;
  for (int64_t v = 0; v < n; v++) top[v] = (int32_t)v;
  int64_t nnz0 = n > 0 ? off0[n] : 0;
  uint64_t* K = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
  uint64_t W = orc_degrees(n, off0, w0, K);
  res->W = W;
  res->n_communities = n;
  if (W == 0) {
    free(K);
    return 0;
  }
  /* the current graph: starts as the input, then each pass's super-vertex graph */
  int64_t cn = n, cnnz = nnz0;
  int64_t* off = copy64(off0, n + 1);
  int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz0 > 0 ? nnz0 : 1));
  uint64_t* w = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(nnz0 > 0 ? nnz0 : 1));
  memcpy(idx, idx0, sizeof(int32_t) * (size_t)nnz0);
  memcpy(w, w0, sizeof(uint64_t) * (size_t)nnz0);
  int32_t* C = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  uint64_t* Sig = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  int32_t* csize = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* map = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int64_t* off2 = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int32_t* idx2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz0 > 0 ? nnz0 : 1));
  uint64_t* w2 = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(nnz0 > 0 ? nnz0 : 1));
  int32_t* cls_verts = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int64_t* cls_start = (int64_t*)malloc(sizeof(int64_t) * (size_t)(substeps + 1));
  int32_t* colour = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (substeps < 1) substeps = 1;

  for (int32_t p = 0; p < max_pass && p < ORC_MAX_PASSES; p++) {
    /* every vertex starts in its own community; K of a super-vertex is its row sum */
    orc_degrees(cn, off, w, K);
    for (int64_t i = 0; i < cn; i++) { C[i] = (int32_t)i; Sig[i] = K[i]; csize[i] = 1; }
    /* modularity before the pass: every vertex of the current graph alone, i.e. the partition
     * of the previous level (aggregation keeps modularity) */
    i128 q_before;
    {
      uint64_t qb[2], Wq = 0;
      orc_modularity(cn, off, idx, w, C, qb, &Wq, NULL);
      q_before = (i128)((u128)qb[0] | ((u128)qb[1] << 64));
    }
    uint64_t Tw[2];
    orc_threshold(W, a, b, p, Tw);
    u128 T = (u128)Tw[0] | ((u128)Tw[1] << 64);
    res->n_pass[p] = cn;
    res->nnz_pass[p] = cnnz;
    res->passes = p + 1;
    /* vertices of each class, ascending within a class: hashed classes, or colour classes */
    {
      if (colour_classes) orc_colour(cn, off, idx, p, substeps, colour);
      int64_t pos = 0;
      for (int32_t k = 0; k < substeps; k++) {
        cls_start[k] = pos;
        for (int64_t v = 0; v < cn; v++) {
          const int32_t cls = substeps == 1 ? 0
                              : colour_classes ? colour[v] : orc_vertex_class(p, substeps, v);
          if (cls == k) cls_verts[pos++] = (int32_t)v;
        }
      }
      cls_start[substeps] = pos;
    }
    int32_t iters = 0, below_tolerance = 0;
    for (int32_t it = 0; it < max_it; it++) {
      uint64_t Sw[2];
      int64_t moved = 0, ncand = 0;
      i128 S = 0;
      if (mode == 0) {
        for (int32_t k = 0; k < substeps; k++) {
          int64_t mk = 0, nk = 0;
          orc_sync_step(cn, off, idx, w, K, W, C, Sig, csize, cls_verts + cls_start[k],
                        cls_start[k + 1] - cls_start[k], nthreads, Sw, &mk, &nk);
          S += (i128)((u128)Sw[0] | ((u128)Sw[1] << 64));
          moved += mk;
          ncand += nk;
        }
      } else {
        orc_async_iteration(cn, off, idx, w, K, W, C, Sig, csize, Sw, &moved);
        S = (i128)((u128)Sw[0] | ((u128)Sw[1] << 64));
      }
      put_i128(Sw, S);
      if (res->n_trace < ORC_MAX_TRACE) {
        int32_t t = res->n_trace++;
        res->trace_pass[t] = p;
        res->trace_moved[t] = moved;
        res->trace_S[2 * t] = Sw[0];
        res->trace_S[2 * t + 1] = Sw[1];
        res->trace_ncand[t] = ncand;
      }
      iters++;
      if (!((u128)S > T)) { below_tolerance = 1; break; } /* the moves just made are kept */
    }
    if (!below_tolerance) res->cap_hits++; /* the phase ran out of iterations */
    res->iterations[p] = iters;
    res->iterations_total += iters;
    i128 q_after;
    {
      uint64_t Wq = 0;
      orc_modularity(cn, off, idx, w, C, res->qnum_pass + 2 * p, &Wq, NULL);
      q_after = (i128)((u128)res->qnum_pass[2 * p] | ((u128)res->qnum_pass[2 * p + 1] << 64));
    }
    /* pass_tolerance = 0: a pass whose increase in modularity is not above it ends the run and
     * its partition is dropped (when nothing moved, it is the previous level anyway) */
    if (!(q_after > q_before)) break;
    int64_t nn = 0, nnz2 = 0;
    orc_aggregate(cn, off, idx, w, C, map, off2, idx2, w2, &nn, &nnz2);
    for (int64_t v = 0; v < n; v++) top[v] = map[top[v]];
    if (levels && n_levels && *n_levels < max_levels) {
      memcpy(levels + (size_t)(*n_levels) * (size_t)n, top, sizeof(int32_t) * (size_t)n);
      (*n_levels)++;
    }
    int shrunk = nn < cn;
    /* the super-vertex graph becomes the current graph */
    memcpy(off, off2, sizeof(int64_t) * (size_t)(nn + 1));
    memcpy(idx, idx2, sizeof(int32_t) * (size_t)nnz2);
    memcpy(w, w2, sizeof(uint64_t) * (size_t)nnz2);
    cn = nn;
    cnnz = nnz2;
    if (!shrunk) break;
  }
  res->n_communities = cn;
  uint64_t Wq = 0;
  orc_modularity(n, off0, idx0, w0, top, res->qnum, &Wq, NULL);
  free(colour); free(cls_start); free(cls_verts);
  free(w2); free(idx2); free(off2); free(map); free(csize); free(Sig); free(C);
  free(w); free(idx); free(off); free(K);
  return 0;
}

int orc_run(int64_t n, const int64_t* off0, const int32_t* idx0, const uint64_t* w0,
            int32_t mode, int32_t a, int32_t b, int32_t max_it, int32_t max_pass,
            int32_t substeps, int32_t nthreads, int32_t* top, orc_result* res) {
  return run_impl(n, off0, idx0, w0, mode, a, b, max_it, max_pass, substeps, nthreads, 0, top,
                  res, NULL, 0, NULL);
}

/* orc_run with every option: colour_classes selects colour classes (orc_colour) instead of
 * hashed ones; levels (may be NULL) keeps every level of the hierarchy (levels[max_levels*n]). */
int orc_run_opts(int64_t n, const int64_t* off0, const int32_t* idx0, const uint64_t* w0,
                 int32_t mode, int32_t a, int32_t b, int32_t max_it, int32_t max_pass,
                 int32_t substeps, int32_t nthreads, int32_t colour_classes, int32_t* top,
                 orc_result* res, int32_t* levels, int32_t max_levels, int32_t* n_levels) {
  return run_impl(n, off0, idx0, w0, mode, a, b, max_it, max_pass, substeps, nthreads,
                  colour_classes, top, res, levels, max_levels, n_levels);
}

/* ---------------------------------------------------------------------------------------------
 * Graph preparation (section 3.1.2 and Table 1, the datasets): every edge is taken as undirected by
 * adding its reverse, edges get a default weight of one, and every vertex receives a self-loop.
 * Written as its plain definition: list every arc, sort the list by (source, neighbour), and
 * combine equal arcs.
 * flags: ORC_PREP_SYM adds (v, u, w) for every edge (u, v, w) with u != v (a self-loop stays one
 * arc); ORC_PREP_LOOPS adds (v, v, 1) for every vertex; equal arcs combine by sum, or by max
 * with ORC_PREP_MAX (which keeps unit weights at one). w == NULL means every weight is 1.
 * Output: off[n+1], idx[nnz], wout[nnz] with rows sorted by neighbour and no repeated
 * neighbour. Returns nnz, or -1 if an endpoint is outside [0, n) or a weight is 0. */
#define ORC_PREP_SYM 0x1u
#define ORC_PREP_LOOPS 0x2u
#define ORC_PREP_MAX 0x4u

typedef struct {
  int32_t u, v;
  uint64_t w;
} prep_arc;

static int cmp_prep_arc(const void* a, const void* b) {
  const prep_arc* x = (const prep_arc*)a;
  const prep_arc* y = (const prep_arc*)b;
  if (x->u != y->u) return x->u < y->u ? -1 : 1;
  if (x->v != y->v) return x->v < y->v ? -1 : 1;
  return 0;
}

int64_t orc_prepare(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                    const uint32_t* w, uint32_t flags, int64_t* off, int32_t* idx,
                    uint64_t* wout) {
  for (int64_t e = 0; e < m; e++) {
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return -1;
    if (w && w[e] == 0) return -1;
  }
  const int64_t cap = m * ((flags & ORC_PREP_SYM) ? 2 : 1) + ((flags & ORC_PREP_LOOPS) ? n : 0);
  prep_arc* a = (prep_arc*)malloc(sizeof(prep_arc) * (size_t)(cap > 0 ? cap : 1));
  int64_t k = 0;
  for (int64_t e = 0; e < m; e++) {
    const uint64_t we = w ? w[e] : 1;
    a[k].u = src[e]; a[k].v = dst[e]; a[k].w = we; k++;
    if ((flags & ORC_PREP_SYM) && src[e] != dst[e]) {
      a[k].u = dst[e]; a[k].v = src[e]; a[k].w = we; k++;
    }
  }
  if (flags & ORC_PREP_LOOPS)
    for (int64_t v = 0; v < n; v++) { a[k].u = (int32_t)v; a[k].v = (int32_t)v; a[k].w = 1; k++; }
  qsort(a, (size_t)k, sizeof(prep_arc), cmp_prep_arc);
  int64_t nnz = 0;
  for (int64_t v = 0; v <= n; v++) off[v] = 0;
  for (int64_t i = 0; i < k; i++) {
    if (nnz > 0 && idx[nnz - 1] == a[i].v && i > 0 && a[i - 1].u == a[i].u) {
      if (flags & ORC_PREP_MAX) {
        if (a[i].w > wout[nnz - 1]) wout[nnz - 1] = a[i].w;
      } else {
        wout[nnz - 1] += a[i].w;
      }
      continue;
    }
    idx[nnz] = a[i].v;
    wout[nnz] = a[i].w;
    off[a[i].u + 1]++;
    nnz++;
  }
  for (int64_t v = 0; v < n; v++) off[v + 1] += off[v];
  free(a);
  return nnz;
}

/* ---------------------------------------------------------------------------------------------
 * Partition and merge (the remedy the paper proposes in section 3.2 and its conclusion for the
 * poor multi-threaded scaling: run partitions of the graph independently, then combine them).
 * Parts are the contiguous vertex ranges [vptr[k], vptr[k+1]). Each part's induced subgraph
 * (the arcs with both ends in the part, ids local to the part) runs the whole method on its own
 * (orc_run with the given rule and parameters). The part communities, numbered part after part,
 * partition the whole graph; the whole graph (every arc, cross-part ones included) is
 * aggregated by that partition, and the method runs again on the super-vertex graph: the merge.
 * top[n]: the final membership (merge community of each vertex's part community).
 * part_comms[P], part_qnum[2P] (may be NULL): communities and W_k^2 Q_k of every part's run;
 * res: the merge run's result (its Q is the final partition's Q on the whole graph). */
int orc_run_partitioned(int64_t n, const int64_t* off, const int32_t* idx, const uint64_t* w,
                        int32_t P, const int64_t* vptr, int32_t mode, int32_t a, int32_t b,
                        int32_t max_it, int32_t max_pass, int32_t substeps, int32_t nthreads,
                        int32_t* top, int64_t* part_comms, uint64_t* part_qnum,
                        orc_result* res) {
  const int64_t nnz = n > 0 ? off[n] : 0;
  int32_t* label = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int64_t* poff = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int32_t* pidx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  uint64_t* pw = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(nnz > 0 ? nnz : 1));
  orc_result* pres = (orc_result*)malloc(sizeof(orc_result));
  int64_t next_label = 0;
  for (int32_t k = 0; k < P; k++) {
    const int64_t v0 = vptr[k], v1 = vptr[k + 1], nk = v1 - v0;
    /* the induced subgraph of part k, local ids */
    int64_t e2 = 0;
    poff[0] = 0;
    for (int64_t v = v0; v < v1; v++) {
      for (int64_t e = off[v]; e < off[v + 1]; e++)
        if (idx[e] >= v0 && idx[e] < v1) {
          pidx[e2] = (int32_t)(idx[e] - v0);
          pw[e2] = w[e];
          e2++;
        }
      poff[v - v0 + 1] = e2;
    }
    run_impl(nk, poff, pidx, pw, mode, a, b, max_it, max_pass, substeps, nthreads, 0,
             label + v0, pres, NULL, 0, NULL);
    for (int64_t v = v0; v < v1; v++) label[v] += (int32_t)next_label;
    next_label += pres->n_communities;
    if (part_comms) part_comms[k] = pres->n_communities;
    if (part_qnum) {
      part_qnum[2 * k] = pres->qnum[0];
      part_qnum[2 * k + 1] = pres->qnum[1];
    }
  }
  /* the merge: aggregate the whole graph by the part communities, run on the super graph */
  int32_t* map = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int64_t* soff = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int32_t* sidx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  uint64_t* sw = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(nnz > 0 ? nnz : 1));
  int64_t sn = 0, snnz = 0;
  if (n > 0) orc_aggregate(n, off, idx, w, label, map, soff, sidx, sw, &sn, &snnz);
  else soff[0] = 0;
  int32_t* stop = (int32_t*)malloc(sizeof(int32_t) * (size_t)(sn > 0 ? sn : 1));
  run_impl(sn, soff, sidx, sw, mode, a, b, max_it, max_pass, substeps, nthreads, 0, stop, res,
           NULL, 0, NULL);
  for (int64_t v = 0; v < n; v++) top[v] = stop[map[v]];
  free(stop); free(sw); free(sidx); free(soff); free(map);
  free(pres); free(pw); free(pidx); free(poff); free(label);
  return 0;
}
