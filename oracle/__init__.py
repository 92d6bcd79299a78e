"""ctypes binding of the Louvain oracle (plain C, ``louvain_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU-baseline leg
use it. The GPU library never imports or links it.

Graphs are passed as numpy arrays: offsets int64[n+1], indices int32[nnz], weights
uint64[nnz]. 128-bit results come back as Python ints.
"""

import ctypes
import os

import numpy as np

from . import build as _build

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

MAX_PASSES = 64
MAX_TRACE = 4096


class OrcResult(ctypes.Structure):
    _fields_ = [
        ("passes", ctypes.c_int32),
        ("iterations_total", ctypes.c_int32),
        ("iterations", ctypes.c_int32 * MAX_PASSES),
        ("n_pass", ctypes.c_int64 * MAX_PASSES),
        ("nnz_pass", ctypes.c_int64 * MAX_PASSES),
        ("cap_hits", ctypes.c_int32),
        ("n_trace", ctypes.c_int32),
        ("trace_pass", ctypes.c_int32 * MAX_TRACE),
        ("trace_moved", ctypes.c_int64 * MAX_TRACE),
        ("trace_S", ctypes.c_uint64 * (2 * MAX_TRACE)),
        ("trace_ncand", ctypes.c_int64 * MAX_TRACE),
        ("qnum_pass", ctypes.c_uint64 * (2 * MAX_PASSES)),
        ("n_communities", ctypes.c_int64),
        ("W", ctypes.c_uint64),
        ("qnum", ctypes.c_uint64 * 2),
    ]


def _i128(lo: int, hi: int) -> int:
    v = (int(hi) << 64) | int(lo)
    return v - (1 << 128) if v >= (1 << 127) else v


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        _LIB = ctypes.CDLL(path)
    return _LIB


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Graph:
    """Host copy of a symmetric CSR for the oracle."""

    def __init__(self, n, offsets, indices, weights):
        self.n = int(n)
        self.off = np.ascontiguousarray(offsets, dtype=np.int64)
        self.idx = np.ascontiguousarray(indices, dtype=np.int32)
        self.w = np.ascontiguousarray(weights, dtype=np.uint64)
        assert self.off.shape == (self.n + 1,)
        assert self.idx.shape == self.w.shape == (int(self.off[-1]) if self.n else 0,)

    @property
    def nnz(self):
        return int(self.idx.shape[0])

    @staticmethod
    def from_csr(g):
        """From a ``graphgen.Csr`` (torch tensors on any device; weights reinterpreted as
        unsigned)."""
        import torch
        w = g.weights.cpu()
        if w.dtype == torch.int32:
            w = w.numpy().view(np.uint32).astype(np.uint64)
        else:
            w = w.numpy().view(np.uint64)
        return Graph(g.n, g.offsets.cpu().numpy().astype(np.int64),
                     g.indices.cpu().numpy(), w)

    def args(self):
        return (ctypes.c_int64(self.n), _p(self.off), _p(self.idx), _p(self.w))


def degrees(g: Graph):
    K = np.zeros(g.n, dtype=np.uint64)
    W = lib().orc_degrees
    W.restype = ctypes.c_uint64
    tot = W(ctypes.c_int64(g.n), _p(g.off), _p(g.w), _p(K))
    return K, int(tot)


def modularity(g: Graph, C):
    """(Qnum, W, sigma_total) for membership C (labels in [0, n))."""
    C = np.ascontiguousarray(C, dtype=np.int32)
    q = np.zeros(2, dtype=np.uint64)
    W = np.zeros(1, dtype=np.uint64)
    s = np.zeros(1, dtype=np.uint64)
    lib().orc_modularity(*g.args(), _p(C), _p(q), _p(W), _p(s))
    return _i128(q[0], q[1]), int(W[0]), int(s[0])


def threshold(W: int, a: int, b: int, p: int) -> int:
    out = np.zeros(2, dtype=np.uint64)
    lib().orc_threshold(ctypes.c_uint64(W), ctypes.c_int32(a), ctypes.c_int32(b),
                        ctypes.c_int32(p), _p(out))
    return int(out[0]) | (int(out[1]) << 64)


def community_state(g: Graph, K, C):
    Sig = np.zeros(g.n, dtype=np.uint64)
    cs = np.zeros(g.n, dtype=np.int32)
    lib().orc_community_state(ctypes.c_int64(g.n), _p(K), _p(np.ascontiguousarray(C, np.int32)),
                              _p(Sig), _p(cs))
    return Sig, cs


class State:
    """Local-moving state of one pass: K, W, C, Sigma, csize (numpy, mutable)."""

    def __init__(self, g: Graph, C=None):
        self.K, self.W = degrees(g)
        self.C = np.arange(g.n, dtype=np.int32) if C is None else np.array(C, dtype=np.int32)
        self.Sig, self.csize = community_state(g, self.K, self.C)

    def copy(self):
        s = State.__new__(State)
        s.K, s.W = self.K.copy(), self.W
        s.C, s.Sig, s.csize = self.C.copy(), self.Sig.copy(), self.csize.copy()
        return s


def sync_iteration(g: Graph, st: State, nthreads: int = 0):
    """One synchronous iteration in place on ``st``; returns (S, moved, candidate pairs)."""
    S = np.zeros(2, dtype=np.uint64)
    moved = ctypes.c_int64(0)
    nc = ctypes.c_int64(0)
    lib().orc_sync_iteration(*g.args(), _p(st.K), ctypes.c_uint64(st.W), _p(st.C), _p(st.Sig),
                             _p(st.csize), ctypes.c_int32(nthreads), _p(S),
                             ctypes.byref(moved), ctypes.byref(nc))
    return _i128(S[0], S[1]), moved.value, nc.value


def vertex_class(p: int, K: int, v: int) -> int:
    f = lib().orc_vertex_class
    f.restype = ctypes.c_int32
    return int(f(ctypes.c_int32(p), ctypes.c_int32(K), ctypes.c_int64(v)))


def sync_step(g: Graph, st: State, verts, nthreads: int = 0):
    """One synchronous step over the listed vertices (others keep their community), in place;
    returns (S, moved, candidate pairs)."""
    verts = np.ascontiguousarray(verts, dtype=np.int32)
    S = np.zeros(2, dtype=np.uint64)
    moved = ctypes.c_int64(0)
    nc = ctypes.c_int64(0)
    lib().orc_sync_step(*g.args(), _p(st.K), ctypes.c_uint64(st.W), _p(st.C), _p(st.Sig),
                        _p(st.csize), _p(verts), ctypes.c_int64(verts.shape[0]),
                        ctypes.c_int32(nthreads), _p(S), ctypes.byref(moved), ctypes.byref(nc))
    return _i128(S[0], S[1]), moved.value, nc.value


def class_lists(n: int, p: int, K: int):
    """Vertices of each class of pass p (ascending)."""
    verts = np.zeros(max(n, 1), dtype=np.int32)
    start = np.zeros(K + 1, dtype=np.int64)
    lib().orc_class_lists(ctypes.c_int64(n), ctypes.c_int32(p), ctypes.c_int32(K), _p(verts),
                          _p(start))
    return [verts[start[k]:start[k + 1]].copy() for k in range(K)]


def substep_iteration(g: Graph, st: State, p: int, K: int, classes=None):
    """One iteration of K class steps in place; returns (S, moved, candidate pairs)."""
    if classes is None:
        classes = class_lists(g.n, p, K)
    S = moved = nc = 0
    for vs in classes:
        a, b, c = sync_step(g, st, vs)
        S += a
        moved += b
        nc += c
    return S, moved, nc


def async_iteration(g: Graph, st: State):
    """One asynchronous (ascending-id) iteration in place; returns (S, moved)."""
    S = np.zeros(2, dtype=np.uint64)
    moved = ctypes.c_int64(0)
    lib().orc_async_iteration(*g.args(), _p(st.K), ctypes.c_uint64(st.W), _p(st.C), _p(st.Sig),
                              _p(st.csize), _p(S), ctypes.byref(moved))
    return _i128(S[0], S[1]), moved.value


def decide_sample(g: Graph, st: State, verts, swap_rule: bool = True):
    """Synchronous-rule decisions of the listed vertices against state ``st`` (not modified).
    Returns (targets int32, gains list of int, candidate counts int64)."""
    verts = np.ascontiguousarray(verts, dtype=np.int64)
    t = np.zeros(verts.shape[0], dtype=np.int32)
    gw = np.zeros(2 * verts.shape[0], dtype=np.uint64)
    nc = np.zeros(verts.shape[0], dtype=np.int64)
    lib().orc_decide_sample(*g.args(), _p(st.K), ctypes.c_uint64(st.W), _p(st.C), _p(st.Sig),
                            _p(st.csize), ctypes.c_int64(verts.shape[0]), _p(verts),
                            ctypes.c_int32(1 if swap_rule else 0), _p(t), _p(gw), _p(nc))
    gains = [_i128(gw[2 * k], gw[2 * k + 1]) for k in range(verts.shape[0])]
    return t, gains, nc


def vertex_gains(g: Graph, st: State, i: int):
    """({community: g_i(community)} over candidate communities other than C[i], stay value)."""
    cap = g.n
    comm = np.zeros(cap, dtype=np.int32)
    gw = np.zeros(2 * cap, dtype=np.uint64)
    stay = np.zeros(2, dtype=np.uint64)
    f = lib().orc_vertex_gains
    f.restype = ctypes.c_int64
    cnt = f(*g.args(), _p(st.K), ctypes.c_uint64(st.W), _p(st.C), _p(st.Sig),
            ctypes.c_int64(i), ctypes.c_int64(cap), _p(comm), _p(gw), _p(stay))
    gains = {int(comm[k]): _i128(gw[2 * k], gw[2 * k + 1]) for k in range(cnt)}
    return gains, _i128(stay[0], stay[1])


def aggregate(g: Graph, C):
    """Super-vertex graph of membership C: (map, Graph') with rows sorted."""
    C = np.ascontiguousarray(C, dtype=np.int32)
    mp = np.zeros(g.n, dtype=np.int32)
    off = np.zeros(g.n + 1, dtype=np.int64)
    idx = np.zeros(max(g.nnz, 1), dtype=np.int32)
    w = np.zeros(max(g.nnz, 1), dtype=np.uint64)
    nn = ctypes.c_int64(0)
    nz = ctypes.c_int64(0)
    lib().orc_aggregate(*g.args(), _p(C), _p(mp), _p(off), _p(idx), _p(w),
                        ctypes.byref(nn), ctypes.byref(nz))
    n2, z2 = nn.value, nz.value
    return mp, Graph(n2, off[:n2 + 1].copy(), idx[:z2].copy(), w[:z2].copy())


def run(g: Graph, mode: str = "sync", a: int = 2, b: int = 1, max_iterations: int = 20,
        max_passes: int = 10, substeps: int = 1, nthreads: int = 0, levels: bool = False,
        colour: bool = False):
    """Whole Louvain run. Returns (membership int32[n], result dict).
    mode "sync": synchronous rule, an iteration being ``substeps`` class steps;
    mode "async": sequential asynchronous rule.
    levels: also return, as result["levels"] (int32[L, n]), the membership of the input
    vertices after each of the L aggregations (the last one equals the membership).
    colour: the classes of every pass are colour classes (``colour_classes``), not hashed."""
    top = np.zeros(max(g.n, 1), dtype=np.int32)
    r = OrcResult()
    max_levels = max(1, min(max_passes, MAX_PASSES))
    lv = np.zeros((max_levels, max(g.n, 1)), dtype=np.int32) if levels else None
    nl = ctypes.c_int32(0)
    lib().orc_run_opts(*g.args(), ctypes.c_int32(0 if mode == "sync" else 1), ctypes.c_int32(a),
                       ctypes.c_int32(b), ctypes.c_int32(max_iterations),
                       ctypes.c_int32(max_passes), ctypes.c_int32(substeps),
                       ctypes.c_int32(nthreads), ctypes.c_int32(1 if colour else 0), _p(top),
                       ctypes.byref(r), _p(lv) if levels else None,
                       ctypes.c_int32(max_levels), ctypes.byref(nl))
    nt = r.n_trace
    res = {
        "passes": r.passes,
        "iterations_total": r.iterations_total,
        "iterations": [r.iterations[p] for p in range(r.passes)],
        "n_pass": [r.n_pass[p] for p in range(r.passes)],
        "nnz_pass": [r.nnz_pass[p] for p in range(r.passes)],
        "cap_hits": r.cap_hits,
        "trace_pass": [r.trace_pass[t] for t in range(nt)],
        "trace_moved": [r.trace_moved[t] for t in range(nt)],
        "trace_S": [_i128(r.trace_S[2 * t], r.trace_S[2 * t + 1]) for t in range(nt)],
        "trace_ncand": [r.trace_ncand[t] for t in range(nt)],
        "qnum_pass": [_i128(r.qnum_pass[2 * p], r.qnum_pass[2 * p + 1]) for p in range(r.passes)],
        "n_communities": r.n_communities,
        "W": r.W,
        "qnum": _i128(r.qnum[0], r.qnum[1]),
    }
    res["q"] = (res["qnum"] / (res["W"] * res["W"])) if res["W"] else 0.0
    if levels:
        res["levels"] = lv[:nl.value, :g.n].copy()
    return top[:g.n].copy(), res


# ----------------------------------------------------------------------------------------------
# graph preparation (section 3.1.2 and Table 1): edge list -> undirected weighted CSR

PREP_SYM = 0x1
PREP_LOOPS = 0x2
PREP_MAX = 0x4


def vertex_priority(p: int, v: int) -> int:
    f = lib().orc_vertex_priority
    f.restype = ctypes.c_uint64
    return int(f(ctypes.c_int32(p), ctypes.c_int64(v)))


def colour_classes(g: Graph, p: int, K: int):
    """Colour class (0..K-1) of every vertex of g in pass p: first-fit colouring in descending
    priority order, colours 0..K-2, the rest in class K-1."""
    out = np.zeros(max(g.n, 1), dtype=np.int32)
    lib().orc_colour(ctypes.c_int64(g.n), _p(g.off), _p(g.idx), ctypes.c_int32(p),
                     ctypes.c_int32(K), _p(out))
    return out[:g.n].copy()


def prepare(n: int, src, dst, w=None, flags: int = PREP_SYM | PREP_LOOPS):
    """Edge list (int32 src, dst; uint32 weights or None for ones) -> (off int64[n+1],
    idx int32[nnz], w uint64[nnz]), rows sorted by neighbour, repeated arcs combined (sum, or
    max with PREP_MAX). Raises ValueError on an endpoint outside [0, n) or a zero weight."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = src.size
    cap = m * (2 if flags & PREP_SYM else 1) + (n if flags & PREP_LOOPS else 0)
    off = np.zeros(n + 1, dtype=np.int64)
    idx = np.zeros(max(cap, 1), dtype=np.int32)
    wo = np.zeros(max(cap, 1), dtype=np.uint64)
    wp = None
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.uint32)
        wp = _p(w)
    f = lib().orc_prepare
    f.restype = ctypes.c_int64
    nnz = f(ctypes.c_int64(n), ctypes.c_int64(m), _p(src), _p(dst), wp, ctypes.c_uint32(flags),
            _p(off), _p(idx), _p(wo))
    if nnz < 0:
        raise ValueError("edge endpoint out of range or zero weight")
    return off, idx[:nnz].copy(), wo[:nnz].copy()


def prepare_row(n: int, src, dst, w, flags: int, r: int):
    """Row r of prepare() computed alone from the edge list (numpy, O(m) per row): the
    neighbours of r with their combined weights, ascending. For checking sampled rows of a
    graph too large to prepare on the host."""
    src = np.asarray(src)
    dst = np.asarray(dst)
    wv = np.ones(src.size, dtype=np.uint64) if w is None else np.asarray(w).astype(np.uint64)
    out_sel = src == r
    nb = [dst[out_sel].astype(np.int64)]
    ws = [wv[out_sel]]
    if flags & PREP_SYM:
        in_sel = (dst == r) & (src != r)
        nb.append(src[in_sel].astype(np.int64))
        ws.append(wv[in_sel])
    if flags & PREP_LOOPS:
        nb.append(np.array([r], dtype=np.int64))
        ws.append(np.ones(1, dtype=np.uint64))
    nb = np.concatenate(nb)
    ws = np.concatenate(ws)
    uniq, inv = np.unique(nb, return_inverse=True)
    acc = np.zeros(uniq.size, dtype=np.uint64)
    if flags & PREP_MAX:
        np.maximum.at(acc, inv, ws)
    else:
        np.add.at(acc, inv, ws)
    return uniq.astype(np.int32), acc


# ----------------------------------------------------------------------------------------------
# partition and merge (section 3.2 and the conclusion: run partitions independently, combine)


def balanced_parts(g: Graph, P: int):
    """Contiguous parts balanced by arcs: part k starts at the least vertex v with
    off[v] >= floor(k * nnz / P) (part 0 at 0, the end at n)."""
    nnz = int(g.off[-1]) if g.n else 0
    vptr = [0]
    for k in range(1, P):
        vptr.append(int(np.searchsorted(g.off[:g.n], (k * nnz) // P, side="left")))
    vptr.append(g.n)
    return vptr


def run_partitioned(g: Graph, vptr, mode: str = "sync", a: int = 2, b: int = 1,
                    max_iterations: int = 20, max_passes: int = 10, substeps: int = 1,
                    nthreads: int = 0):
    """Partition and merge over the contiguous parts [vptr[k], vptr[k+1]). Returns
    (membership int32[n], merge result dict, [per part: {"n_communities", "qnum"}])."""
    P = len(vptr) - 1
    vp = np.ascontiguousarray(vptr, dtype=np.int64)
    top = np.zeros(max(g.n, 1), dtype=np.int32)
    comms = np.zeros(max(P, 1), dtype=np.int64)
    pq = np.zeros(2 * max(P, 1), dtype=np.uint64)
    r = OrcResult()
    lib().orc_run_partitioned(*g.args(), ctypes.c_int32(P), _p(vp),
                              ctypes.c_int32(0 if mode == "sync" else 1), ctypes.c_int32(a),
                              ctypes.c_int32(b), ctypes.c_int32(max_iterations),
                              ctypes.c_int32(max_passes), ctypes.c_int32(substeps),
                              ctypes.c_int32(nthreads), _p(top), _p(comms), _p(pq),
                              ctypes.byref(r))
    res = {"passes": r.passes, "iterations": [r.iterations[p] for p in range(r.passes)],
           "n_communities": r.n_communities, "W": r.W, "qnum": _i128(r.qnum[0], r.qnum[1])}
    parts = [{"n_communities": int(comms[k]), "qnum": _i128(int(pq[2 * k]), int(pq[2 * k + 1]))}
             for k in range(P)]
    return top[:g.n].copy(), res, parts
