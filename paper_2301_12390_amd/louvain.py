"""Python binding of liblouvain.so (the C ABI in include/louvain.h).

Argument marshalling only: every step of the method runs in the library's HIP kernels. Device
buffers are torch tensors on the GPU, streams are torch's current stream. The library must have
been built (``paper_2301_12390_amd.build``); loading fails loudly otherwise.
"""

import ctypes
from dataclasses import dataclass
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblouvain.so")

LV_OK = 0
STATUS = {0: "LV_OK", -1: "LV_EINVAL", -2: "LV_ENOMEM", -3: "LV_EHIP", -4: "LV_EOVERFLOW",
          -5: "LV_EBUDGET", -6: "LV_ECANCELLED", -7: "LV_ETIMEOUT"}
LV_ETIMEOUT = -7

LV_VALIDATE = 0x1
LV_TRACE = 0x2
LV_FORCE_WIDE = 0x4
LV_SMALL_PARTS = 0x8
LV_COLOR_CLASSES = 0x10
LV_GRAPH_REPLAY = 0x20

LV_MAX_PASSES = 64
LV_MAX_TRACE = 1024


class LvI128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_int64)]

    def value(self) -> int:
        return (int(self.hi) << 64) | int(self.lo)


class LvGraph(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("offsets", ctypes.c_void_p),
        ("indices", ctypes.c_void_p),
        ("weights", ctypes.c_void_p),
        ("offsets_64", ctypes.c_int32),
        ("weights_64", ctypes.c_int32),
    ]


class LvParams(ctypes.Structure):
    _fields_ = [
        ("tolerance_exp10", ctypes.c_int32),
        ("decline_exp10", ctypes.c_int32),
        ("max_iterations", ctypes.c_int32),
        ("max_passes", ctypes.c_int32),
        ("substeps", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
    ]


class LvIterTrace(ctypes.Structure):
    _fields_ = [
        ("pass_", ctypes.c_int32),
        ("iteration", ctypes.c_int32),
        ("wide", ctypes.c_int32),
        ("substeps", ctypes.c_int32),
        ("fused_launches", ctypes.c_int32),
        ("wg_launches", ctypes.c_int32),
        ("hub_launches", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("gain_sum", LvI128),
        ("moved", ctypes.c_int64),
        ("candidates", ctypes.c_int64),
        ("fused_vertices", ctypes.c_int64),
        ("fused_arcs", ctypes.c_int64),
        ("fused_candidates", ctypes.c_int64),
        ("wg_vertices", ctypes.c_int64),
        ("wg_arcs", ctypes.c_int64),
        ("wg_candidates", ctypes.c_int64),
        ("hub_vertices", ctypes.c_int64),
        ("hub_arcs", ctypes.c_int64),
        ("fused_ms", ctypes.c_float),
        ("wg_ms", ctypes.c_float),
        ("hub_ms", ctypes.c_float),
        ("update_ms", ctypes.c_float),
        ("iter_ms", ctypes.c_float),
        ("reserved2", ctypes.c_float),
    ]


class LvResult(ctypes.Structure):
    _fields_ = [
        ("passes", ctypes.c_int32),
        ("iterations_total", ctypes.c_int32),
        ("iterations", ctypes.c_int32 * LV_MAX_PASSES),
        ("n_pass", ctypes.c_int64 * LV_MAX_PASSES),
        ("nnz_pass", ctypes.c_int64 * LV_MAX_PASSES),
        ("qnum_pass", LvI128 * LV_MAX_PASSES),
        ("cap_hits", ctypes.c_int32),
        ("n_trace", ctypes.c_int32),
        ("n_communities", ctypes.c_int64),
        ("W", ctypes.c_uint64),
        ("q_num", LvI128),
        ("q", ctypes.c_double),
        ("total_ms", ctypes.c_float),
        ("aggregate_ms", ctypes.c_float * LV_MAX_PASSES),
        ("trace", LvIterTrace * LV_MAX_TRACE),
    ]


class LvMoveStats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32),
        ("hit_cap", ctypes.c_int32),
        ("moved", ctypes.c_int64),
        ("gain_sum", LvI128),
        ("last_gain", LvI128),
        ("last_moved", ctypes.c_int64),
        ("last_candidates", ctypes.c_int64),
    ]


class LvGraphResult(ctypes.Structure):
    _fields_ = [
        ("passes", ctypes.c_int32),
        ("iterations_total", ctypes.c_int32),
        ("iterations", ctypes.c_int32 * LV_MAX_PASSES),
        ("cap_hits", ctypes.c_uint32),
        ("reserved", ctypes.c_int32),
        ("n_communities", ctypes.c_int64),
        ("W", ctypes.c_uint64),
        ("q_num", LvI128),
        ("q", ctypes.c_double),
    ]


class LvPrepStats(ctypes.Structure):
    _fields_ = [
        ("arcs", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("key_bits", ctypes.c_int32),
        ("sort_passes", ctypes.c_int32),
        ("expand_ms", ctypes.c_float),
        ("hist_ms", ctypes.c_float),
        ("scan_ms", ctypes.c_float),
        ("scatter_ms", ctypes.c_float),
        ("emit_ms", ctypes.c_float),
        ("total_ms", ctypes.c_float),
    ]


class LvServerConfig(ctypes.Structure):
    _fields_ = [
        ("slots", ctypes.c_int32),
        ("fail_run", ctypes.c_int32),
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("batch_arcs", ctypes.c_int64),
        ("params", LvParams),
    ]


class LvRequestResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("slot", ctypes.c_int32),
        ("batch_graphs", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("batch_arcs", ctypes.c_int64),
        ("submit_ns", ctypes.c_int64),
        ("start_ns", ctypes.c_int64),
        ("done_ns", ctypes.c_int64),
        ("result", LvGraphResult),
        ("error", ctypes.c_char * 160),
    ]


class LvServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64),
        ("completed", ctypes.c_int64),
        ("failed", ctypes.c_int64),
        ("runs", ctypes.c_int64),
        ("batched_requests", ctypes.c_int64),
        ("slots", ctypes.c_int32),
        ("peak_running", ctypes.c_int32),
        ("trims", ctypes.c_int32),
        ("bound_misses", ctypes.c_int32),
        ("committed_bytes", ctypes.c_uint64),
        ("peak_committed_bytes", ctypes.c_uint64),
        ("peak_held_bytes", ctypes.c_uint64),
    ]


# Every symbol the header declares, with its ctypes signature.
_P = ctypes.c_void_p
SIGNATURES = {
    "louvain_ctx_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(_P)]),
    "louvain_ctx_destroy": (None, [_P]),
    "louvain_last_error": (ctypes.c_char_p, [_P]),
    "louvain_workspace_bytes": (ctypes.c_uint64, [_P]),
    "louvain_run": (ctypes.c_int, [_P, ctypes.POINTER(LvGraph), ctypes.POINTER(LvParams), _P,
                                   ctypes.POINTER(LvResult), _P]),
    "louvain_run_levels": (ctypes.c_int, [_P, ctypes.POINTER(LvGraph), ctypes.POINTER(LvParams),
                                          _P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(LvResult), _P]),
    "louvain_prepare": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _P, _P, _P,
                                       ctypes.c_uint32, _P, ctypes.c_int32, _P, _P,
                                       ctypes.c_int32, ctypes.c_int64,
                                       ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(LvPrepStats), _P]),
    "louvain_colour_classes": (ctypes.c_int, [_P, ctypes.POINTER(LvGraph), ctypes.c_int32,
                                              ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_int32),
                                              _P]),
    "louvain_probe_gather": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_double), _P]),
    "louvain_run_partitioned": (ctypes.c_int, [_P, ctypes.POINTER(LvGraph), ctypes.c_int32,
                                               _P, ctypes.POINTER(LvParams), _P,
                                               ctypes.POINTER(LvGraphResult),
                                               ctypes.POINTER(LvResult), _P]),
    "louvain_move": (ctypes.c_int, [_P, ctypes.POINTER(LvGraph), _P, ctypes.c_uint64,
                                    ctypes.c_int32, ctypes.POINTER(LvParams), _P, _P, _P,
                                    ctypes.POINTER(LvMoveStats), _P]),
    "louvain_aggregate": (ctypes.c_int, [_P, ctypes.POINTER(LvGraph), _P, _P, _P,
                                         ctypes.c_int32, _P, _P, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int64), _P]),
    "louvain_modularity": (ctypes.c_int, [_P, ctypes.POINTER(LvGraph), _P, ctypes.POINTER(LvI128),
                                          ctypes.POINTER(ctypes.c_uint64),
                                          ctypes.POINTER(ctypes.c_double), _P]),
    "louvain_modularity_noalloc": (ctypes.c_int, [_P, ctypes.POINTER(LvGraph), _P,
                                                  ctypes.POINTER(LvI128),
                                                  ctypes.POINTER(ctypes.c_uint64),
                                                  ctypes.POINTER(ctypes.c_double), _P]),
    "louvain_run_batched": (ctypes.c_int, [_P, ctypes.POINTER(LvGraph), ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(LvParams), _P,
                                           ctypes.POINTER(LvGraphResult), _P]),
    "louvain_server_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(LvServerConfig),
                                             ctypes.POINTER(_P)]),
    "louvain_server_destroy": (None, [_P]),
    "louvain_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(LvGraph), _P,
                                             ctypes.POINTER(ctypes.c_uint64)]),
    "louvain_server_wait": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_int64,
                                           ctypes.POINTER(LvRequestResult)]),
    "louvain_server_cancel": (ctypes.c_int, [_P, ctypes.c_uint64,
                                             ctypes.POINTER(ctypes.c_int32)]),
    "louvain_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(LvServerStats)]),
    "louvain_server_clock_ns": (ctypes.c_int64, []),
}

_LIB = None


def load_library(path: str = LIB_PATH):
    """Load liblouvain.so and declare its signatures. Raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_2301_12390_amd.build` "
            "(hipcc, gfx950); there is no fallback implementation")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _LIB = lib
    return lib


class LouvainError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def graph_struct(g) -> LvGraph:
    """lv_graph for a CSR whose tensors are on the GPU (graphgen.Csr or any object with n,
    offsets, indices, weights)."""
    off, idx, w = g.offsets, g.indices, g.weights
    for t in (off, idx, w):
        if not t.is_cuda:
            raise ValueError("graph tensors must be on the GPU")
        if not t.is_contiguous():
            raise ValueError("graph tensors must be contiguous")
    if off.dtype not in (torch.int32, torch.int64) or idx.dtype != torch.int32:
        raise ValueError("offsets must be int32/int64 and indices int32")
    if w.dtype not in (torch.int32, torch.int64):
        raise ValueError("weights must be int32 (uint32 bits) or int64 (uint64 bits)")
    return LvGraph(int(g.n), int(idx.numel()), off.data_ptr(), idx.data_ptr() if idx.numel() else 0,
                   w.data_ptr() if w.numel() else 0, 1 if off.dtype == torch.int64 else 0,
                   1 if w.dtype == torch.int64 else 0)


DEFAULT_SUBSTEPS = 8

LV_PREP_SYMMETRIZE = 0x1
LV_PREP_SELF_LOOPS = 0x2
LV_PREP_MAX = 0x4
LV_PREP_TRACE = 0x8
LV_PREP_TILE_SORT = 0x10
# the paper's input graphs: reversed edges, unit weights, a self-loop on every vertex
LV_PREP_PAPER = LV_PREP_SYMMETRIZE | LV_PREP_SELF_LOOPS | LV_PREP_MAX


@dataclass
class PreparedGraph:
    """CSR written by louvain_prepare (tensors on the GPU; weights int32 holding uint32 bits or
    int64 holding uint64)."""
    n: int
    offsets: torch.Tensor
    indices: torch.Tensor
    weights: torch.Tensor
    name: str = ""
    stats: dict = None

    @property
    def nnz(self) -> int:
        return int(self.indices.numel())


def params_struct(tolerance_exp10=2, decline_exp10=1, max_iterations=20, max_passes=10,
                  substeps=DEFAULT_SUBSTEPS, flags=0):
    return LvParams(tolerance_exp10, decline_exp10, max_iterations, max_passes, substeps, flags)


def result_dict(r: LvResult) -> dict:
    P = r.passes
    tr = []
    for t in range(r.n_trace):
        x = r.trace[t]
        tr.append({
            "pass": x.pass_, "iteration": x.iteration, "wide": x.wide, "substeps": x.substeps,
            "fused_launches": x.fused_launches, "wg_launches": x.wg_launches,
            "hub_launches": x.hub_launches,
            "S": x.gain_sum.value(), "moved": x.moved, "candidates": x.candidates,
            "fused_vertices": x.fused_vertices, "fused_arcs": x.fused_arcs,
            "fused_candidates": x.fused_candidates,
            "wg_vertices": x.wg_vertices, "wg_arcs": x.wg_arcs, "wg_candidates": x.wg_candidates,
            "hub_vertices": x.hub_vertices, "hub_arcs": x.hub_arcs,
            "fused_ms": x.fused_ms, "wg_ms": x.wg_ms, "hub_ms": x.hub_ms,
            "update_ms": x.update_ms, "iter_ms": x.iter_ms,
        })
    return {
        "passes": P,
        "iterations_total": r.iterations_total,
        "iterations": [r.iterations[p] for p in range(P)],
        "n_pass": [r.n_pass[p] for p in range(P)],
        "nnz_pass": [r.nnz_pass[p] for p in range(P)],
        "qnum_pass": [r.qnum_pass[p].value() for p in range(P)],
        "cap_hits": r.cap_hits,
        "n_communities": r.n_communities,
        "W": r.W,
        "qnum": r.q_num.value(),
        "q": r.q,
        "total_ms": r.total_ms,
        "aggregate_ms": [r.aggregate_ms[p] for p in range(P)],
        "trace": tr,
    }


class Louvain:
    """A library context bound to one GPU, with a workspace limited to ``hbm_budget`` bytes
    (0 = unlimited)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        self.lib = load_library()
        self.device = device
        h = ctypes.c_void_p()
        st = self.lib.louvain_ctx_create(device, hbm_budget, ctypes.byref(h))
        if st != LV_OK:
            raise LouvainError(st, "louvain_ctx_create failed")
        self.h = h
        self._result = LvResult()

    def close(self):
        if getattr(self, "h", None):
            self.lib.louvain_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != LV_OK:
            msg = self.lib.louvain_last_error(self.h)
            raise LouvainError(st, msg.decode() if msg else "")

    def workspace_bytes(self) -> int:
        return int(self.lib.louvain_workspace_bytes(self.h))

    def run(self, g, tolerance_exp10=2, decline_exp10=1, max_iterations=20, max_passes=10,
            substeps=DEFAULT_SUBSTEPS, flags=0, membership=None):
        """Whole method. Returns (membership int32 tensor [n], result dict)."""
        gs = graph_struct(g)
        if membership is None:
            membership = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.indices.device)
        p = params_struct(tolerance_exp10, decline_exp10, max_iterations, max_passes, substeps,
                          flags)
        r = self._result
        st = self.lib.louvain_run(self.h, ctypes.byref(gs), ctypes.byref(p), _ptr(membership),
                                  ctypes.byref(r), _stream())
        self._check(st)
        return membership[:g.n], result_dict(r)

    def run_levels(self, g, tolerance_exp10=2, decline_exp10=1, max_iterations=20,
                   max_passes=10, substeps=DEFAULT_SUBSTEPS, flags=0):
        """Whole method keeping the dendrogram. Returns (membership int32 tensor [n], levels
        int32 tensor [L, n] with the membership after each of the L aggregations, result
        dict)."""
        gs = graph_struct(g)
        dev = g.indices.device
        membership = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)
        levels = torch.empty((max_passes, max(g.n, 1)), dtype=torch.int32, device=dev)
        p = params_struct(tolerance_exp10, decline_exp10, max_iterations, max_passes, substeps,
                          flags)
        r = self._result
        nl = ctypes.c_int32(0)
        st = self.lib.louvain_run_levels(self.h, ctypes.byref(gs), ctypes.byref(p),
                                         _ptr(membership), _ptr(levels), max_passes,
                                         ctypes.byref(nl), ctypes.byref(r), _stream())
        self._check(st)
        return membership[:g.n], levels[:nl.value, :g.n], result_dict(r)

    def run_partitioned(self, g, P=8, vptr=None, tolerance_exp10=2, decline_exp10=1,
                        max_iterations=20, max_passes=10, substeps=DEFAULT_SUBSTEPS, flags=0):
        """Partition and merge over P contiguous parts (vptr: host bounds, or None for parts
        balanced by arcs). Returns (membership int32 tensor [n], merge result dict, list of
        per-part result dicts)."""
        gs = graph_struct(g)
        membership = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.indices.device)
        vp = None
        if vptr is not None:
            if len(vptr) != P + 1:
                raise ValueError("vptr must have P + 1 entries")
            vp = (ctypes.c_int64 * (P + 1))(*[int(x) for x in vptr])
        p = params_struct(tolerance_exp10, decline_exp10, max_iterations, max_passes, substeps,
                          flags)
        parts = (LvGraphResult * P)()
        r = self._result
        st = self.lib.louvain_run_partitioned(self.h, ctypes.byref(gs), P, vp, ctypes.byref(p),
                                              _ptr(membership), parts, ctypes.byref(r),
                                              _stream())
        self._check(st)
        out = [{"passes": q.passes, "iterations": [q.iterations[i] for i in range(q.passes)],
                "n_communities": q.n_communities, "W": q.W, "qnum": q.q_num.value(), "q": q.q}
               for q in parts]
        return membership[:g.n], result_dict(r), out

    def colour_classes(self, g, pass_index=0, K=DEFAULT_SUBSTEPS):
        """Colour class of every vertex (uint8 tensor [n]) and the rounds taken."""
        gs = graph_struct(g)
        out = torch.empty(max(g.n, 1), dtype=torch.uint8, device=g.indices.device)
        rounds = ctypes.c_int32(0)
        st = self.lib.louvain_colour_classes(self.h, ctypes.byref(gs), pass_index, K, _ptr(out),
                                             ctypes.byref(rounds), _stream())
        self._check(st)
        return out[:g.n], rounds.value

    def probe_gather(self, table_bytes, slices=1):
        """Random 4-byte gathers per second over a table of table_bytes bytes (measurement:
        the ceiling the move and merge kernels run against; slices > 1 confines workgroup b to
        slice b mod slices)."""
        rate = ctypes.c_double(0)
        st = self.lib.louvain_probe_gather(self.h, int(table_bytes), int(slices),
                                           ctypes.byref(rate), _stream())
        self._check(st)
        return rate.value

    def prepare(self, n, src, dst, weights=None, flags=LV_PREP_PAPER, offsets_64=True,
                weights_64=False, capacity=None) -> PreparedGraph:
        """Edge list (int32 GPU tensors src, dst; weights int32 holding uint32 bits, or None for
        ones) -> the symmetric CSR the method takes. Sizes the outputs with the upper bound
        m (x2 with LV_PREP_SYMMETRIZE) + n (with LV_PREP_SELF_LOOPS) unless capacity is given,
        then trims them to the arcs written."""
        for t in (src, dst) + ((weights,) if weights is not None else ()):
            if not t.is_cuda or not t.is_contiguous() or t.dtype != torch.int32:
                raise ValueError("src, dst and weights must be contiguous int32 GPU tensors")
        m = int(src.numel())
        if int(dst.numel()) != m or (weights is not None and int(weights.numel()) != m):
            raise ValueError("src, dst and weights must have the same length")
        dev = src.device
        if capacity is None:
            capacity = m * (2 if flags & LV_PREP_SYMMETRIZE else 1) + (
                n if flags & LV_PREP_SELF_LOOPS else 0)
        off = torch.empty(n + 1, dtype=torch.int64 if offsets_64 else torch.int32, device=dev)
        idx = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
        w = torch.empty(max(capacity, 1), dtype=torch.int64 if weights_64 else torch.int32,
                        device=dev)
        nnz = ctypes.c_int64(0)
        ps = LvPrepStats()
        st = self.lib.louvain_prepare(self.h, n, m, _ptr(src) if m else None,
                                      _ptr(dst) if m else None,
                                      _ptr(weights) if weights is not None and m else None,
                                      flags, _ptr(off), 1 if offsets_64 else 0, _ptr(idx),
                                      _ptr(w), 1 if weights_64 else 0, capacity,
                                      ctypes.byref(nnz), ctypes.byref(ps), _stream())
        self._check(st)
        k = nnz.value
        stats = {f: getattr(ps, f) for f, _ in LvPrepStats._fields_}
        return PreparedGraph(n, off, idx[:k], w[:k], name="prepared", stats=stats)

    def prepare_count(self, n, src, dst, flags=LV_PREP_PAPER) -> int:
        """Arcs louvain_prepare would write (the size query)."""
        m = int(src.numel())
        nnz = ctypes.c_int64(0)
        st = self.lib.louvain_prepare(self.h, n, m, _ptr(src) if m else None,
                                      _ptr(dst) if m else None, None, flags, None, 1, None,
                                      None, 0, 0, ctypes.byref(nnz), None, _stream())
        self._check(st)
        return nnz.value

    def run_batched(self, packed, vptr, aptr, tolerance_exp10=2, decline_exp10=1,
                    max_iterations=20, max_passes=10, substeps=DEFAULT_SUBSTEPS, flags=0,
                    membership=None):
        """Many graphs in one run. packed: one CSR of the graphs with consecutive vertex ids;
        vptr, aptr: the G + 1 vertex and arc bounds (host sequences). Returns (membership int32
        tensor [n] of ids local to each graph, list of per-graph result dicts)."""
        gs = graph_struct(packed)
        G = len(vptr) - 1
        vp = (ctypes.c_int64 * (G + 1))(*[int(x) for x in vptr])
        ap = (ctypes.c_int64 * (G + 1))(*[int(x) for x in aptr])
        if membership is None:
            membership = torch.empty(max(packed.n, 1), dtype=torch.int32,
                                     device=packed.indices.device)
        p = params_struct(tolerance_exp10, decline_exp10, max_iterations, max_passes, substeps,
                          flags)
        res = (LvGraphResult * G)()
        st = self.lib.louvain_run_batched(self.h, ctypes.byref(gs), G, vp, ap, ctypes.byref(p),
                                          _ptr(membership), res, _stream())
        self._check(st)
        out = []
        for r in res:
            P = r.passes
            out.append({"passes": P, "iterations_total": r.iterations_total,
                        "iterations": [r.iterations[i] for i in range(P)],
                        "cap_hits": r.cap_hits, "n_communities": r.n_communities, "W": r.W,
                        "qnum": r.q_num.value(), "q": r.q})
        return membership[:packed.n], out

    def move(self, g, C, Sigma, csize, K=None, W=0, pass_index=0, tolerance_exp10=2,
             decline_exp10=1, max_iterations=20, substeps=DEFAULT_SUBSTEPS, flags=0) -> dict:
        """One local-moving phase in place on (C, Sigma, csize); Sigma is an int64 tensor of
        uint64 values. Returns the phase statistics."""
        gs = graph_struct(g)
        p = params_struct(tolerance_exp10, decline_exp10, max_iterations, 1, substeps, flags)
        ms = LvMoveStats()
        st = self.lib.louvain_move(self.h, ctypes.byref(gs), _ptr(K), int(W), pass_index,
                                   ctypes.byref(p), _ptr(C), _ptr(Sigma), _ptr(csize),
                                   ctypes.byref(ms), _stream())
        self._check(st)
        return {"iterations": ms.iterations, "hit_cap": ms.hit_cap, "moved": ms.moved,
                "gain_sum": ms.gain_sum.value(), "last_gain": ms.last_gain.value(),
                "last_moved": ms.last_moved, "last_candidates": ms.last_candidates}

    def aggregate(self, g, C, offsets_64=True):
        """Super-vertex graph of C. Returns (map int32 [n], (n', offsets, indices, weights))
        with weights as int64 (uint64 values)."""
        gs = graph_struct(g)
        dev = g.indices.device
        n, nnz = int(g.n), int(g.indices.numel())
        mp = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        off = torch.empty(n + 1, dtype=torch.int64 if offsets_64 else torch.int32, device=dev)
        idx = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        w = torch.empty(max(nnz, 1), dtype=torch.int64, device=dev)
        n_out = ctypes.c_int64()
        nnz_out = ctypes.c_int64()
        st = self.lib.louvain_aggregate(self.h, ctypes.byref(gs), _ptr(C), _ptr(mp), _ptr(off),
                                        1 if offsets_64 else 0, _ptr(idx), _ptr(w),
                                        ctypes.byref(n_out), ctypes.byref(nnz_out), _stream())
        self._check(st)
        n2, z2 = n_out.value, nnz_out.value
        return mp[:n], (n2, off[:n2 + 1], idx[:z2], w[:z2])

    def modularity(self, g, C):
        """(Qnum, W, q) of membership C."""
        gs = graph_struct(g)
        q = LvI128()
        W = ctypes.c_uint64()
        qd = ctypes.c_double()
        st = self.lib.louvain_modularity(self.h, ctypes.byref(gs), _ptr(C), ctypes.byref(q),
                                         ctypes.byref(W), ctypes.byref(qd), _stream())
        self._check(st)
        return q.value(), int(W.value), float(qd.value)

    def modularity_noalloc(self, g, C):
        """(Qnum, W, q) of membership C through louvain_modularity_noalloc (no device
        allocation during the call; temporaries in the library's fixed per-device array)."""
        gs = graph_struct(g)
        q = LvI128()
        W = ctypes.c_uint64()
        qd = ctypes.c_double()
        st = self.lib.louvain_modularity_noalloc(self.h, ctypes.byref(gs), _ptr(C),
                                                 ctypes.byref(q), ctypes.byref(W),
                                                 ctypes.byref(qd), _stream())
        self._check(st)
        return q.value(), int(W.value), float(qd.value)


def graph_result_dict(r: LvGraphResult) -> dict:
    P = r.passes
    return {"passes": P, "iterations_total": r.iterations_total,
            "iterations": [r.iterations[i] for i in range(P)], "cap_hits": r.cap_hits,
            "n_communities": r.n_communities, "W": r.W, "qnum": r.q_num.value(), "q": r.q}


def request_struct(n, offsets, indices, weights, membership=None):
    """(lv_graph with host pointers, membership tensor) for louvain_server_submit, after the
    checks the library cannot make on host memory: the arrays' sizes against n and each other,
    so that the server never reads or writes past a request's buffers."""
    n = int(n)
    if n < 0:
        raise ValueError("n must be >= 0")
    for t in (offsets, indices, weights):
        if t.is_cuda or not t.is_contiguous():
            raise ValueError("request tensors must be contiguous host tensors")
    if offsets.dtype not in (torch.int32, torch.int64) or indices.dtype != torch.int32 \
            or weights.dtype != torch.int32:
        raise ValueError("offsets int32/int64, indices int32, weights int32 (uint32 bits)")
    if offsets.numel() != n + 1 and not (n == 0 and offsets.numel() == 0):
        raise ValueError(f"offsets has {offsets.numel()} entries, n + 1 = {n + 1} expected")
    if indices.numel() != weights.numel():
        raise ValueError("indices and weights differ in length")
    if membership is None:
        membership = torch.empty(max(n, 1), dtype=torch.int32, pin_memory=offsets.is_pinned())
    elif membership.is_cuda or not membership.is_contiguous() or \
            membership.dtype != torch.int32 or membership.numel() < n:
        raise ValueError("membership must be a contiguous int32 host tensor of n entries")
    m = int(indices.numel())
    g = LvGraph(n, m, offsets.data_ptr() if offsets.numel() else 0,
                indices.data_ptr() if m else 0, weights.data_ptr() if m else 0,
                1 if offsets.dtype == torch.int64 else 0, 0)
    return g, membership


class Server:
    """The library's request server (louvain_server_*): ``slots`` runs in flight at once, each
    batching the queued requests up to ``batch_arcs`` arcs, device memory admitted against
    ``hbm_budget`` bytes (0 = no limit). Requests are CSRs in host memory (CPU tensors; pinned
    ones copy fastest); the server keeps them referenced until they are waited for."""

    def __init__(self, device: int = 0, slots: int = 4, hbm_budget: int = 0,
                 batch_arcs: int = 1 << 28, tolerance_exp10=2, decline_exp10=1,
                 max_iterations=20, max_passes=10, substeps=DEFAULT_SUBSTEPS, flags=0,
                 fail_run=0):
        self.lib = load_library()
        cfg = LvServerConfig(slots, fail_run, hbm_budget, batch_arcs,
                             params_struct(tolerance_exp10, decline_exp10, max_iterations,
                                           max_passes, substeps, flags))
        h = ctypes.c_void_p()
        st = self.lib.louvain_server_create(device, ctypes.byref(cfg), ctypes.byref(h))
        if st != LV_OK:
            raise LouvainError(st, "louvain_server_create failed")
        self.h = h
        self._held = {}

    def close(self):
        if getattr(self, "h", None):
            self.lib.louvain_server_destroy(self.h)
            self.h = None
            self._held.clear()

    def __del__(self):
        self.close()

    def clock_ns(self) -> int:
        return int(self.lib.louvain_server_clock_ns())

    def submit(self, n, offsets, indices, weights, membership=None) -> int:
        """Queues one graph (host tensors: offsets int32/int64 [n+1], indices int32, weights
        int32 holding uint32 bits). Returns the ticket; the membership (int32 [n], host) comes
        back from wait()."""
        g, membership = request_struct(n, offsets, indices, weights, membership)
        t = ctypes.c_uint64()
        st = self.lib.louvain_server_submit(self.h, ctypes.byref(g), _ptr(membership),
                                            ctypes.byref(t))
        if st != LV_OK:
            raise LouvainError(st, "louvain_server_submit refused the request")
        self._held[t.value] = (offsets, indices, weights, membership, int(n))
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1):
        """(membership int32 host tensor [n], outcome dict) of a request, or None on a time-out.
        The outcome has the request's status, error text, slot, batch and clock readings, and
        the per-graph result of the run."""
        r = LvRequestResult()
        st = self.lib.louvain_server_wait(self.h, ticket, timeout_ms, ctypes.byref(r))
        if st == LV_ETIMEOUT:
            return None
        if st != LV_OK:
            raise LouvainError(st, f"louvain_server_wait: unknown ticket {ticket}")
        _, _, _, memb, n = self._held.pop(ticket)
        out = {"status": r.status, "error": r.error.decode(), "slot": r.slot,
               "batch_graphs": r.batch_graphs, "batch_arcs": r.batch_arcs,
               "submit_ns": r.submit_ns, "start_ns": r.start_ns, "done_ns": r.done_ns}
        out.update(graph_result_dict(r.result))
        return memb[:n], out

    def cancel(self, ticket: int) -> bool:
        """Drops a request that is still queued (it then completes with LV_ECANCELLED); False
        if it is already running or done."""
        c = ctypes.c_int32(0)
        st = self.lib.louvain_server_cancel(self.h, ticket, ctypes.byref(c))
        if st != LV_OK:
            raise LouvainError(st, f"louvain_server_cancel: unknown ticket {ticket}")
        return bool(c.value)

    def stats(self) -> dict:
        s = LvServerStats()
        self.lib.louvain_server_stats(self.h, ctypes.byref(s))
        return {f: getattr(s, f) for f, _ in LvServerStats._fields_}
