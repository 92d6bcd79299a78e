"""The integer range of the method on the GPU, and the argument checks.

* Weights whose total W lies just below 2^62, the largest the library accepts: every gain
  W*k - K*Sigma then needs its high 64 bits, super-arc weights exceed 32 bits and the hub tables
  hold 64-bit values. Per-iteration state, whole runs, modularity and aggregation are compared
  with the oracle, with and without LV_FORCE_WIDE.
* LV_EOVERFLOW: W above 2^62, including totals of 2^64 or more that a 64-bit sum would wrap
  (run, move, modularity, batch), a batch whose total reaches 2^64, n = 2^31, and nnz >= 2^31
  with int32 offsets.
* LV_EINVAL for null arguments of every entry point, and the context staying usable after.
"""

import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from graphgen import csr_from_edges, pack_graphs, planted_hubs, sbm
from graphgen.csr import Csr

from .gpu_util import assert_state_equal, canonical_rows_fast, gpu_state

pytestmark = pytest.mark.gpu

LV_FORCE_WIDE = 0x4
LV_SMALL_PARTS = 0x8


@pytest.fixture(scope="module")
def lv(gpu_device):
    from paper_2301_12390_amd import Louvain
    ctx = Louvain(0)
    yield ctx
    ctx.close()


def widen(g: Csr, target_exp: int = 62, name: str = "") -> Csr:
    """g with every weight w replaced by (w << s) - (40503 w mod 2^15) (a function of w, so the
    graph stays symmetric), s chosen so that W lies in (2^(target_exp-2), 2^target_exp]."""
    w = g.weights.to(torch.int64)
    W0 = int(w.sum())
    s = target_exp - W0.bit_length()
    nw = (w << s) - ((w * 40503) & 0x7FFF)
    out = Csr(g.n, g.offsets.to(torch.int64), g.indices, nw, name or g.name + "-wide")
    W = int(nw.sum())
    assert 2 ** (target_exp - 2) < W <= 2 ** target_exp
    return out


def star(n_leaves: int) -> Csr:
    """A hub joined to n_leaves leaves, weights 1..13 (one row on the two-phase hub path)."""
    u = torch.zeros(n_leaves, dtype=torch.int64)
    v = torch.arange(1, n_leaves + 1)
    return csr_from_edges(n_leaves + 1, u, v, lambda lo, hi: (hi % 13) + 1,
                          name=f"star{n_leaves}")


def big_graphs():
    base = sbm(1500, 15, 8.0, 2.0, seed=21, weights=(1, 16))
    hubs = planted_hubs(sbm(20000, 200, 8.0, 2.0, seed=22, weights=(1, 16)), [12000, 7000],
                        seed=3, weights=(1, 16))
    return [widen(base), widen(hubs), widen(star(6000))]


BIG = big_graphs()
BIG_IDS = ["sbm1500", "sbm20k+hubs", "star6000"]


def check_run(lv, g, flags, substeps):
    og = O.Graph.from_csr(g)
    top, ref = O.run(og, "sync", substeps=substeps)
    memb, res = lv.run(g.to("cuda:0"), flags=flags, substeps=substeps)
    torch.cuda.synchronize()
    assert res["W"] == ref["W"] and res["W"] > 2 ** 60
    assert np.array_equal(memb.cpu().numpy(), top)
    assert res["qnum"] == ref["qnum"] and res["qnum_pass"] == ref["qnum_pass"]
    assert res["iterations"] == ref["iterations"] and res["passes"] == ref["passes"]
    assert [t["S"] for t in res["trace"]] == ref["trace_S"]
    assert [t["moved"] for t in res["trace"]] == ref["trace_moved"]
    assert [t["candidates"] for t in res["trace"]] == ref["trace_ncand"]
    # the gains of the first iteration need more than 64 bits
    assert all(t["wide"] for t in res["trace"])
    assert abs(ref["trace_S"][0]) >= 2 ** 64


@pytest.mark.parametrize("K", [1, 8])
@pytest.mark.parametrize("flags", [0, LV_FORCE_WIDE, LV_SMALL_PARTS])
@pytest.mark.parametrize("gi", range(len(BIG)), ids=BIG_IDS)
def test_run_weights_near_2_62(lv, gi, flags, K):
    check_run(lv, BIG[gi], flags, K)


@pytest.mark.parametrize("gi", range(len(BIG)), ids=BIG_IDS)
def test_iterations_weights_near_2_62(lv, gi):
    g = BIG[gi]
    og = O.Graph.from_csr(g)
    dg = g.to("cuda:0")
    for K, p in ((1, 0), (8, 3)):
        st = O.State(og)
        C, Sig, cs, Kd = gpu_state(st)
        classes = O.class_lists(og.n, p, K)
        for it in range(5):
            stats = lv.move(dg, C, Sig, cs, K=Kd, W=st.W, max_iterations=1, substeps=K,
                            pass_index=p)
            S, moved, nc = O.substep_iteration(og, st, p, K, classes)
            torch.cuda.synchronize()
            assert_state_equal(st, C, Sig, cs, f"{g.name} K{K} it{it}")
            assert stats["last_gain"] == S and stats["last_moved"] == moved
            assert stats["last_candidates"] == nc
            if moved == 0:
                break


@pytest.mark.parametrize("gi", range(len(BIG)), ids=BIG_IDS)
def test_modularity_and_aggregate_weights_near_2_62(lv, gi):
    g = BIG[gi]
    og = O.Graph.from_csr(g)
    dg = g.to("cuda:0")
    rng = np.random.default_rng(gi)
    for C in (np.arange(g.n, dtype=np.int32), rng.integers(0, 37, g.n).astype(np.int32)):
        Ct = torch.from_numpy(C).to("cuda:0")
        qnum, W, q = lv.modularity(dg, Ct)
        assert (qnum, W) == O.modularity(og, C)[:2]
        mp, (n2, off, idx, w) = lv.aggregate(dg, Ct)
        mo, g2 = O.aggregate(og, C)
        assert np.array_equal(mp.cpu().numpy(), mo) and n2 == g2.n
        off_c, idx_c, w_c = canonical_rows_fast(n2, off.cpu().numpy(), idx.cpu().numpy(),
                                                w.cpu().numpy())
        assert np.array_equal(off_c, g2.off) and np.array_equal(idx_c, g2.idx)
        assert np.array_equal(w_c, g2.w)


def test_batch_weights_near_2_62(lv):
    graphs = [BIG[0], BIG[2], widen(sbm(800, 8, 8.0, 2.0, seed=5, weights=(1, 16)))]
    packed, vptr, aptr = pack_graphs(graphs)
    memb, res = lv.run_batched(packed.to("cuda:0"), vptr, aptr)
    memb = memb.cpu().numpy()
    for g, (gr, r) in enumerate(zip(graphs, res)):
        top, ref = O.run(O.Graph.from_csr(gr), "sync", substeps=8)
        assert np.array_equal(memb[vptr[g]:vptr[g + 1]], top)
        assert r["qnum"] == ref["qnum"] and r["iterations"] == ref["iterations"]


# ----------------------------------------------------------------------------------------------
# LV_EOVERFLOW


def edge_graph(weight: int, dev="cuda:0") -> Csr:
    """Single edge {0, 1} with uint64 weight `weight` on both arcs."""
    w = torch.tensor([weight, weight], dtype=torch.uint64).view(torch.int64)
    return Csr(2, torch.tensor([0, 1, 2], dtype=torch.int64), torch.tensor([1, 0], dtype=torch.int32),
               w, name=f"edge-w{weight}").to(dev)


@pytest.mark.parametrize("weight,ok", [(2 ** 61, True), (2 ** 61 + 1, False), (2 ** 62, False),
                                       (2 ** 63, False), (2 ** 63 + 5, False)])
def test_total_weight_limit(lv, weight, ok):
    """W = 2 * weight: 2^62 is accepted, anything above is LV_EOVERFLOW, also when the 64-bit
    sum wraps to 0 (2^63 + 2^63) or to a small value."""
    from paper_2301_12390_amd import LouvainError
    g = edge_graph(weight)
    C = torch.zeros(2, dtype=torch.int32, device="cuda:0")
    calls = [
        lambda: lv.run(g),
        lambda: lv.modularity(g, C),
        lambda: lv.move(g, torch.arange(2, dtype=torch.int32, device="cuda:0"),
                        g.weights.clone(), torch.ones(2, dtype=torch.int32, device="cuda:0"),
                        max_iterations=1),
    ]
    for call in calls:
        if ok:
            call()
        else:
            with pytest.raises(LouvainError, match="EOVERFLOW"):
                call()
    if ok:
        memb, res = lv.run(g)
        assert memb.cpu().tolist() == [0, 0] and res["W"] == 2 ** 62 and res["qnum"] == 0
    # the context stays usable
    memb, res = lv.run(edge_graph(3))
    assert memb.cpu().tolist() == [0, 0]


def test_batch_total_weight_limit(lv):
    """Graphs of W = 2^62 each are valid; four of them make a batch total of 2^64, which the
    64-bit per-graph sums cannot be trusted with: LV_EOVERFLOW. Three are fine and equal the
    single runs."""
    from paper_2301_12390_amd import LouvainError
    one = edge_graph(2 ** 61, "cpu")
    packed, vptr, aptr = pack_graphs([one] * 3)
    memb, res = lv.run_batched(packed.to("cuda:0"), vptr, aptr)
    assert memb.cpu().tolist() == [0, 0] * 3
    assert all(r["W"] == 2 ** 62 and r["qnum"] == 0 for r in res)
    packed, vptr, aptr = pack_graphs([one] * 4)
    with pytest.raises(LouvainError, match="EOVERFLOW"):
        lv.run_batched(packed.to("cuda:0"), vptr, aptr)
    packed, vptr, aptr = pack_graphs([edge_graph(2 ** 61 + 1, "cpu"), edge_graph(1, "cpu")])
    with pytest.raises(LouvainError, match="EOVERFLOW"):
        lv.run_batched(packed.to("cuda:0"), vptr, aptr)


def raw_graph(n, nnz, off=None, idx=None, w=None, off64=1, w64=0):
    from paper_2301_12390_amd.louvain import LvGraph
    return LvGraph(n, nnz, off or 0, idx or 0, w or 0, off64, w64)


def test_descriptor_overflow(lv):
    """n = 2^31, and nnz >= 2^31 with int32 offsets, are refused before any pointer is read."""
    from paper_2301_12390_amd.louvain import LvParams, LvResult, _stream
    lib = lv.lib
    p = LvParams(2, 1, 20, 10, 8, 0)
    r = LvResult()
    memb = torch.empty(4, dtype=torch.int32, device="cuda:0")
    ok = edge_graph(1)
    cases = [raw_graph(2 ** 31, 2, ok.offsets.data_ptr(), ok.indices.data_ptr(),
                       ok.weights.data_ptr(), 1, 1),
             raw_graph(2, 2 ** 31, ok.offsets.data_ptr(), ok.indices.data_ptr(),
                       ok.weights.data_ptr(), 0, 1)]
    for gs in cases:
        st = lib.louvain_run(lv.h, ctypes.byref(gs), ctypes.byref(p),
                             ctypes.c_void_p(memb.data_ptr()), ctypes.byref(r), _stream())
        assert st == -4, st
        st = lib.louvain_modularity(lv.h, ctypes.byref(gs), ctypes.c_void_p(memb.data_ptr()),
                                    None, None, None, _stream())
        assert st == -4, st


# ----------------------------------------------------------------------------------------------
# LV_EINVAL for null arguments


def test_null_arguments(lv):
    from paper_2301_12390_amd.louvain import (LvGraphResult, LvMoveStats, LvParams, LvResult,
                                              _stream, graph_struct)
    lib = lv.lib
    dev = "cuda:0"
    g = edge_graph(2)
    gs = graph_struct(g)
    p = LvParams(2, 1, 20, 10, 8, 0)
    r = LvResult()
    memb = torch.empty(2, dtype=torch.int32, device=dev)
    mp = ctypes.c_void_p(memb.data_ptr())
    S = _stream()
    EINVAL = -1
    B = ctypes.byref
    assert lib.louvain_run(None, B(gs), B(p), mp, B(r), S) == EINVAL
    assert lib.louvain_run(lv.h, None, B(p), mp, B(r), S) == EINVAL
    assert lib.louvain_run(lv.h, B(gs), None, mp, B(r), S) == EINVAL
    assert lib.louvain_run(lv.h, B(gs), B(p), None, B(r), S) == EINVAL
    assert lib.louvain_run(lv.h, B(gs), B(p), mp, None, S) == EINVAL
    for field in ("offsets", "indices", "weights"):
        bad = graph_struct(g)
        setattr(bad, field, 0)
        assert lib.louvain_run(lv.h, B(bad), B(p), mp, B(r), S) == EINVAL, field
    nl = ctypes.c_int32(0)
    lev = torch.empty(20, dtype=torch.int32, device=dev)
    lp = ctypes.c_void_p(lev.data_ptr())
    assert lib.louvain_run_levels(lv.h, B(gs), B(p), mp, None, 10, B(nl), B(r), S) == EINVAL
    assert lib.louvain_run_levels(lv.h, B(gs), B(p), mp, lp, 10, None, B(r), S) == EINVAL
    C = torch.arange(2, dtype=torch.int32, device=dev)
    Sig = g.weights.clone()
    cs = torch.ones(2, dtype=torch.int32, device=dev)
    cp, sp, csp = (ctypes.c_void_p(t.data_ptr()) for t in (C, Sig, cs))
    ms = LvMoveStats()
    assert lib.louvain_move(lv.h, B(gs), None, 0, 0, B(p), None, sp, csp, B(ms), S) == EINVAL
    assert lib.louvain_move(lv.h, B(gs), None, 0, 0, B(p), cp, None, csp, B(ms), S) == EINVAL
    assert lib.louvain_move(lv.h, B(gs), None, 0, 0, B(p), cp, sp, None, B(ms), S) == EINVAL
    assert lib.louvain_move(lv.h, B(gs), None, 0, 0, None, cp, sp, csp, B(ms), S) == EINVAL
    assert lib.louvain_modularity(lv.h, B(gs), None, None, None, None, S) == EINVAL
    off = torch.empty(3, dtype=torch.int64, device=dev)
    idx = torch.empty(2, dtype=torch.int32, device=dev)
    w = torch.empty(2, dtype=torch.int64, device=dev)
    n2, z2 = ctypes.c_int64(0), ctypes.c_int64(0)
    op, ip, wp = (ctypes.c_void_p(t.data_ptr()) for t in (off, idx, w))
    assert lib.louvain_aggregate(lv.h, B(gs), cp, mp, None, 1, ip, wp, B(n2), B(z2), S) == EINVAL
    assert lib.louvain_aggregate(lv.h, B(gs), None, mp, op, 1, ip, wp, B(n2), B(z2), S) == EINVAL
    assert lib.louvain_aggregate(lv.h, B(gs), cp, mp, op, 1, ip, wp, None, B(z2), S) == EINVAL
    vptr = (ctypes.c_int64 * 2)(0, 2)
    aptr = (ctypes.c_int64 * 2)(0, 2)
    pg = (LvGraphResult * 1)()
    assert lib.louvain_run_batched(lv.h, B(gs), 1, None, aptr, B(p), mp, pg, S) == EINVAL
    assert lib.louvain_run_batched(lv.h, B(gs), 1, vptr, aptr, B(p), mp, None, S) == EINVAL
    assert lib.louvain_run_batched(lv.h, None, 1, vptr, aptr, B(p), mp, pg, S) == EINVAL
    assert lib.louvain_run_batched(lv.h, B(gs), 0, vptr, aptr, B(p), mp, pg, S) == EINVAL
    assert lib.louvain_run_partitioned(lv.h, B(gs), 1, None, B(p), mp, pg, None, S) == EINVAL
    assert lib.louvain_colour_classes(lv.h, B(gs), 0, 8, None, None, S) == EINVAL
    nz = ctypes.c_int64(0)
    assert lib.louvain_prepare(lv.h, 2, 1, None, None, None, 0x3, op, 1, ip, wp, 1, 2, B(nz),
                               None, S) == EINVAL
    assert lib.louvain_prepare(lv.h, 2, 0, None, None, None, 0x3, op, 1, ip, wp, 1, 2, None,
                               None, S) == EINVAL
    assert lib.louvain_ctx_create(0, 0, None) == EINVAL
    # the context still works
    memb2, res = lv.run(g)
    assert memb2.cpu().tolist() == [0, 0]
