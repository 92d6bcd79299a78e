"""Parity at the benchmark's full sizes.

* R-MAT scale 25 (1.05e9 arcs, the timed workload): the whole run against the oracle's whole
  run stored in ``golden/rmat25_run.json`` (membership SHA-256, Qnum of every pass, every
  iteration's S, moves and candidate pairs; written by ``golden/make_rmat25_golden.py``, which
  calls only the oracle), and the quality gate against the stored sequential asynchronous run;
  the whole first local-moving iteration of pass 0 (8 class steps) against the oracle, element
  by element; the modularity of a whole GPU run recomputed by the oracle; aggregation checked
  on every vertex's map, every super-vertex's degree and total weight, and on sampled
  super-rows computed by definition.
* R-MAT scale 22 (1.28e8 arcs): a whole run against the oracle's whole run, and the quality gate
  against the sequential asynchronous oracle.
"""

import hashlib
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
from graphgen import config_graph

from .gpu_util import gpu_state

pytestmark = pytest.mark.gpu

K_CLASSES = 8


@pytest.fixture(scope="module")
def lv(gpu_device):
    from paper_2301_12390_amd import Louvain
    ctx = Louvain(0)
    yield ctx
    ctx.close()


@pytest.fixture(scope="module")
def rmat25(gpu_device):
    print("generating rmat25 on the GPU", flush=True)
    g = config_graph("rmat25", device="cuda:0")
    og = O.Graph.from_csr(g)
    yield g, og
    del g, og
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def rmat25_iter0(rmat25):
    """Oracle state before and after iteration 0 of pass 0."""
    g, og = rmat25
    st0 = O.State(og)
    st = st0.copy()
    classes = O.class_lists(og.n, 0, K_CLASSES)
    print("oracle: iteration 0 of pass 0 on rmat25", flush=True)
    S, moved, nc = O.substep_iteration(og, st, 0, K_CLASSES, classes)
    return st0, st, (S, moved, nc)


GOLDEN25 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rmat25_run.json")


@pytest.mark.timeout(600)
def test_rmat25_whole_run_matches_golden(lv, rmat25):
    """The timed configuration end to end: louvain_run on R-MAT s25 (8 classes, tolerance 10^-2
    declining x10) equals the oracle's stored run bit for bit, and its Q is within 0.01 of the
    sequential asynchronous run's (section 3.2 compares the two rules' quality)."""
    from graphgen.lean import csr_sha256_np
    gold = json.load(open(GOLDEN25))
    g, og = rmat25
    assert (g.n, g.nnz) == (gold["graph"]["n"], gold["graph"]["nnz"])
    print("hashing the rmat25 CSR", flush=True)
    assert csr_sha256_np(og.n, og.off, og.idx, og.w) == gold["graph"]["csr_sha256"]
    memb, res = lv.run(g, substeps=K_CLASSES)
    torch.cuda.synchronize()
    ref = gold["sync"]
    m = memb.cpu().numpy()
    assert hashlib.sha256(np.ascontiguousarray(m, dtype="<i4").tobytes()).hexdigest() == \
        ref["membership_sha256"]
    assert res["W"] == gold["graph"]["W"]
    assert res["qnum"] == ref["qnum"] and res["qnum_pass"] == ref["qnum_pass"]
    assert res["passes"] == ref["passes"] and res["iterations"] == ref["iterations"]
    assert res["n_pass"] == ref["n_pass"] and res["nnz_pass"] == ref["nnz_pass"]
    assert res["n_communities"] == ref["n_communities"] and res["cap_hits"] == ref["cap_hits"]
    assert [t["S"] for t in res["trace"]] == ref["trace_S"]
    assert [t["moved"] for t in res["trace"]] == ref["trace_moved"]
    assert [t["candidates"] for t in res["trace"]] == ref["trace_ncand"]
    q_async = gold["async"]["q"]
    print(f"rmat25: Q gpu {res['q']:.6f}, Q async {q_async:.6f}", flush=True)
    assert res["q"] >= q_async - 0.01


@pytest.mark.timeout(600)
def test_rmat25_first_iteration_exact(lv, rmat25, rmat25_iter0):
    g, og = rmat25
    st0, st, (S, moved, nc) = rmat25_iter0
    C, Sig, cs, K = gpu_state(st0)
    stats = lv.move(g, C, Sig, cs, K=K, W=st0.W, max_iterations=1, substeps=K_CLASSES)
    torch.cuda.synchronize()
    assert stats["last_gain"] == S and stats["last_moved"] == moved
    assert stats["last_candidates"] == nc
    assert np.array_equal(C.cpu().numpy(), st.C)
    assert np.array_equal(Sig.cpu().numpy().view(np.uint64), st.Sig)
    assert np.array_equal(cs.cpu().numpy(), st.csize)


@pytest.mark.timeout(600)
def test_rmat25_run_modularity_and_labels(lv, rmat25, rmat25_iter0):
    g, og = rmat25
    st0, st, (S, moved, _) = rmat25_iter0
    memb, res = lv.run(g, substeps=K_CLASSES)
    torch.cuda.synchronize()
    m = memb.cpu().numpy()
    # the first iteration of the run is the one checked above
    assert res["trace"][0]["S"] == S and res["trace"][0]["moved"] == moved
    assert res["W"] == st0.W
    # labels are dense 0..k-1 and all used
    k = res["n_communities"]
    assert m.min() >= 0 and m.max() == k - 1
    assert np.unique(m).size == k
    qnum, W, _ = O.modularity(og, m)
    assert qnum == res["qnum"] and W == res["W"]


@pytest.mark.timeout(600)
def test_rmat25_levels_properties(lv, rmat25):
    """The dendrogram at full size, through properties that hold at any size: each level's
    modularity on the input graph (oracle) equals the run's Q after that pass (aggregation keeps
    Q), levels nest, the last level is the membership of louvain_run."""
    g, og = rmat25
    memb, res = lv.run(g, substeps=K_CLASSES)
    memb2, levels, res2 = lv.run_levels(g, substeps=K_CLASSES)
    torch.cuda.synchronize()
    assert res2["qnum"] == res["qnum"] and res2["qnum_pass"] == res["qnum_pass"]
    m = memb.cpu().numpy()
    assert np.array_equal(memb2.cpu().numpy(), m)
    L = levels.cpu().numpy()
    assert L.shape[0] >= 1 and np.array_equal(L[-1], m)
    for l in range(L.shape[0]):
        print(f"level {l}: oracle modularity", flush=True)
        qnum, W, _ = O.modularity(og, L[l])
        assert qnum == res["qnum_pass"][l] and W == res["W"], l
        k = int(L[l].max()) + 1
        if l + 1 < res["passes"]:
            assert k == res["n_pass"][l + 1]
        if l > 0:
            # nesting: the finer label determines the coarser one
            coarse = np.full(int(L[l - 1].max()) + 1, -1, dtype=np.int64)
            coarse[L[l - 1]] = L[l]
            assert np.array_equal(coarse[L[l - 1]], L[l]), l


@pytest.mark.timeout(600)
def test_rmat25_aggregate(lv, rmat25, rmat25_iter0):
    g, og = rmat25
    st0, st, _ = rmat25_iter0
    C = st.C
    mp, (n2, off, idx, w) = lv.aggregate(g, torch.from_numpy(C).to("cuda:0"))
    torch.cuda.synchronize()
    labels, inv = np.unique(C, return_inverse=True)
    assert n2 == labels.size
    assert np.array_equal(mp.cpu().numpy(), inv.astype(np.int32))
    off = off.cpu().numpy()
    idx = idx.cpu().numpy()
    w = w.cpu().numpy().view(np.uint64)
    # every super-vertex's weighted degree is its community's Sigma, and W is preserved
    w_ext = np.append(w, np.uint64(0))
    rowsum = np.add.reduceat(w_ext, off[:-1])
    empty = off[1:] == off[:-1]
    rowsum = np.where(empty, np.uint64(0), rowsum)
    assert np.array_equal(rowsum.astype(np.uint64), st.Sig[labels])
    assert int(w.sum(dtype=np.uint64)) == st0.W
    # rows hold distinct neighbours
    rows = np.repeat(np.arange(n2, dtype=np.int64), np.diff(off))
    key = rows * n2 + idx
    assert np.unique(key).size == key.size
    # sampled super-rows against their definition: sum of w over arcs (i, j) with
    # map[i] = a, by target map[j]
    rng = np.random.default_rng(1)
    deg2 = np.diff(off)
    big = np.argsort(deg2)[-20:]
    sample = np.unique(np.concatenate([rng.choice(n2, 200, replace=False), big]))
    newid = inv.astype(np.int64)
    members_mask = np.isin(newid, sample)
    verts = np.nonzero(members_mask)[0]
    starts, ends = og.off[verts], og.off[verts + 1]
    lens = ends - starts
    arc_pos = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens) + \
        np.arange(lens.sum())
    src = np.repeat(newid[verts], lens)
    dst = newid[og.idx[arc_pos]]
    wt = og.w[arc_pos]
    k2 = src * n2 + dst
    order = np.argsort(k2, kind="stable")
    k2, wt = k2[order], wt[order]
    uk, first = np.unique(k2, return_index=True)
    sums = np.add.reduceat(wt, first)
    expect = {}
    for key_, val in zip(uk.tolist(), sums.tolist()):
        expect.setdefault(key_ // n2, {})[key_ % n2] = val
    for a in sample.tolist():
        got = dict(zip(idx[off[a]:off[a + 1]].tolist(), w[off[a]:off[a + 1]].tolist()))
        assert got == expect.get(a, {}), a


@pytest.fixture(scope="module")
def rmat22(gpu_device):
    g = config_graph("rmat22", device="cuda:0")
    return g, O.Graph.from_csr(g)


@pytest.mark.timeout(900)
def test_rmat22_whole_run_exact(lv, rmat22):
    g, og = rmat22
    print("oracle: whole synchronous run on rmat22", flush=True)
    top, ref = O.run(og, "sync", substeps=K_CLASSES, levels=True)
    memb, res = lv.run(g, substeps=K_CLASSES)
    torch.cuda.synchronize()
    assert np.array_equal(memb.cpu().numpy(), top)
    assert res["qnum"] == ref["qnum"] and res["iterations"] == ref["iterations"]
    assert [t["S"] for t in res["trace"]] == ref["trace_S"]
    assert [t["moved"] for t in res["trace"]] == ref["trace_moved"]
    assert res["qnum_pass"] == ref["qnum_pass"] and res["nnz_pass"] == ref["nnz_pass"]
    # per-kernel events: the tiers of s22's class steps run concurrently on three streams
    from .test_gpu_parity import check_trace_times
    traced, res3 = lv.run(g, substeps=K_CLASSES, flags=0x2)
    torch.cuda.synchronize()
    check_trace_times(res3, traced, memb)
    assert sum(t["hub_ms"] for t in res3["trace"]) > 0
    # the dendrogram, level by level
    memb2, levels, res2 = lv.run_levels(g, substeps=K_CLASSES)
    torch.cuda.synchronize()
    assert np.array_equal(memb2.cpu().numpy(), top) and res2["qnum"] == ref["qnum"]
    L = levels.cpu().numpy()
    assert L.shape == ref["levels"].shape
    for l in range(L.shape[0]):
        assert np.array_equal(L[l], ref["levels"][l]), l


@pytest.mark.timeout(900)
def test_rmat22_quality_vs_async(lv, rmat22):
    g, og = rmat22
    print("oracle: sequential asynchronous run on rmat22", flush=True)
    _, ra = O.run(og, "async")
    _, res = lv.run(g, substeps=K_CLASSES)
    print(f"rmat22: Q gpu {res['q']:.6f}, Q async {ra['q']:.6f}", flush=True)
    assert res["q"] >= ra["q"] - 0.01


@pytest.mark.timeout(900)
def test_batched_workload_sampled(lv):
    """The 2048-graph batch in one louvain_run_batched call, as bench.py times it; every graph's
    community count and the Qnum of a sample of graphs (the largest ones and a spread of the
    rest) against the oracle's run on the graph alone."""
    from graphgen import batch_config, pack_graphs
    print("generating the 2048-graph batch on the GPU", flush=True)
    graphs = batch_config(2048, device="cuda:0")
    packed, vptr, aptr = pack_graphs(graphs, device="cuda:0")
    memb, res = lv.run_batched(packed, vptr, aptr, substeps=K_CLASSES)
    torch.cuda.synchronize()
    memb = memb.cpu().numpy()
    for g in range(len(graphs)):
        m = memb[vptr[g]:vptr[g + 1]]
        assert m.min() >= 0 and m.max() == res[g]["n_communities"] - 1, g
    sizes = np.array([gr.n for gr in graphs])
    sample = sorted(set(np.argsort(sizes)[-4:].tolist()) | set(range(0, 2048, 97)))
    worst = 1.0
    for g in sample:
        gr = graphs[g].to("cpu")
        og = O.Graph.from_csr(gr)
        top, ref = O.run(og, "sync", substeps=K_CLASSES)
        assert np.array_equal(memb[vptr[g]:vptr[g + 1]], top), g
        assert res[g]["qnum"] == ref["qnum"] and res[g]["iterations"] == ref["iterations"], g
        # quality gate: within 0.01 of the sequential asynchronous rule on the same graph
        _, ra = O.run(og, "async")
        assert res[g]["q"] >= ra["q"] - 0.01, (g, res[g]["q"], ra["q"])
        worst = min(worst, res[g]["q"] - ra["q"])
    print(f"checked {len(sample)} of 2048 graphs against the oracle; worst Q - Q_async "
          f"{worst:+.5f}", flush=True)


@pytest.mark.timeout(900)
def test_prepare_rmat25_edge_list_sampled(lv):
    """Graph preparation at full size (the raw R-MAT s25 edge list, 5.4e8 edges, with the
    paper's recipe), as bench.py --workload prepare times it: sampled rows (the longest, the
    first, the last and a spread) against the oracle's per-row definition, and properties over
    all rows: one loop per vertex, unit weights, strictly ascending rows, nnz = offsets[n]."""
    from graphgen import rmat_edges
    from paper_2301_12390_amd import LV_PREP_PAPER
    print("generating the rmat25 edge list", flush=True)
    n, u, v = rmat_edges(25, device="cuda:0")
    src = u.to(torch.int32).contiguous()
    dst = v.to(torch.int32).contiguous()
    del u, v
    g = lv.prepare(n, src, dst, flags=LV_PREP_PAPER)
    torch.cuda.synchronize()
    off = g.offsets
    assert int(off[0]) == 0 and int(off[-1]) == g.nnz
    deg = off[1:] - off[:-1]
    assert int(deg.min()) >= 1
    assert bool((g.weights == 1).all())
    rows = torch.repeat_interleave(torch.arange(n, device="cuda:0"), deg)
    same = rows[1:] == rows[:-1]
    assert bool((g.indices[1:][same] > g.indices[:-1][same]).all())
    # every vertex's loop
    assert int(((g.indices.to(torch.int64) == rows)).sum()) == n
    del rows, same
    hs, hd = src.cpu().numpy(), dst.cpu().numpy()
    ho = off.cpu().numpy()
    hi = g.indices.cpu().numpy()
    picks = [int(torch.argmax(deg)), 0, n - 1] + list(range(7, n, n // 5))
    for r in picks:
        print(f"oracle row {r}", flush=True)
        ri, rw = O.prepare_row(n, hs, hd, None, O.PREP_SYM | O.PREP_LOOPS | O.PREP_MAX, r)
        assert np.array_equal(hi[ho[r]:ho[r + 1]], ri), r
        assert (rw == 1).all()


@pytest.mark.timeout(900)
def test_rmat22_partitioned_exact(lv, rmat22):
    """Partition and merge at P = 8 (one part per XCD) on R-MAT s22, whole result exact."""
    g, og = rmat22
    print("oracle: partitioned run on rmat22", flush=True)
    top, ref, parts = O.run_partitioned(og, O.balanced_parts(og, 8), substeps=K_CLASSES)
    memb, res, pr = lv.run_partitioned(g, P=8, substeps=K_CLASSES)
    torch.cuda.synchronize()
    assert np.array_equal(memb.cpu().numpy(), top)
    assert res["qnum"] == ref["qnum"] and res["iterations"] == ref["iterations"]
    assert [p["qnum"] for p in pr] == [p["qnum"] for p in parts]


@pytest.mark.timeout(600)
def test_rmat25_partitioned(lv, rmat25):
    """At full size (1.05e9 arcs, more than one pass of any capped grid covers). P = 1: the one
    part is the whole graph, so its run equals louvain_run exactly (membership and Qnum), a
    property that holds at any size. P = 8: the final partition's Qnum on the input graph,
    recomputed by the oracle, equals the merge run's (aggregation keeps Q); labels dense; and
    every part's W is the weight of its induced subgraph, which the oracle counts directly."""
    g, og = rmat25
    m1, r1 = lv.run(g, substeps=K_CLASSES)
    memb, res, pr = lv.run_partitioned(g, P=1, substeps=K_CLASSES)
    torch.cuda.synchronize()
    assert pr[0]["qnum"] == r1["qnum"] and pr[0]["iterations"] == r1["iterations"]
    assert pr[0]["n_communities"] == r1["n_communities"]
    memb, res, pr = lv.run_partitioned(g, P=8, substeps=K_CLASSES)
    torch.cuda.synchronize()
    m = memb.cpu().numpy()
    k = res["n_communities"]
    assert m.min() >= 0 and m.max() == k - 1 and np.unique(m).size == k
    qnum, W, _ = O.modularity(og, m)
    assert qnum == res["qnum"] and W == res["W"]
    vptr = O.balanced_parts(og, 8)
    for p in range(8):
        lo, hi = vptr[p], vptr[p + 1]
        a0, a1 = og.off[lo], og.off[hi]
        inside = (og.idx[a0:a1] >= lo) & (og.idx[a0:a1] < hi)
        assert pr[p]["W"] == int(og.w[a0:a1][inside].sum()), p
