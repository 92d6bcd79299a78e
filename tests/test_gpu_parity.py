"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit for bit.

Per iteration (louvain_move with max_iterations = 1): C, Sigma, csize, S, moved count and the
number of candidate pairs. Per call: modularity (exact W^2 Q), aggregation (canonicalised
super-vertex CSR and map), and whole runs (membership, exact Q, iterations per pass, per-
iteration S and moves).
"""

import numpy as np
import pytest
import torch

import oracle as O
from graphgen import (add_self_loops, csr_from_arcs, erdos_renyi, lattice_shortcuts,
                      planted_hubs, rmat, ring_of_cliques, sbm, single_edge, two_triangles)
from graphgen.csr import Csr

from .gpu_util import assert_state_equal, canonical_rows_fast, gpu_state

pytestmark = pytest.mark.gpu

LV_FORCE_WIDE = 0x4
LV_SMALL_PARTS = 0x8  # many hash partitions with tiny tables: multi-partition, multi-round paths
LV_GRAPH_REPLAY = 0x20  # iterations of small phases replayed as captured HIP graphs


@pytest.fixture(scope="module")
def lv(gpu_device):
    from paper_2301_12390_amd import Louvain, build as B
    if not __import__("os").path.exists(B.LIB):
        B.build()
    ctx = Louvain(0)
    yield ctx
    ctx.close()


def star(n_leaves: int, weight_fn=None) -> Csr:
    u = torch.zeros(n_leaves, dtype=torch.int64)
    v = torch.arange(1, n_leaves + 1)
    from graphgen import csr_from_edges
    return csr_from_edges(n_leaves + 1, u, v, weight_fn, name=f"star{n_leaves}")


def dup_arcs_graph() -> Csr:
    # duplicate arcs and self-loops in rows (allowed by the input contract)
    src = torch.tensor([0, 0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 4, 4, 4])
    dst = torch.tensor([1, 1, 2, 0, 0, 1, 0, 2, 3, 2, 4, 3, 4, 4])
    w = torch.tensor([2, 3, 1, 3, 2, 7, 1, 5, 4, 4, 2, 2, 1, 1])
    return csr_from_arcs(5, src, dst, w, name="dup-arcs")


def corpus():
    gs = [
        two_triangles(),
        single_edge(),
        ring_of_cliques(8, 5),
        ring_of_cliques(30, 5),
        dup_arcs_graph(),
        add_self_loops(erdos_renyi(300, 0.03, seed=4, weights=(1, 9))),
        erdos_renyi(200, 0.05, seed=5, weights=(1, 9), self_loops=True),
        sbm(3000, 30, 8.0, 2.0, seed=2, weights=(1, 16)),
        lattice_shortcuts(5000, seed=3),
        rmat(12, seed=7),
        rmat(14, seed=3, weights=(1, 16), offsets_dtype=torch.int64),
        star(3000),
    ]
    return gs


CORPUS = corpus()
IDS = [g.name for g in CORPUS]


def run_iterations(lv, g, st, flags=0, max_iters=40, ctx="", substeps=1, pass_index=0):
    """Alternate one GPU iteration and one oracle iteration from the same state."""
    og = O.Graph.from_csr(g)
    dg = g.to("cuda:0")
    C, Sig, cs, K = gpu_state(st)
    classes = O.class_lists(g.n, pass_index, substeps)
    for it in range(max_iters):
        stats = lv.move(dg, C, Sig, cs, K=K, W=st.W, max_iterations=1, flags=flags,
                        substeps=substeps, pass_index=pass_index)
        S, moved, ncand = O.substep_iteration(og, st, pass_index, substeps, classes)
        torch.cuda.synchronize()
        assert_state_equal(st, C, Sig, cs, f"{ctx} iteration {it}")
        assert stats["last_gain"] == S, (ctx, it, stats["last_gain"], S)
        assert stats["last_moved"] == moved, (ctx, it)
        assert stats["last_candidates"] == ncand, (ctx, it, stats["last_candidates"], ncand)
        if moved == 0:
            return it + 1
    return max_iters


@pytest.mark.parametrize("K", [1, 8])
@pytest.mark.parametrize("g", CORPUS, ids=IDS)
def test_move_iterations_from_singletons(lv, g, K):
    st = O.State(O.Graph.from_csr(g))
    run_iterations(lv, g, st, ctx=g.name, substeps=K)


@pytest.mark.parametrize("g", CORPUS, ids=IDS)
def test_move_iterations_wide_arithmetic(lv, g):
    st = O.State(O.Graph.from_csr(g))
    run_iterations(lv, g, st, flags=0x4, max_iters=6, ctx=g.name + " wide")
    st = O.State(O.Graph.from_csr(g))
    run_iterations(lv, g, st, flags=0x4, max_iters=4, ctx=g.name + " wide K3", substeps=3,
                   pass_index=2)


@pytest.mark.parametrize("g", CORPUS[2:], ids=IDS[2:])
def test_move_iterations_from_random_partition(lv, g):
    rng = np.random.default_rng(11)
    C = rng.integers(0, max(2, g.n // 7), size=g.n).astype(np.int32)
    st = O.State(O.Graph.from_csr(g), C)
    run_iterations(lv, g, st, max_iters=5, ctx=g.name + " random")
    st = O.State(O.Graph.from_csr(g), C)
    run_iterations(lv, g, st, max_iters=5, ctx=g.name + " random K5", substeps=5, pass_index=1)


def test_move_hub_with_large_community(lv):
    # a star whose leaves already sit in a few large communities: the hub's row is long and
    # its candidate set small, and the leaves see huge Sigma values
    g = star(5000, weight_fn=lambda lo, hi: (hi % 13) + 1)
    C = (np.arange(g.n) % 4).astype(np.int32)
    st = O.State(O.Graph.from_csr(g), C)
    run_iterations(lv, g, st, max_iters=4, ctx="star partition")


def hub_graphs():
    """Rows far longer than a workgroup table (two-phase hub path of the move, and of the merge
    once the hubs' neighbourhoods form communities)."""
    return [
        planted_hubs(sbm(40000, 400, 8.0, 2.0, seed=4, weights=(1, 16)),
                     [100000, 33000, 17000, 9000, 5000], seed=2, weights=(1, 16)),
        planted_hubs(rmat(14, seed=3), [60000, 20000], seed=5),
    ]


HUBS = hub_graphs()
HUB_IDS = ["sbm40k+hubs", "rmat14+hubs"]
PART_FLAGS = [0, LV_SMALL_PARTS, LV_SMALL_PARTS | LV_FORCE_WIDE]


def test_hub_graphs_have_hub_rows():
    # rows of more than 8192 arcs take the two-phase hub path, in more than one chunk
    for g in HUBS:
        assert int(g.degrees().max()) > 8192


@pytest.mark.parametrize("flags", PART_FLAGS)
@pytest.mark.parametrize("K", [1, 8])
@pytest.mark.parametrize("gi", [0, 1], ids=HUB_IDS)
def test_move_iterations_hub_rows(lv, gi, K, flags):
    g = HUBS[gi]
    st = O.State(O.Graph.from_csr(g))
    run_iterations(lv, g, st, flags=flags, max_iters=8, substeps=K,
                   ctx=f"{g.name} K{K} flags{flags}")
    # hubs whose neighbours sit in a few large communities
    C = (np.arange(g.n) % 5).astype(np.int32)
    st = O.State(O.Graph.from_csr(g), C)
    run_iterations(lv, g, st, flags=flags, max_iters=3, substeps=K, pass_index=1,
                   ctx=f"{g.name} K{K} flags{flags} mod5")


@pytest.mark.parametrize("flags", PART_FLAGS)
@pytest.mark.parametrize("gi", [0, 1], ids=HUB_IDS)
def test_run_hub_graphs(lv, gi, flags):
    check_run(lv, HUBS[gi], flags=flags)


@pytest.mark.parametrize("g", CORPUS, ids=IDS)
def test_run_small_partitions(lv, g):
    # the large communities of the aggregation take the multi-partition, multi-round path
    check_run(lv, g, flags=LV_SMALL_PARTS)


@pytest.mark.parametrize("g", CORPUS, ids=IDS)
def test_modularity(lv, g):
    og = O.Graph.from_csr(g)
    dg = g.to("cuda:0")
    rng = np.random.default_rng(3)
    for C in [np.arange(g.n, dtype=np.int32), np.zeros(g.n, dtype=np.int32),
              rng.integers(0, max(1, g.n // 5), size=g.n).astype(np.int32)]:
        q, W, qd = lv.modularity(dg, torch.from_numpy(C).to("cuda:0"))
        qo, Wo, _ = O.modularity(og, C)
        assert (q, W) == (qo, Wo)
        assert abs(qd - qo / (Wo * Wo)) <= 4e-16 * max(1.0, abs(qd))


@pytest.mark.parametrize("iso", [0, 2, 20])
def test_row_sums_row_spans(lv, iso):
    # row sums (through W and the singleton Qnum) when a 4096-arc tile spans a few hundred, about
    # a thousand, or several thousand rows (isolated vertices between the rows with arcs), with
    # self-loops in the rows, and a whole run on each
    base = erdos_renyi(3000, 0.004, seed=21, weights=(1, 7), self_loops=True)
    n = base.n * (iso + 1)
    off = base.offsets.numpy().astype(np.int64)
    deg = np.diff(off)
    rows = np.repeat(np.arange(base.n) * (iso + 1), deg)
    cols = base.indices.numpy().astype(np.int64) * (iso + 1)
    g = csr_from_arcs(n, torch.from_numpy(rows), torch.from_numpy(cols), base.weights,
                      name=f"er3000x{iso + 1}")
    og = O.Graph.from_csr(g)
    C = np.arange(n, dtype=np.int32)
    q, W, _ = lv.modularity(g.to("cuda:0"), torch.from_numpy(C).to("cuda:0"))
    qo, Wo, _ = O.modularity(og, C)
    assert (q, W) == (qo, Wo)
    check_run(lv, g)


@pytest.mark.parametrize("g", CORPUS, ids=IDS)
@pytest.mark.parametrize("offsets_64", [True, False])
def test_aggregate(lv, g, offsets_64):
    og = O.Graph.from_csr(g)
    dg = g.to("cuda:0")
    rng = np.random.default_rng(5)
    cases = [rng.integers(0, max(1, g.n // 4), size=g.n).astype(np.int32),
             np.arange(g.n, dtype=np.int32), np.zeros(g.n, dtype=np.int32)]
    st = O.State(og)
    O.sync_iteration(og, st)
    cases.append(st.C.copy())
    for C in cases:
        mp, (n2, off, idx, w) = lv.aggregate(dg, torch.from_numpy(C).to("cuda:0"),
                                             offsets_64=offsets_64)
        mo, g2 = O.aggregate(og, C)
        assert np.array_equal(mp.cpu().numpy(), mo)
        assert n2 == g2.n
        off_c, idx_c, w_c = canonical_rows_fast(n2, off.cpu().numpy(), idx.cpu().numpy(),
                                                w.cpu().numpy())
        assert np.array_equal(off_c, g2.off)
        assert np.array_equal(idx_c, g2.idx)
        assert np.array_equal(w_c, g2.w)


@pytest.mark.parametrize("offsets_64", [True, False])
def test_aggregate_community_classes(lv, offsets_64):
    # communities of about 60 to 20,000 arcs, scattered over the vertex ids, so that every
    # aggregation tier gets some: up to 1024 arcs, 1025-2048, 2049-4096 (one workgroup each),
    # 4097-8192 and longer (two-phase)
    g = erdos_renyi(4000, 0.005, seed=11, weights=(1, 9))
    if offsets_64:
        g = g.with_offsets(torch.int64)
    sizes = [3, 30, 60, 120, 250, 500, 1000]
    blocks, v, k = [], 0, 0
    while v < g.n:
        s = min(sizes[k % len(sizes)], g.n - v)
        blocks.append(np.full(s, k, dtype=np.int32))
        v += s
        k += 1
    rng = np.random.default_rng(17)
    labels = rng.permutation(g.n)[:k].astype(np.int32)
    C = labels[np.concatenate(blocks)][rng.permutation(g.n)]
    deg = np.diff(g.offsets.numpy())
    arcs = np.bincount(C, weights=deg, minlength=g.n)
    for lo, hi in [(1024, 2048), (2048, 4096), (4096, 8192), (8192, 1 << 40)]:
        assert ((arcs > lo) & (arcs <= hi)).any(), (lo, hi)
    og = O.Graph.from_csr(g)
    mp, (n2, off, idx, w) = lv.aggregate(g.to("cuda:0"), torch.from_numpy(C).to("cuda:0"),
                                         offsets_64=offsets_64)
    mo, g2 = O.aggregate(og, C)
    assert np.array_equal(mp.cpu().numpy(), mo)
    assert n2 == g2.n
    off_c, idx_c, w_c = canonical_rows_fast(n2, off.cpu().numpy(), idx.cpu().numpy(),
                                            w.cpu().numpy())
    assert np.array_equal(off_c, g2.off)
    assert np.array_equal(idx_c, g2.idx)
    assert np.array_equal(w_c, g2.w)


def check_run(lv, g, flags=0, substeps=8, **kw):
    og = O.Graph.from_csr(g)
    okw = {{"tolerance_exp10": "a", "decline_exp10": "b"}.get(k, k): v for k, v in kw.items()}
    top, ref = O.run(og, "sync", substeps=substeps, **okw)
    memb, res = lv.run(g.to("cuda:0"), flags=flags, substeps=substeps, **kw)
    torch.cuda.synchronize()
    assert np.array_equal(memb.cpu().numpy(), top), g.name
    assert res["qnum"] == ref["qnum"] and res["W"] == ref["W"]
    assert res["passes"] == ref["passes"]
    assert res["iterations"] == ref["iterations"]
    assert res["n_pass"] == ref["n_pass"] and res["nnz_pass"] == ref["nnz_pass"]
    assert res["qnum_pass"] == ref["qnum_pass"]
    assert res["n_communities"] == ref["n_communities"]
    assert res["cap_hits"] == ref["cap_hits"]
    assert [t["S"] for t in res["trace"]] == ref["trace_S"]
    assert [t["moved"] for t in res["trace"]] == ref["trace_moved"]
    assert [t["candidates"] for t in res["trace"]] == ref["trace_ncand"]
    return res, ref


@pytest.mark.parametrize("K", [1, 8])
@pytest.mark.parametrize("g", CORPUS, ids=IDS)
def test_run(lv, g, K):
    check_run(lv, g, substeps=K)


@pytest.mark.parametrize("K", [1, 8])
@pytest.mark.parametrize("g", CORPUS, ids=IDS)
def test_run_graph_replay(lv, g, K):
    # iterations after the first replayed as a HIP graph captured once per phase: the same
    # results as direct launches (both are compared with the oracle)
    check_run(lv, g, flags=LV_GRAPH_REPLAY, substeps=K)


@pytest.mark.parametrize("K", [2, 3, 32])
def test_run_other_class_counts(lv, K):
    check_run(lv, sbm(3000, 30, 8.0, 2.0, seed=2, weights=(1, 16)), substeps=K)
    check_run(lv, rmat(13, seed=9), substeps=K)


def test_run_parameters(lv):
    g = sbm(4000, 40, 8.0, 2.0, seed=9, weights=(1, 16))
    for kw in [dict(tolerance_exp10=0), dict(tolerance_exp10=6, decline_exp10=2),
               dict(max_iterations=1), dict(max_iterations=3, max_passes=2),
               dict(max_passes=1)]:
        check_run(lv, g, **kw)
    check_run(lv, g, flags=0x4)  # 128-bit gains everywhere: identical results
    check_run(lv, g, flags=0x4, substeps=1)


SWEEP = [(0, 1), (1, 1), (3, 1), (4, 1), (6, 1), (8, 1), (12, 1), (2, 2), (2, 3), (2, 4)]


@pytest.mark.parametrize("a,b", SWEEP, ids=[f"tol1e-{a}-decl1e{b}" for a, b in SWEEP])
def test_run_tolerance_sweep(lv, a, b):
    # the tolerance / decline-factor study of bench.py --workload sweep, against the oracle
    check_run(lv, sbm(3000, 30, 8.0, 2.0, seed=2, weights=(1, 16)), tolerance_exp10=a,
              decline_exp10=b)
    check_run(lv, rmat(13, seed=9), tolerance_exp10=a, decline_exp10=b)


def test_run_sbm10k(lv):
    from graphgen import config_graph
    g = config_graph("sbm10k")
    res, ref = check_run(lv, g)
    _, ra = O.run(O.Graph.from_csr(g), "async")
    assert res["q"] >= ra["q"] - 0.01
    check_run(lv, g, substeps=1)


def test_run_rmat16_hubs(lv):
    g = rmat(16, seed=1)
    deg = g.degrees()
    assert int(deg.max()) > 1024  # hub path exercised
    res, ref = check_run(lv, g)
    _, ra = O.run(O.Graph.from_csr(g), "async")
    assert res["q"] >= ra["q"] - 0.01, (res["q"], ra["q"])
    # the fully synchronous rule matches its oracle too (its quality is lower on this graph)
    check_run(lv, g, substeps=1)
    check_run(lv, g, flags=LV_SMALL_PARTS)


def test_run_deterministic(lv):
    g = rmat(15, seed=5, weights=(1, 16))
    dg = g.to("cuda:0")
    a, ra = lv.run(dg)
    b, rb = lv.run(dg)
    assert torch.equal(a, b) and ra["qnum"] == rb["qnum"]
    assert [t["S"] for t in ra["trace"]] == [t["S"] for t in rb["trace"]]


def test_generator_same_on_gpu():
    from graphgen import csr_sha256
    for make in [lambda d: sbm(3000, 30, 8.0, 2.0, seed=2, weights=(1, 16), device=d),
                 lambda d: rmat(14, seed=3, weights=(1, 16), offsets_dtype=torch.int64,
                                device=d)]:
        assert csr_sha256(make("cpu")) == csr_sha256(make("cuda:0"))


def test_empty_and_edgeless(lv):
    dev = "cuda:0"
    g = Csr(0, torch.zeros(1, dtype=torch.int32, device=dev),
            torch.zeros(0, dtype=torch.int32, device=dev),
            torch.zeros(0, dtype=torch.int32, device=dev))
    memb, res = lv.run(g)
    assert memb.numel() == 0 and res["passes"] == 0 and res["qnum"] == 0
    g = Csr(5, torch.zeros(6, dtype=torch.int32, device=dev),
            torch.zeros(0, dtype=torch.int32, device=dev),
            torch.zeros(0, dtype=torch.int32, device=dev))
    memb, res = lv.run(g)
    assert memb.cpu().tolist() == list(range(5)) and res["q"] == 0.0 and res["passes"] == 0
    # only self-loops: nobody has a candidate
    g = csr_from_arcs(4, torch.arange(4), torch.arange(4), torch.tensor([1, 2, 3, 4])).to(dev)
    memb, res = lv.run(g)
    assert memb.cpu().tolist() == [0, 1, 2, 3]
    top, ref = O.run(O.Graph.from_csr(g), "sync")
    assert res["qnum"] == ref["qnum"]


def check_trace_times(res, memb_traced, memb_plain):
    # per-kernel events change nothing, and every time derived from them is non-negative and
    # within its iteration (tier times from the class steps' shared start and end events)
    assert torch.equal(memb_traced, memb_plain)
    for t in res["trace"]:
        for k in ("fused_ms", "wg_ms", "hub_ms", "update_ms"):
            assert 0 <= t[k] <= t["iter_ms"] + 0.5, (k, t)
    for p in range(res["passes"] - 1):
        assert res["aggregate_ms"][p] >= 0


@pytest.mark.parametrize("g", [g for g in CORPUS if g.n >= 1000], ids=[g.name for g in CORPUS
                                                                     if g.n >= 1000])
def test_trace_times_serial_tiers(lv, g):
    # small graphs run their tiers one after another on one stream
    dg = g.to("cuda:0")
    plain, _ = lv.run(dg, substeps=8)
    traced, res = lv.run(dg, substeps=8, flags=0x2)
    torch.cuda.synchronize()
    check_trace_times(res, traced, plain)
    assert sum(t["fused_ms"] for t in res["trace"]) > 0


def test_errors(lv):
    from paper_2301_12390_amd import LouvainError
    g = two_triangles().to("cuda:0")
    with pytest.raises(LouvainError, match="EINVAL"):
        lv.run(g, max_iterations=0)
    with pytest.raises(LouvainError, match="EINVAL"):
        lv.run(g, max_passes=65)
    with pytest.raises(LouvainError, match="EINVAL"):
        lv.run(g, tolerance_exp10=-1)
    bad = Csr(6, g.offsets, g.indices.clone(), g.weights)
    bad.indices[3] = 99
    with pytest.raises(LouvainError, match="EINVAL"):
        lv.run(bad, flags=0x1)
    zero_w = Csr(6, g.offsets, g.indices, torch.zeros_like(g.weights))
    with pytest.raises(LouvainError, match="EINVAL"):
        lv.run(zero_w, flags=0x1)
    # the context stays usable after errors
    memb, res = lv.run(g)
    assert memb.cpu().tolist() == [0, 0, 0, 1, 1, 1]


def test_budget():
    from paper_2301_12390_amd import Louvain, LouvainError
    small = Louvain(0, hbm_budget=1 << 12)
    g = sbm(2000, 20, 8.0, 2.0, seed=1).to("cuda:0")
    with pytest.raises(LouvainError, match="EBUDGET"):
        small.run(g)
    small.close()
    big = Louvain(0, hbm_budget=1 << 30)
    memb, res = big.run(g)
    assert big.workspace_bytes() <= 1 << 30
    big.close()
