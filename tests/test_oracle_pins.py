"""Pins of the CPU oracle against facts that do not come from the oracle itself.

* closed forms (ring of cliques, all-in-one, singletons, single edge);
* a library (networkx modularity on self-loop-free graphs);
* the pairwise Newman-Girvan definition of modularity evaluated with exact fractions;
* brute force over all set partitions of tiny graphs;
* the hand-derived worked example in ``tests/golden/two_triangles.json``;
* invariants (exact modularity change of asynchronous moves, aggregation invariants,
  thread-count independence of the synchronous rule).
"""

import json
import os
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle as O
from graphgen import (csr_from_arcs, csr_from_edges, erdos_renyi, ring_of_cliques, sbm, single_edge,
                      two_triangles, add_self_loops)
from graphgen.rng import splitmix64_sequence

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------------------------
# independent helpers: definitions written from scratch with exact fractions


def arcs_of(g: O.Graph):
    for i in range(g.n):
        for e in range(g.off[i], g.off[i + 1]):
            yield i, int(g.idx[e]), int(g.w[e])


def q_pairwise(g: O.Graph, C) -> Fraction:
    """Newman-Girvan modularity from its pairwise definition,
    Q = (1/W) * sum_{i,j} [A_ij - K_i K_j / W] * delta(C_i, C_j), with A the arc-weight matrix
    (a self-loop's weight on the diagonal once) and K its row sums."""
    n = g.n
    A = {}
    K = [0] * n
    for i, j, w in arcs_of(g):
        A[(i, j)] = A.get((i, j), 0) + w
        K[i] += w
    W = sum(K)
    tot = Fraction(0)
    for i in range(n):
        for j in range(n):
            if C[i] == C[j]:
                tot += Fraction(A.get((i, j), 0)) - Fraction(K[i] * K[j], W)
    return tot / W


def random_partition(n, k, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, k, size=n).astype(np.int32)


def small_graphs():
    out = []
    for s in range(6):
        out.append(O.Graph.from_csr(erdos_renyi(9, 0.35, seed=s, weights=(1, 5))))
    for s in range(3):
        out.append(O.Graph.from_csr(erdos_renyi(8, 0.4, seed=10 + s, weights=(1, 7),
                                                self_loops=True)))
    out.append(O.Graph.from_csr(two_triangles()))
    out.append(O.Graph.from_csr(add_self_loops(two_triangles())))
    return out


# ----------------------------------------------------------------------------------------------
# generator


def test_splitmix64_published_vectors():
    # First outputs of SplitMix64 seeded with 0 (Steele, Lea, Flood 2014 reference generator).
    assert splitmix64_sequence(0, 4) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                         0x06C45D188009454F, 0xF88BB8A8724C81EC]


def test_generator_symmetric_simple():
    g = O.Graph.from_csr(sbm(600, 6, 8.0, 2.0, seed=3, weights=(1, 16)))
    arcs = {}
    for i, j, w in arcs_of(g):
        assert i != j
        assert (i, j) not in arcs
        arcs[(i, j)] = w
    for (i, j), w in arcs.items():
        assert arcs[(j, i)] == w


# ----------------------------------------------------------------------------------------------
# tolerance threshold (integer form of: the iteration's modularity change exceeds the tolerance)


def test_threshold_values():
    assert O.threshold(14, 2, 1, 0) == 0  # 196 / 200
    assert O.threshold(14, 2, 1, 1) == 0
    assert O.threshold(100000, 2, 1, 0) == 5 * 10**7
    assert O.threshold(100000, 2, 1, 1) == 5 * 10**6
    W = 2**62
    assert O.threshold(W, 0, 1, 0) == W * W // 2
    assert O.threshold(W, 2, 1, 3) == W * W // (2 * 10**5)
    assert O.threshold(W, 2, 1, 40) == 0


@pytest.mark.parametrize("W", [1, 7, 14, 999, 10**6 + 3, 2**40 + 1, 2**62])
def test_threshold_is_exact_floor(W):
    for a, b, p in [(2, 1, 0), (2, 1, 1), (2, 1, 5), (0, 1, 0), (3, 2, 2), (12, 4, 1)]:
        T = O.threshold(W, a, b, p)
        tol = Fraction(1, 10 ** (a + b * p))
        # S > T  <=>  2S/W^2 > tol for every integer S around the boundary
        for S in [T - 1, T, T + 1, T + 2]:
            if S < 0:
                continue
            assert (S > T) == (Fraction(2 * S, W * W) > tol)


# ----------------------------------------------------------------------------------------------
# modularity


@pytest.mark.parametrize("nc,k", [(8, 5), (30, 5), (4, 3), (5, 6)])
def test_modularity_ring_of_cliques_closed_form(nc, k):
    g = O.Graph.from_csr(ring_of_cliques(nc, k))
    C = np.repeat(np.arange(nc, dtype=np.int32), k)
    qnum, W, _ = O.modularity(g, C)
    L = k * (k - 1) // 2
    assert Fraction(qnum, W * W) == Fraction(L, L + 1) - Fraction(1, nc)


def test_modularity_closed_form_values():
    # ring of 8 K5 -> 69/88; 30 K5 -> 289/330; 4 K3 -> 1/2
    for (nc, k), q in [((8, 5), Fraction(69, 88)), ((30, 5), Fraction(289, 330)),
                       ((4, 3), Fraction(1, 2))]:
        g = O.Graph.from_csr(ring_of_cliques(nc, k))
        qnum, W, _ = O.modularity(g, np.repeat(np.arange(nc, dtype=np.int32), k))
        assert Fraction(qnum, W * W) == q


def test_modularity_all_in_one_and_singletons():
    for g in small_graphs():
        qnum, W, _ = O.modularity(g, np.zeros(g.n, dtype=np.int32))
        assert qnum == 0
        K = [0] * g.n
        loops = 0
        for i, j, w in arcs_of(g):
            K[i] += w
            if i == j:
                loops += w
        qnum, W, _ = O.modularity(g, np.arange(g.n, dtype=np.int32))
        assert qnum == W * loops - sum(x * x for x in K)


def test_modularity_single_edge():
    g = O.Graph.from_csr(single_edge())
    qnum, W, _ = O.modularity(g, np.array([0, 1], dtype=np.int32))
    assert Fraction(qnum, W * W) == Fraction(-1, 2)
    qnum, W, _ = O.modularity(g, np.array([0, 0], dtype=np.int32))
    assert qnum == 0


def test_modularity_matches_networkx():
    nx = pytest.importorskip("networkx")
    for s in range(8):
        g = O.Graph.from_csr(erdos_renyi(40, 0.12, seed=100 + s, weights=(1, 9)))
        G = nx.Graph()
        G.add_nodes_from(range(g.n))
        for i, j, w in arcs_of(g):
            if i < j:
                G.add_edge(i, j, weight=w)
        C = random_partition(g.n, 5, s)
        comms = [set(np.nonzero(C == c)[0].tolist()) for c in range(5)]
        comms = [c for c in comms if c]
        qnx = nx.community.modularity(G, comms, weight="weight")
        qnum, W, _ = O.modularity(g, C)
        assert abs(qnum / (W * W) - qnx) < 1e-12


def test_modularity_matches_pairwise_definition_with_self_loops():
    for gi, g in enumerate(small_graphs()):
        for s in range(3):
            C = random_partition(g.n, 3, 1000 * gi + s)
            qnum, W, _ = O.modularity(g, C)
            assert Fraction(qnum, W * W) == q_pairwise(g, C)


# ----------------------------------------------------------------------------------------------
# gain formula: single-move identity against the pairwise definition


def test_single_move_identity():
    for gi, g in enumerate(small_graphs()):
        C = random_partition(g.n, 4, 77 + gi)
        st = O.State(g, C)
        q0 = q_pairwise(g, C)
        for i in range(g.n):
            gains, stay = O.vertex_gains(g, st, i)
            for c, gval in gains.items():
                C2 = C.copy()
                C2[i] = c
                dq = q_pairwise(g, C2) - q0
                assert dq == Fraction(2 * (gval - stay), st.W * st.W), (gi, i, c)


# ----------------------------------------------------------------------------------------------
# synchronous rule: every decision checked by brute force over modularity changes


def sync_decisions_bruteforce(g: O.Graph, C, subset=None):
    """Next membership and S under the synchronous rule, from modularity differences only.
    With ``subset``, only those vertices decide; the others keep their community."""
    n = g.n
    q0 = q_pairwise(g, C)
    W = sum(w for _, _, w in arcs_of(g))
    csize = {c: int((C == c).sum()) for c in set(C.tolist())}
    nbr = [set() for _ in range(n)]
    for i, j, _ in arcs_of(g):
        if i != j:
            nbr[i].add(int(C[j]))
    Cn = C.copy()
    S = Fraction(0)
    for i in (range(n) if subset is None else subset):
        d = int(C[i])
        best, best_dq = None, None
        for c in sorted(nbr[i] - {d}):
            C2 = C.copy()
            C2[i] = c
            dq = q_pairwise(g, C2) - q0
            if best is None or dq > best_dq:
                best, best_dq = c, dq
        if best is None or best_dq <= 0:
            continue
        if csize[d] == 1 and csize[best] == 1 and best > d:
            continue
        Cn[i] = best
        S += best_dq * W * W / 2
    assert S.denominator == 1
    return Cn, int(S)


def test_sync_iteration_bruteforce():
    for gi, g in enumerate(small_graphs()):
        for s in range(2):
            C = random_partition(g.n, 4 if s else g.n, 5 + gi * 10 + s)
            if s == 0:
                C = np.arange(g.n, dtype=np.int32)
            st = O.State(g, C)
            S, moved, _ = O.sync_iteration(g, st)
            Cn, Sb = sync_decisions_bruteforce(g, C)
            assert np.array_equal(st.C, Cn), (gi, s)
            assert S == Sb
            assert moved == int((Cn != C).sum())
            Sig2, cs2 = O.community_state(g, st.K, st.C)
            assert np.array_equal(Sig2, st.Sig) and np.array_equal(cs2, st.csize)


def path_graph(n):
    u = torch.arange(n - 1)
    return O.Graph.from_csr(csr_from_edges(n, u, u + 1))


def test_sync_zero_gain_move_not_taken():
    # path 0-1-2 with C = [0, 0, 2]: vertex 1 has stay = 4*1 - 2*(3-2) = 2 and
    # g(2) = 4*1 - 2*1 = 2, a move that does not increase modularity, so it stays
    g = path_graph(3)
    C = np.array([0, 0, 2], dtype=np.int32)
    st = O.State(g, C)
    gains, stay = O.vertex_gains(g, st, 1)
    assert gains == {2: 2} and stay == 2
    S, moved, _ = O.sync_iteration(g, st)
    Cn, Sb = sync_decisions_bruteforce(g, C)
    assert st.C.tolist() == Cn.tolist() == [0, 0, 0] and S == Sb == 1
    # unit-weight graphs have many such ties
    for s in range(4):
        g = O.Graph.from_csr(erdos_renyi(9, 0.4, seed=50 + s))
        C = random_partition(g.n, 3, s)
        st = O.State(g, C)
        O.sync_iteration(g, st)
        Cn, _ = sync_decisions_bruteforce(g, C)
        assert np.array_equal(st.C, Cn)


def test_vertex_class_matches_splitmix64():
    # class of v in pass p: upper 32 bits of the (v+1)-th SplitMix64 output from state p,
    # scaled to [0, K); computed here with Python integers, independently of the C code
    from graphgen.rng import GAMMA, MASK64, mix_int
    for p in (0, 1, 7):
        for K in (2, 3, 8, 32):
            for v in list(range(50)) + [12345, 2**31 - 1]:
                z = (p + (v + 1) * GAMMA) & MASK64
                expect = ((mix_int(z) >> 32) * K) >> 32
                assert O.vertex_class(p, K, v) == expect
    # the classes are near-uniform
    cls = [O.vertex_class(0, 8, v) for v in range(8000)]
    counts = np.bincount(cls, minlength=8)
    assert counts.min() > 850 and counts.max() < 1150


def test_sync_step_on_a_subset_bruteforce():
    for gi, g in enumerate(small_graphs()):
        rng = np.random.default_rng(40 + gi)
        for C in [np.arange(g.n, dtype=np.int32), random_partition(g.n, 3, gi)]:
            subset = sorted(rng.choice(g.n, size=max(1, g.n // 2), replace=False).tolist())
            st = O.State(g, C)
            S, moved, _ = O.sync_step(g, st, subset)
            Cn, Sb = sync_decisions_bruteforce(g, C, subset)
            assert np.array_equal(st.C, Cn) and S == Sb, gi


def test_substep_iteration_is_a_sequence_of_steps():
    g = O.Graph.from_csr(sbm(600, 6, 8.0, 2.0, seed=4, weights=(1, 16)))
    K = 4
    classes = O.class_lists(g.n, 0, K)
    assert sorted(np.concatenate(classes).tolist()) == list(range(g.n))
    st = O.State(g)
    ref = st.copy()
    S, moved, nc = O.substep_iteration(g, st, 0, K)
    S2 = m2 = 0
    for vs in classes:
        a, b, _ = O.sync_step(g, ref, vs)
        S2 += a
        m2 += b
    assert np.array_equal(st.C, ref.C) and S == S2 and moved == m2
    # with one class, a substep iteration is the synchronous iteration
    st1 = O.State(g)
    st2 = O.State(g)
    assert O.substep_iteration(g, st1, 0, 1) == O.sync_iteration(g, st2)
    assert np.array_equal(st1.C, st2.C)


def test_substep_run_bounded_by_optimum():
    for s in range(3):
        g = O.Graph.from_csr(erdos_renyi(8, 0.45, seed=70 + s, weights=(1, 4)))
        qo = q_opt_bruteforce(g)
        for K in (2, 4):
            top, res = O.run(g, "sync", substeps=K)
            assert Fraction(res["qnum"], res["W"] ** 2) <= qo
            assert O.modularity(g, top)[0] == res["qnum"]


def test_quality_substeps_vs_async():
    # the fully synchronous rule oscillates on skewed graphs; classes processed in turn
    # (partial asynchrony) stay within 0.01 of the asynchronous rule
    from graphgen import rmat
    g = O.Graph.from_csr(rmat(16, seed=1))
    _, ra = O.run(g, "async")
    _, r8 = O.run(g, "sync", substeps=8)
    assert r8["q"] >= ra["q"] - 0.01, (r8["q"], ra["q"])


def test_sync_thread_count_invariance():
    g = O.Graph.from_csr(sbm(3000, 30, 8.0, 2.0, seed=7, weights=(1, 16)))
    outs = []
    for t in (1, 3, 8):
        top, res = O.run(g, "sync", nthreads=t)
        outs.append((top.tolist(), res["trace_S"], res["qnum"]))
    assert outs[0] == outs[1] == outs[2]


# ----------------------------------------------------------------------------------------------
# asynchronous rule: every applied gain is the exact modularity change


def test_async_exact_change_per_iteration():
    for gi, g in enumerate(small_graphs() + [O.Graph.from_csr(sbm(500, 5, 8, 2, seed=9,
                                                                     weights=(1, 16)))]):
        st = O.State(g)
        q_prev, W, _ = O.modularity(g, st.C)
        for _ in range(6):
            S, moved = O.async_iteration(g, st)
            q, _, _ = O.modularity(g, st.C)
            assert q - q_prev == 2 * S
            assert S >= 0 and (moved > 0) == (S > 0)
            q_prev = q


# ----------------------------------------------------------------------------------------------
# aggregation invariants


def check_aggregation(g: O.Graph, C):
    st = O.State(g, C)
    mp, g2 = O.aggregate(g, C)
    labels = sorted(set(C.tolist()))
    rank = {c: r for r, c in enumerate(labels)}
    assert g2.n == len(labels)
    assert [rank[int(c)] for c in C] == mp.tolist()
    K2, W2 = O.degrees(g2)
    assert W2 == st.W
    assert K2.tolist() == [int(st.Sig[c]) for c in labels]
    arcs = {}
    for a, b, w in arcs_of(g2):
        assert (a, b) not in arcs
        arcs[(a, b)] = w
    for (a, b), w in arcs.items():
        assert arcs[(b, a)] == w
    for c in labels:
        sigma_c = sum(w for i, j, w in arcs_of(g) if C[i] == c and C[j] == c)
        assert arcs.get((rank[c], rank[c]), 0) == sigma_c
    for a in range(g2.n):
        row = g2.idx[g2.off[a]:g2.off[a + 1]]
        assert np.all(np.diff(row) > 0)
    q1, _, _ = O.modularity(g, C)
    q2, _, _ = O.modularity(g2, np.arange(g2.n, dtype=np.int32))
    assert q1 == q2


def test_aggregation_invariants():
    for gi, g in enumerate(small_graphs()):
        check_aggregation(g, random_partition(g.n, 3, 300 + gi))
        check_aggregation(g, np.arange(g.n, dtype=np.int32))
        check_aggregation(g, np.zeros(g.n, dtype=np.int32))
    g = O.Graph.from_csr(sbm(400, 8, 8, 2, seed=5, weights=(1, 16)))
    st = O.State(g)
    O.sync_iteration(g, st)
    O.sync_iteration(g, st)
    check_aggregation(g, st.C)


def test_aggregation_with_duplicate_arcs():
    # duplicate arcs in a row mean their summed weight
    src = torch.tensor([0, 0, 0, 0, 1, 1, 2, 2, 2])
    dst = torch.tensor([1, 1, 2, 2, 0, 0, 2, 0, 0])
    w = torch.tensor([2, 3, 1, 1, 3, 2, 4, 1, 1])
    g = O.Graph.from_csr(csr_from_arcs(3, src, dst, w))
    mp, g2 = O.aggregate(g, np.array([0, 1, 2], dtype=np.int32))
    rows = {a: dict(zip(g2.idx[g2.off[a]:g2.off[a + 1]].tolist(),
                        g2.w[g2.off[a]:g2.off[a + 1]].tolist())) for a in range(3)}
    assert rows == {0: {1: 5, 2: 2}, 1: {0: 5}, 2: {0: 2, 2: 4}}
    check_aggregation(g, np.array([0, 0, 1], dtype=np.int32))


# ----------------------------------------------------------------------------------------------
# worked example (golden)


def test_worked_example_two_triangles():
    gold = json.load(open(os.path.join(GOLDEN, "two_triangles.json")))
    g = O.Graph.from_csr(two_triangles())
    st = O.State(g)
    assert st.W == gold["W"] and st.K.tolist() == gold["K"]
    assert O.modularity(g, st.C)[0] == gold["qnum_singletons"]
    assert O.threshold(st.W, 2, 1, 0) == gold["threshold_pass0"]
    assert O.threshold(st.W, 2, 1, 1) == gold["threshold_pass1"]
    for i, rec in gold["iteration1_gains"].items():
        gains, stay = O.vertex_gains(g, st, int(i))
        assert {str(c): v for c, v in gains.items()} == rec["candidates"]
        assert stay == rec["stay"]
    for rec in gold["sync_iterations"]:
        S, moved, _ = O.sync_iteration(g, st)
        assert st.C.tolist() == rec["C"]
        assert {str(c): int(st.Sig[c]) for c in range(g.n) if st.csize[c]} == rec["Sigma"]
        assert {str(c): int(st.csize[c]) for c in range(g.n) if st.csize[c]} == rec["csize"]
        assert S == rec["S"] and moved == rec["moved"]
        assert O.modularity(g, st.C)[0] == rec["qnum"]
    mp, g2 = O.aggregate(g, st.C)
    assert mp.tolist() == gold["aggregate"]["map"] and g2.n == gold["aggregate"]["n"]
    arcs = [[a, b, w] for a, b, w in arcs_of(g2)]
    assert arcs == gold["aggregate"]["arcs"]
    st2 = O.State(g2)
    assert st2.K.tolist() == gold["aggregate"]["K"]
    assert O.modularity(g2, st2.C)[0] == gold["aggregate"]["qnum_singletons"]
    gains, stay = O.vertex_gains(g2, st2, 0)
    assert gains == {1: gold["pass1_merge_gain"]} and stay == 0
    top, res = O.run(g, "sync")
    assert top.tolist() == gold["final_membership"] and res["qnum"] == gold["final_qnum"]
    assert Fraction(res["qnum"], res["W"] ** 2) == Fraction(*gold["q_opt"])
    # asynchronous variant
    st = O.State(g)
    for S_exp, q_exp in zip(gold["async_iterations_S"], gold["async_qnum"]):
        S, _ = O.async_iteration(g, st)
        assert S == S_exp and O.modularity(g, st.C)[0] == q_exp
    assert st.C.tolist() == gold["async_labels_before_renumbering"]
    top, res = O.run(g, "async")
    assert top.tolist() == gold["final_membership"]


def test_single_edge_run():
    g = O.Graph.from_csr(single_edge())
    st = O.State(g)
    S, moved, _ = O.sync_iteration(g, st)
    # 1 -> 0 allowed, 0 -> 1 blocked by singleton-swap prevention
    assert st.C.tolist() == [0, 0] and moved == 1
    top, res = O.run(g, "sync")
    assert top.tolist() == [0, 0] and res["qnum"] == 0


def test_empty_graphs():
    g = O.Graph(0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.uint64))
    top, res = O.run(g, "sync")
    assert top.tolist() == [] and res["qnum"] == 0 and res["passes"] == 0
    g = O.Graph(5, np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0, np.uint64))
    top, res = O.run(g, "sync")
    assert top.tolist() == list(range(5)) and res["qnum"] == 0 and res["passes"] == 0


# ----------------------------------------------------------------------------------------------
# whole runs: brute-force optimum bounds the result; planted structure is recovered


def set_partitions(n):
    """Restricted growth strings of length n (every set partition once)."""
    a = [0] * n

    def rec(i, m):
        if i == n:
            yield list(a)
            return
        for v in range(m + 2):
            a[i] = v
            yield from rec(i + 1, max(m, v))

    if n == 0:
        yield []
        return
    a[0] = 0
    yield from rec(1, 0)


def q_opt_bruteforce(g: O.Graph) -> Fraction:
    best = None
    W = None
    for part in set_partitions(g.n):
        qnum, W, _ = O.modularity(g, np.array(part, dtype=np.int32))
        if best is None or qnum > best:
            best = qnum
    return Fraction(best, W * W)


def test_set_partition_count():
    assert sum(1 for _ in set_partitions(6)) == 203
    assert sum(1 for _ in set_partitions(8)) == 4140


def test_bruteforce_bounds_louvain():
    graphs = [O.Graph.from_csr(two_triangles())]
    graphs += [O.Graph.from_csr(erdos_renyi(8, 0.4, seed=s, weights=(1, 4))) for s in range(4)]
    for gi, g in enumerate(graphs):
        qo = q_opt_bruteforce(g)
        for mode in ("sync", "async"):
            top, res = O.run(g, mode)
            q = Fraction(res["qnum"], res["W"] ** 2)
            assert q <= qo, (gi, mode)
            if gi == 0:
                assert q == qo == Fraction(5, 14)


def test_ring_of_cliques_recovered():
    g = O.Graph.from_csr(ring_of_cliques(8, 5))
    for mode in ("sync", "async"):
        top, res = O.run(g, mode)
        assert res["n_communities"] == 8
        assert Fraction(res["qnum"], res["W"] ** 2) == Fraction(69, 88)
        assert top.tolist() == np.repeat(np.arange(8), 5).tolist()
        # the second pass makes no move: a merge gain is 176*1 - 22*22 < 0
        assert res["passes"] == 2 and res["iterations"][1] == 1


def test_quality_sync_vs_async_sbm10k():
    g = O.Graph.from_csr(sbm(10000, 100, 8.0, 2.0, seed=1))
    _, rs = O.run(g, "sync")
    _, ra = O.run(g, "async")
    # async passes never lower Q (every applied move raises it exactly; aggregation keeps it)
    qa = ra["qnum_pass"]
    assert all(qa[p + 1] >= qa[p] for p in range(len(qa) - 1))
    assert rs["q"] >= ra["q"] - 0.01


# ----------------------------------------------------------------------------------------------
# the hierarchy: membership of the input vertices after each aggregation


def check_levels(g: O.Graph, top, res):
    L = res["levels"]
    W = res["W"]
    assert L.shape[1] == g.n
    if W == 0 or len(L) == 0:
        return
    # the last level is the returned membership
    assert (L[-1] == top).all()
    for l in range(len(L)):
        k = int(L[l].max()) + 1
        # dense labels; the l-th aggregation leaves the vertex count the next pass starts with
        assert sorted(set(L[l].tolist())) == list(range(k))
        if l + 1 < res["passes"]:
            assert k == res["n_pass"][l + 1]
        # aggregation keeps Q: the l-th level, evaluated on the INPUT graph with the pairwise
        # definition, has the Q reported after the l-th local-moving phase
        assert q_pairwise(g, L[l]) == Fraction(res["qnum_pass"][l], W * W), l
        if l > 0:
            # each community of level l-1 lies inside one community of level l
            pairs = set(zip(L[l - 1].tolist(), L[l].tolist()))
            assert len(pairs) == len(set(L[l - 1].tolist()))


@pytest.mark.parametrize("mode,sub", [("sync", 1), ("sync", 8), ("async", 1)])
def test_levels_invariants(mode, sub):
    graphs = small_graphs() + [O.Graph.from_csr(ring_of_cliques(30, 3)),
                               O.Graph.from_csr(ring_of_cliques(64, 3))]
    for g in graphs:
        top, res = O.run(g, mode, substeps=sub, levels=True)
        plain, res2 = O.run(g, mode, substeps=sub)
        assert (plain == top).all() and res2["qnum"] == res["qnum"]
        check_levels(g, top, res)
        # an aggregation per pass, except a last pass in which nothing moved
        assert len(res["levels"]) in (res["passes"] - 1, res["passes"])


def test_levels_ring_of_k4_hand_derived():
    """Ring of 16 K4 cliques, asynchronous rule. Pass 0 gathers each clique (as in the (8, 5)
    ring). Pass 1 runs on a ring of 16 super-vertices with self-loop weight 12, ring weight 1,
    K = 14, W = 224: vertex 0 gains 224*1 - 14*14 = 28 towards either ring neighbour and takes
    the smaller id 1; vertex 1 then sees 28 for staying and 28 for moving on, so it stays;
    vertex 2 sees 224 - 14*28 < 0 towards {0, 1} and 28 towards 3, and so on: the cliques pair
    up as {2j, 2j+1}. Pass 2: merging two pairs gains 224*1 - 28*28 < 0, nothing moves.
    Qnum (= W^2 Q) of the two levels: 16 (12*224 - 14^2) and 8 (26*224 - 28^2)."""
    g = O.Graph.from_csr(ring_of_cliques(16, 4))
    top, res = O.run(g, "async", levels=True)
    v = np.arange(64)
    L = res["levels"]
    assert len(L) == 2 and res["passes"] == 3
    assert (L[0] == v // 4).all()
    assert (L[1] == v // 8).all()
    assert res["qnum_pass"][:2] == [16 * (12 * 224 - 14 ** 2), 8 * (26 * 224 - 28 ** 2)]
    check_levels(g, top, res)


def test_levels_edge_cases():
    # no arcs: no level; a single edge: one level joining the two ends
    g = O.Graph.from_csr(single_edge())
    top, res = O.run(g, "sync", levels=True)
    assert res["levels"].tolist() == [[0, 0]]
    # max_passes = 1 caps the hierarchy at one level
    g = O.Graph.from_csr(ring_of_cliques(64, 3))
    top, res = O.run(g, "sync", max_passes=1, levels=True)
    assert len(res["levels"]) == 1 and (res["levels"][0] == top).all()


# ----------------------------------------------------------------------------------------------
# pass_tolerance = 0: a pass that does not raise modularity ends the run and is not kept


def aggregate_by_definition(g: O.Graph, C):
    """Super-vertex graph of labels C written from the definition: labels ranked ascending,
    super-arc (a, b) weighing the sum of the arcs (i, j) with ranks (a, b)."""
    labels = sorted(set(int(c) for c in C))
    rank = {c: r for r, c in enumerate(labels)}
    acc = {}
    for i, j, w in arcs_of(g):
        key = (rank[int(C[i])], rank[int(C[j])])
        acc[key] = acc.get(key, 0) + w
    n2 = len(labels)
    rows = [sorted((b, w) for (a, b), w in acc.items() if a == r) for r in range(n2)]
    off = np.zeros(n2 + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array([b for r in rows for b, _ in r], dtype=np.int32)
    w = np.array([x for r in rows for _, x in r], dtype=np.uint64)
    return [rank[int(c)] for c in C], O.Graph(n2, off, idx, w)


def phase_bruteforce(g: O.Graph, p: int, a: int = 2, b: int = 1, max_it: int = 20):
    """One fully synchronous local-moving phase of pass p from singletons, every decision by
    brute force over modularity differences; stops when S <= floor(W^2 / (2*10^(a+b*p))) or
    after max_it iterations. Returns (C, iterations)."""
    W = sum(w for _, _, w in arcs_of(g))
    T = (W * W) // (2 * 10 ** (a + b * p))
    C = np.arange(g.n, dtype=np.int32)
    for it in range(max_it):
        C, S = sync_decisions_bruteforce(g, C)
        if S <= T:
            return C, it + 1
    return C, max_it


def test_pass_that_lowers_modularity_is_dropped():
    """A 9-vertex graph on which the synchronous rule's second pass oscillates into a partition
    of lower modularity than the first level. Both phases are recomputed here by brute force
    (decisions from modularity differences, aggregation from its definition, Q from the pairwise
    definition); the run must return the first level, report the second pass's Q, and stop."""
    g = O.Graph.from_csr(erdos_renyi(9, 0.45, seed=5098, weights=(1, 5)))
    W = sum(w for _, _, w in arcs_of(g))
    q_single = q_pairwise(g, np.arange(g.n))
    C0, it0 = phase_bruteforce(g, 0)
    level1, g1 = aggregate_by_definition(g, C0)
    q1 = q_pairwise(g, C0)
    C1, it1 = phase_bruteforce(g1, 1)
    q2 = q_pairwise(g, [int(C1[level1[v]]) for v in range(g.n)])
    assert q1 > q_single and q2 <= q1  # the second pass does not raise modularity
    assert (it0, it1) == (3, 20)
    top, res = O.run(g, "sync")
    assert top.tolist() == level1
    assert Fraction(res["qnum"], W * W) == q1
    assert res["passes"] == 2 and res["iterations"] == [it0, it1]
    assert [Fraction(x, W * W) for x in res["qnum_pass"]] == [q1, q2]
    top, res = O.run(g, "sync", levels=True)
    assert res["levels"].tolist() == [level1]


def test_kept_levels_raise_modularity():
    """Q strictly increases from level to level of every run (K = 1 and K = 8 classes, and the
    asynchronous rule), the first level above the singletons; the last pass, if it reports a Q
    that is not higher than the level before it, added no level."""
    from graphgen import lattice_shortcuts, rmat
    graphs = small_graphs() + [O.Graph.from_csr(sbm(3000, 30, 8.0, 2.0, seed=2, weights=(1, 16))),
                               O.Graph.from_csr(lattice_shortcuts(2000, seed=3)),
                               O.Graph.from_csr(rmat(12, seed=7))]
    dropped = 0
    for g in graphs:
        q_single, W, _ = O.modularity(g, np.arange(g.n, dtype=np.int32))
        for mode, K in (("sync", 1), ("sync", 8), ("async", 1)):
            top, res = O.run(g, mode, substeps=K, levels=True)
            if W == 0:
                continue
            L = res["levels"]
            seq = [q_single] + [O.modularity(g, L[l])[0] for l in range(len(L))]
            assert all(seq[l + 1] > seq[l] for l in range(len(seq) - 1)), (g.n, mode, K)
            assert res["qnum"] == seq[-1]
            assert res["qnum_pass"][:len(L)] == seq[1:]
            if len(L) < res["passes"]:
                assert res["qnum_pass"][len(L)] <= seq[-1]
                dropped += res["qnum_pass"][len(L)] < seq[-1]
            if mode == "async":
                assert len(L) + 1 >= res["passes"]
    # the fully synchronous rule lowers modularity in some pass of this corpus (R-MAT s12)
    assert dropped >= 1


# ----------------------------------------------------------------------------------------------
# the run loop's hashed vertex classes (the schedule the GPU runs)


def py_vertex_class(p: int, K: int, v: int) -> int:
    from graphgen.rng import GAMMA, MASK64, mix_int
    return ((mix_int((p + (v + 1) * GAMMA) & MASK64) >> 32) * K) >> 32


def class_steps_python(g: O.Graph, p: int, K: int):
    """First iteration of pass p from singletons: K synchronous steps over classes computed here
    with Python integers. Returns (S, moved, candidate pairs)."""
    st = O.State(g)
    S = moved = nc = 0
    for k in range(K):
        vs = [v for v in range(g.n) if py_vertex_class(p, K, v) == k]
        a, b, c = O.sync_step(g, st, vs)
        S, moved, nc = S + a, moved + b, nc + c
    return S, moved, nc


def test_run_classes_are_the_hashed_classes():
    g = O.Graph.from_csr(sbm(1200, 12, 8.0, 2.0, seed=4, weights=(1, 16)))
    K = 8
    top, res = O.run(g, "sync", substeps=K, max_passes=2)
    assert res["passes"] == 2
    first = {}
    for t, p in enumerate(res["trace_pass"]):
        first.setdefault(p, t)
    t0, t1 = first[0], first[1]
    assert (res["trace_S"][t0], res["trace_moved"][t0], res["trace_ncand"][t0]) == \
        class_steps_python(g, 0, K)
    # pass 1 runs on the aggregate of pass 0's level, with the classes of pass 1
    top1, _ = O.run(g, "sync", substeps=K, max_passes=1)
    _, g1 = aggregate_by_definition(g, top1)
    S1 = class_steps_python(g1, 1, K)
    assert S1[1] > 0
    assert (res["trace_S"][t1], res["trace_moved"][t1], res["trace_ncand"][t1]) == S1


# ----------------------------------------------------------------------------------------------
# weights near 2^62 in total: every product W * k and K * Sigma exceeds 64 bits


def big_weight_graphs():
    """small_graphs() with every weight w replaced by (w << s) - (40503 w mod 2^15), s chosen so
    that W lies just below 2^62 (symmetric: the new weight is a function of the old)."""
    out = []
    for g in small_graphs():
        w = g.w.astype(object)
        W0 = int(sum(int(x) for x in w))
        s = 62 - W0.bit_length()
        nw = np.array([(int(x) << s) - ((40503 * int(x)) & 0x7FFF) for x in w], dtype=np.uint64)
        g2 = O.Graph(g.n, g.off.copy(), g.idx.copy(), nw)
        W = int(sum(int(x) for x in nw))
        K = [0] * g.n
        for i, _, x in arcs_of(g2):
            K[i] += x
        assert 2 ** 60 < W <= 2 ** 62 and W * max(K) >= 2 ** 64
        out.append(g2)
    return out


def test_big_weights_modularity_and_single_moves():
    for gi, g in enumerate(big_weight_graphs()):
        C = random_partition(g.n, 3, 900 + gi)
        qnum, W, _ = O.modularity(g, C)
        assert Fraction(qnum, W * W) == q_pairwise(g, C)
        st = O.State(g, C)
        q0 = q_pairwise(g, C)
        for i in range(g.n):
            gains, stay = O.vertex_gains(g, st, i)
            for c, gval in gains.items():
                C2 = C.copy()
                C2[i] = c
                assert q_pairwise(g, C2) - q0 == Fraction(2 * (gval - stay), W * W), (gi, i, c)


def test_big_weights_sync_async_aggregation():
    for gi, g in enumerate(big_weight_graphs()):
        for C in (np.arange(g.n, dtype=np.int32), random_partition(g.n, 4, 950 + gi)):
            st = O.State(g, C)
            S, moved, _ = O.sync_iteration(g, st)
            Cn, Sb = sync_decisions_bruteforce(g, C)
            assert np.array_equal(st.C, Cn) and S == Sb, gi
        st = O.State(g)
        q_prev, _, _ = O.modularity(g, st.C)
        for _ in range(4):
            S, _ = O.async_iteration(g, st)
            q, _, _ = O.modularity(g, st.C)
            assert q - q_prev == 2 * S
            q_prev = q
        check_aggregation(g, random_partition(g.n, 3, 970 + gi))
    for g in big_weight_graphs()[:4]:
        qo = q_opt_bruteforce(g)
        for mode in ("sync", "async"):
            top, res = O.run(g, mode)
            assert Fraction(res["qnum"], res["W"] ** 2) <= qo
            assert O.modularity(g, top)[0] == res["qnum"]
