"""Pins of the oracle's colour classes (the colouring route to partial asynchrony that section
3.2 cites) against facts from outside it:

* the priority is the SplitMix64 draw, recomputed with Python integers;
* networkx's greedy colouring with the same vertex order (first-fit, no cap);
* a Jones-Plassmann simulation in rounds (a vertex is coloured once every higher-priority
  neighbour is), written here independently, equals the sequential definition;
* so does the shortcut the GPU's rounds take (a vertex is also coloured, with the leftover
  class, once its coloured higher-priority neighbours hold all of 0..K-2), in fewer rounds;
* invariants: classes 0..K-2 are independent sets, first-fit (every smaller colour is held by a
  higher-priority neighbour), the leftover class only when all K-1 colours are taken.
"""

import numpy as np
import pytest

import oracle as O
from graphgen import erdos_renyi, ring_of_cliques, rmat, sbm, add_self_loops
from graphgen.rng import GAMMA, MASK64, mix_int


def prio(p, v):
    return mix_int((p + (v + 1) * GAMMA) & MASK64)


def neighbours(g, v):
    return [int(u) for u in g.idx[g.off[v]:g.off[v + 1]] if u != v]


def graphs():
    out = [O.Graph.from_csr(erdos_renyi(60, 0.1, seed=s, weights=(1, 5))) for s in range(3)]
    out.append(O.Graph.from_csr(add_self_loops(erdos_renyi(40, 0.2, seed=9))))
    out.append(O.Graph.from_csr(ring_of_cliques(6, 5)))
    out.append(O.Graph.from_csr(rmat(9, seed=4)))
    return out


def test_priority_is_splitmix64():
    for p in (0, 1, 5):
        for v in list(range(20)) + [99999, 2**31 - 1]:
            assert O.vertex_priority(p, v) == prio(p, v)


def jp_rounds(g, p, K):
    """Jones-Plassmann in rounds: each round colours every uncoloured vertex whose uncoloured
    neighbours all have lower priority, first-fit over the colours of its coloured neighbours
    (capped: colours 0..K-2, else K-1)."""
    n = g.n
    key = [(prio(p, v), -v) for v in range(n)]
    col = [-1] * n
    rounds = 0
    while any(c < 0 for c in col):
        ready = [v for v in range(n) if col[v] < 0 and
                 all(col[u] >= 0 or key[u] < key[v] for u in neighbours(g, v))]
        assert ready, "the priority order has no cycle"
        for v in ready:
            used = {col[u] for u in neighbours(g, v) if col[u] >= 0}
            col[v] = next((c for c in range(K - 1) if c not in used), K - 1)
        rounds += 1
    return np.array(col, dtype=np.int32), rounds


def jp_rounds_shortcut(g, p, K):
    """Rounds with the shortcut: a vertex is ready when its higher-priority neighbours are all
    coloured, or when those coloured so far hold all of 0..K-2; a ready vertex takes the first
    fit over its coloured higher-priority neighbours' colours (capped as above)."""
    n = g.n
    key = [(prio(p, v), -v) for v in range(n)]
    higher = [[u for u in neighbours(g, v) if key[u] > key[v]] for v in range(n)]
    col = [-1] * n
    rounds = 0
    while any(c < 0 for c in col):
        ready = []
        for v in range(n):
            if col[v] >= 0:
                continue
            held = {col[u] for u in higher[v] if col[u] >= 0}
            if all(col[u] >= 0 for u in higher[v]) or set(range(K - 1)) <= held:
                ready.append((v, held))
        assert ready, "the priority order has no cycle"
        for v, held in ready:
            col[v] = next((c for c in range(K - 1) if c not in held), K - 1)
        rounds += 1
    return np.array(col, dtype=np.int32), rounds


@pytest.mark.parametrize("K", [2, 4, 8, 32])
def test_shortcut_rounds_equal_sequential_first_fit(K):
    fewer = 0
    for gi, g in enumerate(graphs()):
        for p in (0, 3):
            got, r_short = jp_rounds_shortcut(g, p, K)
            assert np.array_equal(O.colour_classes(g, p, K), got), (gi, p, K)
            _, r_plain = jp_rounds(g, p, K)
            assert r_short <= r_plain
            fewer += r_short < r_plain
    if K <= 8:
        assert fewer > 0  # the shortcut fires on these graphs


@pytest.mark.parametrize("K", [2, 4, 8, 32])
def test_matches_jones_plassmann_rounds(K):
    for gi, g in enumerate(graphs()):
        for p in (0, 3):
            expect, _ = jp_rounds(g, p, K)
            assert np.array_equal(O.colour_classes(g, p, K), expect), (gi, p, K)


def test_matches_networkx_greedy_in_priority_order():
    nx = pytest.importorskip("networkx")
    for g in graphs():
        G = nx.Graph()
        G.add_nodes_from(range(g.n))
        for v in range(g.n):
            for u in neighbours(g, v):
                G.add_edge(v, u)
        order = sorted(range(g.n), key=lambda v: (-prio(0, v), v))
        ref = nx.coloring.greedy_color(G, strategy=lambda G_, colors: iter(order))
        assert max(ref.values(), default=0) < 31  # the cap does not bind
        got = O.colour_classes(g, 0, 32)
        assert all(got[v] == ref[v] for v in range(g.n))


@pytest.mark.parametrize("K", [3, 8, 32])
def test_colour_invariants(K):
    for g in graphs() + [O.Graph.from_csr(sbm(2000, 20, 8.0, 2.0, seed=3))]:
        for p in (0, 1):
            c = O.colour_classes(g, p, K)
            assert c.min() >= 0 and c.max() <= K - 1
            for v in range(g.n):
                nb = neighbours(g, v)
                higher = {int(c[u]) for u in nb if prio(p, u) > prio(p, v)}
                if c[v] < K - 1:
                    # an independent set, first fit
                    assert all(c[u] != c[v] for u in nb)
                    assert all(k in higher for k in range(c[v]))
                else:
                    assert all(k in higher for k in range(K - 1))


def test_k1_and_empty():
    g = graphs()[0]
    assert (O.colour_classes(g, 0, 1) == 0).all()
    e = O.Graph(0, np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32),
                np.zeros(0, dtype=np.uint64))
    assert O.colour_classes(e, 0, 8).size == 0


def test_colour_run_classes_are_the_colouring():
    """A colour-class run's first iteration is the sequence of synchronous steps over the colour
    classes of pass 0 (checked step by step with the oracle's step routine)."""
    g = O.Graph.from_csr(sbm(3000, 30, 8.0, 2.0, seed=2, weights=(1, 16)))
    K = 8
    _, res = O.run(g, "sync", substeps=K, colour=True, max_iterations=1, max_passes=1)
    c = O.colour_classes(g, 0, K)
    st = O.State(g)
    S = 0
    for k in range(K):
        verts = np.nonzero(c == k)[0].astype(np.int32)
        S += O.sync_step(g, st, verts)[0]
    assert res["trace_S"][0] == S
