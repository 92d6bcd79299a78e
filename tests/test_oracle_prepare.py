"""Pins of the oracle's graph preparation (section 3.1.2 and Table 1: edges made undirected by
their reverse, unit weights, a self-loop on every vertex) against facts from outside it:

* the hand-derived example ``tests/golden/prepare_small.json``;
* networkx's simple undirected graph of the same edge list (neighbour sets, edge count);
* a dense adjacency matrix accumulated entry by entry;
* invariants: weight conservation (sum), symmetry, strictly ascending rows, one loop per vertex;
* the per-row routine ``prepare_row`` (a second, numpy route) on every row.
"""

import json
import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
FLAG_SETS = [0, O.PREP_SYM, O.PREP_SYM | O.PREP_LOOPS, O.PREP_SYM | O.PREP_LOOPS | O.PREP_MAX,
             O.PREP_LOOPS | O.PREP_MAX, O.PREP_MAX]


def random_edges(n, m, seed, wmax=1, loops=True):
    rng = np.random.default_rng(seed)
    # a skewed endpoint distribution gives many repeated edges
    src = (n * rng.random(m) ** 2).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    if not loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    w = rng.integers(1, wmax + 1, src.size).astype(np.uint32) if wmax > 1 else None
    return src, dst, w


def dense(n, src, dst, w, flags):
    """Adjacency matrix built entry by entry from the edge list."""
    A = np.zeros((n, n), dtype=np.uint64)
    seen = np.zeros((n, n), dtype=bool)

    def put(u, v, x):
        if flags & O.PREP_MAX:
            A[u, v] = max(A[u, v], x) if seen[u, v] else x
        else:
            A[u, v] += x
        seen[u, v] = True

    for e in range(src.size):
        x = 1 if w is None else int(w[e])
        put(src[e], dst[e], x)
        if flags & O.PREP_SYM and src[e] != dst[e]:
            put(dst[e], src[e], x)
    if flags & O.PREP_LOOPS:
        for v in range(n):
            put(v, v, 1)
    return A, seen


def test_golden_small():
    d = json.load(open(os.path.join(GOLDEN, "prepare_small.json")))
    for c in d["cases"]:
        off, idx, w = O.prepare(d["n"], np.array(d["src"]), np.array(d["dst"]), flags=c["flags"])
        assert off.tolist() == c["off"] and idx.tolist() == c["idx"] and w.tolist() == c["w"]


def test_matches_networkx_simple_graph():
    nx = pytest.importorskip("networkx")
    for seed in range(4):
        n = 60
        src, dst, _ = random_edges(n, 400, seed)
        G = nx.Graph()
        G.add_nodes_from(range(n))
        G.add_edges_from(zip(src.tolist(), dst.tolist()))
        off, idx, w = O.prepare(n, src, dst, flags=O.PREP_SYM | O.PREP_MAX)
        loops = nx.number_of_selfloops(G)
        assert idx.size == 2 * (G.number_of_edges() - loops) + loops
        assert (w == 1).all()
        for v in range(n):
            assert set(idx[off[v]:off[v + 1]].tolist()) == set(G.neighbors(v))


@pytest.mark.parametrize("flags", FLAG_SETS)
def test_matches_dense_definition(flags):
    for seed, wmax in [(1, 1), (2, 9), (3, 1000)]:
        n = 40
        src, dst, w = random_edges(n, 300, seed, wmax)
        A, seen = dense(n, src, dst, w, flags)
        off, idx, wo = O.prepare(n, src, dst, w, flags)
        for v in range(n):
            row = idx[off[v]:off[v + 1]]
            assert row.tolist() == np.nonzero(seen[v])[0].tolist()
            assert wo[off[v]:off[v + 1]].tolist() == A[v, row].tolist()


@pytest.mark.parametrize("flags", FLAG_SETS)
def test_invariants_and_rows(flags):
    n = 500
    src, dst, w = random_edges(n, 5000, 7, wmax=50)
    off, idx, wo = O.prepare(n, src, dst, w, flags)
    assert off[0] == 0 and off[-1] == idx.size and (np.diff(off) >= 0).all()
    rows = np.repeat(np.arange(n), np.diff(off))
    # strictly ascending neighbours within each row
    same = rows[1:] == rows[:-1]
    assert (idx[1:][same] > idx[:-1][same]).all()
    if not flags & O.PREP_MAX:
        wsum = int(w.astype(np.uint64).sum())
        if flags & O.PREP_SYM:
            wsum += int(w[src != dst].astype(np.uint64).sum())
        if flags & O.PREP_LOOPS:
            wsum += n
        assert int(wo.sum()) == wsum
    if flags & O.PREP_SYM:
        fwd = {(int(a), int(b)): int(x) for a, b, x in zip(rows, idx, wo)}
        assert all(fwd[(b, a)] == x for (a, b), x in fwd.items())
    if flags & O.PREP_LOOPS:
        assert all((rows == v).any() and v in idx[off[v]:off[v + 1]] for v in range(0, n, 37))
    for r in range(n):
        ri, rw = O.prepare_row(n, src, dst, w, flags, r)
        assert ri.tolist() == idx[off[r]:off[r + 1]].tolist()
        assert rw.tolist() == wo[off[r]:off[r + 1]].tolist()


def test_edge_cases_and_errors():
    # no edges: only the added loops
    off, idx, w = O.prepare(3, np.zeros(0), np.zeros(0))
    assert off.tolist() == [0, 1, 2, 3] and idx.tolist() == [0, 1, 2] and w.tolist() == [1, 1, 1]
    off, idx, w = O.prepare(3, np.zeros(0), np.zeros(0), flags=O.PREP_SYM)
    assert off.tolist() == [0, 0, 0, 0] and idx.size == 0
    off, idx, w = O.prepare(0, np.zeros(0), np.zeros(0))
    assert off.tolist() == [0] and idx.size == 0
    with pytest.raises(ValueError):
        O.prepare(3, np.array([0]), np.array([3]))
    with pytest.raises(ValueError):
        O.prepare(3, np.array([-1]), np.array([0]))
    with pytest.raises(ValueError):
        O.prepare(3, np.array([0]), np.array([1]), np.array([0], dtype=np.uint32))
