"""Pins of the oracle's partition and merge (section 3.2 and the conclusion propose running
partitions of the graph independently and combining them; no procedure is given):

* the hand-derived two triangles split into their triangles;
* the whole procedure composed here from pinned primitives (runs on induced subgraphs built
  independently with numpy, labels offset part by part, aggregation, a run, composition),
  including parts that are whole connected components (no final community spans two);
* the final Q by the pairwise definition; nesting of the part communities in the final ones,
  with the part runs recomputed here on induced subgraphs built independently (numpy);
* P = 1: the run on the whole graph, then a run on its aggregate;
* balanced parts by arcs.
"""

from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from graphgen import erdos_renyi, ring_of_cliques, sbm, two_triangles

from .test_oracle_pins import q_pairwise


def induced(g: O.Graph, v0: int, v1: int) -> O.Graph:
    """Subgraph on [v0, v1) with local ids (numpy, independent of the oracle's C)."""
    off, idx, w = [0], [], []
    for v in range(v0, v1):
        row = g.idx[g.off[v]:g.off[v + 1]]
        wr = g.w[g.off[v]:g.off[v + 1]]
        keep = (row >= v0) & (row < v1)
        idx.extend((row[keep] - v0).tolist())
        w.extend(wr[keep].tolist())
        off.append(len(idx))
    return O.Graph(v1 - v0, np.array(off, dtype=np.int64), np.array(idx, dtype=np.int32),
                   np.array(w, dtype=np.uint64))


def test_two_triangles_hand_derived():
    """Parts {0,1,2} and {3,4,5}: each part is a triangle, which one pass gathers into one
    community (part Q = 0). The merge runs on two super-vertices with self-loops of weight 6 and
    one arc of weight 1 each way (K = 7, W = 14): joining gains 14*1 - 7*7 < 0, so nothing
    moves, and the result is the two triangles, Q = 5/14 (W^2 Q = 70)."""
    g = O.Graph.from_csr(two_triangles())
    top, res, parts = O.run_partitioned(g, [0, 3, 6])
    assert top.tolist() == [0, 0, 0, 1, 1, 1]
    assert res["qnum"] == 70 and res["W"] == 14
    assert [p["n_communities"] for p in parts] == [1, 1]
    assert [p["qnum"] for p in parts] == [0, 0]


def components_graph():
    """Four disjoint graphs placed one after another (no arc between them)."""
    gs = [ring_of_cliques(5, 4), erdos_renyi(40, 0.15, seed=3, weights=(1, 5)),
          sbm(300, 6, 6.0, 1.0, seed=2), ring_of_cliques(7, 3)]
    src, dst, w, base = [], [], [], 0
    for h in gs:
        og = O.Graph.from_csr(h)
        for v in range(og.n):
            for e in range(og.off[v], og.off[v + 1]):
                src.append(v + base)
                dst.append(int(og.idx[e]) + base)
                w.append(int(og.w[e]))
        base += og.n
    n = base
    order = np.lexsort((dst, src))
    src, dst, w = np.array(src)[order], np.array(dst)[order], np.array(w)[order]
    off = np.zeros(n + 1, dtype=np.int64)
    np.add.at(off, src + 1, 1)
    off = np.cumsum(off)
    sizes = [O.Graph.from_csr(h).n for h in gs]
    return O.Graph(n, off, dst.astype(np.int32), w.astype(np.uint64)), sizes


def composed(g, vptr, K):
    """Partition and merge composed here from the pinned primitives: runs on induced subgraphs
    built independently, labels offset part after part, aggregate, run, compose."""
    labels, offset, part = [], 0, []
    for k in range(len(vptr) - 1):
        t, r = O.run(induced(g, vptr[k], vptr[k + 1]), "sync", substeps=K)
        labels.extend((t + offset).tolist())
        offset += r["n_communities"]
        part.append(r)
    mp, agg = O.aggregate(g, np.array(labels, dtype=np.int32))
    t2, r2 = O.run(agg, "sync", substeps=K)
    return t2[mp], r2, part


@pytest.mark.parametrize("K", [1, 8])
def test_components_as_parts(K):
    g, sizes = components_graph()
    vptr = np.concatenate([[0], np.cumsum(sizes)]).tolist()
    top, res, parts = O.run_partitioned(g, vptr, substeps=K)
    expect, r2, part = composed(g, vptr, K)
    assert [p["n_communities"] for p in parts] == [r["n_communities"] for r in part]
    assert [p["qnum"] for p in parts] == [r["qnum"] for r in part]
    assert top.tolist() == expect.tolist() and res["qnum"] == r2["qnum"]
    # no community spans two components
    for k in range(len(sizes)):
        inside = set(top[vptr[k]:vptr[k + 1]].tolist())
        outside = set(top[:vptr[k]].tolist()) | set(top[vptr[k + 1]:].tolist())
        assert not inside & outside


@pytest.mark.parametrize("P", [2, 4, 9])
def test_matches_composition(P):
    g = O.Graph.from_csr(sbm(3000, 30, 8.0, 2.0, seed=7, weights=(1, 16)))
    vptr = O.balanced_parts(g, P)
    top, res, _ = O.run_partitioned(g, vptr, substeps=8)
    expect, r2, _ = composed(g, vptr, 8)
    assert top.tolist() == expect.tolist() and res["qnum"] == r2["qnum"]


@pytest.mark.parametrize("P", [2, 3, 5])
def test_q_and_nesting(P):
    for s in range(3):
        g = O.Graph.from_csr(erdos_renyi(90, 0.06, seed=s, weights=(1, 9)))
        vptr = O.balanced_parts(g, P)
        top, res, parts = O.run_partitioned(g, vptr, substeps=4)
        assert q_pairwise(g, top) == Fraction(res["qnum"], res["W"] ** 2)
        for k in range(P):
            t, r = O.run(induced(g, vptr[k], vptr[k + 1]), "sync", substeps=4)
            assert parts[k]["qnum"] == r["qnum"]
            # each part community lies inside one final community
            seg = top[vptr[k]:vptr[k + 1]]
            for c in set(t.tolist()):
                assert len(set(seg[t == c].tolist())) == 1


def test_single_part_is_run_then_run_on_aggregate():
    g = O.Graph.from_csr(sbm(2000, 20, 8.0, 2.0, seed=5, weights=(1, 16)))
    top, res, _ = O.run_partitioned(g, [0, g.n], substeps=8)
    t1, r1 = O.run(g, "sync", substeps=8)
    mp, agg = O.aggregate(g, t1)
    t2, r2 = O.run(agg, "sync", substeps=8)
    assert top.tolist() == t2[mp].tolist()
    assert res["qnum"] == r2["qnum"]


def test_balanced_parts():
    g = O.Graph.from_csr(sbm(5000, 50, 8.0, 2.0, seed=1))
    for P in (1, 2, 7, 64):
        vptr = O.balanced_parts(g, P)
        assert vptr[0] == 0 and vptr[-1] == g.n and len(vptr) == P + 1
        assert all(vptr[k] <= vptr[k + 1] for k in range(P))
        nnz = int(g.off[-1])
        for k in range(1, P):
            v = vptr[k]
            assert g.off[v] >= (k * nnz) // P and (v == 0 or g.off[v - 1] < (k * nnz) // P)
