"""The live numbering of a run, checked against the oracle's aggregation on the CPU.

From the first aggregation on, louvain_run gives new ids only to communities with arcs, in
label order, and recovers the method's ids (new id = rank of every used label, section 3.2's
renumbering) from two arrays: rep[x], the input vertex whose line of labels names super-vertex
x, and noarc_before[y], the number of input vertices without arcs below y. This test applies
those formulas to random memberships over several levels and compares them with what the
oracle's canonical aggregation gives: the membership of every input vertex, the vertex count
of every level, and the method's id of every super-vertex (which the class hash reads).
"""

import numpy as np
import torch

import oracle as O
from graphgen import csr_from_arcs, erdos_renyi


def spread_graph(factor, seed):
    # an Erdos-Renyi graph whose vertex v becomes factor * v + 1: all other ids have no arcs
    base = erdos_renyi(300, 0.02, seed=seed, weights=(1, 5))
    off = base.offsets.numpy().astype(np.int64)
    src = np.repeat(np.arange(base.n), np.diff(off)) * factor + 1
    dst = base.indices.numpy().astype(np.int64) * factor + 1
    n = base.n * factor + 2
    return csr_from_arcs(n, torch.from_numpy(src), torch.from_numpy(dst), base.weights)


def check(factor, seed, levels=4):
    g = spread_graph(factor, seed)
    og = O.Graph.from_csr(g)
    n0 = g.n
    noarc = np.diff(g.offsets.numpy()) == 0
    noarc_before = np.concatenate([[0], np.cumsum(noarc)])
    rng = np.random.default_rng(seed)
    canon_top = np.arange(n0)     # the method's membership of the input vertices
    live_top = np.arange(n0)      # the live membership (-1: no arcs)
    rep = None                    # level 0: the input itself
    gcan, nlive = og, n0
    live_canon = np.arange(n0)    # method's id of every working vertex
    for level in range(levels):
        has = ~noarc if level == 0 else np.ones(nlive, bool)
        cand = np.flatnonzero(has)
        if len(cand) == 0:
            break
        # a random membership of the working vertices with arcs (labels among them)
        C = np.arange(nlive)
        pick = rng.choice(cand, size=max(1, len(cand) // 4), replace=False)
        C[cand] = rng.choice(pick, size=len(cand))
        # the same membership in the method's numbering (vertices without arcs alone)
        Ccan = np.arange(gcan.n)
        Ccan[live_canon[cand]] = live_canon[C[cand]]
        mo, gnext = O.aggregate(gcan, Ccan.astype(np.int32))
        canon_top = mo[canon_top]
        # the live path: new ids by rank of the labels of vertices with arcs
        labels = np.unique(C[cand])
        newid = -np.ones(nlive, np.int64)
        newid[labels] = np.arange(len(labels))
        live_top = np.where(live_top >= 0, newid[C[np.maximum(live_top, 0)]], -1)
        rep = labels if rep is None else rep[labels]
        nlive = len(labels)
        live_canon = np.arange(nlive) + noarc_before[rep]
        # the formulas of k_canon_membership
        live_below = np.concatenate([[0], np.cumsum(np.bincount(rep, minlength=n0) > 0)])
        got = np.where(live_top >= 0, live_top + noarc_before[rep[np.maximum(live_top, 0)]],
                       live_below[np.arange(n0)] + noarc_before[np.arange(n0)])
        assert np.array_equal(got, canon_top), (factor, seed, level)
        assert gnext.n == nlive + int(noarc.sum()), (factor, seed, level)
        # every working vertex's method id is the id the canonical graph gives its members
        for x in range(0, nlive, max(1, nlive // 64)):
            members = np.flatnonzero(live_top == x)
            assert np.all(canon_top[members] == live_canon[x])
        gcan = gnext


def test_live_numbering_matches_canonical_renumbering():
    for factor in (1, 3, 20):
        for seed in (1, 2):
            check(factor, seed)
