"""Batched runs (louvain_run_batched) against the oracle run on every graph alone.

A batch is the packed union of independent graphs; every graph must come out exactly as a
single run on it: membership (local ids), exact Qnum, passes, iterations per pass, cap hits and
community count. Covers empty and arc-less graphs, self-loops and duplicate arcs, hubs on the
two-phase path, both gain widths, the small-partition testing mode, K = 1 and K = 8 vertex
classes, and the batch validation errors.
"""

import numpy as np
import pytest
import torch

import oracle as O
from graphgen import (add_self_loops, csr_from_arcs, erdos_renyi, lattice_shortcuts, pack_graphs,
                      planted_hubs, rmat, ring_of_cliques, sbm, single_edge, two_triangles)
from graphgen.csr import Csr

pytestmark = pytest.mark.gpu

LV_VALIDATE = 0x1
LV_FORCE_WIDE = 0x4
LV_SMALL_PARTS = 0x8
LV_GRAPH_REPLAY = 0x20


@pytest.fixture(scope="module")
def lv(gpu_device):
    from paper_2301_12390_amd import Louvain
    ctx = Louvain(0)
    yield ctx
    ctx.close()


def empty_graph(n):
    return Csr(n, torch.zeros(n + 1, dtype=torch.int32), torch.zeros(0, dtype=torch.int32),
               torch.zeros(0, dtype=torch.int32), name=f"empty{n}")


def dup_arcs_graph():
    src = torch.tensor([0, 0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 4, 4, 4])
    dst = torch.tensor([1, 1, 2, 0, 0, 1, 0, 2, 3, 2, 4, 3, 4, 4])
    w = torch.tensor([2, 3, 1, 3, 2, 7, 1, 5, 4, 4, 2, 2, 1, 1])
    return csr_from_arcs(5, src, dst, w, name="dup-arcs")


def mixed_batch():
    return [
        two_triangles(),
        empty_graph(0),
        single_edge(),
        empty_graph(7),
        ring_of_cliques(8, 5),
        dup_arcs_graph(),
        add_self_loops(erdos_renyi(300, 0.03, seed=4, weights=(1, 9))),
        sbm(3000, 30, 8.0, 2.0, seed=2, weights=(1, 16)),
        lattice_shortcuts(2000, seed=3),
        rmat(12, seed=7),
        ring_of_cliques(30, 5),
        rmat(13, seed=9, weights=(1, 16)),
    ]


BATCH = mixed_batch()


def check_batch(lv, graphs, flags=0, substeps=8, **kw):
    packed, vptr, aptr = pack_graphs(graphs)
    memb, res = lv.run_batched(packed.to("cuda:0"), vptr, aptr, flags=flags, substeps=substeps,
                               **kw)
    torch.cuda.synchronize()
    memb = memb.cpu().numpy()
    okw = {{"tolerance_exp10": "a", "decline_exp10": "b"}.get(k, k): v for k, v in kw.items()}
    for g, (gr, r) in enumerate(zip(graphs, res)):
        mine = memb[vptr[g]:vptr[g + 1]]
        if gr.nnz == 0:
            assert np.array_equal(mine, np.arange(gr.n)), g
            assert r["passes"] == 0 and r["qnum"] == 0 and r["q"] == 0.0
            assert r["n_communities"] == gr.n
            continue
        top, ref = O.run(O.Graph.from_csr(gr), "sync", substeps=substeps, **okw)
        assert np.array_equal(mine, top), (g, gr.name)
        assert r["qnum"] == ref["qnum"] and r["W"] == ref["W"], (g, gr.name)
        assert r["passes"] == ref["passes"], (g, gr.name, r["passes"], ref["passes"])
        assert r["iterations"] == ref["iterations"], (g, gr.name)
        assert r["cap_hits"] == ref["cap_hits"], (g, gr.name)
        assert r["n_communities"] == ref["n_communities"], (g, gr.name)
    return res


@pytest.mark.parametrize("K", [1, 8])
@pytest.mark.parametrize("flags", [0, LV_FORCE_WIDE, LV_SMALL_PARTS, LV_GRAPH_REPLAY])
def test_batch_matches_single_runs(lv, flags, K):
    check_batch(lv, BATCH, flags=flags, substeps=K)


def test_batch_parameters(lv):
    check_batch(lv, BATCH[4:10], tolerance_exp10=0)
    check_batch(lv, BATCH[4:10], max_iterations=1, max_passes=2)
    check_batch(lv, BATCH[4:10], max_passes=1)


def test_batch_with_hubs(lv):
    hubs = planted_hubs(sbm(40000, 400, 8.0, 2.0, seed=4, weights=(1, 16)),
                        [100000, 33000, 17000], seed=2, weights=(1, 16))
    check_batch(lv, [rmat(12, seed=7), hubs, two_triangles(), sbm(3000, 30, 8.0, 2.0, seed=2)])
    check_batch(lv, [hubs, single_edge()], flags=LV_SMALL_PARTS)


def test_batch_of_one_equals_run(lv):
    g = sbm(4000, 40, 8.0, 2.0, seed=9, weights=(1, 16))
    packed, vptr, aptr = pack_graphs([g])
    m1, r1 = lv.run_batched(packed.to("cuda:0"), vptr, aptr)
    m2, r2 = lv.run(g.to("cuda:0"))
    assert torch.equal(m1, m2)
    assert r1[0]["qnum"] == r2["qnum"] and r1[0]["iterations"] == r2["iterations"]


def test_many_small_graphs(lv):
    gs = []
    for i in range(64):
        n = int(np.exp(np.random.default_rng(i).uniform(np.log(50), np.log(3000))))
        gs.append(sbm(n, max(1, round(n / 100)), 8.0, 2.0, seed=i + 1, weights=(1, 16))
                  if i % 2 == 0 else lattice_shortcuts(n, seed=i + 1))
    check_batch(lv, gs)


def test_batch_validation(lv):
    from paper_2301_12390_amd import LouvainError
    packed, vptr, aptr = pack_graphs([two_triangles(), two_triangles()])
    dev = packed.to("cuda:0")
    with pytest.raises(LouvainError):  # bounds that do not cover the graph
        lv.run_batched(dev, [0, 6, 11], aptr)
    with pytest.raises(LouvainError):  # decreasing bounds
        lv.run_batched(dev, [0, 7, 6, 12], [0, 14, 13, 28])
    with pytest.raises(LouvainError):  # arc bounds that do not match the offsets
        lv.run_batched(dev, vptr, [0, 13, 28], flags=LV_VALIDATE)
    # an arc joining the two graphs
    idx = packed.indices.clone()
    idx[0] = 7
    bad = Csr(packed.n, packed.offsets, idx, packed.weights).to("cuda:0")
    with pytest.raises(LouvainError):
        lv.run_batched(bad, vptr, aptr, flags=LV_VALIDATE)
    # the valid batch still runs on the same context
    m, r = lv.run_batched(dev, vptr, aptr, flags=LV_VALIDATE)
    assert r[0]["qnum"] == r[1]["qnum"]


def test_batch_with_dropped_passes(lv):
    """Fully synchronous runs in which a pass ends below the level before it (that pass is
    dropped: pass 0 of R-MAT s12, pass 1 of the ring of 16 K4, pass 2 of SBM-10k) beside graphs
    whose passes all raise Q: every graph equals its single run, so each dropped graph keeps its
    own earlier level while the others go on."""
    from graphgen import config_graph
    graphs = [ring_of_cliques(16, 4), rmat(12, seed=7), two_triangles(), config_graph("sbm10k"),
              ring_of_cliques(64, 3)]
    dropped = 0
    for g in graphs:
        _, ref = O.run(O.Graph.from_csr(g), "sync", substeps=1, levels=True)
        kept = len(ref["levels"])
        dropped += kept < ref["passes"] and ref["qnum_pass"][kept] < ref["qnum"]
    assert dropped == 3
    check_batch(lv, graphs, substeps=1)
    check_batch(lv, graphs[::-1], substeps=1, flags=LV_SMALL_PARTS)
