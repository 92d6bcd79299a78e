"""GPU parity of the dendrogram (louvain_run_levels) against the oracle's per-level membership.

Every level, the level count, the final membership and the run's exact results must equal the
oracle's run with the same rule and parameters; louvain_run_levels must also agree with
louvain_run on the same input.
"""

import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from graphgen import ring_of_cliques, sbm
from graphgen.csr import Csr

from .test_gpu_parity import CORPUS, HUB_IDS, HUBS, IDS, LV_FORCE_WIDE, LV_SMALL_PARTS

pytestmark = pytest.mark.gpu

LV_COLOR_CLASSES = 0x10


@pytest.fixture(scope="module")
def lv(gpu_device):
    from paper_2301_12390_amd import Louvain, build as B
    if not __import__("os").path.exists(B.LIB):
        B.build()
    ctx = Louvain(0)
    yield ctx
    ctx.close()


def check_levels(lv, g, flags=0, substeps=8, **kw):
    og = O.Graph.from_csr(g)
    okw = {{"tolerance_exp10": "a", "decline_exp10": "b"}.get(k, k): v for k, v in kw.items()}
    if flags & LV_COLOR_CLASSES:
        okw["colour"] = True
    top, ref = O.run(og, "sync", substeps=substeps, levels=True, **okw)
    dg = g.to("cuda:0")
    memb, levels, res = lv.run_levels(dg, flags=flags, substeps=substeps, **kw)
    memb1, res1 = lv.run(dg, flags=flags, substeps=substeps, **kw)
    torch.cuda.synchronize()
    L = levels.cpu().numpy()
    assert L.shape == ref["levels"].shape, (g.name, L.shape, ref["levels"].shape)
    for l in range(L.shape[0]):
        assert np.array_equal(L[l], ref["levels"][l]), (g.name, l)
    assert np.array_equal(memb.cpu().numpy(), top)
    assert np.array_equal(memb1.cpu().numpy(), top)
    for key in ("qnum", "W", "passes", "iterations", "qnum_pass", "n_pass", "nnz_pass"):
        assert res[key] == ref[key], key
        assert res1[key] == res[key], key
    return L, res


@pytest.mark.parametrize("K", [1, 8])
@pytest.mark.parametrize("g", CORPUS, ids=IDS)
def test_levels(lv, g, K):
    check_levels(lv, g, substeps=K)


@pytest.mark.parametrize("flags", [0, LV_SMALL_PARTS | LV_FORCE_WIDE])
@pytest.mark.parametrize("gi", [0, 1], ids=HUB_IDS)
def test_levels_hub_graphs(lv, gi, flags):
    check_levels(lv, HUBS[gi], flags=flags)


def test_levels_deep_hierarchy(lv):
    # rings of small cliques aggregate several times (3 to 8 levels)
    for g in [ring_of_cliques(64, 3), ring_of_cliques(200, 3), ring_of_cliques(16, 4)]:
        for K in (1, 8):
            L, res = check_levels(lv, g, substeps=K)
            if g.name == "ring16xK4" and K == 1:
                # the fully synchronous second pass oscillates for 20 iterations and ends below
                # the first level: it is dropped, so the hierarchy keeps one level
                assert L.shape[0] == 1 and res["passes"] == 2
                assert res["qnum_pass"][1] < res["qnum_pass"][0] == res["qnum"]
            else:
                assert L.shape[0] >= 2


def test_levels_capped_by_max_passes(lv):
    g = sbm(3000, 30, 8.0, 2.0, seed=2, weights=(1, 16))
    for mp in (1, 2):
        L, res = check_levels(lv, g, max_passes=mp)
        assert L.shape[0] <= mp


def test_levels_parameters(lv):
    g = sbm(4000, 40, 8.0, 2.0, seed=9, weights=(1, 16))
    for kw in [dict(tolerance_exp10=0), dict(tolerance_exp10=6, decline_exp10=2)]:
        check_levels(lv, g, **kw)


def spread(g, factor, offset, name):
    # g's vertex v becomes factor * v + offset in a graph of factor * n + offset + 1 vertices:
    # every other id (id 0 and the last one among them when offset > 0) has no arcs
    from graphgen import csr_from_arcs
    off = g.offsets.cpu().numpy().astype(np.int64)
    src = np.repeat(np.arange(g.n), np.diff(off)) * factor + offset
    dst = g.indices.cpu().numpy().astype(np.int64) * factor + offset
    n = g.n * factor + offset + 1
    return csr_from_arcs(n, torch.from_numpy(src), torch.from_numpy(dst), g.weights.cpu(),
                         name=name)



@pytest.mark.parametrize("flags,K", [(0, 1), (0, 8), (LV_COLOR_CLASSES, 8)],
                         ids=["K1", "K8", "colour"])
def test_levels_vertices_without_arcs(lv, flags, K):
    # vertices without arcs leave the working graph after the first aggregation; every level,
    # the per-pass vertex counts and the final membership stay those of the method's numbering
    cases = [
        spread(ring_of_cliques(30, 5), 3, 1, "cliques-x3"),
        spread(sbm(2000, 20, 8.0, 2.0, seed=7, weights=(1, 9)), 20, 7, "sbm-x20"),
        spread(ring_of_cliques(8, 5), 1, 3, "cliques-head3"),
    ]
    for g in cases:
        L, res = check_levels(lv, g, flags=flags, substeps=K)
        assert L.shape[0] >= 1, g.name


def test_levels_empty_and_edgeless(lv):
    dev = "cuda:0"
    for n in (0, 5):
        g = Csr(n, torch.zeros(n + 1, dtype=torch.int32, device=dev),
                torch.zeros(0, dtype=torch.int32, device=dev),
                torch.zeros(0, dtype=torch.int32, device=dev))
        memb, levels, res = lv.run_levels(g)
        assert levels.shape[0] == 0 and memb.cpu().tolist() == list(range(n))


def test_levels_errors(lv):
    """max_levels below max_passes and a NULL n_levels are refused before anything runs."""
    from paper_2301_12390_amd.louvain import graph_struct, params_struct, _ptr
    from graphgen import two_triangles
    g = two_triangles().to("cuda:0")
    gs = graph_struct(g)
    p = params_struct(max_passes=4)
    memb = torch.empty(g.n, dtype=torch.int32, device="cuda:0")
    levels = torch.full((4, g.n), -7, dtype=torch.int32, device="cuda:0")
    nl = ctypes.c_int32(99)
    st = lv.lib.louvain_run_levels(lv.h, ctypes.byref(gs), ctypes.byref(p), _ptr(memb),
                                   _ptr(levels), 3, ctypes.byref(nl), ctypes.byref(lv._result),
                                   None)
    assert st != 0 and nl.value == 0
    assert b"max_levels" in lv.lib.louvain_last_error(lv.h)
    st = lv.lib.louvain_run_levels(lv.h, ctypes.byref(gs), ctypes.byref(p), _ptr(memb),
                                   _ptr(levels), 4, None, ctypes.byref(lv._result), None)
    assert st != 0
    torch.cuda.synchronize()
    assert (levels.cpu() == -7).all()
    # the context stays usable; two triangles aggregate once
    st = lv.lib.louvain_run_levels(lv.h, ctypes.byref(gs), ctypes.byref(p), _ptr(memb),
                                   _ptr(levels), 4, ctypes.byref(nl), ctypes.byref(lv._result),
                                   None)
    torch.cuda.synchronize()
    assert st == 0 and nl.value == 1
    assert levels[0].cpu().tolist() == [0, 0, 0, 1, 1, 1]
    assert (levels[1:].cpu() == -7).all()
