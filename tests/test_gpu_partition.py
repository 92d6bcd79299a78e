"""GPU parity of partition and merge (louvain_run_partitioned) against the oracle's
``run_partitioned``: final membership, the merge run's exact Q and iterations, and every part's
community count and exact Q, for balanced and given parts (empty ones included), on the corpus
and the hub graphs; argument errors.
"""

import numpy as np
import pytest
import torch

import oracle as O
from graphgen import rmat, sbm

from .test_gpu_parity import CORPUS, HUB_IDS, HUBS, IDS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lv(gpu_device):
    from paper_2301_12390_amd import Louvain, build as B
    if not __import__("os").path.exists(B.LIB):
        B.build()
    ctx = Louvain(0)
    yield ctx
    ctx.close()


def check(lv, g, P, vptr=None, substeps=8, flags=0):
    og = O.Graph.from_csr(g)
    ovptr = vptr if vptr is not None else O.balanced_parts(og, P)
    top, ref, parts = O.run_partitioned(og, ovptr, substeps=substeps)
    memb, res, pr = lv.run_partitioned(g.to("cuda:0"), P=P, vptr=vptr, substeps=substeps,
                                       flags=flags)
    torch.cuda.synchronize()
    assert np.array_equal(memb.cpu().numpy(), top), (g.name, P)
    assert res["qnum"] == ref["qnum"] and res["W"] == ref["W"]
    assert res["iterations"] == ref["iterations"] and res["passes"] == ref["passes"]
    assert [p["n_communities"] for p in pr] == [p["n_communities"] for p in parts]
    assert [p["qnum"] for p in pr] == [p["qnum"] for p in parts]
    return res, pr


@pytest.mark.parametrize("P", [1, 2, 5])
@pytest.mark.parametrize("g", CORPUS, ids=IDS)
def test_partitioned(lv, g, P):
    check(lv, g, P)


@pytest.mark.parametrize("K", [1, 32])
def test_partitioned_class_counts(lv, K):
    check(lv, sbm(4000, 40, 8.0, 2.0, seed=9, weights=(1, 16)), 4, substeps=K)


def test_given_parts_with_empty_ones(lv):
    g = sbm(3000, 30, 8.0, 2.0, seed=2, weights=(1, 16))
    check(lv, g, 5, vptr=[0, 0, 1000, 1000, 2500, 3000])
    check(lv, g, 3, vptr=[0, 3000, 3000, 3000])


@pytest.mark.parametrize("flags", [0, 0x8 | 0x4])
@pytest.mark.parametrize("gi", [0, 1], ids=HUB_IDS)
def test_partitioned_hubs(lv, gi, flags):
    check(lv, HUBS[gi], 4, flags=flags)


def test_partitioned_many_parts(lv):
    check(lv, rmat(14, seed=3, weights=(1, 16)), 64)


def test_partitioned_errors(lv):
    from paper_2301_12390_amd import LouvainError
    g = CORPUS[0].to("cuda:0")
    for kw in [dict(P=0), dict(P=2, vptr=[0, 4, 5]), dict(P=2, vptr=[0, 4, 2]),
               dict(P=2, vptr=[1, 3, 6])]:
        with pytest.raises(LouvainError, match="EINVAL"):
            lv.run_partitioned(g, **kw)
    memb, res, pr = lv.run_partitioned(g, P=2)
    torch.cuda.synchronize()
    assert memb.cpu().tolist() == [0, 0, 0, 1, 1, 1]
