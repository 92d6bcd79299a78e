"""GPU parity of graph preparation (louvain_prepare) against the oracle's ``prepare``: offsets,
indices and weights element by element, for every flag set, both offset and weight widths,
inputs spanning many sort tiles with a ragged tail, and the edge cases; then prepared graphs
through the whole method against the oracle's run on the oracle's prepared graph.
"""

import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from graphgen import rmat_edges

pytestmark = pytest.mark.gpu

SYM, LOOPS, MAX = 0x1, 0x2, 0x4
TILE_SORT = 0x10  # the per-digit histogram sort instead of the one-sweep look-back sort
FLAG_SETS = [0, SYM, SYM | LOOPS, SYM | LOOPS | MAX, LOOPS | MAX, MAX, LOOPS]


@pytest.fixture(scope="module")
def lv(gpu_device):
    from paper_2301_12390_amd import Louvain, build as B
    if not __import__("os").path.exists(B.LIB):
        B.build()
    ctx = Louvain(0)
    yield ctx
    ctx.close()


def skewed_edges(n, m, seed, wmax=1):
    """Edge list with many repeats and self-loops (squared uniform sources)."""
    rng = np.random.default_rng(seed)
    src = np.minimum((n * rng.random(m) ** 2).astype(np.int64), n - 1).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    w = rng.integers(1, wmax + 1, m).astype(np.uint32) if wmax > 1 else None
    return src, dst, w


def gpu_prepare(lv, n, src, dst, w, flags, offsets_64=True, weights_64=False):
    d = "cuda:0"
    ts = torch.from_numpy(src.astype(np.int32)).to(d)
    td = torch.from_numpy(dst.astype(np.int32)).to(d)
    tw = None if w is None else torch.from_numpy(w.astype(np.uint32).view(np.int32)).to(d)
    g = lv.prepare(n, ts, td, tw, flags=flags, offsets_64=offsets_64, weights_64=weights_64)
    torch.cuda.synchronize()
    off = g.offsets.cpu().numpy().astype(np.int64)
    idx = g.indices.cpu().numpy()
    wo = g.weights.cpu().numpy()
    wo = wo.view(np.uint64) if weights_64 else wo.view(np.uint32).astype(np.uint64)
    return g, off, idx, wo


def check(lv, n, src, dst, w, flags, **kw):
    ref = O.prepare(n, src, dst, w, flags & (SYM | LOOPS | MAX))
    g, off, idx, wo = gpu_prepare(lv, n, src, dst, w, flags, **kw)
    assert np.array_equal(off, ref[0]), (n, flags)
    assert np.array_equal(idx, ref[1]), (n, flags)
    assert np.array_equal(wo, ref[2]), (n, flags)
    return g, ref


@pytest.mark.parametrize("flags", FLAG_SETS)
def test_prepare_small(lv, flags):
    for seed, (n, m, wmax) in enumerate([(5, 12, 1), (40, 300, 9), (1000, 6000, 1),
                                         (3000, 20000, 70000)]):
        src, dst, w = skewed_edges(n, m, seed, wmax)
        check(lv, n, src, dst, w, flags)


@pytest.mark.parametrize("flags", [SYM | LOOPS | MAX, SYM, LOOPS, SYM | LOOPS | TILE_SORT])
@pytest.mark.parametrize("fmt", [(True, False), (False, False), (True, True), (False, True)],
                         ids=["off64-w32", "off32-w32", "off64-w64", "off32-w64"])
def test_prepare_many_tiles(lv, flags, fmt):
    # 2 * 70001 + 50001 arcs: 47 sort tiles of 4096 and a ragged tail; heavy repeats
    n, m = 50001, 70001
    src, dst, w = skewed_edges(n, m, 11, wmax=1000)
    check(lv, n, src, dst, w, flags, offsets_64=fmt[0], weights_64=fmt[1])


def test_prepare_rmat_edge_list(lv):
    # the paper's recipe on a raw R-MAT edge list (repeats, loops, skewed rows)
    n, u, v = rmat_edges(14, seed=3)
    src, dst = u.numpy().astype(np.int32), v.numpy().astype(np.int32)
    for flags in (SYM | LOOPS | MAX, SYM | LOOPS, SYM, SYM | LOOPS | MAX | TILE_SORT):
        check(lv, n, src, dst, None, flags)
    # n not a power of two
    n, u, v = rmat_edges(13, seed=5, n=6000)
    check(lv, n, u.numpy().astype(np.int32), v.numpy().astype(np.int32), None, SYM | LOOPS | MAX)


def test_prepare_long_runs(lv):
    # one edge repeated across several tiles: a run its head's tile combines over the tiles after
    src = np.array([3] * 20000 + [1, 2] * 5000, dtype=np.int32)
    dst = np.array([7] * 20000 + [2, 1] * 5000, dtype=np.int32)
    w = (np.arange(src.size) % 5 + 1).astype(np.uint32)
    for flags in (0, SYM, SYM | MAX, SYM | LOOPS, SYM | TILE_SORT):
        check(lv, 9, src, dst, w, flags)
    # a hub row spanning many tiles
    src = np.zeros(30000, dtype=np.int32)
    dst = np.arange(30000, dtype=np.int32) % 29999 + 1
    check(lv, 30000, src, dst, None, SYM | LOOPS)


def test_prepare_edge_cases(lv):
    e = np.zeros(0, dtype=np.int32)
    for n, flags in [(0, SYM | LOOPS), (1, SYM | LOOPS), (5, SYM), (5, LOOPS), (1, 0)]:
        check(lv, n, e, e, None, flags)
    check(lv, 1, np.zeros(3, dtype=np.int32), np.zeros(3, dtype=np.int32), None, SYM)
    check(lv, 2, np.array([0, 1], dtype=np.int32), np.array([1, 0], dtype=np.int32), None, SYM)


def test_prepare_count_and_capacity(lv):
    from paper_2301_12390_amd import LouvainError
    src, dst, _ = skewed_edges(500, 4000, 5)
    ref = O.prepare(500, src, dst, None, SYM | LOOPS | MAX)
    ts = torch.from_numpy(src).to("cuda:0")
    td = torch.from_numpy(dst).to("cuda:0")
    assert lv.prepare_count(500, ts, td) == ref[1].size
    # exactly enough room works; one less is refused and reports the size
    g = lv.prepare(500, ts, td, capacity=ref[1].size)
    torch.cuda.synchronize()
    assert np.array_equal(g.indices.cpu().numpy(), ref[1])
    with pytest.raises(LouvainError, match="EINVAL"):
        lv.prepare(500, ts, td, capacity=ref[1].size - 1)


def test_prepare_errors(lv):
    from paper_2301_12390_amd import LouvainError
    d = "cuda:0"
    src = torch.tensor([0, 1, 2], dtype=torch.int32, device=d)
    with pytest.raises(LouvainError, match="EINVAL"):
        lv.prepare(3, src, torch.tensor([1, 3, 0], dtype=torch.int32, device=d))
    with pytest.raises(LouvainError, match="EINVAL"):
        lv.prepare(3, src, torch.tensor([1, -1, 0], dtype=torch.int32, device=d))
    with pytest.raises(LouvainError, match="EINVAL"):
        lv.prepare(3, src, torch.tensor([1, 2, 0], dtype=torch.int32, device=d),
                   torch.tensor([1, 0, 1], dtype=torch.int32, device=d))
    with pytest.raises(LouvainError, match="EINVAL"):
        lv.prepare(3, src, src, flags=0x40)
    # combined weights above 32 bits: refused for uint32 output, exact for uint64
    big = torch.tensor([np.int32(-2**31)] * 3, dtype=torch.int32, device=d)  # 2^31 each
    same = torch.tensor([0, 0, 0], dtype=torch.int32, device=d)
    one = torch.tensor([1, 1, 1], dtype=torch.int32, device=d)
    with pytest.raises(LouvainError, match="EOVERFLOW"):
        lv.prepare(2, same, one, big, flags=SYM)
    g = lv.prepare(2, same, one, big, flags=SYM, weights_64=True)
    torch.cuda.synchronize()
    assert g.weights.cpu().tolist() == [3 * 2**31, 3 * 2**31]
    # the context stays usable
    check(lv, 3, np.array([0, 1], dtype=np.int32), np.array([1, 2], dtype=np.int32), None,
          SYM | LOOPS)


def test_prepare_deterministic(lv):
    src, dst, w = skewed_edges(20000, 100000, 9, wmax=50)
    a = gpu_prepare(lv, 20000, src, dst, w, SYM | LOOPS)
    b = gpu_prepare(lv, 20000, src, dst, w, SYM | LOOPS)
    for x, y in zip(a[1:], b[1:]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("flags", [SYM | LOOPS | MAX, SYM | LOOPS])
def test_prepared_graph_runs_like_oracle(lv, flags):
    """Preparation then the whole method, against the oracle's preparation then its run."""
    n, u, v = rmat_edges(12, seed=7)
    src, dst = u.numpy().astype(np.int32), v.numpy().astype(np.int32)
    off, idx, w = O.prepare(n, src, dst, None, flags)
    og = O.Graph(n, off, idx, w)
    top, ref = O.run(og, "sync", substeps=8)
    g, _, _, _ = gpu_prepare(lv, n, src, dst, None, flags)
    memb, res = lv.run(g, substeps=8)
    torch.cuda.synchronize()
    assert np.array_equal(memb.cpu().numpy(), top)
    assert res["qnum"] == ref["qnum"] and res["iterations"] == ref["iterations"]
