"""Synthetic inputs: the batch packing, the batched workload's size distribution and graph
classes, the serving pool, planted hubs, and the vectorised SBM against a per-block reference.
CPU only."""

import math

import numpy as np
import torch

from graphgen import (batch_graph, batch_sizes, pack_graphs, planted_hubs, sbm, single_edge,
                      two_triangles)
from graphgen.csr import Csr, csr_from_edges
from graphgen.generators import _block_start, _T_SBM_IN
from graphgen.rng import draw, srl, stream_key


def test_pack_graphs_layout():
    gs = [two_triangles(), Csr(3, torch.zeros(4, dtype=torch.int32),
                               torch.zeros(0, dtype=torch.int32),
                               torch.zeros(0, dtype=torch.int32)), single_edge(),
          sbm(300, 3, 8.0, 2.0, seed=1, weights=(1, 16))]
    p, vptr, aptr = pack_graphs(gs)
    assert vptr == [0, 6, 9, 11, 311]
    assert aptr[-1] == p.nnz == sum(g.nnz for g in gs)
    off = p.offsets.long()
    for g, gr in enumerate(gs):
        v0, v1, a0 = vptr[g], vptr[g + 1], aptr[g]
        assert int(off[v0]) == a0
        assert torch.equal(off[v0:v1 + 1] - a0, gr.offsets.long())
        idx = p.indices[aptr[g]:aptr[g + 1]].long()
        assert torch.equal(idx - v0, gr.indices.long())
        assert bool(((idx >= v0) & (idx < v1)).all())
        assert torch.equal(p.weights[aptr[g]:aptr[g + 1]].long(), gr.weights.long())


def test_batch_sizes_log_uniform():
    sz = np.array(batch_sizes(2048))
    assert sz.min() >= 200 and sz.max() <= 200001
    # log-uniform on [ln 200, ln 200001]: mean of ln n and the quartiles
    lo, hi = math.log(200), math.log(200001)
    ln = np.log(sz + 0.5)
    assert abs(ln.mean() - (lo + hi) / 2) < 0.15
    assert abs(np.median(ln) - (lo + hi) / 2) < 0.2
    assert abs(sz.mean() - (200001 - 200) / (hi - lo)) / sz.mean() < 0.1
    assert batch_sizes(2048) == batch_sizes(2048)  # seeded


def test_batch_graph_classes():
    g0 = batch_graph(0, 1000)  # even: SBM, 10 blocks
    g1 = batch_graph(1, 1000)  # odd: lattice + shortcuts
    assert g0.name.startswith("sbm-n1000-b10") and g1.name.startswith("lattice-n1000")
    for g in (g0, g1):
        w = g.weights.long()
        assert int(w.min()) >= 1 and int(w.max()) <= 16
        o = g.offsets.long()
        src = torch.repeat_interleave(torch.arange(g.n), o[1:] - o[:-1])
        # symmetric, no self-loops
        fwd = set(zip(src.tolist(), g.indices.tolist()))
        assert all((b, a) in fwd for a, b in fwd) and all(a != b for a, b in fwd)


def sbm_reference(n, blocks, deg_in, seed):
    """The intra-block edges of sbm() drawn block by block (the definition)."""
    s = n / blocks
    thr = int(min(deg_in / max(s - 1, 1), 1.0) * (1 << 53))
    key = stream_key(seed, _T_SBM_IN, n, blocks)
    us, vs = [], []
    for b in range(blocks):
        lo, hi = _block_start(n, blocks, b), _block_start(n, blocks, b + 1)
        iu, iv = torch.triu_indices(hi - lo, hi - lo, offset=1)
        iu, iv = iu.long() + lo, iv.long() + lo
        keep = srl(draw(key, iu * n + iv), 11) < thr
        us.append(iu[keep])
        vs.append(iv[keep])
    return csr_from_edges(n, torch.cat(us), torch.cat(vs))


def test_sbm_intra_blocks_match_per_block_draws():
    n, blocks = 1234, 17  # two block sizes
    g = sbm(n, blocks, 8.0, 0.0, seed=3)
    ref = sbm_reference(n, blocks, 8.0, 3)
    assert torch.equal(g.offsets.long(), ref.offsets.long())
    assert torch.equal(g.indices, ref.indices)


def test_planted_hubs_degrees():
    base = sbm(2000, 20, 8.0, 2.0, seed=1)
    g = planted_hubs(base, [1500, 700], seed=3)
    deg = g.degrees()
    h0, h1 = 1, 7920 % 2000
    assert int(deg[h0]) > 1000 and int(deg[h1]) > 500
    assert g.nnz > base.nnz
