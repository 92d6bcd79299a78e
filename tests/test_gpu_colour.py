"""GPU parity of colour classes (LV_COLOR_CLASSES, louvain_colour_classes) against the oracle:
the colouring itself element by element, single iterations whose class steps are the colour
classes, whole runs, a batch, and on R-MAT s22 the colouring exactly plus a check that every
vertex holds the first-fit colour of its higher-priority neighbours (a property that holds at
any size and determines the colouring).
"""

import numpy as np
import pytest
import torch

import oracle as O
from graphgen import pack_graphs, planted_hubs, rmat, sbm
from graphgen.rng import GAMMA, MASK64, splitmix64_mix

from .gpu_util import assert_state_equal, gpu_state
from .test_gpu_parity import CORPUS, HUB_IDS, HUBS, IDS

pytestmark = pytest.mark.gpu

COLOUR = 0x10


@pytest.fixture(scope="module")
def lv(gpu_device):
    from paper_2301_12390_amd import Louvain, build as B
    if not __import__("os").path.exists(B.LIB):
        B.build()
    ctx = Louvain(0)
    yield ctx
    ctx.close()


@pytest.mark.parametrize("K", [2, 8, 32])
@pytest.mark.parametrize("g", CORPUS, ids=IDS)
def test_colouring(lv, g, K):
    og = O.Graph.from_csr(g)
    dg = g.to("cuda:0")
    for p in (0, 3):
        c, rounds = lv.colour_classes(dg, p, K)
        torch.cuda.synchronize()
        assert np.array_equal(c.cpu().numpy().astype(np.int32), O.colour_classes(og, p, K)), p
        # vertices without a neighbour take colour 0 in the counting pass; any other vertex
        # is coloured by a round
        assert rounds >= (1 if has_neighbour(g) else 0)


def has_neighbour(g):
    off = g.offsets.cpu().numpy().astype(np.int64)
    src = np.repeat(np.arange(g.n), np.diff(off))
    return bool((g.indices.cpu().numpy().astype(np.int64) != src).any())


def isolated_mix(seed):
    # an Erdos-Renyi graph whose vertex v becomes 3v + 1, plus self loops on every fifth other
    # vertex: a third of the ids hold arcs, the rest none or only a self loop
    from graphgen import csr_from_arcs, erdos_renyi
    base = erdos_renyi(400, 0.015, seed=seed, weights=(1, 5))
    off = base.offsets.numpy().astype(np.int64)
    src = np.repeat(np.arange(base.n), np.diff(off)) * 3 + 1
    dst = base.indices.numpy().astype(np.int64) * 3 + 1
    n = base.n * 3 + 2
    loops = np.array([v for v in range(0, n, 5) if v % 3 != 1], np.int64)
    src = np.concatenate([src, loops])
    dst = np.concatenate([dst, loops])
    w = torch.cat([base.weights, torch.full((len(loops),), 2, dtype=base.weights.dtype)])
    return csr_from_arcs(n, torch.from_numpy(src), torch.from_numpy(dst), w,
                         name=f"isolated-mix-{seed}")


@pytest.mark.parametrize("K", [2, 8, 32])
def test_colouring_vertices_without_neighbours(lv, K):
    for seed in (1, 2):
        g = isolated_mix(seed)
        og = O.Graph.from_csr(g)
        for p in (0, 2):
            c, rounds = lv.colour_classes(g.to("cuda:0"), p, K)
            torch.cuda.synchronize()
            assert np.array_equal(c.cpu().numpy().astype(np.int32), O.colour_classes(og, p, K))
            assert rounds >= 1
    # only self loops: every vertex is colour 0, and no round runs
    from graphgen import csr_from_arcs
    v = torch.arange(50, dtype=torch.int64)
    g = csr_from_arcs(50, v, v, torch.ones(50, dtype=torch.int64), name="loops-only")
    c, rounds = lv.colour_classes(g.to("cuda:0"), 0, K)
    torch.cuda.synchronize()
    assert (c.cpu() == 0).all() and rounds == 0


@pytest.mark.parametrize("gi", [0, 1], ids=HUB_IDS)
def test_colouring_hub_rows(lv, gi):
    g = HUBS[gi]
    og = O.Graph.from_csr(g)
    c, _ = lv.colour_classes(g.to("cuda:0"), 1, 32)
    torch.cuda.synchronize()
    assert np.array_equal(c.cpu().numpy().astype(np.int32), O.colour_classes(og, 1, 32))


def colour_iterations(lv, g, K, flags=0, max_iters=30, pass_index=0):
    og = O.Graph.from_csr(g)
    dg = g.to("cuda:0")
    st = O.State(og)
    C, Sig, cs, Kd = gpu_state(st)
    col = O.colour_classes(og, pass_index, K)
    classes = [np.nonzero(col == k)[0].astype(np.int32) for k in range(K)]
    for it in range(max_iters):
        stats = lv.move(dg, C, Sig, cs, K=Kd, W=st.W, max_iterations=1, flags=COLOUR | flags,
                        substeps=K, pass_index=pass_index)
        S, moved, ncand = O.substep_iteration(og, st, pass_index, K, classes)
        torch.cuda.synchronize()
        assert_state_equal(st, C, Sig, cs, f"iteration {it}")
        assert stats["last_gain"] == S and stats["last_moved"] == moved, it
        assert stats["last_candidates"] == ncand, it
        if moved == 0:
            break


@pytest.mark.parametrize("g", CORPUS[2:], ids=IDS[2:])
def test_colour_class_iterations(lv, g):
    colour_iterations(lv, g, 8)


def test_colour_class_iterations_hubs(lv):
    colour_iterations(lv, HUBS[0], 32, pass_index=2)
    colour_iterations(lv, HUBS[1], 8, flags=0x8)


def check_colour_run(lv, g, K, flags=0):
    og = O.Graph.from_csr(g)
    top, ref = O.run(og, "sync", substeps=K, colour=True)
    memb, res = lv.run(g.to("cuda:0"), flags=COLOUR | flags, substeps=K)
    torch.cuda.synchronize()
    assert np.array_equal(memb.cpu().numpy(), top), g.name
    assert res["qnum"] == ref["qnum"] and res["iterations"] == ref["iterations"]
    assert [t["S"] for t in res["trace"]] == ref["trace_S"]
    assert res["qnum_pass"] == ref["qnum_pass"] and res["nnz_pass"] == ref["nnz_pass"]
    return res, ref


@pytest.mark.parametrize("K", [4, 8, 32])
@pytest.mark.parametrize("g", CORPUS, ids=IDS)
def test_colour_run(lv, g, K):
    check_colour_run(lv, g, K)


@pytest.mark.parametrize("flags", [0, 0x8 | 0x4])
@pytest.mark.parametrize("gi", [0, 1], ids=HUB_IDS)
def test_colour_run_hubs(lv, gi, flags):
    check_colour_run(lv, HUBS[gi], 8, flags)


@pytest.mark.parametrize("K", [2, 8])
@pytest.mark.parametrize("g", [g for g in CORPUS if g.n >= 1000], ids=[g.name for g in CORPUS
                                                                     if g.n >= 1000])
def test_colour_run_small_stages(lv, g, K):
    # LV_SMALL_PARTS also shrinks the colouring's per-workgroup append stages to a few entries,
    # so most frontier appends take the overflow path straight to the global lists
    check_colour_run(lv, g, K, 0x8)


def test_colour_run_levels(lv):
    g = rmat(13, seed=9)
    og = O.Graph.from_csr(g)
    top, ref = O.run(og, "sync", substeps=8, colour=True, levels=True)
    memb, levels, res = lv.run_levels(g.to("cuda:0"), flags=COLOUR, substeps=8)
    torch.cuda.synchronize()
    assert np.array_equal(levels.cpu().numpy(), ref["levels"])


def test_colour_batched(lv):
    graphs = [sbm(3000, 30, 8.0, 2.0, seed=s, weights=(1, 16)) for s in range(3)]
    graphs += [rmat(11, seed=4), planted_hubs(rmat(10, seed=2), [3000], seed=1)]
    packed, vptr, aptr = pack_graphs(graphs, device="cuda:0")
    memb, res = lv.run_batched(packed, vptr, aptr, flags=COLOUR, substeps=8)
    torch.cuda.synchronize()
    m = memb.cpu().numpy()
    for k, g in enumerate(graphs):
        top, ref = O.run(O.Graph.from_csr(g), "sync", substeps=8, colour=True)
        assert np.array_equal(m[vptr[k]:vptr[k + 1]], top), k
        assert res[k]["qnum"] == ref["qnum"] and res[k]["iterations"] == ref["iterations"]


def test_colour_errors(lv):
    from paper_2301_12390_amd import LouvainError
    g = CORPUS[0].to("cuda:0")
    with pytest.raises(LouvainError, match="EINVAL"):
        lv.colour_classes(g, 0, 33)
    with pytest.raises(LouvainError, match="EINVAL"):
        lv.colour_classes(g, -1, 8)
    c, rounds = lv.colour_classes(g, 0, 1)
    torch.cuda.synchronize()
    assert (c.cpu() == 0).all() and rounds == 0


def first_fit_check(g, c, p, K, chunk=1 << 26):
    """Every vertex holds the first-fit colour of its higher-priority neighbours: by induction
    over the priority order this determines the colouring. Checked with torch on the GPU,
    priorities recomputed from the SplitMix64 definition."""
    n = g.n
    v = torch.arange(n, device="cuda:0", dtype=torch.int64)
    z = splitmix64_mix(p + (v + 1) * (GAMMA - (1 << 64)))
    key = z ^ (-(1 << 63))  # unsigned order as signed order
    off = g.offsets.to(torch.int64)
    deg = off[1:] - off[:-1]
    c64 = c.to(torch.int64)
    held = torch.zeros(n * 32, dtype=torch.bool, device="cuda:0")
    for a0 in range(0, g.nnz, chunk):
        a1 = min(g.nnz, a0 + chunk)
        ar = torch.arange(a0, a1, device="cuda:0", dtype=torch.int64)
        src = torch.searchsorted(off, ar, right=True) - 1
        dst = g.indices[a0:a1].to(torch.int64)
        higher = (key[dst] > key[src]) & (dst != src)
        cu = c64[dst]
        sel = higher & (cu < K - 1)
        held[src[sel] * 32 + cu[sel]] = True
        del ar, src, dst, higher, cu, sel
    held = held.view(n, 32)[:, :K - 1]
    free = ~held
    first = torch.where(free.any(dim=1), free.to(torch.int8).argmax(dim=1),
                        torch.full((n,), K - 1, device="cuda:0", dtype=torch.int64))
    bad = int((first != c64).sum())
    assert bad == 0, f"{bad} vertices do not hold their first-fit colour"
    del deg


@pytest.mark.timeout(600)
def test_colouring_rmat22_exact_and_first_fit(lv):
    from graphgen import config_graph
    g = config_graph("rmat22", device="cuda:0")
    c, rounds = lv.colour_classes(g, 0, 32)
    torch.cuda.synchronize()
    og = O.Graph.from_csr(g)
    assert np.array_equal(c.cpu().numpy().astype(np.int32), O.colour_classes(og, 0, 32))
    first_fit_check(g, c, 0, 32)
    print(f"rmat22: {rounds} rounds", flush=True)
