"""Seeded graph generators (integer-only, device independent).

Every random choice is a counter-based SplitMix64 draw (see ``rng``), compared against integer
thresholds, so the CPU and the GPU build identical graphs from the same seed.
"""

import math

import torch

from .csr import Csr, csr_from_arcs, csr_from_edges
from .rng import below, draw, low32, mix_int, srl, stream_key, top32

# stream tags
_T_RMAT = 1
_T_PERM = 2
_T_WEIGHT = 3
_T_SBM_IN = 4
_T_SBM_OUT = 5
_T_LAT = 6
_T_ER = 7
_T_HUBS = 8
_T_BATCH = 9
_T_SERVE = 10


def _pair_weights(key: int, n: int, wmin: int, wmax: int):
    """weight_fn for csr_from_edges: uniform integer in [wmin, wmax] per unordered pair."""
    span = wmax - wmin + 1

    def fn(lo, hi):
        d = draw(key, lo * n + hi)
        if span & (span - 1) == 0:
            shift = 64 - (span.bit_length() - 1)
            r = srl(d, shift) if shift < 64 else torch.zeros_like(d)
        else:
            r = top32(d) % span
        return r + wmin

    return fn


def rmat_edges(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
               c: float = 0.19, seed: int = 1, permute: bool = True, device="cpu",
               chunk: int = 1 << 24, n: int = None):
    """The raw R-MAT edge list behind ``rmat``: (n, u, v) with int64 endpoint tensors of
    ``edge_factor * n`` drawn pairs, self-loops and repeats included (an edge-list file as
    graph preparation receives it)."""
    N = 1 << scale
    if n is None:
        n = N
    assert n <= N
    m = edge_factor * n
    ta = int(round(a * 2**32))
    tb = int(round((a + b) * 2**32))
    tc = int(round((a + b + c) * 2**32))
    key = stream_key(seed, _T_RMAT, scale)
    per_edge = (scale + 1) // 2  # one 64-bit draw covers two levels
    us, vs = [], []
    produced = 0
    counter = 0
    # endpoint pair number e uses draws e*per_edge .. e*per_edge+per_edge-1; the graph keeps the
    # first m pairs (in counter order) whose endpoints are both < n
    while produced < m:
        cnt = min(chunk, m - produced) if n == N else chunk
        e = torch.arange(counter, counter + cnt, dtype=torch.int64, device=device)
        counter += cnt
        u = torch.zeros(cnt, dtype=torch.int64, device=device)
        v = torch.zeros(cnt, dtype=torch.int64, device=device)
        base = e * per_edge
        del e
        for lvl in range(scale):
            d = draw(key, base + lvl // 2)
            r = top32(d) if lvl % 2 == 0 else low32(d)
            del d
            bu = (r >= tb).to(torch.int64)
            bv = (((r >= ta) & (r < tb)) | (r >= tc)).to(torch.int64)
            del r
            u = (u << 1) | bu
            v = (v << 1) | bv
        del base
        if n < N:
            ok = (u < n) & (v < n)
            u, v = u[ok], v[ok]
        us.append(u)
        vs.append(v)
        produced += int(u.numel())
    u = torch.cat(us)[:m]
    v = torch.cat(vs)[:m]
    del us, vs
    if permute:
        pk = stream_key(seed, _T_PERM, scale)
        order = torch.argsort(draw(pk, torch.arange(n, dtype=torch.int64, device=device)))
        newid = torch.empty(n, dtype=torch.int64, device=device)
        newid[order] = torch.arange(n, dtype=torch.int64, device=device)
        del order
        u = newid[u]
        v = newid[v]
        del newid
    return n, u, v


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, permute: bool = True, weights=(1, 1), offsets_dtype=torch.int32,
         device="cpu", chunk: int = 1 << 24, n: int = None) -> Csr:
    """R-MAT graph (Chakrabarti, Zhan, Faloutsos 2004) as a symmetric simple CSR.

    ``edge_factor * 2^scale`` directed endpoint pairs are drawn; each of the ``scale`` levels
    picks a quadrant with probabilities (a, b, c, 1-a-b-c) by comparing a 32-bit draw with
    integer thresholds. Ids are then relabelled by a seeded random permutation (Graph500
    practice), self-loops are dropped, edges are symmetrised and repeats removed. Weights are
    drawn per unordered pair, uniform in ``weights = (wmin, wmax)``.

    If ``n`` is given and is not a power of two, endpoints >= n are redrawn at the next counter
    (the graph then has n vertices and ``scale = ceil(log2 n)``).
    """
    n, u, v = rmat_edges(scale, edge_factor, a, b, c, seed, permute, device, chunk, n)
    wfn = None
    if weights != (1, 1):
        wfn = _pair_weights(stream_key(seed, _T_WEIGHT, scale), n, weights[0], weights[1])
    name = f"rmat-s{scale}-ef{edge_factor}-seed{seed}"
    return csr_from_edges(n, u, v, wfn, offsets_dtype=offsets_dtype, name=name)


def _block_of(n: int, blocks: int, x: torch.Tensor) -> torch.Tensor:
    """Block index of vertex x for ``blocks`` contiguous near-equal blocks of [0, n)."""
    return torch.div(x * blocks, n, rounding_mode="floor")


def _block_start(n: int, blocks: int, b: int) -> int:
    return -(-b * n // blocks)  # ceil(b*n/blocks): the first x with floor(x*blocks/n) == b


def sbm(n: int = 10000, blocks: int = 100, deg_in: float = 8.0, deg_out: float = 2.0,
        seed: int = 1, weights=(1, 1), offsets_dtype=torch.int32, device="cpu",
        p_in: float = None, p_out: float = None) -> Csr:
    """Planted-partition stochastic block model.

    ``blocks`` contiguous blocks of near-equal size s. Each intra-block pair is an edge with
    probability p_in = deg_in/(s-1) (one Bernoulli draw per pair, 53-bit integer threshold).
    Inter-block edges: M = round(p_out * #inter-pairs) uniform random vertex pairs with
    p_out = deg_out/(n-s); pairs inside one block are discarded and repeats collapse, so the
    expected inter-block degree is deg_out up to O(M^2/pairs) collisions.
    """
    s = n / blocks
    if p_in is None:
        p_in = deg_in / max(s - 1, 1)
    if p_out is None:
        p_out = deg_out / max(n - s, 1)
    thr_in = int(min(p_in, 1.0) * (1 << 53))
    key_in = stream_key(seed, _T_SBM_IN, n, blocks)
    key_out = stream_key(seed, _T_SBM_OUT, n, blocks)
    us, vs = [], []
    starts = [_block_start(n, blocks, b) for b in range(blocks + 1)]
    sizes = [starts[b + 1] - starts[b] for b in range(blocks)]
    # intra-block pairs of all blocks of one size at once (block sizes take at most two values);
    # each pair's draw is at its own counter, so the order of generation does not matter
    for sz in sorted(set(sizes)):
        if sz < 2:
            continue
        lo = torch.tensor([starts[b] for b in range(blocks) if sizes[b] == sz], dtype=torch.int64,
                          device=device)
        iu, iv = torch.triu_indices(sz, sz, offset=1, device=device)
        for part in torch.split(lo, max(1, (1 << 24) // iu.numel())):
            bu = (part[:, None] + iu[None, :].to(torch.int64)).reshape(-1)
            bv = (part[:, None] + iv[None, :].to(torch.int64)).reshape(-1)
            keep = srl(draw(key_in, bu * n + bv), 11) < thr_in
            us.append(bu[keep])
            vs.append(bv[keep])
    inter_pairs = (n * n - sum(z * z for z in sizes)) // 2
    M = int(round(p_out * inter_pairs))
    if M > 0:
        ctr = torch.arange(M, dtype=torch.int64, device=device)
        a = below(draw(key_out, 2 * ctr), n)
        b2 = below(draw(key_out, 2 * ctr + 1), n)
        keep = _block_of(n, blocks, a) != _block_of(n, blocks, b2)
        us.append(a[keep])
        vs.append(b2[keep])
    u = torch.cat(us) if us else torch.zeros(0, dtype=torch.int64, device=device)
    v = torch.cat(vs) if vs else torch.zeros(0, dtype=torch.int64, device=device)
    wfn = None
    if weights != (1, 1):
        wfn = _pair_weights(stream_key(seed, _T_WEIGHT, n, blocks), n, weights[0], weights[1])
    return csr_from_edges(n, u, v, wfn, offsets_dtype=offsets_dtype,
                          name=f"sbm-n{n}-b{blocks}-seed{seed}")


def lattice_shortcuts(n: int, shortcut_frac: float = 0.1, seed: int = 1, weights=(1, 16),
                      offsets_dtype=torch.int32, device="cpu") -> Csr:
    """r x c four-neighbour lattice (r = floor(sqrt(n)), c = floor(n/r)) plus
    round(shortcut_frac * |E_lattice|) uniform random shortcut edges (self-loops dropped,
    repeats collapse). Vertices r*c .. n-1, if any, stay isolated."""
    r = max(1, int(math.isqrt(n)))
    c = max(1, n // r)
    ids = torch.arange(r * c, dtype=torch.int64, device=device).view(r, c)
    hu = ids[:, :-1].reshape(-1)
    hv = ids[:, 1:].reshape(-1)
    vu = ids[:-1, :].reshape(-1)
    vv = ids[1:, :].reshape(-1)
    E = hu.numel() + vu.numel()
    M = int(round(shortcut_frac * E))
    key = stream_key(seed, _T_LAT, n)
    ctr = torch.arange(M, dtype=torch.int64, device=device)
    su = below(draw(key, 2 * ctr), n)
    sv = below(draw(key, 2 * ctr + 1), n)
    u = torch.cat([hu, vu, su])
    v = torch.cat([hv, vv, sv])
    wfn = None
    if weights != (1, 1):
        wfn = _pair_weights(stream_key(seed, _T_WEIGHT, n, 7), n, weights[0], weights[1])
    return csr_from_edges(n, u, v, wfn, offsets_dtype=offsets_dtype,
                          name=f"lattice-n{n}-seed{seed}")


def ring_of_cliques(num_cliques: int, k: int, device="cpu", offsets_dtype=torch.int32) -> Csr:
    """``num_cliques`` complete graphs K_k arranged in a ring: the last vertex of clique t is
    joined to the first vertex of clique t+1 (mod num_cliques). Unit weights."""
    us, vs = [], []
    for t in range(num_cliques):
        base = t * k
        for i in range(k):
            for j in range(i + 1, k):
                us.append(base + i)
                vs.append(base + j)
        if num_cliques > 1:
            us.append(base + k - 1)
            vs.append(((t + 1) % num_cliques) * k)
    n = num_cliques * k
    return csr_from_edges(n, torch.tensor(us, device=device), torch.tensor(vs, device=device),
                          None, offsets_dtype=offsets_dtype, name=f"ring{num_cliques}xK{k}")


def two_triangles(device="cpu") -> Csr:
    """Triangles {0,1,2} and {3,4,5} joined by the edge 2-3 (unit weights)."""
    u = torch.tensor([0, 0, 1, 3, 3, 4, 2], device=device)
    v = torch.tensor([1, 2, 2, 4, 5, 5, 3], device=device)
    return csr_from_edges(6, u, v, None, name="two-triangles")


def single_edge(device="cpu") -> Csr:
    return csr_from_edges(2, torch.tensor([0], device=device), torch.tensor([1], device=device),
                          None, name="single-edge")


def erdos_renyi(n: int, p: float, seed: int = 1, weights=(1, 1), self_loops: bool = False,
                offsets_dtype=torch.int32, device="cpu") -> Csr:
    """G(n, p) by one Bernoulli draw per unordered pair (small n only). With ``self_loops``
    each vertex also gets a loop with probability p."""
    key = stream_key(seed, _T_ER, n)
    iu, iv = torch.triu_indices(n, n, offset=0 if self_loops else 1, device=device)
    iu = iu.to(torch.int64)
    iv = iv.to(torch.int64)
    thr = int(min(p, 1.0) * (1 << 53))
    keep = srl(draw(key, iu * n + iv), 11) < thr
    u, v = iu[keep], iv[keep]
    wfn = None
    if weights != (1, 1):
        wfn = _pair_weights(stream_key(seed, _T_WEIGHT, n, 11), n, weights[0], weights[1])
    return csr_from_edges(n, u, v, wfn, offsets_dtype=offsets_dtype, keep_self_loops=self_loops,
                          name=f"er-n{n}-p{p}-seed{seed}")


def planted_hubs(base: Csr, hub_degrees, seed: int = 1, weights=(1, 1)) -> Csr:
    """``base`` plus hub vertices: hub i (vertex (i * 7919 + 1) mod n) gets edges to
    hub_degrees[i] uniform random vertices (repeats collapse, so its degree is at most that).
    Gives power-law-like rows far longer than one workgroup's table on a small graph."""
    n = base.n
    dev = base.device
    o = base.offsets.to(torch.int64)
    src = torch.repeat_interleave(torch.arange(n, dtype=torch.int64, device=dev), o[1:] - o[:-1])
    dst = base.indices.to(torch.int64)
    keep = src < dst
    us, vs = [src[keep]], [dst[keep]]
    key = stream_key(seed, _T_HUBS, n, len(hub_degrees))
    start = 0
    for i, d in enumerate(hub_degrees):
        h = (i * 7919 + 1) % n
        ctr = torch.arange(start, start + d, dtype=torch.int64, device=dev)
        start += d
        us.append(torch.full((d,), h, dtype=torch.int64, device=dev))
        vs.append(below(draw(key, ctr), n))
    wfn = None
    if weights != (1, 1):
        wfn = _pair_weights(stream_key(seed, _T_WEIGHT, n, 12), n, weights[0], weights[1])
    return csr_from_edges(n, torch.cat(us), torch.cat(vs), wfn,
                          offsets_dtype=base.offsets.dtype,
                          name=f"{base.name}+hubs{list(hub_degrees)}-seed{seed}")


def add_self_loops(g: Csr, weight: int = 1) -> Csr:
    """The paper's preprocessing (its dataset section): add a self-loop of the given weight to
    every vertex that has none. Returns a new CSR with rows re-sorted."""
    o = g.offsets.to(torch.int64)
    deg = o[1:] - o[:-1]
    src = torch.repeat_interleave(torch.arange(g.n, dtype=torch.int64, device=g.device), deg)
    dst = g.indices.to(torch.int64)
    has = torch.zeros(g.n, dtype=torch.bool, device=g.device)
    has[src[src == dst]] = True
    add = torch.nonzero(~has).flatten()
    src = torch.cat([src, add])
    dst = torch.cat([dst, add])
    w = torch.cat([g.weights.to(torch.int64),
                   torch.full((add.numel(),), weight, dtype=torch.int64, device=g.device)])
    return csr_from_arcs(g.n, src, dst, w, offsets_dtype=g.offsets.dtype,
                         weights_dtype=g.weights.dtype, name=g.name + "+loops")


def batch_sizes(count: int = 2048, seed: int = 1, nmin: int = 200, nmax: int = 200001):
    """Vertex counts of a batch: n_g = floor(exp(U(ln nmin, ln nmax))) with U from the 53 top
    bits of draw g of the batch's stream."""
    key = stream_key(seed, _T_BATCH, count)
    u = srl(draw(key, torch.arange(count, dtype=torch.int64)), 11).tolist()
    lo, hi = math.log(nmin), math.log(nmax)
    return [int(math.floor(math.exp(lo + (x / float(1 << 53)) * (hi - lo)))) for x in u]


def batch_graph(g: int, n: int, seed: int = 1, device="cpu") -> Csr:
    """Graph g of a batch: even g an SBM with max(1, round(n/100)) near-equal blocks, expected
    intra/inter degree 8/2; odd g an r x c lattice plus 10% shortcuts; weights 1..16; graph
    seed = SplitMix64 finaliser of (seed xor g)."""
    gseed = mix_int(seed ^ g)
    if g % 2 == 0:
        return sbm(n, max(1, round(n / 100)), 8.0, 2.0, seed=gseed, weights=(1, 16),
                   device=device)
    return lattice_shortcuts(n, 0.1, seed=gseed, weights=(1, 16), device=device)


def batch_config(count: int = 2048, seed: int = 1, device="cpu"):
    """The batched workload: ``count`` graphs (see batch_sizes and batch_graph)."""
    return [batch_graph(g, n, seed, device) for g, n in enumerate(batch_sizes(count, seed))]


def serving_pool(count: int = 32, seed: int = 1, nmin: int = 1000, nmax: int = 4000000,
                 device="cpu"):
    """Request graphs of the serving workload: n log-uniform in [nmin, nmax]; R-MAT (0.57,
    0.19, 0.19, 0.05, edge factor 16, scale ceil(log2 n), endpoints >= n redrawn) or SBM
    (round(n / 100) blocks, expected intra/inter degree 8/2) with probability 1/2 each; weights
    1..16. Returns the graphs (a pool that requests draw from)."""
    key = stream_key(seed, _T_SERVE, count)
    d = draw(key, torch.arange(2 * count, dtype=torch.int64)).tolist()
    lo, hi = math.log(nmin), math.log(nmax + 1)
    out = []
    for i in range(count):
        u = ((d[2 * i] >> 11) & ((1 << 53) - 1)) / float(1 << 53)
        n = int(math.floor(math.exp(lo + u * (hi - lo))))
        gseed = mix_int(seed ^ (i + 0x5E5E))
        if (d[2 * i + 1] >> 63) & 1:
            sc = max(1, (n - 1).bit_length())
            out.append(rmat(sc, 16, seed=gseed, weights=(1, 16), device=device, n=n))
        else:
            out.append(sbm(n, max(1, round(n / 100)), 8.0, 2.0, seed=gseed, weights=(1, 16),
                           device=device))
    return out


def config_graph(name: str, device="cpu") -> Csr:
    """The named benchmark workloads.

    * ``sbm10k``: 10,000 vertices, 100 blocks, expected intra/inter degree 8/2, unit weights,
      int32 offsets, seed 1.
    * ``rmat22``: R-MAT scale 22, edge factor 16, (0.57, 0.19, 0.19, 0.05), unit weights, int32
      offsets, seed 1.
    * ``rmat25``: R-MAT scale 25, same parameters, weights uniform 1..16, int64 offsets, seed 1.
    * ``rmatNN`` for other scales: unit weights, int32 offsets (int64 from scale 25 on, with
      weights 1..16).
    """
    if name == "sbm10k":
        return sbm(10000, 100, 8.0, 2.0, seed=1, device=device)
    if name.startswith("rmat"):
        s = int(name[4:])
        if s >= 25:
            return rmat(s, 16, seed=1, weights=(1, 16), offsets_dtype=torch.int64, device=device)
        return rmat(s, 16, seed=1, device=device)
    raise ValueError(name)
