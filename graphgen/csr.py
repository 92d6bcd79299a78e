"""Symmetric CSR container and builders.

A graph is stored as arcs: an undirected edge {u, v} with u != v appears as the two arcs
(u, v) and (v, u); a self-loop (u, u) appears once. This is the paper's convention of
duplicating each edge in the reverse direction (its Table 1 caption), so the arc count is the
paper's |E|.
"""

import hashlib
from dataclasses import dataclass

import torch


@dataclass
class Csr:
    n: int
    offsets: torch.Tensor  # int32 or int64 [n+1]
    indices: torch.Tensor  # int32 [nnz]
    weights: torch.Tensor  # int32 (uint32 bit patterns) or int64 (uint64) [nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.indices.numel())

    @property
    def device(self):
        return self.indices.device

    def to(self, device) -> "Csr":
        return Csr(self.n, self.offsets.to(device), self.indices.to(device),
                   self.weights.to(device), self.name)

    def with_offsets(self, dtype) -> "Csr":
        return Csr(self.n, self.offsets.to(dtype), self.indices, self.weights, self.name)

    def total_weight(self) -> int:
        return int(self.weights.to(torch.int64).sum().item())

    def degrees(self) -> torch.Tensor:
        o = self.offsets.to(torch.int64)
        return o[1:] - o[:-1]


def csr_from_arcs(n: int, src: torch.Tensor, dst: torch.Tensor, w: torch.Tensor,
                  offsets_dtype=torch.int32, weights_dtype=torch.int32, name="") -> Csr:
    """CSR from an arc list, rows sorted by (src, dst); duplicate arcs are kept as given."""
    src = src.to(torch.int64)
    dst = dst.to(torch.int64)
    key = src * n + dst
    order = torch.argsort(key, stable=True)
    src = src[order]
    dst = dst[order]
    w = w.to(torch.int64)[order]
    counts = torch.bincount(src, minlength=n) if src.numel() else torch.zeros(
        n, dtype=torch.int64, device=src.device)
    offsets = torch.zeros(n + 1, dtype=torch.int64, device=src.device)
    offsets[1:] = torch.cumsum(counts, 0)
    if offsets_dtype == torch.int32:
        assert int(offsets[-1]) < (1 << 31)
    return Csr(n, offsets.to(offsets_dtype), dst.to(torch.int32), w.to(weights_dtype), name)


def csr_from_edges(n: int, u: torch.Tensor, v: torch.Tensor, weight_fn=None,
                   offsets_dtype=torch.int32, keep_self_loops=False, name="",
                   chunk: int = 1 << 27) -> Csr:
    """Symmetric simple graph from an undirected edge list.

    Self-loops are dropped (unless ``keep_self_loops``), every edge becomes two arcs, and
    repeated pairs collapse to one. ``weight_fn(lo, hi)`` gives the weight of the unordered pair
    {lo, hi} (lo <= hi) as an int64 tensor; it must depend on the pair only, so both arcs of an
    edge and every repeat of it carry the same weight. ``None`` means unit weights.
    """
    dev = u.device
    u = u.to(torch.int64)
    v = v.to(torch.int64)
    if not keep_self_loops:
        m = u != v
        u, v = u[m], v[m]
    lo = torch.minimum(u, v)
    hi = torch.maximum(u, v)
    del u, v
    # unique undirected pairs (sorted keys), then expand to arcs
    pk = torch.unique(lo * n + hi)
    del lo, hi
    lo = torch.div(pk, n, rounding_mode="floor")
    hi = pk - lo * n
    del pk
    if weight_fn is None:
        wp = None
    else:
        wp = weight_fn(lo, hi)
    loop = lo == hi
    a_src = torch.cat([lo, hi[~loop]])
    a_dst = torch.cat([hi, lo[~loop]])
    if wp is not None:
        a_w = torch.cat([wp, wp[~loop]])
    del lo, hi
    key = a_src * n + a_dst
    del a_src
    order = torch.argsort(key)
    key = key[order]
    if wp is not None:
        a_w = a_w[order]
    del order, a_dst
    rows = torch.div(key, n, rounding_mode="floor")
    cols = (key - rows * n).to(torch.int32)
    del key
    counts = torch.bincount(rows, minlength=n)
    del rows
    offsets = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    offsets[1:] = torch.cumsum(counts, 0)
    del counts
    if offsets_dtype == torch.int32:
        assert int(offsets[-1]) < (1 << 31)
        offsets = offsets.to(torch.int32)
    if wp is None:
        weights = torch.ones(cols.numel(), dtype=torch.int32, device=dev)
    else:
        weights = a_w.to(torch.int32)
    return Csr(n, offsets, cols, weights, name)


def csr_sha256(g: Csr) -> str:
    """SHA-256 over (n, offsets as int64, indices as int32, weights as int64), little endian."""
    h = hashlib.sha256()
    h.update(int(g.n).to_bytes(8, "little"))
    h.update(g.offsets.to(torch.int64).cpu().numpy().tobytes())
    h.update(g.indices.to(torch.int32).cpu().numpy().tobytes())
    h.update(g.weights.to(torch.int64).cpu().numpy().tobytes())
    return h.hexdigest()


def pack_graphs(graphs, device=None, offsets_dtype=None):
    """One CSR holding the given graphs with consecutive vertex ids (graph g owns vertices
    vptr[g] .. vptr[g+1]-1 and arcs aptr[g] .. aptr[g+1]-1). Returns (packed, vptr, aptr) with
    vptr and aptr as Python lists. Weights are widened to the widest input type."""
    assert graphs, "no graphs"
    dev = device if device is not None else graphs[0].device
    wdt = torch.int64 if any(g.weights.dtype == torch.int64 for g in graphs) else torch.int32
    vptr, aptr = [0], [0]
    offs, idxs, ws = [], [], []
    for g in graphs:
        offs.append(g.offsets[:-1].to(dev, torch.int64) + aptr[-1])
        idxs.append(g.indices.to(dev, torch.int64) + vptr[-1])
        ws.append(g.weights.to(dev, wdt))
        vptr.append(vptr[-1] + g.n)
        aptr.append(aptr[-1] + g.nnz)
    nnz = aptr[-1]
    if offsets_dtype is None:
        offsets_dtype = torch.int64 if nnz >= (1 << 31) else torch.int32
    offs.append(torch.tensor([nnz], dtype=torch.int64, device=dev))
    packed = Csr(vptr[-1], torch.cat(offs).to(offsets_dtype), torch.cat(idxs).to(torch.int32),
                 torch.cat(ws), name=f"batch-{len(graphs)}")
    return packed, vptr, aptr
