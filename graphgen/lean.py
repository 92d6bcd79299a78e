"""Memory-lean construction of a large R-MAT CSR on the host.

``rmat`` builds its CSR with whole-array torch sorts, which need several copies of the arc list
at once; at scale 25 (1.05e9 arcs) that exceeds a 64 GB host. This module builds the identical
graph (same endpoint draws, permutation, pair set, weights and row order; checked against
``rmat`` at small scales) with in-place numpy sorts of 8-byte pair keys and chunked passes, and
keeps the result in ``.npy`` files that can be memory-mapped.

Row r of the CSR holds its neighbours in ascending order: first the smaller ends of the pairs
{x, r} with x < r, then the larger ends of the pairs {r, y} with y > r. Both halves come out of
one sorted list of pair keys each, so no arc-level sort is needed.
"""

import hashlib
import os

import numpy as np
import torch

from .generators import _T_WEIGHT, rmat_edges
from .rng import draw, srl, stream_key, top32

_CHUNK = 1 << 26


def _pair_weight_np(wkey: int, n: int, wmin: int, wmax: int, lo: np.ndarray, hi: np.ndarray):
    """The per-pair weight of ``rmat`` (uniform in [wmin, wmax], drawn at counter lo*n + hi)."""
    span = wmax - wmin + 1
    d = draw(wkey, torch.from_numpy(lo * n + hi))
    if span & (span - 1) == 0:
        shift = 64 - (span.bit_length() - 1)
        r = srl(d, shift) if shift < 64 else torch.zeros_like(d)
    else:
        r = top32(d) % span
    return (r + wmin).numpy()


def _sorted_unique_inplace(keys: np.ndarray) -> np.ndarray:
    keys.sort()
    if keys.size == 0:
        return keys
    keep = np.empty(keys.size, dtype=bool)
    keep[0] = True
    np.not_equal(keys[1:], keys[:-1], out=keep[1:])
    return keys[keep]


def rmat_csr_files(scale: int, out_dir: str, seed: int = 1, weights=(1, 16),
                   edge_factor: int = 16, log=print):
    """Writes ``off.npy`` (int64[n+1]), ``idx.npy`` (int32[nnz]) and ``w.npy`` (uint32[nnz]) of
    ``rmat(scale, edge_factor, seed=seed, weights=weights)`` to ``out_dir`` (reused if present)
    and returns (n, off, idx, w) as read-only memory maps."""
    paths = [os.path.join(out_dir, f) for f in ("off.npy", "idx.npy", "w.npy")]
    if all(os.path.exists(p) for p in paths):
        off, idx, w = (np.load(p, mmap_mode="r") for p in paths)
        return off.shape[0] - 1, off, idx, w
    os.makedirs(out_dir, exist_ok=True)
    n, u, v = rmat_edges(scale, edge_factor, seed=seed)
    log(f"lean rmat s{scale}: {u.numel()} endpoint pairs drawn")
    m = int(u.numel())
    keys = np.empty(m, dtype=np.int64)
    pos = 0
    un, vn = u.numpy(), v.numpy()
    for s in range(0, m, _CHUNK):
        a, b = un[s:s + _CHUNK], vn[s:s + _CHUNK]
        ok = a != b
        lo = np.minimum(a, b)[ok]
        hi = np.maximum(a, b)[ok]
        keys[pos:pos + lo.size] = lo * n + hi
        pos += lo.size
    del u, v, un, vn
    keys = _sorted_unique_inplace(keys[:pos].copy())
    P = keys.size
    log(f"lean rmat s{scale}: {P} distinct pairs")
    # arcs per row: as the smaller end (lo -> hi) and as the larger end (hi -> lo)
    cnt_lo = np.zeros(n, dtype=np.int64)
    cnt_hi = np.zeros(n, dtype=np.int64)
    for s in range(0, P, _CHUNK):
        k = keys[s:s + _CHUNK]
        cnt_lo += np.bincount(k // n, minlength=n)
        cnt_hi += np.bincount(k % n, minlength=n)
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt_lo + cnt_hi, out=off[1:])
    nnz = int(off[-1])
    start_lo = np.zeros(n, dtype=np.int64)
    np.cumsum(cnt_lo[:-1], out=start_lo[1:])
    start_hi = np.zeros(n, dtype=np.int64)
    np.cumsum(cnt_hi[:-1], out=start_hi[1:])
    idx = np.lib.format.open_memmap(paths[1] + ".tmp.npy", mode="w+", dtype=np.int32,
                                    shape=(nnz,))
    w = np.lib.format.open_memmap(paths[2] + ".tmp.npy", mode="w+", dtype=np.uint32,
                                  shape=(nnz,))
    wkey = stream_key(seed, _T_WEIGHT, scale)
    # second half of each row: pairs in (lo, hi) order, arc lo -> hi
    for s in range(0, P, _CHUNK):
        k = keys[s:s + _CHUNK]
        lo, hi = k // n, k % n
        j = np.arange(s, s + k.size, dtype=np.int64)
        at = off[lo] + cnt_hi[lo] + (j - start_lo[lo])
        idx[at] = hi.astype(np.int32)
        w[at] = _pair_weight_np(wkey, n, weights[0], weights[1], lo, hi).astype(np.uint32)
    log(f"lean rmat s{scale}: forward arcs written")
    # first half: pairs in (hi, lo) order, arc hi -> lo
    keys = (keys % n) * n + keys // n
    keys.sort()
    for s in range(0, P, _CHUNK):
        k = keys[s:s + _CHUNK]
        hi, lo = k // n, k % n
        j = np.arange(s, s + k.size, dtype=np.int64)
        at = off[hi] + (j - start_hi[hi])
        idx[at] = lo.astype(np.int32)
        w[at] = _pair_weight_np(wkey, n, weights[0], weights[1], lo, hi).astype(np.uint32)
    del keys
    idx.flush()
    w.flush()
    del idx, w
    np.save(paths[0], off)
    os.replace(paths[1] + ".tmp.npy", paths[1])
    os.replace(paths[2] + ".tmp.npy", paths[2])
    log(f"lean rmat s{scale}: n={n} nnz={nnz}")
    off, idx, w = (np.load(p, mmap_mode="r") for p in paths)
    return n, off, idx, w


def csr_sha256_np(n: int, off, idx, w) -> str:
    """``csr_sha256`` of numpy arrays: SHA-256 over (n, offsets as int64, indices as int32,
    weights as int64), little endian, streamed in chunks."""
    h = hashlib.sha256()
    h.update(int(n).to_bytes(8, "little"))
    h.update(np.ascontiguousarray(off, dtype=np.int64).tobytes())
    for s in range(0, idx.shape[0], _CHUNK):
        h.update(np.ascontiguousarray(idx[s:s + _CHUNK], dtype=np.int32).tobytes())
    for s in range(0, w.shape[0], _CHUNK):
        h.update(np.asarray(w[s:s + _CHUNK]).astype(np.int64).tobytes())
    return h.hexdigest()
