"""Helpers shared by the GPU tests: move graphs to the device, compare GPU state with the
oracle's."""

import numpy as np
import torch

import oracle as O


def dev_graph(g, device="cuda:0"):
    return g.to(device)


def gpu_state(st: O.State, device="cuda:0"):
    """Device tensors (C, Sigma, csize, K) holding the oracle state's values."""
    C = torch.from_numpy(st.C.copy()).to(device)
    Sig = torch.from_numpy(st.Sig.view(np.int64).copy()).to(device)
    cs = torch.from_numpy(st.csize.copy()).to(device)
    K = torch.from_numpy(st.K.view(np.int64).copy()).to(device)
    return C, Sig, cs, K


def assert_state_equal(st: O.State, C, Sig, cs, ctx=""):
    Cg = C.cpu().numpy()
    Sg = Sig.cpu().numpy().view(np.uint64)
    cg = cs.cpu().numpy()
    if not np.array_equal(Cg, st.C):
        bad = np.nonzero(Cg != st.C)[0]
        raise AssertionError(f"{ctx}: C differs at {bad[:10]} (gpu {Cg[bad[:10]]}, "
                             f"oracle {st.C[bad[:10]]}), {bad.size} total")
    if not np.array_equal(Sg, st.Sig):
        bad = np.nonzero(Sg != st.Sig)[0]
        raise AssertionError(f"{ctx}: Sigma differs at {bad[:10]}")
    if not np.array_equal(cg, st.csize):
        bad = np.nonzero(cg != st.csize)[0]
        raise AssertionError(f"{ctx}: csize differs at {bad[:10]}")


def canonical_rows(n, off, idx, w):
    """Rows sorted by neighbour id: (off int64, idx int32, w uint64) numpy arrays."""
    off = np.asarray(off, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int32).copy()
    w = np.asarray(w).astype(np.int64).view(np.uint64).copy()
    for r in range(n):
        a, b = off[r], off[r + 1]
        o = np.argsort(idx[a:b], kind="stable")
        idx[a:b] = idx[a:b][o]
        w[a:b] = w[a:b][o]
    return off, idx, w


def canonical_rows_fast(n, off, idx, w):
    """Vectorised row sort: order arcs by (row, neighbour)."""
    off = np.asarray(off, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    w = np.asarray(w).astype(np.int64).view(np.uint64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
    o = np.lexsort((idx, rows))
    return off, idx[o].astype(np.int32), w[o]
