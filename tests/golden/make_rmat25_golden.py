"""Writes ``rmat25_run.json``: the oracle's whole Louvain runs on the R-MAT scale-25 benchmark
graph, for the full-size GPU parity test.

Calls only the oracle (``oracle/``) and the seeded generators (``graphgen/``). The graph is
built on the host with ``graphgen.lean`` (identical to ``config_graph("rmat25")``; its SHA-256
is stored so that the GPU test can confirm it ran on the same input). Stored:
* the synchronous class-step run (8 classes, tolerance 10^-2 declining x10 per pass, 20
  iterations, 10 passes): SHA-256 of the membership (int32, little endian), its Qnum, every
  pass's Qnum, vertex and arc counts, iterations, and every iteration's S, moves and candidate
  pairs;
* the sequential asynchronous run (the quality reference): Qnum, Q, passes, iterations, every
  pass's Qnum;
* Qnum of the singleton partition (the modularity before pass 0).

Needs about 45 GB of host memory and 20-40 minutes on 8 cores. Run from the repository root:
    python tests/golden/make_rmat25_golden.py [--cache DIR]
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from graphgen.lean import csr_sha256_np, rmat_csr_files  # noqa: E402

OUT = os.path.join(HERE, "rmat25_run.json")


def log(*a):
    print(time.strftime("%H:%M:%S"), *a, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cache", default="/tmp/lv_rmat25", help="directory for the graph's files")
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()
    n, off, idx, w = rmat_csr_files(25, args.cache, seed=1, weights=(1, 16), log=log)
    sha = csr_sha256_np(n, off, idx, w)
    log(f"graph n={n} nnz={idx.shape[0]} sha256={sha}")
    g = O.Graph(n, np.asarray(off), idx, np.asarray(w).astype(np.uint64))
    del w
    q0, W, _ = O.modularity(g, np.arange(n, dtype=np.int32))
    log(f"W={W}, singleton Qnum={q0}")
    t = time.time()
    top, rs = O.run(g, "sync", substeps=8)
    t_sync = time.time() - t
    msha = hashlib.sha256(np.ascontiguousarray(top, dtype="<i4").tobytes()).hexdigest()
    log(f"sync K=8: {t_sync:.0f}s Q={rs['q']:.6f} iterations={rs['iterations']}")
    del top
    t = time.time()
    _, ra = O.run(g, "async")
    t_async = time.time() - t
    log(f"async: {t_async:.0f}s Q={ra['q']:.6f} iterations={ra['iterations']}")
    out = {
        "graph": {"name": "rmat25", "n": n, "nnz": int(g.nnz), "W": W, "csr_sha256": sha},
        "params": {"tolerance_exp10": 2, "decline_exp10": 1, "max_iterations": 20,
                   "max_passes": 10, "substeps": 8},
        "singleton_qnum": q0,
        "sync": {
            "membership_sha256": msha,
            "qnum": rs["qnum"], "q": rs["q"], "passes": rs["passes"],
            "iterations": rs["iterations"], "cap_hits": rs["cap_hits"],
            "n_pass": rs["n_pass"], "nnz_pass": rs["nnz_pass"], "qnum_pass": rs["qnum_pass"],
            "n_communities": rs["n_communities"],
            "trace_pass": rs["trace_pass"], "trace_S": rs["trace_S"],
            "trace_moved": rs["trace_moved"], "trace_ncand": rs["trace_ncand"],
            "seconds": round(t_sync, 1),
        },
        "async": {
            "qnum": ra["qnum"], "q": ra["q"], "passes": ra["passes"],
            "iterations": ra["iterations"], "qnum_pass": ra["qnum_pass"],
            "n_communities": ra["n_communities"], "seconds_one_core": round(t_async, 1),
        },
        "host": {"threads_sync": os.cpu_count()},
    }
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    log(f"wrote {args.out}")


if __name__ == "__main__":
    main()
