"""The C-ABI library loads without a GPU, exports every function include/louvain.h declares, and
the Python binding's structures have the C layout (checked against a gcc-compiled probe of the
header). No compute call is made."""

import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "louvain.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(louvain_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2301_12390_amd import build as B
    if B.needs_build():
        B.build()
    from paper_2301_12390_amd.louvain import load_library
    return load_library()


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) == 22, names
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_header():
    from paper_2301_12390_amd.louvain import SIGNATURES
    assert sorted(SIGNATURES) == header_functions()


def test_missing_library_fails_loudly(tmp_path):
    from paper_2301_12390_amd import louvain as L
    saved = L._LIB
    L._LIB = None
    try:
        with pytest.raises(ImportError, match="missing"):
            L.load_library(str(tmp_path / "nope.so"))
    finally:
        L._LIB = saved


PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "louvain.h"
#define F(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
#define S(T) printf(#T " %zu\n", sizeof(T));
int main(void) {
  S(lv_graph) F(lv_graph, nnz) F(lv_graph, offsets) F(lv_graph, indices) F(lv_graph, weights)
  F(lv_graph, offsets_64) F(lv_graph, weights_64)
  S(lv_params) F(lv_params, flags)
  S(lv_iter_trace) F(lv_iter_trace, wg_launches) F(lv_iter_trace, gain_sum)
  F(lv_iter_trace, fused_candidates) F(lv_iter_trace, hub_arcs) F(lv_iter_trace, fused_ms)
  F(lv_iter_trace, iter_ms)
  S(lv_result) F(lv_result, iterations) F(lv_result, n_pass) F(lv_result, qnum_pass)
  F(lv_result, cap_hits) F(lv_result, n_communities) F(lv_result, W) F(lv_result, q_num)
  F(lv_result, q) F(lv_result, total_ms) F(lv_result, aggregate_ms) F(lv_result, trace)
  S(lv_move_stats) F(lv_move_stats, moved) F(lv_move_stats, gain_sum)
  F(lv_move_stats, last_candidates)
  S(lv_graph_result) F(lv_graph_result, iterations) F(lv_graph_result, cap_hits)
  F(lv_graph_result, n_communities) F(lv_graph_result, W) F(lv_graph_result, q_num)
  F(lv_graph_result, q)
  S(lv_prep_stats) F(lv_prep_stats, nnz) F(lv_prep_stats, sort_passes)
  F(lv_prep_stats, scatter_ms) F(lv_prep_stats, total_ms)
  S(lv_server_config) F(lv_server_config, hbm_budget_bytes) F(lv_server_config, batch_arcs)
  F(lv_server_config, fail_run) F(lv_server_config, params)
  S(lv_request_result) F(lv_request_result, batch_arcs) F(lv_request_result, done_ns)
  F(lv_request_result, result) F(lv_request_result, error)
  S(lv_server_stats) F(lv_server_stats, slots) F(lv_server_stats, bound_misses)
  F(lv_server_stats, peak_held_bytes)
  return 0;
}
"""


def test_struct_layout_matches_header():
    from paper_2301_12390_amd import louvain as L
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(src, "w").write(PROBE)
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), src,
                               "-o", exe])
        out = subprocess.check_output([exe]).decode().split("\n")
    cmap = {"lv_graph": L.LvGraph, "lv_params": L.LvParams, "lv_iter_trace": L.LvIterTrace,
            "lv_result": L.LvResult, "lv_move_stats": L.LvMoveStats,
            "lv_graph_result": L.LvGraphResult, "lv_prep_stats": L.LvPrepStats,
            "lv_server_config": L.LvServerConfig, "lv_request_result": L.LvRequestResult,
            "lv_server_stats": L.LvServerStats}
    checked = 0
    for line in out:
        if not line:
            continue
        key, val = line.split()
        val = int(val)
        if "." in key:
            t, f = key.split(".")
            assert getattr(cmap[t], f).offset == val, key
        else:
            assert ctypes.sizeof(cmap[key]) == val, key
        checked += 1
    assert checked > 20
