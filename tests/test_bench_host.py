"""Host logic without a GPU: bench.py's one-GPU refusal, its graph cache format and its
rocprofv3 summaries (counter scaling by the calibration copy, per-launch bytes, the source hash
that invalidates a stale traffic figure); and the binding's checks of server requests."""

import json
import os
import subprocess
import sys

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_graph_cache_round_trip(tmp_path):
    from graphgen import rmat
    g = rmat(8, seed=3, weights=(1, 16))
    p = str(tmp_path / "g.bin")
    bench.save_graph(p, "rmat8", g)
    h = bench.load_graph(p, "rmat8", "cpu")
    assert h.n == g.n
    for a, b in ((h.offsets, g.offsets), (h.indices, g.indices), (h.weights, g.weights)):
        assert a.dtype == b.dtype and torch.equal(a, b)
    with pytest.raises(AssertionError):
        bench.load_graph(p, "rmat9", "cpu")


def test_short_name():
    assert bench._short_name("void lv::(anonymous namespace)::k_move_lds<false, unsigned int>"
                             "(lv::MoveArgs<unsigned int>)") == "void k_move_lds<false, unsigned int>"
    assert bench._short_name("lv::k_apply_moves(int const*, long)") == "k_apply_moves"


def write_csv(path, rows):
    keys = ["Kernel_Name", "Counter_Name", "Counter_Value", "Grid_Size"]
    with open(path, "w") as f:
        f.write(",".join(keys) + "\n")
        for r in rows:
            f.write(",".join(f'"{r[k]}"' for k in keys) + "\n")


def pmc_inputs(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    mv = "void lv::k_move_lds<false, unsigned int>(lv::MoveArgs<unsigned int>)"
    other = "lv::k_apply_moves(int const*, long)"
    fetch = [{"Kernel_Name": copy, "Counter_Name": "FETCH_SIZE", "Counter_Value": 524288,
              "Grid_Size": 1024},
             {"Kernel_Name": copy, "Counter_Name": "FETCH_SIZE", "Counter_Value": 7,
              "Grid_Size": 64},
             {"Kernel_Name": mv, "Counter_Name": "FETCH_SIZE", "Counter_Value": 1000,
              "Grid_Size": 4096},
             {"Kernel_Name": mv, "Counter_Name": "FETCH_SIZE", "Counter_Value": 3000,
              "Grid_Size": 4096},
             {"Kernel_Name": other, "Counter_Name": "FETCH_SIZE", "Counter_Value": 5,
              "Grid_Size": 256}]
    write = [{"Kernel_Name": copy, "Counter_Name": "WRITE_SIZE", "Counter_Value": 1048576,
              "Grid_Size": 1024},
             {"Kernel_Name": mv, "Counter_Name": "WRITE_SIZE", "Counter_Value": 10,
              "Grid_Size": 4096},
             {"Kernel_Name": mv, "Counter_Name": "WRITE_SIZE", "Counter_Value": 30,
              "Grid_Size": 4096}]
    fp, wp, bp = (str(tmp_path / n) for n in ("fetch.csv", "write.csv", "bench.json"))
    write_csv(fp, fetch)
    write_csv(wp, write)
    json.dump({"roofline": {"algorithmic_bytes_per_launch": 1.0e6}}, open(bp, "w"))
    return fp, wp, bp


def test_pmc_summary_scales_by_the_calibration_copy(tmp_path, monkeypatch):
    fp, wp, bp = pmc_inputs(tmp_path)
    out = str(tmp_path / "pmc.md")
    bench.summarize_pmc(fp, wp, bp, out, "the commands", "rmat25", 1024)
    text = open(out).read()
    d = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    # the 1 GiB copy reads 524288 KiB of FETCH_SIZE (x2) and 1048576 KiB of WRITE_SIZE (x1)
    assert d["calibration"]["fetch_scale"] == 2.0 and d["calibration"]["write_scale"] == 1.0
    assert d["launches"] == 2
    assert d["fetch_bytes_per_launch"] == 2000 * 1024 * 2.0
    assert d["write_bytes_per_launch"] == 20 * 1024 * 1.0
    assert d["bytes_per_launch"] == d["fetch_bytes_per_launch"] + d["write_bytes_per_launch"]
    assert d["kernel_src_sha256"] == bench.kernel_src_sha("k_move_lds")
    assert "the commands" in text
    # load_traffic takes the figure only for the same workload and kernel source
    monkeypatch.setitem(bench.PMC_KERNELS, "k_move_lds",
                        (bench.PMC_KERNELS["k_move_lds"][0], out))
    assert bench.load_traffic("rmat25") == d["bytes_per_launch"]
    assert bench.load_traffic("rmat22") is None
    monkeypatch.setattr(bench, "kernel_src_sha", lambda kernel="k_move_lds": "0" * 64)
    assert bench.load_traffic("rmat25") is None


def test_pmc_summary_needs_the_calibration_copy(tmp_path):
    fp, wp, bp = pmc_inputs(tmp_path)
    rows = [r for r in open(fp).read().splitlines() if "copyBuffer" not in r]
    open(fp, "w").write("\n".join(rows) + "\n")
    with pytest.raises(SystemExit, match="calibration"):
        bench.summarize_pmc(fp, wp, bp, str(tmp_path / "x.md"), "", "rmat25", 1024)


def test_stats_summary(tmp_path):
    p = str(tmp_path / "stats.csv")
    keys = ["Name", "Calls", "TotalDurationNs", "AverageNs"]
    rows = [("lv::k_apply_moves(int const*)", 4, 4.0e6, 1.0e6),
            ("void lv::k_move_lds<false, unsigned int>(lv::MoveArgs<unsigned int>)", 8, 12.0e6,
             1.5e6),
            ("at::native::vectorized_elementwise_kernel<4>", 100, 50.0e6, 0.5e6)]
    with open(p, "w") as f:
        f.write(",".join(keys) + "\n")
        for r in rows:
            f.write(",".join(f'"{x}"' for x in r) + "\n")
    out = str(tmp_path / "stats.md")
    bench.summarize_stats(p, out, "cmd", "a test")
    text = open(out).read()
    assert "Library kernels total: 16.0 ms" in text
    lines = [ln for ln in text.splitlines() if ln.startswith("| `")]
    # library kernels only, longest first, shares of the library total
    assert len(lines) == 2
    assert "k_move_lds" in lines[0] and "75.0%" in lines[0]
    assert "k_apply_moves" in lines[1] and "25.0%" in lines[1]
    assert "vectorized_elementwise" not in text


def test_server_request_checks():
    """The binding's host-side checks of a server request (no GPU needed): sizes against n,
    dtypes, devices; a good request maps onto lv_graph."""
    from paper_2301_12390_amd.louvain import request_struct
    i32, i64 = torch.int32, torch.int64
    off = torch.tensor([0, 2, 3, 4], dtype=i64)
    idx = torch.tensor([1, 2, 0, 0], dtype=i32)
    w = torch.ones(4, dtype=i32)
    g, memb = request_struct(3, off, idx, w)
    assert (g.n, g.nnz, g.offsets_64, g.weights_64) == (3, 4, 1, 0)
    assert memb.dtype == i32 and memb.numel() == 3
    g, _ = request_struct(3, off.to(i32), idx, w)
    assert g.offsets_64 == 0
    g, _ = request_struct(0, torch.zeros(1, dtype=i32), idx[:0], w[:0])
    assert g.n == 0 and g.nnz == 0
    bad = [
        (4, off, idx, w, None),                           # offsets too short for n
        (2, off, idx, w, None),                           # offsets too long for n
        (3, off, idx, w[:3], None),                       # weights shorter than indices
        (3, off, idx.to(i64), w, None),                   # 64-bit indices
        (3, off, idx, w.to(i64), None),                   # 64-bit weights
        (3, off.to(torch.float32), idx, w, None),         # float offsets
        (3, off, idx, w, torch.empty(2, dtype=i32)),      # membership too short
        (3, off, idx, w, torch.empty(3, dtype=i64)),      # membership of the wrong type
        (-1, off, idx, w, None),
        (3, off, idx[:0], w, None),                       # indices shorter than weights
        (3, off, torch.stack([idx, idx], 1)[:, 0], w, None),  # not contiguous
    ]
    for n, o, i, ww, m in bad:
        with pytest.raises(ValueError):
            request_struct(n, o, i, ww, m)
