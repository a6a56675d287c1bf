"""CPU checks of bench.py's contract pieces: the one-GPU guard, the byte
model of Section 3.2 that prices the roofline, and the sampled-row picker
(no GPU is touched)."""
import json
import os
import subprocess
import sys

import numpy as np

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_model_bytes_is_the_paper_formula():
    # A: 2 bytes per non-empty row header (SCSR) and per entry, 8 per tile;
    # X: the distinct columns each tile touches, k values each; Y written once
    m = bench.model_bytes(T=10, R=100, C=300, nnz=1000, n=64, k=4)
    assert m["A"] == 2 * 100 + 2 * 1000 + 8 * 10
    assert m["X"] == 300 * 4 * 4 and m["Y"] == 64 * 4 * 4
    assert m["total"] == m["A"] + m["X"] + m["Y"]
    assert m["floor"] == m["A"] + 64 * 4 * 4 + m["Y"]
    # for a binary matrix the A term is the SCSR size (no value bytes) plus
    # the tile headers
    assert m["A"] == oracle.scsr_bytes(100, 1000, 0) + 8 * 10


def test_sample_rows_cover_hubs_and_spread_blocks():
    n = 1 << 16
    rp = np.arange(0, 8 * n + 1, 8, dtype=np.int64)          # degree 8 everywhere
    sel = bench.sample_rows(rp, n, 200_000)
    assert np.all(np.diff(sel) > 0) and sel[0] == 0 and sel[-1] < n
    assert set(range(64)) <= set(sel.tolist())
    nnz = int(np.diff(rp)[sel].sum())
    assert 0.5 * 200_000 <= nnz - 64 * 8 <= 2 * 200_000
    # blocks spread over the whole range
    assert sel[-1] > 0.9 * n


def test_traffic_reported_only_for_the_profiled_kernel(monkeypatch):
    """The committed counter summary prices the dominant launch only while
    it was taken on this kernel source and column chunk."""
    recorded = {}
    for line in open(bench.TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            a, b = line.split("=", 1)
            recorded[a.strip()] = b.strip()
    got = bench.measured_traffic(int(recorded["kc"]))
    if recorded["kernel_source_sha256_16"] == bench.kernel_source_hash():
        assert got == int(recorded["hbm_bytes_per_launch"])
    else:
        assert got is None
    assert bench.measured_traffic(int(recorded["kc"]) // 2) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic(int(recorded["kc"])) is None
