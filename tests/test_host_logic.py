"""Host-side logic on the CPU: the benchmark's algorithmic byte counts and its
gate on committed counter profiles, the serving loop's bookkeeping (sequential
replay, latency summary) and the serving trace's recipe."""

import math
import os
import shutil

import numpy as np
import pytest

import bench
import workloads
from paper_1712_09999_amd import serving

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_kernel_bytes_of_the_iteration():
    dims, ranks, s = (64, 64, 64, 64), (6, 6, 6, 6), 8
    L = math.prod(dims)
    pb = sum(r * L // d * s for d, r in zip(dims, ranks))  # one pass over every P_n
    # no merged mode: GEMM-M reads D and Y_n for every mode
    kb = bench.kernel_bytes(dims, ranks, s, 0)
    assert kb["fused"] == 10 * L * s + pb
    assert kb["gemm_p"] == 8 * L * s + pb
    assert kb["gemm_m"] == 8 * L * s + pb
    # modes 0 and 1 merged: GEMM-M streams modes 2 and 3 and their P_n
    kb = bench.kernel_bytes(dims, ranks, s, 2)
    assert kb["gemm_m"] == 4 * L * s + pb // 2
    # every mode merged: the pass writes one I_n x R_n partial of modes 2 and 3
    # per block, and k_msum reads them and writes 64 group sums
    kb = bench.kernel_bytes(dims, ranks, s, 4, 4096)
    part = 8 * 4096 * (64 * 6 + 64 * 6)
    assert kb["fused"] == 10 * L * s + pb + part
    assert kb["gemm_m"] == part + 8 * 64 * (64 * 6 + 64 * 6)
    assert round(kb["gemm_p"] / 1e6, 1) == 1124.1
    # the last two modes' GEMM-P as one pass: one read of D fewer
    kb = bench.kernel_bytes(dims, ranks, s, 4, 4096, 1)
    assert kb["gemm_p"] == 7 * L * s + pb
    # the headline's figures (FP64): 1417.7 MB, 989.9 MB, 25.6 MB
    assert round(kb["fused"] / 1e6, 1) == 1417.7
    assert round(kb["gemm_p"] / 1e6, 1) == 989.9
    assert round(kb["gemm_m"] / 1e6, 1) == 25.6


def test_measured_traffic_needs_the_measured_source(tmp_path, monkeypatch):
    # a copy of the profile whose recorded checksum no longer matches gives
    # None, as does a missing profile; an intact copy gives the recorded bytes
    prof = tmp_path / "profiles"
    prof.mkdir()
    src = os.path.join(ROOT, "profiles", "pasd_c4_fp64_hbm_traffic.md")
    text = open(src).read()
    lines = [ln for ln in text.splitlines() if ln.strip().startswith("fused_source_sha256:")]
    assert len(lines) == 1
    (prof / "stale.md").write_text(text.replace(lines[0], "    fused_source_sha256: 00"))
    shutil.copytree(os.path.join(ROOT, "paper_1712_09999_amd"), tmp_path / "paper_1712_09999_amd",
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    monkeypatch.setattr(bench, "__file__", str(tmp_path / "bench.py"))
    assert bench._measured_traffic("fused", "stale.md") is None
    assert bench._measured_traffic("fused", "missing.md") is None
    import hashlib
    digest = hashlib.sha256(
        open(tmp_path / "paper_1712_09999_amd" / "csrc" / "kernels_elem.hip", "rb").read()).hexdigest()
    (prof / "fresh.md").write_text(text.replace(lines[0], "    fused_source_sha256: " + digest))
    rec = [ln for ln in text.splitlines() if ln.strip().startswith("fused_traffic_bytes_per_launch:")]
    assert bench._measured_traffic("fused", "fresh.md") == int(rec[0].split(":")[1])


def test_sequential_replay_queues_in_arrival_order():
    reqs = [serving.Request(0, 0.0, None, (3, 3, 3)), serving.Request(1, 0.5, None, (3, 3, 3)),
            serving.Request(2, 3.0, None, (3, 3, 3)), serving.Request(3, 0.2, None, (3, 3, 3))]
    service = {0: 1.0, 1: 1.0, 2: 0.5, 3: 0.25}
    res = {r.rid: r for r in serving.sequential_replay(reqs, service)}
    # order of service: 0 (0 -> 1), 3 (1 -> 1.25), 1 (1.25 -> 2.25), 2 (3 -> 3.5)
    assert res[0].completed == 1.0
    assert res[3].admitted == 1.0 and res[3].completed == 1.25
    assert res[1].admitted == 1.25 and res[1].completed == 2.25
    assert res[2].admitted == 3.0 and res[2].completed == 3.5
    summary = serving.latency_summary(list(res.values()))
    lat = np.array([1.0, 1.75, 0.5, 1.05])
    assert summary["count"] == 4
    assert summary["p50_ms"] == pytest.approx(np.percentile(lat, 50) * 1e3)
    assert summary["p99_ms"] == pytest.approx(np.percentile(lat, 99) * 1e3)
    assert summary["solves_per_s"] == pytest.approx(4 / 3.5)


def test_serving_trace_recipe():
    trace = workloads.serving_trace(count=512, qps=100.0)
    assert len(trace) == 512
    arrivals = [t["arrival"] for t in trace]
    assert all(b > a for a, b in zip(arrivals, arrivals[1:]))
    # Poisson arrivals at the stated rate (mean gap 1/qps within a few percent)
    assert np.mean(np.diff([0.0] + arrivals)) == pytest.approx(0.01, rel=0.1)
    for t in trace:
        d, r = t["dims"], t["ranks"]
        assert len(d) == 3 and all(32 <= x <= 256 for x in d)
        assert all(3 <= x <= 15 for x in r)
        # Tucker feasibility: r_n <= prod of the other ranks, and r_n <= I_n
        for n in range(3):
            assert r[n] <= r[(n + 1) % 3] * r[(n + 2) % 3] and r[n] <= d[n]
        assert 0.05 <= t["frac"] <= 0.20
    # seeded: the same trace twice
    assert workloads.serving_trace(count=8, qps=100.0) == trace[:8]


def test_bench_refuses_more_than_one_gpu():
    # the benchmark measures one GPU; asking for more ends at once with a
    # message and exit status 2, before anything touches a device
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "--gpus 2 is not supported" in r.stderr
    assert r.stdout == ""
