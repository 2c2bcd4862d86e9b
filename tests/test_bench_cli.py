"""Host-side checks of bench.py (no device): the one-GPU contract, the
refusal without a GPU, and the lookup of the committed HBM-traffic figures,
which must go null once the leaf-product kernel source changes."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=300)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU may be present")
def test_without_a_gpu_the_bench_refuses():
    r = run_bench("--steps", "1", "--warmup", "0")
    assert r.returncode == 2
    assert "needs a GPU" in r.stderr


def test_traffic_lookup_follows_the_kernel_source(tmp_path, monkeypatch):
    data = json.load(open(bench.TRAFFIC_FILE))
    kernel, workloads = next(iter(data.items()))
    workload, ent = next(iter(workloads.items()))
    got = bench.measured_traffic(kernel, workload)
    if ent["source_sha"] == bench.source_sha(bench.GEMM_SOURCE):
        assert got == ent["bytes_per_dispatch"] > 0
    else:
        assert got is None
    # Unknown entries and a changed kernel source give null.
    assert bench.measured_traffic(kernel, "no such workload") is None
    assert bench.measured_traffic("no such kernel", workload) is None
    other = tmp_path / "leafgemm.hip"
    other.write_text("// a different kernel source\n")
    monkeypatch.setattr(bench, "GEMM_SOURCE", str(other))
    assert bench.measured_traffic(kernel, workload) is None


def test_percentile():
    assert bench.percentile([], 50) is None
    assert bench.percentile([1.0, 2.0, 3.0], 50) == 2.0
    assert bench.percentile([1.0, 2.0, 3.0, 4.0], 99) == pytest.approx(3.97)
