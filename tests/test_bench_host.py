"""Host-side pieces of bench.py (no GPU): the one-GPU refusal, the
algorithmic byte model of a dense sweep, the traffic summary's validity
check, and the rank-accuracy report."""

import hashlib
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr)


def test_dense_sweep_bytes():
    # offsets 4(n+1) + indices 4m + out-degrees 4n + x read/write 8nS + FP64 scores 16nS
    n, m = 1 << 20, 17271734
    assert bench.dense_sweep_bytes(n, m) == 4 * (n + 1) + 4 * m + 4 * n + 8 * n + 16 * n
    assert bench.dense_sweep_bytes(10, 100, S=4) == 44 + 400 + 40 + 320 + 640


def test_traffic_summary_checks_the_kernel_source(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel source")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    summ = tmp_path / "t.md"
    summ.write_text(f"- kernel_source_sha256: `{sha}`\n- algorithmic_bytes_per_sweep: `1000`\n"
                    f"- hbm_bytes_per_sweep: `1500`\n")
    monkeypatch.setattr(bench, "SWEEP_SOURCE", str(src))
    assert bench.measured_traffic(1000, str(summ)) == 1500.0
    # the same workload, a few edges apart
    assert bench.measured_traffic(1000.5, str(summ)) == 1500.0 * 1000.5 / 1000
    assert bench.measured_traffic(2000, str(summ)) is None  # another workload
    assert bench.measured_traffic(1000, str(tmp_path / "missing.md")) is None
    src.write_text("changed kernel source")
    assert bench.measured_traffic(1000, str(summ)) is None  # the counters no longer describe the kernel


def test_host_cpu_model_is_named():
    name = bench.host_cpu_model()
    assert isinstance(name, str) and name


def test_rank_accuracy_report():
    from paper_1712_00595_amd import accuracy

    ref = np.linspace(1.0, 0.0, 2000)
    out = bench.rank_accuracy(accuracy, ref + 1e-12, ref)
    assert set(out) == {"spearman", "top10_overlap", "top100_overlap", "top1000_overlap"}
    assert out["spearman"] > 0.999999 and out["top1000_overlap"] == 1.0
