"""Host-side pieces of bench.py that need no GPU: the refusal of more than
one GPU, the ALU peak, the operation model the ALU roofline divides by, and
the lookup of committed HBM counters keyed by the kernel source's hash."""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2506_14781_amd import tdpt as T  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_alu_peak_is_the_published_vector_rate():
    # 157.3 TFLOP/s fp32 with a fused multiply-add counted as 2 operations
    assert bench.PEAK_LANE_OPS == 256 * 128 * 2.4e9
    assert abs(bench.PEAK_LANE_OPS - 157.3e12 / 2) / bench.PEAK_LANE_OPS < 1e-3


def test_operation_model_of_the_workloads():
    """Per update: one multiply-add per problem neighbour, the copy term (4),
    the bias (1), a quarter Philox4x32-10 (25), the decision (6) and the
    cheaper f/g bookkeeping: d + 15 + 32 + min(4, (d + 3) / mcs)."""
    from synth.configs import wishart_n1000, wishart_n200
    for w, mcs in ((wishart_n1000(), 50), (wishart_n200(), 1)):
        info = T.Instance.from_synth(w.instance).info()
        d = info["nnz"] / info["n"]
        want = d + 4 + 1 + 25 + 6 + min(4.0, (d + 3) / mcs)
        assert bench.alu_ops_per_update(info, mcs=mcs) == pytest.approx(want)
    assert bench.alu_ops_per_update(T.Instance.from_synth(wishart_n1000().instance).info(),
                                    mcs=50) == pytest.approx(40.12, abs=0.01)


def test_measured_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    key = "wishart-N1000-D6-64x32"
    m = bench.MEASURED_TRAFFIC[key]
    with open(bench.KERNEL_SRC, "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()[:16]
    current = m["kernel_sha256"] == digest  # counters taken on this kernel source
    assert bench.measured_traffic(key, m["kernel"], 4) == (4 * m["bytes_per_round"] if current else None)
    assert bench.measured_traffic(key, "k_persistent", 4) is None
    assert bench.measured_traffic("no-such-workload", m["kernel"], 4) is None
    changed = tmp_path / "kernels.hip"
    changed.write_bytes(open(bench.KERNEL_SRC, "rb").read() + b"\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(changed))
    assert bench.measured_traffic(key, m["kernel"], 4) is None
