"""Host-side checks of bench.py: its byte models against the committed HBM
counters, the counter readers, and the one-GPU refusal (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("variant,nc", [("plain", 3), ("boussinesq", 4)])
def test_counters_match_byte_model(variant, nc):
    """Where the stored counters were taken with the current kernel sources,
    every pass of the step moves its kept-modes byte model within 15 % (the
    counters never undercount it: each pass must move at least its model);
    p1, run once per call, also reads the forcing band and writes the tile
    padding, within 25 %."""
    tr = bench.read_traffic(variant)
    assert tr is not None and tr["n"] == 512
    if tr["source_hash"] != bench.kernel_source_hash():
        pytest.skip("counters taken with other kernel sources (bench reports them as null)")
    alg = bench.algorithmic_bytes(512, 10, nc=nc)
    for name, measured in tr["bytes_per_launch"].items():
        tot, launches = alg[name]
        model = tot / launches
        hi = 1.25 if name == "p1" else 1.15
        assert 0.99 * model <= measured <= hi * model, (name, measured, model)


def test_unknown_traffic_variant():
    assert bench.read_traffic(None) is None
    assert bench.read_traffic("rotating") is None


def test_ensemble_byte_model_resident_runs():
    """A block-resident run moves only its state and accumulator: 3 state and
    3 accumulator reads, 3 accumulator writes and one state write per step."""
    n = 128
    K = (n - 1) // 3
    us = (2 * K + 1) * (K + 1) * 8.0
    un = n * (K + 1) * 8.0
    assert bench.ensemble_alg_bytes([n]) == 10 * us
    assert bench.ensemble_alg_bytes([n], resident=()) == 4 * (10 * un + 3 * us) + us
    assert bench.ensemble_alg_bytes([256]) == bench.ensemble_alg_bytes([256], resident=())


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
