"""Host-side parts of the benchmark contract: more than one GPU is refused with a message, and the
profile-derived constants (row-sweep HBM bytes, executed flops) are reported only while the kernel
sources and build flags they were measured with are unchanged."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_profile_constants_are_reported_only_for_their_sources():
    # measured bytes are reported for the workload and sources they were measured on, else null
    sys.path.insert(0, ROOT)
    import bench
    match = bench._sources_match(bench.ROW_SWEEP_TRAFFIC["sources"])
    t = bench._row_sweep_traffic("z3_16x16_d6")
    assert (t is not None and t > 0) if match else t is None
    assert bench._row_sweep_traffic("z2_16x16_d4") is None
    ex = bench._row_sweep_executed("z3_16x16_d6", 30.0)
    assert (ex is not None) == bench._sources_match(bench.ROW_SWEEP_EXECUTED["sources"])
