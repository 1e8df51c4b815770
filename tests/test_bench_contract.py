"""Host-side checks of bench.py: the single-GPU contract and the bookkeeping
behind its roofline object (no GPU needed)."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


def test_traffic_figure_is_reported_only_for_the_sources_it_was_counted_on(tmp_path, monkeypatch):
    """roofline.traffic is the HBM byte count taken on the dominant kernel's
    sources with the recorded hash, at the recorded schedule; once either
    differs, bench.py reports null rather than a stale figure.  When reported,
    it is at least the algorithmic bytes of a launch at that schedule (11
    items per node of 1e5 paths, 4096 nodes, each (160 x 8 + 48) B)."""
    b = _bench()
    sched = dict(b.TRAFFIC_SCHEDULE)
    t = b.traffic_bytes(sched)
    assert t is None or t >= 4096 * 11 * (160 * 8 + 48)
    other = dict(sched, chunk_paths=16384)
    assert b.traffic_bytes(other) is None
    monkeypatch.setattr(b, "TRAFFIC_SHA256", "0" * 64)
    assert b.traffic_bytes(sched) is None


def test_op_table_and_peak():
    b = _bench()
    assert b.OPS_PER_PS_FWD == 120.0 and b.OPS_PER_PS_ADJ == 180.0
    # 256 CUs x 128 FP32 lanes x 2.4 GHz: half the published 157.3 TFLOP/s (FMA = 2 flops)
    assert abs(b.PEAK_LANE_OPS * 2 - 157.3e12) / 157.3e12 < 1e-3
