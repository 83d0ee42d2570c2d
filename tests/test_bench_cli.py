"""bench.py's command line on the host: it runs on one GPU only and says so
when asked for more, before touching a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_record_matches_workload_variant_and_batches():
    """The committed counter record is for the current kernel source and holds
    one entry per launch shape it was measured in (the benchmark's variants,
    one batch and four concurrent batches); nothing is reported for a shape
    or variant it does not hold.  Measured bytes lie between the least a
    launch must move (one read and one write of its populations) and 1.3
    times that."""
    b = _bench_module()
    cases = [("laplace_sweep", "twostep-58x32", 1, 72 * 24 * 256 * 256),
             ("laplace_sweep", "twostep-58x32", 4, 72 * 6 * 256 * 256),
             ("collapse_large", "twostep-58x24", 1, 72 * 8192 * 4096)]
    for wl, v, nb, model in cases:
        e = b.measured_traffic(wl, v, nb)
        assert e is not None, (wl, v, nb)
        assert e["min_hbm_bytes_per_launch"] == model
        assert model <= e["bytes_per_launch"] < 1.3 * model
    assert b.measured_traffic("laplace_sweep", "twostep-58x32", 2) is None
    assert b.measured_traffic("laplace_sweep", "fused2-128x16", 1) is None
    assert b.measured_traffic("single_small", "twostep-58x32", 1) is None


def test_timing_parts_cover_the_steps_in_whole_graphs():
    """The timed parts add up to exactly the timed steps, none longer than one
    captured graph (256 steps), and none depends on the warm-up length."""
    b = _bench_module()
    for steps in (1280, 20, 1, 255, 256, 257, 1000):
        parts = b.timing_parts(steps)
        assert sum(parts) == steps
        assert all(0 < n <= 256 for n in parts)
        assert all(n == 256 for n in parts[:-1])
