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
    one batch and four concurrent batches, with the stores the benchmark picks
    for each); nothing is reported for a shape, variant or store kind it does
    not hold.  Measured bytes lie between the least a
    launch must move (one read and one write of its populations) and 1.3
    times that."""
    b = _bench_module()
    cases = [("laplace_sweep", "twostep-58x32", 1, True, 72 * 24 * 256 * 256),
             ("laplace_sweep", "twostep-58x32", 4, True, 72 * 6 * 256 * 256),
             ("collapse_large", "twostep-58x24", 1, False, 72 * 8192 * 4096)]
    for wl, v, nb, wt, model in cases:
        e = b.measured_traffic(wl, v, nb, wt)
        assert e is not None, (wl, v, nb, wt)
        assert e["min_hbm_bytes_per_launch"] == model
        assert model <= e["bytes_per_launch"] < 1.3 * model
    for wl, v, nb, wt, sites in (("laplace_sweep", "twostep-58x32", 1, True, 24 * 256 * 256),
                                 ("collapse_large", "twostep-58x24", 1, False, 8192 * 4096)):
        r = b.valu_roofline(b.measured_traffic(wl, v, nb, wt), 1.0, 2 * sites)
        assert r is not None and r["bound"] == "alu" and 150 < r["lane_slots_per_site_update"] < 600
    assert b.valu_roofline(None, 1.0, 1) is None
    assert b.measured_traffic("laplace_sweep", "twostep-58x32", 2, True) is None
    assert b.measured_traffic("laplace_sweep", "twostep-58x32", 4, False) is None
    assert b.measured_traffic("laplace_sweep", "fused2-128x16", 1, False) is None
    assert b.measured_traffic("single_small", "twostep-58x32", 1, False) is None


def test_timing_parts_cover_the_steps_in_whole_graphs():
    """The timed parts add up to exactly the timed steps, none longer than one
    captured graph (256 steps), and none depends on the warm-up length."""
    b = _bench_module()
    for steps in (1280, 20, 1, 255, 256, 257, 1000):
        parts = b.timing_parts(steps)
        assert sum(parts) == steps
        assert all(0 < n <= 256 for n in parts)
        assert all(n == 256 for n in parts[:-1])


class _Stream:
    """A stream of a simulated device: `t` is the time (us) its work reaches."""

    def __init__(self, us_per_step):
        self.t = 0.0
        self.us_per_step = us_per_step

    def wait_event(self, ev):
        self.t = max(self.t, ev.ts) + 2.0          # a cross-stream wait costs 2 us


class _Event:
    def __init__(self, enable_timing=False):
        self.timing = enable_timing
        self.ts = None

    def record(self, stream):
        self.ts = stream.t

    def elapsed_time(self, other):
        assert self.timing and other.timing, "a timed interval needs timing events"
        return (other.ts - self.ts) / 1000.0


class _Cuda:
    Event = _Event

    @staticmethod
    def synchronize():
        pass


class _Torch:
    cuda = _Cuda


class _Clock:
    """lbm_device_clock / lbm_hold_until on the simulated device (1 MHz, so a
    tick is a microsecond); the host reads the clock at 100 us."""
    rate = 1000000

    def device_clock(self):
        return 100, self.rate

    def hold_until(self, tick, max_ticks, stream):
        assert max_ticks <= self.rate
        stream.t = max(stream.t, float(tick))


class _Runner:
    def __init__(self, streams):
        self.streams = streams

    def step(self, n):
        for st in self.streams:
            st.t += n * st.us_per_step

    def prepare(self, n):
        pass

    def sync(self):
        pass


def test_timed_region_brackets_every_stream_and_its_parts_add_up():
    """On a simulated device whose four streams take 1.0, 1.2, 0.9 and 1.0 us
    a step: every stream starts at the common hold, the streams are aligned
    (with untimed events) before each later part, and the region runs from
    the hold's end to the slowest stream's end: the steps of the slowest
    stream plus the waits of the alignments, no more.  One stream alone is
    timed the same way."""
    b = _bench_module()
    for per_step, steps in (([1.0, 1.2, 0.9, 1.0], 600), ([1.0, 1.2, 0.9, 1.0], 20), ([1.5], 600)):
        streams = [_Stream(u) for u in per_step]
        ms, median, nparts = b.timed_region(_Torch, _Clock(), _Runner(streams), streams, steps, 5)
        parts = b.timing_parts(steps)
        assert nparts == len(parts)
        hold_end = 100 + 1000.0 * max(1.0, 0.5 * len(streams))
        # the region is exactly the span from the hold's end to the last stream's end
        assert abs(ms * 1000.0 - (max(st.t for st in streams) - hold_end)) < 1e-6
        slow = sum(n * max(per_step) for n in parts)
        # a join (one wait per other stream) and a fork (one wait) at each later part
        align = (len(streams) - 1 + 1) * 2.0 * (len(parts) - 1) if len(streams) > 1 else 0.0
        assert slow - 1e-6 <= ms * 1000.0 <= slow + align + 1e-6, (ms, slow, align)
        assert max(per_step) - 1e-9 <= median * 1000.0 <= max(per_step) + align / min(parts) + 1e-9
