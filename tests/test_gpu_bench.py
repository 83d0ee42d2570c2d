"""bench.py's timed region measures the kernels, also at a short run.

The region times steps replayed from graphs prepared during the warm-up
(lbm_batch_prepare), behind holds that release every stream at one instant of
the device clock once the host has enqueued the whole region.  At 20 timed
steps after 5 warm-up steps its time per step must then be that of a long run
(no per-part transfer, host gap or cross-stream wait inside), on one stream
(the roofline launch) and on four concurrent streams (the `value`).  Preparing
changes neither results nor state.
"""
import importlib.util
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_1605_01800_amd.lbm")
from paper_1605_01800_amd import studies  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _one_batch(sims):
    b = L.Batch(precision="fp32", max_instances=len(sims),
                max_tiles=sum(L.tile_count(s.params) for s in sims))
    for s in sims:
        b.attach(s)
    b.set_variant(L.variant_names().index("twostep-58x32"))
    return b


def test_short_region_times_the_kernel_on_one_stream():
    print("case bench one stream", flush=True)
    bench = _bench()
    sims = studies.laplace_sweep_sims(L, "fp32", "cuda:0")
    b = _one_batch(sims)
    short = min(bench.timed_region(torch, L, b, [b.stream], 20, 5)[0] / 20 for _ in range(3))
    long_ = bench.timed_region(torch, L, b, [b.stream], 768, 64)[0] / 768
    _, ms_pair = b.step_timed(40)
    pair = ms_pair / 40
    print("ms/step: 20 steps %.4f, 768 steps %.4f, event pair per launch %.4f" % (short, long_, pair),
          flush=True)
    assert short < 1.10 * long_
    # an event pair around one launch also holds its dispatch: never shorter
    assert short < 1.05 * pair
    b.close()
    for s in sims:
        s.close()


def test_short_region_times_the_kernels_on_four_streams():
    print("case bench four streams", flush=True)
    bench = _bench()
    sims = studies.laplace_sweep_sims(L, "fp32", "cuda:0")
    g = L.BatchGroup(sims, precision="fp32", n_batches=4)
    g.set_variant(L.variant_names().index("twostep-58x32"))
    short = min(bench.timed_region(torch, L, g, g.streams, 20, 5)[0] / 20 for _ in range(3))
    long_ = bench.timed_region(torch, L, g, g.streams, 768, 64)[0] / 768
    print("ms/step: 20 steps %.4f, 768 steps %.4f" % (short, long_), flush=True)
    assert short < 1.15 * long_
    g.close()
    for s in sims:
        s.close()


def test_prepare_changes_neither_results_nor_state():
    """Two copies of the sweep's first six instances step 300 + 37 steps, one
    with lbm_batch_prepare before each call (and a prepare of another count
    that is never run in between), one without: bitwise the same populations
    and step counts."""
    print("case prepare", flush=True)
    out = []
    for prepared in (False, True):
        sims = studies.laplace_sweep_sims(L, "fp32", "cuda:0")[:6]
        b = _one_batch(sims)
        for n in (300, 37):
            if prepared:
                b.prepare(n + 5)
                b.prepare(n)
            b.step(n)
        b.sync()
        out.append(([s.populations().cpu().numpy() for s in sims], [s.diag()["step"] for s in sims]))
        b.close()
        for s in sims:
            s.close()
    (fa, sa), (fb, sb) = out
    assert sa == sb == [337] * 6
    for a, c in zip(fa, fb):
        assert np.array_equal(a, c)


def test_holds_release_their_streams_together():
    """lbm_hold_until on four streams with one target: each stream's next
    event comes at the target (within 50 us of each other), not before it,
    although the holds were enqueued one after another; a hold longer than a
    second is refused."""
    print("case hold", flush=True)
    streams = [torch.cuda.Stream() for _ in range(4)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in streams]
    ref = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    tick, rate = L.device_clock()
    assert rate > 0
    ref.record(streams[0])
    until = tick + int(20e-3 * rate)          # far beyond the host's enqueueing
    for st in streams:
        L.hold_until(until, rate // 2, st)
    for e, st in zip(ev, streams):
        e.record(st)
    torch.cuda.synchronize()
    t = [ref.elapsed_time(e) for e in ev]
    print("release after the first event (ms):", ["%.4f" % v for v in t], flush=True)
    assert max(t) - min(t) < 0.05
    assert min(t) > 10.0
    with pytest.raises(L.LbmError):
        L.hold_until(until, 2 * rate, streams[0])
