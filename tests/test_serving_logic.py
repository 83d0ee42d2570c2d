"""Scheduling logic of the continuous-batching server, on the CPU with a
counting backend and a simulated clock (no device, no physics)."""
import pytest

from paper_1605_01800_amd import inputs
from paper_1605_01800_amd.serving import Request, Server, make_requests, percentile


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class CountingBackend:
    """Steps nothing; advances the fake clock by sites * steps / rate and
    records what the server asked for."""

    def __init__(self, clock, rate=1e9, bytes_per_site=76):
        self.clock = clock
        self.rate = rate
        self.bps = bytes_per_site
        self.attached = []
        self.resident = 0
        self.max_resident = 0
        self.steps_done = {}
        self.order = []

    def footprint(self, r):
        return r.sites * self.bps

    def prepare(self, r):
        self.order.append(r.id)
        return {"req": r}

    def attach(self, h):
        self.attached.append(h)
        self.resident += self.footprint(h["req"])
        self.max_resident = max(self.max_resident, self.resident)

    def step(self, handles, counts):
        assert [h["req"].id for h in handles] == [h["req"].id for h in self.attached]
        for h, c in zip(handles, counts):
            assert c > 0
            self.steps_done[h["req"].id] = self.steps_done.get(h["req"].id, 0) + c
            self.clock.t += c * h["req"].sites / self.rate

    def sync(self):
        pass

    def failed(self, h):
        return False

    def finish(self, h):
        self.attached.remove(h)
        self.resident -= self.footprint(h["req"])
        return {"step": self.steps_done[h["req"].id]}, None


def _trace(n, rate, seed=0, steps=(5000, 40000)):
    tr = inputs.request_trace(n, seed, steps_lo=steps[0], steps_hi=steps[1])
    arr = inputs.poisson_arrivals(n, rate, seed + 1)
    return make_requests(tr, arr)


def test_every_request_completes_with_its_step_count():
    clock = FakeClock()
    be = CountingBackend(clock)
    reqs = _trace(60, rate=5.0)
    srv = Server(be, budget_bytes=10 ** 10, chunk_steps=500, clock=clock, sleep=clock.sleep)
    results, stats = srv.run(reqs)
    assert len(results) == 60
    for r, q in zip(results, sorted(reqs, key=lambda q: q.id)):
        assert r.id == q.id and r.diag["step"] == q.steps
        assert r.finish >= r.first_chunk >= r.admit >= r.arrival
    assert stats["p50_s"] <= stats["p99_s"]
    assert stats["site_updates"] == sum(q.sites * q.steps for q in reqs)


@pytest.mark.parametrize("budget_mb", [60, 200])
def test_resident_footprint_never_exceeds_the_budget(budget_mb):
    clock = FakeClock()
    be = CountingBackend(clock)
    reqs = _trace(80, rate=50.0, seed=3)
    budget = budget_mb * 10 ** 6
    srv = Server(be, budget_bytes=budget, chunk_steps=400, clock=clock, sleep=clock.sleep)
    results, stats = srv.run(reqs)
    assert len(results) == 80
    assert be.max_resident <= budget
    assert stats["peak_resident_bytes"] <= budget


def test_admission_is_fifo_and_slots_are_bounded():
    clock = FakeClock()
    be = CountingBackend(clock)
    reqs = _trace(40, rate=100.0, seed=5)
    srv = Server(be, budget_bytes=10 ** 12, max_slots=4, chunk_steps=300, clock=clock, sleep=clock.sleep)
    srv.run(reqs)
    assert be.order == [q.id for q in sorted(reqs, key=lambda q: (q.arrival, q.id))]
    assert srv.peak_slots <= 4


def test_oversized_request_is_rejected():
    clock = FakeClock()
    be = CountingBackend(clock)
    big = Request(id=0, nx=1024, ny=1024, walls=False, T_over_Tc=0.7, steps=10, bubbles=[])
    with pytest.raises(ValueError):
        Server(be, budget_bytes=1000, clock=clock, sleep=clock.sleep).run([big])


def test_idle_server_waits_for_the_next_arrival():
    clock = FakeClock()
    be = CountingBackend(clock, rate=1e12)
    reqs = [Request(id=k, nx=64, ny=64, walls=False, T_over_Tc=0.7, steps=100, bubbles=[],
                    arrival=10.0 * k) for k in range(3)]
    results, _ = Server(be, budget_bytes=10 ** 9, clock=clock, sleep=clock.sleep).run(reqs)
    for k, r in enumerate(results):
        assert r.admit >= 10.0 * k
        assert r.latency < 1.0


def test_percentile_nearest_rank():
    assert percentile([5, 1, 3, 2, 4], 50) == 3
    assert percentile(list(range(1, 101)), 99) == 99
    assert percentile([7], 99) == 7


def test_request_trace_matches_the_served_workload():
    tr = inputs.request_trace(512, 0)
    assert len(tr) == 512
    for t in tr:
        assert 64 <= min(t["nx"], t["ny"]) and max(t["nx"], t["ny"]) <= 1024 + 1
        assert 5000 <= t["steps"] <= 40000
        assert 0.6 <= t["T_over_Tc"] <= 0.9
        if t["walls"]:
            assert 0.005 <= t["delta"] <= 0.03
    frac = sum(t["walls"] for t in tr) / 512
    assert 0.4 < frac < 0.6


class FailingBackend(CountingBackend):
    """Marks the requests in `bad` as non-finite once they have been stepped."""

    def __init__(self, clock, bad):
        super().__init__(clock)
        self.bad = set(bad)

    def failed(self, h):
        return h["req"].id in self.bad and self.steps_done.get(h["req"].id, 0) > 0


def test_failed_requests_are_retired_after_their_first_chunk():
    clock = FakeClock()
    be = FailingBackend(clock, bad={3, 7})
    reqs = _trace(20, rate=5.0)
    srv = Server(be, budget_bytes=10 ** 10, chunk_steps=500, clock=clock, sleep=clock.sleep)
    results, stats = srv.run(reqs)
    assert len(results) == 20 and stats["failed"] == 2
    for r, q in zip(results, sorted(reqs, key=lambda q: q.id)):
        if q.id in (3, 7):
            assert r.failed and r.diag["step"] == 500 < q.steps
        else:
            assert not r.failed and r.diag["step"] == q.steps
    assert stats["site_updates"] == sum(q.sites * (500 if q.id in (3, 7) else q.steps) for q in reqs)
    assert be.resident == 0


def test_served_autotune_candidates_accept_any_width():
    """The served autotuner only weighs variants that take odd grid widths, so
    a pick made on a sample of even widths cannot refuse a later request."""
    from paper_1605_01800_amd.serving import served_variants
    names = ["2pass-64x4", "fused-64x16", "fused2-128x16", "fused2-128x32", "fused-64x32"]
    assert served_variants(names) == [0, 1, 4]
    L = pytest.importorskip("paper_1605_01800_amd.lbm")
    all_names = L.variant_names()
    picks = served_variants(all_names)
    assert picks and all(not all_names[i].startswith("fused2") for i in picks)
