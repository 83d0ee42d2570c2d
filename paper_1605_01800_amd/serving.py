"""Continuous-batching server for independent lattice Boltzmann runs.

Requests (a grid, a temperature, an initial state of Eq. 16 and a step count)
arrive over time.  The server keeps every admitted request's populations
resident in HBM and steps all of them together, one launch per step over the
tiles of every resident instance (lbm.Batch).  Work proceeds in chunks of
`chunk_steps` steps; at each chunk boundary finished requests are retired and
newly arrived ones admitted, as long as the resident footprint stays within
the HBM budget and a slot is free.  New requests are initialised on their own
streams while the current chunk runs, so admission overlaps device work.  A
request's result is bitwise the same alone and in any mix (the batch kernels
compute each instance independently).

The control loop only schedules; all stepping goes through the backend (the
GPU backend below drives liblbm; tests can substitute a counting backend).
A request whose state turns non-finite (psi^2 < 0 or an overflow, latched on
the device) is retired at the end of the chunk in which it is seen, marked
failed; the others continue unaffected.
"""
import json
import math
import time
from dataclasses import dataclass, field


@dataclass
class Request:
    id: int
    nx: int
    ny: int
    walls: bool
    T_over_Tc: float
    steps: int
    bubbles: list
    delta: float = 0.0
    arrival: float = 0.0       # seconds after the start of the run
    tau_nu: float = 0.6
    W: float = 5.0
    noise_amp: float = 0.0
    seed: int = 0

    @property
    def sites(self):
        return self.nx * self.ny


@dataclass
class Result:
    id: int
    arrival: float
    admit: float
    first_chunk: float
    finish: float
    sites: int
    steps: int
    footprint: int
    diag: dict = field(default_factory=dict)
    state: object = None
    failed: bool = False         # turned non-finite; retired at the chunk where it was seen

    @property
    def latency(self):
        return self.finish - self.arrival


def percentile(values, q):
    """Nearest-rank percentile (q in [0, 100])."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(0, min(len(v) - 1, int(math.ceil(q / 100.0 * len(v))) - 1))
    return v[k]


def served_variants(names):
    """Indices of the tile variants a server may pick: those that accept any
    grid width (the paired "fused2-*" variants need an even nx, and requests
    of any width may still arrive)."""
    return [i for i, n in enumerate(names) if not n.startswith("fused2")]


class GpuBackend:
    """Backend over liblbm: one lbm.Sim per admitted request, resident in one
    of `n_batches` lbm.Batch objects, each on its own stream (default
    priority).  With several batches their launches overlap, so one batch's
    start-up, tail and kernel boundary run under another's work; a new
    request joins the batch with the fewest resident sites.  Results do not
    depend on the batch a request is in, nor on `write_through` (write-through
    population stores, Batch.set_write_through)."""

    def __init__(self, precision="fp32", device="cuda", max_instances=64, max_tiles=1 << 20,
                 variant=None, keep_state=False, n_batches=1, write_through=False):
        from . import lbm
        self.lbm = lbm
        self.precision = precision
        self.device = device
        self.keep_state = keep_state
        self.batches = [lbm.Batch(precision=precision, max_instances=max_instances,
                                  max_tiles=max_tiles, device=device) for _ in range(max(1, int(n_batches)))]
        for b in self.batches:
            b.set_write_through(write_through)
        self._where = {}                # id(handle) -> its batch
        self._sites = [0] * len(self.batches)
        self.variant = variant
        if variant is not None:
            for b in self.batches:
                b.set_variant(variant)
        self._bad = {}

    def params(self, req):
        return self.lbm.make_params(req.nx, req.ny, T_over_Tc=req.T_over_Tc, walls=req.walls,
                                    precision=self.precision, tau_nu=req.tau_nu)

    def footprint(self, req):
        return self.lbm.workspace_bytes(self.params(req))

    def prepare(self, req):
        """Allocates and initialises the instance on its own stream (overlaps
        the running chunk); returns a handle."""
        sim = self.lbm.Sim(self.params(req), device=self.device)
        sim.init_bubble(req.bubbles, W=req.W, delta=req.delta, noise_amp=req.noise_amp,
                        seed=req.seed)
        return sim

    def attach(self, h):
        k = min(range(len(self.batches)), key=lambda i: self._sites[i])
        self.batches[k].attach(h)
        self._where[id(h)] = k
        self._sites[k] += h.nx * h.ny

    def step(self, handles, counts):
        n = {id(h): c for h, c in zip(handles, counts)}
        for b in self.batches:
            if b.members:
                b.step_each([n.get(id(m), 0) for m in b.members])

    def sync(self):
        # one transfer per batch reads its resident requests' latches
        self._bad = {}
        for b in self.batches:
            if b.members:
                self._bad.update({id(m): bad for m, bad in zip(b.members, b.status())})

    def failed(self, h):
        return self._bad.get(id(h), False)

    def finish(self, h):
        out = h.macros(fields=False, check=False)["diag"]
        state = h.populations().cpu() if self.keep_state and not out["nonfinite"] else None
        k = self._where.pop(id(h))
        self.batches[k].detach(h)
        self._sites[k] -= h.nx * h.ny
        h.close()
        return out, state

    def autotune(self, reqs, reps=20, passes=3):
        """Picks the tile variant on throwaway instances shaped like reqs and
        returns (variant, aggregate MLUPS of the tuned run).  Only variants
        that accept any grid width compete (served_variants): a paired variant
        picked on a sample of even widths would refuse a later odd-width
        request.  Each candidate is timed with HIP events over `reps` steps
        after a warm-up, `passes` times, and scored by its fastest pass."""
        import torch
        lbm = self.lbm
        tmp = lbm.Batch(precision=self.precision, max_instances=len(reqs),
                        max_tiles=sum(lbm.tile_count(self.params(r)) for r in reqs), device=self.device)
        sims = [self.prepare(r) for r in reqs]
        for s in sims:
            tmp.attach(s)
        best = {}
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(passes):
            for v in served_variants(lbm.variant_names()):
                tmp.set_variant(v)
                tmp.step(min(reps, 8))
                tmp.prepare(reps)
                e0.record(tmp.stream)
                tmp.step(reps)
                e1.record(tmp.stream)
                e1.synchronize()
                ms = e0.elapsed_time(e1) / reps
                best[v] = min(best.get(v, float("inf")), ms)
        tmp.close()
        for s in sims:
            s.close()
        variant = min(best, key=best.get)
        self.variant = variant
        for b in self.batches:
            b.set_variant(variant)
        sites = sum(r.sites for r in reqs)
        return variant, sites / (best[variant] * 1e-3) / 1e6

    def close(self):
        for b in self.batches:
            b.close()


class Server:
    """Admission by footprint, continuous batching in chunks, FIFO order."""

    def __init__(self, backend, budget_bytes, max_slots=64, chunk_steps=500, clock=None,
                 sleep=None, log=None):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.chunk = int(chunk_steps)
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep
        self.log = log                  # optional file-like object for JSONL records
        self.peak_resident = 0
        self.peak_slots = 0

    def run(self, requests):
        pending = sorted(requests, key=lambda r: (r.arrival, r.id))
        for r in pending:
            if self.backend.footprint(r) > self.budget:
                raise ValueError("request %d needs more than the whole budget" % r.id)
        active = []                     # [req, handle, remaining, result]
        results = []
        resident = 0
        t0 = self.clock()
        now = lambda: self.clock() - t0
        updates = 0
        failures = 0
        busy = 0.0
        staged = []                     # prepared, attached at the next chunk boundary

        def admit():
            # in arrival order, every arrived request that fits the budget and a slot
            nonlocal resident
            while (pending and pending[0].arrival <= now()
                   and len(active) + len(staged) < self.max_slots):
                r = pending[0]
                need = self.backend.footprint(r)
                if resident + need > self.budget:
                    break
                pending.pop(0)
                resident += need
                h = self.backend.prepare(r)
                res = Result(r.id, r.arrival, now(), float("nan"), float("nan"), r.sites, r.steps, need)
                staged.append([r, h, r.steps, res])

        while pending or active or staged:
            admit()
            for a in staged:
                self.backend.attach(a[1])
                active.append(a)
            staged = []
            self.peak_resident = max(self.peak_resident, resident)
            self.peak_slots = max(self.peak_slots, len(active))
            if not active:
                if pending:
                    wait = pending[0].arrival - now()
                    if wait > 0:
                        self.sleep(wait)
                continue
            counts = [min(self.chunk, a[2]) for a in active]
            tc = now()
            for a in active:
                if math.isnan(a[3].first_chunk):
                    a[3].first_chunk = tc
            self.backend.step([a[1] for a in active], counts)
            admit()                     # initialise arrivals while the chunk runs
            self.backend.sync()
            busy += now() - tc
            updates += sum(c * a[0].sites for c, a in zip(counts, active))
            t_done = now()
            still = []
            for c, a in zip(counts, active):
                a[2] -= c
                # a request whose state turned non-finite is retired now, so
                # that it neither wastes steps nor stops the batch
                bad = self.backend.failed(a[1])
                if a[2] == 0 or bad:
                    diag, state = self.backend.finish(a[1])
                    a[3].finish = t_done
                    a[3].diag = diag
                    a[3].state = state
                    a[3].failed = bad
                    resident -= a[3].footprint
                    results.append(a[3])
                    if bad:
                        failures += 1
                    if self.log is not None:
                        self.log.write(json.dumps({
                            "id": a[3].id, "arrival": a[3].arrival, "admit": a[3].admit,
                            "first_chunk": a[3].first_chunk, "finish": a[3].finish,
                            "sites": a[3].sites, "steps": a[3].steps, "footprint": a[3].footprint,
                            "latency": a[3].latency, "failed": bad, "diag": diag}) + "\n")
                else:
                    still.append(a)
            active = still
        total = now()
        lat = [r.latency for r in results]
        stats = {"requests": len(results), "wall_s": total, "busy_s": busy,
                 "site_updates": updates, "mlups": updates / total / 1e6 if total > 0 else 0.0,
                 "busy_mlups": updates / busy / 1e6 if busy > 0 else 0.0,
                 "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99),
                 "mean_s": sum(lat) / len(lat) if lat else float("nan"),
                 "peak_resident_bytes": self.peak_resident, "peak_slots": self.peak_slots,
                 "failed": failures}
        return sorted(results, key=lambda r: r.id), stats


def make_requests(trace, arrivals, **extra):
    """Requests from inputs.request_trace dicts and arrival times."""
    out = []
    for t, a in zip(trace, arrivals):
        d = dict(t)
        d.update(extra)
        out.append(Request(id=d["id"], nx=d["nx"], ny=d["ny"], walls=d["walls"],
                           T_over_Tc=d["T_over_Tc"], steps=d["steps"], bubbles=d["bubbles"],
                           delta=d.get("delta", 0.0), arrival=float(a),
                           tau_nu=d.get("tau_nu", 0.6)))
    return out
