"""Benchmark of the D2Q9 pseudopotential MRT lattice Boltzmann timestep on one
MI355X.

Default workload: the Laplace-law and coexistence sweep (configuration c2: 24
instances of a 256 x 256 periodic grid, discs of radius 20..60 at T/Tc
0.6..0.9 plus one liquid slab per temperature), binary32, with the tile variant
the autotuner picks (normally the two-step kernel: one launch per two steps),
replayed from captured HIP graphs.  A "step" advances all 24 instances by one timestep.  The
steps are timed twice: as one batch over the tiles of all 24 instances on one
stream (one launch per step over every site), then spread over four batches on
four streams whose launches run concurrently, with write-through population
stores (`value`).

Prints one JSON line: aggregate MLUPS (million lattice-site updates per second)
of the concurrent run, the roofline of the dominant kernel from the one-stream
run (algorithmic HBM bytes of the stated per-site model over its timed launch
duration, and the measured HBM traffic when a counter record for the current
kernel source exists) with the concurrent run's figures beside it, the
oracle's CPU rate on
a bounded sample, the plain per-instance binary64 rate (one instance at a time,
direct launches, no graph, no batch) and the served-batch latencies.

Other workloads: collapse_large (configuration c5: one 8192 x 4096
wall-bounded grid, HBM resident), single_small (c1) and the experiment drivers
of paper_1605_01800_amd.studies, each printing its own JSON line.  The served
batch follows configuration c4.  The configurations are the JSON files of
paper_1605_01800_amd/configs.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per site per launch (read 9 f and write psi / read 9 f,
# read psi, write 9 f), by element size
BYTES_PSI = {4: 9 * 4 + 4, 8: 9 * 8 + 8}
BYTES_COLLIDE = {4: 9 * 4 + 4 + 9 * 4, 8: 9 * 8 + 8 + 9 * 8}
# the fused kernel reads the nine populations and writes nine (psi stays in LDS)
BYTES_FUSED = {4: 18 * 4, 8: 18 * 8}


def timing_parts(steps):
    """Step counts of the timed parts: 256 steps each (the longest chunk one
    captured graph holds) and the remainder, so that every part replays graphs
    prepared during the warm-up and the steps need no host-to-device transfer
    (the descriptors already hold the parts' chunk length)."""
    full, rest = divmod(steps, 256)
    return [256] * full + ([rest] if rest else [])


def hold(L, streams, ms):
    """Holds every stream until one common instant of the device clock, about
    `ms` milliseconds ahead (lbm_hold_until): the host enqueues the timed
    region's first part on every stream meanwhile, and the streams then start
    together, so that the region times the device work alone, neither the
    host's enqueueing nor a cross-stream wait (a fork of four streams from one
    and their join back cost about 30 us, measured with tiny kernels)."""
    tick, rate = L.device_clock()
    until = tick + int(ms * 1e-3 * rate)
    for st in streams:
        L.hold_until(until, rate // 2, st)


def timed_region(torch, L, runner, streams, steps, warmup):
    """Times `steps` steps of `runner` (a Batch on streams[0], or a
    BatchGroup whose batches run on `streams`) with HIP events; returns (ms,
    median ms per step of the parts, parts).  The warm-up runs `warmup` steps,
    then readies the timed steps' graphs and descriptors without running them
    (lbm_batch_prepare), so the timed region enqueues nothing but graph
    launches.  The timed steps run as parts of up to 256 steps.  Every stream
    records a start event after the common hold and an end event after its
    last part; the region runs from the earliest start to the latest end, so
    it brackets the work of every stream without timing a cross-stream wait.
    Between parts the streams are aligned again (the first waits for the
    others, they for it; events without timing, which cost less in a busy
    stream), and the first stream records a timed event there: left to drift
    apart, four concurrent batches ran 3 % slower over 1280 steps.  The parts
    add up to the region (for the median)."""
    parts = timing_parts(steps)
    if warmup > 0:
        runner.step(warmup)
    runner.prepare(steps)
    runner.sync()
    start = [torch.cuda.Event(enable_timing=True) for _ in streams]
    end = [torch.cuda.Event(enable_timing=True) for _ in streams]
    mid = [torch.cuda.Event(enable_timing=True) for _ in parts[1:]]
    torch.cuda.synchronize()
    ref = torch.cuda.Event(enable_timing=True)
    ref.record(streams[0])                  # before every hold ends
    # long enough for the host to enqueue the first part on every stream (the
    # later parts are enqueued while it runs), and no longer: an idle device
    # lowers its clocks, and after a 20 ms hold the first 512 steps ran 10 %
    # slower
    hold(L, streams, max(1.0, 0.5 * len(streams)))
    for e, st in zip(start, streams):
        e.record(st)
    for i, n in enumerate(parts):
        if i > 0:
            for st in streams[1:]:
                done = torch.cuda.Event()
                done.record(st)
                streams[0].wait_event(done)
            mid[i - 1].record(streams[0])
            go = torch.cuda.Event()
            go.record(streams[0])
            for st in streams[1:]:
                st.wait_event(go)
        runner.step(n)
    for e, st in zip(end, streams):
        e.record(st)
    torch.cuda.synchronize()
    bounds = ([min(ref.elapsed_time(e) for e in start)] + [ref.elapsed_time(e) for e in mid] +
              [max(ref.elapsed_time(e) for e in end)])            # ms after `ref`
    ms = bounds[-1] - bounds[0]
    part_ms = sorted((bounds[i + 1] - bounds[i]) / n for i, n in enumerate(parts))
    return ms, part_ms[len(part_ms) // 2], len(part_ms)


def measured_traffic(workload, variant_name, batches, write_through):
    """The rocprofv3 FETCH_SIZE and WRITE_SIZE record of the dominant kernel
    for this workload, tile variant, number of concurrent batches and store
    kind (write-through or not), from
    profiles/traffic.json (HBM bytes per launch, each counter scaled by what
    it reads for a copy kernel of known size), or None when there is no such
    record or the kernel source (lbm_kernels.hip and lbm_rounding.h) has
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    csrc = os.path.join(ROOT, "paper_1605_01800_amd", "csrc")
    try:
        with open(path) as fh:
            rec = json.load(fh)
        h = hashlib.sha256()
        for name in ("lbm_kernels.hip", "lbm_rounding.h"):    # the kernels' device code
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(fh.read())
        sha = h.hexdigest()
    except (OSError, ValueError):
        return None
    if not isinstance(rec, dict) or rec.get("kernels_source_sha256") != sha:
        return None
    found = rec.get("entries", {}).get(workload, [])
    for e in (found if isinstance(found, list) else [found]):
        if (isinstance(e, dict) and e.get("variant") == variant_name and e.get("batches") == batches
                and e.get("write_through") == bool(write_through) and "bytes_per_launch" in e):
            return e
    return None


# Vector-ALU issue peak of the MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz,
# one lane-operation per lane and clock (a wave64 instruction issues over four
# clocks; no packed or dual-issued forms, which the build switches off):
# 39.3 T lane-operations/s, the fp32 vector peak of 157.3 TFLOP/s counted as
# one lane-operation per fused multiply-add and without packing.
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9


def valu_roofline(rec, launch_ms, site_updates):
    """The launch against the vector-ALU issue peak, from the SQ_INSTS_VALU
    count in the counter record (wave instructions per launch, x 64 lanes),
    or None without such a record."""
    if not rec or "valu_insts_per_launch" not in rec:
        return None
    lane_slots = rec["valu_insts_per_launch"] * 64
    achieved = lane_slots / (launch_ms * 1e-3)
    return {"bound": "alu", "achieved": round(achieved / 1e12, 2), "peak": round(VALU_PEAK_LANE_OPS / 1e12, 2),
            "unit": "T lane-ops/s", "frac": round(achieved / VALU_PEAK_LANE_OPS, 4),
            "valu_insts_per_launch": rec["valu_insts_per_launch"],
            "lane_slots_per_site_update": round(lane_slots / site_updates, 1),
            "issue_floor_ms": round(lane_slots / VALU_PEAK_LANE_OPS * 1e3, 5)}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1280)
    ap.add_argument("--warmup", type=int, default=256)
    ap.add_argument("--workload", default="laplace_sweep",
                    choices=["laplace_sweep", "collapse_large", "collapse_shard", "precision_large",
                             "collapse_horizon",
                             "laplace_physics", "coexistence_sweep", "critical_nucleus", "paper_collapse",
                             "single_small"])
    ap.add_argument("--streams", type=int, default=0,
                    help="batches (one stream each) the instances are spread over; 0: 4 for "
                         "workloads of several instances, 1 otherwise")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-plain", action="store_true")
    ap.add_argument("--variant", type=int, default=-1, help="tile variant; -1 autotunes")
    ap.add_argument("--write-through", default="auto", choices=["auto", "0", "1"],
                    help="write-through stores for the one-batch run; auto: the faster, by timing")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-served", action="store_true", help="skip the served-batch latency run")
    ap.add_argument("--tau-nu", type=float, default=None,
                    help="tau_nu of the collapse studies (default: the configured one)")
    ap.add_argument("--delta", type=float, default=None,
                    help="liquid over-density of the collapse studies (default: the configured one)")
    ap.add_argument("--sigma", type=float, default=0.0111,
                    help="surface tension for the critical-nucleus study (this model's Laplace fit at 0.5 Tc)")
    ap.add_argument("--tau-nu-list", type=float, nargs="+", default=[0.51, 0.6],
                    help="tau_nu values of the paper_collapse study")
    ap.add_argument("--delta-list", type=float, nargs="+", default=[0.13],
                    help="liquid over-densities of the paper_collapse study")
    ap.add_argument("--record-every", type=int, default=0, help="record interval of the paper_collapse study")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "fp32_mixed"],
                    help="precision of the paper_collapse study")
    from paper_1605_01800_amd import inputs
    c4 = inputs.load_config("c4")
    ap.add_argument("--served-requests", type=int, default=c4["trace"]["n_requests"])
    ap.add_argument("--served-budget-gb", type=float, default=c4["serving"]["budget_gb"])
    ap.add_argument("--served-batches", type=int, default=c4["serving"]["batches"],
                    help="batches (one stream each) the served requests are spread over")
    ap.add_argument("--served-write-through", type=int, default=int(c4["serving"]["write_through"]),
                    choices=[0, 1], help="write-through population stores in the served batches")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run liblbm's plain copy kernel over MIB MiB, 5 times, and exit "
                         "(reference for the memory-traffic counters)")
    return ap.parse_args()


def calibrate_copy(mib):
    import torch
    from paper_1605_01800_amd import lbm as L
    n = mib << 20
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    L.copy_kernel(dst, src, n, st)
    e0.record(st)
    for _ in range(5):
        L.copy_kernel(dst, src, n, st)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / 5
    assert torch.equal(dst, src)
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "ms": ms,
                      "GB_s": 2 * n / (ms * 1e-3) / 1e9}), flush=True)


def copy_rate(L, nbytes, stream, reps=50):
    """GB/s of the library's plain copy kernel moving nbytes into another nbytes
    (so 2 nbytes of traffic per launch), launched back to back on `stream`:
    what the memory system delivers for a launch's worth of bytes, launch cost
    included."""
    import torch
    n = max(16, (int(nbytes) + 15) // 16 * 16)
    with torch.cuda.stream(stream):
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
    for _ in range(5):
        L.copy_kernel(dst, src, n, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        L.copy_kernel(dst, src, n, stream)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * n / (ms * 1e-3) / 1e9


def collapse_large_sims(L, precision, device):
    """The 8192 x 4096 three-disc collapse of configuration c5."""
    from paper_1605_01800_amd import inputs, studies
    (inst,) = inputs.config_instances(inputs.load_config("c5"))
    return [studies.sim_from_instance(L, inst, precision, device)]


def collapse_shard_sims(L, precision, device):
    """One GPU's share of the 8192 x 4096 grid split in y over 8 GPUs: the
    lowest 512 rows (lower wall; the cut at the top would exchange a halo
    with the next GPU and is a wall here), with the part of the largest
    disc that falls into them."""
    from paper_1605_01800_amd import inputs, studies
    (inst,) = inputs.config_instances(inputs.load_config("c5"))
    inside = [b for b in inst["bubbles"] if b[1] - b[2] < 512]
    shard = dict(inst, ny=512, bubbles=inside or [(4095.5, 255.5, 150.0)])
    return [studies.sim_from_instance(L, shard, precision, device)]


def single_small(device, steps, warmup):
    """One 64 x 64 periodic instance in binary64 (T = 0.7 T_c, a disc of
    radius 16 at the centre, W = 2, tau_nu = 0.8, the 64^2 check of
    Section 3.1): a launch-bound case (0.3 MB of populations), stepped through
    captured graphs of 256 steps on the instance's own stream, for each tile
    variant."""
    import torch
    from paper_1605_01800_amd import inputs, studies
    from paper_1605_01800_amd import lbm as L
    cfg = inputs.load_config("c1")
    (inst,) = inputs.config_instances(cfg)
    out = {"metric": "single_instance_mlups", "grid": "%dx%d" % (inst["nx"], inst["ny"]),
           "precision": cfg["precision"], "steps": steps, "variants": {}}
    for v, name in enumerate(L.variant_names()):
        s = studies.sim_from_instance(L, inst, cfg["precision"], device)
        s.set_variant(v)
        s.step(warmup)
        s.sync()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        s.step(steps)
        e1.record(s.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        out["variants"][name] = {"mlups": round(inst["nx"] * inst["ny"] * steps / (ms * 1e-3) / 1e6, 1),
                                 "us_per_step": round(ms * 1e3 / steps, 3)}
        s.close()
    best = max(out["variants"].items(), key=lambda kv: kv[1]["mlups"])
    out["best"] = {"variant": best[0], **best[1]}
    print(json.dumps(out), flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(seconds):
    """The FP64 oracle on one 256 x 256 instance of the sweep (R = 40 at
    0.7 T_c), steps sized to take about `seconds` on all the threads its
    OpenMP runtime uses, then a shorter sample on one thread."""
    from oracle import coexist, stepper
    from oracle import build as obuild
    obuild.ensure_built()
    T = coexist.temperature(0.7)
    rg, rl, _ = coexist.maxwell(T)
    P = stepper.make_params(256, 256, T, tau_nu=0.6)

    def timed(secs):
        f = stepper.init_populations(P, stepper.init_density(P, bubbles=[(127.5, 127.5, 40.0)],
                                                             rho_l=rl, rho_g=rg, W=5.0))
        t0 = time.perf_counter()
        stepper.step(P, f, 3)
        per = (time.perf_counter() - t0) / 3
        n = max(3, int(secs / per))
        t0 = time.perf_counter()
        rc = stepper.step(P, f, n)
        dt = time.perf_counter() - t0
        assert rc == 0
        return n, dt

    threads = stepper.threads()
    n, dt = timed(seconds)
    stepper.set_threads(1)
    n1, dt1 = timed(seconds / 5)
    stepper.set_threads(threads)
    return {"value": 256 * 256 * n / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "1 of the 24 sweep instances (256x256, R=40, 0.7 Tc), %d steps, %.1f s" % (n, dt),
            "single_thread_value": 256 * 256 * n1 / dt1 / 1e6,
            "single_thread_sample": "%d steps, %.1f s" % (n1, dt1), "cpu_model": _cpu_model()}


def fp64_plain(L, device, steps):
    """Each sweep instance in binary64, one at a time, direct launches on the
    null stream (no graph, no batching)."""
    import torch
    sims = []
    from paper_1605_01800_amd import inputs
    null = torch.cuda.default_stream(torch.device(device))
    for case in inputs.laplace_sweep_cases(256):
        p = L.make_params(256, 256, T_over_Tc=case["T_over_Tc"], precision="fp64", tau_nu=0.6)
        s = L.Sim(p, device=device, stream=null)
        s.init_bubble(case["bubbles"], slab_rows=case["slab_rows"], W=5.0)
        sims.append(s)
    for s in sims:
        s.step(5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sims:
        s.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for s in sims:
        s.close()
    return len(sims) * 256 * 256 * steps / dt / 1e6


def served_run(device, n_requests, budget_gb, load=None, chunk=None, seed=None, batches=1, write_through=False):
    """The served batch: n_requests requests of the served-batch trace (sides
    log-uniform in [64, 1024], aspect 1, 4/3 or 2, half periodic bubbles and
    half wall-bounded collapses, T/Tc in [0.6, 0.9], 5,000-40,000 steps),
    Poisson arrivals at a rate that loads the GPU to `load` of the throughput
    measured by the autotuner on the first 16 requests (one batch).  The
    resident requests are spread over `batches` batches on their own streams."""
    import numpy as np
    from paper_1605_01800_amd import inputs, serving
    c4 = inputs.load_config("c4")
    load = c4["serving"]["load"] if load is None else load
    chunk = c4["serving"]["chunk_steps"] if chunk is None else chunk
    seed = c4["trace"]["seed"] if seed is None else seed
    trace = inputs.request_trace(n_requests, seed)
    reqs0 = serving.make_requests(trace, [0.0] * n_requests)
    be = serving.GpuBackend(precision="fp32", device=device, max_instances=64, max_tiles=1 << 19,
                            n_batches=batches, write_through=write_through)
    variant, cal_mlups = be.autotune(reqs0[:c4["serving"]["autotune_requests"]])
    work = np.mean([r.sites * r.steps for r in reqs0])
    rate = load * cal_mlups * 1e6 / work
    arrivals = inputs.poisson_arrivals(n_requests, rate, seed + 1)
    reqs = serving.make_requests(trace, arrivals)
    srv = serving.Server(be, budget_bytes=int(budget_gb * 1e9), max_slots=64, chunk_steps=chunk)
    results, stats = srv.run(reqs)
    be.close()
    bad = [r.id for r in results if r.diag.get("nonfinite")]
    from paper_1605_01800_amd import lbm as L
    errs = served_reference_errors(device, reqs, results)
    compact = [[e["id"]] + (["failed"] if e.get("failed") else
                            [float("%.2g" % e["radius"]), float("%.2g" % e["mass"]),
                             None if e["wall_p"] is None else float("%.2g" % e["wall_p"])])
               for e in errs["per_request"]]
    return {"error_vs_fp64": {"summary": errs["summary"],
                              "per_request": "[id, radius, mass, wall-pressure peak] relative errors "
                                             "of the final result against the same request in binary64",
                              "values": compact},
            "requests": len(results), "arrival_rate_per_s": round(rate, 3), "load": load,
            "calibrated_mlups": round(cal_mlups, 1), "tile": L.variant_names()[variant],
            "budget_GB": budget_gb, "chunk_steps": chunk, "batches": batches,
            "write_through": bool(write_through),
            "wall_s": round(stats["wall_s"], 3),
            "busy_s": round(stats["busy_s"], 3), "aggregate_mlups": round(stats["mlups"], 1),
            "busy_mlups": round(stats["busy_mlups"], 1), "p50_s": round(stats["p50_s"], 4),
            "p99_s": round(stats["p99_s"], 4), "mean_s": round(stats["mean_s"], 4),
            "peak_resident_GB": round(stats["peak_resident_bytes"] / 1e9, 3),
            "peak_slots": stats["peak_slots"], "nonfinite_requests": bad}


def served_reference_errors(device, reqs, results, chunk=500):
    """Every served result against the same request stepped in binary64 (the
    path held to the oracle at 1e-12): relative errors of the final bubble
    radius, total mass and, with walls, the wall-pressure peak.  The binary64
    runs go through the same server, all arrived at once, with a budget that
    never binds."""
    from paper_1605_01800_amd import lbm as L
    from paper_1605_01800_amd import serving
    ref_reqs = [serving.Request(**{**r.__dict__, "arrival": 0.0}) for r in reqs]
    be = serving.GpuBackend(precision="fp64", device=device, max_instances=64, max_tiles=1 << 19,
                            n_batches=2, variant=L.variant_names().index("fused-64x16"))
    srv = serving.Server(be, budget_bytes=64 * 10 ** 9, max_slots=64, chunk_steps=chunk)
    ref, _ = srv.run(ref_reqs)
    be.close()
    by_id = {r.id: r for r in ref}
    rel = lambda a, b: abs(a - b) / abs(b)
    per = []
    for r in results:
        q = by_id[r.id]
        if r.failed or q.failed:
            per.append({"id": r.id, "failed": True})
            continue
        e = {"id": r.id, "radius": max((rel(a, b) for a, b in zip(r.diag["radius"], q.diag["radius"])),
                                       default=0.0),
             "mass": rel(r.diag["mass"], q.diag["mass"]),
             "wall_p": None}
        if q.diag["wall_p_step"] >= 0:
            e["wall_p"] = rel(r.diag["wall_p_max"], q.diag["wall_p_max"])
            e["wall_p_same_step"] = r.diag["wall_p_step"] == q.diag["wall_p_step"]
        per.append(e)
    ok = [e for e in per if not e.get("failed")]
    summary = {}
    for k in ("radius", "mass", "wall_p"):
        v = sorted(e[k] for e in ok if e.get(k) is not None)
        if v:
            summary[k] = {"max": v[-1], "median": v[len(v) // 2]}
    summary["wall_p_same_step"] = sum(1 for e in ok if e.get("wall_p_same_step"))
    summary["with_walls"] = sum(1 for e in ok if e.get("wall_p") is not None)
    return {"per_request": per, "summary": summary}


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1605_01800_amd import lbm as L

    device = "cuda:0"
    torch.cuda.set_device(0)
    from paper_1605_01800_amd import studies
    if args.workload == "precision_large":
        studies.precision_study(device, True, steps=args.steps, every=max(1, args.steps // 20),
                                tau_nu=args.tau_nu, delta=args.delta)
        return
    if args.workload == "collapse_horizon":
        studies.precision_study(device, False, steps=args.steps, every=max(1, args.steps // 100),
                                tau_nu=args.tau_nu, delta=args.delta)
        return
    if args.workload == "laplace_physics":
        studies.laplace_physics(device, steps=args.steps)
        return
    if args.workload == "single_small":
        single_small(device, steps=args.steps, warmup=args.warmup)
        return
    if args.workload == "coexistence_sweep":
        studies.coexistence_sweep(device, steps=args.steps)
        return
    if args.workload == "critical_nucleus":
        studies.critical_nucleus(device, steps=args.steps, sigma=args.sigma)
        return
    if args.workload == "paper_collapse":
        studies.paper_collapse(device, steps=args.steps, every=args.record_every or max(1, args.steps // 200),
                               tau_nu=args.tau_nu_list, delta=args.delta_list, precision=args.precision)
        return
    precision = "fp32"
    es = 4
    from paper_1605_01800_amd import inputs
    if args.workload == "laplace_sweep":
        sims = studies.laplace_sweep_sims(L, precision, device)
        cfg = inputs.load_config("c2")
        sw, d = cfg["sweep"], cfg["defaults"]
        workload = {"workload": "laplace_sweep", "configuration": "c2", "instances": len(sims),
                    "grid": "%dx%d" % (sw["nx"], sw["ny"]), "periodic": not d["walls"],
                    "T_over_Tc": sw["T_over_Tc"], "radii": sw["radii"], "slab_rows": sw["slab_rows"],
                    "tau_nu": d["tau_nu"], "eps": d["eps"]}
    else:
        (inst,) = inputs.config_instances(inputs.load_config("c5"))
        common = {"instances": 1, "walls_y": inst["walls"], "T_over_Tc": inst["T_over_Tc"],
                  "delta": inst["delta"], "tau_nu": inst["tau_nu"], "eps": inst["eps"]}
        if args.workload == "collapse_shard":
            sims = collapse_shard_sims(L, precision, device)
            workload = {"workload": "collapse_shard", "configuration": "c5", "grid": "%dx512" % inst["nx"],
                        "shard_of": "%dx%d over 8 GPUs (rows 0-511, lower wall)" % (inst["nx"], inst["ny"]),
                        **common}
        else:
            sims = collapse_large_sims(L, precision, device)
            workload = {"workload": "collapse_large", "configuration": "c5",
                        "grid": "%dx%d" % (inst["nx"], inst["ny"]),
                        "radii": [b[2] for b in inst["bubbles"]], **common}
    sites = sum(s.nx * s.ny for s in sims)
    max_tiles = sum(L.tile_count(s.params) for s in sims)
    batch = L.Batch(precision=precision, max_instances=len(sims), max_tiles=max_tiles, device=device)
    for s in sims:
        batch.attach(s)
    if args.variant >= 0:
        batch.set_variant(args.variant)
        variant = args.variant
    else:
        variant, _ = batch.autotune(reps=20)
    workload["tile"] = L.variant_names()[variant]
    # write-through stores for the one-batch run, by timing (they pay where the
    # populations stay in the caches and cost where they stream from HBM)
    if args.write_through == "auto":
        wt1, _ = batch.tune_write_through(reps=20)
    else:
        batch.set_write_through(args.write_through == "1")
        wt1 = batch.write_through
    workload["write_through_one_batch"] = wt1
    # Independent instances can also be spread over several batches, one
    # stream each, whose kernels then run concurrently (one batch's start-up,
    # tail and kernel boundary overlap another's work); a step is then one
    # launch per batch.
    n_streams = args.streams if args.streams > 0 else (4 if len(sims) >= 4 else 1)
    n_streams = min(n_streams, len(sims))
    vname = L.variant_names()[variant]
    fused = not vname.startswith("2pass")
    if not fused:
        n_streams = 1                     # their launches are timed one batch at a time
    workload["streams"] = n_streams
    print("# workload %s sites %d variant %s streams %d" % (args.workload, sites, vname, n_streams),
          file=sys.stderr, flush=True)

    # First the whole batch on one stream: one launch per step over every
    # site, timed as a region with HIP events on that stream.  This gives the
    # dominant kernel's launch duration for the roofline, and matches a
    # kernel trace launch for launch (a profiler serialises concurrent
    # streams, so their launches cannot be checked against a trace).
    ms1, median1, nparts1 = timed_region(torch, L, batch, [batch.stream], args.steps, args.warmup)
    for s in sims:
        s.sync()                          # raises if a non-finite value was latched
    print("# one stream, %d steps: %.4f ms/step, %.0f MLUPS" % (args.steps, ms1 / args.steps,
                                                                sites * args.steps / (ms1 * 1e-3) / 1e6),
          file=sys.stderr, flush=True)

    # Then the job as it runs best: with several streams, the instances in
    # n_streams batches stepped concurrently.  `value` is this region.
    group = None
    if n_streams > 1:
        for s in sims:
            batch.detach(s)
        group = L.BatchGroup(sims, precision=precision, n_batches=n_streams, device=device)
        group.set_variant(variant)
        group_wt = group.batches[0].write_through
        workload["write_through"] = group_wt
        ms, median_ms, nparts = timed_region(torch, L, group, group.streams, args.steps, args.warmup)
    else:
        workload["write_through"] = wt1
        ms, median_ms, nparts = ms1, median1, nparts1
    for s in sims:
        s.sync()
    mlups = sites * args.steps / (ms * 1e-3) / 1e6
    print("# timed %d steps on %d stream(s): %.4f ms/step, %.0f MLUPS" % (args.steps, n_streams,
                                                                        ms / args.steps, mlups),
          file=sys.stderr, flush=True)

    # Dominant kernel.  Fused variants launch one kernel per step, replayed
    # back to back from prepared graphs, so on one stream a launch lasts the
    # timed region over the step count (an upper bound: it includes the
    # kernel boundaries and one end-of-chunk kernel per graph) and moves the
    # bytes of all sites; a kernel trace of the same command gives the same
    # average launch.  Two-pass variants time each launch with its own event
    # pair on the batch's stream.
    # A two-step launch advances every site by two steps: its algorithmic
    # bytes are those of two site updates (2 x 72 B a site), while the bytes
    # it must move are one read and one write of the populations (72 B a
    # site), reported beside them as min_hbm_*.
    nk = min(args.steps, 100)
    nk += nk % 2
    spl = 2 if vname.startswith("twostep") else 1          # site updates per launch
    if group is not None:
        group.close()
        for s in sims:
            batch.attach(s)
    ms_psi, ms_col = batch.step_timed(nk)
    if fused:
        t_dom = ms1 / args.steps * spl
        kname = {"fused2": "fused2_kernel", "fused": "fused_kernel",
                 "twostep": "twostep_kernel"}[vname.split("-")[0]]
        dominant = (kname, t_dom, BYTES_FUSED[es] * spl)
        kernels = {kname: {"ms_region_avg": t_dom, "ms_event_pair_avg": ms_col / (nk // spl),
                           "site_updates_per_launch": spl,
                           "bytes_per_site": BYTES_FUSED[es] * spl,
                           "GB_s": round(BYTES_FUSED[es] * spl * sites / (t_dom * 1e-3) / 1e9, 1)}}
    else:
        t_psi, t_col = ms_psi / nk, ms_col / nk
        dominant = ("collide_stream_kernel", t_col, BYTES_COLLIDE[es]) if t_col >= t_psi else \
            ("psi_pass_kernel", t_psi, BYTES_PSI[es])
        kernels = {"psi_pass_kernel": {"ms": t_psi, "bytes_per_site": BYTES_PSI[es],
                                       "GB_s": round(BYTES_PSI[es] * sites / (t_psi * 1e-3) / 1e9, 1)},
                   "collide_stream_kernel": {"ms": t_col, "bytes_per_site": BYTES_COLLIDE[es],
                                             "GB_s": round(BYTES_COLLIDE[es] * sites / (t_col * 1e-3) / 1e9, 1)}}
    achieved = dominant[2] * sites / (dominant[1] * 1e-3) / 1e9
    print("# dominant %s %.4f ms/launch, %.0f GB/s of %d B/site" % (dominant[0], dominant[1], achieved,
                                                                     dominant[2]), file=sys.stderr, flush=True)

    trec = measured_traffic(args.workload, vname, 1, wt1)
    traffic = trec["bytes_per_launch"] if trec else None
    # The MI355X's Infinity Cache (256 MB) sits between the L2s and HBM: a
    # working set that fits it is served from there, and the FETCH_SIZE and
    # WRITE_SIZE counters (L2 to fabric) then count cache bytes, not only
    # DRAM bytes.
    working_set = sum(L.workspace_bytes(s.params) for s in sims)
    cache_resident = working_set < 256e6
    min_hbm = BYTES_FUSED[es] * sites if fused else dominant[2] * sites    # bytes a launch must move
    min_hbm_gbs = min_hbm / (dominant[1] * 1e-3) / 1e9
    copy_gbs = copy_rate(L, min_hbm // 2, batch.stream)
    out = {
        "metric": "aggregate MLUPS + %HBM roofline (FP32 batched vs FP64 plain); p50/p99 latency",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "ms_per_step_median_of_parts": median_ms,
        "timed_parts": nparts,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (Eq. 16 initial states)",
        "config": workload,
        "roofline": {
            "bound": "hbm",
            "kernel": dominant[0],
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "launch_ms": dominant[1],
            "traffic": traffic,
            "traffic_counters": "FETCH_SIZE + WRITE_SIZE per launch, scaled by a copy of known size: "
                                "bytes from the L2s to the fabric" +
                                (" (the working set fits the 256 MB Infinity Cache, so not all of "
                                 "them reach DRAM)" if cache_resident else ""),
            "working_set_bytes": working_set,
            "cache_resident": cache_resident,
            "bytes_per_site": dominant[2],
            "site_updates_per_launch": spl,
            "algorithmic_bytes_per_launch": dominant[2] * sites,
            "traffic_over_algorithmic": None if traffic is None else round(traffic / (dominant[2] * sites), 4),
            "min_hbm_bytes_per_launch": min_hbm,
            "min_hbm_GB_s": round(min_hbm_gbs, 1),
            "traffic_over_min_hbm": None if traffic is None else round(traffic / min_hbm, 4),
            # a plain copy of the bytes a launch must move (half read, half
            # written), back to back on one stream: what this traffic can
            # reach on this part, launch cost included
            "copy_same_bytes_GB_s": round(copy_gbs, 1),
            "frac_of_copy": round(min_hbm_gbs / copy_gbs, 4),
            "valu": valu_roofline(trec, dominant[1], sites * spl),
        },
        "kernels": kernels,
    }
    if group is not None:
        # the step's launches on all streams, each over its batch's share of
        # the sites: the step's algorithmic bytes over the step's time, and
        # the step's measured bytes (launches of a quarter of the grid)
        step_ms = ms / args.steps
        crec = measured_traffic(args.workload, vname, n_streams, group_wt)
        # bytes of one step: every batch's launches in it (a two-step launch
        # counts for two steps)
        c_traffic = round(crec["bytes_per_launch"] * crec["launches_per_step"]) if crec else None
        c_achieved = BYTES_FUSED[es] * sites / (step_ms * 1e-3) / 1e9
        out["roofline"]["concurrent_streams"] = {
            "streams": n_streams, "launches_per_step": n_streams / spl, "write_through": group_wt,
            "step_ms": step_ms,
            "achieved": round(c_achieved, 1), "frac": round(c_achieved / HBM_PEAK_GBS, 4),
            "frac_of_copy": round(c_achieved / spl / copy_gbs, 4), "traffic": c_traffic,
            "traffic_over_algorithmic": None if c_traffic is None else
            round(c_traffic / (BYTES_FUSED[es] * sites), 4)}
    batch.close()
    for s in sims:
        s.close()
    torch.cuda.synchronize()

    if args.workload == "laplace_sweep" and not args.no_fp64_plain:
        plain = fp64_plain(L, device, steps=40)
        out["fp64_plain_mlups"] = round(plain, 1)
        out["speedup_vs_fp64_plain"] = round(mlups / plain, 2)
        print("# fp64 plain per-instance %.0f MLUPS" % plain, file=sys.stderr, flush=True)

    if args.workload == "laplace_sweep" and not args.no_served:
        sv = served_run(device, args.served_requests, args.served_budget_gb, batches=args.served_batches,
                        write_through=bool(args.served_write_through))
        out["served"] = sv
        out["p50_s"] = sv["p50_s"]
        out["p99_s"] = sv["p99_s"]
        print("# served %d requests: %.0f MLUPS aggregate, p50 %.3f s, p99 %.3f s"
              % (sv["requests"], sv["aggregate_mlups"], sv["p50_s"], sv["p99_s"]), file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        print("# cpu baseline %.2f MLUPS" % out["cpu_baseline"]["value"], file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
