"""Writes the oracle's references for the long-horizon parity tests and times
the oracle on those workloads.

  sweep     the Laplace-law and coexistence sweep: 24 periodic 256 x 256
            instances (discs of radius 20 .. 60 at T/T_c 0.6 .. 0.9, plus one
            liquid slab of 128 rows per temperature), tau_nu = 0.6, W = 5,
            40,000 steps; bubble radius and mass every 1000 steps, density
            snapshots at 10,000, 20,000 and 40,000 steps (every fourth site in
            x and y, and the full row and column through the centre), the
            final pressure jump of each disc (Eq. 17, p of Eq. 15) and the
            coexisting densities of each slab.
  collapse  the wall-bounded collapse on 1024 x 768 (x periodic, halfway
            bounce-back walls in y, T = 0.6 T_c, tau_nu = 0.6, a disc of radius
            120 centred at (511.5, 200), W = 5, liquid at rho_l (1 + delta),
            +-0.1 % seeded noise), 50,000 steps; radius and mass every 100 steps,
            the wall-pressure reading of every step (kept as its running maximum
            and step, and the maximum of each 100-step block), and density
            snapshots (every fourth site, the row through the centre and the
            column through x = 511) at steps 1000, 5000, 10000, 20000, 50000.

TEST INFRASTRUCTURE: calls only oracle/ (the binary64 CPU stepper, its
multiprecision coexistence solver and its post-processing) and the seeded
layouts of paper_1605_01800_amd.inputs, which hold none of the method's
arithmetic.  Every stored value is the oracle's.  The wall time of every run is
stored with the thread count and the CPU model.

    python tests/golden/make_horizon_goldens.py sweep|collapse [--delta D --seed S] [--threads N]
                                                [--out DIR]   (default: tests/golden)
    python tests/golden/make_horizon_goldens.py sweep --part I --parts N   (cases I, I+N, ...)
    python tests/golden/make_horizon_goldens.py merge-sweep --parts N      (joins the parts)
    python tests/golden/make_horizon_goldens.py timing [--max-steps K]     (1 thread and all)
"""
import argparse
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import coexist, diagnostics, stepper  # noqa: E402
from paper_1605_01800_amd import inputs  # noqa: E402

OUT_DIR = HERE


def sweep_file():
    return os.path.join(OUT_DIR, "laplace_sweep_40k.npz")


SNAP_STEPS = (1000, 5000, 10000, 20000, 50000)


def collapse_file(delta, seed):
    return os.path.join(OUT_DIR, "collapse_1024x768_50k_d%03d_s%d.npz" % (round(delta * 1000), seed))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def sample(rho, stride=4):
    return np.ascontiguousarray(rho[::stride, ::stride])


SWEEP_SNAPS = (10000, 20000, 40000)
SWEEP_PER_CASE = ("radius", "mass", "rho_sampled", "rho_centre_row", "rho_centre_col", "T_over_Tc", "T", "R",
                  "slab_rows", "rho_l", "rho_g", "dp", "p_in", "p_out", "slab_rho_g", "slab_rho_l", "wall_s")


def part_file(i):
    return os.path.join(OUT_DIR, "laplace_sweep_40k_part%d.npz" % i)


def merge_sweep(parts):
    """Joins the parts written by `sweep --part i --parts n` (cases i, i + n,
    ...) into the one reference file, in case order."""
    ps = [np.load(part_file(i), allow_pickle=False) for i in range(parts)]
    ncase = sum(len(p["case_index"]) for p in ps)
    out = {}
    for key in SWEEP_PER_CASE:
        a = None
        for p in ps:
            v = p[key]
            if a is None:
                a = np.zeros((ncase,) + v.shape[1:], dtype=v.dtype)
            a[p["case_index"]] = v
        out[key] = a
    total = float(np.sum(out["wall_s"]))
    n = 256
    steps = int(ps[0]["steps"])
    np.savez_compressed(sweep_file(), steps=steps, every=int(ps[0]["every"]), stride=4,
                        snap_steps=np.array(ps[0]["snap_steps"]),
                        threads=int(ps[0]["threads"]), cpu=str(ps[0]["cpu"]), total_wall_s=total,
                        mlups=ncase * n * n * steps / total / 1e6, **out)
    print("wrote", sweep_file(), "oracle %.2f MLUPS" % (ncase * n * n * steps / total / 1e6), flush=True)


def run_sweep(steps=40000, every=1000, part=0, parts=1):
    n = 256
    all_cases = inputs.laplace_sweep_cases(n)
    index = list(range(part, len(all_cases), parts))
    cases = [all_cases[i] for i in index]
    ncase = len(cases)
    nrec = steps // every + 1
    radius = np.full((ncase, nrec), np.nan)
    mass = np.full((ncase, nrec), np.nan)
    nsnap = len(SWEEP_SNAPS)
    rho_s = np.zeros((ncase, nsnap, n // 4, n // 4))
    row_c = np.zeros((ncase, nsnap, n))
    col_c = np.zeros((ncase, nsnap, n))
    meta = {k: np.zeros(ncase) for k in ("T_over_Tc", "T", "R", "slab_rows", "rho_l", "rho_g",
                                          "dp", "p_in", "p_out", "slab_rho_g", "slab_rho_l", "wall_s")}
    for i, case in enumerate(cases):
        tr = case["T_over_Tc"]
        T = coexist.temperature(tr)
        rg, rl, _ = coexist.maxwell(T)
        P = stepper.make_params(n, n, T, tau_nu=0.6)
        rho0 = stepper.init_density(P, bubbles=case["bubbles"], slab_rows=case["slab_rows"],
                                    rho_l=rl, rho_g=rg, W=5.0)
        f = stepper.init_populations(P, rho0)
        t0 = time.perf_counter()
        for k in range(nrec):
            if k > 0:
                rc = stepper.step(P, f, every)
                if rc != 0:
                    raise RuntimeError("case %d turned non-finite before step %d" % (i, k * every))
            rho = stepper.density(P, f)
            mass[i, k] = diagnostics.neumaier_sum(rho)
            if case["bubbles"]:
                radius[i, k] = diagnostics.bubble_radius(rho, rl, rg)
            if k * every in SWEEP_SNAPS:
                j = SWEEP_SNAPS.index(k * every)
                rho_s[i, j] = sample(rho)
                row_c[i, j] = rho[n // 2]
                col_c[i, j] = rho[:, n // 2]
        wall = time.perf_counter() - t0
        rho, _, _, p = stepper.macros(P, f)
        R = case["bubbles"][0][2] if case["bubbles"] else 0.0
        meta["T_over_Tc"][i], meta["T"][i], meta["R"][i] = tr, T, R
        meta["slab_rows"][i], meta["rho_l"][i], meta["rho_g"][i] = case["slab_rows"], rl, rg
        meta["wall_s"][i] = wall
        if case["bubbles"]:
            cx, cy, _ = case["bubbles"][0]
            dp, p_in, p_out = diagnostics.pressure_jump(p, (cx, cy), radius[i, -1], 5.0)
            meta["dp"][i], meta["p_in"][i], meta["p_out"][i] = dp, p_in, p_out
            meta["slab_rho_g"][i] = meta["slab_rho_l"][i] = np.nan
        else:
            g, l = diagnostics.slab_densities(rho, case["slab_rows"])
            meta["slab_rho_g"][i], meta["slab_rho_l"][i] = g, l
            meta["dp"][i] = meta["p_in"][i] = meta["p_out"][i] = np.nan
        print("sweep case %2d T/Tc %.1f R %4.0f slab %3d: %.1f s (%.2f MLUPS), radius %.6f, dp %.4e"
              % (i, tr, R, case["slab_rows"], wall, n * n * steps / wall / 1e6, radius[i, -1],
                 meta["dp"][i]), flush=True)
    total = float(np.sum(meta["wall_s"]))
    np.savez_compressed(
        sweep_file() if parts == 1 else part_file(part), case_index=np.array(index),
        steps=steps, every=every, stride=4, snap_steps=np.array(SWEEP_SNAPS), radius=radius, mass=mass,
        rho_sampled=rho_s.astype(np.float32), rho_centre_row=row_c, rho_centre_col=col_c,
        threads=stepper.threads(), cpu=cpu_model(), total_wall_s=total,
        mlups=ncase * n * n * steps / total / 1e6, **meta)
    print("wrote", sweep_file() if parts == 1 else part_file(part),
          "oracle %.2f MLUPS on %d threads" % (ncase * n * n * steps / total / 1e6, stepper.threads()), flush=True)


def run_collapse(delta, seed, steps=50000, every=100):
    nx, ny = 1024, 768
    T = coexist.temperature(0.6)
    rg, rl, _ = coexist.maxwell(T)
    P = stepper.make_params(nx, ny, T, walls=True, tau_nu=0.6)
    bub = [(511.5, 200.0, 120.0)]
    rho0 = stepper.init_density(P, bubbles=bub, rho_l=rl, rho_g=rg, W=5.0, delta=delta,
                                noise_amp=1e-3, seed=seed)
    f = stepper.init_populations(P, rho0)
    nrec = steps // every + 1
    radius = np.full(nrec, np.nan)
    mass = np.full(nrec, np.nan)
    block_wall_max = np.full(nrec - 1, np.nan)
    snaps, rows, cols = {}, {}, {}
    best, best_step = -np.inf, -1
    t0 = time.perf_counter()
    for k in range(nrec):
        if k > 0:
            rc, w = stepper.step_wall_pressure(P, f, every)
            if rc != 0:
                raise RuntimeError("collapse turned non-finite before step %d" % (k * every))
            block_wall_max[k - 1] = np.max(w)
            j = int(np.argmax(w))
            if w[j] > best:
                best, best_step = float(w[j]), (k - 1) * every + j
        rho = stepper.density(P, f)
        mass[k] = diagnostics.neumaier_sum(rho)
        radius[k] = diagnostics.bubble_radius(rho, rl, rg)
        if k * every in SNAP_STEPS:
            snaps[k * every] = sample(rho)
            rows[k * every] = rho[200].copy()
            cols[k * every] = rho[:, 511].copy()
        if k % 50 == 0:
            el = time.perf_counter() - t0
            print("collapse d=%.3f s=%d step %6d radius %.6f mass %.10e wall max %.6e (%.0f s)"
                  % (delta, seed, k * every, radius[k], mass[k], best, el), flush=True)
    wall = time.perf_counter() - t0
    out = collapse_file(delta, seed)
    np.savez_compressed(
        out, steps=steps, every=every, stride=4, delta=delta, seed=seed, T=T, T_over_Tc=0.6,
        rho_l=rl, rho_g=rg, bubble=np.array(bub[0]), noise_amp=1e-3, W=5.0, tau_nu=0.6,
        radius=radius, mass=mass, block_wall_p_max=block_wall_max, wall_p_max=best,
        wall_p_step=best_step, snap_steps=np.array(sorted(snaps)),
        snaps=np.stack([snaps[s] for s in sorted(snaps)]),
        snap_rows=np.stack([rows[s] for s in sorted(rows)]),
        snap_cols=np.stack([cols[s] for s in sorted(cols)]),
        threads=stepper.threads(), cpu=cpu_model(), total_wall_s=wall,
        mlups=nx * ny * steps / wall / 1e6)
    print("wrote", out, "oracle %.2f MLUPS on %d threads, %.0f s" % (nx * ny * steps / wall / 1e6,
                                                                    stepper.threads(), wall), flush=True)


def run_timing(max_steps):
    """Oracle MLUPS on the three parity workloads, on one thread and on all
    the threads of its OpenMP runtime: the 64 x 64 binary64 check case
    (10,000 steps, in full), one instance of the sweep (256 x 256, R = 40 at
    0.7 T_c) and the 1024 x 768 collapse, each for min(its steps, max_steps)
    steps (the full sweep and collapse runs are timed when their references
    are written)."""
    nthreads = stepper.threads()
    cases = []
    T7 = coexist.temperature(0.7)
    rg, rl, _ = coexist.maxwell(T7)
    P = stepper.make_params(64, 64, T7, tau_nu=0.8)
    cases.append(("64x64 periodic, binary64", P,
                  dict(bubbles=[(31.5, 31.5, 16.0)], rho_l=rl, rho_g=rg, W=2.0), 10000))
    P = stepper.make_params(256, 256, T7, tau_nu=0.6)
    cases.append(("256x256 sweep instance", P, dict(bubbles=[(127.5, 127.5, 40.0)], rho_l=rl, rho_g=rg, W=5.0),
                  min(40000, max_steps)))
    T6 = coexist.temperature(0.6)
    g6, l6, _ = coexist.maxwell(T6)
    P = stepper.make_params(1024, 768, T6, walls=True, tau_nu=0.6)
    cases.append(("1024x768 collapse", P, dict(bubbles=[(511.5, 200.0, 120.0)], rho_l=l6, rho_g=g6, W=5.0,
                                                delta=0.02, noise_amp=1e-3, seed=1), min(50000, max_steps)))
    for name, P, init, steps in cases:
        for th in (1, nthreads):
            stepper.set_threads(th)
            f = stepper.init_populations(P, stepper.init_density(P, **init))
            t0 = time.perf_counter()
            assert stepper.step(P, f, steps) == 0
            dt = time.perf_counter() - t0
            print("oracle timing: %s, %d steps, %d thread(s): %.1f s, %.2f MLUPS (%s)"
                  % (name, steps, th, dt, P.nx * P.ny * steps / dt / 1e6, cpu_model()), flush=True)
    stepper.set_threads(nthreads)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["sweep", "collapse", "merge-sweep", "timing"])
    ap.add_argument("--max-steps", type=int, default=2000)
    ap.add_argument("--part", type=int, default=0)
    ap.add_argument("--parts", type=int, default=1)
    ap.add_argument("--delta", type=float, default=0.02)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--out", default=HERE)
    a = ap.parse_args()
    global OUT_DIR
    OUT_DIR = a.out
    os.makedirs(OUT_DIR, exist_ok=True)
    if a.threads > 0:
        stepper.set_threads(a.threads)
    if a.what == "sweep":
        run_sweep(part=a.part, parts=a.parts)
    elif a.what == "merge-sweep":
        merge_sweep(a.parts)
    elif a.what == "timing":
        run_timing(a.max_steps)
    else:
        run_collapse(a.delta, a.seed)


if __name__ == "__main__":
    main()
