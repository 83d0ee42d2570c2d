"""Seeded synthetic inputs shared by the tests, the benchmark and the serving
loop, and the workload configurations (configs/c1 ... c5) they are built
from.  Holds none of the method's arithmetic: only configurations, random
layouts, request traces and population perturbations, all from numpy
generators with fixed seeds.
"""
import json
import math
import os

import numpy as np

CONFIG_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs")


def load_config(cid):
    """The workload configuration `cid` ("c1" ... "c5") from
    configs/<cid>_*.json: grid, boundaries, temperature, initial state, step
    count and what the run records."""
    names = [n for n in sorted(os.listdir(CONFIG_DIR)) if n.startswith(cid + "_") and n.endswith(".json")]
    if len(names) != 1:
        raise KeyError("no single configuration file for %r in %s" % (cid, CONFIG_DIR))
    with open(os.path.join(CONFIG_DIR, names[0])) as fh:
        return json.load(fh)


def config_instances(cfg):
    """The instances of a configuration as plain dicts (nx, ny, walls,
    T_over_Tc, tau_nu, eps, W, bubbles [(x, y, R)], slab_rows, delta,
    noise_amp, seed), each the configuration's defaults overridden by its own
    entries.  A "sweep" expands to the discs of every radius and then one slab
    at each temperature; "seeded_discs" places discs with
    non_overlapping_discs."""
    base = dict(cfg.get("defaults", {}))
    out = []
    if "sweep" in cfg:
        sw = cfg["sweep"]
        for case in _sweep_cases(sw, sw["nx"]):
            out.append({**base, "nx": sw["nx"], "ny": sw["ny"], **case})
    for inst in cfg.get("instances", []):
        e = {**base, **inst}
        b = e.get("bubbles", [])
        if isinstance(b, dict):
            sd = b["seeded_discs"]
            e["bubbles"] = non_overlapping_discs(e["nx"], e["ny"], sd["radii"], W=e["W"], seed=sd["seed"],
                                                 walls=e["walls"])
        else:
            e["bubbles"] = [tuple(float(v) for v in x) for x in b]
        out.append(e)
    return out


def _sweep_cases(sw, n):
    c = 0.5 * (n - 1)
    slab = sw["slab_rows"] * n // sw["ny"]
    cases = []
    for tr in sw["T_over_Tc"]:
        for R in sw["radii"]:
            cases.append({"T_over_Tc": float(tr), "bubbles": [(c, c, float(R))], "slab_rows": 0})
        cases.append({"T_over_Tc": float(tr), "bubbles": [], "slab_rows": slab})
    return cases


def random_populations(rho, seed, amp=0.3):
    """Populations (ny, nx, 9) whose sum is close to the density field rho:
    f_a = rho / 9 * (1 + amp * U(-1, 1)), independently per site and direction.
    A generic state for one-step comparisons, not an equilibrium."""
    rng = np.random.default_rng(seed)
    f = np.repeat(rho[:, :, None] / 9.0, 9, axis=2)
    return f * (1.0 + amp * rng.uniform(-1.0, 1.0, f.shape))


def non_overlapping_discs(nx, ny, radii, W, seed, walls=True, max_tries=100000):
    """Centres for discs of the given radii, at least R_i + R_j + 4W apart and,
    with walls, at least R_i + 2W from the rows y = 0 and y = ny - 1; x is
    periodic, so distances in x wrap."""
    rng = np.random.default_rng(seed)
    placed = []
    for R in radii:
        for _ in range(max_tries):
            x = rng.uniform(0, nx)
            lo, hi = (R + 2 * W, ny - 1 - R - 2 * W) if walls else (0, ny)
            if hi <= lo:
                raise ValueError("disc does not fit")
            y = rng.uniform(lo, hi)
            ok = True
            for (px, py, pr) in placed:
                dx = abs(x - px)
                dx = min(dx, nx - dx)
                if math.hypot(dx, y - py) < R + pr + 4 * W:
                    ok = False
                    break
            if ok:
                placed.append((x, y, float(R)))
                break
        else:
            raise ValueError("could not place disc of radius %g" % R)
    return placed


def laplace_sweep_cases(n=256):
    """The Laplace-law and coexistence sweep of configuration c2 on an n x n
    periodic grid: discs of every radius at every temperature, centred on
    ((n-1)/2, (n-1)/2), plus one flat liquid slab (the configured share of the
    rows) per temperature."""
    return _sweep_cases(load_config("c2")["sweep"], n)


def request_trace(n_requests=None, seed=None, side_lo=None, side_hi=None, steps_lo=None, steps_hi=None):
    """Served-batch requests of configuration c4 (any argument given overrides
    it): sides log-uniform with the aspect ratio drawn from the configured set
    (both sides within [side_lo, side_hi]), a 50/50 mix of periodic stationary
    discs and wall-bounded collapses (centre at a third of the height), the
    radius a uniform share of the short side, delta, T/Tc and the step count
    uniform in their configured ranges.  Arrival times are not included."""
    tr = load_config("c4")["trace"]
    n_requests = tr["n_requests"] if n_requests is None else n_requests
    seed = tr["seed"] if seed is None else seed
    side_lo = tr["side_lo"] if side_lo is None else side_lo
    side_hi = tr["side_hi"] if side_hi is None else side_hi
    steps_lo = tr["steps_lo"] if steps_lo is None else steps_lo
    steps_hi = tr["steps_hi"] if steps_hi is None else steps_hi
    aspects = tr["aspects"]
    t_lo, t_hi = tr["T_over_Tc"]
    r_lo, r_hi = tr["radius_of_short_side"]
    d_lo, d_hi = tr["delta"]
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_requests):
        aspect = aspects[rng.integers(0, len(aspects))]
        short = int(round(math.exp(rng.uniform(math.log(side_lo), math.log(side_hi / aspect)))))
        long_ = int(round(aspect * short))
        collapse = bool(rng.integers(0, 2))
        trr = float(rng.uniform(t_lo, t_hi))
        steps = int(rng.integers(steps_lo, steps_hi + 1))
        if collapse:
            nx, ny = long_, short
            R = float(rng.uniform(r_lo, r_hi)) * short
            y0 = ny / 3.0
            R = min(R, y0 - 6.0)
            req = {"id": k, "nx": nx, "ny": ny, "walls": True, "T_over_Tc": trr, "steps": steps,
                   "bubbles": [(0.5 * (nx - 1), y0, R)], "delta": float(rng.uniform(d_lo, d_hi))}
        else:
            nx, ny = long_, short
            R = float(rng.uniform(r_lo, r_hi)) * short
            req = {"id": k, "nx": nx, "ny": ny, "walls": False, "T_over_Tc": trr, "steps": steps,
                   "bubbles": [(0.5 * (nx - 1), 0.5 * (ny - 1), R)], "delta": 0.0}
        out.append(req)
    return out


def poisson_arrivals(n, rate, seed):
    """Arrival times (seconds) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))
