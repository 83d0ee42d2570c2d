"""Seeded synthetic inputs shared by the tests, the benchmark and the serving
loop.  Holds none of the method's arithmetic: only random layouts, request
traces and population perturbations, all from numpy generators with fixed
seeds.
"""
import math

import numpy as np

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
    """The Laplace-law and coexistence sweep on an n x n periodic grid: discs of
    radius {20, 30, 40, 50, 60} at T/Tc {0.6, 0.7, 0.8, 0.9} centred on
    ((n-1)/2, (n-1)/2), plus one flat liquid slab of n/2 rows per temperature."""
    c = 0.5 * (n - 1)
    cases = []
    for tr in (0.6, 0.7, 0.8, 0.9):
        for R in (20, 30, 40, 50, 60):
            cases.append({"T_over_Tc": tr, "bubbles": [(c, c, float(R))], "slab_rows": 0})
        cases.append({"T_over_Tc": tr, "bubbles": [], "slab_rows": n // 2})
    return cases


def request_trace(n_requests, seed, side_lo=64, side_hi=1024, steps_lo=5000, steps_hi=40000):
    """Served-batch requests: sides log-uniform with aspect ratio in {1, 4/3, 2}
    (both sides within [side_lo, side_hi]), a 50/50 mix of periodic stationary
    discs (R = 0.15-0.3 of the short side) and wall-bounded collapses (delta in
    [0.005, 0.03], centre at a third of the height), T/Tc in [0.6, 0.9], and a
    step count in [steps_lo, steps_hi].  Arrival times are not included."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_requests):
        aspect = [1.0, 4.0 / 3.0, 2.0][rng.integers(0, 3)]
        short = int(round(math.exp(rng.uniform(math.log(side_lo), math.log(side_hi / aspect)))))
        long_ = int(round(aspect * short))
        collapse = bool(rng.integers(0, 2))
        tr = float(rng.uniform(0.6, 0.9))
        steps = int(rng.integers(steps_lo, steps_hi + 1))
        if collapse:
            nx, ny = long_, short
            R = float(rng.uniform(0.15, 0.3)) * short
            y0 = ny / 3.0
            R = min(R, y0 - 6.0)
            req = {"id": k, "nx": nx, "ny": ny, "walls": True, "T_over_Tc": tr, "steps": steps,
                   "bubbles": [(0.5 * (nx - 1), y0, R)], "delta": float(rng.uniform(0.005, 0.03))}
        else:
            nx, ny = long_, short
            R = float(rng.uniform(0.15, 0.3)) * short
            req = {"id": k, "nx": nx, "ny": ny, "walls": False, "T_over_Tc": tr, "steps": steps,
                   "bubbles": [(0.5 * (nx - 1), 0.5 * (ny - 1), R)], "delta": 0.0}
        out.append(req)
    return out


def poisson_arrivals(n, rate, seed):
    """Arrival times (seconds) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))
