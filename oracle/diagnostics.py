"""Post-processing of density and pressure fields, in float64 numpy.

Test infrastructure only (see oracle/__init__.py).  The paper defines the
pressure jump of the Laplace law (Eq. 17) but not how a radius or the two
pressures are sampled from a diffuse interface; the readings used here are:

  radius  -- area-equivalent radius sqrt(A / pi), A = sum of the gas fraction
             clip((rho_l - rho) / (rho_l - rho_g), 0, 1) over the nodes; with
             several bubbles each node counts for the nearest initial centre
             (the reading has no value in the paper to compare against; the
             code is pinned to gas regions of known area)
  p_in    -- mean pressure over nodes closer than R - 2W to the centre
  p_out   -- mean pressure over nodes farther than R + 2W from the centre
  slab    -- densities averaged over the 17 central rows of each phase

The pressure jump is reported as p_in - p_out, positive for a gas bubble (Eq. 17
writes the opposite difference; its magnitude sigma / r is what is fitted).
"""
import math

import numpy as np


def neumaier_sum(values):
    """Compensated sum (Neumaier's variant of Kahan summation), fixed order."""
    s = 0.0
    c = 0.0
    for v in np.asarray(values, dtype=np.float64).ravel():
        t = s + v
        if abs(s) >= abs(v):
            c += (s - t) + v
        else:
            c += (v - t) + s
        s = t
    return s + c


def gas_fraction(rho, rho_l, rho_g):
    return np.clip((rho_l - rho) / (rho_l - rho_g), 0.0, 1.0)


def bubble_radius(rho, rho_l, rho_g):
    return math.sqrt(float(np.sum(gas_fraction(rho, rho_l, rho_g))) / math.pi)


def bubble_radii(rho, centres, rho_l, rho_g):
    """Per-bubble radii, each node counted for the nearest initial centre."""
    ny, nx = rho.shape
    yy, xx = np.mgrid[0:ny, 0:nx]
    d2 = np.stack([(xx - cx) ** 2 + (yy - cy) ** 2 for cx, cy in centres])
    owner = np.argmin(d2, axis=0)
    frac = gas_fraction(rho, rho_l, rho_g)
    return [math.sqrt(float(np.sum(frac[owner == k])) / math.pi) for k in range(len(centres))]


def pressure_jump(p, centre, R, W):
    """(p_in - p_out, p_in, p_out) around a bubble of radius R."""
    ny, nx = p.shape
    yy, xx = np.mgrid[0:ny, 0:nx]
    r = np.hypot(xx - centre[0], yy - centre[1])
    p_in = float(np.mean(p[r < R - 2 * W]))
    p_out = float(np.mean(p[r > R + 2 * W]))
    return p_in - p_out, p_in, p_out


def slab_densities(rho, slab_rows):
    """(rho_g, rho_l) of a liquid slab of slab_rows rows centred on (ny-1)/2,
    each averaged over the 17 rows at the middle of its phase."""
    ny = rho.shape[0]
    prof = rho.mean(axis=1)
    yc = 0.5 * (ny - 1)
    liquid_mid = int(round(yc))
    gas_mid = int(round(yc + 0.5 * ny)) % ny
    rows_l = [(liquid_mid + k) % ny for k in range(-8, 9)]
    rows_g = [(gas_mid + k) % ny for k in range(-8, 9)]
    return float(np.mean(prof[rows_g])), float(np.mean(prof[rows_l]))


def laplace_fit(radii, jumps):
    """Least-squares line dp = sigma / R + c; returns (sigma, c, r^2)."""
    x = 1.0 / np.asarray(radii, dtype=np.float64)
    y = np.asarray(jumps, dtype=np.float64)
    A = np.vstack([x, np.ones_like(x)]).T
    (sigma, c), *_ = np.linalg.lstsq(A, y, rcond=None)
    yfit = sigma * x + c
    ss_res = float(np.sum((y - yfit) ** 2))
    ss_tot = float(np.sum((y - y.mean()) ** 2))
    return float(sigma), float(c), 1.0 - ss_res / ss_tot
