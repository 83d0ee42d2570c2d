"""Pins of the oracle's post-processing (oracle/diagnostics.py) against values
fixed by elementary geometry and arithmetic, not by the functions' own
formulas: the area-equivalent radius of gas regions whose area is known
(squares and rectangles of whole sites), fractional gas sites, the clip of
over- and under-shooting densities, nearest-centre ownership of several
bubbles, the compensated sum against math.fsum, the pressure jump of a step
field and the Laplace fit of exact lines.

The radius reading (the paper defines none): R = sqrt(A / pi), with A the sum
over sites of the gas fraction clip((rho_l - rho) / (rho_l - rho_g), 0, 1).

The module under test is oracle.diagnostics, or the file that the
ORACLE_DIAGNOSTICS environment variable names (the mutation tests load copies
with a planted mistake this way).
"""
import importlib.util
import math
import os

import numpy as np
import pytest

from oracle import diagnostics as _faithful


def _module():
    path = os.environ.get("ORACLE_DIAGNOSTICS")
    if not path:
        return _faithful
    spec = importlib.util.spec_from_file_location("diagnostics_under_test", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


D = _module()

RHO_L, RHO_G = 0.3581309, 9.294146e-3        # Maxwell densities at 0.7 T_c


def _field(ny, nx, value=RHO_L):
    return np.full((ny, nx), value, dtype=np.float64)


def test_sharp_square_has_the_radius_of_its_area():
    # 12 x 12 gas sites: A = 144, R = 12 / sqrt(pi)
    rho = _field(64, 80)
    rho[20:32, 30:42] = RHO_G
    assert D.bubble_radius(rho, RHO_L, RHO_G) == pytest.approx(12.0 / math.sqrt(math.pi), rel=1e-14)


def test_sharp_rectangle_and_single_site():
    rho = _field(40, 50)
    rho[5:8, 10:37] = RHO_G                       # 3 x 27 = 81 sites
    assert D.bubble_radius(rho, RHO_L, RHO_G) == pytest.approx(9.0 / math.sqrt(math.pi), rel=1e-14)
    one = _field(8, 8)
    one[3, 4] = RHO_G
    assert D.bubble_radius(one, RHO_L, RHO_G) == pytest.approx(1.0 / math.sqrt(math.pi), rel=1e-14)
    assert D.bubble_radius(_field(8, 8), RHO_L, RHO_G) == 0.0


def test_half_density_counts_half_a_site():
    # every site at the mid density is half gas: A = nx ny / 2
    mid = 0.5 * (RHO_L + RHO_G)
    rho = _field(30, 42, mid)
    assert D.bubble_radius(rho, RHO_L, RHO_G) == pytest.approx(math.sqrt(30 * 42 / 2 / math.pi), rel=1e-13)
    # a quarter of the way from the liquid: a quarter of a site each
    q = RHO_L - 0.25 * (RHO_L - RHO_G)
    rho = _field(16, 16, q)
    assert D.bubble_radius(rho, RHO_L, RHO_G) == pytest.approx(math.sqrt(64 / math.pi), rel=1e-13)


def test_overshooting_densities_are_clipped():
    # compressed liquid (rho > rho_l) adds no negative area, and vapour below
    # rho_g adds no more than one site each: same radius as the sharp square
    rho = _field(64, 64, RHO_L * 1.02)
    rho[10:20, 10:20] = 0.5 * RHO_G
    assert D.bubble_radius(rho, RHO_L, RHO_G) == pytest.approx(10.0 / math.sqrt(math.pi), rel=1e-14)
    f = D.gas_fraction(np.array([RHO_L * 1.5, RHO_L, RHO_G, 0.1 * RHO_G]), RHO_L, RHO_G)
    assert f.tolist() == [0.0, 0.0, 1.0, 1.0]


def test_each_site_counts_for_the_nearest_centre():
    # two gas squares, 6 x 6 around (14.5, 20.5) and 4 x 4 around (45.5, 20.5);
    # the centres passed are the squares' centres
    rho = _field(48, 64)
    rho[18:24, 12:18] = RHO_G
    rho[19:23, 44:48] = RHO_G
    r = D.bubble_radii(rho, [(14.5, 20.5), (45.5, 20.5)], RHO_L, RHO_G)
    assert r[0] == pytest.approx(6.0 / math.sqrt(math.pi), rel=1e-14)
    assert r[1] == pytest.approx(4.0 / math.sqrt(math.pi), rel=1e-14)
    # a gas column at x = 28 is nearer the first centre (13.5 columns) than the
    # second (17.5), one at x = 33 nearer the second (12.5 against 18.5)
    rho[0:5, 28] = RHO_G
    rho[0:3, 33] = RHO_G
    r = D.bubble_radii(rho, [(14.5, 20.5), (45.5, 20.5)], RHO_L, RHO_G)
    assert r[0] == pytest.approx(math.sqrt(41 / math.pi), rel=1e-14)
    assert r[1] == pytest.approx(math.sqrt(19 / math.pi), rel=1e-14)
    # one centre: the same as the whole-field radius
    assert D.bubble_radii(rho, [(30.0, 30.0)], RHO_L, RHO_G)[0] == pytest.approx(
        D.bubble_radius(rho, RHO_L, RHO_G), rel=1e-15)


def test_ownership_uses_both_coordinates():
    # centres stacked in y: a square above sits with the upper centre
    rho = _field(60, 20)
    rho[40:45, 8:13] = RHO_G
    r = D.bubble_radii(rho, [(10.0, 10.0), (10.0, 42.0)], RHO_L, RHO_G)
    assert r[0] == 0.0
    assert r[1] == pytest.approx(5.0 / math.sqrt(math.pi), rel=1e-14)


def test_compensated_sum_matches_exact_summation():
    # cancellations that a plain or Kahan sum loses entirely
    for vals in ([1.0, 1e100, 1.0, -1e100], [1e16, 1.0, -1e16], [3.0, 1e17, -1e17, 0.5]):
        assert D.neumaier_sum(vals) == math.fsum(vals)
    rng = np.random.default_rng(7)
    v = rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000)
    assert D.neumaier_sum(v) == pytest.approx(math.fsum(v.tolist()), rel=1e-15, abs=1e-15)
    # a density field: the mass of 64 x 64 sites of 0.3581309
    m = D.neumaier_sum(_field(64, 64))
    assert m == pytest.approx(math.fsum([RHO_L] * 4096), rel=1e-16)


def test_pressure_jump_of_a_step_field():
    # p = 1 inside radius 20, 0 outside: p_in - p_out = 1, sampled away from
    # the interface (r < R - 2W inside, r > R + 2W outside)
    ny, nx = 101, 101
    yy, xx = np.mgrid[0:ny, 0:nx]
    r = np.hypot(xx - 50.0, yy - 50.0)
    p = np.where(r < 20.0, 1.0, 0.0) + 0.25
    dp, p_in, p_out = D.pressure_jump(p, (50.0, 50.0), 20.0, 5.0)
    assert (dp, p_in, p_out) == (1.0, 1.25, 0.25)
    # the band R - 2W <= r <= R + 2W is left out: values there do not count
    p[(r >= 10.0) & (r <= 30.0)] = 100.0
    assert D.pressure_jump(p, (50.0, 50.0), 20.0, 5.0)[0] == 1.0


def test_slab_densities_of_a_two_phase_profile():
    # liquid in the middle half of the rows, gas elsewhere; the 17 central
    # rows of each phase are away from the interfaces
    ny, nx = 128, 8
    rho = np.full((ny, nx), RHO_G)
    rho[32:96, :] = RHO_L
    g, l = D.slab_densities(rho, 64)
    assert g == pytest.approx(RHO_G, rel=1e-15) and l == pytest.approx(RHO_L, rel=1e-15)
    # a gas row inside the liquid's 17 central rows, or a liquid row inside
    # the gas's, moves the averages by 1/17 of the density difference
    rho[64, :] = RHO_G
    rho[0, :] = RHO_L
    g, l = D.slab_densities(rho, 64)
    assert l == pytest.approx(RHO_L - (RHO_L - RHO_G) / 17, rel=1e-14)
    assert g == pytest.approx(RHO_G + (RHO_L - RHO_G) / 17, rel=1e-14)


def test_laplace_fit_of_exact_lines():
    R = np.array([20.0, 30.0, 40.0, 50.0])
    sigma, c, r2 = D.laplace_fit(R, 0.01 / R + 2e-5)
    assert sigma == pytest.approx(0.01, rel=1e-12)
    assert c == pytest.approx(2e-5, rel=1e-9)
    assert r2 == pytest.approx(1.0, abs=1e-12)
