"""Pins of the oracle's equation of state and coexistence solvers against the
numbers the paper prints and against independent evaluation routes."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import coexist, stepper


def _cs_pressure(rho, T, a=0.5, eta_per_rho=1.0, R=1.0):
    eta = eta_per_rho * rho
    return rho * R * T * (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3 - a * rho ** 2


def test_critical_density_matches_printed(paper_values):
    val, unit, _ = paper_values["rho_c"]
    Tc, rho_c, pc = coexist.critical_point()
    assert abs(rho_c - val) <= unit
    # first and second derivatives of Eq. 15 vanish there: the closed-form p'
    # and a central difference of it
    h = 1e-5
    p = lambda r: _cs_pressure(r, Tc)
    d1 = _dpdrho(rho_c, Tc)
    d2 = (_dpdrho(rho_c + h, Tc) - _dpdrho(rho_c - h, Tc)) / (2 * h)
    assert abs(d1) < 1e-13 and abs(d2) < 1e-8
    assert math.isclose(pc, p(rho_c), rel_tol=1e-12)


def test_literal_b1_contradicts_printed_critical_density(paper_values):
    """Reading of Eq. 15's b: with b = 1 as printed the critical density is four
    times the printed one, so b = 4 (eta = rho) is used."""
    _, rho_c_b1, _ = coexist.critical_point(b=1.0)
    val, unit, _ = paper_values["rho_c"]
    assert abs(rho_c_b1 - 4 * 0.1304438842) < 1e-6
    assert abs(rho_c_b1 - val) > 100 * unit


def test_maxwell_matches_printed_half_Tc(paper_values, coexistence_table):
    rg, rl, p0 = coexist.maxwell(coexist.temperature(0.5))
    val_l, unit_l, _ = paper_values["rho_l_half_Tc"]
    val_g, _, _ = paper_values["rho_g_half_Tc"]
    assert abs(rl - val_l) <= unit_l
    # the printed vapour density is a simulation result near the Maxwell value
    assert abs(rg - val_g) / val_g < 1e-3
    assert rl / rg > paper_values["density_ratio_min"][0]
    row = coexistence_table[0.5]["maxwell"]
    assert np.allclose((rg, rl, p0), row, rtol=1e-10)


def _chemical_potential(rho, T, a=0.5, R=1.0):
    """Closed-form chemical potential of the CS fluid with eta = rho:
    mu = RT [ln rho + (8 eta - 9 eta^2 + 3 eta^3) / (1 - eta)^3] - 2 a rho."""
    eta = rho
    return R * T * (math.log(rho) + (8 * eta - 9 * eta ** 2 + 3 * eta ** 3) / (1 - eta) ** 3) - 2 * a * rho


@pytest.mark.parametrize("tr", [0.5, 0.6, 0.7, 0.8, 0.9])
def test_maxwell_equal_chemical_potential(tr, coexistence_table):
    row = coexistence_table[tr]
    rg, rl, p0 = row["maxwell"]
    T = row["T"]
    assert math.isclose(_cs_pressure(rg, T), p0, rel_tol=1e-9)
    # the liquid pressure is a difference of O(0.1) terms: compare on that scale
    assert abs(_cs_pressure(rl, T) - p0) < 1e-12
    mg, ml = _chemical_potential(rg, T), _chemical_potential(rl, T)
    assert abs(mg - ml) < 1e-11 * abs(mg)


def _dpdrho(rho, T, a=0.5, R=1.0):
    """Closed-form derivative of Eq. 15 with eta = rho."""
    e = rho
    return R * T * (1 + 4 * e + 4 * e ** 2 - 4 * e ** 3 + e ** 4) / (1 - e) ** 4 - 2 * a * rho


@pytest.mark.parametrize("tr,eps", [(0.6, 1.86), (0.7, 1.0), (0.8, 0.0), (0.9, 2.0)])
def test_mechanical_stability_by_parts(tr, eps, coexistence_table):
    """Eq. 9 integrated by parts: the boundary terms vanish, leaving
    int p'(rho) psi^(-eps) drho = 0 (or int p' ln psi drho = 0 at eps = 0).
    Checked with scipy quadrature and the closed-form p', so it shares no step
    with the multiprecision solver."""
    row = coexistence_table[tr]
    T = row["T"]
    rg, rl = row[("eq9", eps)]
    ps = lambda r: math.sqrt(2 * (r / 3 - _cs_pressure(r, T)))
    if eps == 0.0:
        g = lambda r: _dpdrho(r, T) * math.log(ps(r))
    else:
        g = lambda r: _dpdrho(r, T) * ps(r) ** (-eps)
    sg, sl = row["spinodal"]
    val = sum(integrate.quad(g, lo, hi, limit=200, epsabs=0, epsrel=1e-12)[0]
              for lo, hi in ((rg, sg), (sg, sl), (sl, rl)))
    scale = sum(integrate.quad(lambda r: abs(g(r)), lo, hi, limit=200)[0]
                for lo, hi in ((rg, sg), (sg, sl), (sl, rl)))
    assert abs(val) < 1e-8 * scale


def test_eps_one_lowest_temperature_is_near_0p7(coexistence_table):
    """Section 3.1: with eps = 1.0 the lowest reachable reduced temperature is
    about 0.7 T_c.  Eq. 9 has a solution at 0.7 T_c and none below."""
    assert coexistence_table[0.7][("eq9", 1.0)] is not None
    assert coexistence_table[0.6][("eq9", 1.0)] is None
    assert coexistence_table[0.5][("eq9", 1.0)] is None


def test_eps_1p86_tracks_maxwell_liquid_branch(coexistence_table):
    """Section 3.1: with eps = 1.86 the coexistence curve agrees well with the
    Maxwell construction; the liquid branch agrees to 0.05 % from 0.5 to 0.9 T_c
    and the gas branch to 20 % at 0.5 T_c and 1 % from 0.7 T_c up."""
    for tr, row in coexistence_table.items():
        g, l = row[("eq9", 1.86)]
        mg, ml, _ = row["maxwell"]
        assert abs(l - ml) / ml < 5e-4
        assert abs(g - mg) / mg < (0.2 if tr < 0.7 else 0.01)


@pytest.mark.slow
def test_table_regenerates_from_oracle(coexistence_table):
    row = coexistence_table[0.7]
    T = coexist.temperature(0.7)
    assert math.isclose(T, row["T"], rel_tol=1e-11)
    g, l = coexist.mechanical_stability(T, 1.86)[:2]
    assert np.allclose((g, l), row[("eq9", 1.86)], rtol=1e-9)


def test_c_oracle_eos_and_psi_match_definitions():
    """The C oracle's Eq. 15 against the multiprecision one, and Eq. 13's psi
    inserted in Eq. 10 (p = rho c_s^2 + G c^2 psi^2 / 2) gives back p_EOS."""
    T = coexist.temperature(0.7)
    P = stepper.make_params(4, 4, T)
    for rho in (1e-3, 0.01, 0.0931, 0.2, 0.35, 0.45):
        p = stepper.eos_pressure(P, rho)
        assert math.isclose(p, float(coexist.eos_pressure(rho, T)), rel_tol=1e-13, abs_tol=1e-18)
        psi = stepper.psi(P, rho)
        assert math.isclose(rho / 3.0 + (-1.0) * psi ** 2 / 2.0, p, rel_tol=1e-12, abs_tol=1e-16)


def test_psi_is_nan_near_the_pole():
    """Close below the EOS pole (eta -> 1) p_EOS grows without bound, psi^2 of
    Eq. 13 turns negative and the oracle propagates NaN instead of clamping."""
    T = coexist.temperature(0.7)
    P = stepper.make_params(4, 4, T)
    assert math.isnan(stepper.psi(P, 0.99))
    assert not math.isnan(stepper.psi(P, 0.45))
