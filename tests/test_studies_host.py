"""Host-side helpers of the experiment drivers (CPU only): the gas-region
shape analysis, the slab sampling and the liquid density for a prescribed
pressure, each against values computed independently here or by the
oracle."""
import math

import numpy as np
import pytest

from paper_1605_01800_amd import studies


def test_gas_shape_counts_components_across_the_periodic_edge():
    rho = np.full((40, 60), 0.45)
    rho[10:20, 0:3] = 0.001          # one disc cut by the x edge ...
    rho[10:20, 57:60] = 0.001        # ... continues here
    rho[30:35, 28:33] = 0.001        # a second one
    s = studies.gas_shape(rho, 0.2, x_c=30, y_c=32, dy=2)
    assert s["components"] == 2
    assert s["gas_columns"] == 3 + 3 + 5
    assert s["gas_rows"] == 10 + 5
    assert s["neck_rows"] == 5
    assert s["waist"] == 5 and s["lobes"] == 5
    assert s["gas_radius"] == pytest.approx(math.sqrt((60 + 25) / math.pi))
    assert s["rho_max"] == 0.45


def test_gas_shape_dumbbell_waist():
    y, x = np.mgrid[0:61, 0:81]
    gas = ((x - 40) ** 2 / 15 ** 2 + (y - 15) ** 2 / 12 ** 2 < 1) | ((x - 40) ** 2 / 15 ** 2 + (y - 45) ** 2 / 12 ** 2 < 1)
    gas |= (abs(x - 40) <= 2) & (abs(y - 30) <= 4)
    rho = np.where(gas, 0.001, 0.45)
    s = studies.gas_shape(rho, 0.2, x_c=40, y_c=30, dy=15)
    assert s["components"] == 1
    assert s["waist"] == 5 and s["lobes"] == 29


def test_slab_densities_sample_the_centres():
    ny, nx = 64, 8
    prof = np.where(np.abs(np.arange(ny) - 31.5) < 16, 0.4, 0.01)
    rho = np.tile(prof[:, None], (1, nx))
    rl, rg = studies._slab_densities(rho)
    assert rl == pytest.approx(0.4) and rg == pytest.approx(0.01)


def test_cs_pressure_matches_the_oracle():
    from oracle import build, coexist, stepper
    build.ensure_built()
    T = coexist.temperature(0.6)
    P = stepper.make_params(4, 4, T)
    rho = np.array([1e-3, 0.05, 0.13, 0.3, 0.45])
    ref = stepper.eos_pressure(P, rho)
    assert np.allclose(studies.cs_pressure(rho, T), ref, rtol=1e-13, atol=1e-17)


def test_liquid_density_for_pressure_is_on_the_liquid_branch():
    from oracle import coexist
    T = coexist.temperature(0.5)
    g, l, p0 = coexist.maxwell(T)
    rho = studies.liquid_density_for_pressure(T, p0)
    assert rho == pytest.approx(l, rel=1e-9)
    rho2 = studies.liquid_density_for_pressure(T, p0 - 1e-3)
    assert rho2 < l and abs(studies.cs_pressure(rho2, T) - (p0 - 1e-3)) < 1e-13
    s_g, s_l = coexist.spinodals(T)
    assert rho2 > s_l
