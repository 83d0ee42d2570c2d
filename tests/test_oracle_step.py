"""Whole-step pins of the oracle: invariants, symmetry, an independent BGK
stepper in the equal-rate limit, the initial state of Eq. 16 and the noise
generator."""
import math

import numpy as np
import pytest

from oracle import coexist, diagnostics, stepper

E = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
WF = np.array([0] + [1 / 3] * 4 + [1 / 12] * 4)
T07 = coexist.temperature(0.7)
RG07, RL07, _ = coexist.maxwell(T07)


def _bubble(nx, ny, T, R, walls=False, W_=5.0, **kw):
    P = stepper.make_params(nx, ny, T, walls=walls, **kw)
    rg, rl, _ = coexist.maxwell(T)
    rho = stepper.init_density(P, bubbles=[(0.5 * (nx - 1), 0.5 * (ny - 1), R)],
                               rho_l=rl, rho_g=rg, W=W_)
    return P, stepper.init_populations(P, rho)


@pytest.mark.parametrize("walls", [False, True])
def test_uniform_state_is_a_fixed_point(walls):
    P = stepper.make_params(9, 7, T07, walls=walls)
    f = stepper.init_populations(P, np.full((7, 9), 0.2))
    f0 = f.copy()
    assert stepper.step(P, f, 50) == 0
    # bitwise identical across nodes (translation invariance) ...
    assert np.all(f == f[0, 0][None, None, :])
    # ... and equal to the start up to rounding
    assert np.allclose(f, f0, rtol=1e-14, atol=0)


@pytest.mark.parametrize("walls", [False, True])
def test_mass_is_conserved(walls):
    P, f = _bubble(40, 36, T07, 9, walls=walls, tau_nu=0.8)
    m0 = diagnostics.neumaier_sum(stepper.density(P, f))
    assert stepper.step(P, f, 1500) == 0
    m1 = diagnostics.neumaier_sum(stepper.density(P, f))
    assert abs(m1 - m0) / m0 < 1e-13


def test_total_momentum_stays_zero_on_periodic_grid():
    """The pairwise force sums to zero and the collision adds exactly F, so
    the total momentum of a periodic system stays at its initial value, 0."""
    P, f = _bubble(40, 34, T07, 9, tau_nu=0.6)
    rng = np.random.default_rng(2)
    f *= 1 + 1e-3 * rng.standard_normal(f.shape)     # break the symmetry
    j0 = np.einsum("yxa,ad->d", f, E)
    assert stepper.step(P, f, 800) == 0
    rho, vx, vy, _ = stepper.macros(P, f)
    # rho v = j + F/2 and sum F = 0, so sum rho v is the total momentum
    mom = np.array([np.sum(rho * vx), np.sum(rho * vy)])
    assert np.all(np.abs(mom - j0) < 1e-13)


@pytest.mark.parametrize("walls", [False, True])
def test_centred_bubble_keeps_mirror_symmetry(walls):
    nx, ny = 34, 30
    P, f = _bubble(nx, ny, T07, 8, walls=walls, tau_nu=0.8)
    assert stepper.step(P, f, 600) == 0
    rho = stepper.density(P, f)
    assert np.allclose(rho, rho[:, ::-1], rtol=0, atol=1e-13)
    assert np.allclose(rho, rho[::-1, :], rtol=0, atol=1e-13)
    if not walls:
        # a square-symmetric start on a square grid stays symmetric under x <-> y
        P2, f2 = _bubble(30, 30, T07, 8, tau_nu=0.8)
        stepper.step(P2, f2, 600)
        r2 = stepper.density(P2, f2)
        assert np.allclose(r2, r2.T, rtol=0, atol=1e-13)


def _cs_pressure(rho, T):
    eta = rho
    return rho * T * (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3 - 0.5 * rho ** 2


def _bgk_guo_step(f, T, tau):
    """Independent velocity-space stepper: BGK collision with Guo's forcing,
    psi from the CS pressure, the force with numpy rolls, streaming with rolls
    (periodic)."""
    rho = f.sum(axis=2)
    psi = np.sqrt(2 * (rho / 3 - _cs_pressure(rho, T)))
    Fx = np.zeros_like(rho)
    Fy = np.zeros_like(rho)
    for a in range(1, 9):
        nb = np.roll(psi, shift=(-E[a, 1], -E[a, 0]), axis=(0, 1))
        Fx += WF[a] * nb * E[a, 0]
        Fy += WF[a] * nb * E[a, 1]
    Fx *= psi
    Fy *= psi
    vx = (f @ E[:, 0] + 0.5 * Fx) / rho
    vy = (f @ E[:, 1] + 0.5 * Fy) / rho
    out = np.empty_like(f)
    for a in range(9):
        eu = E[a, 0] * vx + E[a, 1] * vy
        feq = W[a] * rho * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (vx ** 2 + vy ** 2))
        eF = E[a, 0] * Fx + E[a, 1] * Fy
        guo = W[a] * (3 * ((E[a, 0] - vx) * Fx + (E[a, 1] - vy) * Fy) + 9 * eu * eF)
        post = f[:, :, a] - (f[:, :, a] - feq) / tau + (1 - 0.5 / tau) * guo
        out[:, :, a] = np.roll(post, shift=(E[a, 1], E[a, 0]), axis=(0, 1))
    return out


def test_whole_steps_equal_independent_bgk_stepper_at_equal_rates():
    """At 0.9 T_c, where the eps = 0 scheme has a coexistence solution."""
    tau = 0.9
    nx, ny = 26, 22
    T = coexist.temperature(0.9)
    rg, rl, _ = coexist.maxwell(T)
    P = stepper.make_params(nx, ny, T, eps=0.0, s=[1 / tau] * 9)
    rho = stepper.init_density(P, bubbles=[(11.0, 10.5, 6.0)], rho_l=rl, rho_g=rg, W=3.0)
    f = stepper.init_populations(P, rho)
    g = f.copy()
    for _ in range(60):
        g = _bgk_guo_step(g, T, tau)
    assert stepper.step(P, f, 60) == 0
    assert np.max(np.abs(f - g)) < 1e-14


def test_initial_density_follows_eq16():
    nx, ny = 41, 37
    P = stepper.make_params(nx, ny, T07)
    x0, y0, r0, Wd = 20.0, 18.0, 9.0, 5.0
    rho = stepper.init_density(P, bubbles=[(x0, y0, r0)], rho_l=RL07, rho_g=RG07, W=Wd)
    yy, xx = np.mgrid[0:ny, 0:nx]
    r = np.hypot(xx - x0, yy - y0)
    # exactly at r = r0: the mean of the two densities; the tanh is odd around r0
    assert rho[18, 29] == pytest.approx(0.5 * (RL07 + RG07), abs=1e-16)
    assert rho[18, 20] == pytest.approx(RG07 + (RL07 - RG07) * 0.5 * (1 + math.tanh(-2 * 9 / 5)), rel=1e-14)
    assert np.all(np.diff(rho[18, 20:]) > 0)
    assert rho.max() < RL07 and rho.min() > RG07
    # rest-state populations: f_a = w_a rho, no momentum
    f = stepper.init_populations(P, rho)
    assert np.allclose(f.sum(axis=2), rho, rtol=1e-15)
    assert np.allclose(f @ E, 0, atol=1e-18)


def test_liquid_overpressure_and_slab():
    P = stepper.make_params(8, 128, T07)
    rho = stepper.init_density(P, slab_rows=64, rho_l=RL07, rho_g=RG07, W=5.0, delta=0.02)
    rg, rl = diagnostics.slab_densities(rho, 64)
    assert rl == pytest.approx(RL07 * 1.02, rel=1e-6)
    assert rg == pytest.approx(RG07, rel=1e-6)
    assert rho[0, 0] == rho[0, 7] and rho[63, 0] > rho[0, 0]


def test_splitmix64_reference_outputs():
    """SplitMix64 seeded with 0: its first three outputs are the published
    values 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f; the
    k-th output is the hash of 0 + (k-1) * golden gamma, i.e. the oracle's
    uniform deviate of index (k-1) * 0x9E3779B97F4A7C15 with seed 0."""
    g = 0x9E3779B97F4A7C15
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    for k, w in enumerate(want):
        u = stepper.uniform(0, (k * g) & (2 ** 64 - 1))
        assert u == (w >> 11) * 2.0 ** -53


def _splitmix64(s):
    """One SplitMix64 output from state s (Steele, Lea and Flood, 2014),
    written here from its published definition, apart from the oracle's."""
    m = 2 ** 64 - 1
    z = (s + 0x9E3779B97F4A7C15) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def test_noise_of_each_site_uses_its_row_major_index():
    """The noise reading: site (x, y) is scaled by 1 + amp (2u - 1), u the
    SplitMix64 deviate of seed XOR (y nx + x) taken to 53 bits.  On a
    non-square grid, so a transposed index fails."""
    nx, ny, amp, seed = 23, 17, 1e-3, 0x5EED1234
    P = stepper.make_params(nx, ny, T07)
    kw = dict(bubbles=[(11.0, 8.0, 5.0)], rho_l=RL07, rho_g=RG07, W=5.0)
    base = stepper.init_density(P, **kw)
    noisy = stepper.init_density(P, noise_amp=amp, seed=seed, **kw)
    for y in range(ny):
        for x in range(nx):
            u = (_splitmix64(seed ^ (y * nx + x)) >> 11) * 2.0 ** -53
            assert noisy[y, x] == base[y, x] * (1.0 + amp * (2.0 * u - 1.0)), (x, y)


def test_noise_is_bounded_and_seeded():
    P = stepper.make_params(50, 40, T07)
    base = stepper.init_density(P, bubbles=[(25, 20, 8)], rho_l=RL07, rho_g=RG07, W=5.0)
    n1 = stepper.init_density(P, bubbles=[(25, 20, 8)], rho_l=RL07, rho_g=RG07, W=5.0,
                              noise_amp=1e-3, seed=1)
    n2 = stepper.init_density(P, bubbles=[(25, 20, 8)], rho_l=RL07, rho_g=RG07, W=5.0,
                              noise_amp=1e-3, seed=2)
    rel = n1 / base - 1
    assert np.all(np.abs(rel) <= 1e-3) and rel.std() > 4e-4
    assert not np.array_equal(n1, n2)
    assert abs(rel.mean()) < 1e-4


def test_nonfinite_state_is_reported():
    P = stepper.make_params(6, 6, T07)
    rho = np.full((6, 6), 0.2)
    rho[2, 3] = 0.99           # psi^2 < 0 next to the EOS pole
    f = stepper.init_populations(P, rho)
    assert stepper.step(P, f, 1) == -4


@pytest.mark.parametrize("gap", [9.3, 4.0])
def test_walls_are_planes_of_mirror_symmetry(gap):
    """Halfway bounce-back at y = -1/2 and y = ny - 1/2 with the mirrored psi
    of the solid rows, on states uniform in x and at rest (where reversing a
    diagonal population and reflecting it in y give the same value), must
    reproduce the lower half of a periodic channel of 2 ny rows whose upper
    half is the mirror image of the lower: both walls are then planes of
    symmetry of the periodic run.  A liquid layer on the lower wall, vapour,
    and a thinner layer on the upper wall; pins the wall position, the
    bounce-back of every population and the psi mirror against the periodic
    path."""
    nx, ny = 3, 24
    y = np.arange(ny)
    mid, half = 0.5 * (RL07 + RG07), 0.5 * (RL07 - RG07)
    col = mid - half * np.tanh(2 * (y - gap) / 5.0) * np.tanh(2 * (ny - 4.5 - y) / 5.0)
    Pw = stepper.make_params(nx, ny, T07, walls=True, tau_nu=0.7)
    fw = stepper.init_populations(Pw, np.tile(col[:, None], (1, nx)))
    Pp = stepper.make_params(nx, 2 * ny, T07, walls=False, tau_nu=0.7)
    colp = np.concatenate([col, col[::-1]])
    fp = stepper.init_populations(Pp, np.tile(colp[:, None], (1, nx)))
    assert stepper.step(Pw, fw, 300) == 0
    assert stepper.step(Pp, fp, 300) == 0
    assert np.max(np.abs(fw - fp[:ny])) < 1e-13 * np.max(np.abs(fw))
    # the periodic run itself stays mirror symmetric (y -> 2 ny - 1 - y, e_y -> -e_y)
    refl = [0, 1, 4, 3, 2, 8, 7, 6, 5]
    assert np.max(np.abs(fp[ny:][::-1][:, :, refl] - fp[:ny])) < 1e-13 * np.max(np.abs(fw))
    # and the state has moved away from the start (the test is not vacuous)
    f0 = stepper.init_populations(Pw, np.tile(col[:, None], (1, nx)))
    assert np.max(np.abs(fw - f0)) > 1e-4


def test_wall_pressure_of_a_uniform_critical_state_is_the_critical_pressure():
    """At the critical point (rho_c, T_c) of Eq. 15, found by the multiprecision
    solver, a uniform state at rest between walls stays uniform, and the wall
    pressure of every step is the critical pressure p_c (0.00220840670051 for
    a = 0.5, b = 4, R = 1)."""
    Tc, rc, pc = coexist.critical_point()
    P = stepper.make_params(12, 10, float(Tc), walls=True)
    f = stepper.init_populations(P, np.full((10, 12), float(rc)))
    rc_, w = stepper.step_wall_pressure(P, f, 6)
    assert rc_ == 0
    assert np.allclose(w, float(pc), rtol=1e-12, atol=0)
    assert float(pc) == pytest.approx(0.00220840670051, rel=1e-10)


def test_wall_pressure_reads_only_the_wall_rows_of_each_steps_start():
    """The recorded value of step t is the largest Eq. 15 pressure on rows 0 and
    ny - 1 of the state before step t: a denser row next to the wall does not
    count, the densest wall row does, and the values follow the state step by
    step."""
    ny, nx = 16, 10
    P = stepper.make_params(nx, ny, T07, walls=True, tau_nu=0.8)
    rho = np.full((ny, nx), RL07)
    rho[ny - 2, :] = RL07 * 1.05           # not a wall row
    rho[ny - 1, 3] = RL07 * 1.02           # the densest wall site
    rho[0, :] = RL07 * 1.01
    f = stepper.init_populations(P, rho)
    g = f.copy()
    rc_, w = stepper.step_wall_pressure(P, f, 8)
    assert rc_ == 0
    assert w[0] == pytest.approx(stepper.eos_pressure(P, RL07 * 1.02), rel=1e-13)
    for t in range(8):
        d = stepper.density(P, g)
        want = max(np.max(stepper.eos_pressure(P, d[0])), np.max(stepper.eos_pressure(P, d[-1])))
        assert w[t] == want
        assert stepper.step(P, g, 1) == 0
    assert np.array_equal(f, g)
    # the bottom wall row counts as well
    rho[0, 5] = RL07 * 1.03
    rc_, w = stepper.step_wall_pressure(P, stepper.init_populations(P, rho), 1)
    assert rc_ == 0 and w[0] == pytest.approx(stepper.eos_pressure(P, RL07 * 1.03), rel=1e-13)
