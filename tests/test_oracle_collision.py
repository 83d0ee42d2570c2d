"""Pins of the oracle's moment transform, equilibrium, source term and
relaxation (Eqs. 2-4, 6, 8, 14) against textbook forms written in velocity
space and against invariants of the collision."""
import numpy as np
import pytest

from oracle import coexist, stepper

# Textbook D2Q9 set in the order rest, +x, +y, -x, -y, then the diagonals.
E = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def textbook_feq(rho, v):
    """Second-order Maxwell-Boltzmann equilibrium of the D2Q9 lattice."""
    eu = E @ v
    return W * rho * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (v @ v))


def guo_forcing(v, F):
    """Guo, Zheng and Shi's discrete forcing term w_a [3 (e_a - v).F + 9 (e_a.v)(e_a.F)]."""
    return W * (3 * ((E - v) @ F) + 9 * (E @ v) * (E @ F))


def test_velocity_order():
    assert np.array_equal(stepper.velocities(), E)


def test_transform_is_orthogonal_with_integer_rows():
    M, Minv = stepper.transform()
    assert np.array_equal(M, np.round(M))
    G = M @ M.T
    assert np.array_equal(G, np.diag(np.diag(G)))
    assert np.allclose(M @ Minv, np.eye(9), atol=1e-15)


def test_equilibrium_moments_are_moments_of_textbook_feq():
    """Eq. 4 must equal M applied to the textbook equilibrium for any rho, v;
    a wrong sign or a swapped row of M fails this."""
    rng = np.random.default_rng(1)
    for _ in range(50):
        rho = rng.uniform(0.001, 0.5)
        v = rng.uniform(-0.2, 0.2, 2)
        m = stepper.moments(textbook_feq(rho, v))
        meq = stepper.equilibrium_moments(rho, v[0], v[1])
        assert np.allclose(m, meq, rtol=0, atol=1e-15)


def _params(rates, eps=0.0):
    P = stepper.make_params(4, 4, coexist.temperature(0.7), eps=eps, s=rates)
    return P


def _random_node(rng):
    rho = rng.uniform(0.01, 0.45)
    f = W * rho * (1 + rng.uniform(-0.3, 0.3, 9))
    F = rng.uniform(-1e-3, 1e-3, 2)
    psi = rng.uniform(0.05, 0.4)
    return f, F, psi


@pytest.mark.parametrize("tau", [0.51, 0.6, 1.0, 1.7])
def test_mrt_equals_bgk_with_guo_forcing_at_equal_rates(tau):
    """With all rates equal to 1/tau and eps = 0, Eq. 3 with the source of
    Eq. 8 is the BGK collision with Guo's forcing term."""
    rng = np.random.default_rng(int(tau * 100))
    P = _params([1 / tau] * 9, eps=0.0)
    for _ in range(40):
        f, F, psi = _random_node(rng)
        rho = f.sum()
        v = (E.T @ f + 0.5 * F) / rho
        bgk = f - (f - textbook_feq(rho, v)) / tau + (1 - 0.5 / tau) * guo_forcing(v, F)
        got = stepper.collide_node(P, f, psi, F[0], F[1])
        assert np.allclose(got, bgk, rtol=0, atol=2e-15)


def test_collision_conserves_mass_and_adds_the_force():
    """For any rates: rho* = rho and j* = j + F (Eq. 6's half-force velocity
    makes the relaxation of j exactly cancel the (1 - s_j/2) F source)."""
    rng = np.random.default_rng(7)
    for _ in range(40):
        rates = rng.uniform(0.5, 1.9, 9)
        rates[5] = rates[3]
        P = _params(rates, eps=rng.uniform(0, 2))
        f, F, psi = _random_node(rng)
        out = stepper.collide_node(P, f, psi, F[0], F[1])
        assert abs(out.sum() - f.sum()) < 1e-15
        assert np.allclose(E.T @ out, E.T @ f + F, rtol=0, atol=1e-16)


def test_li_term_properties():
    """Eq. 14's extra term: it leaves mass and momentum unchanged, is linear in
    eps, scales as 1/psi^2 and (at fixed velocity) as |F|^2."""
    rng = np.random.default_rng(11)
    rates = stepper.relaxation_rates(0.6)
    for _ in range(20):
        f, F, psi = _random_node(rng)
        base = stepper.collide_node(_params(rates, 0.0), f, psi, F[0], F[1])
        d1 = stepper.collide_node(_params(rates, 1.0), f, psi, F[0], F[1]) - base
        d2 = stepper.collide_node(_params(rates, 2.0), f, psi, F[0], F[1]) - base
        dh = stepper.collide_node(_params(rates, 1.0), f, psi / 2, F[0], F[1]) - base
        assert np.max(np.abs(d1)) > 0
        # the differences carry the rounding of O(0.1) populations, ~1e-17
        assert abs(d1.sum()) < 1e-16 and np.allclose(E.T @ d1, 0, atol=1e-16)
        assert np.allclose(d2, 2 * d1, rtol=1e-8, atol=1e-16)
        assert np.allclose(dh, 4 * d1, rtol=1e-8, atol=1e-16)


def test_li_term_through_the_collision_in_closed_form():
    """Eq. 14's extra terms after (I - Lambda/2) of Eq. 3: since
    (1 - s/2) / (tau - 1/2) = s for tau = 1/s, they add s_e Y to m*_e and
    -s_zeta Y to m*_zeta, Y = 0.75 eps |F|^2 / psi^2, and nothing elsewhere.
    Through the e row (-4, -1 x4, 2 x4) and the zeta row (4, -2 x4, 1 x4) of
    M, whose squared norms are 36, f* changes by Y/36 times -4 s_e - 4 s_zeta
    at rest, 2 s_zeta - s_e on the axes and 2 s_e - s_zeta on the diagonals.
    With s_e != s_zeta, so that a rate taken from the other row fails (the
    zeta part changes neither mass, momentum nor the second-order pressure
    tensor, so the coexistence pins cannot see it)."""
    rng = np.random.default_rng(12)
    s_e, s_z = 0.8, 1.3
    rates = np.array([1.0, s_e, s_z, 1.0, 1.1, 1.0, 1.1, 1.0 / 0.8, 1.0 / 0.8])
    for eps in (1.0, 1.86):
        for _ in range(10):
            f, F, psi = _random_node(rng)
            base = stepper.collide_node(_params(rates, 0.0), f, psi, F[0], F[1])
            d = stepper.collide_node(_params(rates, eps), f, psi, F[0], F[1]) - base
            Y = 0.75 * eps * (F[0] ** 2 + F[1] ** 2) / psi ** 2
            want = Y / 36.0 * np.array([-4 * s_e - 4 * s_z] + [2 * s_z - s_e] * 4 + [2 * s_e - s_z] * 4)
            assert np.allclose(d, want, rtol=1e-9, atol=1e-16), (d, want)


def test_each_moment_relaxes_at_its_own_rate():
    """Eqs. 2-3 without force: a perturbation delta placed in one
    non-conserved moment alone (f = f_eq + delta M^-1 e_k) leaves the
    collision as (1 - s_k) delta in that moment and nothing in the others,
    with s in the order (rho, e, zeta, jx, qx, jy, qy, pxx, pxy) of Eq. 2.
    Distinct rates per group, so relaxing a moment at another moment's rate
    fails."""
    M, Minv = stepper.transform()
    s_rho, s_e, s_z, s_j, s_q, s_nu = 1.0, 0.7, 1.3, 1.0, 1.6, 0.9
    rates = np.array([s_rho, s_e, s_z, s_j, s_q, s_j, s_q, s_nu, s_nu])
    P = _params(rates)
    rng = np.random.default_rng(5)
    for k in (1, 2, 4, 6, 7, 8):
        rho = rng.uniform(0.05, 0.45)
        v = rng.uniform(-0.1, 0.1, 2)
        delta = 1e-3 * rho
        f = textbook_feq(rho, v) + delta * Minv[:, k]
        out = stepper.collide_node(P, f, 0.3, 0.0, 0.0)
        dm = M @ out - stepper.equilibrium_moments(rho, v[0], v[1])
        want = np.zeros(9)
        want[k] = (1.0 - rates[k]) * delta
        assert np.allclose(dm, want, rtol=0, atol=1e-15), (k, dm, want)
