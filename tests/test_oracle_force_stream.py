"""Pins of the oracle's interaction force (Eq. 7) and streaming (Eq. 5) with
periodic and halfway bounce-back boundaries."""
import numpy as np
import pytest

from oracle import coexist, stepper

T07 = coexist.temperature(0.7)


def test_uniform_psi_gives_zero_force():
    for walls in (False, True):
        P = stepper.make_params(7, 5, T07, walls=walls)
        Fx, Fy = stepper.force(P, np.full((5, 7), 0.3))
        assert np.all(Fx == 0) and np.all(Fy == 0)


def test_force_of_a_sinusoid_is_exact():
    """psi = sin(kx x) sin(ky y) on a periodic grid: by the sum-to-product
    identities, sum_a w_a psi(x + e_a) e_ax = 2 cos(kx x) sin(kx) sin(ky y)
    (1/3 + cos(ky) / 6), and the same with x and y exchanged."""
    nx, ny = 24, 18
    kx, ky = 2 * np.pi * 3 / nx, 2 * np.pi * 2 / ny
    y, x = np.mgrid[0:ny, 0:nx]
    psi = 1.5 + np.sin(kx * x) * np.sin(ky * y)
    P = stepper.make_params(nx, ny, T07)
    Fx, Fy = stepper.force(P, psi)
    gx = 2 * np.cos(kx * x) * np.sin(kx) * np.sin(ky * y) * (1 / 3 + np.cos(ky) / 6)
    gy = 2 * np.cos(ky * y) * np.sin(ky) * np.sin(kx * x) * (1 / 3 + np.cos(kx) / 6)
    # -G = 1
    assert np.allclose(Fx, psi * gx, atol=1e-14)
    assert np.allclose(Fy, psi * gy, atol=1e-14)


@pytest.mark.parametrize("a,ex,ey,w", [(1, 1, 0, 1 / 3), (2, 0, 1, 1 / 3), (3, -1, 0, 1 / 3),
                                       (4, 0, -1, 1 / 3), (5, 1, 1, 1 / 12), (6, -1, 1, 1 / 12),
                                       (7, -1, -1, 1 / 12), (8, 1, -1, 1 / 12)])
def test_force_from_a_single_raised_site(a, ex, ey, w):
    """psi = 1 plus d at one site s: the node s - e_a feels exactly w_a d e_a."""
    nx, ny, d = 9, 8, 0.25
    psi = np.ones((ny, nx))
    sx, sy = 4, 3
    psi[sy, sx] += d
    P = stepper.make_params(nx, ny, T07)
    Fx, Fy = stepper.force(P, psi)
    assert Fx[sy - ey, sx - ex] == pytest.approx(w * d * ex, abs=1e-16)
    assert Fy[sy - ey, sx - ex] == pytest.approx(w * d * ey, abs=1e-16)


def test_total_force_vanishes_on_periodic_grid():
    rng = np.random.default_rng(3)
    P = stepper.make_params(13, 11, T07)
    Fx, Fy = stepper.force(P, rng.uniform(0.1, 0.4, (11, 13)))
    assert abs(Fx.sum()) < 1e-15 and abs(Fy.sum()) < 1e-15


def test_wall_rows_use_mirrored_psi():
    """Reading for solid sites: psi(x, -1) = psi(x, 0), psi(x, ny) = psi(x, ny-1).
    For psi depending on y only, Fy at the bottom row is psi0 (psi1 - psi0) / 2
    and at the top row psi_t (psi_t - psi_{t-1}) / 2 with the sign of -e_y."""
    nx, ny = 5, 6
    prof = np.array([0.2, 0.25, 0.3, 0.33, 0.31, 0.28])
    psi = np.repeat(prof[:, None], nx, axis=1)
    P = stepper.make_params(nx, ny, T07, walls=True)
    Fx, Fy = stepper.force(P, psi)
    assert np.allclose(Fx, 0, atol=1e-17)
    assert np.allclose(Fy[0], prof[0] * (prof[1] - prof[0]) / 2, atol=1e-16)
    assert np.allclose(Fy[-1], prof[-1] * (prof[-1] - prof[-2]) / 2, atol=1e-16)
    mid = prof[1:-1] * (prof[2:] - prof[:-2]) / 2
    assert np.allclose(Fy[1:-1], mid[:, None], atol=1e-16)


def _delta_state(nx, ny, x, y, a):
    f = np.zeros((ny, nx, 9))
    f[y, x, a] = 1.0
    return f


def test_periodic_streaming_moves_each_population_along_its_velocity():
    nx, ny = 6, 5
    P = stepper.make_params(nx, ny, T07)
    E = stepper.velocities()
    for a in range(9):
        for (x, y) in [(0, 0), (5, 4), (2, 3)]:
            out = stepper.stream(P, _delta_state(nx, ny, x, y, a))
            xd, yd = (x + E[a, 0]) % nx, (y + E[a, 1]) % ny
            assert out[yd, xd, a] == 1.0
            assert np.nansum(out) == 1.0


@pytest.mark.parametrize("x,y,a,expect", [
    (2, 0, 4, (2, 0, 2)),     # moving -y at the bottom row comes back as +y
    (2, 0, 7, (2, 0, 5)),     # (-1,-1) -> (1,1) at the same node
    (2, 0, 8, (2, 0, 6)),     # (1,-1) -> (-1,1)
    (0, 3, 2, (0, 3, 4)),     # moving +y at the top row
    (0, 3, 5, (0, 3, 7)),
    (5, 3, 6, (5, 3, 8)),
    (5, 0, 1, (0, 0, 1)),     # x stays periodic next to a wall
    (5, 0, 5, (0, 1, 5)),     # diagonal leaving through x only wraps
])
def test_halfway_bounce_back_at_walls(x, y, a, expect):
    nx, ny = 6, 4
    P = stepper.make_params(nx, ny, T07, walls=True)
    out = stepper.stream(P, _delta_state(nx, ny, x, y, a))
    ex, ey, ea = expect
    assert out[ey, ex, ea] == 1.0
    assert np.nansum(out) == 1.0


def test_streaming_is_a_permutation():
    rng = np.random.default_rng(5)
    for walls in (False, True):
        P = stepper.make_params(7, 6, T07, walls=walls)
        f = rng.random((6, 7, 9))
        out = stepper.stream(P, f)
        assert not np.any(np.isnan(out))
        assert np.array_equal(np.sort(out.ravel()), np.sort(f.ravel()))
