"""The stochastic rounding of the binary32 rest population
(paper_1605_01800_amd/csrc/lbm_rounding.h), compiled for the host with g++
through tests/rounding_harness.cpp and run over every one of the 2^24 keys
the rounding tells apart:

  * it returns only the binary32 values next to the exact sum a + b (the
    exact sum itself when it is representable), so no rounding moves a site's
    mass by more than one unit in the last place of its rest population;
  * its mean over the keys is the exact sum to within 2^-24 of the gap
    between those values, so each site keeps its mass on average;
  * the random words are the same for sites that the grid's reflections map
    onto each other, and at any site their top bits, which the rounding
    reads, are spread evenly over the steps."""
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1605_01800_amd", "csrc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("rounding") / "rounding_harness")
    subprocess.run([gxx, "-O2", "-std=c++17", "-ffp-contract=off", "-Wall", "-Wno-unknown-pragmas", "-I" + CSRC,
                    "-o", exe, os.path.join(ROOT, "tests", "rounding_harness.cpp")], check=True)
    return exe


def _bits(x):
    return "%08x" % int(np.float32(x).view(np.uint32))


def _float(h):
    return np.uint32(int(h, 16)).view(np.float32)


def _cases():
    rng = np.random.default_rng(11)
    out = [(1.0, 2.0 ** -24 + 2.0 ** -47),          # just above the midpoint
           (1.0, -2.0 ** -30),                        # below a power of two: the gap halves
           (-1.0, 2.0 ** -30), (-0.25, -3e-9),
           (0.125, 0.0), (0.5, 0.25),                 # exact sums
           (0.1, -0.1),                               # exact cancellation
           (3e-7, 0.4),                               # the increment larger than the population
           (-0.0123, 0.0123 + 1e-9)]
    for _ in range(24):                               # populations and increments of the collision
        out.append((rng.uniform(-0.2, 0.2), rng.uniform(-1e-3, 1e-3) * 10.0 ** rng.integers(-4, 1)))
    return [(np.float32(a), np.float32(b)) for a, b in out]


@pytest.mark.parametrize("a,b", _cases())
def test_rounding_returns_the_neighbours_and_is_exact_on_average(harness, a, b):
    out = subprocess.run([harness, "sum", _bits(a), _bits(b)], check=True, capture_output=True,
                         text=True).stdout.split()
    v0, n0, v1, n1, others = _float(out[0]), int(out[1]), _float(out[2]), int(out[3]), int(out[4])
    assert others == 0 and n0 + n1 == 1 << 24
    exact = Fraction(float(a)) + Fraction(float(b))
    near = np.float32(float(exact))                   # to nearest
    if Fraction(float(near)) == exact:
        assert n1 == 0 and v0 == near
        return
    lo = near if Fraction(float(near)) < exact else np.nextafter(near, np.float32(-np.inf))
    hi = np.nextafter(lo, np.float32(np.inf))
    assert Fraction(float(lo)) < exact < Fraction(float(hi))
    assert {float(v0), float(v1)} == {float(lo), float(hi)}
    gap = Fraction(float(hi)) - Fraction(float(lo))
    mean = (n0 * Fraction(float(v0)) + n1 * Fraction(float(v1))) / (1 << 24)
    assert abs(mean - exact) <= gap / (1 << 24)


@pytest.mark.parametrize("nx,ny", [(7, 10), (8, 1), (256, 256), (1024, 767)])
def test_words_are_mirror_symmetric(harness, nx, ny):
    out = subprocess.run([harness, "words", str(nx), str(ny)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout


@pytest.mark.parametrize("x,y", [(0, 0), (17, 100), (127, 255), (5000, 3000)])
def test_a_sites_words_spread_evenly_over_the_steps(harness, x, y):
    """The rounding is exact on average at a site if its word's top bits are
    uniform over the steps: the top byte of site (x, y)'s word over 65,536
    steps, a chi-square test of 256 equal bins at the 0.1 % level."""
    out = subprocess.run([harness, "steps", "8192", "4096", str(x), str(y), "65536"], check=True,
                         capture_output=True, text=True).stdout.split()
    counts = np.array([int(c) for c in out], dtype=np.float64)
    assert counts.size == 256 and counts.sum() == 65536
    chi2 = float(np.sum((counts - 256.0) ** 2 / 256.0))
    assert chi2 < 330.5, chi2                         # 255 degrees of freedom, p = 0.001
