"""Mutation tests of the oracle's pins.

Each case plants one plausible mistake in a copy of oracle/lbm_oracle.c (a
dropped term, a wrong sign, coefficient, index or direction), compiles it with
the oracle's flags, and runs the oracle's own tests (tests/test_oracle_*.py)
against it in a separate process: a pin must fail for every mistake.  The
oracle source itself is not changed; the copy is loaded through ORACLE_LIB.

The post-processing of oracle/diagnostics.py (bubble radius, ownership of
sites by bubbles, compensated sums, pressure jump, slab densities) is checked
the same way: a copy with one planted mistake is loaded through
ORACLE_DIAGNOSTICS by its pins (tests/test_oracle_diagnostics.py).
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

from oracle import build as obuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, text in lbm_oracle.c, the mistaken text); each text occurs once
MUTANTS = [
    ("eos_numerator_sign",          # Eq. 15, Z = (1 + eta + eta^2 - eta^3) / (1 - eta)^3
     "double num = 1.0 + eta + eta * eta - eta * eta * eta;",
     "double num = 1.0 + eta + eta * eta + eta * eta * eta;"),
    ("psi_factor_two",              # Eq. 13 without its factor 2
     "return sqrt(2.0 * (p - rho * cs2) / (P->G * c * c));",
     "return sqrt((p - rho * cs2) / (P->G * c * c));"),
    ("force_diagonal_weight",       # Eq. 7, w = 1/12 on the diagonals
     "return (a <= 4) ? 1.0 / 3.0 : 1.0 / 12.0;",
     "return (a <= 4) ? 1.0 / 3.0 : 1.0 / 6.0;"),
    ("force_x_sign",                # Eq. 7, -G in front of the x component only
     "Fx[i] = -P->G * psi[i] * sx;",
     "Fx[i] = P->G * psi[i] * sx;"),
    ("velocity_half_force",         # Eq. 6, half the force
     "double vx = (jx + 0.5 * dt * Fx) / rho;",
     "double vx = (jx + dt * Fx) / rho;"),
    ("moment_matrix_entry",         # a q_x row with two diagonal entries swapped
     "{ 0, -2,  0,  2,  0,  1, -1, -1,  1},   /* qx   */",
     "{ 0, -2,  0,  2,  0,  1, -1,  1, -1},   /* qx   */"),
    ("equilibrium_e_coefficient",   # Eq. 4, e row rho (-2 + 3 v^2)
     "meq[1] = rho * (-2.0 + 3.0 * v2);",
     "meq[1] = rho * (-2.0 + 2.0 * v2);"),
    ("li_term_zeta_uses_tau_e",     # Eq. 14, tau_zeta in the zeta row
     "- 0.75 * P->eps * F2 / (psi * psi * dt * (tau_z - 0.5));",
     "- 0.75 * P->eps * F2 / (psi * psi * dt * (tau_e - 0.5));"),
    ("li_term_dropped_from_zeta",   # Eq. 14 zeta row without Li's term
     "S[2] = -6.0 * vF - 0.75 * P->eps * F2 / (psi * psi * dt * (tau_z - 0.5));",
     "S[2] = -6.0 * vF;"),
    ("source_without_half_rate",    # Eq. 3, (I - Lambda/2) S
     "+ dt * (1.0 - 0.5 * P->s[k]) * S[k];",
     "+ dt * (1.0 - P->s[k]) * S[k];"),
    ("bounce_back_not_reversed",    # halfway bounce-back returns the opposite population
     "fnew[((long)y * nx + x) * 9 + opposite(a)] = fstar[src];",
     "fnew[((long)y * nx + x) * 9 + a] = fstar[src];"),
    ("stream_x_backwards",          # Eq. 5, f_a moves to x + e_a
     "int xd = ((x + EX[a]) % nx + nx) % nx;",
     "int xd = ((x - EX[a]) % nx + nx) % nx;"),
    ("wall_psi_zero",               # psi at solid sites: mirror, not 0
     "if (y < 0) y = 0;\n        if (y > ny - 1) y = ny - 1;",
     "if (y < 0 || y > ny - 1) return 0.0;"),
    ("rest_weight",                 # f_a = w_a rho with w_0 = 4/9
     "if (a == 0) return 4.0 / 9.0;",
     "if (a == 0) return 1.0 / 3.0;"),
    ("source_pxx_factor",           # Eq. 14, 2 (vx Fx - vy Fy) in the pxx row
     "S[7] = 2.0 * (vx * Fx - vy * Fy);",
     "S[7] = (vx * Fx - vy * Fy);"),
    ("equilibrium_qx_sign",         # Eq. 4, q_x^eq = -rho vx
     "meq[4] = -rho * vx;",
     "meq[4] = rho * vx;"),
    ("wall_psi_periodic",           # psi at solid sites wrapped around instead of mirrored
     "    if (P->walls) {\n        if (y < 0) y = 0;\n        if (y > ny - 1) y = ny - 1;\n    } else {\n"
     "        y = ((y % ny) + ny) % ny;\n    }",
     "    y = ((y % ny) + ny) % ny;"),
    ("interface_width",             # Eq. 16, tanh(2 d / W)
     "tanh(2.0 * d / W)",
     "tanh(d / W)"),
    ("noise_site_index",            # noise of site (x, y) drawn with index y nx + x
     "oracle_uniform(seed, (uint64_t)i)",
     "oracle_uniform(seed, (uint64_t)((long)x * ny + y))"),
    ("wall_pressure_row",           # the wall-pressure reading on the row next to the top wall
     "const int rows[2] = {0, P->ny - 1};",
     "const int rows[2] = {0, P->ny - 2};"),
    ("wall_pressure_bottom_row",    # ... and on the row next to the bottom wall
     "const int rows[2] = {0, P->ny - 1};",
     "const int rows[2] = {1, P->ny - 1};"),
    ("macros_velocity_half_force",  # Eq. 6 in the reported velocity field
     "vx[i] = (jx + 0.5 * Fx[i]) / rho[i];",
     "vx[i] = jx / rho[i];"),
]


# (name, text in oracle/diagnostics.py, the mistaken text); each text occurs once
PY_MUTANTS = [
    ("radius_sqrt_area_over_pi",    # sqrt(A) / pi instead of sqrt(A / pi)
     "math.sqrt(float(np.sum(gas_fraction(rho, rho_l, rho_g))) / math.pi)",
     "math.sqrt(float(np.sum(gas_fraction(rho, rho_l, rho_g)))) / math.pi"),
    ("gas_fraction_not_clipped",    # fraction outside [0, 1] counted
     "return np.clip((rho_l - rho) / (rho_l - rho_g), 0.0, 1.0)",
     "return (rho_l - rho) / (rho_l - rho_g)"),
    ("gas_fraction_densities_swapped",
     "return np.clip((rho_l - rho) / (rho_l - rho_g), 0.0, 1.0)",
     "return np.clip((rho_g - rho) / (rho_g - rho_l), 0.0, 1.0)"),
    ("radii_farthest_centre",       # each site counted for the farthest centre
     "owner = np.argmin(d2, axis=0)",
     "owner = np.argmax(d2, axis=0)"),
    ("radii_distance_in_x_only",
     "(xx - cx) ** 2 + (yy - cy) ** 2",
     "(xx - cx) ** 2"),
    ("radii_sqrt_area_over_pi",
     "math.sqrt(float(np.sum(frac[owner == k])) / math.pi)",
     "math.sqrt(float(np.sum(frac[owner == k]))) / math.pi"),
    ("kahan_instead_of_neumaier",   # compensation without Neumaier's branch
     "        if abs(s) >= abs(v):\n            c += (s - t) + v\n        else:\n            c += (v - t) + s\n",
     "        c += (s - t) + v\n"),
    ("pressure_jump_sign",          # p_out - p_in, negative for a bubble
     "return p_in - p_out, p_in, p_out",
     "return p_out - p_in, p_in, p_out"),
    ("pressure_jump_band",          # inner sample reaching into the interface
     "p_in = float(np.mean(p[r < R - 2 * W]))",
     "p_in = float(np.mean(p[r < R - W]))"),
    ("slab_sixteen_rows",           # 16 rows instead of the 17 central ones
     "rows_l = [(liquid_mid + k) % ny for k in range(-8, 9)]",
     "rows_l = [(liquid_mid + k) % ny for k in range(-8, 8)]"),
]


def _source():
    with open(obuild.SRC) as fh:
        return fh.read()


def _run_pins(lib_path):
    env = dict(os.environ, ORACLE_LIB=lib_path, OMP_NUM_THREADS="2")
    tests = sorted(os.path.join(ROOT, "tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
                   if f.startswith("test_oracle_") and f.endswith(".py") and "mutants" not in f)
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"] + tests
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def _py_source():
    with open(os.path.join(ROOT, "oracle", "diagnostics.py")) as fh:
        return fh.read()


def _run_py_pins(path):
    env = dict(os.environ, ORACLE_DIAGNOSTICS=path)
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_oracle_diagnostics.py")]
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def _survivors(runs):
    survivors = []
    for name, r in runs.items():
        tail = r.stdout.strip().splitlines()[-1] if r.stdout.strip() else r.stderr[-300:]
        print(name, "->", tail)
        # exit status 1 with a failed test: a pin caught it (2 and up would be
        # a collection or usage error, which proves nothing)
        if not (r.returncode == 1 and "failed" in tail):
            survivors.append((name, r.returncode, tail))
    return survivors


def test_every_mutation_applies_once():
    src = _source()
    for name, old, new in MUTANTS:
        assert src.count(old) == 1, name
        assert old != new, name
    src = _py_source()
    for name, old, new in PY_MUTANTS:
        assert src.count(old) == 1, name
        assert old != new, name


def test_every_planted_mistake_fails_a_pin(tmp_path):
    """Every mutant fails a pin; a faithful copy, run through the same
    harness alongside them, passes (so the failures are the mistakes')."""
    src = _source()
    libs = {}
    for name, old, new in MUTANTS + [("faithful_copy", "", "")]:
        c = tmp_path / (name + ".c")
        c.write_text(src.replace(old, new) if old else src)
        libs[name] = obuild.compile_source(str(c), str(tmp_path / (name + ".so")), quiet=True)
    with ThreadPoolExecutor(max_workers=4) as pool:
        runs = dict(zip(libs, pool.map(_run_pins, libs.values())))
    control = runs.pop("faithful_copy")
    assert control.returncode == 0, control.stdout[-2000:]
    survivors = _survivors(runs)
    assert not survivors, survivors


def test_every_planted_diagnostics_mistake_fails_a_pin(tmp_path):
    """The same for oracle/diagnostics.py: every mutant fails a pin of
    tests/test_oracle_diagnostics.py, and a faithful copy passes them."""
    src = _py_source()
    files = {}
    for name, old, new in PY_MUTANTS + [("faithful_copy", "", "")]:
        p = tmp_path / (name + ".py")
        p.write_text(src.replace(old, new) if old else src)
        files[name] = str(p)
    with ThreadPoolExecutor(max_workers=4) as pool:
        runs = dict(zip(files, pool.map(_run_py_pins, files.values())))
    control = runs.pop("faithful_copy")
    assert control.returncode == 0, control.stdout[-2000:]
    survivors = _survivors(runs)
    assert not survivors, survivors
