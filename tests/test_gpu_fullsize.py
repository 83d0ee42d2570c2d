"""Parity at the workloads' full sizes, in the launch configuration bench.py
times (one batch over all instances, the tile variant its autotuner picks):

  * the Laplace-law sweep, 24 instances of 256 x 256: after 300 steps every
    site of every instance is compared with one oracle step from the same state
    (and, for the two-step kernel, with two: one launch of its pair path);
  * the 8192 x 4096 wall-bounded three-disc collapse: after 200 steps, windows
    at the walls, across the periodic x edge, across strip edges and on a disc
    interface are compared with one oracle step of the window (for the
    two-step kernel its odd last step; two steps cannot be compared on a
    window, whose wrapped edges the oracle steps as a discontinuity that
    leaves Eq. 13's range).  A window's outer three rows and columns are left
    out where the window is not bounded by a wall (one step reaches two sites:
    psi of a neighbour, then streaming), so the compared sites see exactly the
    state the GPU saw.

Tolerances as for single steps: 1e-14 relative (binary64), 2e-6 (binary32);
the many-step tests state their own.
"""
import numpy as np
import pytest

from oracle import stepper as ostep
from tests.helpers import oracle_params, rel_inf, to_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_1605_01800_amd.lbm")
from paper_1605_01800_amd import inputs, studies  # noqa: E402

STEP_TOL = {"fp64": 1e-14, "fp32": 2e-6, "fp32_mixed": 2e-6}


def _batch(sims, precision, variant):
    b = L.Batch(precision=precision, max_instances=len(sims),
                max_tiles=sum(L.tile_count(s.params) for s in sims))
    for s in sims:
        b.attach(s)
    b.set_variant(L.variant_names().index(variant))
    return b


@pytest.mark.parametrize("variant,n", [("fused-64x16", 1), ("fused2-128x16", 1), ("twostep-58x32", 1),
                                       ("twostep-58x32", 2)])
def test_laplace_sweep_full_size_one_step(variant, n):
    print("case sweep", variant, n, flush=True)
    sims = studies.laplace_sweep_sims(L, "fp32", "cuda:0")
    b = _batch(sims, "fp32", variant)
    b.step(300)
    b.sync()
    starts = [s.populations() for s in sims]
    b.step(n)
    b.sync()
    for s, f0 in zip(sims, starts):
        want = to_oracle(f0)
        assert ostep.step(oracle_params(s.params), want, n) == 0
        got = to_oracle(s.populations())
        assert rel_inf(got, want) < n * STEP_TOL["fp32"]
    b.close()
    for s in sims:
        s.close()


def _windows(nx, ny, bub, h=32, w=40):
    """(rows, columns, bottom wall, top wall) of the sample windows."""
    x0, y0, r0 = bub[0]
    xi, yi = int(x0 + r0) - w // 2, int(y0) - h // 2           # across the first disc's interface
    out = [
        (np.arange(0, h), np.arange(1000, 1000 + w), True, False),                 # bottom wall
        (np.arange(ny - h, ny), np.arange(5000, 5000 + w), False, True),           # top wall
        (np.arange(ny // 2, ny // 2 + h), np.r_[nx - w // 2:nx, 0:w // 2], False, False),  # x edge
        (np.arange(0, h), np.r_[nx - w // 2:nx, 0:w // 2], True, False),           # corner
        (np.arange(1717, 1717 + h), np.arange(128 * 20 - w // 2, 128 * 20 + w // 2), False, False),  # strips
        (np.arange(yi, yi + h), np.arange(xi, xi + w), False, False),              # interface
    ]
    return out


@pytest.mark.parametrize("prec,variant,n", [("fp32", "fused2-128x16", 1), ("fp32", "fused-64x16", 1),
                                            ("fp64", "fused-64x16", 1), ("fp32_mixed", "fused2-128x16", 1),
                                            ("fp32", "twostep-58x24", 1), ("fp64", "twostep-58x24", 1)])
def test_collapse_large_full_size_sampled_windows(prec, variant, n):
    print("case large", prec, variant, n, flush=True)
    nx, ny = 8192, 4096
    bub = inputs.non_overlapping_discs(nx, ny, [300, 200, 150], W=5.0, seed=0, walls=True)
    p = L.make_params(nx, ny, T_over_Tc=0.6, walls=True, precision=prec, tau_nu=0.6)
    sim = L.Sim(p)
    sim.init_bubble(bub, W=5.0, delta=0.02)
    b = _batch([sim], prec, variant)
    b.step(200)
    b.sync()
    f0 = sim.populations()
    b.step(n)
    b.sync()
    f1 = sim.populations()
    P = oracle_params(p)
    m = 3 * n                                     # rows and columns a window's edge can reach in
    for rows, cols, bottom, top in _windows(nx, ny, bub):
        r = torch.as_tensor(rows, device=f0.device)
        c = torch.as_tensor(cols, device=f0.device)
        sub0 = f0.index_select(1, r).index_select(2, c)
        sub1 = f1.index_select(1, r).index_select(2, c)
        h, w = len(rows), len(cols)
        Pw = ostep.with_grid(P, w, h, walls=bottom or top)
        want = to_oracle(sub0)
        assert ostep.step(Pw, want, n) == 0
        got = to_oracle(sub1)
        ylo = 0 if bottom else m
        yhi = h if top else h - m
        sl = (slice(ylo, yhi), slice(m, w - m))
        err = rel_inf(got[sl], want[sl])
        print("window rows %d.. cols %d.. err %.2e" % (rows[0], cols[0], err), flush=True)
        assert err < n * STEP_TOL[prec]
    b.close()
    sim.close()


def test_largest_plane_sampled_windows():
    """The largest accepted binary32 grid, 32768 x 32767 with walls: every
    population plane just under 4 GiB (76 GB of workspace).  From an Eq. 16
    state, one step of each single-pass kernel family is compared with the
    oracle on windows at the far ends of the planes (the largest offsets)."""
    free, _ = torch.cuda.mem_get_info()
    if free < 170e9:
        pytest.skip("needs about 160 GB of free device memory")
    print("case largest plane", flush=True)
    nx, ny = 32768, 32767
    bub = [(nx - 1000.5, ny - 800.0, 300.0), (700.0, 600.0, 200.0)]
    p = L.make_params(nx, ny, T_over_Tc=0.7, walls=True, precision="fp32", tau_nu=0.6)
    sim = L.Sim(p)
    sim.init_bubble(bub, W=5.0, delta=0.02)
    sim.set_variant(L.variant_names().index("fused2-128x16"))
    sim.step(3)
    sim.sync()
    f0 = sim.populations()
    P = oracle_params(p)
    h, w = 32, 40
    windows = [
        (np.arange(ny - h, ny), np.r_[nx - w // 2:nx, 0:w // 2], False, True),     # top corner, x edge
        (np.arange(0, h), np.arange(nx - w, nx), True, False),                     # bottom, last columns
        (np.arange(ny - 816, ny - 816 + h), np.arange(nx - 720, nx - 720 + w), False, False),  # interface
        (np.arange(ny // 2, ny // 2 + h), np.arange(nx // 2 - w // 2, nx // 2 + w // 2), False, False),
    ]
    for variant in ("fused2-128x16", "fused-64x16", "2pass-64x4"):
        sim.set_populations(f0)
        sim.set_variant(L.variant_names().index(variant))
        sim.step(1)
        sim.sync()
        f1 = sim.populations()
        for rows, cols, bottom, top in windows:
            r = torch.as_tensor(rows, device=f0.device)
            c = torch.as_tensor(cols, device=f0.device)
            want = to_oracle(f0.index_select(1, r).index_select(2, c))
            assert ostep.step(ostep.with_grid(P, w, h, walls=bottom or top), want, 1) == 0
            got = to_oracle(f1.index_select(1, r).index_select(2, c))
            sl = (slice(0 if bottom else 3, h if top else h - 3), slice(3, w - 3))
            err = rel_inf(got[sl], want[sl])
            print(variant, "window rows %d.. cols %d.. err %.2e" % (rows[0], cols[0], err), flush=True)
            assert err < STEP_TOL["fp32"]
        del f1
    sim.close()
    del f0
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 1e-4)])
def test_collapse_horizon_grid_many_steps_against_the_oracle(prec, tol):
    """The 1024 x 768 wall-bounded collapse grid (0.6 T_c, a disc of radius 120
    at (511.5, 200), delta = 0.02, noise 1e-3, tau_nu = 0.6) at full size:
    1000 steps of the GPU path in the benchmark's launch configuration against
    1000 oracle steps from the same initial state; density field and bubble
    radius within the precision's tolerance.  The binary64 bound is derived
    from the arithmetic: this flow amplifies rounding, and the oracle itself,
    perturbed by half an ulp of random noise on every population at every
    step, drifts by 3.7e-12 (max norm, relative) in 1000 steps; the GPU rounds
    differently (fused multiply-adds, another summation order) by about that
    much per step, so 1e-11 bounds it; a wrong term shows as 1e-6 or more."""
    print("case horizon", prec, flush=True)
    from oracle import coexist, diagnostics
    nx, ny, steps = 1024, 768, 1000
    p = L.make_params(nx, ny, T_over_Tc=0.6, walls=True, precision=prec, tau_nu=0.6)
    bub = [(511.5, 200.0, 120.0)]
    sim = L.Sim(p)
    sim.init_bubble(bub, W=5.0, delta=0.02, noise_amp=1e-3, seed=1)
    f0 = to_oracle(sim.populations())
    b = _batch([sim], prec, "fused-64x16" if prec == "fp64" else "fused2-128x16")
    b.step(steps)
    b.sync()
    m = sim.macros()
    rho = m["rho"].double().cpu().numpy()
    P = oracle_params(p)
    assert ostep.step(P, f0, steps) == 0
    ref = ostep.density(P, f0)
    err = float(np.max(np.abs(rho - ref)) / np.max(np.abs(ref)))
    rg, rl, _ = coexist.maxwell(p.T)
    r_ref = diagnostics.bubble_radius(ref, rl, rg)
    r_gpu = m["diag"]["radius"][0]
    print("rho err %.2e radius %.6f vs %.6f" % (err, r_gpu, r_ref), flush=True)
    assert err < tol
    assert abs(r_gpu - r_ref) / r_ref < tol
    b.close()
    sim.close()


def test_batch_group_equals_one_batch_bitwise():
    """The sweep's 24 instances spread over four batches on four streams, as
    bench.py times them (write-through stores), step bitwise like the same
    instances in one batch."""
    print("case batch group", flush=True)
    out = []
    for n_batches in (1, 4):
        sims = studies.laplace_sweep_sims(L, "fp32", "cuda:0")
        if n_batches == 1:
            runner = _batch(sims, "fp32", "twostep-58x32")
        else:
            runner = L.BatchGroup(sims, precision="fp32", n_batches=n_batches)
            assert runner.batches[0].write_through
            runner.set_variant(L.variant_names().index("twostep-58x32"))
        runner.step(300)
        runner.sync()
        out.append([s.populations().cpu().numpy() for s in sims])
        runner.close()
        for s in sims:
            s.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_precision_study_large_grid_reduced_steps():
    """The 8192 x 4096 three-disc collapse (configuration c5: T = 0.6 T_c,
    delta = 0.02, tau_nu = 0.6) over its first 6000 steps, which include the
    wall-pressure peak (step 5297) and end before the first bubble vanishes
    completely (the model then leaves the range where Eq. 13 gives a real
    psi, near step 6400), in binary32 and in binary32 with binary64 EOS and
    psi near the spinodal, against the binary64 GPU path (held to the oracle
    at 1e-12): total mass, every bubble's radius history and the wall-pressure
    peak within 1e-4, the peak at the same step."""
    print("case precision large", flush=True)
    out = studies.precision_study("cuda:0", True, steps=6000, every=300)
    ref = out["runs"]["fp64"]
    assert not ref["nonfinite"] and ref["steps_done"] == 6000
    for prec in ("fp32", "fp32_mixed"):
        e = out["runs"][prec]
        print(prec, e["mass_max_rel_err"], e["radius_max_rel_err"], e.get("wall_p_max_rel_err"),
              e.get("wall_p_step"), ref["wall_p_step"], flush=True)
        assert not e["nonfinite"] and e["steps_done"] == 6000
        assert e["mass_max_rel_err"] < 1e-4
        assert max(e["radius_max_rel_err"]) < 1e-4
        assert e["wall_p_max_rel_err"] < 1e-4
        assert e["wall_p_step"] == ref["wall_p_step"]
