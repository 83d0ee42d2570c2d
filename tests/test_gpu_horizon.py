"""Binary32 GPU runs against the binary64 oracle over the workloads' full
horizons, in the launch configurations bench.py times.  The oracle's values
come from tests/golden/make_horizon_goldens.py (which calls only oracle/):

  * the Laplace-law / coexistence sweep (24 periodic 256 x 256 instances,
    40,000 steps), as four concurrent batches with write-through stores and
    the 64-column fused kernel: bubble radius and mass every 1000 steps, the
    final density field (every fourth site, plus the full row and column
    through the centre), the final pressure jump of every disc and the
    coexisting densities of every slab;
  * the 1024 x 768 wall-bounded collapse (50,000 steps) as one batch with the
    paired kernel: radius and mass every 100 steps, the wall-pressure peak
    and its step, and density snapshots.

Tolerances (the binary32 bar): 1e-4 relative on densities (max norm over the
compared sites, relative to the largest reference density) and on the radius
history and mass.  Derived quantities take the bound that 1e-4 on the
densities implies: the pressure jump, |d dp| <= 2 max|dp/drho| 1e-4 rho_max
over the densities of the run.  The collapse's density field holds 1e-4 up to
5000 steps; from 10,000 steps on its largest differences sit on the ringing
interface and exceed it (a known failure of binary32 storage, kept as a
strict expected failure so that a change in either direction shows).
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_1605_01800_amd.lbm")
from oracle import diagnostics, stepper  # noqa: E402
from paper_1605_01800_amd import inputs  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SWEEP = os.path.join(GOLDEN, "laplace_sweep_40k.npz")
COLLAPSE = os.path.join(GOLDEN, "collapse_1024x768_50k_d020_s1.npz")
TOL = 1e-4


def _load(path):
    if not os.path.exists(path):
        pytest.skip("oracle reference %s not generated" % os.path.basename(path))
    return np.load(path, allow_pickle=False)


def _eos_slope_bound(T, lo, hi):
    """max |dp/drho| of Eq. 15 over [lo, hi], from the oracle's EOS."""
    P = stepper.make_params(4, 4, T)
    r = np.linspace(lo, hi, 4001)
    p = stepper.eos_pressure(P, r)
    return float(np.max(np.abs(np.diff(p) / np.diff(r))))


def _field_err(got, want):
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


@pytest.fixture(scope="module")
def sweep_run():
    g = _load(SWEEP)
    steps, every = int(g["steps"]), int(g["every"])
    cases = inputs.laplace_sweep_cases(256)
    sims = []
    for i, case in enumerate(cases):
        p = L.make_params(256, 256, T=float(g["T"][i]), precision="fp32", tau_nu=0.6)
        s = L.Sim(p)
        s.init_bubble(case["bubbles"], slab_rows=case["slab_rows"], rho_l=float(g["rho_l"][i]),
                      rho_g=float(g["rho_g"][i]), W=5.0)
        sims.append(s)
    group = L.BatchGroup(sims, precision="fp32", n_batches=4)
    group.set_variant(L.variant_names().index("fused-64x16"))
    radius = np.full(g["radius"].shape, np.nan)
    mass = np.full(g["mass"].shape, np.nan)
    for k in range(steps // every + 1):
        if k:
            group.step(every)
            group.sync()
        for i, s in enumerate(sims):
            d = s.diag()
            assert not d["nonfinite"] and d["step"] == k * every
            mass[i, k] = d["mass"]
            if d["radius"]:
                radius[i, k] = d["radius"][0]
    fields = [s.macros() for s in sims]
    rho = [f["rho"].double().cpu().numpy() for f in fields]
    pres = [f["p"].cpu().numpy() for f in fields]
    group.close()
    for s in sims:
        s.close()
    return g, cases, radius, mass, rho, pres


def test_sweep_radius_and_mass_histories(sweep_run):
    g, cases, radius, mass, _, _ = sweep_run
    disc = ~np.isnan(g["radius"][:, 0])
    er = np.abs(radius[disc] - g["radius"][disc]) / g["radius"][disc]
    em = np.abs(mass - g["mass"]) / g["mass"]
    print("radius history max rel err %.2e, mass %.2e" % (er.max(), em.max()), flush=True)
    for i, case in enumerate(cases):
        print("case %2d T/Tc %.1f: radius %.2e mass %.2e (final mass gpu %.10e oracle %.10e)"
              % (i, case["T_over_Tc"], np.nanmax(np.abs(radius[i] - g["radius"][i]) / g["radius"][i])
                 if disc[i] else 0.0, em[i].max(), mass[i, -1], g["mass"][i, -1]), flush=True)
    assert er.max() < TOL
    assert em.max() < TOL


def _centroid(rho, rho_l):
    """Centre of the density deficit rho_l - rho (x, y) of a sampled field."""
    d = np.clip(rho_l - rho, 0.0, None)
    yy, xx = np.mgrid[0:rho.shape[0], 0:rho.shape[1]]
    return float(np.sum(d * xx) / np.sum(d)), float(np.sum(d * yy) / np.sum(d))


def test_sweep_final_density_fields(sweep_run):
    g, cases, _, _, rho, _ = sweep_run
    worst = 0.0
    for i, case in enumerate(cases):
        ref_s = g["rho_sampled"][i].astype(np.float64)
        scale = max(np.max(np.abs(g["rho_centre_row"][i])), np.max(np.abs(ref_s)))
        e_row = np.abs(rho[i][128] - g["rho_centre_row"][i])
        e_col = np.abs(rho[i][:, 128] - g["rho_centre_col"][i])
        e = max(np.max(np.abs(rho[i][::4, ::4] - ref_s)), np.max(e_row), np.max(e_col)) / scale
        cg = _centroid(rho[i][::4, ::4], float(g["rho_l"][i]))
        co = _centroid(ref_s, float(g["rho_l"][i]))
        print("case %2d T/Tc %.1f R %2g slab %3d: max rel err %.2e (row max at x=%d, column max at y=%d), "
              "deficit centre shift (%.2e, %.2e) sites"
              % (i, case["T_over_Tc"], case["bubbles"][0][2] if case["bubbles"] else 0, case["slab_rows"], e,
                 int(np.argmax(e_row)), int(np.argmax(e_col)), 4 * (cg[0] - co[0]), 4 * (cg[1] - co[1])),
              flush=True)
        worst = max(worst, e)
    print("final density fields max rel err %.2e" % worst, flush=True)
    assert worst < TOL


def test_sweep_pressure_jumps_and_slab_densities(sweep_run):
    g, cases, radius, _, rho, pres = sweep_run
    for i, case in enumerate(cases):
        T = float(g["T"][i])
        if case["bubbles"]:
            cx, cy, _ = case["bubbles"][0]
            dp = diagnostics.pressure_jump(pres[i], (cx, cy), float(g["radius"][i, -1]), 5.0)[0]
            bound = 2 * _eos_slope_bound(T, float(g["rho_g"][i]) * 0.5, float(g["rho_l"][i]) * 1.02) \
                * TOL * float(g["rho_l"][i])
            print("case %d T/Tc %.1f R %g dp %.6e oracle %.6e diff %.2e bound %.2e"
                  % (i, case["T_over_Tc"], case["bubbles"][0][2], dp, g["dp"][i], dp - g["dp"][i], bound),
                  flush=True)
            assert abs(dp - g["dp"][i]) <= bound
        else:
            gs, ls = diagnostics.slab_densities(rho[i], case["slab_rows"])
            scale = float(g["slab_rho_l"][i])
            print("slab T/Tc %.1f rho_g %.6e (oracle %.6e, rel %.1e) rho_l %.6f (oracle %.6f)"
                  % (case["T_over_Tc"], gs, g["slab_rho_g"][i], abs(gs / g["slab_rho_g"][i] - 1), ls,
                     g["slab_rho_l"][i]), flush=True)
            assert abs(gs - g["slab_rho_g"][i]) / scale < TOL
            assert abs(ls - g["slab_rho_l"][i]) / scale < TOL


@pytest.fixture(scope="module")
def collapse_run():
    g = _load(COLLAPSE)
    steps, every = int(g["steps"]), int(g["every"])
    nx, ny = 1024, 768
    p = L.make_params(nx, ny, T=float(g["T"]), walls=True, precision="fp32", tau_nu=float(g["tau_nu"]))
    sim = L.Sim(p)
    sim.init_bubble([tuple(g["bubble"])], rho_l=float(g["rho_l"]), rho_g=float(g["rho_g"]), W=float(g["W"]),
                    delta=float(g["delta"]), noise_amp=float(g["noise_amp"]), seed=int(g["seed"]))
    b = L.Batch(precision="fp32", max_instances=1, max_tiles=L.tile_count(p))
    b.attach(sim)
    b.set_variant(L.variant_names().index("fused2-128x16"))
    radius = np.full(g["radius"].shape, np.nan)
    mass = np.full(g["mass"].shape, np.nan)
    snaps = {}
    snap_steps = [int(s) for s in g["snap_steps"]]
    for k in range(steps // every + 1):
        if k:
            b.step(every)
            b.sync()
        d = sim.diag()
        assert not d["nonfinite"]
        radius[k], mass[k] = d["radius"][0], d["mass"]
        if k * every in snap_steps:
            snaps[k * every] = sim.macros()["rho"].double().cpu().numpy()
    d = sim.diag()
    b.close()
    sim.close()
    return g, radius, mass, snaps, d


def test_collapse_radius_mass_and_wall_peak(collapse_run):
    g, radius, mass, _, d = collapse_run
    er = np.max(np.abs(radius - g["radius"]) / g["radius"])
    em = np.max(np.abs(mass - g["mass"]) / g["mass"])
    ew = abs(d["wall_p_max"] - float(g["wall_p_max"])) / abs(float(g["wall_p_max"]))
    print("radius history max rel err %.2e, mass %.2e, wall peak %.2e (step %d, oracle %d)"
          % (er, em, ew, d["wall_p_step"], int(g["wall_p_step"])), flush=True)
    assert er < TOL and em < TOL and ew < TOL


def _snapshot_err(g, snaps, step):
    j = [int(s) for s in g["snap_steps"]].index(step)
    rho = snaps[step]
    ref = g["snaps"][j]
    e = max(np.max(np.abs(rho[::4, ::4] - ref)), np.max(np.abs(rho[200] - g["snap_rows"][j])),
            np.max(np.abs(rho[:, 511] - g["snap_cols"][j])))
    return float(e / np.max(np.abs(ref)))


@pytest.mark.parametrize("step", [1000, 5000])
def test_collapse_density_field_early(collapse_run, step):
    g, _, _, snaps, _ = collapse_run
    e = _snapshot_err(g, snaps, step)
    print("density field at step %d: max rel err %.2e" % (step, e), flush=True)
    assert e < TOL


@pytest.mark.xfail(strict=True, reason="binary32 storage: the ringing interface drifts past 1e-4 "
                                       "of the density range after about 7000 steps")
@pytest.mark.parametrize("step", [10000, 20000, 50000])
def test_collapse_density_field_late(collapse_run, step):
    g, _, _, snaps, _ = collapse_run
    e = _snapshot_err(g, snaps, step)
    print("density field at step %d: max rel err %.2e" % (step, e), flush=True)
    assert e < TOL
