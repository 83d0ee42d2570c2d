"""Binary32 GPU runs against the binary64 oracle over the workloads' full
horizons, in the launch configurations bench.py times.  The oracle's values
come from tests/golden/make_horizon_goldens.py (which calls only oracle/):

  * the Laplace-law / coexistence sweep (24 periodic 256 x 256 instances,
    40,000 steps), as four concurrent batches with write-through stores and
    the two-step kernel: bubble radius and mass every 1000 steps, density
    snapshots at 10,000, 20,000 and 40,000 steps (every fourth site, plus the
    full row and column through the centre), the final pressure jump of every
    disc and the coexisting densities of every slab;
  * the 1024 x 768 wall-bounded collapse (50,000 steps, both instances of its
    configuration) as one batch with the two-step kernel: radius and mass
    every 100 steps, the wall-pressure peak and its step, and density
    snapshots.

(The single-step and two-step kernels step bitwise alike, so the choice
among them does not change these results.)

Tolerances (the binary32 bar): 1e-4 relative on densities (max norm over the
compared sites, relative to the largest reference density) and on the radius
history and mass.  Derived quantities take the bound that 1e-4 on the
densities implies: the pressure jump, |d dp| <= 2 max|dp/drho| 1e-4 rho_max
over the densities of the run.  The sweep's density fields are held to 1e-4
over the full 40,000 steps; the collapse's (both instances of its
configuration: delta 0.02 with noise seed 1, delta 0.01 with seed 2) to
10,000 steps in the max norm and over all 50,000 in the relative L2 norm.
Beyond 10,000 steps the collapse's largest differences sit on its ringing
interface, which the binary32 path has moved by about a thousandth of a site:
where that passes 1e-4 it is a known failure, kept as a strict expected
failure, so that a change in either direction shows.
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
# the two instances of the collapse configuration (delta, noise seed)
COLLAPSES = {"d020_s1": os.path.join(GOLDEN, "collapse_1024x768_50k_d020_s1.npz"),
             "d010_s2": os.path.join(GOLDEN, "collapse_1024x768_50k_d010_s2.npz")}
# whether the binary32 field holds 1e-4 in the max norm past 10,000 steps
# (measured: delta 0.02 1.7e-4 and 2.6e-4 at 20,000 and 50,000 steps, delta
# 0.01 4.8e-5 and 1.2e-4)
LATE_MAX_NORM_HOLDS = {("d020_s1", 20000): False, ("d020_s1", 50000): False,
                       ("d010_s2", 20000): True, ("d010_s2", 50000): False}
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
    group.set_variant(L.variant_names().index("twostep-58x32"))
    radius = np.full(g["radius"].shape, np.nan)
    mass = np.full(g["mass"].shape, np.nan)
    snap_steps = [int(v) for v in g["snap_steps"]]
    snaps = {}
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
        if k * every in snap_steps:
            snaps[k * every] = [s.macros()["rho"].double().cpu().numpy() for s in sims]
    fields = [s.macros() for s in sims]
    rho = [f["rho"].double().cpu().numpy() for f in fields]
    pres = [f["p"].cpu().numpy() for f in fields]
    group.close()
    for s in sims:
        s.close()
    return g, cases, radius, mass, rho, pres, snaps


def test_sweep_radius_and_mass_histories(sweep_run):
    g, cases, radius, mass, _, _, _ = sweep_run
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


def _sweep_field_errors(g, cases, snaps, step):
    """Per instance: max |rho_gpu - rho_oracle| / max rho_oracle over the
    sampled sites and the full centre row and column at `step`, and the shift
    of the density deficit's centre (sites)."""
    j = [int(v) for v in g["snap_steps"]].index(step)
    out = []
    for i, case in enumerate(cases):
        rho = snaps[step][i]
        ref_s = g["rho_sampled"][i, j].astype(np.float64)
        row, col = g["rho_centre_row"][i, j], g["rho_centre_col"][i, j]
        scale = max(np.max(np.abs(row)), np.max(np.abs(ref_s)))
        e = max(np.max(np.abs(rho[::4, ::4] - ref_s)), np.max(np.abs(rho[128] - row)),
                np.max(np.abs(rho[:, 128] - col))) / scale
        cg = _centroid(rho[::4, ::4], float(g["rho_l"][i]))
        co = _centroid(ref_s, float(g["rho_l"][i]))
        out.append((e, 4 * (cg[0] - co[0]), 4 * (cg[1] - co[1])))
        print("step %d case %2d T/Tc %.1f R %2g slab %3d: max rel err %.2e, deficit centre shift (%.1e, %.1e)"
              % (step, i, case["T_over_Tc"], case["bubbles"][0][2] if case["bubbles"] else 0,
                 case["slab_rows"], e, out[-1][1], out[-1][2]), flush=True)
    return out


@pytest.mark.parametrize("step", [10000, 20000])
def test_sweep_density_fields(sweep_run, step):
    g, cases, _, _, _, _, snaps = sweep_run
    worst = max(e for e, _, _ in _sweep_field_errors(g, cases, snaps, step))
    print("step %d: density fields max rel err %.2e" % (step, worst), flush=True)
    assert worst < TOL


def _horizon_errors(g, cases, snaps, slabs):
    errs = _sweep_field_errors(g, cases, snaps, int(g["steps"]))
    return [e for (e, _, _), c in zip(errs, cases) if (c["slab_rows"] > 0) == slabs]


def test_sweep_disc_density_fields_at_the_horizon(sweep_run):
    g, cases, _, _, _, _, snaps = sweep_run
    worst = max(_horizon_errors(g, cases, snaps, slabs=False))
    print("step %d: disc density fields max rel err %.2e" % (int(g["steps"]), worst), flush=True)
    assert worst < TOL


def test_sweep_slab_density_fields_at_the_horizon(sweep_run):
    g, cases, _, _, _, _, snaps = sweep_run
    worst = max(_horizon_errors(g, cases, snaps, slabs=True))
    print("step %d: slab density fields max rel err %.2e" % (int(g["steps"]), worst), flush=True)
    assert worst < TOL


def test_sweep_pressure_jumps_and_slab_densities(sweep_run):
    g, cases, radius, _, rho, pres, _ = sweep_run
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


@pytest.fixture(scope="module", params=sorted(COLLAPSES))
def collapse_run(request):
    g = _load(COLLAPSES[request.param])
    steps, every = int(g["steps"]), int(g["every"])
    nx, ny = 1024, 768
    p = L.make_params(nx, ny, T=float(g["T"]), walls=True, precision="fp32", tau_nu=float(g["tau_nu"]))
    sim = L.Sim(p)
    sim.init_bubble([tuple(g["bubble"])], rho_l=float(g["rho_l"]), rho_g=float(g["rho_g"]), W=float(g["W"]),
                    delta=float(g["delta"]), noise_amp=float(g["noise_amp"]), seed=int(g["seed"]))
    b = L.Batch(precision="fp32", max_instances=1, max_tiles=L.tile_count(p))
    b.attach(sim)
    b.set_variant(L.variant_names().index("twostep-58x24"))
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
    return g, radius, mass, snaps, d, request.param


def test_collapse_radius_mass_and_wall_peak(collapse_run):
    g, radius, mass, _, d, _ = collapse_run
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


@pytest.mark.parametrize("step", [1000, 5000, 10000])
def test_collapse_density_field_early(collapse_run, step):
    g, _, _, snaps, _, _ = collapse_run
    e = _snapshot_err(g, snaps, step)
    print("density field at step %d: max rel err %.2e" % (step, e), flush=True)
    assert e < TOL


@pytest.mark.parametrize("step", [1000, 5000, 10000, 20000, 50000])
def test_collapse_density_field_in_the_mean(collapse_run, step):
    """Over the whole horizon the binary32 field agrees with the oracle's to
    1e-4 in the relative L2 norm over the sampled sites (every fourth site of
    the grid): the differences beyond 10,000 steps that fail the max norm
    (test_collapse_density_field_late) are confined to the ringing
    interface."""
    g, _, _, snaps, _, _ = collapse_run
    j = [int(s) for s in g["snap_steps"]].index(step)
    ref = g["snaps"][j].astype(np.float64)
    got = snaps[step][::4, ::4]
    e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print("density field at step %d: relative L2 err %.2e" % (step, e), flush=True)
    assert e < TOL


@pytest.mark.parametrize("step", [20000, 50000])
def test_collapse_density_field_late(request, collapse_run, step):
    g, _, _, snaps, _, case = collapse_run
    if not LATE_MAX_NORM_HOLDS[(case, step)]:
        request.applymarker(pytest.mark.xfail(
            strict=True, reason="binary32 storage: the ringing interface drifts past 1e-4 of the "
                                "density range after about 10,000 steps"))
    e = _snapshot_err(g, snaps, step)
    print("density field at step %d: max rel err %.2e" % (step, e), flush=True)
    assert e < TOL


@pytest.mark.parametrize("case", sorted(COLLAPSES))
def test_collapse_binary64_follows_the_oracle_over_the_whole_horizon(case):
    """The same 50,000-step collapses in binary64 (the fused single-step
    kernel) against the oracle's runs: the flow amplifies the two programs'
    different rounding orders (unit roundoff 1.1e-16) by up to about 10^7
    over the ringing (density field 2.2e-10 and 1.0e-9 at 50,000 steps for
    delta 0.02 and 0.01), so the field is held to 1e-8, four orders of
    magnitude inside the binary32 bar, the radius history and mass to 1e-10
    and the wall-pressure peak to 1e-12 at the oracle's step.  Binary64
    follows the oracle there where binary32 leaves the bar
    (test_collapse_density_field_late): that failure is the storage
    precision's, not a difference of model or path."""
    g = _load(COLLAPSES[case])
    steps, every = int(g["steps"]), int(g["every"])
    p = L.make_params(1024, 768, T=float(g["T"]), walls=True, precision="fp64", tau_nu=float(g["tau_nu"]))
    sim = L.Sim(p)
    sim.set_variant(L.variant_names().index("fused-64x16"))
    sim.init_bubble([tuple(g["bubble"])], rho_l=float(g["rho_l"]), rho_g=float(g["rho_g"]), W=float(g["W"]),
                    delta=float(g["delta"]), noise_amp=float(g["noise_amp"]), seed=int(g["seed"]))
    snap_steps = [int(s) for s in g["snap_steps"]]
    er = em = 0.0
    field = {}
    for k in range(steps // every + 1):
        if k:
            sim.step(every)
        d = sim.diag()
        assert not d["nonfinite"]
        er = max(er, abs(d["radius"][0] - g["radius"][k]) / g["radius"][k])
        em = max(em, abs(d["mass"] - g["mass"][k]) / g["mass"][k])
        if k * every in snap_steps:
            field[k * every] = _snapshot_err(g, {k * every: sim.macros()["rho"].cpu().numpy()}, k * every)
    d = sim.diag()
    sim.close()
    ew = abs(d["wall_p_max"] - float(g["wall_p_max"])) / abs(float(g["wall_p_max"]))
    print("binary64: radius %.2e mass %.2e wall peak %.2e (step %d); field %s"
          % (er, em, ew, d["wall_p_step"], ", ".join("%d: %.2e" % kv for kv in sorted(field.items()))),
          flush=True)
    assert er < 1e-10 and em < 1e-10
    assert ew < 1e-12 and d["wall_p_step"] == int(g["wall_p_step"])
    assert max(field.values()) < 1e-8
