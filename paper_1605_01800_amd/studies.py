"""The paper's experiments run on the GPU path, each printing one JSON line.

  precision_study     a wall-bounded collapse in binary64, binary32 and binary32
                      with a binary64 EOS: MLUPS, and the error of total mass,
                      bubble radii and the wall-pressure peak against binary64
  laplace_physics     the Laplace-law sweep (Section 3.1, Eq. 17) run to
                      equilibrium: surface tension per temperature, slab
                      densities against the Maxwell rule (Eq. 11)
  coexistence_sweep   flat-interface coexistence densities for several Li
                      coefficients eps (Eq. 14) and viscosities tau_nu
                      (Section 3.1): the eps dependence of the coexistence
                      curve, its independence of tau_nu
  critical_nucleus    heterogeneous cavitation (Section 3.2, Eq. 18): discs
                      of several radii in a stretched liquid; the radius that
                      separates condensing from growing bubbles
  paper_collapse      the collapse between two walls of Section 4 (1801 x 301,
                      R0 = 138, d = 150, T = 0.5 Tc): bubble shape, topology and
                      wall pressure over time

Every input is synthetic (the Eq. 16 profiles with the stated parameters).
Host-side analysis reads the macroscopic fields the library computes; every
lattice update runs in liblbm.
"""
import json
import sys
import time

import numpy as np


def _log(msg):
    print("# " + msg, file=sys.stderr, flush=True)


def record(sim):
    d = sim.diag()
    return {"step": d["step"], "mass": d["mass"], "radius": d["radius"], "wall_p_max": d["wall_p_max"],
            "wall_p_step": d["wall_p_step"], "nonfinite": d["nonfinite"]}


def run_history(L, params, init, steps, every, device, variant=None, extra=None):
    """Steps one instance, recording record(sim) (and extra(sim), merged in)
    every `every` steps; stops at a non-finite state.  Returns the history,
    the stepping MLUPS and the wall time."""
    import torch
    sim = L.Sim(params, device=device)
    if variant is not None:
        sim.set_variant(variant)
    sim.init_bubble(**init)

    def rec():
        r = record(sim)
        if extra is not None:
            r.update(extra(sim))
        return r

    hist = [rec()]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_s = 0.0
    done = 0
    while done < steps:
        n = min(every, steps - done)
        t1 = time.perf_counter()
        try:
            sim.step(n)
            sim.stream.synchronize()
        except L.NonFiniteError:
            hist.append({"step": done + n, "nonfinite": True})
            break
        step_s += time.perf_counter() - t1
        done += n
        try:
            hist.append(rec())
        except L.NonFiniteError:
            hist.append({"step": done, "nonfinite": True})
            break
    total = time.perf_counter() - t0
    sim.close()
    return hist, params.nx * params.ny * done / max(step_s, 1e-9) / 1e6, total


def rel_err_history(h, ref, key, k=None):
    out = []
    for a, b in zip(h, ref):
        if a.get("nonfinite") or b.get("nonfinite"):
            break
        va = a[key] if k is None else a[key][k]
        vb = b[key] if k is None else b[key][k]
        out.append((a["step"], abs(va - vb) / abs(vb) if vb != 0 else abs(va - vb)))
    return out


# ---------------------------------------------------------------------------
def precision_study(device, large, steps, every, tau_nu=None, delta=None):
    """The same wall-bounded collapse in binary64, binary32 and binary32 with
    binary64 EOS/psi: MLUPS of each and the relative error of total mass,
    bubble radii and the wall-pressure peak against binary64.  The grid is the
    first instance of configuration c5 (large) or c3; tau_nu and delta, when
    given, replace the configured ones."""
    from . import inputs
    from . import lbm as L
    inst = inputs.config_instances(inputs.load_config("c5" if large else "c3"))[0]
    name = "precision_large" if large else "collapse_horizon"
    nx, ny, bub = inst["nx"], inst["ny"], inst["bubbles"]
    tau_nu = inst["tau_nu"] if tau_nu is None else tau_nu
    delta = inst["delta"] if delta is None else delta
    init = dict(bubbles=bub, W=inst["W"], delta=delta, noise_amp=inst["noise_amp"], seed=inst["seed"])
    runs = {}
    for prec in ("fp64", "fp32", "fp32_mixed"):
        p = L.make_params(nx, ny, T_over_Tc=inst["T_over_Tc"], walls=inst["walls"], precision=prec,
                          tau_nu=tau_nu, eps=inst["eps"])
        hist, mlups, total = run_history(L, p, init, steps, every, device,
                                         variant=L.variant_names().index("fused-64x16"))
        runs[prec] = {"hist": hist, "mlups": mlups}
        _log("%s %s: %.0f MLUPS over %d steps (%.1f s)" % (name, prec, mlups, hist[-1]["step"], total))
    ref = runs["fp64"]["hist"]
    out = {"metric": name, "grid": "%dx%d" % (nx, ny), "walls_y": inst["walls"], "T_over_Tc": inst["T_over_Tc"],
           "tau_nu": tau_nu, "eps": inst["eps"], "delta": delta, "bubbles": [list(b) for b in bub], "steps": steps, "record_every": every,
           "reference": "binary64 GPU path (within 1e-12 of the FP64 oracle over 10^4 steps)", "runs": {}}
    for prec, r in runs.items():
        h = r["hist"]
        e = {"mlups": round(r["mlups"], 1),
             "bytes_per_site": 144 if prec == "fp64" else 72,
             "frac_of_8TBs": round(r["mlups"] * 1e6 * (144 if prec == "fp64" else 72) / 8e12, 4),
             "steps_done": h[-1]["step"], "nonfinite": bool(h[-1].get("nonfinite"))}
        if prec != "fp64":
            em = rel_err_history(h, ref, "mass")
            e["mass_max_rel_err"] = max(v for _, v in em)
            er = [rel_err_history(h, ref, "radius", k) for k in range(len(bub))]
            e["radius_max_rel_err"] = [max(v for _, v in x) for x in er]
            e["radius_rel_err_vs_step"] = [[s_, max(x[i][1] for x in er)] for i, (s_, _) in enumerate(er[0])]
            hl, rl = h[-1], ref[min(len(ref), len(h)) - 1]
            if not hl.get("nonfinite") and not rl.get("nonfinite"):
                e["wall_p_max"] = hl["wall_p_max"]
                e["wall_p_max_rel_err"] = abs(hl["wall_p_max"] - rl["wall_p_max"]) / abs(rl["wall_p_max"])
                e["wall_p_step"] = hl["wall_p_step"]
                e["wall_p_step_ref"] = rl["wall_p_step"]
        else:
            e["radius_history"] = [[x["step"]] + list(x["radius"]) for x in h if not x.get("nonfinite")]
            e["wall_p_max"] = h[-1].get("wall_p_max")
            e["wall_p_step"] = h[-1].get("wall_p_step")
        out["runs"][prec] = e
    print(json.dumps(out), flush=True)
    return out


# ---------------------------------------------------------------------------
def sim_from_instance(L, inst, precision, device):
    """A Sim in the initial state of one configuration instance
    (inputs.config_instances)."""
    p = L.make_params(inst["nx"], inst["ny"], T_over_Tc=inst["T_over_Tc"], walls=inst["walls"],
                      precision=precision, tau_nu=inst["tau_nu"], eps=inst["eps"])
    s = L.Sim(p, device=device)
    s.init_bubble(inst["bubbles"], slab_rows=inst.get("slab_rows", 0), W=inst["W"], delta=inst.get("delta", 0.0),
                  noise_amp=inst.get("noise_amp", 0.0), seed=inst.get("seed", 0))
    return s


def laplace_sweep_sims(L, precision, device, n=256):
    """The 24 instances of the Laplace-law / coexistence sweep (configuration
    c2) on n x n grids."""
    from . import inputs
    base = inputs.load_config("c2")["defaults"]
    return [sim_from_instance(L, {**base, "nx": n, "ny": n, **case}, precision, device)
            for case in inputs.laplace_sweep_cases(n)]


def _batch_of(L, sims, precision, device, variant="fused-64x16"):
    batch = L.Batch(precision=precision, max_instances=len(sims),
                    max_tiles=sum(L.tile_count(s.params) for s in sims), device=device)
    for s in sims:
        batch.attach(s)
    batch.set_variant(L.variant_names().index(variant))
    return batch


def _slab_densities(rho, half=8):
    """Coexisting densities of a periodic slab: means over 2 half + 1 rows
    around the liquid centre (row (ny-1)/2) and the gas centre half a period
    away, each row averaged over x."""
    ny = rho.shape[0]
    prof = rho.mean(axis=1)
    lm = int(round(0.5 * (ny - 1)))
    gm = (lm + ny // 2) % ny
    rl = float(np.mean(prof[[(lm + j) % ny for j in range(-half, half + 1)]]))
    rg = float(np.mean(prof[[(gm + j) % ny for j in range(-half, half + 1)]]))
    return rl, rg


def laplace_physics(device, steps, n=256):
    """The sweep run to equilibrium in binary32: per temperature the surface
    tension from a least-squares line of the pressure jump against 1/R (Eq. 17,
    reported as p_in - p_out), and the slab's coexisting densities against the
    Maxwell rule (Eq. 11).  A disc whose centre density has risen past the
    mid-density (rho_l + rho_g) / 2 has dissolved and is left out of the fit."""
    from . import inputs
    from . import lbm as L
    sims = laplace_sweep_sims(L, "fp32", device, n)
    cases = inputs.laplace_sweep_cases(n)
    batch = _batch_of(L, sims, "fp32", device)
    # The acoustic transient of the initial profile decays slowly at tau_nu
    # = 0.6 (the slowest mode of a 256 box has a decay time of ~2e4 steps), so
    # the pressure jump and the slab densities are averaged over samples
    # every 250 steps in the last quarter of the run.
    yy, xx = np.mgrid[0:n, 0:n]
    c = 0.5 * (n - 1)
    r = np.hypot(xx - c, yy - c)
    t0 = time.perf_counter()
    batch.step(steps - steps // 4)
    batch.sync()
    dt = time.perf_counter() - t0
    sample_every = 250
    nsamp = max(1, (steps // 4) // sample_every)
    acc = [dict(dp=0.0, R=0.0, rl=0.0, rg=0.0, centre=0.0) for _ in sims]
    for k in range(nsamp):
        t1 = time.perf_counter()
        batch.step(sample_every)
        batch.sync()
        dt += time.perf_counter() - t1
        for a, s, case in zip(acc, sims, cases):
            m = s.macros()
            rho = m["rho"].double().cpu().numpy()
            if case["slab_rows"]:
                rl, rg = _slab_densities(rho)
                a["rl"] += rl / nsamp
                a["rg"] += rg / nsamp
            else:
                p = m["p"].cpu().numpy()
                R = m["diag"]["radius"][0]
                a["R"] += R / nsamp
                a["centre"] += float(rho[r < 2.0].mean()) / nsamp
                inside, outside = r < R - 10.0, r > R + 10.0
                if inside.any():
                    a["dp"] += float(p[inside].mean() - p[outside].mean()) / nsamp
    per_T = {}
    for a, case in zip(acc, cases):
        tr = case["T_over_Tc"]
        g, l, _ = L.maxwell(L.temperature(tr))
        e = per_T.setdefault(tr, {"R": [], "dp": [], "R0": [], "dissolved": [], "maxwell": (g, l)})
        if case["slab_rows"]:
            e["slab_rho_l"], e["slab_rho_g"] = a["rl"], a["rg"]
        elif a["centre"] > 0.5 * (g + l):
            e["dissolved"].append(case["bubbles"][0][2])
        else:
            e["R"].append(a["R"])
            e["dp"].append(a["dp"])
            e["R0"].append(case["bubbles"][0][2])
    out = {"metric": "laplace_physics", "grid": "%dx%d" % (n, n), "steps": steps, "tau_nu": 0.6, "eps": 1.86,
           "averaged_over": "%d samples every %d steps in the last quarter" % (nsamp, sample_every),
           "precision": "fp32", "seconds": round(dt, 2), "mlups": round(len(sims) * n * n * steps / dt / 1e6, 1),
           "temperatures": {}}
    for tr, e in sorted(per_T.items()):
        g, l = e["maxwell"]
        t = {"initial_radii": e["R0"], "radii": [round(v, 3) for v in e["R"]], "dp": e["dp"],
             "dissolved_initial_radii": e["dissolved"],
             "slab_rho_l": e.get("slab_rho_l"), "slab_rho_g": e.get("slab_rho_g"),
             "maxwell_rho_l": l, "maxwell_rho_g": g,
             "rho_l_rel_dev": (e["slab_rho_l"] - l) / l, "rho_g_rel_dev": (e["slab_rho_g"] - g) / g}
        if len(e["R"]) >= 2:
            x = 1.0 / np.array(e["R"])
            y = np.array(e["dp"])
            A = np.vstack([x, np.ones_like(x)]).T
            (sig, c0), *_ = np.linalg.lstsq(A, y, rcond=None)
            yf = sig * x + c0
            r2 = 1 - np.sum((y - yf) ** 2) / np.sum((y - y.mean()) ** 2) if len(x) > 2 else 1.0
            t.update({"sigma": float(sig), "intercept": float(c0), "r2": float(r2)})
        out["temperatures"][str(tr)] = t
    batch.close()
    for s in sims:
        s.close()
    print(json.dumps(out), flush=True)
    return out


# ---------------------------------------------------------------------------
def coexistence_sweep(device, steps, T_over_Tc=(0.5, 0.6, 0.7, 0.8, 0.9), eps=(1.0, 1.86, 2.0),
                      tau_nu=(0.51, 0.6, 0.8), nx=64, ny=256, precision="fp64"):
    """Flat liquid slabs (ny / 2 liquid rows in a periodic nx x ny box), one
    instance per (T, eps, tau_nu), each stepped on its own stream in chunks of
    1000 steps and averaged over the last quarter of the run: the coexisting
    densities against the Maxwell rule and against the mechanical-stability
    condition of Eq. 9 for the instance's eps (None where it has no
    solution).  An instance that turns non-finite is
    reported with the step count at which its latch was first seen (a
    multiple of 1000) and stops alone; the others go on."""
    from . import lbm as L
    cases, sims = [], []
    for tr in T_over_Tc:
        for e in eps:
            for tn in tau_nu:
                p = L.make_params(nx, ny, T_over_Tc=tr, precision=precision, tau_nu=tn, eps=e)
                s = L.Sim(p, device=device)
                s.set_variant(L.variant_names().index("fused-64x16"))
                s.init_bubble([], slab_rows=ny // 2, W=5.0)
                sims.append(s)
                cases.append({"T_over_Tc": tr, "eps": e, "tau_nu": tn})
    t0 = time.perf_counter()
    alive = list(range(len(sims)))
    acc = {i: [0.0, 0.0, 0] for i in alive}
    bad = {}
    chunk = 1000
    done = 0
    while done < steps and alive:
        n = min(chunk, steps - done)
        for i in list(alive):
            try:
                sims[i].step(n)
            except L.NonFiniteError:
                bad[i] = done
                alive.remove(i)
        for i in list(alive):
            try:
                sims[i].sync()
            except L.NonFiniteError:
                bad[i] = done + n
                alive.remove(i)
        done += n
        if done > steps - steps // 4:
            for i in list(alive):
                try:
                    rho = sims[i].macros()["rho"].double().cpu().numpy()
                except L.NonFiniteError:
                    bad[i] = done
                    alive.remove(i)
                    continue
                rl, rg = _slab_densities(rho)
                acc[i][0] += rl
                acc[i][1] += rg
                acc[i][2] += 1
    dt = time.perf_counter() - t0
    out = {"metric": "coexistence_sweep", "grid": "%dx%d" % (nx, ny), "slab_rows": ny // 2, "steps": steps,
           "precision": precision, "averaged_over": "the records every %d steps in the last quarter" % chunk,
           "seconds": round(dt, 2), "cases": []}
    for i, c in enumerate(cases):
        T = L.temperature(c["T_over_Tc"])
        g, l, _ = L.maxwell(T)
        try:
            g9, l9, _ = L.mechanical_stability(T, c["eps"])
        except L.LbmError:
            g9 = l9 = None
        e = dict(c)
        e.update({"maxwell_rho_g": g, "maxwell_rho_l": l, "eq9_rho_g": g9, "eq9_rho_l": l9})
        if i in bad or acc[i][2] == 0:
            e["nonfinite_step"] = bad.get(i)
        else:
            e["rho_l"] = acc[i][0] / acc[i][2]
            e["rho_g"] = acc[i][1] / acc[i][2]
            e["rho_l_rel_dev"] = (e["rho_l"] - l) / l
            e["rho_g_rel_dev"] = (e["rho_g"] - g) / g
            if g9 is not None:
                e["rho_l_rel_dev_eq9"] = (e["rho_l"] - l9) / l9
                e["rho_g_rel_dev_eq9"] = (e["rho_g"] - g9) / g9
        out["cases"].append(e)
    for s in sims:
        s.close()
    print(json.dumps(out), flush=True)
    return out


# ---------------------------------------------------------------------------
def cs_pressure(rho, T, a=0.5, b=4.0, R=1.0):
    """Carnahan-Starling pressure, Eq. 15 (eta = b rho / 4), for setting up
    initial states and reading results on the host."""
    eta = b * rho / 4.0
    return rho * R * T * (1 + eta + eta * eta - eta ** 3) / (1 - eta) ** 3 - a * rho * rho


def liquid_density_for_pressure(T, p_target, a=0.5, b=4.0, R=1.0):
    """Density on the liquid branch (above the liquid spinodal) where the
    Carnahan-Starling pressure (Eq. 15) equals p_target, by bisection."""
    def p_eos(rho):
        return cs_pressure(rho, T, a, b, R)

    # liquid spinodal: the largest local minimum of p below the pole
    rs = np.linspace(1e-4, 4.0 / b * 0.999, 200001)
    ps = p_eos(rs)
    k = int(np.argmin(np.where(rs > 0.1, ps, np.inf)))
    lo, hi = rs[k], 4.0 / b * 0.999
    if not (p_eos(lo) < p_target < p_eos(hi)):
        raise ValueError("no liquid density with p = %g at T = %g" % (p_target, T))
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if p_eos(mid) < p_target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def critical_nucleus(device, steps, sigma, r_star=11.3, radii=None, n=401, T_over_Tc=0.5, tau_nu=0.6,
                     precision="fp32"):
    """Eq. 18: a vapour disc in liquid whose pressure lies dP = sigma / r_star
    below the flat-interface coexistence pressure is in unstable equilibrium
    at r_star; smaller discs condense and larger ones grow.  The liquid density
    is set from the pressure (the liquid branch of Eq. 15), the vapour at the
    Maxwell gas density, and one periodic n x n instance per initial radius is
    stepped (all in one batch).  Reports each disc's gas radius (cells below
    the mid density) and centre density over time, which discs condensed and
    which grew, and so the measured threshold between the largest condensing
    and the smallest growing disc."""
    from . import lbm as L
    T = L.temperature(T_over_Tc)
    g, l, p0 = L.maxwell(T)
    dP = sigma / r_star
    rho_liq = liquid_density_for_pressure(T, p0 - dP)
    if radii is None:
        radii = [r_star + d for d in (-4, -3, -2, -1.5, -1, -0.5, 0.5, 1, 1.5, 2, 3, 4)]
    c = 0.5 * (n - 1)
    sims = []
    for R0 in radii:
        p = L.make_params(n, n, T_over_Tc=T_over_Tc, precision=precision, tau_nu=tau_nu)
        s = L.Sim(p, device=device)
        s.init_bubble([(c, c, float(R0))], rho_l=rho_liq, rho_g=g, W=5.0)
        sims.append(s)
    batch = _batch_of(L, sims, precision, device)
    ic = int(round(c))
    mid = 0.5 * (rho_liq + g)

    def state():
        # gas radius sqrt(A / pi) of the cells below the mid density, and the
        # centre density (the area-weighted radius of the diagnostics cannot
        # tell a condensed disc from a stretched liquid: both hold the same
        # mass deficit)
        out = []
        for s in sims:
            rho = s.macros()["rho"].double().cpu().numpy()
            out.append((float(np.sqrt((rho < mid).sum() / np.pi)), float(rho[ic, ic])))
        return out

    t0 = time.perf_counter()
    hist = [state()]
    every = max(1, steps // 20)
    done = 0
    while done < steps:
        k = min(every, steps - done)
        batch.step(k)
        batch.sync()
        done += k
        hist.append(state())
    dt = time.perf_counter() - t0
    first, final = hist[0], hist[-1]
    condensed = [R0 for R0, f in zip(radii, final) if f[1] > mid]
    grown = [R0 for R0, f0, f in zip(radii, first, final) if f[1] <= mid and f[0] > f0[0] + 0.5]
    steady = [R0 for R0 in radii if R0 not in condensed and R0 not in grown]
    out = {"metric": "critical_nucleus", "grid": "%dx%d" % (n, n), "T_over_Tc": T_over_Tc, "tau_nu": tau_nu,
           "eps": 1.86, "precision": precision, "steps": steps, "sigma": sigma, "r_star_target": r_star,
           "dP": dP, "p_coexistence": p0, "rho_liquid": rho_liq, "rho_vapour": g,
           "initial_radii": list(radii), "final_gas_radii": [f[0] for f in final],
           "final_centre_density": [f[1] for f in final],
           "gas_radius_history": [[i * every] + [round(x[0], 3) for x in h] for i, h in enumerate(hist)],
           "condensed": condensed, "grown": grown, "neither": steady,
           "largest_condensing": max(condensed) if condensed else None,
           "smallest_growing": min(grown) if grown else None,
           "seconds": round(dt, 2)}
    batch.close()
    for s in sims:
        s.close()
    print(json.dumps(out), flush=True)
    return out


# ---------------------------------------------------------------------------
def gas_shape(rho, mid, x_c, y_c, dy):
    """Shape of the gas region rho < mid: connected components (4-neighbour,
    periodic in x), columns and rows containing gas, gas rows in column x_c,
    and the gas width (cells) of row y_c (the waist of a dumbbell) and the
    larger of rows y_c - dy and y_c + dy (its lobes)."""
    from scipy import ndimage
    gas = rho < mid
    lab, nlab = ndimage.label(gas)
    # join components that meet across the periodic x boundary
    parent = list(range(nlab + 1))

    def find(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i

    for y in range(rho.shape[0]):
        a, b = lab[y, 0], lab[y, -1]
        if a and b:
            parent[find(a)] = find(b)
    comps = {find(i) for i in range(1, nlab + 1)}
    cols = np.flatnonzero(gas.any(axis=0))
    rows = np.flatnonzero(gas.any(axis=1))
    return {"components": len(comps), "gas_radius": float(np.sqrt(gas.sum() / np.pi)),
            "gas_columns": int(cols.size), "gas_rows": int(rows.size), "neck_rows": int(gas[:, x_c].sum()),
            "waist": int(gas[y_c].sum()), "lobes": int(max(gas[y_c - dy].sum(), gas[y_c + dy].sum())),
            "rho_max": float(rho.max())}


def paper_collapse(device, steps, every, tau_nu=(0.51, 0.6), delta=(0.13,), precision="fp32",
                   nx=1801, ny=301, R0=138.0, d=150.0, T_over_Tc=0.5):
    """Section 4: a vapour disc of radius R0 centred d rows above the lower
    wall of a channel of ny rows (walls at y = -1/2 and ny - 1/2, x periodic),
    at T = 0.5 Tc, the liquid over-dense by delta so that the ambient pressure
    exceeds the vapour pressure.  In the closed channel the mass balance lets
    the disc vanish only if delta exceeds its area over the liquid's area
    (12.4% here); below that it shrinks to a new equilibrium.  Per (tau_nu,
    delta): the shape of the gas region over time (components, lateral and
    longitudinal extent, gas rows at the centre column, widths of the waist
    and the lobes of the dumbbell), the densest site, the step it splits in
    two, the step the gas vanishes, and the wall-pressure peak with its
    step.  A run that turns non-finite is reported up to that step."""
    from . import lbm as L
    T = L.temperature(T_over_Tc)
    g, l, _ = L.maxwell(T)
    mid = 0.5 * (g + l)
    xc = 0.5 * (nx - 1)
    runs = []
    for tn in tau_nu:
        for dl in delta:
            p = L.make_params(nx, ny, T_over_Tc=T_over_Tc, walls=True, precision=precision, tau_nu=tn)

            def shape(sim):
                rho = sim.macros()["rho"].double().cpu().numpy()
                return gas_shape(rho, mid, int(round(xc)), int(round(d)), int(0.6 * R0))

            init = dict(bubbles=[(xc, d, R0)], W=5.0, delta=dl)
            hist, mlups, total = run_history(L, p, init, steps, every, device,
                                             variant=L.variant_names().index("fused-64x16"), extra=shape)
            ok = [h for h in hist if not h.get("nonfinite")]
            split = next((h["step"] for h in ok if h["components"] >= 2), None)
            gone = next((h["step"] for h in ok if h["components"] == 0), None)
            e = {"tau_nu": tn, "delta": dl, "mlups": round(mlups, 1), "seconds": round(total, 2),
                 "steps_done": hist[-1]["step"], "nonfinite": bool(hist[-1].get("nonfinite")),
                 "split_step": split, "vanish_step": gone,
                 "wall_p_max": ok[-1]["wall_p_max"], "wall_p_step": ok[-1]["wall_p_step"],
                 "history": [[h["step"], round(h["gas_radius"], 3), h["components"], h["gas_columns"],
                              h["gas_rows"], h["neck_rows"], h["waist"], h["lobes"], round(h["rho_max"], 5)]
                             for h in ok]}
            _log("paper_collapse tau_nu %.2f delta %.3f: %d steps, split %s, vanish %s, nonfinite %s"
                 % (tn, dl, e["steps_done"], split, gone, e["nonfinite"]))
            runs.append(e)
    # Eq. 13 has a real psi only while p_EOS(rho) < rho / 3 (c_s^2 = 1/3)
    lo, hi = l, 0.999999
    for _ in range(200):
        m = 0.5 * (lo + hi)
        lo, hi = (m, hi) if cs_pressure(m, T) < m / 3.0 else (lo, m)
    out = {"metric": "paper_collapse", "grid": "%dx%d" % (nx, ny), "walls_y": True, "R0": R0, "d": d,
           "rho_psi_limit": lo,
           "lambda": R0 / d, "kappa": d / ny, "T_over_Tc": T_over_Tc, "eps": 1.86,
           "precision": precision, "history_columns": ["step", "gas_radius", "components", "gas_columns",
                                                        "gas_rows", "neck_rows", "waist", "lobes", "rho_max"],
           "runs": runs}
    print(json.dumps(out), flush=True)
    return out
