"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: binary64 GPU path within 1e-12 relative (max norm) of the oracle;
binary32 paths within 1e-4 on density fields and bubble radii.  Single steps
from generic states are compared population by population."""
import math

import numpy as np
import pytest

from oracle import coexist, diagnostics, stepper as ostep
from tests.helpers import oracle_params, rel_inf, to_device, to_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_1605_01800_amd.lbm")
from paper_1605_01800_amd import inputs  # noqa: E402

TOL = {"fp64": 1e-12, "fp32": 1e-4, "fp32_mixed": 1e-4}
STEP_TOL = {"fp64": 1e-14, "fp32": 2e-6, "fp32_mixed": 2e-6}


def _bubble_rho(P, T, R, walls=False, W=4.0):
    rg, rl, _ = coexist.maxwell(T)
    c = (0.5 * (P.nx - 1), 0.5 * (P.ny - 1) if not walls else P.ny / 3.0)
    return ostep.init_density(P, bubbles=[(c[0], c[1], R)], rho_l=rl, rho_g=rg, W=W), rg, rl


def _variant(name):
    return L.variant_names().index(name)


@pytest.mark.parametrize("variant,shift", [("2pass-64x4", False), ("fused-64x16", False),
                                           ("fused-64x128", False), ("2pass-64x8", True),
                                           ("fused-64x32", True), ("fused2-128x16", False),
                                           ("fused2-128x64", True), ("twostep-58x32", False),
                                           ("twostep-58x64", True)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_mixed"])
@pytest.mark.parametrize("nx,ny,walls", [(100, 37, False), (100, 37, True), (64, 8, False),
                                         (130, 5, True), (1, 6, False), (3, 1, True),
                                         (200, 131, True), (2, 3, False), (258, 9, True)])
def test_single_step_from_random_state(prec, nx, ny, walls, variant, shift):
    """One step from a generic state on ragged grids (x not a multiple of 64,
    tiny and degenerate sizes, both boundary kinds), for the two-pass and the
    fused kernels, with populations stored plain (reference density 0) or
    shifted by the rest equilibrium of the liquid density."""
    print("case", prec, nx, ny, walls, variant, shift, flush=True)
    if variant.startswith("fused2") and nx % 2:
        pytest.skip("paired variants need an even nx")
    T = coexist.temperature(0.7)
    p = L.make_params(nx, ny, T=T, walls=walls, precision=prec, tau_nu=0.6)
    P = oracle_params(p)
    rho, _, _ = _bubble_rho(P, T, min(nx, ny) / 4.0 + 0.5, walls)
    f0 = inputs.random_populations(rho, seed=nx * 1000 + ny, amp=0.3)
    sim = L.Sim(p)
    sim.set_variant(_variant(variant))
    if shift:
        sim.init_density(rho)            # sets the shift reference to rho_l
    dt = sim.dtype
    sim.set_populations(to_device(f0, dt))
    start = to_oracle(sim.populations())          # the state as the device holds it
    sim.step(1)
    got = to_oracle(sim.populations())
    want = start.copy()
    assert ostep.step(P, want, 1) == 0
    assert rel_inf(got, want) < STEP_TOL[prec]
    sim.close()


@pytest.mark.parametrize("variant,shift", [("twostep-58x16", False), ("twostep-58x24", True),
                                           ("twostep-58x32", False), ("twostep-58x48", True)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_mixed"])
@pytest.mark.parametrize("nx,ny,walls", [(100, 37, False), (100, 37, True), (64, 8, False),
                                         (130, 5, True), (1, 6, False), (3, 1, True),
                                         (200, 131, True), (2, 3, False), (258, 9, True), (59, 2, False)])
@pytest.mark.parametrize("nsteps", [2, 3])
def test_two_step_kernel_from_random_state(prec, nx, ny, walls, variant, shift, nsteps):
    """The two-step kernel from a generic state: two steps in one launch (the
    intermediate state only in LDS) and three (a launch of two, then the odd
    last step alone), on the ragged and degenerate grids of the single-step
    test (strips of 58 columns: x edges inside strips, grids narrower than
    the lane's reach, periodic grids of one and two rows)."""
    print("case", prec, nx, ny, walls, variant, shift, nsteps, flush=True)
    T = coexist.temperature(0.7)
    p = L.make_params(nx, ny, T=T, walls=walls, precision=prec, tau_nu=0.6)
    P = oracle_params(p)
    rho, _, _ = _bubble_rho(P, T, min(nx, ny) / 4.0 + 0.5, walls)
    f0 = inputs.random_populations(rho, seed=nx * 1000 + ny, amp=0.3)
    sim = L.Sim(p)
    sim.set_variant(_variant(variant))
    if shift:
        sim.init_density(rho)
    sim.set_populations(to_device(f0, sim.dtype))
    start = to_oracle(sim.populations())
    sim.step(nsteps)
    got = to_oracle(sim.populations())
    assert sim.diag()["step"] == nsteps
    want = start.copy()
    assert ostep.step(P, want, nsteps) == 0
    assert rel_inf(got, want) < nsteps * STEP_TOL[prec]
    sim.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_variants_are_bitwise_identical(prec):
    """Every tile shape of every kernel family (two-pass, fused, paired,
    two-step) gives the same bits: no halo or ring race, no change of
    arithmetic order, and no fused multiply-add left to the compiler's choice
    (the site arithmetic writes each one out)."""
    T = coexist.temperature(0.7)
    p = L.make_params(150, 70, T=T, walls=True, precision=prec, tau_nu=0.8)
    names = L.variant_names()
    outs = []
    for v in range(len(names)):
        sim = L.Sim(p)
        sim.set_variant(v)
        sim.init_bubble([(74.5, 30.0, 14.0)], W=4.0)
        sim.step(40)
        outs.append(sim.populations().cpu())
        sim.close()
    ref = outs[0]
    for name, o in zip(names, outs):
        err = float((o - ref).abs().max() / ref.abs().max())
        print(name, err, "bitwise" if torch.equal(o, ref) else "differs")
        assert torch.equal(o, ref), name


def test_periodic_64x64_fp64_matches_oracle_over_10000_steps():
    """64 x 64 periodic, FP64, T = 0.7 T_c, bubble R = 16 at the centre, W = 2,
    tau_nu = 0.8 (nu = 0.1); rho field, mass and radius every 500 steps."""
    T = coexist.temperature(0.7)
    rg, rl, _ = coexist.maxwell(T)
    p = L.make_params(64, 64, T=T, precision="fp64", tau_nu=0.8)
    P = oracle_params(p)
    bub = [(31.5, 31.5, 16.0)]
    sim = L.Sim(p).init_bubble(bub, rho_l=rl, rho_g=rg, W=2.0)
    f = ostep.init_populations(P, ostep.init_density(P, bubbles=bub, rho_l=rl, rho_g=rg, W=2.0))
    worst = 0.0
    for k in range(20):
        sim.step(500)
        assert ostep.step(P, f, 500) == 0
        m = sim.macros()
        rho_o = ostep.density(P, f)
        err = rel_inf(m["rho"].cpu().numpy(), rho_o)
        worst = max(worst, err)
        assert err < TOL["fp64"], (k, err)
        mass_o = diagnostics.neumaier_sum(rho_o)
        assert abs(m["diag"]["mass"] - mass_o) / mass_o < 1e-13
        r_o = diagnostics.bubble_radius(rho_o, rl, rg)
        assert abs(m["diag"]["radius"][0] - r_o) / r_o < TOL["fp64"]
        assert m["diag"]["step"] == 500 * (k + 1)
    print("max rel err", worst)
    sim.close()


@pytest.mark.parametrize("prec", ["fp32", "fp32_mixed"])
def test_periodic_64x64_fp32_within_1e4(prec):
    T = coexist.temperature(0.7)
    rg, rl, _ = coexist.maxwell(T)
    p = L.make_params(64, 64, T=T, precision=prec, tau_nu=0.8)
    P = oracle_params(p)
    bub = [(31.5, 31.5, 16.0)]
    sim = L.Sim(p).init_bubble(bub, rho_l=rl, rho_g=rg, W=2.0)
    f = ostep.init_populations(P, ostep.init_density(P, bubbles=bub, rho_l=rl, rho_g=rg, W=2.0))
    for k in range(4):
        sim.step(1000)
        assert ostep.step(P, f, 1000) == 0
        m = sim.macros()
        rho_o = ostep.density(P, f)
        assert rel_inf(m["rho"].cpu().numpy(), rho_o) < TOL[prec]
        r_o = diagnostics.bubble_radius(rho_o, rl, rg)
        assert abs(m["diag"]["radius"][0] - r_o) / r_o < TOL[prec]
    sim.close()


@pytest.mark.parametrize("variant", ["2pass-64x8", "fused-64x32", "fused2-128x32"])
def test_walls_collapse_fp64_matches_oracle(variant):
    """Wall-bounded collapse set-up (Section 4.1): liquid at rho_l (1 + delta),
    seeded noise, halfway bounce-back at both walls."""
    T = coexist.temperature(0.6)
    rg, rl, _ = coexist.maxwell(T)
    p = L.make_params(96, 80, T=T, walls=True, precision="fp64", tau_nu=0.6)
    P = oracle_params(p)
    bub = [(47.5, 30.0, 18.0)]
    kw = dict(rho_l=rl, rho_g=rg, W=5.0, delta=0.02, noise_amp=1e-3, seed=7)
    sim = L.Sim(p)
    sim.set_variant(_variant(variant))
    sim.init_bubble(bub, **kw)
    f = ostep.init_populations(P, ostep.init_density(P, bubbles=bub, **kw))
    assert rel_inf(to_oracle(sim.populations()), f) < 1e-15
    for _ in range(3):
        sim.step(200)
        assert ostep.step(P, f, 200) == 0
        m = sim.macros()
        assert rel_inf(m["rho"].cpu().numpy(), ostep.density(P, f)) < TOL["fp64"]
    sim.close()


def test_macros_match_oracle_fields():
    T = coexist.temperature(0.8)
    p = L.make_params(70, 50, T=T, walls=True, precision="fp64", tau_nu=0.6)
    P = oracle_params(p)
    sim = L.Sim(p).init_bubble([(34.5, 20.0, 10.0)], W=4.0)
    sim.step(300)
    m = sim.macros()
    f = to_oracle(sim.populations())
    rho, vx, vy, pr = ostep.macros(P, f)
    assert rel_inf(m["rho"].cpu().numpy(), rho) < 1e-15
    assert np.max(np.abs(m["ux"].cpu().numpy() - vx)) < 1e-15
    assert np.max(np.abs(m["uy"].cpu().numpy() - vy)) < 1e-15
    assert np.max(np.abs(m["p"].cpu().numpy() - pr)) < 1e-15
    d = m["diag"]
    assert abs(d["mom_x"] - np.sum(rho * vx)) < 1e-13
    assert abs(d["mom_y"] - np.sum(rho * vy)) < 1e-13
    sim.close()


@pytest.mark.parametrize("variant", ["2pass-64x4", "fused-64x64", "fused2-128x32", "twostep-58x64"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_equals_alone_bitwise(prec, variant):
    """Uneven grids stepped together give the bits of each stepped alone, also
    with different step counts per instance."""
    T6, T8 = coexist.temperature(0.6), coexist.temperature(0.8)
    nx3 = 78 if variant.startswith("fused2") else 77
    specs = [(L.make_params(64, 64, T=T8, precision=prec), [(31.5, 31.5, 12.0)]),
             (L.make_params(200, 90, T=T6, walls=True, precision=prec, tau_nu=0.8), [(99.5, 30.0, 20.0)]),
             (L.make_params(nx3, 129, T=T8, precision=prec, tau_nu=0.51), [(38.0, 64.0, 15.0)])]
    counts = [300, 173, 256]
    alone = []
    v = _variant(variant)
    for (p, b), n in zip(specs, counts):
        s = L.Sim(p)
        s.set_variant(v)
        s.init_bubble(b, W=5.0)
        s.step(n)
        alone.append(s.populations().cpu())
        s.close()
    batch = L.Batch(precision=prec, max_instances=4, max_tiles=4096)
    batch.set_variant(v)
    sims = [L.Sim(p).init_bubble(b, W=5.0) for p, b in specs]
    for s in sims:
        batch.attach(s)
    batch.step_each(counts)
    batch.sync()
    for s, a, n in zip(sims, alone, counts):
        assert s.diag()["step"] == n
        assert torch.equal(s.populations().cpu(), a)
    batch.close()


@pytest.mark.parametrize("prec,variant", [("fp32", "fused-64x16"), ("fp64", "fused-64x16"),
                                          ("fp32", "fused2-128x16"), ("fp32_mixed", "fused2-128x16")])
def test_walk_order_does_not_change_results(prec, variant):
    """A fused launch whose tiles all fit on the device walks every other band
    of tiles downwards, a larger one walks them all upwards: the same two
    instances stepped alone (small launches) and beside a filler grid that
    makes the launch too large give the same bits."""
    T6, T8 = coexist.temperature(0.6), coexist.temperature(0.8)
    specs = [(L.make_params(200, 90, T=T6, walls=True, precision=prec, tau_nu=0.8), [(99.5, 30.0, 20.0)]),
             (L.make_params(78, 129, T=T8, precision=prec, tau_nu=0.51), [(38.0, 64.0, 15.0)])]
    v = _variant(variant)
    alone = []
    for p, b in specs:
        s = L.Sim(p)
        s.set_variant(v)
        s.init_bubble(b, W=5.0)
        s.step(150)
        alone.append(s.populations().cpu())
        s.close()
    cap = L.resident_blocks(prec, v)
    assert cap > 0
    assert max(L.tile_count(p) for p, _ in specs) <= cap
    cols = 128 if variant.startswith("fused2") else 64
    nx = cols * (cap // 64 + 1)                   # 1024 rows: 64 bands of 16
    fill = L.Sim(L.make_params(nx, 1024, T=T8, precision=prec)).init_bubble([(nx / 2, 512.0, 100.0)], W=5.0)
    sims = [L.Sim(p).init_bubble(b, W=5.0) for p, b in specs]
    tiles = sum(L.tile_count(s.params) for s in sims + [fill])
    assert tiles > cap, (tiles, cap)
    batch = L.Batch(precision=prec, max_instances=3, max_tiles=tiles)
    batch.set_variant(v)
    for s in sims + [fill]:
        batch.attach(s)
    batch.step_each([150, 150, 1])
    batch.sync()
    for s, a in zip(sims, alone):
        assert torch.equal(s.populations().cpu(), a)
    batch.close()
    for s in sims + [fill]:
        s.close()


@pytest.mark.parametrize("prec,variant", [("fp64", "fused-64x16"), ("fp32", "fused-64x32"),
                                          ("fp32_mixed", "fused-64x16"), ("fp32", "fused2-128x16"),
                                          ("fp32", "twostep-58x32"), ("fp64", "twostep-58x24")])
def test_write_through_stores_do_not_change_results(prec, variant):
    """A batch with write-through population stores steps bitwise like one
    without (the paired kernels ignore the setting), over an odd number of
    steps, so that a two-step batch also takes its last step alone."""
    T6, T8 = coexist.temperature(0.6), coexist.temperature(0.8)
    specs = [(L.make_params(200, 90, T=T6, walls=True, precision=prec, tau_nu=0.8), [(99.5, 30.0, 20.0)]),
             (L.make_params(78, 129, T=T8, precision=prec, tau_nu=0.51), [(38.0, 64.0, 15.0)])]
    out = []
    for wt in (False, True):
        sims = [L.Sim(p).init_bubble(b, W=5.0) for p, b in specs]
        batch = L.Batch(precision=prec, max_instances=2, max_tiles=sum(L.tile_count(p) for p, _ in specs))
        batch.set_variant(_variant(variant))
        batch.set_write_through(wt)
        for s in sims:
            batch.attach(s)
        batch.step(141)
        batch.sync()
        out.append([s.populations().cpu() for s in sims])
        batch.close()
        for s in sims:
            s.close()
    for a, b in zip(*out):
        assert torch.equal(a, b)


def test_write_through_tuning_keeps_a_setting_the_batch_then_uses():
    """lbm_batch_tune_write_through times a two-step batch both ways and keeps
    one setting (returned, with a positive time per step); for a paired
    variant, which ignores the setting, it times nothing and keeps the
    current one.  Results stay bitwise those of an untuned batch."""
    p = L.make_params(130, 66, T=coexist.temperature(0.7), walls=True, precision="fp32", tau_nu=0.8)
    out = []
    for tune in (False, True):
        sim = L.Sim(p).init_bubble([(64.5, 30.0, 12.0)], W=4.0)
        b = L.Batch(precision="fp32", max_instances=1, max_tiles=L.tile_count(p))
        b.attach(sim)
        b.set_variant(_variant("twostep-58x24"))
        if tune:
            on, ms = b.tune_write_through(reps=4)
            assert on in (True, False) and on == b.write_through and ms > 0
            b.set_variant(_variant("fused2-128x16"))
            b.set_write_through(True)
            on2, ms2 = b.tune_write_through(reps=4)
            assert on2 is True and ms2 != ms2                      # NaN: nothing timed
            b.set_variant(_variant("twostep-58x24"))
            b.set_write_through(on)
        else:
            b.step(3 * 2 * (4 + 4))             # the steps the tuning takes: 3 passes x 2 settings
        b.step(41)
        b.sync()
        out.append(sim.populations().cpu())
        b.close()
        sim.close()
    assert torch.equal(out[0], out[1])


def test_paired_variant_rejects_odd_nx():
    p = L.make_params(77, 20, T_over_Tc=0.7, precision="fp32")
    s = L.Sim(p)
    with pytest.raises(L.LbmError):
        s.set_variant(_variant("fused2-128x16"))
    s.close()


def test_checkpoint_roundtrip_is_bitwise():
    T = coexist.temperature(0.7)
    p = L.make_params(90, 60, T=T, walls=True, precision="fp32", tau_nu=0.6)
    a = L.Sim(p).init_bubble([(44.5, 25.0, 12.0)], W=5.0, delta=0.01)
    a.step(123)
    img = a.save()
    a.step(200)
    ref = a.populations().cpu()
    b = L.Sim(p).load(img)
    assert b.diag()["step"] == 123
    b.step(200)
    assert torch.equal(b.populations().cpu(), ref)
    a.close()
    b.close()


def test_nonfinite_state_latches_and_refuses_to_step():
    """A density next to the EOS pole makes psi^2 < 0 (Eq. 13): the step
    latches the error, the next sync reports it, further steps are refused."""
    T = coexist.temperature(0.7)
    p = L.make_params(32, 16, T=T, precision="fp64")
    rho = np.full((16, 32), 0.2)
    rho[5, 7] = 0.99
    f = inputs.random_populations(rho, 0, amp=0.0)
    sim = L.Sim(p)
    sim.set_populations(to_device(f, sim.dtype))
    sim.step(1)
    with pytest.raises(L.NonFiniteError):
        sim.sync()
    with pytest.raises(L.NonFiniteError):
        sim.step(1)
    sim.init_bubble([(15.5, 7.5, 4.0)], W=3.0)      # a fresh state clears the latch
    sim.step(5)
    sim.sync()
    sim.close()


@pytest.mark.parametrize("variant", ["2pass-64x4", "fused-64x16", "fused2-128x16"])
def test_wall_pressure_peak_matches_oracle(variant):
    T = coexist.temperature(0.6)
    rg, rl, _ = coexist.maxwell(T)
    p = L.make_params(80, 48, T=T, walls=True, precision="fp64", tau_nu=0.6)
    P = oracle_params(p)
    bub = [(39.5, 14.0, 9.0)]
    kw = dict(rho_l=rl, rho_g=rg, W=4.0, delta=0.03)
    sim = L.Sim(p)
    sim.set_variant(_variant(variant))
    sim.init_bubble(bub, **kw)
    f = ostep.init_populations(P, ostep.init_density(P, bubbles=bub, **kw))
    best, best_step = -math.inf, -1
    for t in range(300):
        rho = ostep.density(P, f)
        pw = max(np.max(ostep.eos_pressure(P, rho[0])), np.max(ostep.eos_pressure(P, rho[-1])))
        if pw > best:
            best, best_step = pw, t
        ostep.step(P, f, 1)
    sim.step(300)
    d = sim.diag()
    assert d["wall_p_step"] == best_step
    assert abs(d["wall_p_max"] - best) <= 1e-12 * abs(best)
    sim.close()


def test_attached_instance_reads_follow_batch_work():
    """Reads of an instance attached to a batch run on the batch's stream, so
    a read right after batch steps (no explicit sync) sees those steps: the
    populations equal the ones read after a sync and a detach, and the
    diagnostics count the steps."""
    print("case attached reads", flush=True)
    p = L.make_params(2048, 1024, T_over_Tc=0.7, walls=True, precision="fp32", tau_nu=0.6)
    sim = L.Sim(p).init_bubble([(1023.5, 400.0, 150.0)], W=5.0, delta=0.02)
    b = L.Batch(precision="fp32", max_instances=1, max_tiles=L.tile_count(p))
    b.attach(sim)
    b.set_variant(_variant("fused2-128x16"))
    for k in range(3):
        b.step(40)
        early = sim.populations()
        b.sync()
        assert sim.diag()["step"] == 40 * (k + 1)
        assert torch.equal(early, sim.populations())
    b.step(40)
    rho = sim.macros()["rho"]
    b.detach(sim)
    late = sim.populations()
    assert torch.equal(rho, sim.macros()["rho"])
    assert sim.diag()["step"] == 160
    assert late.shape == (9, 1024, 2048)
    b.close()
    sim.close()


def test_poll_reports_completion():
    """lbm_poll / lbm_batch_poll never block and report done once the work
    has finished."""
    print("case poll", flush=True)
    p = L.make_params(1024, 1024, T_over_Tc=0.7, precision="fp32", tau_nu=0.6)
    sim = L.Sim(p).init_bubble([(511.5, 511.5, 100.0)], W=5.0)
    sim.step(500)
    assert isinstance(sim.poll(), bool)
    sim.sync()
    assert sim.poll()
    b = L.Batch(precision="fp32", max_instances=1, max_tiles=L.tile_count(p))
    b.attach(sim)
    b.step(500)
    assert isinstance(b.poll(), bool) and isinstance(sim.poll(), bool)
    b.sync()
    assert b.poll() and sim.poll()
    assert sim.diag()["step"] == 1000
    b.close()
    sim.close()


def test_empty_and_zero_step_calls_are_no_ops():
    """An empty batch steps without error; zero steps, alone or per instance
    in a batch, leave the state and the step counter bitwise unchanged."""
    print("case empty", flush=True)
    p = L.make_params(70, 33, T_over_Tc=0.7, walls=True, precision="fp32", tau_nu=0.6)
    empty = L.Batch(precision="fp32", max_instances=2, max_tiles=64)
    empty.step(10)
    empty.sync()
    assert empty.status() == [] and empty.poll()
    sim = L.Sim(p).init_bubble([(34.5, 12.0, 6.0)], W=4.0, delta=0.01)
    sim.step(5)
    before = sim.populations()
    sim.step(0)
    assert torch.equal(before, sim.populations()) and sim.diag()["step"] == 5
    other = L.Sim(p).init_bubble([(20.5, 20.0, 5.0)], W=4.0)
    b = L.Batch(precision="fp32", max_instances=2, max_tiles=2 * L.tile_count(p))
    b.attach(sim)
    b.attach(other)
    b.step_each([0, 7])
    b.sync()
    assert torch.equal(before, sim.populations()) and sim.diag()["step"] == 5
    assert other.diag()["step"] == 7
    b.close()
    empty.close()
    sim.close()
    other.close()


@pytest.mark.parametrize("variant", ["fused-64x16", "fused2-128x16", "2pass-64x4"])
def test_mixed_precision_uses_binary64_only_in_the_spinodal_interval(variant):
    """LBM_FP32_MIXED evaluates Eqs. 15 and 13 in binary64 only at sites whose
    density lies in the spinodal interval at T widened by a tenth of its width
    on each side.  A state whose densities all lie outside it (gas and liquid
    with a one-site jump, both perturbed by 1 %) steps bitwise like LBM_FP32;
    a state with an Eq. 16 interface, whose densities cross the interval, does
    not, and both stay within the single-step tolerance of the oracle."""
    print("case mixed", variant, flush=True)
    nx, ny = 96, 40
    T = coexist.temperature(0.7)
    rg, rl, _ = coexist.maxwell(T)
    sg, sl = L.spinodals(T)
    pad = 0.1 * (sl - sg)
    rng = np.random.default_rng(5)
    jump = np.where(np.arange(ny)[:, None] < ny // 2, rg, rl) * np.ones((1, nx))
    jump = jump * (1 + 0.01 * (2 * rng.random((ny, nx)) - 1))
    assert not np.any((jump > sg - pad) & (jump < sl + pad))
    p64 = L.make_params(nx, ny, T=T, precision="fp64", tau_nu=0.6)
    bubble, _, _ = _bubble_rho(oracle_params(p64), T, 12.5)
    assert np.any((bubble > sg - pad) & (bubble < sl + pad))
    for rho, same in ((jump, True), (bubble, False)):
        out = {}
        for prec in ("fp32", "fp32_mixed"):
            sim = L.Sim(L.make_params(nx, ny, T=T, precision=prec, tau_nu=0.6))
            sim.set_variant(_variant(variant))
            sim.init_density(rho)
            start = to_oracle(sim.populations())
            sim.step(1)
            got = sim.populations()
            out[prec] = got.cpu().numpy()
            want = start.copy()
            assert ostep.step(oracle_params(sim.params), want, 1) == 0
            assert rel_inf(to_oracle(got), want) < STEP_TOL[prec]
            sim.close()
        assert np.array_equal(out["fp32"], out["fp32_mixed"]) == same


# mirror images of the D2Q9 directions: x -> -x and y -> -y
_MIRROR_X = [0, 3, 2, 1, 4, 6, 5, 8, 7]
_MIRROR_Y = [0, 1, 4, 3, 2, 8, 7, 6, 5]


@pytest.mark.parametrize("variant", ["2pass-64x4", "fused-64x16", "fused2-128x16", "twostep-58x24"])
@pytest.mark.parametrize("prec,walls", [("fp32", False), ("fp32", True), ("fp64", False), ("fp32_mixed", True)])
def test_mirror_symmetric_state_stays_bitwise_symmetric(prec, walls, variant):
    """A disc at the centre of the grid is symmetric under both reflections
    (with walls, the walls are the y mirror's planes too); every kernel's
    rounding is mirror-symmetric, so after 3001 steps the populations are
    still bit for bit their own mirror images (population a at (x, y) equals
    the mirrored population at the mirrored site): the disc cannot drift."""
    print("case mirror", prec, walls, variant, flush=True)
    nx, ny = 96, 70
    p = L.make_params(nx, ny, T_over_Tc=0.7, walls=walls, precision=prec, tau_nu=0.6)
    s = L.Sim(p)
    s.set_variant(_variant(variant))
    s.init_bubble([(0.5 * (nx - 1), 0.5 * (ny - 1), 17.0)], W=5.0, delta=0.01 if walls else 0.0)
    s.step(3001)
    f = s.populations().cpu()
    s.close()
    fx = f[_MIRROR_X].flip(2)
    fy = f[_MIRROR_Y].flip(1)
    assert torch.equal(f, fx)
    assert torch.equal(f, fy)


@pytest.mark.parametrize("walls", [False, True])
def test_binary32_slab_keeps_its_mass(walls):
    """A flat liquid slab is the same in every column, so every column rounds
    alike at every step; with the binary32 rest population rounded
    stochastically each site keeps its mass on average, and the slab's total
    mass stays within 5e-7 over 20,000 steps (rounded to nearest, the
    sweep's 256 x 256 slabs drifted coherently by 4-6e-6 in 40,000 steps).
    The run is bitwise reproducible: the random words come from the site and
    the step counter."""
    print("case slab mass walls", walls, flush=True)
    T = coexist.temperature(0.6)
    p = L.make_params(128, 128, T=T, walls=walls, precision="fp32", tau_nu=0.6)
    out = []
    for _ in range(2):
        s = L.Sim(p)
        s.set_variant(_variant("twostep-58x32"))
        s.init_bubble([], slab_rows=64, W=5.0)
        m0 = s.diag()["mass"]
        s.step(20000)
        d = s.diag()
        assert not d["nonfinite"] and d["step"] == 20000
        out.append((d["mass"] / m0 - 1.0, s.populations().cpu()))
        s.close()
    print("relative mass change %.2e" % out[0][0], flush=True)
    assert abs(out[0][0]) < 5e-7
    assert torch.equal(out[0][1], out[1][1])
