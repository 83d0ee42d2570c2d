"""The workload configurations (paper_1605_01800_amd/configs/c1 ... c5) are
the ones the benchmark, the studies and the oracle references run: each
expands to the instances its description names, and the stored oracle
references were written for exactly those parameters."""
import os

import numpy as np
import pytest

from paper_1605_01800_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_every_configuration_loads_once():
    ids = [inputs.load_config("c%d" % k)["id"] for k in range(1, 6)]
    assert ids == ["c1", "c2", "c3", "c4", "c5"]
    with pytest.raises(KeyError):
        inputs.load_config("c9")


def test_c1_is_the_64x64_binary64_disc():
    cfg = inputs.load_config("c1")
    (i,) = inputs.config_instances(cfg)
    assert cfg["precision"] == "fp64" and cfg["steps"] == 10000 and cfg["record_every"] == 500
    assert (i["nx"], i["ny"], i["walls"], i["T_over_Tc"], i["W"]) == (64, 64, False, 0.7, 2.0)
    assert i["bubbles"] == [(31.5, 31.5, 16.0)]
    # kinematic viscosity 0.1 = c_s^2 (tau_nu - 1/2)
    assert abs((i["tau_nu"] - 0.5) / 3.0 - 0.1) < 1e-15


def test_c2_expands_to_the_24_sweep_instances_of_the_oracle_reference():
    inst = inputs.config_instances(inputs.load_config("c2"))
    assert len(inst) == 24
    assert all((i["nx"], i["ny"], i["walls"], i["tau_nu"], i["W"]) == (256, 256, False, 0.6, 5.0) for i in inst)
    assert [i["slab_rows"] for i in inst].count(128) == 4
    assert inputs.laplace_sweep_cases(256) == [{k: i[k] for k in ("T_over_Tc", "bubbles", "slab_rows")}
                                              for i in inst]
    path = os.path.join(GOLDEN, "laplace_sweep_40k.npz")
    if not os.path.exists(path):
        pytest.skip("oracle reference not generated")
    g = np.load(path, allow_pickle=False)
    assert int(g["steps"]) == inputs.load_config("c2")["steps"]
    assert np.array_equal(g["T_over_Tc"], [i["T_over_Tc"] for i in inst])
    assert np.array_equal(g["slab_rows"], [i["slab_rows"] for i in inst])
    radii = [i["bubbles"][0][2] if i["bubbles"] else 0.0 for i in inst]
    assert np.array_equal(np.nan_to_num(g["R"]), radii)


def test_c3_instances_are_the_oracle_reference_collapses():
    cfg = inputs.load_config("c3")
    inst = inputs.config_instances(cfg)
    assert [(i["delta"], i["seed"]) for i in inst] == [(0.02, 1), (0.01, 2)]
    for i in inst:
        assert (i["nx"], i["ny"], i["walls"], i["T_over_Tc"]) == (1024, 768, True, 0.6)
        path = os.path.join(GOLDEN, "collapse_1024x768_50k_d%03d_s%d.npz" % (round(i["delta"] * 1000), i["seed"]))
        if not os.path.exists(path):
            pytest.skip("oracle reference %s not generated" % os.path.basename(path))
        g = np.load(path, allow_pickle=False)
        assert int(g["steps"]) == cfg["steps"] and int(g["every"]) == cfg["record_every"]
        assert float(g["delta"]) == i["delta"] and int(g["seed"]) == i["seed"]
        assert float(g["noise_amp"]) == i["noise_amp"] and float(g["W"]) == i["W"]
        assert float(g["tau_nu"]) == i["tau_nu"] and float(g["T_over_Tc"]) == i["T_over_Tc"]
        assert tuple(float(v) for v in g["bubble"]) == i["bubbles"][0]


def test_c4_trace_follows_its_configuration():
    cfg = inputs.load_config("c4")
    tr = cfg["trace"]
    reqs = inputs.request_trace()
    assert len(reqs) == tr["n_requests"] == 512
    for r in reqs:
        assert tr["side_lo"] <= min(r["nx"], r["ny"]) and max(r["nx"], r["ny"]) <= tr["side_hi"]
        assert tr["T_over_Tc"][0] <= r["T_over_Tc"] <= tr["T_over_Tc"][1]
        assert tr["steps_lo"] <= r["steps"] <= tr["steps_hi"]
        if r["walls"]:
            assert tr["delta"][0] <= r["delta"] <= tr["delta"][1]
    walls = sum(r["walls"] for r in reqs)
    assert 200 < walls < 312                       # a fair coin per request
    assert inputs.request_trace(5, 3) == inputs.request_trace(5, 3)


def test_c5_places_three_discs_inside_the_walls():
    (i,) = inputs.config_instances(inputs.load_config("c5"))
    assert (i["nx"], i["ny"], i["walls"], i["T_over_Tc"], i["delta"]) == (8192, 4096, True, 0.6, 0.02)
    assert sorted(b[2] for b in i["bubbles"]) == [150.0, 200.0, 300.0]
    for k, (x, y, R) in enumerate(i["bubbles"]):
        assert R + 2 * i["W"] <= y <= i["ny"] - 1 - R - 2 * i["W"]
        for (x2, y2, R2) in i["bubbles"][k + 1:]:
            dx = min(abs(x - x2), i["nx"] - abs(x - x2))
            assert np.hypot(dx, y - y2) >= R + R2 + 4 * i["W"]
