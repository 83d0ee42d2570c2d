"""The allocation-free batch (lbm_batch_create_static: the workspace is the
library's static device array) against the batch on a caller-owned workspace
(lbm_batch_create), through the C ABI: two batches in a row on the same
array, the second with fewer and smaller instances, each stepped bitwise like
the ordinary batch; the limits and the one-per-device rule are refused with
their status codes."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_1605_01800_amd.lbm")


def _sims(specs):
    out = []
    for (nx, ny, walls, tr, bub, delta) in specs:
        p = L.make_params(nx, ny, T_over_Tc=tr, walls=walls, precision="fp32", tau_nu=0.6)
        s = L.Sim(p)
        s.init_bubble(bub, W=4.0, delta=delta, noise_amp=1e-3 if walls else 0.0, seed=3)
        out.append(s)
    return out


def _run(specs, static, variant, counts):
    sims = _sims(specs)
    b = L.Batch(precision="fp32", max_instances=len(sims),
                max_tiles=sum(L.tile_count(s.params) for s in sims), static=static)
    for s in sims:
        b.attach(s)
    b.set_variant(L.variant_names().index(variant))
    for c in counts:
        if isinstance(c, int):
            b.step(c)
        else:
            b.step_each(c)
    status = b.status()
    out = ([s.populations().cpu().numpy() for s in sims], [s.diag() for s in sims], status)
    b.close()
    for s in sims:
        s.close()
    return out


def _same(a, b):
    (fa, da, sa), (fb, db, sb) = a, b
    assert sa == sb == [False] * len(fa)
    for x, y in zip(fa, fb):
        assert np.array_equal(x, y)
    for x, y in zip(da, db):
        assert x == y


BIG = [(200, 90, True, 0.6, [(99.5, 30.0, 20.0)], 0.02),
       (129, 77, False, 0.7, [(64.0, 38.0, 15.0)], 0.0),
       (256, 256, False, 0.8, [(127.5, 127.5, 40.0)], 0.0),
       (70, 150, True, 0.65, [(35.0, 50.0, 12.0)], 0.01),
       (96, 64, False, 0.9, [(47.5, 31.5, 14.0)], 0.0)]
SMALL = [(64, 40, True, 0.7, [(31.5, 14.0, 8.0)], 0.02),
         (80, 48, False, 0.75, [(39.5, 23.5, 10.0)], 0.0)]


def test_static_batch_steps_like_the_ordinary_one_twice_in_a_row():
    print("case static batch: five instances, fused-64x16", flush=True)
    counts = [300, [17, 5, 17, 0, 9], 120]
    _same(_run(BIG, True, "fused-64x16", counts), _run(BIG, False, "fused-64x16", counts))
    # the second batch on the same array: fewer, smaller instances, another
    # kernel family (even nx for the paired kernel)
    print("case static batch: two smaller instances, fused2-128x16", flush=True)
    counts = [50, [7, 3], 256 + 31]
    _same(_run(SMALL, True, "fused2-128x16", counts), _run(SMALL, False, "fused2-128x16", counts))


def test_static_batch_limits_and_one_per_device():
    print("case static batch limits", flush=True)
    lib = L.lib()
    import ctypes
    st = torch.cuda.current_stream().cuda_stream
    b = ctypes.c_void_p()
    assert lib.lbm_batch_create_static(1, 65, 16, st, ctypes.byref(b)) == -2          # LBM_ENOMEM
    assert lib.lbm_batch_create_static(1, 4, 65537, st, ctypes.byref(b)) == -2
    assert lib.lbm_batch_create_static(1, 0, 16, st, ctypes.byref(b)) == -1           # LBM_EINVAL
    assert lib.lbm_batch_create_static(1, 4, 16, st, ctypes.byref(b)) == 0
    c = ctypes.c_void_p()
    assert lib.lbm_batch_create_static(1, 4, 16, st, ctypes.byref(c)) == -5           # LBM_ESTATE
    lib.lbm_batch_destroy(b)
    assert lib.lbm_batch_create_static(1, 4, 16, st, ctypes.byref(c)) == 0
    lib.lbm_batch_destroy(c)
