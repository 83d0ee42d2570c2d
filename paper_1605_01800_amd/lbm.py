"""Python binding of liblbm (include/lbm.h): argument marshalling only.

Every step of the method runs in the HIP kernels of liblbm.so; PyTorch only
provides device memory (the workspaces and output tensors) and streams.  The
library must be built in-tree first (python -m paper_1605_01800_amd.build);
importing this module on a machine without it raises, it never falls back to
another implementation.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_LIB selects another build of the same library (e.g. a tuning experiment)
LIB_PATH = os.environ.get("LBM_LIB") or os.path.join(_HERE, "_lib", "liblbm.so")

FP64, FP32, FP32_MIXED = 0, 1, 2
_PREC = {"fp64": FP64, "fp32": FP32, "fp32_mixed": FP32_MIXED, FP64: FP64, FP32: FP32,
         FP32_MIXED: FP32_MIXED}
MAX_BUBBLES = 8

STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EHIP",
          -4: "LBM_ENONFINITE", -5: "LBM_ESTATE"}


class LbmError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = lib().lbm_strerror(code).decode() if _lib is not None else ""
        super().__init__("%s failed: %s (%s)" % (where, STATUS.get(code, code), msg))


class NonFiniteError(LbmError):
    pass


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("walls_y", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("R", ctypes.c_double), ("T", ctypes.c_double),
                ("G", ctypes.c_double), ("eps", ctypes.c_double),
                ("s_rho", ctypes.c_double), ("s_e", ctypes.c_double),
                ("s_zeta", ctypes.c_double), ("s_j", ctypes.c_double),
                ("s_q", ctypes.c_double), ("s_nu", ctypes.c_double)]


class Bubble(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double), ("r0", ctypes.c_double)]


class Diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("mass", ctypes.c_double),
                ("mom_x", ctypes.c_double), ("mom_y", ctypes.c_double),
                ("n_bubbles", ctypes.c_int32), ("nonfinite", ctypes.c_int32),
                ("gas_area", ctypes.c_double * MAX_BUBBLES),
                ("radius", ctypes.c_double * MAX_BUBBLES),
                ("wall_p_max", ctypes.c_double), ("wall_p_step", ctypes.c_int64)]

    def to_dict(self):
        n = self.n_bubbles
        return {"step": self.step, "mass": self.mass, "mom_x": self.mom_x, "mom_y": self.mom_y,
                "nonfinite": bool(self.nonfinite), "gas_area": list(self.gas_area[:n]),
                "radius": list(self.radius[:n]), "wall_p_max": self.wall_p_max,
                "wall_p_step": self.wall_p_step}


_lib = None

_SIGS = {
    "lbm_workspace_bytes": [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)],
    "lbm_tile_count": [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_int64)],
    "lbm_create": [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                   ctypes.POINTER(ctypes.c_void_p)],
    "lbm_init_bubble": [ctypes.c_void_p, ctypes.POINTER(Bubble), ctypes.c_int, ctypes.c_int,
                        ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                        ctypes.c_double, ctypes.c_uint64],
    "lbm_init_density": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double],
    "lbm_step": [ctypes.c_void_p, ctypes.c_int64],
    "lbm_step_timed": [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_float)],
    "lbm_macros": [ctypes.c_void_p] + [ctypes.c_void_p] * 4 + [ctypes.POINTER(Diag)],
    "lbm_get_populations": [ctypes.c_void_p, ctypes.c_void_p],
    "lbm_set_populations": [ctypes.c_void_p, ctypes.c_void_p],
    "lbm_checkpoint_bytes": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "lbm_save": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t],
    "lbm_load": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t],
    "lbm_sync": [ctypes.c_void_p],
    "lbm_poll": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)],
    "lbm_destroy": [ctypes.c_void_p],
    "lbm_strerror": [ctypes.c_int],
    "lbm_batch_workspace_bytes": [ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)],
    "lbm_batch_create": [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                         ctypes.c_size_t, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)],
    "lbm_batch_attach": [ctypes.c_void_p, ctypes.c_void_p],
    "lbm_batch_detach": [ctypes.c_void_p, ctypes.c_void_p],
    "lbm_batch_step": [ctypes.c_void_p, ctypes.c_int64],
    "lbm_batch_step_each": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int],
    "lbm_batch_prepare": [ctypes.c_void_p, ctypes.c_int64],
    "lbm_batch_create_static": [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                ctypes.POINTER(ctypes.c_void_p)],
    "lbm_batch_step_timed": [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_float)],
    "lbm_batch_size": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)],
    "lbm_batch_poll": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)],
    "lbm_batch_status": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int],
    "lbm_batch_destroy": [ctypes.c_void_p],
    "lbm_batch_set_variant": [ctypes.c_void_p, ctypes.c_int],
    "lbm_batch_set_write_through": [ctypes.c_void_p, ctypes.c_int],
    "lbm_batch_tune_write_through": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_float)],
    "lbm_batch_autotune": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                           ctypes.POINTER(ctypes.c_float)],
    "lbm_variant_count": [],
    "lbm_variant_name": [ctypes.c_int],
    "lbm_resident_blocks": [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
    "lbm_set_variant": [ctypes.c_void_p, ctypes.c_int],
    "lbm_critical_point": [ctypes.c_double] * 3 + [ctypes.POINTER(ctypes.c_double)] * 3,
    "lbm_maxwell": [ctypes.c_double] * 4 + [ctypes.POINTER(ctypes.c_double)] * 3,
    "lbm_mechanical_stability": [ctypes.c_double] * 6 + [ctypes.POINTER(ctypes.c_double)] * 3,
    "lbm_spinodals": [ctypes.c_double] * 4 + [ctypes.POINTER(ctypes.c_double)] * 2,
    "lbm_copy_kernel": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "lbm_device_clock": [ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)],
    "lbm_hold_until": [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p],
}


def lib():
    """The loaded liblbm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblbm.so is not built (%s); run python -m paper_1605_01800_amd.build"
                              % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.lbm_strerror.restype = ctypes.c_char_p
        L.lbm_variant_name.restype = ctypes.c_char_p
        L.lbm_destroy.restype = None
        L.lbm_batch_destroy.restype = None
        _lib = L
    return _lib


def _check(code, where):
    if code == -4:
        raise NonFiniteError(code, where)
    if code != 0:
        raise LbmError(code, where)


# ---- host helpers ----------------------------------------------------------

def critical_point(a=0.5, b=4.0, R=1.0):
    """(T_c, rho_c, p_c) of Eq. 15."""
    out = [ctypes.c_double() for _ in range(3)]
    _check(lib().lbm_critical_point(a, b, R, *[ctypes.byref(o) for o in out]), "lbm_critical_point")
    return tuple(o.value for o in out)


def spinodals(T, a=0.5, b=4.0, R=1.0):
    """(rho_sg, rho_sl): where dp/drho of Eq. 15 vanishes at temperature T."""
    out = [ctypes.c_double() for _ in range(2)]
    _check(lib().lbm_spinodals(a, b, R, T, *[ctypes.byref(o) for o in out]), "lbm_spinodals")
    return tuple(o.value for o in out)


def maxwell(T, a=0.5, b=4.0, R=1.0):
    """(rho_g, rho_l, p0) of the Maxwell rule (Eq. 11) at temperature T."""
    out = [ctypes.c_double() for _ in range(3)]
    _check(lib().lbm_maxwell(a, b, R, T, *[ctypes.byref(o) for o in out]), "lbm_maxwell")
    return tuple(o.value for o in out)


def mechanical_stability(T, eps=1.86, a=0.5, b=4.0, R=1.0, G=-1.0):
    """(rho_g, rho_l, p0) that the lattice model with Li's term settles to by
    the mechanical-stability condition, Eq. 9; LbmError when it has none."""
    out = [ctypes.c_double() for _ in range(3)]
    _check(lib().lbm_mechanical_stability(a, b, R, T, G, eps, *[ctypes.byref(o) for o in out]),
           "lbm_mechanical_stability")
    return tuple(o.value for o in out)


def temperature(T_over_Tc, a=0.5, b=4.0, R=1.0):
    return T_over_Tc * critical_point(a, b, R)[0]


def make_params(nx, ny, T=None, T_over_Tc=None, walls=False, precision="fp32", a=0.5, b=4.0,
                R=1.0, G=-1.0, eps=1.86, tau_nu=0.6, s_rho=1.0, s_e=1.1, s_zeta=1.1, s_j=1.0,
                s_q=1.1, s_nu=None):
    """Parameters with the defaults of Section 3.1 (a = 0.5, b = 4, R = 1, G = -1,
    eps = 1.86, s_rho = s_j = 1.0, s_e = s_zeta = s_q = 1.1, s_nu = 1 / tau_nu)."""
    if T is None:
        if T_over_Tc is None:
            raise ValueError("give T or T_over_Tc")
        T = temperature(T_over_Tc, a, b, R)
    p = Params()
    p.nx, p.ny, p.walls_y, p.precision = int(nx), int(ny), int(bool(walls)), _PREC[precision]
    p.a, p.b, p.R, p.T, p.G, p.eps = a, b, R, T, G, eps
    p.s_rho, p.s_e, p.s_zeta, p.s_j, p.s_q = s_rho, s_e, s_zeta, s_j, s_q
    p.s_nu = (1.0 / tau_nu) if s_nu is None else s_nu
    return p


def workspace_bytes(p):
    n = ctypes.c_size_t()
    _check(lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n)), "lbm_workspace_bytes")
    return n.value


def tile_count(p):
    n = ctypes.c_int64()
    _check(lib().lbm_tile_count(ctypes.byref(p), ctypes.byref(n)), "lbm_tile_count")
    return n.value


def variant_names():
    L = lib()
    return [L.lbm_variant_name(i).decode() for i in range(L.lbm_variant_count())]


def resident_blocks(precision, variant):
    """Blocks of a fused variant's kernel the device holds at once (known after
    the first Sim or Batch is created; 0 for the two-pass variants)."""
    n = ctypes.c_int()
    _check(lib().lbm_resident_blocks(_PREC[precision], int(variant), ctypes.byref(n)), "lbm_resident_blocks")
    return n.value


def _dtype(precision):
    return torch.float64 if precision == FP64 else torch.float32


def _alloc_bytes(nbytes, device):
    # torch's caching allocator returns 512-byte aligned blocks
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    if t.data_ptr() % 256:
        raise RuntimeError("workspace is not 256-byte aligned")
    return t


def _bubbles(bubbles):
    arr = (Bubble * max(1, len(bubbles)))()
    for k, (x0, y0, r0) in enumerate(bubbles):
        arr[k].x0, arr[k].y0, arr[k].r0 = x0, y0, r0
    return arr


class Sim:
    """One instance in a torch-allocated workspace, stepped on its own stream."""

    def __init__(self, params, device="cuda", stream=None):
        self.params = params
        self.device = torch.device(device)
        self.nx, self.ny = params.nx, params.ny
        self.dtype = _dtype(params.precision)
        self.ws_bytes = workspace_bytes(params)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        with torch.cuda.stream(self.stream):
            self.ws = _alloc_bytes(self.ws_bytes, self.device)
        h = ctypes.c_void_p()
        _check(lib().lbm_create(ctypes.byref(params), self.ws.data_ptr(), self.ws_bytes,
                                self.stream.cuda_stream, ctypes.byref(h)), "lbm_create")
        self.h = h
        self.rho_l = self.rho_g = None
        self._batch = None

    @property
    def work_stream(self):
        """The stream the library enqueues this instance's work on: its own, or
        the batch's while it is attached to one."""
        return self._batch.stream if self._batch is not None else self.stream

    # -- state --------------------------------------------------------------
    def init_bubble(self, bubbles=(), slab_rows=0, rho_l=None, rho_g=None, W=5.0, delta=0.0,
                    noise_amp=0.0, seed=0):
        if rho_l is None or rho_g is None:
            g, l, _ = maxwell(self.params.T, self.params.a, self.params.b, self.params.R)
            rho_l = l if rho_l is None else rho_l
            rho_g = g if rho_g is None else rho_g
        self.rho_l, self.rho_g = rho_l, rho_g
        arr = _bubbles(bubbles)
        _check(lib().lbm_init_bubble(self.h, arr, len(bubbles), int(slab_rows), rho_l, rho_g, W,
                                     delta, noise_amp, int(seed)), "lbm_init_bubble")
        return self

    def init_density(self, rho, rho_l=None, rho_g=None):
        """Rest state f_a = w_a rho from a (ny, nx) density field."""
        if rho_l is None or rho_g is None:
            g, l, _ = maxwell(self.params.T, self.params.a, self.params.b, self.params.R)
            rho_l = l if rho_l is None else rho_l
            rho_g = g if rho_g is None else rho_g
        self.rho_l, self.rho_g = rho_l, rho_g
        ws = self.work_stream
        with torch.cuda.stream(ws):
            r = torch.as_tensor(rho, dtype=torch.float64).to(self.device).contiguous()
        assert r.shape == (self.ny, self.nx)
        _check(lib().lbm_init_density(self.h, r.data_ptr(), rho_l, rho_g), "lbm_init_density")
        ws.synchronize()
        return self

    def step(self, n=1):
        _check(lib().lbm_step(self.h, int(n)), "lbm_step")
        return self

    def step_timed(self, n):
        """Steps n times with events around every kernel; returns the summed
        device milliseconds (psi pass, force+collide+stream pass)."""
        ms = (ctypes.c_float * 2)()
        _check(lib().lbm_step_timed(self.h, int(n), ms), "lbm_step_timed")
        return ms[0], ms[1]

    def set_variant(self, v):
        _check(lib().lbm_set_variant(self.h, int(v)), "lbm_set_variant")

    def sync(self):
        _check(lib().lbm_sync(self.h), "lbm_sync")

    def failed(self):
        """Waits for the instance's work and tells whether its state has
        turned non-finite (the latch of lbm_sync)."""
        try:
            self.sync()
        except NonFiniteError:
            return True
        return False

    def poll(self):
        """True when all work enqueued for this instance has finished."""
        done = ctypes.c_int()
        _check(lib().lbm_poll(self.h, ctypes.byref(done)), "lbm_poll")
        return bool(done.value)

    def macros(self, fields=True, check=True):
        """dict with rho, ux, uy (population precision), p (float64) tensors of
        shape (ny, nx) when fields is true, and the diagnostics.  With check
        false a latched non-finite state is reported in diag["nonfinite"]
        instead of raising NonFiniteError."""
        out = {}
        ptrs = [None] * 4
        if fields:
            with torch.cuda.stream(self.work_stream):
                for k, dt in zip(("rho", "ux", "uy", "p"), (self.dtype,) * 3 + (torch.float64,)):
                    out[k] = torch.empty((self.ny, self.nx), dtype=dt, device=self.device)
            ptrs = [out[k].data_ptr() for k in ("rho", "ux", "uy", "p")]
        d = Diag()
        rc = lib().lbm_macros(self.h, *ptrs, ctypes.byref(d))
        if rc != -4 or check:
            _check(rc, "lbm_macros")
        out["diag"] = d.to_dict()
        return out

    def diag(self):
        return self.macros(fields=False)["diag"]

    def populations(self):
        """Post-streaming populations, tensor (9, ny, nx)."""
        ws = self.work_stream
        with torch.cuda.stream(ws):
            f = torch.empty((9, self.ny, self.nx), dtype=self.dtype, device=self.device)
        _check(lib().lbm_get_populations(self.h, f.data_ptr()), "lbm_get_populations")
        ws.synchronize()
        return f

    def set_populations(self, f):
        f = f.to(device=self.device, dtype=self.dtype).contiguous()
        assert f.shape == (9, self.ny, self.nx)
        ws = self.work_stream
        ws.wait_stream(torch.cuda.current_stream(self.device))
        _check(lib().lbm_set_populations(self.h, f.data_ptr()), "lbm_set_populations")
        ws.synchronize()
        return self

    def save(self):
        n = ctypes.c_size_t()
        _check(lib().lbm_checkpoint_bytes(self.h, ctypes.byref(n)), "lbm_checkpoint_bytes")
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().lbm_save(self.h, buf, n.value), "lbm_save")
        return buf.raw

    def load(self, image):
        buf = ctypes.create_string_buffer(image, len(image))
        _check(lib().lbm_load(self.h, buf, len(image)), "lbm_load")
        return self

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            # lbm_destroy detaches the instance from its batch (after the
            # batch's pending work); keep the binding's view in step
            b = getattr(self, "_batch", None)
            if b is not None and self in b.members:
                b.members.remove(self)
            self._batch = None
            lib().lbm_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Instances stepped together, one launch per pass over all their tiles."""

    def __init__(self, precision="fp32", max_instances=64, max_tiles=1 << 16, device="cuda",
                 stream=None, static=False):
        """static: the batch's workspace is the library's static device array
        (lbm_batch_create_static: no allocation at all, one such batch per
        device at a time, at most LBM_STATIC_MAX_INSTANCES instances and
        LBM_STATIC_MAX_TILES tiles)."""
        self.precision = _PREC[precision]
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        b = ctypes.c_void_p()
        if static:
            self.ws = None
            with torch.cuda.device(self.device):
                _check(lib().lbm_batch_create_static(self.precision, int(max_instances), int(max_tiles),
                                                     self.stream.cuda_stream, ctypes.byref(b)),
                       "lbm_batch_create_static")
        else:
            n = ctypes.c_size_t()
            _check(lib().lbm_batch_workspace_bytes(int(max_instances), int(max_tiles), ctypes.byref(n)),
                   "lbm_batch_workspace_bytes")
            with torch.cuda.stream(self.stream):
                self.ws = _alloc_bytes(n.value, self.device)
            _check(lib().lbm_batch_create(self.precision, int(max_instances), int(max_tiles),
                                          self.ws.data_ptr(), n.value, self.stream.cuda_stream,
                                          ctypes.byref(b)), "lbm_batch_create")
        self.b = b
        self.members = []
        self.write_through = False

    def attach(self, sim):
        _check(lib().lbm_batch_attach(self.b, sim.h), "lbm_batch_attach")
        self.members.append(sim)
        sim._batch = self

    def detach(self, sim):
        _check(lib().lbm_batch_detach(self.b, sim.h), "lbm_batch_detach")
        self.members.remove(sim)
        sim._batch = None

    def set_write_through(self, on):
        """Write-through population stores in the fused 64-column and the
        two-step kernels: faster when several batches run concurrently or the
        grids stay in the caches, slower on grids streamed from HBM; results
        are bitwise the same."""
        _check(lib().lbm_batch_set_write_through(self.b, 1 if on else 0), "lbm_batch_set_write_through")
        self.write_through = bool(on)

    def tune_write_through(self, reps=20):
        """Times the current variant with write-through stores off and on and
        keeps the faster setting; returns (on, ms per step or NaN)."""
        on = ctypes.c_int()
        ms = ctypes.c_float()
        _check(lib().lbm_batch_tune_write_through(self.b, int(reps), ctypes.byref(on), ctypes.byref(ms)),
               "lbm_batch_tune_write_through")
        self.write_through = bool(on.value)
        return self.write_through, ms.value

    def step(self, n=1):
        _check(lib().lbm_batch_step(self.b, int(n)), "lbm_batch_step")

    def prepare(self, n):
        """Readies a following step(n) so that it enqueues only its graph
        launches: descriptors sent, chunk graphs captured and uploaded."""
        _check(lib().lbm_batch_prepare(self.b, int(n)), "lbm_batch_prepare")

    def step_each(self, counts):
        arr = (ctypes.c_int64 * max(1, len(counts)))(*[int(c) for c in counts])
        _check(lib().lbm_batch_step_each(self.b, arr, len(counts)), "lbm_batch_step_each")

    def step_timed(self, n):
        ms = (ctypes.c_float * 2)()
        _check(lib().lbm_batch_step_timed(self.b, int(n), ms), "lbm_batch_step_timed")
        return ms[0], ms[1]

    def set_variant(self, v):
        _check(lib().lbm_batch_set_variant(self.b, int(v)), "lbm_batch_set_variant")

    def autotune(self, reps=20):
        best = ctypes.c_int()
        ms = ctypes.c_float()
        _check(lib().lbm_batch_autotune(self.b, int(reps), ctypes.byref(best), ctypes.byref(ms)),
               "lbm_batch_autotune")
        return best.value, ms.value

    def sync(self):
        self.stream.synchronize()

    def status(self):
        """Non-finite latch of every attached instance (attach order) as of the
        last chunk end, read in one transfer; synchronises the batch."""
        n = len(self.members)
        arr = (ctypes.c_int * max(n, 1))()
        _check(lib().lbm_batch_status(self.b, arr, max(n, 1)), "lbm_batch_status")
        return [bool(arr[i]) for i in range(n)]

    def poll(self):
        """True when all work enqueued on the batch's stream has finished."""
        done = ctypes.c_int()
        _check(lib().lbm_batch_poll(self.b, ctypes.byref(done)), "lbm_batch_poll")
        return bool(done.value)

    def close(self):
        if getattr(self, "b", None) is not None and self.b.value:
            lib().lbm_batch_destroy(self.b)
            self.b = ctypes.c_void_p()
            for m in self.members:
                m._batch = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchGroup:
    """Independent instances spread round-robin over several batches, each on
    its own stream (default priority), stepped together: the batches' kernels
    run concurrently, so one batch's start-up and tail, and the gap at its
    kernel boundaries, overlap another's work.  With more than one batch the
    batches use write-through stores (Batch.set_write_through), so that each
    kernel end has little dirty L2 to write back.  Results are bitwise those
    of one batch (the same kernels on the same tiles)."""

    def __init__(self, sims, precision="fp32", n_batches=4, device="cuda", write_through=None):
        n = max(1, min(int(n_batches), len(sims)))
        if write_through is None:
            write_through = n > 1
        groups = [list(sims[i::n]) for i in range(n)]
        self.batches = []
        for g in groups:
            b = Batch(precision=precision, max_instances=len(g),
                      max_tiles=sum(tile_count(s.params) for s in g), device=device)
            for s in g:
                b.attach(s)
            b.set_write_through(write_through)
            self.batches.append(b)

    @property
    def streams(self):
        return [b.stream for b in self.batches]

    def set_variant(self, v):
        for b in self.batches:
            b.set_variant(v)

    def step(self, n=1):
        for b in self.batches:
            b.step(n)

    def prepare(self, n):
        for b in self.batches:
            b.prepare(n)

    def fork(self, event):
        """Makes every batch's stream wait for `event` (recorded by the caller)."""
        for st in self.streams:
            st.wait_event(event)

    def join(self, stream):
        """Makes `stream` wait for all work enqueued so far on every batch."""
        for st in self.streams:
            if st != stream:
                e = torch.cuda.Event()
                e.record(st)
                stream.wait_event(e)

    def sync(self):
        for b in self.batches:
            b.sync()

    def close(self):
        for b in self.batches:
            b.close()
        self.batches = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def copy_kernel(dst, src, nbytes, stream=None):
    """Plain device copy of nbytes (multiple of 16) with liblbm's copy kernel."""
    s = stream.cuda_stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check(lib().lbm_copy_kernel(dst.data_ptr(), src.data_ptr(), int(nbytes), s), "lbm_copy_kernel")


def device_clock():
    """(tick, rate in Hz) of the current device's constant-rate clock."""
    t, r = ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().lbm_device_clock(ctypes.byref(t), ctypes.byref(r)), "lbm_device_clock")
    return t.value, r.value


def hold_until(tick, max_ticks, stream=None):
    """Holds `stream` until the device clock reaches `tick` (at most
    `max_ticks`, no more than one second's worth)."""
    s = stream.cuda_stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check(lib().lbm_hold_until(int(tick), int(max_ticks), s), "lbm_hold_until")

