"""ctypes binding of the C oracle (lbm_oracle.c).  Test infrastructure only.

Arrays are numpy float64 in the oracle's own layout: populations f[y, x, a]
(shape (ny, nx, 9)), fields g[y, x] (shape (ny, nx)).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


class OracleParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("walls", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("a", ctypes.c_double), ("b", ctypes.c_double),
        ("R", ctypes.c_double), ("T", ctypes.c_double),
        ("G", ctypes.c_double), ("eps", ctypes.c_double),
        ("s", ctypes.c_double * 9),
    ]


def lib():
    """The oracle library: the build of lbm_oracle.c, or the library that the
    ORACLE_LIB environment variable names (the mutation tests load copies of
    the oracle with a planted mistake this way)."""
    global _lib
    if _lib is None:
        L = ctypes.CDLL(os.environ.get("ORACLE_LIB") or _build.ensure_built())
        P = ctypes.POINTER(OracleParams)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_eos_pressure.argtypes = [P, ctypes.c_double]
        L.oracle_eos_pressure.restype = ctypes.c_double
        L.oracle_psi.argtypes = [P, ctypes.c_double]
        L.oracle_psi.restype = ctypes.c_double
        L.oracle_density.argtypes = [P, dp, dp]
        L.oracle_force.argtypes = [P, dp, dp, dp]
        L.oracle_moments.argtypes = [dp, dp]
        L.oracle_equilibrium_moments.argtypes = [ctypes.c_double] * 3 + [dp]
        L.oracle_source.argtypes = [P] + [ctypes.c_double] * 5 + [dp]
        L.oracle_collide_node.argtypes = [P, dp] + [ctypes.c_double] * 3 + [dp]
        L.oracle_collide.argtypes = [P, dp, dp, dp, dp, dp]
        L.oracle_stream.argtypes = [P, dp, dp]
        L.oracle_step.argtypes = [P, dp, ctypes.c_int64]
        L.oracle_step.restype = ctypes.c_int
        L.oracle_step_wall_pressure.argtypes = [P, dp, ctypes.c_int64, dp]
        L.oracle_step_wall_pressure.restype = ctypes.c_int
        L.oracle_macros.argtypes = [P, dp, dp, dp, dp, dp]
        L.oracle_macros.restype = ctypes.c_int
        L.oracle_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.oracle_uniform.restype = ctypes.c_double
        L.oracle_init_density.argtypes = [P, dp, ctypes.c_int, ctypes.c_int] + \
            [ctypes.c_double] * 5 + [ctypes.c_uint64, dp]
        L.oracle_init_populations.argtypes = [P, dp, dp]
        L.oracle_transform.argtypes = [dp, dp]
        L.oracle_velocities.argtypes = [ctypes.POINTER(ctypes.c_int)]
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def relaxation_rates(tau_nu, s_rho=1.0, s_e=1.1, s_zeta=1.1, s_j=1.0, s_q=1.1):
    """Diagonal of Lambda (Eq. 2) in moment order; defaults are the rates of
    Section 3.1 (s_rho = s_j = 1.0, s_e = s_zeta = s_q = 1.1) and s_nu = 1/tau_nu."""
    s_nu = 1.0 / tau_nu
    return (s_rho, s_e, s_zeta, s_j, s_q, s_j, s_q, s_nu, s_nu)


def make_params(nx, ny, T, walls=False, a=0.5, b=4.0, R=1.0, G=-1.0, eps=1.86,
                tau_nu=0.6, s=None):
    P = OracleParams()
    P.nx, P.ny, P.walls = int(nx), int(ny), int(bool(walls))
    P.a, P.b, P.R, P.T, P.G, P.eps = a, b, R, T, G, eps
    rates = s if s is not None else relaxation_rates(tau_nu)
    for k in range(9):
        P.s[k] = float(rates[k])
    return P


def with_grid(P, nx, ny, walls=None):
    """Copy of P on another grid."""
    Q = OracleParams()
    ctypes.pointer(Q)[0] = P
    Q.nx, Q.ny = int(nx), int(ny)
    if walls is not None:
        Q.walls = int(bool(walls))
    return Q


def eos_pressure(P, rho):
    L = lib()
    r = np.asarray(rho, dtype=np.float64)
    out = np.array([L.oracle_eos_pressure(ctypes.byref(P), float(v)) for v in r.ravel()])
    return out.reshape(r.shape) if r.shape else float(out[0])


def psi(P, rho):
    L = lib()
    r = np.asarray(rho, dtype=np.float64)
    out = np.array([L.oracle_psi(ctypes.byref(P), float(v)) for v in r.ravel()])
    return out.reshape(r.shape) if r.shape else float(out[0])


def density(P, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    rho = np.empty((P.ny, P.nx))
    lib().oracle_density(ctypes.byref(P), _ptr(f), _ptr(rho))
    return rho


def force(P, psi_field):
    ps = np.ascontiguousarray(psi_field, dtype=np.float64)
    assert ps.shape == (P.ny, P.nx)
    Fx = np.empty_like(ps)
    Fy = np.empty_like(ps)
    lib().oracle_force(ctypes.byref(P), _ptr(ps), _ptr(Fx), _ptr(Fy))
    return Fx, Fy


def moments(f9):
    f9 = np.ascontiguousarray(f9, dtype=np.float64)
    m = np.empty(9)
    lib().oracle_moments(_ptr(f9), _ptr(m))
    return m


def equilibrium_moments(rho, vx, vy):
    m = np.empty(9)
    lib().oracle_equilibrium_moments(rho, vx, vy, _ptr(m))
    return m


def source(P, vx, vy, Fx, Fy, psi_value):
    S = np.empty(9)
    lib().oracle_source(ctypes.byref(P), vx, vy, Fx, Fy, psi_value, _ptr(S))
    return S


def collide_node(P, f9, psi_value, Fx, Fy):
    f9 = np.ascontiguousarray(f9, dtype=np.float64)
    out = np.empty(9)
    lib().oracle_collide_node(ctypes.byref(P), _ptr(f9), psi_value, Fx, Fy, _ptr(out))
    return out


def collide(P, f, psi_field, Fx, Fy):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    args = [np.ascontiguousarray(x, dtype=np.float64) for x in (psi_field, Fx, Fy)]
    lib().oracle_collide(ctypes.byref(P), _ptr(f), *[_ptr(x) for x in args], _ptr(out))
    return out


def stream(P, fstar):
    fstar = np.ascontiguousarray(fstar, dtype=np.float64)
    out = np.full_like(fstar, np.nan)
    lib().oracle_stream(ctypes.byref(P), _ptr(fstar), _ptr(out))
    return out


def step(P, f, nsteps=1):
    """Advances f (float64, shape (ny, nx, 9), C-contiguous) in place; returns
    the oracle's status (0, or -4 for a non-finite state)."""
    assert f.shape == (P.ny, P.nx, 9)
    return lib().oracle_step(ctypes.byref(P), _ptr(f), int(nsteps))


def step_wall_pressure(P, f, nsteps):
    """Advances f by nsteps steps in place, as step(); returns (status, w) with
    w[t] the largest pressure of Eq. 15 on the wall rows y = 0 and y = ny - 1
    of the state at the start of step t (the wall-pressure reading)."""
    assert f.shape == (P.ny, P.nx, 9)
    w = np.full(int(nsteps), np.nan)
    rc = lib().oracle_step_wall_pressure(ctypes.byref(P), _ptr(f), int(nsteps), _ptr(w))
    return rc, w


def macros(P, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    rho, vx, vy, p = (np.empty((P.ny, P.nx)) for _ in range(4))
    rc = lib().oracle_macros(ctypes.byref(P), _ptr(f), _ptr(rho), _ptr(vx), _ptr(vy), _ptr(p))
    assert rc == 0
    return rho, vx, vy, p


def uniform(seed, i):
    return lib().oracle_uniform(int(seed), int(i))


def init_density(P, bubbles=(), slab_rows=0, rho_l=0.0, rho_g=0.0, W=5.0, delta=0.0,
                 noise_amp=0.0, seed=0):
    b = np.ascontiguousarray(np.asarray(bubbles, dtype=np.float64).reshape(-1))
    if b.size == 0:
        b = np.zeros(3)
    rho = np.empty((P.ny, P.nx))
    lib().oracle_init_density(ctypes.byref(P), _ptr(b), len(bubbles), int(slab_rows),
                              rho_l, rho_g, W, delta, noise_amp, int(seed), _ptr(rho))
    return rho


def init_populations(P, rho):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    f = np.empty((P.ny, P.nx, 9))
    lib().oracle_init_populations(ctypes.byref(P), _ptr(rho), _ptr(f))
    return f


def transform():
    M = np.empty((9, 9))
    Minv = np.empty((9, 9))
    lib().oracle_transform(_ptr(M), _ptr(Minv))
    return M, Minv


def velocities():
    e = (ctypes.c_int * 18)()
    lib().oracle_velocities(e)
    return np.array(list(e)).reshape(9, 2)


def threads():
    """Threads the oracle's OpenMP loops use."""
    return lib().oracle_threads()


def set_threads(n):
    lib().oracle_set_threads(int(n))
