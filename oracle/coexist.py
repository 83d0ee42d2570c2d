"""Coexistence densities of the Carnahan-Starling fluid in multiprecision.

Test infrastructure only (see oracle/__init__.py).

  critical_point        -- the point where dp/drho = d2p/drho2 = 0 (Section 3.1)
  spinodals             -- the two roots of dp/drho = 0 below T_c
  maxwell               -- the equal-area rule of Eq. 11
  mechanical_stability  -- the condition of Eq. 9 with psi from Eq. 13

Every quantity is evaluated from its definition with mpmath (derivatives by
mpmath.diff, integrals by mpmath.quad); the pressure p0 of the two coexisting
phases is found by bisection on the sign of the equal-area integral, which is
monotone in p0 because the integrand's weight is positive.
"""
import functools

import mpmath as mp

DPS = 20


def _ctx():
    mp.mp.dps = DPS


def eos_pressure(rho, T, a=0.5, b=4.0, R=1.0):
    """Eq. 15: p = rho R T (1 + eta + eta^2 - eta^3) / (1 - eta)^3 - a rho^2,
    eta = b rho / 4."""
    rho = mp.mpf(rho)
    eta = mp.mpf(b) * rho / 4
    return rho * R * T * (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3 - a * rho ** 2


def psi(rho, T, a=0.5, b=4.0, R=1.0, G=-1.0):
    """Eq. 13 with c = 1, c_s^2 = 1/3."""
    return mp.sqrt(2 * (eos_pressure(rho, T, a, b, R) - mp.mpf(rho) / 3) / G)


@functools.lru_cache(maxsize=None)
def critical_point(a=0.5, b=4.0, R=1.0):
    """(T_c, rho_c, p_c) where dp/drho = d2p/drho2 = 0 (Section 3.1)."""
    _ctx()

    def eqs(rho, T):
        f = lambda r: eos_pressure(r, T, a, b, R)
        return [mp.diff(f, rho, 1), mp.diff(f, rho, 2)]

    # rho_c depends on b only; start from a coarse scan of the inflection.
    rho_c, T_c = mp.findroot(eqs, (mp.mpf("0.52") / b, mp.mpf("0.09") * a))
    return float(T_c), float(rho_c), float(eos_pressure(rho_c, T_c, a, b, R))


def _dp(rho, T, a, b, R):
    return mp.diff(lambda r: eos_pressure(r, T, a, b, R), rho)


@functools.lru_cache(maxsize=None)
def spinodals(T, a=0.5, b=4.0, R=1.0):
    """Gas-side and liquid-side roots of dp/drho = 0 at temperature T < T_c."""
    _ctx()
    T = mp.mpf(T)
    Tc, rho_c, _ = critical_point(a, b, R)
    if T >= Tc:
        raise ValueError("T must be below T_c")
    g = lambda r: _dp(r, T, a, b, R)
    rho_sg = _bisect(g, mp.mpf(1e-12), mp.mpf(rho_c))
    rho_sl = _bisect(g, mp.mpf(rho_c), mp.mpf(4.0 / b) * (1 - mp.mpf(1e-9)))
    return float(rho_sg), float(rho_sl)


def _bisect(fn, lo, hi, iters=200):
    flo = fn(lo)
    fhi = fn(hi)
    if flo * fhi > 0:
        raise ValueError("no sign change in bracket")
    for _ in range(iters):
        mid = (lo + hi) / 2
        fm = fn(mid)
        if fm == 0:
            return mid
        if (fm > 0) == (flo > 0):
            lo, flo = mid, fm
        else:
            hi, fhi = mid, fm
        if hi - lo < mp.mpf(10) ** (-DPS + 4) * max(abs(hi), mp.mpf(1)):
            break
    return (lo + hi) / 2


def _phase_roots(p0, T, a, b, R):
    """Gas and liquid roots of p(rho) = p0 outside the spinodal interval."""
    rho_sg, rho_sl = (mp.mpf(v) for v in spinodals(float(T), a, b, R))
    h = lambda r: eos_pressure(r, T, a, b, R) - p0
    rg = _bisect(h, mp.mpf(10) ** (-DPS + 6), rho_sg)
    rl = _bisect(h, rho_sl, mp.mpf(4.0 / b) * (1 - mp.mpf(1e-12)))
    return rg, rl


def _coexistence(T, weight, a, b, R):
    """Solves p(rho_g) = p(rho_l) = p0 and int_{rho_g}^{rho_l} (p0 - p) w drho = 0."""
    _ctx()
    T = mp.mpf(T)
    rho_sg, rho_sl = (mp.mpf(v) for v in spinodals(float(T), a, b, R))
    p_hi = eos_pressure(rho_sg, T, a, b, R)          # local maximum (gas spinodal)
    p_lo = max(eos_pressure(rho_sl, T, a, b, R), mp.mpf(0))  # local minimum, or 0

    def area(p0):
        rg, rl = _phase_roots(p0, T, a, b, R)
        integrand = lambda r: (p0 - eos_pressure(r, T, a, b, R)) * weight(r)
        return mp.quad(integrand, [rg, rho_sg, rho_sl, rl]), rg, rl

    eps_p = (p_hi - p_lo) * mp.mpf(10) ** (-DPS + 8)
    lo, hi = p_lo + eps_p, p_hi - eps_p
    a_lo, _, _ = area(lo)
    a_hi, _, _ = area(hi)
    if a_lo * a_hi > 0:
        return None
    for _ in range(120):
        mid = (lo + hi) / 2
        am, rg, rl = area(mid)
        if (am > 0) == (a_lo > 0):
            lo, a_lo = mid, am
        else:
            hi = mid
        if hi - lo < abs(mid) * mp.mpf(10) ** (-DPS + 6):
            break
    p0 = (lo + hi) / 2
    rg, rl = _phase_roots(p0, T, a, b, R)
    return float(rg), float(rl), float(p0)


@functools.lru_cache(maxsize=None)
def maxwell(T, a=0.5, b=4.0, R=1.0):
    """Thermodynamic coexistence (rho_g, rho_l, p0) by the equal-area rule,
    Eq. 11: int (p0 - p_EOS) / rho^2 drho = 0."""
    return _coexistence(T, lambda r: 1 / r ** 2, a, b, R)


@functools.lru_cache(maxsize=None)
def mechanical_stability(T, eps, a=0.5, b=4.0, R=1.0, G=-1.0):
    """Coexistence (rho_g, rho_l, p0) predicted for the lattice model by Eq. 9,
    int (p0 - p_EOS) psi' / psi^(1+eps) drho = 0, psi from Eq. 13 (so that
    p_EOS-PL of Eq. 10 equals p_EOS), psi' = dpsi/drho.  None when no p0 in
    the admissible range makes the integral vanish."""
    _ctx()
    Tm = mp.mpf(T)
    ps = lambda r: psi(r, Tm, a, b, R, G)
    weight = lambda r: mp.diff(ps, r) / ps(r) ** (1 + mp.mpf(eps))
    return _coexistence(T, weight, a, b, R)


def temperature(T_over_Tc, a=0.5, b=4.0, R=1.0):
    """Absolute temperature for a reduced temperature T/T_c."""
    return T_over_Tc * critical_point(a, b, R)[0]
