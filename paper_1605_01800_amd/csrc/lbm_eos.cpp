// Host helpers for the Carnahan-Starling equation of state (Eq. 15):
// its critical point and the Maxwell coexistence densities (Eq. 11), in long
// double.  They serve callers that set up runs by reduced temperature and by
// the coexisting densities (the initial profile of Eq. 16 needs rho_l, rho_g).
//
// With eta = (b/4) rho the pressure is p = rho R T Z(eta) - a rho^2,
// Z = (1 + eta + eta^2 - eta^3) / (1 - eta)^3, and
//   dp/drho = R T A(eta) - 2 a rho,  A = (1 + 4eta + 4eta^2 - 4eta^3 + eta^4) / (1 - eta)^4,
//   mu(rho) = R T [ln rho + (8eta - 9eta^2 + 3eta^3) / (1 - eta)^3] - 2 a rho
// (mu is the chemical potential, d mu = dp / rho).  The equal-area rule of
// Eq. 11 is equivalent to p(rho_g) = p(rho_l) and mu(rho_g) = mu(rho_l).
#include <math.h>

#include "lbm.h"

namespace {

typedef long double ld;

struct Cs {
    ld a, k, R, T;   // k = b / 4
    ld p(ld rho) const
    {
        const ld e = k * rho;
        return rho * R * T * (1 + e + e * e - e * e * e) / ((1 - e) * (1 - e) * (1 - e)) - a * rho * rho;
    }
    ld dp(ld rho) const
    {
        const ld e = k * rho;
        const ld om = 1 - e;
        return R * T * (1 + 4 * e + 4 * e * e - 4 * e * e * e + e * e * e * e) / (om * om * om * om) -
               2 * a * rho;
    }
    ld mu(ld rho) const
    {
        const ld e = k * rho;
        const ld om = 1 - e;
        return R * T * (logl(rho) + (8 * e - 9 * e * e + 3 * e * e * e) / (om * om * om)) - 2 * a * rho;
    }
};

// Root of fn on [lo, hi] by bisection; fn(lo) and fn(hi) must differ in sign.
template <typename F>
ld bisect(F fn, ld lo, ld hi)
{
    ld flo = fn(lo);
    for (int i = 0; i < 200; ++i) {
        const ld mid = 0.5L * (lo + hi);
        const ld fm = fn(mid);
        if (fm == 0) return mid;
        if ((fm > 0) == (flo > 0)) {
            lo = mid;
            flo = fm;
        } else {
            hi = mid;
        }
        if (hi - lo <= 1e-19L * fabsl(hi)) break;
    }
    return 0.5L * (lo + hi);
}

// eta at the critical point: d(A(eta)/eta)/deta = 0, i.e. eta A'(eta) = A(eta),
// independent of a, b, R.  Numerator of eta A' - A over (1 - eta)^5.
ld critical_eta()
{
    auto g = [](ld e) {
        const ld N = 1 + 4 * e + 4 * e * e - 4 * e * e * e + e * e * e * e;
        const ld dN = 4 + 8 * e - 12 * e * e + 4 * e * e * e;
        return e * dN * (1 - e) + N * (5 * e - 1);
    };
    return bisect(g, 0.01L, 0.5L);
}

}  // namespace

extern "C" int lbm_critical_point(double a, double b, double R, double *T_c, double *rho_c, double *p_c)
{
    if (!(a > 0) || !(b > 0) || !(R > 0)) return LBM_EINVAL;
    const ld e = critical_eta();
    const ld k = (ld)b / 4;
    const ld rho = e / k;
    const ld om = 1 - e;
    const ld A = (1 + 4 * e + 4 * e * e - 4 * e * e * e + e * e * e * e) / (om * om * om * om);
    // dp/drho = 0 at the critical point: R T A = 2 a rho
    const ld T = 2 * (ld)a * rho / ((ld)R * A);
    Cs cs{(ld)a, k, (ld)R, T};
    if (T_c) *T_c = (double)T;
    if (rho_c) *rho_c = (double)rho;
    if (p_c) *p_c = (double)cs.p(rho);
    return LBM_OK;
}

extern "C" int lbm_spinodals(double a, double b, double R, double T, double *rho_sg, double *rho_sl)
{
    double Tc, rc;
    if (lbm_critical_point(a, b, R, &Tc, &rc, nullptr) != LBM_OK) return LBM_EINVAL;
    if (!(T > 0) || !(T < Tc)) return LBM_EINVAL;
    const Cs cs{(ld)a, (ld)b / 4, (ld)R, (ld)T};
    const ld pole = 4.0L / b;
    // dp/drho = 0 on each side of the critical density: the local maximum of
    // p on the gas side and the local minimum on the liquid side
    if (rho_sg) *rho_sg = (double)bisect([&](ld r) { return cs.dp(r); }, 1e-12L, (ld)rc);
    if (rho_sl) *rho_sl = (double)bisect([&](ld r) { return cs.dp(r); }, (ld)rc, pole * (1 - 1e-12L));
    return LBM_OK;
}

extern "C" int lbm_maxwell(double a, double b, double R, double T, double *rho_g, double *rho_l,
                           double *p0)
{
    double Tc, rc;
    if (lbm_critical_point(a, b, R, &Tc, &rc, nullptr) != LBM_OK) return LBM_EINVAL;
    if (!(T > 0) || !(T < Tc)) return LBM_EINVAL;
    const Cs cs{(ld)a, (ld)b / 4, (ld)R, (ld)T};
    const ld pole = 4.0L / b;
    // spinodals: dp/drho = 0 on each side of the critical density
    const ld sg = bisect([&](ld r) { return cs.dp(r); }, 1e-12L, (ld)rc);
    const ld sl = bisect([&](ld r) { return cs.dp(r); }, (ld)rc, pole * (1 - 1e-12L));
    const ld p_hi = cs.p(sg);
    ld p_lo = cs.p(sl);
    if (p_lo < 0) p_lo = 0;
    auto roots = [&](ld P, ld &g, ld &l) {
        g = bisect([&](ld r) { return cs.p(r) - P; }, 1e-30L, sg);
        l = bisect([&](ld r) { return cs.p(r) - P; }, sl, pole * (1 - 1e-15L));
    };
    // mu_l - mu_g is monotone in p0 (its derivative is 1/rho_l - 1/rho_g); the
    // root is bracketed by the two ends of the admissible pressure range
    auto gap = [&](ld P) {
        ld g, l;
        roots(P, g, l);
        return cs.mu(l) - cs.mu(g);
    };
    const ld lo = p_lo + (p_hi - p_lo) * 1e-15L;
    const ld hi = p_hi - (p_hi - p_lo) * 1e-15L;
    if ((gap(lo) > 0) == (gap(hi) > 0)) return LBM_EINVAL;
    const ld P = bisect(gap, lo, hi);
    ld g, l;
    roots(P, g, l);
    if (rho_g) *rho_g = (double)g;
    if (rho_l) *rho_l = (double)l;
    if (p0) *p0 = (double)P;
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// Coexistence of the lattice model with Li's term: the mechanical-stability
// condition of Eq. 9 for a flat interface,
//   int_{rho_g}^{rho_l} (p0 - p(rho)) psi'(rho) / psi(rho)^(1+eps) drho = 0,
// with p(rho_g) = p(rho_l) = p0 and psi of Eq. 13, psi^2 = 2 (rho/3 - p) / (-G)
// (c = 1, c_s^2 = 1/3), so psi' = (1/3 - dp/drho) / (-G psi).
namespace {

struct Eq9 {
    Cs cs;
    ld mG;    // -G > 0
    ld eps;
    ld p0;
    ld psi(ld rho) const { return sqrtl(2 * (rho / 3 - cs.p(rho)) / mG); }
    // integrand in u = ln rho (d rho = rho du)
    ld f(ld u) const
    {
        const ld rho = expl(u);
        const ld s = psi(rho);
        const ld ds = (1.0L / 3 - cs.dp(rho)) / (mG * s);
        return (p0 - cs.p(rho)) * ds * powl(s, -1 - eps) * rho;
    }
};

// n-point Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on
// P_n from the Chebyshev-like first guess, P_n by the three-term recurrence.
struct GaussLegendre {
    static const int n = 12;
    ld x[n], w[n];
    GaussLegendre()
    {
        const ld pi = 3.14159265358979323846264338327950288L;
        for (int i = 0; i < n; ++i) {
            ld z = cosl(pi * (i + 0.75L) / (n + 0.5L)), dP = 1;
            for (int it = 0; it < 100; ++it) {
                ld p0 = 1, p1 = z;
                for (int k = 2; k <= n; ++k) {
                    const ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dP = n * (z * p1 - p0) / (z * z - 1);
                const ld dz = p1 / dP;
                z -= dz;
                if (fabsl(dz) < 1e-20L) break;
            }
            x[i] = z;
            w[i] = 2 / ((1 - z * z) * dP * dP);
        }
    }
};

// Composite Gauss-Legendre over [ln rho_g, ln rho_l]: the integrand is smooth
// there (psi > 0, and psi' stays finite through the spinodals), and ln rho
// spreads the steep gas side over as many panels as the liquid side.
ld eq9_integral(const Eq9 &q, ld rho_g, ld rho_l)
{
    static const GaussLegendre gl;
    const ld u0 = logl(rho_g), u1 = logl(rho_l);
    const int panels = 96;
    const ld h = (u1 - u0) / panels;
    ld sum = 0;
    for (int i = 0; i < panels; ++i) {
        const ld c = u0 + (i + 0.5L) * h;
        ld part = 0;
        for (int k = 0; k < GaussLegendre::n; ++k) part += gl.w[k] * q.f(c + 0.5L * h * gl.x[k]);
        sum += 0.5L * h * part;
    }
    return sum;
}

}  // namespace

extern "C" int lbm_mechanical_stability(double a, double b, double R, double T, double G, double eps,
                                        double *rho_g, double *rho_l, double *p0)
{
    double Tc, rc;
    if (lbm_critical_point(a, b, R, &Tc, &rc, nullptr) != LBM_OK) return LBM_EINVAL;
    if (!(T > 0) || !(T < Tc) || !(G < 0) || !(eps >= 0)) return LBM_EINVAL;
    Eq9 q{Cs{(ld)a, (ld)b / 4, (ld)R, (ld)T}, -(ld)G, (ld)eps, 0};
    const Cs &cs = q.cs;
    const ld pole = 4.0L / b;
    const ld sg = bisect([&](ld r) { return cs.dp(r); }, 1e-12L, (ld)rc);
    const ld sl = bisect([&](ld r) { return cs.dp(r); }, (ld)rc, pole * (1 - 1e-12L));
    const ld p_hi = cs.p(sg);
    // a gas root needs p0 > 0 (p -> 0+ as rho -> 0); a liquid root p0 > p(sl)
    const ld p_lo = cs.p(sl) > 0 ? cs.p(sl) : 0;
    auto roots = [&](ld P, ld &g, ld &l) {
        g = bisect([&](ld r) { return cs.p(r) - P; }, 1e-300L, sg);
        l = bisect([&](ld r) { return cs.p(r) - P; }, sl, pole * (1 - 1e-15L));
    };
    auto I = [&](ld P) {
        ld g, l;
        roots(P, g, l);
        Eq9 qq = q;
        qq.p0 = P;
        return eq9_integral(qq, g, l);
    };
    // scan the admissible pressures (geometrically near 0) for a sign change
    const int n = 400;
    ld prev_p = 0, prev_i = 0;
    bool have = false, found = false;
    ld lo = 0, hi = 0;
    for (int i = 1; i < n; ++i) {
        const ld t = (ld)i / n;
        const ld P = p_lo > 0 ? p_lo + (p_hi - p_lo) * t : p_hi * powl(1e-12L, 1 - t);
        const ld v = I(P);
        if (!isfinite((double)v)) continue;
        if (have && ((v > 0) != (prev_i > 0))) {
            lo = prev_p;
            hi = P;
            found = true;
            break;
        }
        prev_p = P;
        prev_i = v;
        have = true;
    }
    if (!found) return LBM_EINVAL;   // Eq. 9 has no coexistence at this T and eps
    const ld P = bisect(I, lo, hi);
    ld g, l;
    roots(P, g, l);
    if (rho_g) *rho_g = (double)g;
    if (rho_l) *rho_l = (double)l;
    if (p0) *p0 = (double)P;
    return LBM_OK;
}
