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
