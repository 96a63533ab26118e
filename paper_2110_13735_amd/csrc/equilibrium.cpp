// Limit states of the space-homogeneous equation (section 'Convergence
// towards a steady state', its practical computations): for given mass rho,
// mean velocity u and internal energy e, the classical Maxwellian (alpha = 0),
// the quantum Maxwellian (1/|alpha|) / (z^-1 exp(|v-u|^2 / 2T) + sgn alpha)
// whose fugacity solves eq. eq_fugacity, the 3-D Bose-Einstein condensate
// (eqs. Tcritical_bosons_3d, m0critical_bosons_3d) or the saturated
// Fermi-Dirac state chi (eqs. def_chi, critical_FD).  Host code: a few
// hundred evaluations of the complete Fermi-Dirac / Bose-Einstein integrals
// per solve.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "../../include/bnq.h"
#include "bnq_internal.h"

namespace bnq {
namespace {

constexpr int kGL = 16;

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_16)
struct GL {
    double x[kGL], w[kGL];
    GL() {
        for (int i = 0; i < kGL; ++i) {
            double t = std::cos(M_PI * (i + 0.75) / (kGL + 0.5)), dp = 1.0;
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = t;
                for (int k = 2; k <= kGL; ++k) {
                    const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = kGL * (t * p1 - p0) / (t * t - 1.0);
                const double dt = p1 / dp;
                t -= dt;
                if (std::fabs(dt) < 1e-16) break;
            }
            x[i] = t;
            w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
        }
    }
};

const GL &gl() {
    static const GL g;
    return g;
}

// Integrand of K_nu without its leading factor: FD, mu <= 0: x^(nu-1) e^-x /
// (1 + e^(mu - x)) (K = e^mu I); FD, mu > 0: x^(nu-1) / (e^(x - mu) + 1)
// (K = I); BE with delta = -ln z >= 0: x^(nu-1) e^-x / (1 - e^(-x - delta))
// (K = e^-delta I).  All over Gamma(nu).
struct Integrand {
    double nu;
    bool fermi;
    double p;  // mu (FD) or delta (BE)
    double core(double x) const {  // the factor besides x^(nu-1)
        if (fermi) return p <= 0 ? std::exp(-x) / (1.0 + std::exp(p - x)) : 1.0 / (std::exp(x - p) + 1.0);
        return std::exp(-x) / -std::expm1(-x - p);
    }
};

// Sum of GL16 over [a, b] in x
double panel_x(const Integrand &f, double a, double b) {
    const GL &g = gl();
    const double c = 0.5 * (a + b), h = 0.5 * (b - a);
    double s = 0;
    for (int i = 0; i < kGL; ++i) {
        const double x = c + h * g.x[i];
        s += g.w[i] * std::pow(x, f.nu - 1.0) * f.core(x);
    }
    return s * h;
}

// GL16 over [sa, sb] in s, x = s^2: integrand 2 s^(2 nu - 1) core(s^2)
double panel_s(const Integrand &f, double sa, double sb) {
    const GL &g = gl();
    const double c = 0.5 * (sa + sb), h = 0.5 * (sb - sa);
    double s = 0;
    for (int i = 0; i < kGL; ++i) {
        const double t = c + h * g.x[i];
        s += g.w[i] * 2.0 * std::pow(t, 2.0 * f.nu - 1.0) * f.core(t * t);
    }
    return s * h;
}

// ln K_nu (FD: p = mu = ln z; BE: p = delta = -ln z >= 0).  Composite
// Gauss-Legendre: the first panel in s = sqrt(x) (removes the x^(nu - 1)
// branch point and, for BE, resolves the pole at x = -delta), geometric panels
// up to x = 1 (and on through the flat part of a degenerate FD integrand),
// then unit panels through the Fermi step and the exponential tail.
double log_K(double nu, bool fermi, double p) {
    Integrand f{nu, fermi, p};
    double a0 = 1.0;
    if (!fermi && p > 0) a0 = std::fmin(p, 1.0);
    const double sa = std::sqrt(a0);
    double sum = panel_s(f, 0.0, 0.5 * sa) + panel_s(f, 0.5 * sa, sa);
    double x = a0;
    while (x < 1.0) {
        const double nx = std::fmin(2.0 * x, 1.0);
        sum += panel_x(f, x, nx);
        x = nx;
    }
    const double mu = fermi ? std::fmax(p, 0.0) : 0.0;
    while (x < mu - 40.0) {  // the flat part of a degenerate FD integrand
        const double nx = std::fmin(2.0 * x, mu - 40.0);
        sum += panel_x(f, x, nx);
        x = nx;
    }
    const double end = mu + 60.0;
    while (x < end) {
        const double nx = std::fmin(x + 1.0, end);
        sum += panel_x(f, x, nx);
        x = nx;
    }
    const double lead = fermi ? (p <= 0 ? p : 0.0) : -p;
    return lead + std::log(sum) - std::lgamma(nu);
}

// ln of K_nu^(nu+1) / K_(nu+1)^nu
double log_ratio(double nu, bool fermi, double p) {
    return (nu + 1.0) * log_K(nu, fermi, p) - nu * log_K(nu + 1.0, fermi, p);
}

// Brent's method (R. P. Brent, Algorithms for Minimization without
// Derivatives, 1973, ch. 4) for a root of g in [a, b], g(a) g(b) <= 0:
// inverse quadratic or secant steps kept inside the bracket, bisection
// whenever they do not shrink it fast enough.
template <typename F>
double brent(F g, double a, double b, double fa, double fb, double tol) {
    double c = a, fc = fa, d = b - a, e = d;
    for (int it = 0; it < 200; ++it) {
        if ((fb > 0) == (fc > 0)) {
            c = a;
            fc = fa;
            d = e = b - a;
        }
        if (std::fabs(fc) < std::fabs(fb)) {
            a = b;
            b = c;
            c = a;
            fa = fb;
            fb = fc;
            fc = fa;
        }
        const double t = 2.0 * 2.2e-16 * std::fabs(b) + 0.5 * tol;
        const double m = 0.5 * (c - b);
        if (std::fabs(m) <= t || fb == 0.0) return b;
        if (std::fabs(e) >= t && std::fabs(fa) > std::fabs(fb)) {
            double p, q, r;
            const double s = fb / fa;
            if (a == c) {
                p = 2.0 * m * s;
                q = 1.0 - s;
            } else {
                q = fa / fc;
                r = fb / fc;
                p = s * (2.0 * m * q * (q - r) - (b - a) * (r - 1.0));
                q = (q - 1.0) * (r - 1.0) * (s - 1.0);
            }
            if (p > 0)
                q = -q;
            else
                p = -p;
            if (2.0 * p < std::fmin(3.0 * m * q - std::fabs(t * q), std::fabs(e * q))) {
                e = d;
                d = p / q;
            } else {
                d = m;
                e = m;
            }
        } else {
            d = m;
            e = m;
        }
        a = b;
        fa = fb;
        b += std::fabs(d) > t ? d : (m > 0 ? t : -t);
        fb = g(b);
    }
    return b;
}

}  // namespace

double complete_fd_be_log(double nu, int fermi, double p) { return log_K(nu, fermi != 0, p); }

int solve_equilibrium(int d, double alpha, double rho, const double *u, double e, bnq_equilibrium *out, char *err,
                      size_t errlen) {
    std::memset(out, 0, sizeof *out);
    out->d = d;
    out->alpha = alpha;
    out->rho = rho;
    for (int i = 0; i < d; ++i) out->u[i] = u ? u[i] : 0.0;
    out->e = e;
    if ((d != 2 && d != 3) || !(rho > 0) || !(e > 0) || !std::isfinite(rho) || !std::isfinite(e) ||
        !std::isfinite(alpha)) {
        std::snprintf(err, errlen, "need d in {2, 3}, finite rho > 0 and e > 0");
        return BNQ_EINVAL;
    }
    const double nu = 0.5 * d;
    if (alpha == 0.0) {
        out->kind = BNQ_EQ_MAXWELL;
        out->T = e / nu;
        return BNQ_OK;
    }
    const bool fermi = alpha > 0;
    const double ratio = std::fabs(alpha) * rho * std::pow(d / (4.0 * M_PI * e), nu);
    out->ratio = ratio;
    const double lx = std::log(ratio);
    if (fermi) {
        // upper end of I_eq: (nu + 1)^nu / Gamma(nu + 1), the ratio of the
        // saturated state chi
        const double upper = std::pow(nu + 1.0, nu) / std::tgamma(nu + 1.0);
        out->A = std::sqrt(2.0 * e * (d + 2.0) / d);
        if (std::fabs(ratio / upper - 1.0) <= 1e-9) {
            out->kind = BNQ_EQ_SATURATED;
            return BNQ_OK;
        }
        if (ratio > upper) {
            out->kind = BNQ_EQ_UNKNOWN;
            return BNQ_OK;
        }
        auto g = [&](double mu) { return log_ratio(nu, true, mu) - lx; };
        // g ~ mu - ln(ratio) as mu -> -inf; g grows to ln(upper / ratio) > 0
        double lo = std::fmin(lx, 0.0) - 4.0, hi = std::fmax(lx, 0.0) + 4.0;
        double glo = g(lo), ghi = g(hi);
        for (int k = 0; glo > 0 && k < 60; ++k) glo = g(lo = 2.0 * lo - 1.0);
        for (int k = 0; ghi < 0 && k < 60; ++k) ghi = g(hi = 2.0 * hi + 1.0);
        if (glo > 0 || ghi < 0) {
            std::snprintf(err, errlen, "no bracket for the Fermi-Dirac fugacity (ratio %.17g)", ratio);
            return BNQ_EINVAL;
        }
        const double mu = brent(g, lo, hi, glo, ghi, 1e-15 * std::fmax(1.0, std::fabs(hi)));
        out->kind = BNQ_EQ_QUANTUM;
        out->log_z = mu;
        out->z = std::exp(mu);
        out->T = e * std::exp(log_K(nu, true, mu) - log_K(nu + 1.0, true, mu)) / nu;
        return BNQ_OK;
    }
    // Bose-Einstein: z = e^-delta in (0, 1]; 3-D has a finite ratio at z = 1
    if (d == 3) {
        const double upper = std::exp(log_ratio(nu, false, 0.0));
        if (ratio >= upper) {
            const double z32 = std::exp(log_K(1.5, false, 0.0)), z52 = std::exp(log_K(2.5, false, 0.0));
            out->kind = BNQ_EQ_CONDENSATE;
            out->z = 1.0;
            out->log_z = 0.0;
            // the z = 1 part carries all the internal energy rho e (the
            // condensate sits at v = u), as in step 3(b) of the rescaled
            // Euler scheme; eq. Tcritical_bosons_3d gives the same T only at
            // the critical ratio, where m0 = 0
            out->T = std::pow(std::fabs(alpha) * rho * e / (std::pow(2.0 * M_PI, 1.5) * 1.5 * z52), 0.4);
            out->m0 = rho - std::pow(2.0 * M_PI * out->T, 1.5) * z32 / std::fabs(alpha);
            return BNQ_OK;
        }
    }
    // root in w = ln delta: g decreases from its z -> 1 value to -inf
    auto g = [&](double w) { return log_ratio(nu, false, std::exp(w)) - lx; };
    double lo = -2.0, hi = std::log(std::fmax(-lx, 0.0) + 8.0);
    double glo = g(lo), ghi = g(hi);
    for (int k = 0; glo < 0 && k < 40; ++k) glo = g(lo = 2.0 * lo - 2.0);
    for (int k = 0; ghi > 0 && k < 40; ++k) ghi = g(hi = hi + 1.0);
    if (glo < 0 || ghi > 0) {
        std::snprintf(err, errlen, "no bracket for the Bose-Einstein fugacity (ratio %.17g)", ratio);
        return BNQ_EINVAL;
    }
    const double w = brent(g, lo, hi, glo, ghi, 1e-15 * std::fmax(1.0, std::fabs(lo)));
    const double delta = std::exp(w);
    out->kind = BNQ_EQ_QUANTUM;
    out->log_z = -delta;
    out->z = std::exp(-delta);
    out->T = e * std::exp(log_K(nu, false, delta) - log_K(nu + 1.0, false, delta)) / nu;
    return BNQ_OK;
}

}  // namespace bnq
