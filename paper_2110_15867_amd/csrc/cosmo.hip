// Background expansion for comoving runs (Eqs. 1, 2 with a(t)): host code.
//
// A flat universe of matter and a cosmological constant (radiation
// neglected): H(a) = H0 sqrt(Om a^-3 + 1 - Om), whose Friedmann equation
// da/dt = a H(a) integrates in closed form,
//   Om < 1:  a(t) = (Om / OL)^(1/3) sinh^(2/3)(3/2 sqrt(OL) H0 t),  OL = 1 - Om
//   Om = 1:  a(t) = (3/2 H0 t)^(2/3),
// with the inverse t(a) = 2 / (3 sqrt(OL) H0) asinh(sqrt(OL / Om) a^(3/2)).
// A drift over [t0, t1] moves a comoving position by u times the integral of
// dt / a(t)^2 (Eq. 1, with u constant during the drift): evaluated by
// adaptive 16-point Gauss-Legendre quadrature (nodes from Newton's method on
// the Legendre polynomial), to about 1e-14 relative.
#include <math.h>
#include <stddef.h>

#include "../../include/vlasov.h"

namespace {

constexpr int GL_N = 16;

struct GaussLegendre {
    double x[GL_N], w[GL_N];
    GaussLegendre()
    {
        for (int i = 0; i < GL_N; ++i) {
            double z = cos(M_PI * (i + 0.75) / (GL_N + 0.5)), dp = 1.0;
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = z;                  // P_0, P_1
                for (int k = 2; k <= GL_N; ++k) {
                    const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = GL_N * (z * p1 - p0) / (z * z - 1.0);  // P_n'(z)
                const double dz = p1 / dp;
                z -= dz;
                if (fabs(dz) < 1e-17) break;
            }
            x[i] = z;
            w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
};

const GaussLegendre& gl()
{
    static const GaussLegendre r;
    return r;
}

bool cosmo_ok(const vlasov_cosmology* c)
{
    return isfinite(c->omega_m) && isfinite(c->H0) && c->omega_m > 0.0 && c->omega_m <= 1.0 &&
           c->H0 > 0.0;
}

double scale_factor(const vlasov_cosmology* c, double t)
{
    const double om = c->omega_m, ol = 1.0 - om;
    if (ol == 0.0) return pow(1.5 * c->H0 * t, 2.0 / 3.0);
    return cbrt(om / ol) * pow(sinh(1.5 * sqrt(ol) * c->H0 * t), 2.0 / 3.0);
}

double cosmic_time(const vlasov_cosmology* c, double a)
{
    const double om = c->omega_m, ol = 1.0 - om;
    if (ol == 0.0) return pow(a, 1.5) / (1.5 * c->H0);
    return asinh(sqrt(ol / om) * pow(a, 1.5)) / (1.5 * sqrt(ol) * c->H0);
}

double gl_inv_a2(const vlasov_cosmology* c, double t0, double t1)
{
    const GaussLegendre& q = gl();
    const double h = 0.5 * (t1 - t0), m = 0.5 * (t1 + t0);
    double s = 0.0;
    for (int i = 0; i < GL_N; ++i) {
        const double a = scale_factor(c, m + h * q.x[i]);
        s += q.w[i] / (a * a);
    }
    return s * h;
}

// whole-interval rule against the sum over its halves, halving where they
// differ by more than 1e-14 of the value (a 16-node rule on a smooth
// integrand is then exact to rounding).  `budget` bounds the rule
// evaluations, so intervals whose two estimates differ only by rounding
// cannot recurse without end.
double drift_integral(const vlasov_cosmology* c, double t0, double t1, double whole, int depth,
                      long& budget)
{
    const double tm = 0.5 * (t0 + t1);
    const double l = gl_inv_a2(c, t0, tm), r = gl_inv_a2(c, tm, t1);
    budget -= 2;
    if (depth >= 40 || budget <= 0 || fabs(l + r - whole) <= 1e-14 * fabs(l + r)) return l + r;
    return drift_integral(c, t0, tm, l, depth + 1, budget) +
           drift_integral(c, tm, t1, r, depth + 1, budget);
}

}  // namespace

extern "C" {

int vlasov_cosmo_a(const vlasov_cosmology* c, double t, double* a)
{
    if (c == nullptr || a == nullptr) return VLASOV_ERR_NULL;
    if (!isfinite(t)) return VLASOV_ERR_NONFINITE;
    if (!cosmo_ok(c) || !(t > 0.0)) return VLASOV_ERR_SHAPE;
    *a = scale_factor(c, t);
    return isfinite(*a) ? VLASOV_OK : VLASOV_ERR_NONFINITE;
}

int vlasov_cosmo_t(const vlasov_cosmology* c, double a, double* t)
{
    if (c == nullptr || t == nullptr) return VLASOV_ERR_NULL;
    if (!isfinite(a)) return VLASOV_ERR_NONFINITE;
    if (!cosmo_ok(c) || !(a > 0.0)) return VLASOV_ERR_SHAPE;
    *t = cosmic_time(c, a);
    return VLASOV_OK;
}

int vlasov_cosmo_steps(const vlasov_cosmology* c, double t0, double dt, int nsteps, double* a,
                       double* a2inv)
{
    if (c == nullptr || a2inv == nullptr) return VLASOV_ERR_NULL;
    if (!isfinite(t0) || !isfinite(dt)) return VLASOV_ERR_NONFINITE;
    if (!cosmo_ok(c) || !(t0 > 0.0) || !(dt > 0.0) || nsteps < 1) return VLASOV_ERR_SHAPE;
    for (int n = 0; n < nsteps; ++n) {
        const double ta = t0 + n * dt, tb = t0 + (n + 1) * dt;
        long budget = 1 << 16;
        a2inv[n] = drift_integral(c, ta, tb, gl_inv_a2(c, ta, tb), 0, budget) / dt;
        if (!isfinite(a2inv[n])) return VLASOV_ERR_NONFINITE;
    }
    if (a != nullptr)
        for (int k = 0; k <= nsteps; ++k) {
            a[k] = scale_factor(c, t0 + k * dt);
            if (!isfinite(a[k])) return VLASOV_ERR_NONFINITE;
        }
    return VLASOV_OK;
}

}  // extern "C"
