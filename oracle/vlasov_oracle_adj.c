/*
 * FP64 CPU oracle of the sweep derivatives -- TEST INFRASTRUCTURE ONLY.
 *
 * The SL-MPP5 update of a line is piecewise linear in the cell values: every
 * minimum, maximum, median and minmod of the Suresh-Huynh bounds and the
 * positivity clamp selects one of its arguments, and every argument is a
 * linear form of the five stencil values.  With the selections frozen at the
 * forward input, the sweep is the linear map f' = J f, and it depends on the
 * fractional shift nu smoothly (through the semi-Lagrangian weights and the
 * factor nu of the flux).  This file builds, for one line, the dense matrix J
 * and the column df'/dnu by evaluating the forward formulas of
 * vlasov_oracle.c on dual numbers (value, gradient with respect to the five
 * stencil values, derivative with respect to the fraction).  Tangents are
 * J v + (df'/dnu) dnu; adjoints are J^T lambda and lambda . df'/dnu.  The
 * fraction enters through the weights, the factor mu of the flux and the
 * alpha(mu) of the bounds' upper limit.
 *
 * Selection rule at ties (equal values, where the derivative is not unique):
 * min and max keep their first argument, the median is max(min(x,y),
 * min(max(x,y),z)) built from those, minmod returns 0 unless all four
 * arguments are strictly of one sign.
 *
 * Parity status: pinned in the CPU test-suite by J f = f' (the frozen map
 * reproduces the forward result), by central finite differences of the
 * forward oracle in f and in the shift, and by the chain through the 6D
 * operators and the Strang step.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "vlasov_oracle.h"

typedef struct {
    double v;       /* value */
    double g[5];    /* d/d(f_{j-2} .. f_{j+2}) in the upwind frame */
    double dmu;     /* d/d(mu) */
} dual;

static dual dconst(double v)
{
    dual r;
    memset(&r, 0, sizeof(r));
    r.v = v;
    return r;
}
static dual dvar(double v, int k)
{
    dual r = dconst(v);
    r.g[k] = 1.0;
    return r;
}
static dual dlin(double p, dual x, double q, dual y)  /* p x + q y */
{
    dual r;
    r.v = p * x.v + q * y.v;
    for (int k = 0; k < 5; ++k) r.g[k] = p * x.g[k] + q * y.g[k];
    r.dmu = p * x.dmu + q * y.dmu;
    return r;
}
static dual dadd(dual x, dual y) { return dlin(1.0, x, 1.0, y); }
static dual dsub(dual x, dual y) { return dlin(1.0, x, -1.0, y); }
static dual dscale(double p, dual x) { return dlin(p, x, 0.0, x); }
/* Selection margins.  Every comparison of two values x, y records the gap
 * |x - y| / max(|x|, |y|, S), S the largest |value| of the interface's
 * stencil; the smallest gap since the last reset (per thread) tells how
 * close the interface is to a selection that another rounding of the same
 * arithmetic (FP32 on the device) could take the other way.  A tie is gap 0
 * unless both values are exact in any rounding: constants, stencil values,
 * or combinations of stencil values that are all zero (tl_x holds the
 * stencil while margins are taken; NULL otherwise, and then nothing is
 * recorded). */
static _Thread_local double tl_gap = INFINITY;
static _Thread_local double tl_scale = 0.0;
static _Thread_local const double* tl_x = NULL;
static int exact_in_any_rounding(dual z)
{
    int nz = 0, unit = 0;
    double contrib = 0.0;
    for (int k = 0; k < 5; ++k) {
        if (z.g[k] != 0.0) {
            ++nz;
            unit = z.g[k] == 1.0;
            contrib += fabs(z.g[k] * tl_x[k]);
        }
    }
    if (nz == 0) return 1;
    if (nz == 1 && unit) return 1;
    return contrib == 0.0;
}
static void note_gap(dual x, dual y)
{
    if (tl_x == NULL) return;
    if (x.v == y.v) {
        if (!(exact_in_any_rounding(x) && exact_in_any_rounding(y))) tl_gap = 0.0;
        return;
    }
    double m = fabs(x.v) > fabs(y.v) ? fabs(x.v) : fabs(y.v);
    if (tl_scale > m) m = tl_scale;
    const double g = fabs(x.v - y.v) / m;
    if (g < tl_gap) tl_gap = g;
}
static dual dmin2(dual x, dual y) { note_gap(x, y); return x.v <= y.v ? x : y; }
static dual dmax2(dual x, dual y) { note_gap(x, y); return x.v >= y.v ? x : y; }
static dual dmin3(dual x, dual y, dual z) { return dmin2(dmin2(x, y), z); }
static dual dmax3(dual x, dual y, dual z) { return dmax2(dmax2(x, y), z); }
static dual dmed3(dual x, dual y, dual z) { return dmax2(dmin2(x, y), dmin2(dmax2(x, y), z)); }
static dual dminmod4(dual w, dual x, dual y, dual z)
{
    const dual zero = dconst(0.0);
    note_gap(w, zero);
    note_gap(x, zero);
    note_gap(y, zero);
    note_gap(z, zero);
    if (w.v > 0 && x.v > 0 && y.v > 0 && z.v > 0) return dmin2(dmin2(w, x), dmin2(y, z));
    if (w.v < 0 && x.v < 0 && y.v < 0 && z.v < 0) return dmax2(dmax2(w, x), dmax2(y, z));
    return dconst(0.0);
}
/* product of a function of mu alone (x: only value and dmu) with a dual */
static dual dmul_mu(dual m, dual y)
{
    dual r;
    r.v = m.v * y.v;
    for (int k = 0; k < 5; ++k) r.g[k] = m.v * y.g[k];
    r.dmu = m.dmu * y.v + m.v * y.dmu;
    return r;
}

/* The interface-value weights of vlasov_oracle.c as functions of a dual mu. */
static void dweights(double mu, dual w[5])
{
    dual m = dconst(mu);
    m.dmu = 1.0;
    dual one = dconst(1.0), m2 = dmul_mu(m, m);
    /* products of functions of mu only: dmul_mu works for them too */
#define P(x, y) dmul_mu((x), (y))
    dual t1 = dsub(m2, one);                                   /* mu^2 - 1 */
    dual t4 = dsub(m2, dconst(4.0));                           /* mu^2 - 4 */
    dual mp1 = dadd(m, one), mp2 = dadd(m, dconst(2.0));
    dual mm1 = dsub(m, one), mm2 = dsub(m, dconst(2.0)), mm3 = dsub(m, dconst(3.0));
    w[0] = dscale(1.0 / 120.0, P(t1, t4));
    w[1] = dscale(-1.0 / 120.0, P(P(t1, mp2), dsub(dscale(4.0, m), dconst(13.0))));
    w[2] = dscale(1.0 / 120.0,
                  P(P(mp1, mp2), dadd(dsub(dscale(6.0, m2), dscale(33.0, m)), dconst(47.0))));
    w[3] = dscale(-1.0 / 120.0, P(P(P(mm1, mm2), mm3), dadd(dscale(4.0, m), dconst(9.0))));
    w[4] = dscale(1.0 / 120.0, P(P(P(mp1, mm1), mm2), mm3));
#undef P
}

/* Linearised flux magnitude through an interface in its upwind frame:
 * stencil values x[0..4] = f_{j-2..j+2} (a..e), fraction mu > 0.  Returns the
 * dual of the flux magnitude.  Mirrors vor_interface_flux / vor_mp5_limit. */
static dual dflux(const double x[5], double mu, int limiter)
{
    dual a = dvar(x[0], 0), b = dvar(x[1], 1), c = dvar(x[2], 2), d = dvar(x[3], 3),
         e = dvar(x[4], 4);
    dual w[5];
    dweights(mu, w);
    dual st[5] = {a, b, c, d, e};
    dual fhat = dconst(0.0);
    for (int k = 0; k < 5; ++k) fhat = dadd(fhat, dmul_mu(w[k], st[k]));
    dual lim = fhat;
    if (limiter) {
        /* alpha(mu) of vor_mp_alpha with its derivative -1/mu^2 (0 where capped) */
        dual alpha = dconst(vor_mp_alpha(mu));
        if (mu * (VOR_ALPHA_CAP + 1.0) > 1.0) alpha.dmu = -1.0 / (mu * mu);
        dual Dm = dadd(dsub(a, dscale(2.0, b)), c);
        dual D0 = dadd(dsub(b, dscale(2.0, c)), d);
        dual Dp = dadd(dsub(c, dscale(2.0, d)), e);
        dual dM4p = dminmod4(dsub(dscale(4.0, D0), Dp), dsub(dscale(4.0, Dp), D0), D0, Dp);
        dual dM4m = dminmod4(dsub(dscale(4.0, D0), Dm), dsub(dscale(4.0, Dm), D0), D0, Dm);
        dual fUL = dadd(c, dmul_mu(alpha, dsub(c, b)));
        dual fAV = dscale(0.5, dadd(c, d));
        dual fMD = dsub(fAV, dscale(0.5, dM4p));
        dual fLC = dadd(dadd(c, dscale(0.5, dsub(c, b))), dscale(4.0 / 3.0, dM4m));
        dual fmin = dmax2(dmin3(c, d, fMD), dmin3(c, fUL, fLC));
        dual fmax = dmin2(dmax3(c, d, fMD), dmax3(c, fUL, fLC));
        lim = dmed3(fhat, fmin, fmax);
    }
    dual mud = dconst(mu);
    mud.dmu = 1.0;
    return dmed3(dmul_mu(mud, lim), dconst(0.0), c);
}

static long wrap_or_drop(long j, long M, int periodic)
{
    if (periodic) {
        long r = j % M;
        return r < 0 ? r + M : r;
    }
    return (j >= 0 && j < M) ? j : -1;
}

/* Frozen Jacobian of one line sweep: J (M x M, row-major, J[i*M + j] =
 * d out_i / d f_j) and dnu[i] = d out_i / d nu, at the forward input f and
 * shift s.  With limiter = 0 the bounds are skipped (unlimited scheme). */
void vor_sweep_line_jacobian(const double* f, long M, double s, int periodic, int limiter,
                             double* J, double* dnu)
{
    long N;
    double nu;
    vor_split_shift(s, &N, &nu);
    memset(J, 0, sizeof(double) * M * M);
    memset(dnu, 0, sizeof(double) * M);
    const double mu = fabs(nu);
    /* The upwind side follows the sign of nu; at a whole-cell shift (nu = 0)
     * the flux vanishes and its derivative is the one-sided limit from the
     * side of s's sign, i.e. for a growing |s| (the flux is mu times the
     * limited value, and a tie between that product and 0 in the clamp keeps
     * the product). */
    const int neg = nu < 0.0 || (nu == 0.0 && s < 0.0);
    for (long i = 0; i < M; ++i) {
        long j = i - N;
        long src = wrap_or_drop(j, M, periodic);
        if (src >= 0) J[i * M + src] += 1.0;
        /* out_i -= Phi_{j+1/2}; out_i += Phi_{j-1/2} */
        for (int side = 0; side < 2; ++side) {
            long jj = side == 0 ? j : j - 1;          /* interface jj + 1/2 */
            double sign = side == 0 ? -1.0 : 1.0;
            long cols[5];
            double x[5];
            for (int k = 0; k < 5; ++k) {
                /* upwind frame: f_{jj-2..jj+2} for nu > 0, f_{jj+3..jj-1} for nu < 0 */
                long idx = neg ? jj + 3 - k : jj - 2 + k;
                cols[k] = wrap_or_drop(idx, M, periodic);
                x[k] = cols[k] >= 0 ? f[cols[k]] : 0.0;
            }
            dual phi = dflux(x, mu, limiter);
            /* physical flux = +phi (nu > 0) or -phi (nu < 0); d mu / d nu = +1 or -1 */
            double fs = neg ? -1.0 : 1.0;
            for (int k = 0; k < 5; ++k)
                if (cols[k] >= 0) J[i * M + cols[k]] += sign * fs * phi.g[k];
            dnu[i] += sign * fs * phi.dmu * fs;
        }
    }
}

/* Selection margin of every input cell of one line sweep: margin[r] is the
 * smallest gap (see note_gap) of the limiter and clamp of the interfaces
 * whose stencils read cell r -- the interfaces that make column r of the
 * frozen Jacobian, so the adjoint lam_in[r] = sum_i J[i][r] lam[i] depends
 * on no other selection (+inf where none reads it). */
void vor_sweep_line_margin(const double* f, long M, double s, int periodic, double* margin)
{
    long N;
    double nu;
    vor_split_shift(s, &N, &nu);
    const double mu = fabs(nu);
    const int neg = nu < 0.0 || (nu == 0.0 && s < 0.0);
    for (long i = 0; i < M; ++i) margin[i] = INFINITY;
    if (nu == 0.0) return;
    for (long i = 0; i < M; ++i) {
        long jj = i - N;                          /* interface jj + 1/2 */
        double x[5], S = 0.0;
        long cols[5];
        for (int k = 0; k < 5; ++k) {
            long idx = neg ? jj + 3 - k : jj - 2 + k;
            cols[k] = wrap_or_drop(idx, M, periodic);
            x[k] = cols[k] >= 0 ? f[cols[k]] : 0.0;
            if (fabs(x[k]) > S) S = fabs(x[k]);
        }
        tl_gap = INFINITY;
        tl_scale = S;
        tl_x = x;
        (void)dflux(x, mu, 1);
        tl_x = NULL;
        for (int k = 0; k < 5; ++k)
            if (cols[k] >= 0 && tl_gap < margin[cols[k]]) margin[cols[k]] = tl_gap;
    }
    /* the interface below output 0 (jj = -N-1) also enters the update */
    {
        long jj = -N - 1;
        double x[5], S = 0.0;
        long cols[5];
        for (int k = 0; k < 5; ++k) {
            long idx = neg ? jj + 3 - k : jj - 2 + k;
            cols[k] = wrap_or_drop(idx, M, periodic);
            x[k] = cols[k] >= 0 ? f[cols[k]] : 0.0;
            if (fabs(x[k]) > S) S = fabs(x[k]);
        }
        tl_gap = INFINITY;
        tl_scale = S;
        tl_x = x;
        (void)dflux(x, mu, 1);
        tl_x = NULL;
        for (int k = 0; k < 5; ++k)
            if (cols[k] >= 0 && tl_gap < margin[cols[k]]) margin[cols[k]] = tl_gap;
    }
}

/* Tangent and adjoint of a line sweep through its frozen Jacobian. */
void vor_sweep_line_tangent(const double* f, long M, double s, int periodic, const double* v,
                            double nu_dot, double* out_dot)
{
    double* J = (double*)malloc(sizeof(double) * M * M);
    double* dn = (double*)malloc(sizeof(double) * M);
    vor_sweep_line_jacobian(f, M, s, periodic, 1, J, dn);
    for (long i = 0; i < M; ++i) {
        double acc = dn[i] * nu_dot;
        for (long j = 0; j < M; ++j) acc += J[i * M + j] * v[j];
        out_dot[i] = acc;
    }
    free(J);
    free(dn);
}

void vor_sweep_line_adjoint(const double* f, long M, double s, int periodic, const double* lam,
                            double* lam_in, double* lam_nu)
{
    double* J = (double*)malloc(sizeof(double) * M * M);
    double* dn = (double*)malloc(sizeof(double) * M);
    vor_sweep_line_jacobian(f, M, s, periodic, 1, J, dn);
    double ln = 0.0;
    for (long j = 0; j < M; ++j) {
        double acc = 0.0;
        for (long i = 0; i < M; ++i) acc += J[i * M + j] * lam[i];
        lam_in[j] = acc;
    }
    for (long i = 0; i < M; ++i) ln += dn[i] * lam[i];
    *lam_nu = ln;
    free(J);
    free(dn);
}

/* ------------------------------------------------------------------------ */
/* 6D adjoints.  Line bookkeeping as in vor_advect_position/velocity.       */
/* ------------------------------------------------------------------------ */

/* lam_in = J^T lam_out for the position sweep along a (periodic). */
int vor_advect_position_adj(const vor_grid* g, int a, const double* fin, const double* lam_out,
                            double* lam_in, double dt_over_a2)
{
    int rc = vor_check_grid(g);
    if (rc) return rc;
    long n[3] = {g->n[0], g->n[1], g->n[2]};
    long nu[3] = {g->nu[0], g->nu[1], g->nu[2]};
    long Nu = nu[0] * nu[1] * nu[2];
    long stride_sp[3] = {n[1] * n[2] * Nu, n[2] * Nu, Nu};
    int b0 = (a == 0) ? 1 : 0;
    int b1 = (a == 2) ? 1 : 2;
    long nplanes = n[b0] * n[b1];
    #pragma omp parallel for schedule(static)
    for (long p = 0; p < nplanes; ++p) {
        long i0 = p / n[b1], i1 = p % n[b1], M = n[a];
        double *line = malloc(sizeof(double) * M), *lam = malloc(sizeof(double) * M),
               *res = malloc(sizeof(double) * M);
        for (long ju = 0; ju < Nu; ++ju) {
            long jv[3] = {ju / (nu[1] * nu[2]), (ju / nu[2]) % nu[1], ju % nu[2]};
            double s = vor_position_shift(g, a, jv[a], dt_over_a2), lnu;
            long base = i0 * stride_sp[b0] + i1 * stride_sp[b1] + ju;
            for (long i = 0; i < M; ++i) {
                line[i] = fin[base + i * stride_sp[a]];
                lam[i] = lam_out[base + i * stride_sp[a]];
            }
            vor_sweep_line_adjoint(line, M, s, 1, lam, res, &lnu);
            for (long i = 0; i < M; ++i) lam_in[base + i * stride_sp[a]] = res[i];
        }
        free(line);
        free(lam);
        free(res);
    }
    return 0;
}

/* lam_in = J^T lam_out for the velocity sweep along a; lam_g[a][cell] +=
 * sum over the cell's lines of lam . d out / d nu times dt/du. */
int vor_advect_velocity_adj(const vor_grid* g, int a, int vbc, const double* fin,
                            const float* gfield, double dt, const double* lam_out,
                            double* lam_in, double* lam_g)
{
    int rc = vor_check_grid(g);
    if (rc) return rc;
    long nu[3] = {g->nu[0], g->nu[1], g->nu[2]};
    long Nx = (long)g->n[0] * g->n[1] * g->n[2], Nu = nu[0] * nu[1] * nu[2];
    long stride_u[3] = {nu[1] * nu[2], nu[2], 1};
    int b0 = (a == 0) ? 1 : 0;
    int b1 = (a == 2) ? 1 : 2;
    double du = 2.0 * g->umax[a] / g->nu[a];
    #pragma omp parallel for schedule(static)
    for (long c = 0; c < Nx; ++c) {
        long M = nu[a];
        double *line = malloc(sizeof(double) * M), *lam = malloc(sizeof(double) * M),
               *res = malloc(sizeof(double) * M);
        double s = vor_velocity_shift(g, a, gfield[(long)a * Nx + c], dt), tot = 0.0, lnu;
        for (long j0 = 0; j0 < nu[b0]; ++j0) {
            for (long j1 = 0; j1 < nu[b1]; ++j1) {
                long base = c * Nu + j0 * stride_u[b0] + j1 * stride_u[b1];
                for (long i = 0; i < M; ++i) {
                    line[i] = fin[base + i * stride_u[a]];
                    lam[i] = lam_out[base + i * stride_u[a]];
                }
                vor_sweep_line_adjoint(line, M, s, vbc == 1, lam, res, &lnu);
                for (long i = 0; i < M; ++i) lam_in[base + i * stride_u[a]] = res[i];
                tot += lnu;
            }
        }
        if (lam_g) lam_g[(long)a * Nx + c] += tot * (dt / du);
        free(line);
        free(lam);
        free(res);
    }
    return 0;
}

/* Selection margins of a position / velocity sweep: margin has the layout of
 * f and holds, at every cell, the margin vor_sweep_line_margin gives it in
 * its line. */
int vor_advect_position_margin(const vor_grid* g, int a, const double* fin, double* margin,
                               double dt_over_a2)
{
    int rc = vor_check_grid(g);
    if (rc) return rc;
    long n[3] = {g->n[0], g->n[1], g->n[2]};
    long nu[3] = {g->nu[0], g->nu[1], g->nu[2]};
    long Nu = nu[0] * nu[1] * nu[2];
    long stride_sp[3] = {n[1] * n[2] * Nu, n[2] * Nu, Nu};
    int b0 = (a == 0) ? 1 : 0;
    int b1 = (a == 2) ? 1 : 2;
    long nplanes = n[b0] * n[b1];
    #pragma omp parallel for schedule(static)
    for (long p = 0; p < nplanes; ++p) {
        long i0 = p / n[b1], i1 = p % n[b1], M = n[a];
        double *line = malloc(sizeof(double) * M), *mg = malloc(sizeof(double) * M);
        for (long ju = 0; ju < Nu; ++ju) {
            long jv[3] = {ju / (nu[1] * nu[2]), (ju / nu[2]) % nu[1], ju % nu[2]};
            double s = vor_position_shift(g, a, jv[a], dt_over_a2);
            long base = i0 * stride_sp[b0] + i1 * stride_sp[b1] + ju;
            for (long i = 0; i < M; ++i) line[i] = fin[base + i * stride_sp[a]];
            vor_sweep_line_margin(line, M, s, 1, mg);
            for (long i = 0; i < M; ++i) margin[base + i * stride_sp[a]] = mg[i];
        }
        free(line);
        free(mg);
    }
    return 0;
}

int vor_advect_velocity_margin(const vor_grid* g, int a, int vbc, const double* fin,
                               const float* gfield, double dt, double* margin)
{
    int rc = vor_check_grid(g);
    if (rc) return rc;
    long nu[3] = {g->nu[0], g->nu[1], g->nu[2]};
    long Nx = (long)g->n[0] * g->n[1] * g->n[2], Nu = nu[0] * nu[1] * nu[2];
    long stride_u[3] = {nu[1] * nu[2], nu[2], 1};
    int b0 = (a == 0) ? 1 : 0;
    int b1 = (a == 2) ? 1 : 2;
    #pragma omp parallel for schedule(static)
    for (long c = 0; c < Nx; ++c) {
        long M = nu[a];
        double *line = malloc(sizeof(double) * M), *mg = malloc(sizeof(double) * M);
        double s = vor_velocity_shift(g, a, gfield[(long)a * Nx + c], dt);
        for (long j0 = 0; j0 < nu[b0]; ++j0) {
            for (long j1 = 0; j1 < nu[b1]; ++j1) {
                long base = c * Nu + j0 * stride_u[b0] + j1 * stride_u[b1];
                for (long i = 0; i < M; ++i) line[i] = fin[base + i * stride_u[a]];
                vor_sweep_line_margin(line, M, s, vbc == 1, mg);
                for (long i = 0; i < M; ++i) margin[base + i * stride_u[a]] = mg[i];
            }
        }
        free(line);
        free(mg);
    }
    return 0;
}

/* Tangent of the velocity sweep: out_dot = J v + d out/d nu * (g_dot dt/du). */
int vor_advect_velocity_tan(const vor_grid* g, int a, int vbc, const double* fin,
                            const float* gfield, const double* g_dot, double dt, const double* v,
                            double* out_dot)
{
    int rc = vor_check_grid(g);
    if (rc) return rc;
    long nu[3] = {g->nu[0], g->nu[1], g->nu[2]};
    long Nx = (long)g->n[0] * g->n[1] * g->n[2], Nu = nu[0] * nu[1] * nu[2];
    long stride_u[3] = {nu[1] * nu[2], nu[2], 1};
    int b0 = (a == 0) ? 1 : 0;
    int b1 = (a == 2) ? 1 : 2;
    double du = 2.0 * g->umax[a] / g->nu[a];
    #pragma omp parallel for schedule(static)
    for (long c = 0; c < Nx; ++c) {
        long M = nu[a];
        double *line = malloc(sizeof(double) * M), *vl = malloc(sizeof(double) * M),
               *res = malloc(sizeof(double) * M);
        double s = vor_velocity_shift(g, a, gfield[(long)a * Nx + c], dt);
        double nu_dot = g_dot ? g_dot[(long)a * Nx + c] * (dt / du) : 0.0;
        for (long j0 = 0; j0 < nu[b0]; ++j0) {
            for (long j1 = 0; j1 < nu[b1]; ++j1) {
                long base = c * Nu + j0 * stride_u[b0] + j1 * stride_u[b1];
                for (long i = 0; i < M; ++i) {
                    line[i] = fin[base + i * stride_u[a]];
                    vl[i] = v[base + i * stride_u[a]];
                }
                vor_sweep_line_tangent(line, M, s, vbc == 1, vl, nu_dot, res);
                for (long i = 0; i < M; ++i) out_dot[base + i * stride_u[a]] = res[i];
            }
        }
        free(line);
        free(vl);
        free(res);
    }
    return 0;
}

/* Tangent of the position sweep (no shift derivative: the drift shift does
 * not depend on the field). */
int vor_advect_position_tan(const vor_grid* g, int a, const double* fin, const double* v,
                            double* out_dot, double dt_over_a2)
{
    int rc = vor_check_grid(g);
    if (rc) return rc;
    long n[3] = {g->n[0], g->n[1], g->n[2]};
    long nu[3] = {g->nu[0], g->nu[1], g->nu[2]};
    long Nu = nu[0] * nu[1] * nu[2];
    long stride_sp[3] = {n[1] * n[2] * Nu, n[2] * Nu, Nu};
    int b0 = (a == 0) ? 1 : 0;
    int b1 = (a == 2) ? 1 : 2;
    long nplanes = n[b0] * n[b1];
    #pragma omp parallel for schedule(static)
    for (long p = 0; p < nplanes; ++p) {
        long i0 = p / n[b1], i1 = p % n[b1], M = n[a];
        double *line = malloc(sizeof(double) * M), *vl = malloc(sizeof(double) * M),
               *res = malloc(sizeof(double) * M);
        for (long ju = 0; ju < Nu; ++ju) {
            long jv[3] = {ju / (nu[1] * nu[2]), (ju / nu[2]) % nu[1], ju % nu[2]};
            double s = vor_position_shift(g, a, jv[a], dt_over_a2);
            long base = i0 * stride_sp[b0] + i1 * stride_sp[b1] + ju;
            for (long i = 0; i < M; ++i) {
                line[i] = fin[base + i * stride_sp[a]];
                vl[i] = v[base + i * stride_sp[a]];
            }
            vor_sweep_line_tangent(line, M, s, 1, vl, 0.0, res);
            for (long i = 0; i < M; ++i) out_dot[base + i * stride_sp[a]] = res[i];
        }
        free(line);
        free(vl);
        free(res);
    }
    return 0;
}

/* Adjoint of one Strang step (Eq. 5): forward stages are recomputed from
 * fin, then the sweeps are transposed in reverse order.  lam_g_n and
 * lam_g_np1 ([3][cells]) are accumulated. */
int vor_step_adj(const vor_grid* g, int vbc, const double* fin, const float* g_n,
                 const float* g_np1, double dt, double a2inv, const double* lam_out,
                 double* lam_in, double* lam_g_n, double* lam_g_np1)
{
    int rc = vor_check_grid(g);
    if (rc) return rc;
    long total = (long)g->n[0] * g->n[1] * g->n[2] * g->nu[0] * g->nu[1] * g->nu[2];
    double* st[9];
    for (int k = 0; k < 9; ++k) st[k] = (double*)malloc(sizeof(double) * total);
    double* lam = (double*)malloc(sizeof(double) * total);
    double* tmp = (double*)malloc(sizeof(double) * total);
    double h = 0.5 * dt, dta = dt * a2inv;
    /* st[k] = input of sweep k */
    memcpy(st[0], fin, sizeof(double) * total);
    rc |= vor_advect_velocity(g, 0, vbc, st[0], st[1], g_n, h, NULL);
    rc |= vor_advect_velocity(g, 1, vbc, st[1], st[2], g_n, h, NULL);
    rc |= vor_advect_velocity(g, 2, vbc, st[2], st[3], g_n, h, NULL);
    rc |= vor_advect_position(g, 2, st[3], st[4], dta);
    rc |= vor_advect_position(g, 1, st[4], st[5], dta);
    rc |= vor_advect_position(g, 0, st[5], st[6], dta);
    rc |= vor_advect_velocity(g, 0, vbc, st[6], st[7], g_np1, h, NULL);
    rc |= vor_advect_velocity(g, 1, vbc, st[7], st[8], g_np1, h, NULL);
    memcpy(lam, lam_out, sizeof(double) * total);
    rc |= vor_advect_velocity_adj(g, 2, vbc, st[8], g_np1, h, lam, tmp, lam_g_np1);
    rc |= vor_advect_velocity_adj(g, 1, vbc, st[7], g_np1, h, tmp, lam, lam_g_np1);
    rc |= vor_advect_velocity_adj(g, 0, vbc, st[6], g_np1, h, lam, tmp, lam_g_np1);
    rc |= vor_advect_position_adj(g, 0, st[5], tmp, lam, dta);
    rc |= vor_advect_position_adj(g, 1, st[4], lam, tmp, dta);
    rc |= vor_advect_position_adj(g, 2, st[3], tmp, lam, dta);
    rc |= vor_advect_velocity_adj(g, 2, vbc, st[2], g_n, h, lam, tmp, lam_g_n);
    rc |= vor_advect_velocity_adj(g, 1, vbc, st[1], g_n, h, tmp, lam, lam_g_n);
    rc |= vor_advect_velocity_adj(g, 0, vbc, st[0], g_n, h, lam, lam_in, lam_g_n);
    for (int k = 0; k < 9; ++k) free(st[k]);
    free(lam);
    free(tmp);
    return rc;
}

/* Adjoint of the moments: lam_f += du^3 lam_rho + du^3 sum_a lam_umean[a]
 * (u_a - umean_a) / rho, at the forward input f (cells with rho = 0 get only
 * the density term).  lam_umean may be NULL. */
int vor_moments_adj(const vor_grid* g, const double* f, const double* lam_rho,
                    const double* lam_umean, double* lam_f)
{
    int rc = vor_check_grid(g);
    if (rc) return rc;
    long Nx = (long)g->n[0] * g->n[1] * g->n[2];
    long Nu = (long)g->nu[0] * g->nu[1] * g->nu[2];
    double* rho = (double*)malloc(sizeof(double) * Nx);
    double* um = (double*)malloc(sizeof(double) * 3 * Nx);
    vor_moments(g, f, rho, um, NULL);
    double du[3], du3 = 1.0;
    for (int a = 0; a < 3; ++a) {
        du[a] = 2.0 * g->umax[a] / g->nu[a];
        du3 *= du[a];
    }
    #pragma omp parallel for schedule(static)
    for (long c = 0; c < Nx; ++c) {
        for (long ju = 0; ju < Nu; ++ju) {
            long jv[3] = {ju / ((long)g->nu[1] * g->nu[2]), (ju / g->nu[2]) % g->nu[1],
                          ju % g->nu[2]};
            double t = du3 * lam_rho[c];
            if (lam_umean && rho[c] != 0.0) {
                for (int a = 0; a < 3; ++a) {
                    double u = -g->umax[a] + (jv[a] + 0.5) * du[a];
                    t += du3 * lam_umean[(long)a * Nx + c] * (u - um[(long)a * Nx + c]) / rho[c];
                }
            }
            lam_f[c * Nu + ju] += t;
        }
    }
    free(rho);
    free(um);
    return 0;
}
