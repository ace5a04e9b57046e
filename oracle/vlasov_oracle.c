/*
 * FP64 CPU oracle for the split SL-MPP5 advection of the neutrino
 * distribution function f(x,u) on a 6D phase-space grid.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link,
 * load or call this file: only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the HIP
 * library: it has its own grid struct, its own shift formulas and its own
 * scheme arithmetic, all written as plainly as the definitions allow.
 *
 * What it computes (Yoshikawa, Tanaka & Yoshida, SC'21):
 *   - the Vlasov equation, Eq. (1), split into three position advections
 *     (Eq. 3, speed u_i / a^2) and three velocity advections (Eq. 4, speed
 *     g_i = -d(phi)/dx_i), section 5.1.1;
 *   - one full step composed as in Eq. (5): half kicks ux,uy,uz with the field
 *     at t^n, drifts z,y,x over dt, half kicks ux,uy,uz with the field at
 *     t^{n+1} (operators act right to left);
 *   - each 1D operator is SL-MPP5 (section 5.2): a fifth-order finite-volume
 *     update whose interface flux is the conservative semi-Lagrangian flux
 *     (the exact integral of the reconstruction over the upwind departure
 *     interval), limited by the Suresh-Huynh monotonicity-preserving bounds
 *     and by a positivity clamp, evaluated once per step (single stage);
 *   - velocity moments per spatial cell (section 5.1.3): density, mean
 *     velocity and the velocity dispersion tensor.
 * The paper prints no formula for the scheme; the readings taken here (the
 * shift split and the shift-dependent alpha of the bounds, epsilon, the
 * positivity form, the velocity boundary, the time level of the field in the
 * second half kick) are listed with the build's design notes.
 *
 * Layout: f[ix][iy][iz][jx][jy][jz], jz fastest (the per-cell velocity block
 * of List 1 without its header).  Cell centres x_i = (i+1/2) dx and
 * u_j = -umax + (j+1/2) du, du = 2 umax / nu (domain of section 5.1.3).
 *
 * Parity status: the SL weights, the limiter, the line sweep, the composed
 * step and the moments are pinned by closed forms and invariants in the
 * CPU test-suite, among them the property the paper names for the scheme:
 * repeated sweeps of monotone data create no new extrema at any shift.  The
 * form of alpha, the positivity clamp, the vacuum velocity boundary and the
 * field time level are readings of a silent paper: parity against the paper
 * itself is unpinned for those choices.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "vlasov_oracle.h"

/* ------------------------------------------------------------------------ */
/* Elementary selections.                                                    */
/* ------------------------------------------------------------------------ */

static double dmin2(double a, double b) { return a <= b ? a : b; }
static double dmax2(double a, double b) { return a >= b ? a : b; }
static double dmin3(double a, double b, double c) { return dmin2(dmin2(a, b), c); }
static double dmax3(double a, double b, double c) { return dmax2(dmax2(a, b), c); }

/* median of three values */
double vor_median3(double x, double y, double z)
{
    return dmax2(dmin2(x, y), dmin2(dmax2(x, y), z));
}

/* minmod of four arguments: the argument of least magnitude when all four
 * are strictly of one sign, zero otherwise (Suresh & Huynh 1997). */
double vor_minmod4(double w, double x, double y, double z)
{
    if (w > 0 && x > 0 && y > 0 && z > 0) return dmin2(dmin2(w, x), dmin2(y, z));
    if (w < 0 && x < 0 && y < 0 && z < 0) return dmax2(dmax2(w, x), dmax2(y, z));
    return 0.0;
}

/* ------------------------------------------------------------------------ */
/* Conservative semi-Lagrangian interface value (section 5.2).               */
/*                                                                           */
/* For a rightward shift by a fraction mu of a cell, the mass crossing the   */
/* interface j+1/2 is the integral, over the departure interval              */
/* [x_{j+1/2} - mu dx, x_{j+1/2}], of the quartic that reproduces the cell   */
/* averages f_{j-2..j+2}.  That flux equals sum_k c_k(mu) f_{j+k} with       */
/*   c_{-2} =  mu (mu^2-1)(mu^2-4) / 120                                     */
/*   c_{-1} = -mu (mu^2-1)(mu+2)(4mu-13) / 120                               */
/*   c_{0}  =  mu (mu+1)(mu+2)(6mu^2-33mu+47) / 120                          */
/*   c_{+1} = -mu (mu-1)(mu-2)(mu-3)(4mu+9) / 120                            */
/*   c_{+2} =  mu (mu+1)(mu-1)(mu-2)(mu-3) / 120                             */
/* The interface value is the mean over the departure interval, i.e. the    */
/* flux divided by mu; w_k = c_k / mu are the quartics below, which stay     */
/* finite at mu = 0 where they reduce to the fifth-order upwind point value. */
/* ------------------------------------------------------------------------ */
void vor_sl5_weights(double mu, double w[5])
{
    w[0] = (mu * mu - 1.0) * (mu * mu - 4.0) / 120.0;
    w[1] = -(mu * mu - 1.0) * (mu + 2.0) * (4.0 * mu - 13.0) / 120.0;
    w[2] = (mu + 1.0) * (mu + 2.0) * (6.0 * mu * mu - 33.0 * mu + 47.0) / 120.0;
    w[3] = -(mu - 1.0) * (mu - 2.0) * (mu - 3.0) * (4.0 * mu + 9.0) / 120.0;
    w[4] = (mu + 1.0) * (mu - 1.0) * (mu - 2.0) * (mu - 3.0) / 120.0;
}

/* ------------------------------------------------------------------------ */
/* Monotonicity-preserving bounds of Suresh & Huynh (1997), the "standard   */
/* MP preserving scheme" whose polynomial flux SL-MPP5 replaces (section     */
/* 5.2).  Stencil a..e = f_{j-2..j+2} seen from the upwind side of the       */
/* interface j+1/2.  epsilon = 0, so the limited value is the median of the  */
/* unlimited value and the two bounds; alpha scales the upper limit          */
/* f_UL = f_j + alpha (f_j - f_{j-1}).                                       */
/* ------------------------------------------------------------------------ */
double vor_mp5_limit(double fhat, double a, double b, double c, double d, double e, double alpha)
{
    double Dm = a - 2.0 * b + c;          /* curvature at j-1 */
    double D0 = b - 2.0 * c + d;          /* curvature at j   */
    double Dp = c - 2.0 * d + e;          /* curvature at j+1 */
    double dM4p = vor_minmod4(4.0 * D0 - Dp, 4.0 * Dp - D0, D0, Dp);   /* at j+1/2 */
    double dM4m = vor_minmod4(4.0 * D0 - Dm, 4.0 * Dm - D0, D0, Dm);   /* at j-1/2 */
    double fUL = c + alpha * (c - b);
    double fAV = 0.5 * (c + d);
    double fMD = fAV - 0.5 * dM4p;
    double fLC = c + 0.5 * (c - b) + (4.0 / 3.0) * dM4m;
    double fmin = dmax2(dmin3(c, d, fMD), dmin3(c, fUL, fLC));
    double fmax = dmin2(dmax3(c, d, fMD), dmax3(c, fUL, fLC));
    return vor_median3(fhat, fmin, fmax);
}

/* alpha for a single-stage update with Courant number mu (0 <= mu <= 1/2).
 * The new value of cell j is f_j - mu (fhat_{j+1/2} - fhat_{j-1/2}).  On
 * monotone data, with fhat_{j-1/2} between f_{j-1} and f_j and fhat_{j+1/2}
 * between f_j and f_j + alpha (f_j - f_{j-1}), it stays between f_{j-1} and
 * f_j as long as mu (1 + alpha) <= 1: the largest such alpha is (1-mu)/mu
 * (Suresh and Huynh's fixed alpha = 4 is this bound at mu = 0.2, the
 * Courant number their Runge-Kutta stages allow).  The split of the shift
 * keeps mu <= 1/2, so alpha >= 1.  Below mu = 1/(1 + 2^20) alpha stays at
 * 2^20: the bound remains finite at a whole-cell shift, and any smaller
 * alpha keeps the property. */
double vor_mp_alpha(double mu)
{
    const double cap = VOR_ALPHA_CAP;
    if (mu * (cap + 1.0) <= 1.0) return cap;
    return (1.0 - mu) / mu;
}

/* ------------------------------------------------------------------------ */
/* One line of M cells.                                                      */
/* ------------------------------------------------------------------------ */

/* Value of the line extended beyond [0, M): periodic wrap, or zero ghosts   */
/* (vacuum outside the velocity domain).                                     */
static double ext(const double* f, long M, long j, int periodic)
{
    if (periodic) {
        long r = j % M;
        if (r < 0) r += M;
        return f[r];
    }
    return (j >= 0 && j < M) ? f[j] : 0.0;
}

/* Split a shift s (in cells) into the nearest integer N (halves rounded    */
/* away from zero) and a fraction nu = s - N with |nu| <= 1/2: the integer   */
/* part is an exact translation and the fraction, at most half a cell either */
/* way, goes through the flux.  (Splitting at the floor instead leaves       */
/* fractions up to a whole cell, where the bounds of vor_mp5_limit cannot    */
/* keep the update monotone: the fixed 1/2 of f_LC exceeds (1-mu)/mu above   */
/* mu = 2/3.)                                                                */
void vor_split_shift(double s, long* N, double* nu)
{
    double n = round(s);
    *N = (long)n;
    *nu = s - n;
}

/* Numerical flux through the interface j+1/2 for a fractional shift nu.    */
/* limiter = 0 switches the MP bounds off (used only to measure the order of */
/* the unlimited scheme).                                                    */
double vor_interface_flux(const double* f, long M, long j, double nu, int periodic, int limiter)
{
    double a, b, c, d, e, mu, w[5], fhat, lim, phi;
    if (nu == 0.0) return 0.0;
    if (nu > 0.0) {                       /* upwind side is cell j */
        a = ext(f, M, j - 2, periodic);
        b = ext(f, M, j - 1, periodic);
        c = ext(f, M, j, periodic);
        d = ext(f, M, j + 1, periodic);
        e = ext(f, M, j + 2, periodic);
        mu = nu;
    } else {                              /* upwind side is cell j+1: mirror */
        a = ext(f, M, j + 3, periodic);
        b = ext(f, M, j + 2, periodic);
        c = ext(f, M, j + 1, periodic);
        d = ext(f, M, j, periodic);
        e = ext(f, M, j - 1, periodic);
        mu = -nu;
    }
    vor_sl5_weights(mu, w);
    fhat = w[0] * a + w[1] * b + w[2] * c + w[3] * d + w[4] * e;
    lim = limiter ? vor_mp5_limit(fhat, a, b, c, d, e, vor_mp_alpha(mu)) : fhat;
    /* positivity: the mass leaving the upwind cell lies between 0 and the
     * content of that cell */
    phi = vor_median3(mu * lim, 0.0, c);
    return nu > 0.0 ? phi : -phi;
}

/* Advance one line by the shift s: f'_i = f_{i-N} - (Phi_{i-N+1/2} -
 * Phi_{i-N-1/2}).  With zero ghosts, *outflow (if not NULL) receives the
 * content that left the line through its two faces: the cells shifted past
 * a face plus the fractional flux through it. */
void vor_sweep_line_opt(const double* f, double* out, long M, double s, int periodic,
                        int limiter, double* outflow)
{
    long N, i, j;
    double nu, sum;
    vor_split_shift(s, &N, &nu);
    for (i = 0; i < M; ++i) {
        j = i - N;
        out[i] = ext(f, M, j, periodic)
               - (vor_interface_flux(f, M, j, nu, periodic, limiter)
                  - vor_interface_flux(f, M, j - 1, nu, periodic, limiter));
    }
    if (outflow) {
        sum = 0.0;
        if (!periodic) {
            if (s >= 0.0) {               /* through the upper face */
                for (j = M - N; j < M; ++j) sum += ext(f, M, j, 0);
                sum += vor_interface_flux(f, M, M - N - 1, nu, 0, limiter);
            } else {                      /* through the lower face */
                for (j = 0; j < -N; ++j) sum += ext(f, M, j, 0);
                sum -= vor_interface_flux(f, M, -N - 1, nu, 0, limiter);
            }
        }
        *outflow = sum;
    }
}

void vor_sweep_line(const double* f, double* out, long M, double s, int periodic, double* outflow)
{
    vor_sweep_line_opt(f, out, M, s, periodic, 1, outflow);
}

/* ------------------------------------------------------------------------ */
/* 6D operators.                                                             */
/* ------------------------------------------------------------------------ */

static long ncell_x(const vor_grid* g) { return (long)g->n[0] * g->n[1] * g->n[2]; }
static long ncell_u(const vor_grid* g) { return (long)g->nu[0] * g->nu[1] * g->nu[2]; }

/* Shift of the position sweep along axis a for velocity index j (Eq. 3):
 * s = u_j * dt a^-2 / dx. */
double vor_position_shift(const vor_grid* g, int a, long j, double dt_over_a2)
{
    double dx = g->L[a] / g->n[a];
    double factor = dt_over_a2 / dx;
    double du = 2.0 * g->umax[a] / g->nu[a];
    double u = -g->umax[a] + (j + 0.5) * du;
    return u * factor;
}

/* Shift of the velocity sweep along axis a for a spatial cell whose field
 * component is ga (Eq. 4): s = g_a * dt / du. */
double vor_velocity_shift(const vor_grid* g, int a, float ga, double dt)
{
    double du = 2.0 * g->umax[a] / g->nu[a];
    double factor = dt / du;
    return (double)ga * factor;
}

int vor_check_grid(const vor_grid* g)
{
    int a;
    if (!g) return -1;
    for (a = 0; a < 3; ++a) {
        if (g->n[a] < 1 || g->nu[a] < 1) return -2;
        if (!(g->L[a] > 0) || !(g->umax[a] > 0)) return -2;
    }
    return 0;
}

/* Position sweep along axis a in {0,1,2} (periodic box). */
int vor_advect_position(const vor_grid* g, int a, const double* fin, double* fout,
                        double dt_over_a2)
{
    long n[3], nu[3], Nu, stride_sp[3], p;
    int rc = vor_check_grid(g);
    if (rc) return rc;
    if (a < 0 || a > 2) return -2;
    for (int k = 0; k < 3; ++k) { n[k] = g->n[k]; nu[k] = g->nu[k]; }
    Nu = ncell_u(g);
    /* stride between neighbouring spatial cells along each axis, in floats */
    stride_sp[2] = Nu;
    stride_sp[1] = n[2] * Nu;
    stride_sp[0] = n[1] * n[2] * Nu;
    /* the two spatial axes other than a */
    int b0 = (a == 0) ? 1 : 0;
    int b1 = (a == 2) ? 1 : 2;
    long nplanes = n[b0] * n[b1];
    #pragma omp parallel for schedule(static)
    for (p = 0; p < nplanes; ++p) {
        long i0 = p / n[b1], i1 = p % n[b1];
        long M = n[a];
        double* line = (double*)malloc(sizeof(double) * M);
        double* res = (double*)malloc(sizeof(double) * M);
        for (long ju = 0; ju < Nu; ++ju) {
            long jv[3];
            jv[0] = ju / (nu[1] * nu[2]);
            jv[1] = (ju / nu[2]) % nu[1];
            jv[2] = ju % nu[2];
            double s = vor_position_shift(g, a, jv[a], dt_over_a2);
            long base = i0 * stride_sp[b0] + i1 * stride_sp[b1] + ju;
            for (long i = 0; i < M; ++i) line[i] = fin[base + i * stride_sp[a]];
            vor_sweep_line(line, res, M, s, 1, NULL);
            for (long i = 0; i < M; ++i) fout[base + i * stride_sp[a]] = res[i];
        }
        free(line);
        free(res);
    }
    return 0;
}

/* Velocity sweep along axis a in {0,1,2} (ux,uy,uz).  gfield is FP32
 * [3][nx][ny][nz].  vbc = 0: vacuum outside [-umax, umax), the content that
 * leaves is added to outflow[cell] (density units, i.e. times du^3) when
 * outflow is not NULL; vbc = 1: periodic velocity axis. */
int vor_advect_velocity(const vor_grid* g, int a, int vbc, const double* fin, double* fout,
                        const float* gfield, double dt, double* outflow)
{
    long nu[3], Nx, Nu, c;
    int rc = vor_check_grid(g);
    if (rc) return rc;
    if (a < 0 || a > 2 || vbc < 0 || vbc > 1) return -2;
    for (int k = 0; k < 3; ++k) nu[k] = g->nu[k];
    Nx = ncell_x(g);
    Nu = ncell_u(g);
    double du3 = (2.0 * g->umax[0] / g->nu[0]) * (2.0 * g->umax[1] / g->nu[1])
               * (2.0 * g->umax[2] / g->nu[2]);
    long stride_u[3];
    stride_u[2] = 1;
    stride_u[1] = nu[2];
    stride_u[0] = nu[1] * nu[2];
    int b0 = (a == 0) ? 1 : 0;
    int b1 = (a == 2) ? 1 : 2;
    #pragma omp parallel for schedule(static)
    for (c = 0; c < Nx; ++c) {
        long M = nu[a];
        double* line = (double*)malloc(sizeof(double) * M);
        double* res = (double*)malloc(sizeof(double) * M);
        double s = vor_velocity_shift(g, a, gfield[(long)a * Nx + c], dt);
        double out_sum = 0.0;
        for (long j0 = 0; j0 < nu[b0]; ++j0) {
            for (long j1 = 0; j1 < nu[b1]; ++j1) {
                long base = c * Nu + j0 * stride_u[b0] + j1 * stride_u[b1];
                double ofl = 0.0;
                for (long i = 0; i < M; ++i) line[i] = fin[base + i * stride_u[a]];
                vor_sweep_line(line, res, M, s, vbc == 1, &ofl);
                for (long i = 0; i < M; ++i) fout[base + i * stride_u[a]] = res[i];
                out_sum += ofl;
            }
        }
        if (outflow) outflow[c] += out_sum * du3;
        free(line);
        free(res);
    }
    return 0;
}

/* One full step, Eq. (5): D_uz D_uy D_ux (dt/2, g_np1) D_x D_y D_z (dt)
 * D_uz D_uy D_ux (dt/2, g_n) applied right to left.  work must hold one
 * copy of f; fout receives the result. */
int vor_step(const vor_grid* g, int vbc, const double* fin, double* fout, double* work,
             const float* g_n, const float* g_np1, double dt, double a2inv, double* outflow)
{
    int rc = vor_check_grid(g);
    if (rc) return rc;
    double h = 0.5 * dt;
    double dta = dt * a2inv;
    /* first half kick with the field at t^n */
    rc |= vor_advect_velocity(g, 0, vbc, fin, fout, g_n, h, outflow);
    rc |= vor_advect_velocity(g, 1, vbc, fout, work, g_n, h, outflow);
    rc |= vor_advect_velocity(g, 2, vbc, work, fout, g_n, h, outflow);
    /* drift z, y, x */
    rc |= vor_advect_position(g, 2, fout, work, dta);
    rc |= vor_advect_position(g, 1, work, fout, dta);
    rc |= vor_advect_position(g, 0, fout, work, dta);
    /* second half kick with the field at t^{n+1} */
    rc |= vor_advect_velocity(g, 0, vbc, work, fout, g_np1, h, outflow);
    rc |= vor_advect_velocity(g, 1, vbc, fout, work, g_np1, h, outflow);
    rc |= vor_advect_velocity(g, 2, vbc, work, fout, g_np1, h, outflow);
    return rc;
}

/* Velocity moments per spatial cell (section 5.1.3):
 *   rho(x)   = sum_u f du^3
 *   umean(x) = sum_u u f du^3 / rho   (0 where rho = 0), layout [3][cells]
 *   mass     = sum_x rho dx^3 */
int vor_moments(const vor_grid* g, const double* f, double* rho, double* umean, double* mass)
{
    long Nx, Nu, c;
    int rc = vor_check_grid(g);
    if (rc) return rc;
    Nx = ncell_x(g);
    Nu = ncell_u(g);
    double du[3], dx3 = 1.0, du3 = 1.0;
    for (int a = 0; a < 3; ++a) {
        du[a] = 2.0 * g->umax[a] / g->nu[a];
        du3 *= du[a];
        dx3 *= g->L[a] / g->n[a];
    }
    #pragma omp parallel for schedule(static)
    for (c = 0; c < Nx; ++c) {
        double m0 = 0.0, m1[3] = {0.0, 0.0, 0.0};
        for (long ju = 0; ju < Nu; ++ju) {
            long jx = ju / ((long)g->nu[1] * g->nu[2]);
            long jy = (ju / g->nu[2]) % g->nu[1];
            long jz = ju % g->nu[2];
            double u[3];
            u[0] = -g->umax[0] + (jx + 0.5) * du[0];
            u[1] = -g->umax[1] + (jy + 0.5) * du[1];
            u[2] = -g->umax[2] + (jz + 0.5) * du[2];
            double v = f[c * Nu + ju];
            m0 += v;
            for (int a = 0; a < 3; ++a) m1[a] += u[a] * v;
        }
        rho[c] = m0 * du3;
        if (umean) {
            for (int a = 0; a < 3; ++a) umean[(long)a * Nx + c] = (m0 != 0.0) ? m1[a] / m0 : 0.0;
        }
    }
    if (mass) {
        double m = 0.0;
        for (c = 0; c < Nx; ++c) m += rho[c];
        *mass = m * dx3;
    }
    return 0;
}

/* Velocity dispersion tensor per spatial cell (section 5.1.3 lists it with
 * the density and mean velocity among the moments taken without data
 * exchange; the paper gives no formula).  Read as the density-weighted
 * covariance of u over the cell's velocity block:
 *   sigma_lm(x) = sum_u (u_l - umean_l)(u_m - umean_m) f / sum_u f,
 * 0 where sum_u f = 0.  Written as its definition: a first pass for the mean,
 * a second for the central products.  Layout [6][cells], components in the
 * order xx, xy, xz, yy, yz, zz. */
int vor_dispersion(const vor_grid* g, const double* f, double* sigma)
{
    long Nx, Nu, c;
    int rc = vor_check_grid(g);
    if (rc) return rc;
    Nx = ncell_x(g);
    Nu = ncell_u(g);
    double du[3];
    for (int a = 0; a < 3; ++a) du[a] = 2.0 * g->umax[a] / g->nu[a];
    static const int comp[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    #pragma omp parallel for schedule(static)
    for (c = 0; c < Nx; ++c) {
        const double* blk = f + c * Nu;
        double m0 = 0.0, mean[3] = {0.0, 0.0, 0.0};
        for (long ju = 0; ju < Nu; ++ju) {
            double u[3];
            u[0] = -g->umax[0] + (ju / ((long)g->nu[1] * g->nu[2]) + 0.5) * du[0];
            u[1] = -g->umax[1] + ((ju / g->nu[2]) % g->nu[1] + 0.5) * du[1];
            u[2] = -g->umax[2] + (ju % g->nu[2] + 0.5) * du[2];
            m0 += blk[ju];
            for (int a = 0; a < 3; ++a) mean[a] += u[a] * blk[ju];
        }
        double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (m0 != 0.0) {
            for (int a = 0; a < 3; ++a) mean[a] /= m0;
            for (long ju = 0; ju < Nu; ++ju) {
                double d[3];
                d[0] = -g->umax[0] + (ju / ((long)g->nu[1] * g->nu[2]) + 0.5) * du[0] - mean[0];
                d[1] = -g->umax[1] + ((ju / g->nu[2]) % g->nu[1] + 0.5) * du[1] - mean[1];
                d[2] = -g->umax[2] + (ju % g->nu[2] + 0.5) * du[2] - mean[2];
                for (int k = 0; k < 6; ++k) s[k] += d[comp[k][0]] * d[comp[k][1]] * blk[ju];
            }
            for (int k = 0; k < 6; ++k) s[k] /= m0;
        }
        for (int k = 0; k < 6; ++k) sigma[(long)k * Nx + c] = s[k];
    }
    return 0;
}
