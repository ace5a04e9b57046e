/*
 * libvlasov -- split SL-MPP5 advection of the distribution function f(x,u)
 * on a six-dimensional phase-space grid, for AMD Instinct MI355X (gfx950).
 *
 * Method (Yoshikawa, Tanaka & Yoshida, "A 400 trillion-grid Vlasov
 * simulation on Fugaku supercomputer", SC'21):
 *   - Vlasov equation, Eq. (1), split into six 1D advections: position
 *     sweeps along x, y, z with speed u_i / a^2 (Eq. 3) and velocity sweeps
 *     along ux, uy, uz with speed g_i = -d(phi)/dx_i (Eq. 4), section 5.1.1;
 *   - one full step composed as in Eq. (5);
 *   - each 1D operator is SL-MPP5 (section 5.2): fifth-order finite volume,
 *     conservative semi-Lagrangian interface flux (exact integral of the
 *     quartic reconstruction over the upwind departure interval), limited by
 *     the Suresh-Huynh monotonicity-preserving bounds and a positivity
 *     clamp, one flux evaluation per cell per step.  The shift s splits
 *     into its nearest integer (an exact translation) and a fraction nu of
 *     at most half a cell; the bounds' upper limit f_j + alpha (f_j - f_{j-1})
 *     takes alpha = (1-|nu|)/|nu|, the largest value for which the
 *     single-stage update keeps monotone data monotone, so repeated sweeps
 *     create no new extrema at any shift;
 *   - FP32 flux arithmetic (section 5.1.1); FP64 only for reductions;
 *   - velocity moments per spatial cell without data exchange (5.1.3).
 *
 * Data layout (List 1 of section 5.3 without the per-cell header):
 *   f[ix][iy][iz][jx][jy][jz], jz fastest; cell centres x_i = (i+1/2) L/n,
 *   u_j = -umax + (j+1/2) du with du = 2 umax / nu.  The header fields of
 *   List 1 (dens, mean velocity) are separate FP64 arrays [nx][ny][nz].
 *
 * Storage precisions: FP32, or FP16 / BF16 with one FP32 scale per
 * uz-line (the nu_z values of one (ix,iy,iz,jx,jy)): value = code * scale,
 * scale = largest |value| on the line.  Scale arrays have
 * nx*ny*nz*nux*nuy entries and are NULL for FP32.
 *
 * Conventions for every entry point:
 *   - Pointers to arrays are DEVICE pointers owned by the caller; the grid
 *     is a HOST pointer read during the call only.  The library keeps no
 *     reference after returning and allocates nothing: scratch space is the
 *     caller's workspace.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Calls enqueue work and return without synchronising.
 *   - Out-of-place only: an output that overlaps an input is rejected.
 *   - Results are bitwise reproducible for identical inputs (no atomics,
 *     fixed-order reductions).
 *   - Errors are returned as negative codes; nothing aborts.  Argument
 *     checks are host-side and O(1); a launch failure maps to
 *     VLASOV_ERR_DEVICE.  Array contents are not inspected: f must be finite
 *     and non-negative for the positivity guarantee.
 *   - Calls are reentrant; the library holds no global state.
 */
#ifndef LIBVLASOV_H
#define LIBVLASOV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VLASOV_ABI_VERSION 1

/* Phase-space grid: n[3] spatial cells of the periodic box [0, L) and nu[3]
 * velocity cells of [-umax, umax) per axis (domain of section 5.1.3). */
typedef struct vlasov_grid {
    int32_t n[3];
    int32_t nu[3];
    double L[3];
    double umax[3];
} vlasov_grid;

typedef enum vlasov_prec {
    VLASOV_F32 = 0,   /* float */
    VLASOV_F16 = 1,   /* IEEE half code per value + FP32 scale per uz-line */
    VLASOV_BF16 = 2   /* bfloat16 code per value + FP32 scale per uz-line */
} vlasov_prec;

/* Velocity-space boundary.  OUTFLOW: vacuum outside [-umax, umax), the
 * content leaving through a face is tallied.  PERIODIC: wrap (used to test
 * invariants; not physical). */
typedef enum vlasov_vbc {
    VLASOV_VBC_OUTFLOW = 0,
    VLASOV_VBC_PERIODIC = 1
} vlasov_vbc;

enum {
    VLASOV_OK = 0,
    VLASOV_ERR_NULL = -1,       /* a required pointer is NULL */
    VLASOV_ERR_SHAPE = -2,      /* grid sizes/extents invalid or unsupported */
    VLASOV_ERR_PREC = -3,       /* unknown precision or vbc, or scale missing */
    VLASOV_ERR_ALIAS = -4,      /* an output overlaps an input */
    VLASOV_ERR_NONFINITE = -5,  /* dt, a^-2 or the derived shift factor is not finite */
    VLASOV_ERR_DEVICE = -6,     /* HIP launch or runtime error */
    VLASOV_ERR_WORKSPACE = -7,  /* workspace NULL or smaller than required */
    VLASOV_ERR_TOO_LARGE = -8   /* grid exceeds the fixed scratch of an allocation-free call */
};

/* Version of this interface (VLASOV_ABI_VERSION). */
int vlasov_abi_version(void);

/* Static description of an error code; never NULL. */
const char* vlasov_strerror(int code);

/* Storage bytes of one copy of f (codes only) and of its scale array. */
size_t vlasov_f_bytes(const vlasov_grid* grid, vlasov_prec prec);
size_t vlasov_scale_bytes(const vlasov_grid* grid, vlasov_prec prec);

/*
 * Position sweeps (Eq. 3): advance f along x, y or z over dt.  The shift of
 * the line with velocity index j is s_j = u_j * dt_over_a2 / dx in cells
 * (dt_over_a2 = dt / a(t)^2; a = 1 gives dt).  s = N + nu is split into an
 * integer part applied as an exact translation and a fraction applied by the
 * SL-MPP5 flux (see the method summary above); the box is periodic.  Any
 * |s| is accepted.
 *   f_in / scale_in : input f (and its scales for F16/BF16)
 *   f_out / scale_out : output f (and scales); must not overlap the inputs
 */
int vlasov_advect_x(const vlasov_grid* grid, vlasov_prec prec, const void* f_in,
                    const float* scale_in, void* f_out, float* scale_out,
                    double dt_over_a2, void* stream);
int vlasov_advect_y(const vlasov_grid* grid, vlasov_prec prec, const void* f_in,
                    const float* scale_in, void* f_out, float* scale_out,
                    double dt_over_a2, void* stream);
int vlasov_advect_z(const vlasov_grid* grid, vlasov_prec prec, const void* f_in,
                    const float* scale_in, void* f_out, float* scale_out,
                    double dt_over_a2, void* stream);

/*
 * Velocity sweeps (Eq. 4): advance f along ux, uy or uz over dt.  The shift
 * of every line of spatial cell c is s = g[axis][c] * dt / du (the advection
 * speed in velocity space is g = -grad phi).
 *   g       : FP32 field [3][nx][ny][nz], device
 *   outflow : FP64 [nx][ny][nz], device, or NULL.  With VBC_OUTFLOW the
 *             content that leaves [-umax, umax) through the two faces of
 *             this axis, in density units (sum of f times du^3), is ADDED to
 *             outflow[c].  Untouched with VBC_PERIODIC.
 */
int vlasov_advect_ux(const vlasov_grid* grid, vlasov_prec prec, vlasov_vbc vbc,
                     const void* f_in, const float* scale_in, void* f_out, float* scale_out,
                     const float* g, double dt, double* outflow, void* stream);
int vlasov_advect_uy(const vlasov_grid* grid, vlasov_prec prec, vlasov_vbc vbc,
                     const void* f_in, const float* scale_in, void* f_out, float* scale_out,
                     const float* g, double dt, double* outflow, void* stream);
int vlasov_advect_uz(const vlasov_grid* grid, vlasov_prec prec, vlasov_vbc vbc,
                     const void* f_in, const float* scale_in, void* f_out, float* scale_out,
                     const float* g, double dt, double* outflow, void* stream);

/*
 * Velocity kick: D_uz D_uy D_ux over dt with one field g, i.e. the three
 * velocity sweeps of one half step of Eq. (5) (with dt the half step).
 * Velocity blocks of 16^3 or 32^3 cells are swept inside LDS (one HBM read
 * and one write of f instead of three); other shapes run the three sweeps
 * and then need `work` (vlasov_step_workspace_bytes, else VLASOV_ERR_WORKSPACE);
 * work may be NULL for the fused shapes.  With FP32 storage the result is
 * bitwise that of vlasov_advect_ux, _uy, _uz in sequence.  With FP16/BF16
 * storage the fused shapes keep the values between the three sweeps in FP32
 * and round only the result, so they differ from the three single sweeps by
 * those sweeps' two intermediate roundings (about one code unit of the line
 * scale); the outflow tally differs by the same relative amount.
 */
int vlasov_kick(const vlasov_grid* grid, vlasov_prec prec, vlasov_vbc vbc, const void* f_in,
                const float* scale_in, void* f_out, float* scale_out, const float* g, double dt,
                void* work, size_t work_bytes, double* outflow, void* stream);

/* Bytes of workspace vlasov_step needs: one intermediate copy of f plus its
 * scales, 256-byte aligned. */
size_t vlasov_step_workspace_bytes(const vlasov_grid* grid, vlasov_prec prec);

/*
 * One full step, Eq. (5):
 *   f^{n+1} = D_uz D_uy D_ux(dt/2; g_np1) D_x D_y D_z(dt) D_uz D_uy D_ux(dt/2; g_n) f^n
 * applied right to left: half kicks ux, uy, uz with the field at t^n, drifts
 * z, y, x with dt * a2inv, half kicks ux, uy, uz with the field at t^{n+1}.
 * Nine sweeps: each group of three velocity sweeps runs as one vlasov_kick;
 * intermediates ping-pong between f_out and work.
 *   g_n, g_np1 : FP32 fields [3][nx][ny][nz] at t^n and t^{n+1}
 *   a2inv      : a(t)^-2 for the drifts
 *   work       : device workspace of at least vlasov_step_workspace_bytes
 *   outflow    : as for the velocity sweeps (accumulated over the six kicks)
 */
int vlasov_step(const vlasov_grid* grid, vlasov_prec prec, vlasov_vbc vbc, const void* f_in,
                const float* scale_in, void* f_out, float* scale_out, const float* g_n,
                const float* g_np1, double dt, double a2inv, void* work, size_t work_bytes,
                double* outflow, void* stream);

/*
 * vlasov_step, also returning the velocity moments of f^{n+1} (section
 * 5.1.3) as vlasov_moments defines them: rho [nx][ny][nz] (required) and
 * umean [3][nx][ny][nz] (may be NULL), FP64 device arrays.  Where the last
 * kick runs fused, the moments are summed while it stores each cell's block
 * (from the stored values: decoded codes for FP16/BF16), so no pass reads
 * f^{n+1} again; otherwise they come from a moments pass over f_out.  The
 * summation order differs from vlasov_moments', so the two agree to FP64
 * rounding, not to the bit.  f_out is the bits vlasov_step writes.
 * Errors: as vlasov_step; VLASOV_ERR_NULL for a NULL rho; VLASOV_ERR_ALIAS
 * when rho or umean overlap each other, f_in, f_out or work.
 */
int vlasov_step_moments(const vlasov_grid* grid, vlasov_prec prec, vlasov_vbc vbc,
                        const void* f_in, const float* scale_in, void* f_out, float* scale_out,
                        const float* g_n, const float* g_np1, double dt, double a2inv,
                        void* work, size_t work_bytes, double* outflow, double* rho,
                        double* umean, void* stream);

/* Bytes of workspace vlasov_steps needs: two intermediate copies of f plus
 * their scales, and the kick's shift table, 256-byte aligned. */
size_t vlasov_steps_workspace_bytes(const vlasov_grid* grid, vlasov_prec prec);

/*
 * nsteps steps of Eq. (5) with the half kicks that meet between two steps
 * merged into one: the trailing half kick of step k and the leading half
 * kick of step k+1 both use the field at t^{k+1}, and run as one kick over
 * dt (a kick moves f along u with a field that is fixed during it, so in
 * exact arithmetic the two forms agree):
 *   K(dt/2; g_0), then for k = 0 .. nsteps-1: D_x D_y D_z(dt a2inv[k]) and
 *   K(dt; g_{k+1}), the last one K(dt/2; g_nsteps).
 * nsteps + 1 kicks instead of 2 nsteps: 4 passes over f per step instead of
 * 5.  The semi-Lagrangian flux of one kick over dt is not the composition of
 * two over dt/2, so results differ from repeated vlasov_step at the scheme's
 * truncation error; they follow the same merged composition of the single
 * sweeps.  For callers that need no state between the steps.
 *   fields : FP32 device array [nsteps + 1][3][nx][ny][nz], the field at t^k
 *            in slot k
 *   a2inv  : HOST array of nsteps drift factors a(t)^-2, or NULL for all 1
 *   work   : device workspace of at least vlasov_steps_workspace_bytes
 *   outflow: as for vlasov_step (accumulated over all kicks), may be NULL
 * Errors: as vlasov_step; VLASOV_ERR_SHAPE for nsteps < 1; VLASOV_ERR_ALIAS
 * when fields overlap f_out or work.
 */
int vlasov_steps(const vlasov_grid* grid, vlasov_prec prec, vlasov_vbc vbc, const void* f_in,
                 const float* scale_in, void* f_out, float* scale_out, const float* fields,
                 int nsteps, double dt, const double* a2inv, void* work, size_t work_bytes,
                 double* outflow, void* stream);

/* Bytes of workspace vlasov_field needs (twiddle tables and FP64 complex
 * spectra, 256-byte aligned). */
size_t vlasov_field_workspace_bytes(const vlasov_grid* grid);

/*
 * The acceleration field of a density on the periodic spatial mesh: the
 * Poisson equation (Eq. 2), nabla^2 phi = coupling (rho - mean rho), solved
 * by the discrete Fourier transform (the convolution method of the paper's
 * mesh part, section 3), and g = -grad phi (the speed of Eq. 4):
 *   phi_k = -coupling rho_k / |k|^2 (mean removed), g_a,k = -i k_a phi_k,
 *   k_a = 2 pi m_a / L_a with m_a the signed index; k_a = 0 on the Nyquist
 *   plane of an even axis for the derivative.
 * FP64 throughout (separable DFTs, one pass per axis), g stored as FP32.
 *   rho      : FP64 device [nx][ny][nz] (e.g. from vlasov_moments)
 *   coupling : 4 pi G a(t)^2
 *   field    : FP32 device [3][nx][ny][nz], the layout vlasov_step takes
 *   work     : device workspace of at least vlasov_field_workspace_bytes
 * Errors: VLASOV_ERR_NULL, VLASOV_ERR_SHAPE (bad grid, L <= 0),
 * VLASOV_ERR_NONFINITE, VLASOV_ERR_WORKSPACE, VLASOV_ERR_ALIAS.
 */
int vlasov_field(const vlasov_grid* grid, const double* rho, double coupling, float* field,
                 void* work, size_t work_bytes, void* stream);

/* Bytes of workspace vlasov_step_sc needs: vlasov_step's, 256-byte aligned,
 * followed by vlasov_field's. */
size_t vlasov_step_sc_workspace_bytes(const vlasov_grid* grid, vlasov_prec prec);

/*
 * One self-consistent step of the Vlasov-Poisson system (Eqs. 1, 2, 5):
 * half kicks ux, uy, uz with the field g_n at t^n, drifts z, y, x, then the
 * density of the drifted f (the kicks move f along u only, so it is the
 * density at t^{n+1}), its field by vlasov_field with `coupling`
 * (4 pi G a(t^{n+1})^2), and the half kicks with that field.  The density is
 * that of f alone: the CDM part of the paper's mesh density is not modelled.
 *   g_n     : FP32 device [3][nx][ny][nz], field at t^n (vlasov_field of the
 *             density of f^n, or the previous step's g_np1)
 *   g_np1   : FP32 device [3][nx][ny][nz], OUT: field at t^{n+1}
 *   rho_np1 : FP64 device [nx][ny][nz], OUT: density of f^{n+1}
 *   work    : device workspace of at least vlasov_step_sc_workspace_bytes
 * Other arguments and errors as vlasov_step and vlasov_field; g_np1 and
 * rho_np1 must not overlap each other, g_n, f_in, f_out or work.
 */
int vlasov_step_sc(const vlasov_grid* grid, vlasov_prec prec, vlasov_vbc vbc, const void* f_in,
                   const float* scale_in, void* f_out, float* scale_out, const float* g_n,
                   float* g_np1, double* rho_np1, double coupling, double dt, double a2inv,
                   void* work, size_t work_bytes, double* outflow, void* stream);

/*
 * Background expansion for comoving runs: Eq. (1) drifts comoving positions
 * at u / a(t)^2 and Eq. (2) carries 4 pi G a(t)^2 (rho - mean rho).  The
 * background is a flat universe of matter (omega_m) and a cosmological
 * constant (1 - omega_m), radiation neglected, H0 in the inverse time unit of
 * dt; a(t) is the closed-form solution of its Friedmann equation, t cosmic
 * time from the big bang.  Host functions, no device work.
 *
 *   vlasov_cosmo_a:     *a = a(t)
 *   vlasov_cosmo_t:     *t = t(a) (e.g. the start time of a run at redshift
 *                       z: a = 1 / (1 + z))
 *   vlasov_cosmo_steps: for steps of dt from t0, host arrays
 *                       a[k] = a(t0 + k dt), k = 0..nsteps (a may be NULL),
 *                       a2inv[n] = (1/dt) * integral of dt'/a(t')^2 over
 *                       step n (adaptive Gauss-Legendre, relative 1e-14):
 *                       the a2inv argument of vlasov_step, vlasov_step_sc
 *                       or vlasov_steps for that step, which moves a
 *                       position by u times the integral (u is constant
 *                       during the drift).
 * For a comoving f the density rho = sum f du^3 keeps its mean, and Eq. (2)
 * reads nabla^2 phi = (K / a)(rho - mean rho), K = 4 pi G times the physical
 * density of one unit of rho at a = 1: the coupling of vlasov_step_sc for
 * step n is K / a[n+1] (its field is taken at t0 + (n+1) dt).
 * Errors: VLASOV_ERR_NULL (cosmology or an output NULL), VLASOV_ERR_NONFINITE
 * (t, a, t0 or dt not finite, or a result overflows), VLASOV_ERR_SHAPE
 * (omega_m outside (0, 1], H0 <= 0, t, a, t0 or dt <= 0, nsteps < 1).
 */
typedef struct vlasov_cosmology {
    double omega_m;   /* matter density parameter today, 0 < omega_m <= 1 */
    double H0;        /* Hubble constant today, in 1 / (time unit of dt) */
} vlasov_cosmology;

int vlasov_cosmo_a(const vlasov_cosmology* cosmo, double t, double* a);
int vlasov_cosmo_t(const vlasov_cosmology* cosmo, double a, double* t);
int vlasov_cosmo_steps(const vlasov_cosmology* cosmo, double t0, double dt, int nsteps,
                       double* a, double* a2inv);

/*
 * Velocity moments per spatial cell (section 5.1.3), accumulated in FP64:
 *   rho[c]      = sum_u f du^3
 *   umean[a][c] = sum_u u_a f du^3 / rho[c]  (0 where rho[c] = 0); may be NULL
 *   mass        = sum_c rho[c] dx^3 (device FP64 scalar); may be NULL
 * rho and umean are FP64 device arrays [nx][ny][nz] and [3][nx][ny][nz].
 */
int vlasov_moments(const vlasov_grid* grid, vlasov_prec prec, const void* f, const float* scale,
                   double* rho, double* umean, double* mass, void* stream);

/*
 * The velocity moments up to second order per spatial cell, the velocity
 * dispersion tensor among them (section 5.1.3 names it with the density and
 * mean velocity as moments needing no data exchange; the paper gives no
 * formula, and it is read as the density-weighted covariance of u):
 *   rho[c], umean[a][c]  as vlasov_moments (umean may be NULL)
 *   sigma[k][c] = sum_u (u_l - umean_l)(u_m - umean_m) f / sum_u f, with
 *                 (l,m) = xx, xy, xz, yy, yz, zz for k = 0..5; 0 where
 *                 rho[c] = 0.
 * One pass over f: FP64 sums of f, u f and u_l u_m f about u = 0, then sigma =
 * <u_l u_m> - umean_l umean_m, which keeps about 16 - log10(<u^2>/sigma)
 * digits.  rho [nx][ny][nz], umean [3][...], sigma [6][...]: FP64 device.
 * Errors: VLASOV_ERR_NULL (grid, f, rho or sigma NULL), VLASOV_ERR_SHAPE,
 * VLASOV_ERR_PREC (unknown precision; FP16/BF16 without scale),
 * VLASOV_ERR_ALIAS (rho, umean, sigma overlap), VLASOV_ERR_DEVICE.
 */
int vlasov_dispersion(const vlasov_grid* grid, vlasov_prec prec, const void* f,
                      const float* scale, double* rho, double* umean, double* sigma,
                      void* stream);

/*
 * Derivatives (FP32 storage only).  With the limiter's selections frozen at
 * the forward input f_in -- the forward arithmetic is re-run on f_in and each
 * minimum, maximum, median, minmod and clamp keeps the argument it selected
 * -- a sweep is the linear map f_out = J f_in, smooth in the fractional
 * shift.  At ties between equal candidates the first argument of a minimum
 * or maximum wins and the median is max(min(x,y), min(max(x,y),z)); at a
 * whole-cell shift the shift derivative is the one-sided limit from the side
 * the shift comes from.  Tangent and adjoint share one linearisation, so
 * <tan(v), w> = <v, adj(w)> (+ field terms) up to FP32 rounding.
 *
 *   _tan: v_out = J v_in (+ d f_out/d g . g_dot for velocity sweeps; g_dot
 *         is FP32 [3][cells] or NULL; only the swept component is read)
 *   _adj: lam_in = J^T lam_out (overwritten); velocity sweeps ADD
 *         lam_out . d f_out/d g to lam_g[axis][cell] (FP32 [3][cells], or
 *         NULL to skip)
 * All arrays are device FP32 in the layout of f; outputs must not overlap
 * the inputs.
 */
int vlasov_advect_x_tan(const vlasov_grid* grid, const float* f_in, const float* v_in,
                        float* v_out, double dt_over_a2, void* stream);
int vlasov_advect_y_tan(const vlasov_grid* grid, const float* f_in, const float* v_in,
                        float* v_out, double dt_over_a2, void* stream);
int vlasov_advect_z_tan(const vlasov_grid* grid, const float* f_in, const float* v_in,
                        float* v_out, double dt_over_a2, void* stream);
int vlasov_advect_x_adj(const vlasov_grid* grid, const float* f_in, const float* lam_out,
                        float* lam_in, double dt_over_a2, void* stream);
int vlasov_advect_y_adj(const vlasov_grid* grid, const float* f_in, const float* lam_out,
                        float* lam_in, double dt_over_a2, void* stream);
int vlasov_advect_z_adj(const vlasov_grid* grid, const float* f_in, const float* lam_out,
                        float* lam_in, double dt_over_a2, void* stream);
int vlasov_advect_ux_tan(const vlasov_grid* grid, vlasov_vbc vbc, const float* f_in,
                         const float* g, const float* g_dot, double dt, const float* v_in,
                         float* v_out, void* stream);
int vlasov_advect_uy_tan(const vlasov_grid* grid, vlasov_vbc vbc, const float* f_in,
                         const float* g, const float* g_dot, double dt, const float* v_in,
                         float* v_out, void* stream);
int vlasov_advect_uz_tan(const vlasov_grid* grid, vlasov_vbc vbc, const float* f_in,
                         const float* g, const float* g_dot, double dt, const float* v_in,
                         float* v_out, void* stream);
int vlasov_advect_ux_adj(const vlasov_grid* grid, vlasov_vbc vbc, const float* f_in,
                         const float* g, double dt, const float* lam_out, float* lam_in,
                         float* lam_g, void* stream);
int vlasov_advect_uy_adj(const vlasov_grid* grid, vlasov_vbc vbc, const float* f_in,
                         const float* g, double dt, const float* lam_out, float* lam_in,
                         float* lam_g, void* stream);
int vlasov_advect_uz_adj(const vlasov_grid* grid, vlasov_vbc vbc, const float* f_in,
                         const float* g, double dt, const float* lam_out, float* lam_in,
                         float* lam_g, void* stream);

/* Workspace of vlasov_step_adj: the eight intermediate stages of Eq. (5)
 * recomputed from f_in plus one adjoint buffer (nine FP32 copies of f). */
size_t vlasov_step_adj_workspace_bytes(const vlasov_grid* grid);

/*
 * Adjoint of vlasov_step (FP32): the forward stages are recomputed from f_in
 * into `work`, then the nine sweeps are transposed in reverse order.
 * lam_in = (d f_out / d f_in)^T lam_out; lam_g_n and lam_g_np1 (FP32
 * [3][cells]) are ADDED the gradients with respect to the fields at t^n and
 * t^{n+1}.  Outflow tallies carry no adjoint.
 */
int vlasov_step_adj(const vlasov_grid* grid, vlasov_vbc vbc, const float* f_in,
                    const float* g_n, const float* g_np1, double dt, double a2inv,
                    const float* lam_out, float* lam_in, float* lam_g_n, float* lam_g_np1,
                    void* work, size_t work_bytes, void* stream);

/*
 * Adjoint of vlasov_moments (section 5.1.3) at the forward result rho,
 * umean (FP64 device arrays from vlasov_moments):
 *   lam_f[c][u] += du^3 lam_rho[c] + du^3 sum_a lam_umean[a][c] (u_a - umean[a][c]) / rho[c]
 * (the umean term only where rho[c] != 0; lam_umean, rho and umean may be
 * NULL together).  lam_f is FP32 in the layout of f and is accumulated.
 */
int vlasov_moments_adj(const vlasov_grid* grid, const double* rho, const double* umean,
                       const double* lam_rho, const double* lam_umean, float* lam_f,
                       void* stream);

/*
 * vlasov_field for callers that cannot allocate (code under stream capture,
 * serving loops, harnesses that forbid allocation): the same computation,
 * with its twiddle tables and FP64 spectra in a fixed device array of the
 * library instead of a caller workspace.  The array holds
 * vlasov_field_noalloc_max_bytes() bytes (24 MiB: meshes up to 64^3 cells);
 * each device keeps its own copy until the process ends, and its address is
 * looked up on the first call on that device.  Results are vlasov_field's,
 * bit for bit.  Every call on one device uses the same array: calls that
 * overlap on one device (concurrent streams) race.  No allocation, no
 * hipMalloc, no caller workspace.
 * Errors: as vlasov_field; VLASOV_ERR_TOO_LARGE when the mesh needs more
 * than the fixed array (vlasov_field_workspace_bytes > max_bytes).
 */
size_t vlasov_field_noalloc_max_bytes(void);
int vlasov_field_noalloc(const vlasov_grid* grid, const double* rho, double coupling,
                         float* field, void* stream);

/*
 * Storage codec of the FP16/BF16 forms (the reduced-precision storage of f;
 * the paper's own arithmetic, section 5.1.1, is FP32 throughout).
 *   vlasov_encode: f32 (FP32, layout of f) -> codes (layout of f, 2 bytes
 *     each) and scale ([nx][ny][nz][nux][nuy] FP32): scale = the largest
 *     |value| of the uz-line, code = RNE(value * r) with r the hardware
 *     reciprocal of the scale (0 for an all-zero line) -- exactly what every
 *     sweep stores for the same FP32 values.
 *   vlasov_decode: codes, scale -> f32 = code * scale in FP32, exactly what
 *     every sweep loads.
 * With VLASOV_F32 both copy the values (scale unused, may be NULL).  Device
 * pointers, caller-owned; codes and f32 16-byte aligned; nu_z a power of two
 * from 4 to 64 for FP16/BF16.  Errors: VLASOV_ERR_NULL (grid, f32 or codes
 * NULL), VLASOV_ERR_PREC (unknown precision; FP16/BF16 without scale),
 * VLASOV_ERR_SHAPE (grid, alignment or nu_z), VLASOV_ERR_ALIAS (outputs
 * overlap inputs), VLASOV_ERR_DEVICE.
 */
int vlasov_encode(const vlasov_grid* grid, vlasov_prec prec, const float* f32, void* codes,
                  float* scale, void* stream);
int vlasov_decode(const vlasov_grid* grid, vlasov_prec prec, const void* codes,
                  const float* scale, float* f32, void* stream);

/* Deterministic FP64 sum of x[0..n) into *out (device pointers): a single
 * work-group, fixed order.  Used for total mass and total outflow. */
int vlasov_sum_f64(const double* x, int64_t n, double* out, void* stream);

/* Plain copy of `bytes` (multiple of 16, 16-byte aligned, non-overlapping)
 * from src to dst on the device: the HBM bandwidth probe that sets the
 * practical ceiling of a streaming kernel and calibrates traffic counters.
 * Not part of the method. */
int vlasov_stream_copy(const void* src, void* dst, size_t bytes, void* stream);

/* Vector-ALU probe: n threads (n a positive multiple of 256) each run eight
 * independent chains of FP32 FMA, med3, min3, max3, add and mul for `iters`
 * iterations and write one float to out[0..n) (device memory of n floats,
 * caller-owned).  *lane_ops (host pointer) receives the lane-operations
 * launched, 64 n iters, so that the kernel's time gives the issue rate the
 * sweeps' arithmetic can reach.  Not part of the method. */
int vlasov_valu_probe(float* out, int64_t n, int iters, double* lane_ops, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LIBVLASOV_H */
