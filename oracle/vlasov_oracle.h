/*
 * FP64 CPU oracle (test infrastructure only; see vlasov_oracle.c).
 * Independent of the HIP library: this header is included by the oracle
 * sources alone.
 */
#ifndef VLASOV_ORACLE_H
#define VLASOV_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* spatial cells n[3] in a periodic box [0, L), velocity cells nu[3] on
 * [-umax, umax) per axis */
typedef struct {
    int n[3];
    int nu[3];
    double L[3];
    double umax[3];
} vor_grid;

double vor_median3(double x, double y, double z);
double vor_minmod4(double w, double x, double y, double z);
void vor_sl5_weights(double mu, double w[5]);
/* largest alpha of the upper limit used by the bounds (see vor_mp_alpha) */
#define VOR_ALPHA_CAP 1048576.0
double vor_mp5_limit(double fhat, double a, double b, double c, double d, double e, double alpha);
double vor_mp_alpha(double mu);
void vor_split_shift(double s, long* N, double* nu);
double vor_interface_flux(const double* f, long M, long j, double nu, int periodic, int limiter);
void vor_sweep_line_opt(const double* f, double* out, long M, double s, int periodic,
                        int limiter, double* outflow);
void vor_sweep_line(const double* f, double* out, long M, double s, int periodic, double* outflow);

double vor_position_shift(const vor_grid* g, int a, long j, double dt_over_a2);
double vor_velocity_shift(const vor_grid* g, int a, float ga, double dt);
int vor_check_grid(const vor_grid* g);
int vor_advect_position(const vor_grid* g, int a, const double* fin, double* fout,
                        double dt_over_a2);
int vor_advect_velocity(const vor_grid* g, int a, int vbc, const double* fin, double* fout,
                        const float* gfield, double dt, double* outflow);
int vor_step(const vor_grid* g, int vbc, const double* fin, double* fout, double* work,
             const float* g_n, const float* g_np1, double dt, double a2inv, double* outflow);
int vor_moments(const vor_grid* g, const double* f, double* rho, double* umean, double* mass);
int vor_dispersion(const vor_grid* g, const double* f, double* sigma);

/* derivatives (vlasov_oracle_adj.c) */
void vor_sweep_line_jacobian(const double* f, long M, double s, int periodic, int limiter,
                             double* J, double* dnu);
void vor_sweep_line_tangent(const double* f, long M, double s, int periodic, const double* v,
                            double nu_dot, double* out_dot);
void vor_sweep_line_adjoint(const double* f, long M, double s, int periodic, const double* lam,
                            double* lam_in, double* lam_nu);
void vor_sweep_line_margin(const double* f, long M, double s, int periodic, double* margin);
int vor_advect_position_margin(const vor_grid* g, int a, const double* fin, double* margin,
                               double dt_over_a2);
int vor_advect_velocity_margin(const vor_grid* g, int a, int vbc, const double* fin,
                               const float* gfield, double dt, double* margin);
int vor_advect_position_adj(const vor_grid* g, int a, const double* fin, const double* lam_out,
                            double* lam_in, double dt_over_a2);
int vor_advect_velocity_adj(const vor_grid* g, int a, int vbc, const double* fin,
                            const float* gfield, double dt, const double* lam_out,
                            double* lam_in, double* lam_g);
int vor_advect_velocity_tan(const vor_grid* g, int a, int vbc, const double* fin,
                            const float* gfield, const double* g_dot, double dt, const double* v,
                            double* out_dot);
int vor_advect_position_tan(const vor_grid* g, int a, const double* fin, const double* v,
                            double* out_dot, double dt_over_a2);
int vor_step_adj(const vor_grid* g, int vbc, const double* fin, const float* g_n,
                 const float* g_np1, double dt, double a2inv, const double* lam_out,
                 double* lam_in, double* lam_g_n, double* lam_g_np1);
int vor_moments_adj(const vor_grid* g, const double* f, const double* lam_rho,
                    const double* lam_umean, double* lam_f);

#ifdef __cplusplus
}
#endif
#endif
