// C-ABI of libvlasov: argument checks, per-line shift tables and the launch
// sequence of each entry point.  Declarations and their contracts are in
// include/vlasov.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "../../include/vlasov.h"
#include "launch.hpp"

using namespace vlasov;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Dims {
    long n[3], nu[3];
    long cells, Nu, total;
};

bool dims_of(const vlasov_grid* g, Dims& d)
{
    if (g == nullptr) return false;
    for (int a = 0; a < 3; ++a) {
        if (g->n[a] < 1 || g->nu[a] < 1) return false;
        if (!(g->L[a] > 0.0) || !isfinite(g->L[a])) return false;
        if (!(g->umax[a] > 0.0) || !isfinite(g->umax[a])) return false;
        d.n[a] = g->n[a];
        d.nu[a] = g->nu[a];
    }
    d.cells = d.n[0] * d.n[1] * d.n[2];
    d.Nu = d.nu[0] * d.nu[1] * d.nu[2];
    if (d.cells > 0x7fffffffL) return false;          // one work-group per cell
    if (d.Nu > 0x7fffffffL) return false;
    d.total = d.cells * d.Nu;
    return true;
}

size_t elem_bytes(int prec) { return prec == VLASOV_F32 ? 4 : 2; }

bool prec_ok(int prec) { return prec == VLASOV_F32 || prec == VLASOV_F16 || prec == VLASOV_BF16; }

// Scaled storage keeps one scale per uz-line; the kernels spread a uz-line
// over a power-of-two group of lanes.
bool scaled_shape_ok(const Dims& d)
{
    const long z = d.nu[2];
    return z >= 4 && z <= 64 && (z & (z - 1)) == 0;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb)
{
    if (a == nullptr || b == nullptr || na == 0 || nb == 0) return false;
    const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
    return pa < pb + nb && pb < pa + na;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

int vector_width(long nuz) { return nuz % 4 == 0 ? 4 : (nuz % 2 == 0 ? 2 : 1); }

// Common checks of a sweep's storage arguments.
int check_io(const Dims& d, int prec, const void* fin, const float* sin, const void* fout,
             const float* sout)
{
    if (!prec_ok(prec)) return VLASOV_ERR_PREC;
    if (fin == nullptr || fout == nullptr) return VLASOV_ERR_NULL;
    if (!aligned16(fin) || !aligned16(fout)) return VLASOV_ERR_SHAPE;
    const size_t fb = (size_t)d.total * elem_bytes(prec);
    if (prec != VLASOV_F32) {
        if (sin == nullptr || sout == nullptr) return VLASOV_ERR_PREC;
        if (!scaled_shape_ok(d)) return VLASOV_ERR_SHAPE;
        const size_t sb = (size_t)(d.total / d.nu[2]) * sizeof(float);
        if (overlap(sout, sb, sin, sb) || overlap(sout, sb, fin, fb) || overlap(fout, fb, sin, sb))
            return VLASOV_ERR_ALIAS;
    }
    if (overlap(fout, fb, fin, fb)) return VLASOV_ERR_ALIAS;
    return VLASOV_OK;
}

int from_hip(hipError_t e) { return e == hipSuccess ? VLASOV_OK : VLASOV_ERR_DEVICE; }

// Shift of the position sweep along axis a for velocity index j (Eq. 3):
// s_j = u_j * dt a^-2 / dx with u_j the cell centre of velocity cell j.
double position_shift(const vlasov_grid* g, int a, long j, double dt_over_a2)
{
#pragma clang fp contract(off)
    const double dx = g->L[a] / g->n[a];
    const double factor = dt_over_a2 / dx;
    const double du = 2.0 * g->umax[a] / g->nu[a];
    const double u = -g->umax[a] + (j + 0.5) * du;
    return u * factor;
}

// Integer part of a periodic line's shift in its upwind frame, as the
// kernels split it (floor of |s|, reduced mod M), and its direction.
void split_integer(double s, int M, int* N, bool* neg)
{
    const double n = (s >= 0.0) ? floor(s) : ceil(s);
    *neg = s < 0.0;
    *N = (int)fmod(*neg ? -n : n, (double)M);
}

// Whether the z sweep can pair the two halves of each uz-line in one lane
// (see k_position_pair): every line of the upper half must move up and every
// line of the lower half down, all by less than one cell; the half length
// must divide the wave, a row must hold whole waves of lanes and the line
// length must have a compiled walk.  Returns 1 when it can, else 0.
int pair_mode(const PosArgs& a)
{
    const long nuz = a.nuz;
    const long H = nuz / 2;
    if (a.V != 1 || a.pst != 1 || a.nshift != nuz || nuz % 2 != 0) return 0;
    if (H != 8 && H != 16 && H != 32) return 0;
    if ((a.I / 2) % 64 != 0) return 0;
    if (a.M != 16 && a.M != 32 && a.M != 64) return 0;
    for (long j = 0; j < nuz; ++j) {
        int n;
        bool neg;
        split_integer(a.shift[j], a.M, &n, &neg);
        if (n != 0 || neg != (j < H)) return 0;
    }
    return 1;
}

int make_pos_args(const vlasov_grid* g, const Dims& d, int axis, double dt_over_a2, PosArgs& a)
{
    if (!isfinite(dt_over_a2)) return VLASOV_ERR_NONFINITE;
    if (d.nu[axis] > kMaxShiftTable) return VLASOV_ERR_SHAPE;
    memset(&a, 0, sizeof(a));
    a.O = 1;
    for (int b = 0; b < axis; ++b) a.O *= d.n[b];
    a.M = (int)d.n[axis];
    a.I = d.Nu;
    for (int b = axis + 1; b < 3; ++b) a.I *= d.n[b];
    a.Nu = d.Nu;
    a.pst = axis == 0 ? d.nu[1] * d.nu[2] : (axis == 1 ? d.nu[2] : 1);
    a.nshift = (int)d.nu[axis];
    a.nuz = d.nu[2];
    a.nux = d.nu[0];
    a.V = axis == 2 ? 1 : vector_width(d.nu[2]);
    a.G = (int)(d.nu[2] / a.V);
    for (long j = 0; j < d.nu[axis]; ++j) {
        a.shift[j] = position_shift(g, axis, j, dt_over_a2);
        if (!isfinite(a.shift[j])) return VLASOV_ERR_NONFINITE;
    }
    if (axis == 2) a.pair = pair_mode(a);
    a.skew = axis != 2;
    // a wave covers 64 V consecutive inner elements; they share the shift
    // when the velocity index that sets it changes only every pst elements
    a.us = a.pst % (64L * a.V) == 0 ? 1 : 0;
    // y sweep: the shift follows u_y, which changes every nu_z elements.  A
    // wave can still hold one u_y value if its lanes take R = 64 V / nu_z
    // whole uz-lines from R consecutive u_x rows (k_position's gathered
    // mapping): nu_z / V lanes per uz-line making up the wave, R dividing
    // nu_x, nu_y a multiple of 4 (4 waves of a work-group share a unit),
    // rows of whole work-groups and units filling groups of eight.
    a.ug = 0;
    // (taken for FP32 storage only -- k_position decides: an FP16/BF16
    // uz-line is 64 bytes, and a gathered wave would read half cache lines)
    if (axis == 1 && !a.us && a.V == 4 && (64L * a.V) % a.nuz == 0 &&
        (a.I / a.V) % 256 == 0 && d.nu[1] % 4 == 0) {
        const long R = 64L * a.V / a.nuz;
        const long units = a.O * (a.I / a.Nu) * (d.nu[0] / (R > 0 ? R : 1));
        if (R > 1 && d.nu[0] % R == 0 && (a.nuz / a.V) * R == 64 && units % 8 == 0) a.ug = (int)R;
    }
    // whether a wave-aligned block of 64 V inner elements can hold lanes of
    // both directions (shift signs); the inner index repeats with period Nu
    a.mix = 0;
    const long span = 64L * a.V;
    if (a.V != 4 || (a.I / a.V) % 64 != 0) {
        a.mix = 1;
    } else {
        for (long k0 = 0; k0 < a.Nu && !a.mix; k0 += span) {
            const long j_lo = (k0 / a.pst) % a.nshift;
            const long j_hi = ((k0 + span - 1) / a.pst) % a.nshift;
            const bool n_lo = a.shift[j_lo] < 0.0, n_hi = a.shift[j_hi] < 0.0;
            // within a block the index runs monotonically from j_lo to j_hi
            // (span divides Nu), and u_j, hence the shift, is monotone in j
            if (n_lo != n_hi || j_hi < j_lo) a.mix = 1;
        }
    }
    return VLASOV_OK;
}

int run_position(const vlasov_grid* g, const Dims& d, int axis, int prec, const void* fin,
                 const float* sin, void* fout, float* sout, double dt_over_a2, hipStream_t st)
{
    PosArgs a;
    const int rc = make_pos_args(g, d, axis, dt_over_a2, a);
    if (rc) return rc;
    return from_hip(launch_position(prec, fin, sin, fout, sout, a, st));
}

int make_vel_args(const vlasov_grid* g, const Dims& d, int axis, int vbc, const float* field,
                  double dt, double* outflow, VelArgs& a)
{
    if (!isfinite(dt)) return VLASOV_ERR_NONFINITE;
    const double du = 2.0 * g->umax[axis] / g->nu[axis];
    const double factor = dt / du;
    if (!isfinite(factor)) return VLASOV_ERR_NONFINITE;
    memset(&a, 0, sizeof(a));
    a.g = field + (long)axis * d.cells;
    a.factor = factor;
    a.M = (int)d.nu[axis];
    a.nuz = d.nu[2];
    a.periodic = vbc == VLASOV_VBC_PERIODIC;
    a.outflow = outflow;
    a.du3 = (2.0 * g->umax[0] / g->nu[0]) * (2.0 * g->umax[1] / g->nu[1]) *
            (2.0 * g->umax[2] / g->nu[2]);
    a.cells = d.cells;
    if (axis == 2) {
        a.I = 1;
        a.nsub = d.nu[0] * d.nu[1];
        a.V = 1;
        a.G = 1;
    } else {
        a.I = axis == 0 ? d.nu[1] * d.nu[2] : d.nu[2];
        a.nsub = axis == 0 ? 1 : d.nu[0];
        a.V = vector_width(d.nu[2]);
        a.G = (int)(d.nu[2] / a.V);
    }
    return VLASOV_OK;
}

int run_velocity(const vlasov_grid* g, const Dims& d, int axis, int prec, int vbc,
                 const void* fin, const float* sin, void* fout, float* sout, const float* field,
                 double dt, double* outflow, hipStream_t st)
{
    VelArgs a;
    const int rc = make_vel_args(g, d, axis, vbc, field, dt, outflow, a);
    if (rc) return rc;
    if (axis == 2) return from_hip(launch_vel_uz(prec, fin, sin, fout, sout, a, st));
    return from_hip(launch_vel_strided(prec, fin, sin, fout, sout, a, st));
}

size_t lds_limit()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 0;
    return (size_t)v;
}

// D_uz D_uy D_ux over dt with one field: fused in LDS where the velocity
// block fits, otherwise three single sweeps through `mid` buffers.
// Moments of f (arguments checked by the caller): rho, umean per cell, and the
// total mass when `mass` is given.
int run_moments(const vlasov_grid* g, const Dims& d, int prec, const void* f, const float* scale,
                double* rho, double* umean, double* mass, hipStream_t st, double* sigma = nullptr)
{
    MomArgs a;
    memset(&a, 0, sizeof(a));
    a.cells = d.cells;
    a.Nu = d.Nu;
    a.nuz = d.nu[2];
    a.du3 = 1.0;
    for (int k = 0; k < 3; ++k) {
        a.nu[k] = (int)d.nu[k];
        a.umin[k] = -g->umax[k];
        a.du[k] = 2.0 * g->umax[k] / g->nu[k];
        a.du3 *= a.du[k];
    }
    a.rho = rho;
    a.umean = umean;
    a.sigma = sigma;
    int rc = from_hip(launch_moments(prec, f, scale, a, st));
    if (rc || mass == nullptr) return rc;
    const double dx3 = (g->L[0] / g->n[0]) * (g->L[1] / g->n[1]) * (g->L[2] / g->n[2]);
    return from_hip(launch_sum(rho, d.cells, dx3, mass, st));
}

int run_kick(const vlasov_grid* g, const Dims& d, int prec, int vbc, const void* fin,
             const float* sin, void* fout, float* sout, void* midf, float* mids,
             const float* field, double dt, double* outflow, KickShift* shifts, hipStream_t st,
             double* rho = nullptr, double* umean = nullptr)
{
    if (!isfinite(dt)) return VLASOV_ERR_NONFINITE;
    int nu[3] = {(int)d.nu[0], (int)d.nu[1], (int)d.nu[2]};
    const bool yz64 = kick_yz64_supported(nu, lds_limit());
    if (kick_supported(nu, lds_limit()) || yz64) {
        KickArgs a;
        memset(&a, 0, sizeof(a));
        a.g = field;
        for (int k = 0; k < 3; ++k) {
            a.factor[k] = dt / (2.0 * g->umax[k] / g->nu[k]);
            if (!isfinite(a.factor[k])) return VLASOV_ERR_NONFINITE;
            a.nu[k] = nu[k];
        }
        a.periodic = vbc == VLASOV_VBC_PERIODIC;
        a.outflow = outflow;
        a.du3 = (2.0 * g->umax[0] / g->nu[0]) * (2.0 * g->umax[1] / g->nu[1]) *
                (2.0 * g->umax[2] / g->nu[2]);
        a.cells = d.cells;
        a.rho = rho;
        a.umean = umean;
        for (int k = 0; k < 3; ++k) {
            a.umin[k] = -g->umax[k];
            a.du[k] = 2.0 * g->umax[k] / g->nu[k];
        }
        if (!yz64) return from_hip(launch_kick(prec, fin, sin, fout, sout, a, shifts, st));
        // 64^3 blocks: ux on its own, then uy and uz fused on slabs of the
        // block (in place on the output when there is no middle buffer)
        void* mf = midf != nullptr ? midf : fout;
        float* ms = midf != nullptr ? mids : sout;
        int rc = run_velocity(g, d, 0, prec, vbc, fin, sin, mf, ms, field, dt, outflow, st);
        if (rc) return rc;
        rc = from_hip(launch_kick_yz64(prec, mf, ms, fout, sout, a, shifts, st));
        if (rc || rho == nullptr) return rc;
        return run_moments(g, d, prec, fout, sout, rho, umean, nullptr, st);
    }
    if (midf == nullptr) return VLASOV_ERR_WORKSPACE;
    int rc = run_velocity(g, d, 0, prec, vbc, fin, sin, fout, sout, field, dt, outflow, st);
    if (rc) return rc;
    rc = run_velocity(g, d, 1, prec, vbc, fout, sout, midf, mids, field, dt, outflow, st);
    if (rc) return rc;
    rc = run_velocity(g, d, 2, prec, vbc, midf, mids, fout, sout, field, dt, outflow, st);
    if (rc || rho == nullptr) return rc;
    return run_moments(g, d, prec, fout, sout, rho, umean, nullptr, st);
}

int advect_position(const vlasov_grid* g, int axis, int prec, const void* fin, const float* sin,
                    void* fout, float* sout, double dt_over_a2, void* stream)
{
    Dims d;
    if (g == nullptr) return VLASOV_ERR_NULL;
    if (!dims_of(g, d)) return VLASOV_ERR_SHAPE;
    const int rc = check_io(d, prec, fin, sin, fout, sout);
    if (rc) return rc;
    return run_position(g, d, axis, prec, fin, sin, fout, sout, dt_over_a2, (hipStream_t)stream);
}

int advect_velocity(const vlasov_grid* g, int axis, int prec, int vbc, const void* fin,
                    const float* sin, void* fout, float* sout, const float* field, double dt,
                    double* outflow, void* stream)
{
    Dims d;
    if (g == nullptr) return VLASOV_ERR_NULL;
    if (!dims_of(g, d)) return VLASOV_ERR_SHAPE;
    if (vbc != VLASOV_VBC_OUTFLOW && vbc != VLASOV_VBC_PERIODIC) return VLASOV_ERR_PREC;
    if (field == nullptr) return VLASOV_ERR_NULL;
    const int rc = check_io(d, prec, fin, sin, fout, sout);
    if (rc) return rc;
    const size_t fb = (size_t)d.total * elem_bytes(prec);
    if (overlap(fout, fb, field, 3 * d.cells * sizeof(float))) return VLASOV_ERR_ALIAS;
    if (outflow != nullptr && overlap(fout, fb, outflow, d.cells * sizeof(double)))
        return VLASOV_ERR_ALIAS;
    return run_velocity(g, d, axis, prec, vbc, fin, sin, fout, sout, field, dt, outflow,
                        (hipStream_t)stream);
}

}  // namespace

extern "C" {

int vlasov_abi_version(void) { return VLASOV_ABI_VERSION; }

const char* vlasov_strerror(int code)
{
    switch (code) {
        case VLASOV_OK: return "success";
        case VLASOV_ERR_NULL: return "a required pointer is NULL";
        case VLASOV_ERR_SHAPE: return "grid sizes, extents or alignment invalid or unsupported";
        case VLASOV_ERR_PREC: return "unknown precision or velocity boundary, or scale array missing";
        case VLASOV_ERR_ALIAS: return "an output overlaps an input";
        case VLASOV_ERR_NONFINITE: return "time step or shift factor is not finite";
        case VLASOV_ERR_DEVICE: return "HIP launch or runtime error";
        case VLASOV_ERR_WORKSPACE: return "workspace missing or too small";
        case VLASOV_ERR_TOO_LARGE: return "grid exceeds the fixed scratch of the allocation-free call";
        default: return "unknown error code";
    }
}

size_t vlasov_f_bytes(const vlasov_grid* grid, vlasov_prec prec)
{
    Dims d;
    if (!dims_of(grid, d) || !prec_ok(prec)) return 0;
    return (size_t)d.total * elem_bytes(prec);
}

size_t vlasov_scale_bytes(const vlasov_grid* grid, vlasov_prec prec)
{
    Dims d;
    if (!dims_of(grid, d) || !prec_ok(prec) || prec == VLASOV_F32) return 0;
    return (size_t)(d.total / d.nu[2]) * sizeof(float);
}

int vlasov_advect_x(const vlasov_grid* g, vlasov_prec p, const void* fin, const float* sin,
                    void* fout, float* sout, double dt_over_a2, void* stream)
{
    return advect_position(g, 0, p, fin, sin, fout, sout, dt_over_a2, stream);
}
int vlasov_advect_y(const vlasov_grid* g, vlasov_prec p, const void* fin, const float* sin,
                    void* fout, float* sout, double dt_over_a2, void* stream)
{
    return advect_position(g, 1, p, fin, sin, fout, sout, dt_over_a2, stream);
}
int vlasov_advect_z(const vlasov_grid* g, vlasov_prec p, const void* fin, const float* sin,
                    void* fout, float* sout, double dt_over_a2, void* stream)
{
    return advect_position(g, 2, p, fin, sin, fout, sout, dt_over_a2, stream);
}

int vlasov_advect_ux(const vlasov_grid* g, vlasov_prec p, vlasov_vbc vbc, const void* fin,
                     const float* sin, void* fout, float* sout, const float* field, double dt,
                     double* outflow, void* stream)
{
    return advect_velocity(g, 0, p, vbc, fin, sin, fout, sout, field, dt, outflow, stream);
}
int vlasov_advect_uy(const vlasov_grid* g, vlasov_prec p, vlasov_vbc vbc, const void* fin,
                     const float* sin, void* fout, float* sout, const float* field, double dt,
                     double* outflow, void* stream)
{
    return advect_velocity(g, 1, p, vbc, fin, sin, fout, sout, field, dt, outflow, stream);
}
int vlasov_advect_uz(const vlasov_grid* g, vlasov_prec p, vlasov_vbc vbc, const void* fin,
                     const float* sin, void* fout, float* sout, const float* field, double dt,
                     double* outflow, void* stream)
{
    return advect_velocity(g, 2, p, vbc, fin, sin, fout, sout, field, dt, outflow, stream);
}

// Step workspace: one copy of f, its scales, then the kick's shift table.
static size_t shift_table_offset(const Dims& d, int prec)
{
    size_t b = align_up((size_t)d.total * elem_bytes(prec));
    if (prec != VLASOV_F32) b += align_up((size_t)(d.total / d.nu[2]) * sizeof(float));
    return b;
}

size_t vlasov_step_workspace_bytes(const vlasov_grid* grid, vlasov_prec prec)
{
    Dims d;
    if (!dims_of(grid, d) || !prec_ok(prec)) return 0;
    return shift_table_offset(d, prec) + align_up((size_t)(3 * d.cells) * sizeof(KickShift));
}

static int step_impl(const vlasov_grid* g, vlasov_prec prec, vlasov_vbc vbc, const void* fin,
                     const float* sin, void* fout, float* sout, const float* g_n,
                     const float* g_np1, double dt, double a2inv, void* work, size_t work_bytes,
                     double* outflow, double* rho, double* umean, void* stream)
{
    Dims d;
    if (g == nullptr) return VLASOV_ERR_NULL;
    if (!dims_of(g, d)) return VLASOV_ERR_SHAPE;
    if (vbc != VLASOV_VBC_OUTFLOW && vbc != VLASOV_VBC_PERIODIC) return VLASOV_ERR_PREC;
    if (g_n == nullptr || g_np1 == nullptr) return VLASOV_ERR_NULL;
    int rc = check_io(d, prec, fin, sin, fout, sout);
    if (rc) return rc;
    if (!isfinite(dt) || !isfinite(a2inv) || !isfinite(dt * a2inv)) return VLASOV_ERR_NONFINITE;
    for (int a = 0; a < 3; ++a)
        if (d.nu[a] > kMaxShiftTable) return VLASOV_ERR_SHAPE;
    const size_t need = vlasov_step_workspace_bytes(g, prec);
    if (work == nullptr || work_bytes < need) return VLASOV_ERR_WORKSPACE;
    const size_t fb = (size_t)d.total * elem_bytes(prec);
    const size_t sb = prec == VLASOV_F32 ? 0 : (size_t)(d.total / d.nu[2]) * sizeof(float);
    void* wf = work;
    float* ws = prec == VLASOV_F32 ? nullptr : (float*)((char*)work + align_up(fb));
    if (overlap(work, need, fin, fb) || overlap(work, need, fout, fb) ||
        overlap(work, need, sin, sb) || overlap(work, need, sout, sb))
        return VLASOV_ERR_ALIAS;
    if (overlap(fout, fb, g_n, 3 * d.cells * sizeof(float)) ||
        overlap(fout, fb, g_np1, 3 * d.cells * sizeof(float)))
        return VLASOV_ERR_ALIAS;
    hipStream_t st = (hipStream_t)stream;
    KickShift* tab = (KickShift*)((char*)work + shift_table_offset(d, prec));
    const double h = 0.5 * dt;
    const double dta = dt * a2inv;
    // Eq. (5) right to left: kick(g_n) -> z -> y -> x -> kick(g_np1).
    // Buffers: in -> out (kick) -> work (z) -> out (y) -> work (x) -> out (kick);
    // a kick that cannot run fused uses the other buffer as its middle stage.
    if ((rc = run_kick(g, d, prec, vbc, fin, sin, fout, sout, wf, ws, g_n, h, outflow, tab, st)))
        return rc;
    if ((rc = run_position(g, d, 2, prec, fout, sout, wf, ws, dta, st))) return rc;
    if ((rc = run_position(g, d, 1, prec, wf, ws, fout, sout, dta, st))) return rc;
    if ((rc = run_position(g, d, 0, prec, fout, sout, wf, ws, dta, st))) return rc;
    if ((rc = run_kick(g, d, prec, vbc, wf, ws, fout, sout, nullptr, nullptr, g_np1, h, outflow,
                       tab, st, rho, umean)) == VLASOV_ERR_WORKSPACE) {
        // unfused last kick: x result is in work; go work -> out -> work -> out
        if ((rc = run_velocity(g, d, 0, prec, vbc, wf, ws, fout, sout, g_np1, h, outflow, st)))
            return rc;
        if ((rc = run_velocity(g, d, 1, prec, vbc, fout, sout, wf, ws, g_np1, h, outflow, st)))
            return rc;
        rc = run_velocity(g, d, 2, prec, vbc, wf, ws, fout, sout, g_np1, h, outflow, st);
        if (rc == VLASOV_OK && rho != nullptr)
            rc = run_moments(g, d, prec, fout, sout, rho, umean, nullptr, st);
    }
    return rc;
}

int vlasov_step(const vlasov_grid* g, vlasov_prec prec, vlasov_vbc vbc, const void* fin,
                const float* sin, void* fout, float* sout, const float* g_n, const float* g_np1,
                double dt, double a2inv, void* work, size_t work_bytes, double* outflow,
                void* stream)
{
    return step_impl(g, prec, vbc, fin, sin, fout, sout, g_n, g_np1, dt, a2inv, work, work_bytes,
                     outflow, nullptr, nullptr, stream);
}

int vlasov_step_moments(const vlasov_grid* g, vlasov_prec prec, vlasov_vbc vbc, const void* fin,
                        const float* sin, void* fout, float* sout, const float* g_n,
                        const float* g_np1, double dt, double a2inv, void* work,
                        size_t work_bytes, double* outflow, double* rho, double* umean,
                        void* stream)
{
    Dims d;
    if (g == nullptr) return VLASOV_ERR_NULL;
    if (!dims_of(g, d)) return VLASOV_ERR_SHAPE;
    if (rho == nullptr) return VLASOV_ERR_NULL;
    const size_t nb = (size_t)d.cells * sizeof(double);
    if (umean != nullptr && overlap(rho, nb, umean, 3 * nb)) return VLASOV_ERR_ALIAS;
    const size_t fb = (size_t)d.total * elem_bytes(prec);
    if (overlap(fout, fb, rho, nb) || overlap(fout, fb, umean, 3 * nb) ||
        overlap(fin, fb, rho, nb) || overlap(fin, fb, umean, 3 * nb) ||
        overlap(work, work_bytes, rho, nb) || overlap(work, work_bytes, umean, 3 * nb))
        return VLASOV_ERR_ALIAS;
    return step_impl(g, prec, vbc, fin, sin, fout, sout, g_n, g_np1, dt, a2inv, work, work_bytes,
                     outflow, rho, umean, stream);
}

size_t vlasov_steps_workspace_bytes(const vlasov_grid* grid, vlasov_prec prec)
{
    Dims d;
    if (!dims_of(grid, d) || !prec_ok(prec)) return 0;
    return 2 * shift_table_offset(d, prec) + align_up((size_t)(3 * d.cells) * sizeof(KickShift));
}

int vlasov_steps(const vlasov_grid* g, vlasov_prec prec, vlasov_vbc vbc, const void* fin,
                 const float* sin, void* fout, float* sout, const float* fields, int nsteps,
                 double dt, const double* a2inv, void* work, size_t work_bytes, double* outflow,
                 void* stream)
{
    Dims d;
    if (g == nullptr) return VLASOV_ERR_NULL;
    if (!dims_of(g, d)) return VLASOV_ERR_SHAPE;
    if (vbc != VLASOV_VBC_OUTFLOW && vbc != VLASOV_VBC_PERIODIC) return VLASOV_ERR_PREC;
    if (fields == nullptr) return VLASOV_ERR_NULL;
    if (nsteps < 1) return VLASOV_ERR_SHAPE;
    int rc = check_io(d, prec, fin, sin, fout, sout);
    if (rc) return rc;
    if (!isfinite(dt)) return VLASOV_ERR_NONFINITE;
    for (int k = 0; k < nsteps; ++k) {
        const double a = a2inv != nullptr ? a2inv[k] : 1.0;
        if (!isfinite(a) || !isfinite(dt * a)) return VLASOV_ERR_NONFINITE;
    }
    for (int a = 0; a < 3; ++a)
        if (d.nu[a] > kMaxShiftTable) return VLASOV_ERR_SHAPE;
    const size_t need = vlasov_steps_workspace_bytes(g, prec);
    if (work == nullptr || work_bytes < need) return VLASOV_ERR_WORKSPACE;
    const size_t fb = (size_t)d.total * elem_bytes(prec);
    const size_t sb = prec == VLASOV_F32 ? 0 : (size_t)(d.total / d.nu[2]) * sizeof(float);
    const size_t gb = (size_t)(nsteps + 1) * 3 * d.cells * sizeof(float);
    if (overlap(work, need, fin, fb) || overlap(work, need, fout, fb) ||
        overlap(work, need, sin, sb) || overlap(work, need, sout, sb) ||
        overlap(work, need, fields, gb) || overlap(fout, fb, fields, gb))
        return VLASOV_ERR_ALIAS;
    // two intermediate copies: the drifts ping-pong between f_out and the
    // first; a kick that cannot run fused uses the second as its middle stage
    const size_t one = shift_table_offset(d, prec);
    void* w1 = work;
    float* s1 = prec == VLASOV_F32 ? nullptr : (float*)((char*)w1 + align_up(fb));
    void* w2 = (char*)work + one;
    float* s2 = prec == VLASOV_F32 ? nullptr : (float*)((char*)w2 + align_up(fb));
    KickShift* tab = (KickShift*)((char*)work + 2 * one);
    hipStream_t st = (hipStream_t)stream;
    const size_t gstride = (size_t)3 * d.cells;
    // K(dt/2; g_0), then per step: z, y, x over dt a^-2 and the merged kick
    // K(dt; g_{k+1}) (K(dt/2; g_n) after the last step)
    if ((rc = run_kick(g, d, prec, vbc, fin, sin, fout, sout, w1, s1, fields, 0.5 * dt, outflow,
                       tab, st)))
        return rc;
    for (int k = 0; k < nsteps; ++k) {
        const double dta = dt * (a2inv != nullptr ? a2inv[k] : 1.0);
        if ((rc = run_position(g, d, 2, prec, fout, sout, w1, s1, dta, st))) return rc;
        if ((rc = run_position(g, d, 1, prec, w1, s1, fout, sout, dta, st))) return rc;
        if ((rc = run_position(g, d, 0, prec, fout, sout, w1, s1, dta, st))) return rc;
        const double h = k + 1 < nsteps ? dt : 0.5 * dt;
        if ((rc = run_kick(g, d, prec, vbc, w1, s1, fout, sout, w2, s2,
                           fields + (size_t)(k + 1) * gstride, h, outflow, tab, st)))
            return rc;
    }
    return VLASOV_OK;
}

int vlasov_kick(const vlasov_grid* g, vlasov_prec prec, vlasov_vbc vbc, const void* fin,
                const float* sin, void* fout, float* sout, const float* field, double dt,
                void* work, size_t work_bytes, double* outflow, void* stream)
{
    Dims d;
    if (g == nullptr) return VLASOV_ERR_NULL;
    if (!dims_of(g, d)) return VLASOV_ERR_SHAPE;
    if (vbc != VLASOV_VBC_OUTFLOW && vbc != VLASOV_VBC_PERIODIC) return VLASOV_ERR_PREC;
    if (field == nullptr) return VLASOV_ERR_NULL;
    int rc = check_io(d, prec, fin, sin, fout, sout);
    if (rc) return rc;
    const size_t fb = (size_t)d.total * elem_bytes(prec);
    if (overlap(fout, fb, field, 3 * d.cells * sizeof(float))) return VLASOV_ERR_ALIAS;
    if (outflow != nullptr && overlap(fout, fb, outflow, d.cells * sizeof(double)))
        return VLASOV_ERR_ALIAS;
    void* wf = nullptr;
    float* ws = nullptr;
    KickShift* tab = nullptr;
    int nu[3] = {(int)d.nu[0], (int)d.nu[1], (int)d.nu[2]};
    const bool fused = kick_supported(nu, lds_limit());
    const size_t need = vlasov_step_workspace_bytes(g, prec);
    // fused shapes run without a workspace (then every work-group splits its
    // own shifts); with one they precompute the shift table into it
    if (!fused && (work == nullptr || work_bytes < need)) return VLASOV_ERR_WORKSPACE;
    if (work != nullptr && work_bytes >= need) {
        const size_t sb = prec == VLASOV_F32 ? 0 : (size_t)(d.total / d.nu[2]) * sizeof(float);
        if (overlap(work, need, fin, fb) || overlap(work, need, fout, fb) ||
            overlap(work, need, sin, sb) || overlap(work, need, sout, sb) ||
            overlap(work, need, field, 3 * d.cells * sizeof(float)) ||
            (outflow != nullptr && overlap(work, need, outflow, d.cells * sizeof(double))))
            return VLASOV_ERR_ALIAS;
        wf = work;
        ws = prec == VLASOV_F32 ? nullptr : (float*)((char*)work + align_up(fb));
        tab = (KickShift*)((char*)work + shift_table_offset(d, prec));
    }
    return run_kick(g, d, prec, vbc, fin, sin, fout, sout, wf, ws, field, dt, outflow, tab,
                    (hipStream_t)stream);
}

int vlasov_moments(const vlasov_grid* g, vlasov_prec prec, const void* f, const float* scale,
                   double* rho, double* umean, double* mass, void* stream)
{
    Dims d;
    if (g == nullptr) return VLASOV_ERR_NULL;
    if (!dims_of(g, d)) return VLASOV_ERR_SHAPE;
    if (!prec_ok(prec)) return VLASOV_ERR_PREC;
    if (f == nullptr || rho == nullptr) return VLASOV_ERR_NULL;
    if (!aligned16(f)) return VLASOV_ERR_SHAPE;
    if (prec != VLASOV_F32) {
        if (scale == nullptr) return VLASOV_ERR_PREC;
        if (!scaled_shape_ok(d)) return VLASOV_ERR_SHAPE;
    }
    const size_t nb = (size_t)d.cells * sizeof(double);
    if (umean != nullptr && overlap(rho, nb, umean, 3 * nb)) return VLASOV_ERR_ALIAS;
    if (mass != nullptr && (overlap(mass, 8, rho, nb) || overlap(mass, 8, umean, 3 * nb)))
        return VLASOV_ERR_ALIAS;
    return run_moments(g, d, prec, f, scale, rho, umean, mass, (hipStream_t)stream);
}

int vlasov_dispersion(const vlasov_grid* g, vlasov_prec prec, const void* f, const float* scale,
                      double* rho, double* umean, double* sigma, void* stream)
{
    Dims d;
    if (g == nullptr) return VLASOV_ERR_NULL;
    if (!dims_of(g, d)) return VLASOV_ERR_SHAPE;
    if (!prec_ok(prec)) return VLASOV_ERR_PREC;
    if (f == nullptr || rho == nullptr || sigma == nullptr) return VLASOV_ERR_NULL;
    if (!aligned16(f)) return VLASOV_ERR_SHAPE;
    if (prec != VLASOV_F32) {
        if (scale == nullptr) return VLASOV_ERR_PREC;
        if (!scaled_shape_ok(d)) return VLASOV_ERR_SHAPE;
    }
    const size_t nb = (size_t)d.cells * sizeof(double);
    if (overlap(rho, nb, sigma, 6 * nb) || overlap(umean, 3 * nb, rho, nb) ||
        overlap(umean, 3 * nb, sigma, 6 * nb))
        return VLASOV_ERR_ALIAS;
    return run_moments(g, d, prec, f, scale, rho, umean, nullptr, (hipStream_t)stream, sigma);
}

size_t vlasov_step_sc_workspace_bytes(const vlasov_grid* grid, vlasov_prec prec)
{
    Dims d;
    if (!dims_of(grid, d) || !prec_ok(prec)) return 0;
    const int n[3] = {(int)d.n[0], (int)d.n[1], (int)d.n[2]};
    return align_up(vlasov_step_workspace_bytes(grid, prec)) + field_workspace_bytes(n);
}

int vlasov_step_sc(const vlasov_grid* g, vlasov_prec prec, vlasov_vbc vbc, const void* fin,
                   const float* sin, void* fout, float* sout, const float* g_n, float* g_np1,
                   double* rho_np1, double coupling, double dt, double a2inv, void* work,
                   size_t work_bytes, double* outflow, void* stream)
{
    Dims d;
    if (g == nullptr) return VLASOV_ERR_NULL;
    if (!dims_of(g, d)) return VLASOV_ERR_SHAPE;
    if (vbc != VLASOV_VBC_OUTFLOW && vbc != VLASOV_VBC_PERIODIC) return VLASOV_ERR_PREC;
    if (g_n == nullptr || g_np1 == nullptr || rho_np1 == nullptr) return VLASOV_ERR_NULL;
    int rc = check_io(d, prec, fin, sin, fout, sout);
    if (rc) return rc;
    if (!isfinite(dt) || !isfinite(a2inv) || !isfinite(dt * a2inv) || !isfinite(coupling))
        return VLASOV_ERR_NONFINITE;
    for (int a = 0; a < 3; ++a) {
        if (d.nu[a] > kMaxShiftTable) return VLASOV_ERR_SHAPE;
        if (!(g->L[a] > 0.0) || !isfinite(g->L[a])) return VLASOV_ERR_SHAPE;
    }
    const size_t need = vlasov_step_sc_workspace_bytes(g, prec);
    if (work == nullptr || work_bytes < need) return VLASOV_ERR_WORKSPACE;
    const size_t fb = (size_t)d.total * elem_bytes(prec);
    const size_t sb = prec == VLASOV_F32 ? 0 : (size_t)(d.total / d.nu[2]) * sizeof(float);
    const size_t gb = 3 * (size_t)d.cells * sizeof(float);
    const size_t rb = (size_t)d.cells * sizeof(double);
    if (overlap(work, need, fin, fb) || overlap(work, need, fout, fb) ||
        overlap(work, need, sin, sb) || overlap(work, need, sout, sb) ||
        overlap(work, need, g_n, gb) || overlap(work, need, g_np1, gb) ||
        overlap(work, need, rho_np1, rb) || overlap(fout, fb, g_n, gb) ||
        overlap(fout, fb, g_np1, gb) || overlap(fout, fb, rho_np1, rb) ||
        overlap(g_np1, gb, g_n, gb) || overlap(g_np1, gb, rho_np1, rb) ||
        overlap(fin, fb, g_np1, gb) || overlap(fin, fb, rho_np1, rb))
        return VLASOV_ERR_ALIAS;
    hipStream_t st = (hipStream_t)stream;
    void* wf = work;
    float* ws = prec == VLASOV_F32 ? nullptr : (float*)((char*)work + align_up(fb));
    KickShift* tab = (KickShift*)((char*)work + shift_table_offset(d, prec));
    void* fwork = (char*)work + align_up(vlasov_step_workspace_bytes(g, prec));
    const double h = 0.5 * dt;
    const double dta = dt * a2inv;
    // kick(g_n) -> z -> y -> x; the kicks leave the density alone, so the
    // drifted f has the density of f^{n+1}: its field drives the last kick
    if ((rc = run_kick(g, d, prec, vbc, fin, sin, fout, sout, wf, ws, g_n, h, outflow, tab, st)))
        return rc;
    if ((rc = run_position(g, d, 2, prec, fout, sout, wf, ws, dta, st))) return rc;
    if ((rc = run_position(g, d, 1, prec, wf, ws, fout, sout, dta, st))) return rc;
    if ((rc = run_position(g, d, 0, prec, fout, sout, wf, ws, dta, st))) return rc;
    if ((rc = run_moments(g, d, prec, wf, ws, rho_np1, nullptr, nullptr, st))) return rc;
    FieldArgs fa;
    memset(&fa, 0, sizeof(fa));
    for (int k = 0; k < 3; ++k) {
        fa.n[k] = (int)d.n[k];
        fa.L[k] = g->L[k];
    }
    fa.coupling = coupling;
    fa.cells = d.cells;
    if ((rc = from_hip(launch_field(rho_np1, g_np1, fa, fwork, st)))) return rc;
    if ((rc = run_kick(g, d, prec, vbc, wf, ws, fout, sout, nullptr, nullptr, g_np1, h, outflow,
                       tab, st)) == VLASOV_ERR_WORKSPACE) {
        if ((rc = run_velocity(g, d, 0, prec, vbc, wf, ws, fout, sout, g_np1, h, outflow, st)))
            return rc;
        if ((rc = run_velocity(g, d, 1, prec, vbc, fout, sout, wf, ws, g_np1, h, outflow, st)))
            return rc;
        rc = run_velocity(g, d, 2, prec, vbc, wf, ws, fout, sout, g_np1, h, outflow, st);
    }
    return rc;
}

size_t vlasov_field_workspace_bytes(const vlasov_grid* grid)
{
    Dims d;
    if (!dims_of(grid, d)) return 0;
    const int n[3] = {(int)d.n[0], (int)d.n[1], (int)d.n[2]};
    return field_workspace_bytes(n);
}

int vlasov_field(const vlasov_grid* g, const double* rho, double coupling, float* field,
                 void* work, size_t work_bytes, void* stream)
{
    Dims d;
    if (g == nullptr) return VLASOV_ERR_NULL;
    if (!dims_of(g, d)) return VLASOV_ERR_SHAPE;
    if (rho == nullptr || field == nullptr) return VLASOV_ERR_NULL;
    if (!isfinite(coupling)) return VLASOV_ERR_NONFINITE;
    for (int a = 0; a < 3; ++a)
        if (!(g->L[a] > 0.0) || !isfinite(g->L[a])) return VLASOV_ERR_SHAPE;
    const size_t need = vlasov_field_workspace_bytes(g);
    if (work == nullptr || work_bytes < need) return VLASOV_ERR_WORKSPACE;
    const size_t nb = (size_t)d.cells * sizeof(double);
    const size_t fb = 3 * (size_t)d.cells * sizeof(float);
    if (overlap(work, need, rho, nb) || overlap(work, need, field, fb) ||
        overlap(rho, nb, field, fb))
        return VLASOV_ERR_ALIAS;
    FieldArgs a;
    memset(&a, 0, sizeof(a));
    for (int k = 0; k < 3; ++k) {
        a.n[k] = (int)d.n[k];
        a.L[k] = g->L[k];
    }
    a.coupling = coupling;
    a.cells = d.cells;
    return from_hip(launch_field(rho, field, a, work, (hipStream_t)stream));
}

// ---------------------------------------------------------------------------
// Tangents and adjoints (FP32 storage)
// ---------------------------------------------------------------------------
static int check_adj_io(const vlasov_grid* g, Dims& d, const void* a, const void* b, const void* out)
{
    if (g == nullptr) return VLASOV_ERR_NULL;
    if (!dims_of(g, d)) return VLASOV_ERR_SHAPE;
    if (a == nullptr || b == nullptr || out == nullptr) return VLASOV_ERR_NULL;
    const size_t fb = (size_t)d.total * sizeof(float);
    if (overlap(out, fb, a, fb) || overlap(out, fb, b, fb)) return VLASOV_ERR_ALIAS;
    return VLASOV_OK;
}

static int position_tan(const vlasov_grid* g, int axis, const float* f, const float* v,
                        float* out, double dta, void* stream)
{
    Dims d;
    int rc = check_adj_io(g, d, f, v, out);
    if (rc) return rc;
    PosArgs a;
    if ((rc = make_pos_args(g, d, axis, dta, a))) return rc;
    return from_hip(launch_position_tan(f, v, out, a, (hipStream_t)stream));
}

static int position_adj(const vlasov_grid* g, int axis, const float* f, const float* lam,
                        float* lam_in, double dta, void* stream)
{
    Dims d;
    int rc = check_adj_io(g, d, f, lam, lam_in);
    if (rc) return rc;
    PosArgs a;
    if ((rc = make_pos_args(g, d, axis, dta, a))) return rc;
    return from_hip(launch_position_adj(f, lam, lam_in, a, (hipStream_t)stream));
}

static int velocity_tan(const vlasov_grid* g, int axis, int vbc, const float* f,
                        const float* field, const float* g_dot, double dt, const float* v,
                        float* out, void* stream)
{
    Dims d;
    int rc = check_adj_io(g, d, f, v, out);
    if (rc) return rc;
    if (vbc != VLASOV_VBC_OUTFLOW && vbc != VLASOV_VBC_PERIODIC) return VLASOV_ERR_PREC;
    if (field == nullptr) return VLASOV_ERR_NULL;
    VelArgs a;
    if ((rc = make_vel_args(g, d, axis, vbc, field, dt, nullptr, a))) return rc;
    const float* gd = g_dot != nullptr ? g_dot + (long)axis * d.cells : nullptr;
    return from_hip(launch_velocity_tan(f, v, out, gd, a, (hipStream_t)stream));
}

static int velocity_adj(const vlasov_grid* g, int axis, int vbc, const float* f,
                        const float* field, double dt, const float* lam, float* lam_in,
                        float* lam_g, void* stream)
{
    Dims d;
    int rc = check_adj_io(g, d, f, lam, lam_in);
    if (rc) return rc;
    if (vbc != VLASOV_VBC_OUTFLOW && vbc != VLASOV_VBC_PERIODIC) return VLASOV_ERR_PREC;
    if (field == nullptr) return VLASOV_ERR_NULL;
    if (lam_g != nullptr && overlap(lam_in, (size_t)d.total * 4, lam_g, 3 * d.cells * 4))
        return VLASOV_ERR_ALIAS;
    VelArgs a;
    if ((rc = make_vel_args(g, d, axis, vbc, field, dt, nullptr, a))) return rc;
    float* lg = lam_g != nullptr ? lam_g + (long)axis * d.cells : nullptr;
    return from_hip(launch_velocity_adj(f, lam, lam_in, lg, a, (hipStream_t)stream));
}

#define VL_POS_DERIV(ax, idx)                                                                  \
    int vlasov_advect_##ax##_tan(const vlasov_grid* g, const float* f_in, const float* v_in,    \
                                 float* v_out, double dt_over_a2, void* stream)                 \
    {                                                                                          \
        return position_tan(g, idx, f_in, v_in, v_out, dt_over_a2, stream);                     \
    }                                                                                          \
    int vlasov_advect_##ax##_adj(const vlasov_grid* g, const float* f_in, const float* lam_out, \
                                 float* lam_in, double dt_over_a2, void* stream)                \
    {                                                                                          \
        return position_adj(g, idx, f_in, lam_out, lam_in, dt_over_a2, stream);                 \
    }
VL_POS_DERIV(x, 0)
VL_POS_DERIV(y, 1)
VL_POS_DERIV(z, 2)
#undef VL_POS_DERIV

#define VL_VEL_DERIV(ax, idx)                                                                   \
    int vlasov_advect_u##ax##_tan(const vlasov_grid* g, vlasov_vbc vbc, const float* f_in,       \
                                  const float* field, const float* g_dot, double dt,             \
                                  const float* v_in, float* v_out, void* stream)                 \
    {                                                                                           \
        return velocity_tan(g, idx, vbc, f_in, field, g_dot, dt, v_in, v_out, stream);           \
    }                                                                                           \
    int vlasov_advect_u##ax##_adj(const vlasov_grid* g, vlasov_vbc vbc, const float* f_in,       \
                                  const float* field, double dt, const float* lam_out,           \
                                  float* lam_in, float* lam_g, void* stream)                     \
    {                                                                                           \
        return velocity_adj(g, idx, vbc, f_in, field, dt, lam_out, lam_in, lam_g, stream);       \
    }
VL_VEL_DERIV(x, 0)
VL_VEL_DERIV(y, 1)
VL_VEL_DERIV(z, 2)
#undef VL_VEL_DERIV

size_t vlasov_step_adj_workspace_bytes(const vlasov_grid* grid)
{
    Dims d;
    if (!dims_of(grid, d)) return 0;
    return 9 * align_up((size_t)d.total * sizeof(float));
}

int vlasov_step_adj(const vlasov_grid* g, vlasov_vbc vbc, const float* fin, const float* g_n,
                    const float* g_np1, double dt, double a2inv, const float* lam_out,
                    float* lam_in, float* lam_g_n, float* lam_g_np1, void* work,
                    size_t work_bytes, void* stream)
{
    Dims d;
    int rc = check_adj_io(g, d, fin, lam_out, lam_in);
    if (rc) return rc;
    if (vbc != VLASOV_VBC_OUTFLOW && vbc != VLASOV_VBC_PERIODIC) return VLASOV_ERR_PREC;
    if (g_n == nullptr || g_np1 == nullptr) return VLASOV_ERR_NULL;
    if (!isfinite(dt) || !isfinite(a2inv) || !isfinite(dt * a2inv)) return VLASOV_ERR_NONFINITE;
    const size_t need = vlasov_step_adj_workspace_bytes(g);
    if (work == nullptr || work_bytes < need) return VLASOV_ERR_WORKSPACE;
    const size_t fb = (size_t)d.total * sizeof(float);
    if (overlap(work, need, fin, fb) || overlap(work, need, lam_out, fb) ||
        overlap(work, need, lam_in, fb))
        return VLASOV_ERR_ALIAS;
    hipStream_t st = (hipStream_t)stream;
    const size_t slot = align_up(fb);
    float* stage[9];
    stage[0] = const_cast<float*>(fin);
    for (int k = 1; k < 9; ++k) stage[k] = (float*)((char*)work + (k - 1) * slot);
    float* lw = (float*)((char*)work + 8 * slot);
    const double h = 0.5 * dt, dta = dt * a2inv;
    // forward stages: stage[k] is the input of sweep k of Eq. (5)
    if ((rc = run_velocity(g, d, 0, VLASOV_F32, vbc, stage[0], nullptr, stage[1], nullptr, g_n, h, nullptr, st))) return rc;
    if ((rc = run_velocity(g, d, 1, VLASOV_F32, vbc, stage[1], nullptr, stage[2], nullptr, g_n, h, nullptr, st))) return rc;
    if ((rc = run_velocity(g, d, 2, VLASOV_F32, vbc, stage[2], nullptr, stage[3], nullptr, g_n, h, nullptr, st))) return rc;
    if ((rc = run_position(g, d, 2, VLASOV_F32, stage[3], nullptr, stage[4], nullptr, dta, st))) return rc;
    if ((rc = run_position(g, d, 1, VLASOV_F32, stage[4], nullptr, stage[5], nullptr, dta, st))) return rc;
    if ((rc = run_position(g, d, 0, VLASOV_F32, stage[5], nullptr, stage[6], nullptr, dta, st))) return rc;
    if ((rc = run_velocity(g, d, 0, VLASOV_F32, vbc, stage[6], nullptr, stage[7], nullptr, g_np1, h, nullptr, st))) return rc;
    if ((rc = run_velocity(g, d, 1, VLASOV_F32, vbc, stage[7], nullptr, stage[8], nullptr, g_np1, h, nullptr, st))) return rc;
    // reverse: lam_out -> lam_in -> lw -> lam_in -> ... -> lam_in (nine transposed sweeps)
    const float* src = lam_out;
    float* bufs[2] = {lam_in, lw};
    int b = 0;
    auto vadj = [&](int axis, int k, const float* field, float* lg) {
        const int r = velocity_adj(g, axis, vbc, stage[k], field, h, src, bufs[b], lg, stream);
        src = bufs[b];
        b ^= 1;
        return r;
    };
    auto padj = [&](int axis, int k) {
        const int r = position_adj(g, axis, stage[k], src, bufs[b], dta, stream);
        src = bufs[b];
        b ^= 1;
        return r;
    };
    if ((rc = vadj(2, 8, g_np1, lam_g_np1))) return rc;
    if ((rc = vadj(1, 7, g_np1, lam_g_np1))) return rc;
    if ((rc = vadj(0, 6, g_np1, lam_g_np1))) return rc;
    if ((rc = padj(0, 5))) return rc;
    if ((rc = padj(1, 4))) return rc;
    if ((rc = padj(2, 3))) return rc;
    if ((rc = vadj(2, 2, g_n, lam_g_n))) return rc;
    if ((rc = vadj(1, 1, g_n, lam_g_n))) return rc;
    return vadj(0, 0, g_n, lam_g_n);
}

int vlasov_moments_adj(const vlasov_grid* g, const double* rho, const double* umean,
                       const double* lam_rho, const double* lam_umean, float* lam_f,
                       void* stream)
{
    Dims d;
    if (g == nullptr) return VLASOV_ERR_NULL;
    if (!dims_of(g, d)) return VLASOV_ERR_SHAPE;
    if (lam_f == nullptr || lam_rho == nullptr) return VLASOV_ERR_NULL;
    if (lam_umean != nullptr && (rho == nullptr || umean == nullptr)) return VLASOV_ERR_NULL;
    MomArgs a;
    memset(&a, 0, sizeof(a));
    a.cells = d.cells;
    a.Nu = d.Nu;
    a.nuz = d.nu[2];
    a.du3 = 1.0;
    for (int k = 0; k < 3; ++k) {
        a.nu[k] = (int)d.nu[k];
        a.umin[k] = -g->umax[k];
        a.du[k] = 2.0 * g->umax[k] / g->nu[k];
        a.du3 *= a.du[k];
    }
    a.rho = const_cast<double*>(rho);
    a.umean = const_cast<double*>(umean);
    return from_hip(launch_moments_adj(a, lam_rho, lam_umean, lam_f, (hipStream_t)stream));
}

static int codec_args(const vlasov_grid* g, vlasov_prec prec, const void* f32, const void* codes,
                      const void* scale, Dims& d)
{
    if (g == nullptr || f32 == nullptr || codes == nullptr) return VLASOV_ERR_NULL;
    if (!dims_of(g, d)) return VLASOV_ERR_SHAPE;
    if (!prec_ok(prec)) return VLASOV_ERR_PREC;
    if (!aligned16(f32) || !aligned16(codes)) return VLASOV_ERR_SHAPE;
    const size_t fb = (size_t)d.total * 4, cb = (size_t)d.total * elem_bytes(prec);
    if (overlap(f32, fb, codes, cb)) return VLASOV_ERR_ALIAS;
    if (prec == VLASOV_F32) return VLASOV_OK;
    if (scale == nullptr) return VLASOV_ERR_PREC;
    if (!scaled_shape_ok(d)) return VLASOV_ERR_SHAPE;
    const size_t sb = (size_t)(d.total / d.nu[2]) * sizeof(float);
    if (overlap(scale, sb, f32, fb) || overlap(scale, sb, codes, cb)) return VLASOV_ERR_ALIAS;
    return VLASOV_OK;
}

int vlasov_encode(const vlasov_grid* g, vlasov_prec prec, const float* f32, void* codes,
                  float* scale, void* stream)
{
    Dims d;
    const int rc = codec_args(g, prec, f32, codes, scale, d);
    if (rc) return rc;
    if (prec == VLASOV_F32)
        return from_hip(hipMemcpyAsync(codes, f32, (size_t)d.total * 4, hipMemcpyDeviceToDevice,
                                       (hipStream_t)stream));
    return from_hip(launch_encode(prec, f32, codes, scale, d.total, d.nu[2], (hipStream_t)stream));
}

int vlasov_decode(const vlasov_grid* g, vlasov_prec prec, const void* codes, const float* scale,
                  float* f32, void* stream)
{
    Dims d;
    const int rc = codec_args(g, prec, f32, codes, scale, d);
    if (rc) return rc;
    if (prec == VLASOV_F32)
        return from_hip(hipMemcpyAsync(f32, codes, (size_t)d.total * 4, hipMemcpyDeviceToDevice,
                                       (hipStream_t)stream));
    return from_hip(launch_decode(prec, codes, scale, f32, d.total, d.nu[2], (hipStream_t)stream));
}

int vlasov_sum_f64(const double* x, int64_t n, double* out, void* stream)
{
    if (x == nullptr || out == nullptr) return VLASOV_ERR_NULL;
    if (n < 0) return VLASOV_ERR_SHAPE;
    if (overlap(out, 8, x, (size_t)n * 8)) return VLASOV_ERR_ALIAS;
    return from_hip(launch_sum(x, n, 1.0, out, (hipStream_t)stream));
}

}  // extern "C"
