// Tangent-linear and adjoint sweeps (FP32 storage only).
//
// With the limiter's selections frozen at the forward input, one sweep of a
// line is a linear map of the cell values, f' = J f, and a smooth function of
// the fractional shift nu (through the semi-Lagrangian weights and the
// factor mu of the flux).  Each interface flux is linearised as
//   Phi = sum_k W_k f_{j+k} (upwind frame, k = -2..2),  dPhi/dmu,
// by re-running the forward arithmetic of flux_mag on the forward input with
// the same FP32 operations, so every selection (early-out, curvature
// minmods, bounds, median, positivity clamp) is the forward's own, and then
// reading off which candidate each selection returned.  Ties between equal
// candidates are resolved as in the FP64 oracle: min and max keep their first
// argument, the median is max(min(x,y), min(max(x,y),z)).
//
//  tangent: out_dot_i = v_{i-N} - (Phi_dot_{j+1/2} - Phi_dot_{j-1/2}), j = i-N,
//           Phi_dot = W . v + dPhi/dmu * mu_dot
//  adjoint: lam_in_r = lam_{r+N} + sum_{k} psi_{r-k} W_{r-k}[k],
//           psi_j = lam_{j+N+1} - lam_{j+N}, lam_mu = sum_j psi_j dPhi_j/dmu
// (all in the walk frame of the line; lines with a negative shift are walked
// mirrored, where mu = -nu).  The adjoint gathers: each input cell is written
// once, from a sliding window of the five interfaces that read it.
//
// One thread per line.  Lines along x, y, z, ux and uy are read with direct
// strided loads (neighbouring lanes take neighbouring elements of a row, so
// every access is coalesced); the contiguous uz-lines go through LDS tiles of
// whole lines, loaded and stored with 16-byte accesses, as in the forward uz
// sweep.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.hpp"
#include "rows.hpp"
#include "sl_mpp5.hpp"

namespace vlasov {

namespace {

// Derivatives of the interface-value weights with respect to mu.
struct WeightSlopes {
    float d0, d1, d2, d3, d4;
};

__device__ __forceinline__ WeightSlopes sl5_weight_slopes(float mu)
{
    const float m2 = mu * mu, m3 = m2 * mu;
    const float k = 1.0f / 120.0f;
    WeightSlopes s;
    s.d0 = (4.0f * m3 - 10.0f * mu) * k;
    s.d1 = -(16.0f * m3 - 15.0f * m2 - 60.0f * mu + 5.0f) * k;
    s.d2 = (24.0f * m3 - 45.0f * m2 - 80.0f * mu + 75.0f) * k;
    s.d3 = -(16.0f * m3 - 45.0f * m2 - 20.0f * mu + 75.0f) * k;
    s.d4 = (4.0f * m3 - 15.0f * m2 + 10.0f * mu + 5.0f) * k;
    return s;
}

// Linear form over the stencil (a, b, c, d, e), with the derivative with
// respect to mu in slot 5 (the stencil values do not depend on mu).
struct Lin {
    float w[6];
};

__device__ __forceinline__ Lin lin_zero()
{
    Lin r;
#pragma unroll
    for (int q = 0; q < 6; ++q) r.w[q] = 0.0f;
    return r;
}

__device__ __forceinline__ Lin lin_unit(int k)
{
    Lin r = lin_zero();
    r.w[k] = 1.0f;
    return r;
}

__device__ __forceinline__ Lin lin_comb(float p, const Lin& x, float q, const Lin& y)
{
    Lin r;
#pragma unroll
    for (int i = 0; i < 6; ++i) r.w[i] = p * x.w[i] + q * y.w[i];
    return r;
}

__device__ __forceinline__ Lin lin_scale(float p, const Lin& x)
{
    Lin r;
#pragma unroll
    for (int i = 0; i < 6; ++i) r.w[i] = p * x.w[i];
    return r;
}

// A value with its linear form.
struct VL {
    float v;
    Lin l;
};
struct FluxLin {
    float W[5];     // d phi / d (a..e)
    float dmu;      // d phi / d mu
};

// Selections on (value, candidate index) pairs with the FP64 oracle's tie
// rules (min and max keep their first argument on a tie; the median is
// max(min(x,y), min(max(x,y),z))): every selection is decided on the
// values, and the linear form is built for the winning candidate only.
struct Pick {
    float v;
    int id;
};
__device__ __forceinline__ Pick pmin2(const Pick& x, const Pick& y) { return x.v <= y.v ? x : y; }
__device__ __forceinline__ Pick pmax2(const Pick& x, const Pick& y) { return x.v >= y.v ? x : y; }
__device__ __forceinline__ Pick pmed3(const Pick& x, const Pick& y, const Pick& z)
{
    return pmax2(pmin2(x, y), pmin2(pmax2(x, y), z));
}
// minmod of four; id 4 stands for the zero it returns when signs differ
__device__ __forceinline__ Pick pminmod4(const Pick& w, const Pick& x, const Pick& y, const Pick& z)
{
    if (w.v > 0.0f && x.v > 0.0f && y.v > 0.0f && z.v > 0.0f)
        return pmin2(pmin2(w, x), pmin2(y, z));
    if (w.v < 0.0f && x.v < 0.0f && y.v < 0.0f && z.v < 0.0f)
        return pmax2(pmax2(w, x), pmax2(y, z));
    return Pick{0.0f, 4};
}

// curv_minmod on (value, candidate): the value with curv_minmod's FP32
// operations (so the bounds that use it are the forward's), the candidate
// the oracle's minmod of four picks where its value is the same, else the
// one the value came from (m = minmod(Da, Db), or 4m - o with o the other).
__device__ __forceinline__ Pick pcurv_minmod(float Da, float Db)
{
    const float v = curv_minmod(Da, Db);
    const Pick w = pminmod4(Pick{fmaf(4.0f, Da, -Db), 0}, Pick{fmaf(4.0f, Db, -Da), 1},
                            Pick{Da, 2}, Pick{Db, 3});
    if (w.v == v) return Pick{v, w.id};
    if (v == 0.0f) return Pick{v, 4};
    const bool a_least = med3(Da, Db, 0.0f) == Da;
    if (v == (a_least ? Da : Db)) return Pick{v, a_least ? 2 : 3};
    return Pick{v, a_least ? 0 : 1};
}

// Form of the curvature minmod that won: candidates 4 Da - Db (0),
// 4 Db - Da (1), Da (2), Db (3), zero (4).
__device__ __forceinline__ Lin minmod_form(int id, const Lin& Da, const Lin& Db)
{
    switch (id) {
        case 0: return lin_comb(4.0f, Da, -1.0f, Db);
        case 1: return lin_comb(4.0f, Db, -1.0f, Da);
        case 2: return Da;
        case 3: return Db;
        default: return lin_zero();
    }
}

__device__ __forceinline__ Lin curvature_form(const Lin& l, const Lin& m, const Lin& r)
{
    return lin_comb(1.0f, lin_comb(1.0f, l, -2.0f, m), 1.0f, r);
}

// mp_bounded on (value, form) pairs: the values with mp_bounded's FP32
// operations, so every selection is the forward's.  u[] are the forms of the
// stencil's a..e (the upwind frame's cells, or mirrored for a comp line);
// the upper-limit factor alpha carries its mu-derivative alpha_mu.  The
// candidates of the bounds are c (0), d (1), fMD (2), fUL (3), fLC (4) and
// the unlimited value fhat (5).
__device__ VL mp_bounded_lin(const VL& fhat, const Stencil& s, const Lin (&u)[5], float alpha,
                             float alpha_mu)
{
    const float Dmv = s.dm1 - s.dm2, D0v = s.d0 - s.dm1, Dpv = s.dp1 - s.d0;
    // curv_minmod(Da, Db) = minmod(4Da-Db, 4Db-Da, Da, Db)
    const Pick Mp = pcurv_minmod(D0v, Dpv);
    const Pick Mm = pcurv_minmod(Dmv, D0v);
    const Pick c{s.c, 0};
    const Pick d{s.d, 1};
    const Pick fMD{fmaf(-0.5f, Mp.v, fmaf(0.5f, s.d0, s.c)), 2};
    const Pick fUL{fmaf(alpha, s.dm1, s.c), 3};
    const Pick fLC{fmaf(4.0f / 3.0f, Mm.v, fmaf(0.5f, s.dm1, s.c)), 4};
    const Pick lo = pmax2(pmin2(pmin2(c, d), fMD), pmin2(pmin2(c, fUL), fLC));
    const Pick hi = pmin2(pmax2(pmax2(c, d), fMD), pmax2(pmax2(c, fUL), fLC));
    const Pick r = pmed3(Pick{fhat.v, 5}, lo, hi);
    VL out;
    out.v = r.v;
    switch (r.id) {
        case 5: out.l = fhat.l; break;
        case 0: out.l = u[2]; break;
        case 1: out.l = u[3]; break;
        case 3: {
            const Lin cb = lin_comb(1.0f, u[2], -1.0f, u[1]);                 // c - b
            out.l = lin_comb(alpha, cb, 1.0f, u[2]);
            out.l.w[5] += alpha_mu * s.dm1;
            break;
        }
        case 2: {
            const Lin D0 = curvature_form(u[1], u[2], u[3]);
            const Lin Dp = curvature_form(u[2], u[3], u[4]);
            out.l = lin_comb(0.5f, lin_comb(1.0f, u[2], 1.0f, u[3]), -0.5f,
                             minmod_form(Mp.id, D0, Dp));
            break;
        }
        default: {
            const Lin cb = lin_comb(1.0f, u[2], -1.0f, u[1]);
            const Lin Dm = curvature_form(u[0], u[1], u[2]);
            const Lin D0 = curvature_form(u[1], u[2], u[3]);
            out.l = lin_comb(4.0f / 3.0f, minmod_form(Mm.id, Dm, D0), 1.0f,
                             lin_comb(0.5f, cb, 1.0f, u[2]));
            break;
        }
    }
    return out;
}

// The forward flux with its frozen linearisation.  The values follow
// flux_mag / mp_flux / mp_bounded operation by operation, so every selection
// is the forward's (the clamp of a comp line is read on the complement, see
// below).
__device__ FluxLin flux_lin(const Stencil& s, const LineShift& sh, const WeightSlopes& ds)
{
    float y = sh.v0 * s.dm2;
    y = fmaf(sh.v1, s.dm1, y);
    y = fmaf(sh.v2, s.d0, y);
    y = fmaf(sh.v3, s.dp1, y);
    const float m = med3(s.d0, sh.alpha * s.dm1, 0.0f);
    // y = fhat - c as a form: the weights, and d fhat / d mu
    VL Y;
    Y.v = y;
    Y.l.w[0] = sh.w0; Y.l.w[1] = sh.w1; Y.l.w[2] = sh.w2 - 1.0f; Y.l.w[3] = sh.w3;
    Y.l.w[4] = sh.w4;
    float ydmu = ds.d0 * s.a;
    ydmu = fmaf(ds.d1, s.b, ydmu);
    ydmu = fmaf(ds.d2, s.c, ydmu);
    ydmu = fmaf(ds.d3, s.d, ydmu);
    ydmu = fmaf(ds.d4, s.e, ydmu);
    Y.l.w[5] = ydmu;
    const Lin uc = lin_unit(2);
    const bool early = med3(y, 0.0f, m) == y;
    FluxLin out;
    VL r;
    if (!sh.comp) {
        VL F{s.c + y, lin_comb(1.0f, uc, 1.0f, Y.l)};
        if (!early) {
            // d alpha / d mu = -1/mu^2 (0 where alpha is held at its cap)
            const float a_mu = sh.mu * (kAlphaCap + 1.0f) <= 1.0f ? 0.0f : -1.0f / (sh.mu * sh.mu);
            const Lin u[5] = {lin_unit(0), lin_unit(1), lin_unit(2), lin_unit(3), lin_unit(4)};
            F = mp_bounded_lin(F, s, u, sh.alpha, a_mu);
        }
        // positivity clamp med3(mu L, 0, c), oracle tie rules
        VL pre{sh.mu * F.v, lin_scale(sh.mu, F.l)};
        pre.l.w[5] = fmaf(sh.mu, F.l.w[5], F.v);
        const Pick k = pmed3(Pick{pre.v, 0}, Pick{0.0f, 1}, Pick{s.c, 2});
        r.v = k.v;
        r.l = k.id == 0 ? pre.l : (k.id == 1 ? lin_zero() : uc);
    } else {
        // complement: ghat = c - q y on the mirrored stencil with alpha_c; what
        // leaves through the complement side is Psi = med3(mu' ghat_lim, 0, c)
        // and Phi = c - Psi.  The selections of that clamp are taken on Psi,
        // as the split at the nearest integer takes them (its tie rules differ
        // from those of the same clamp written on Phi where c = 0).
        // dq/dmu = 1/mu'^2, d alpha_c/dmu = 1/mu'^2 (0 where held at its cap),
        // dmu'/dmu = -1.
        const float q_mu = 1.0f / (sh.muc * sh.muc);
        VL G{fmaf(-sh.q, y, s.c), lin_comb(1.0f, uc, -sh.q, Y.l)};
        G.l.w[5] = -sh.q * Y.l.w[5] - q_mu * y;
        if (!early) {
            const float ac_mu = sh.muc * (kAlphaCap + 1.0f) <= 1.0f ? 0.0f : q_mu;
            const Stencil mst{s.e, s.d, s.c, s.b, s.a, -s.dp1, -s.d0, -s.dm1, -s.dm2};
            const Lin u[5] = {lin_unit(4), lin_unit(3), lin_unit(2), lin_unit(1), lin_unit(0)};
            G = mp_bounded_lin(G, mst, u, sh.alpha_c, ac_mu);
        }
        VL P{sh.muc * G.v, lin_scale(sh.muc, G.l)};
        P.l.w[5] = sh.muc * G.l.w[5] - G.v;
        const Pick k = pmed3(Pick{P.v, 0}, Pick{0.0f, 1}, Pick{s.c, 2});
        const Lin psi = k.id == 0 ? P.l : (k.id == 1 ? lin_zero() : uc);
        r.v = s.c - k.v;
        r.l = lin_comb(1.0f, uc, -1.0f, psi);
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) out.W[q] = r.l.w[q];
    out.dmu = r.l.w[5];
    return out;
}

// Stencil of interface j+1/2 in the walk frame from a 5-value window.
__device__ __forceinline__ Stencil make_stencil(const float* w)
{
    return Stencil{w[0], w[1], w[2], w[3], w[4], w[1] - w[0], w[2] - w[1], w[3] - w[2],
                   w[4] - w[3]};
}

using Reader32 = GlobalReader<PREC_F32, 1, false>;

// Tangent of one line: x = forward input, v = input tangent, mu_dot = d mu.
__device__ void line_tangent(Reader32& rx, Reader32& rv, float* out, long stride, int M, int dir,
                             const LineShift& sh, bool periodic, float mu_dot)
{
    const WeightSlopes ds = sl5_weight_slopes(sh.mu);
    const int N = sh.N;
    float wx[5], wv[5];
    rx.seek(-N - 3);
    rv.seek(-N - 3);
    for (int q = 0; q < 5; ++q) {
        rx.next(&wx[q]);
        rv.next(&wv[q]);
    }
    auto dphi = [&](const float* xs, const float* vs) {
        const FluxLin fl = flux_lin(make_stencil(xs), sh, ds);
        float t = fl.dmu * mu_dot;
#pragma unroll
        for (int q = 0; q < 5; ++q) t = fmaf(fl.W[q], vs[q], t);
        return t;
    };
    float old = dphi(wx, wv);                     // interface j0 - 1/2
    for (int i = 0; i < M; ++i) {
        for (int q = 0; q < 4; ++q) {
            wx[q] = wx[q + 1];
            wv[q] = wv[q + 1];
        }
        rx.next(&wx[4]);
        rv.next(&wv[4]);
        const float nw = dphi(wx, wv);            // interface j + 1/2, j = i - N
        const int p = dir > 0 ? i : M - 1 - i;
        out[(long)p * stride] = wv[2] - (nw - old);
        old = nw;
    }
}

// Adjoint of one line: x = forward input, lam = output adjoint (frame rows
// read through rl, which starts N rows later).  Writes lam_in and returns
// lam_mu.  R: a row reader of global memory (Reader32) or of an LDS tile.
template <int MT, class R>
__device__ float line_adjoint(R& rx, R& rl, float* lam_in, long stride, int Mrt, int dir,
                              const LineShift& sh, bool periodic)
{
    // MT > 0: the line length at compile time.  The walk is unrolled by five,
    // the length of the interface window below, so that its slots are renamed
    // instead of moved at every interface (unrolled whole, its inlined
    // linearisations need more registers than a SIMD has for two waves)
    const int M = MT > 0 ? MT : Mrt;
    const WeightSlopes ds = sl5_weight_slopes(sh.mu);
    const int N = sh.N;
    // interfaces j = -2 .. M+1 ; interface j reads x_{j-2..j+2}, psi_j needs
    // lam_{j+N}, lam_{j+N+1}
    float wx[5];
    rx.seek(-4);
    for (int q = 0; q < 5; ++q) rx.next(&wx[q]);    // x_{-4..0}: stencil of j = -2
    rl.seek(N - 2);
    float lam_lo, lam_hi;
    rl.next(&lam_lo);                                // lam_{-2+N}
    // window of the last five interfaces: psi and weights
    float psi[5], W[5][5];
    float lam_mu = 0.0f;
    // identity term source: lam_{r+N} for r = j-2 -> read separately
    R rid = rl;
    rid.seek(N);                                     // lam_{0+N}
#pragma unroll 5
    for (int j = -2; j <= M + 1; ++j) {
        if (j > -2) {
            for (int q = 0; q < 4; ++q) wx[q] = wx[q + 1];
            rx.next(&wx[4]);                         // x_{j+2}
        }
        rl.next(&lam_hi);                            // lam_{j+N+1}
        const FluxLin fl = flux_lin(make_stencil(wx), sh, ds);
        const float ps = lam_hi - lam_lo;
        lam_lo = lam_hi;
        if (periodic ? (j >= 0 && j < M) : true) lam_mu = fmaf(ps, fl.dmu, lam_mu);
        // slide the interface window: slot 4 holds interface j
        for (int q = 0; q < 4; ++q) {
            psi[q] = psi[q + 1];
            for (int k = 0; k < 5; ++k) W[q][k] = W[q + 1][k];
        }
        psi[4] = ps;
        for (int k = 0; k < 5; ++k) W[4][k] = fl.W[k];
        if (j >= 2) {
            // row r = j-2 is read by interfaces r-2..r+2 = slots 0..4 at offsets k = 2..-2
            const int r = j - 2;
            float id;
            rid.next(&id);                           // lam_{r+N}
            float acc = id;
            for (int q = 0; q < 5; ++q) acc = fmaf(psi[q], W[q][4 - q], acc);
            const int p = dir > 0 ? r : M - 1 - r;
            lam_in[(long)p * stride] = acc;
        }
    }
    return lam_mu;
}

}  // namespace

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_position_tan(const float* __restrict__ f,
                                                      const float* __restrict__ v,
                                                      float* __restrict__ out, PosArgs a)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.O * a.I) return;
    const long o = t / a.I, k = t - (t / a.I) * a.I;
    const int jl = (int)(((k % a.Nu) / a.pst) % a.nshift);
    const LineShift sh = split_shift(a.shift[jl], a.M, true);
    const int dir = sh.neg ? -1 : 1;
    const long base = o * (long)a.M * a.I + k;
    Reader32 rx{f + base, nullptr, a.I, 0, a.M, dir, true, 0};
    Reader32 rv{v + base, nullptr, a.I, 0, a.M, dir, true, 0};
    line_tangent(rx, rv, out + base, a.I, a.M, dir, sh, true, 0.0f);
}

template <int MT>
__global__ void __launch_bounds__(256) k_position_adj(const float* __restrict__ f,
                                                      const float* __restrict__ lam,
                                                      float* __restrict__ lam_in, PosArgs a)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.O * a.I) return;
    const long o = t / a.I;
    long k = t - o * a.I;
    // y sweeps (the shift follows u_y, pst = nu_z): consecutive lanes would
    // cover 64 / nu_z values of u_y, and a wave would run both sides of every
    // branch on the shift.  Instead each wave takes one u_y: 64 / nu_z whole
    // uz-lines from consecutive u_x rows -- a permutation of k within groups
    // of 64 nu_y elements (64 / nu_z u_x rows), which tile every row
    if (a.pst == a.nuz && a.nshift > 1 && a.nshift * a.nuz * a.nux == a.Nu && a.nuz <= 64 &&
        64 % a.nuz == 0 && a.nux % (64 / a.nuz) == 0) {
        const long G = 64L * a.nshift;
        const long l = k & 63;
        const long rr = l / a.nuz;
        k = (k / G) * G + (rr * a.nshift + (k % G) / 64) * a.nuz + (l - rr * a.nuz);
    }
    const int jl = (int)(((k % a.Nu) / a.pst) % a.nshift);
    const LineShift sh = split_shift(a.shift[jl], a.M, true);
    const int dir = sh.neg ? -1 : 1;
    const long base = o * (long)a.M * a.I + k;
    Reader32 rx{f + base, nullptr, a.I, 0, a.M, dir, true, 0};
    Reader32 rl{lam + base, nullptr, a.I, 0, a.M, dir, true, 0};
    line_adjoint<MT>(rx, rl, lam_in + base, a.I, a.M, dir, sh, true);
}

// Velocity sweeps: one work-group per spatial cell; lines of the cell are
// (sub, k) with line start ((cell*nsub + sub) * M) * I + k.
__global__ void __launch_bounds__(256) k_velocity_tan(const float* __restrict__ f,
                                                      const float* __restrict__ v,
                                                      float* __restrict__ out,
                                                      const float* __restrict__ g_dot, VelArgs a)
{
    const long cell = blockIdx.x;
    const double s = (double)a.g[cell] * a.factor;
    const LineShift sh = split_shift(s, a.M, a.periodic);
    const int dir = sh.neg ? -1 : 1;
    // d mu / d s = +1 (rightward) or -1 (walked mirrored); s_dot = g_dot dt / du
    const float s_dot = g_dot != nullptr ? (float)((double)g_dot[cell] * a.factor) : 0.0f;
    const float mu_dot = sh.neg ? -s_dot : s_dot;
    const long lpc = a.nsub * a.I;
    for (long l = threadIdx.x; l < lpc; l += blockDim.x) {
        const long sub = l / a.I, k = l - (l / a.I) * a.I;
        const long base = ((cell * a.nsub + sub) * a.M) * a.I + k;
        Reader32 rx{f + base, nullptr, a.I, 0, a.M, dir, a.periodic, 0};
        Reader32 rv{v + base, nullptr, a.I, 0, a.M, dir, a.periodic, 0};
        line_tangent(rx, rv, out + base, a.I, a.M, dir, sh, a.periodic, mu_dot);
    }
}

template <int MT>
__global__ void __launch_bounds__(256) k_velocity_adj(const float* __restrict__ f,
                                                      const float* __restrict__ lam,
                                                      float* __restrict__ lam_in,
                                                      float* __restrict__ lam_g, VelArgs a)
{
    __shared__ double red[4];
    const long cell = blockIdx.x;
    const double s = (double)a.g[cell] * a.factor;
    const LineShift sh = split_shift(s, a.M, a.periodic);
    const int dir = sh.neg ? -1 : 1;
    const long lpc = a.nsub * a.I;
    double mine = 0.0;
    for (long l = threadIdx.x; l < lpc; l += blockDim.x) {
        const long sub = l / a.I, k = l - (l / a.I) * a.I;
        const long base = ((cell * a.nsub + sub) * a.M) * a.I + k;
        Reader32 rx{f + base, nullptr, a.I, 0, a.M, dir, a.periodic, 0};
        Reader32 rl{lam + base, nullptr, a.I, 0, a.M, dir, a.periodic, 0};
        mine += (double)line_adjoint<MT>(rx, rl, lam_in + base, a.I, a.M, dir, sh, a.periodic);
    }
    if (lam_g != nullptr) {
        const double tot = block_sum(mine, red);
        // lam_s = +lam_mu (rightward) or -lam_mu (mirrored); ds/dg = dt/du
        if (threadIdx.x == 0) lam_g[cell] += (float)((sh.neg ? -tot : tot) * a.factor);
    }
}

// Adjoint of the uz sweep: the lines are contiguous (M values), so a
// work-group stages NT whole lines of f and of lam through LDS with 16-byte
// loads, each thread walks one line out of LDS into a third tile, and the
// results leave with 16-byte stores.  lam_mu is summed per cell as in
// k_velocity_adj (per thread over its lines, then over the work-group).
template <int MT, int NT>
__global__ void __launch_bounds__(NT) k_velocity_adj_uz(const float* __restrict__ f,
                                                        const float* __restrict__ lam,
                                                        float* __restrict__ lam_in,
                                                        float* __restrict__ lam_g, VelArgs a)
{
    constexpr int LS = MT + 1;                  // padded line stride in LDS
    __shared__ float tf[NT * LS], tl[NT * LS], to[NT * LS];
    __shared__ double red[NT / 64];
    const long cell = blockIdx.x;
    const double s = (double)a.g[cell] * a.factor;
    const LineShift sh = split_shift(s, MT, a.periodic);
    const int dir = sh.neg ? -1 : 1;
    const long lpc = a.nsub;                    // lines per cell = nux * nuy
    const long cbase = cell * lpc;
    double mine = 0.0;
    for (long l0 = 0; l0 < lpc; l0 += NT) {
        const int nl = (int)((lpc - l0) < NT ? (lpc - l0) : NT);
        const long off0 = (cbase + l0) * MT;
        for (int e = threadIdx.x * 4; e < nl * MT; e += NT * 4) {
            const int ln = e / MT;
            const int off = e - ln * MT;
            const float4 x = *reinterpret_cast<const float4*>(f + off0 + e);
            const float4 y = *reinterpret_cast<const float4*>(lam + off0 + e);
            float* df = tf + ln * LS + off;
            float* dl = tl + ln * LS + off;
            df[0] = x.x; df[1] = x.y; df[2] = x.z; df[3] = x.w;
            dl[0] = y.x; dl[1] = y.y; dl[2] = y.z; dl[3] = y.w;
        }
        __syncthreads();
        if (threadIdx.x < nl) {
            LdsReader rx{tf + threadIdx.x * LS, 1, MT, dir, a.periodic, 0};
            LdsReader rl{tl + threadIdx.x * LS, 1, MT, dir, a.periodic, 0};
            mine += (double)line_adjoint<MT>(rx, rl, to + threadIdx.x * LS, 1, MT, dir, sh,
                                         a.periodic);
        }
        __syncthreads();
        for (int e = threadIdx.x * 4; e < nl * MT; e += NT * 4) {
            const int ln = e / MT;
            const int off = e - ln * MT;
            const float* src = to + ln * LS + off;
            *reinterpret_cast<float4*>(lam_in + off0 + e) = make_float4(src[0], src[1], src[2], src[3]);
        }
        __syncthreads();
    }
    if (lam_g != nullptr) {
        const double tot = block_sum(mine, red);
        if (threadIdx.x == 0) lam_g[cell] += (float)((sh.neg ? -tot : tot) * a.factor);
    }
}

hipError_t launch_position_tan(const float* f, const float* v, float* out, const PosArgs& a,
                               hipStream_t st)
{
    const long total = a.O * a.I;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_position_tan, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, f,
                       v, out, a);
    return hipGetLastError();
}

hipError_t launch_position_adj(const float* f, const float* lam, float* lam_in, const PosArgs& a,
                               hipStream_t st)
{
    const long total = a.O * a.I;
    if (total == 0) return hipSuccess;
    const dim3 grid((unsigned)((total + 255) / 256));
    switch (a.M) {
        case 16: hipLaunchKernelGGL(k_position_adj<16>, grid, dim3(256), 0, st, f, lam, lam_in, a); break;
        case 32: hipLaunchKernelGGL(k_position_adj<32>, grid, dim3(256), 0, st, f, lam, lam_in, a); break;
        case 64: hipLaunchKernelGGL(k_position_adj<64>, grid, dim3(256), 0, st, f, lam, lam_in, a); break;
        default: hipLaunchKernelGGL(k_position_adj<0>, grid, dim3(256), 0, st, f, lam, lam_in, a); break;
    }
    return hipGetLastError();
}

static unsigned vel_block(const VelArgs& a)
{
    long bs = ((a.nsub * a.I + 63) / 64) * 64;
    return (unsigned)(bs > 256 ? 256 : bs);
}

hipError_t launch_velocity_tan(const float* f, const float* v, float* out, const float* g_dot,
                               const VelArgs& a, hipStream_t st)
{
    if (a.cells == 0) return hipSuccess;
    hipLaunchKernelGGL(k_velocity_tan, dim3((unsigned)a.cells), dim3(vel_block(a)), 0, st, f, v,
                       out, g_dot, a);
    return hipGetLastError();
}

hipError_t launch_velocity_adj(const float* f, const float* lam, float* lam_in, float* lam_g,
                               const VelArgs& a, hipStream_t st)
{
    if (a.cells == 0) return hipSuccess;
    // uz (contiguous lines of 16, 32 or 64 values, 16-byte aligned cells):
    // LDS tiles of 4096 values per array
    const bool al = ((uintptr_t)f | (uintptr_t)lam | (uintptr_t)lam_in) % 16 == 0;
    if (a.I == 1 && al) {
        const dim3 grid((unsigned)a.cells);
        switch (a.M) {
            case 16:
                hipLaunchKernelGGL((k_velocity_adj_uz<16, 256>), grid, dim3(256), 0, st, f, lam, lam_in, lam_g, a);
                return hipGetLastError();
            case 32:
                hipLaunchKernelGGL((k_velocity_adj_uz<32, 128>), grid, dim3(128), 0, st, f, lam, lam_in, lam_g, a);
                return hipGetLastError();
            case 64:
                hipLaunchKernelGGL((k_velocity_adj_uz<64, 64>), grid, dim3(64), 0, st, f, lam, lam_in, lam_g, a);
                return hipGetLastError();
            default:
                break;
        }
    }
    const dim3 cg((unsigned)a.cells), cb(vel_block(a));
    switch (a.M) {
        case 16: hipLaunchKernelGGL(k_velocity_adj<16>, cg, cb, 0, st, f, lam, lam_in, lam_g, a); break;
        case 32: hipLaunchKernelGGL(k_velocity_adj<32>, cg, cb, 0, st, f, lam, lam_in, lam_g, a); break;
        case 64: hipLaunchKernelGGL(k_velocity_adj<64>, cg, cb, 0, st, f, lam, lam_in, lam_g, a); break;
        default: hipLaunchKernelGGL(k_velocity_adj<0>, cg, cb, 0, st, f, lam, lam_in, lam_g, a); break;
    }
    return hipGetLastError();
}

}  // namespace vlasov
