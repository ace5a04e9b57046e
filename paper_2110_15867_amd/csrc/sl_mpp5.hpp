// Device building blocks of the SL-MPP5 sweep (section 5.2): storage codecs,
// the per-line shift split, the conservative semi-Lagrangian weights, the
// Suresh-Huynh bounds and the two line walkers that every sweep kernel uses.
//
// All flux arithmetic is FP32 (section 5.1.1).  Each walker streams one line
// (or V lines side by side) through a register window, so every cell is
// loaded once, every interface flux is evaluated once, and every curvature
// and curvature-minmod is computed once and reused by its neighbours.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vlasov {

enum Prec { PREC_F32 = 0, PREC_F16 = 1, PREC_BF16 = 2 };

// ---------------------------------------------------------------------------
// Storage codecs.  FP32 stores the value; FP16/BF16 store value/scale with
// round-to-nearest-even, the scale being the largest |value| of the uz-line.
// ---------------------------------------------------------------------------
template <int P> struct Codec;
template <> struct Codec<PREC_F32> {
    using T = float;
    static constexpr bool scaled = false;
    __device__ static float dec(T v) { return v; }
    __device__ static T enc(float x) { return x; }
};
template <> struct Codec<PREC_F16> {
    using T = _Float16;
    static constexpr bool scaled = true;
    __device__ static float dec(T v) { return (float)v; }
    __device__ static T enc(float x) { return (_Float16)x; }
};
template <> struct Codec<PREC_BF16> {
    using T = __bf16;
    static constexpr bool scaled = true;
    __device__ static float dec(T v) { return (float)v; }
    __device__ static T enc(float x) { return (__bf16)x; }
};

template <typename T, int V> struct alignas(sizeof(T) * V) Pack { T v[V]; };

// Code of value x with inverse scale inv: the FP32 product, rounded once to
// FP32, then rounded to the storage type.  The empty asm pins the FP32
// product so instruction selection cannot merge the multiply into a
// mixed-precision FMA with a single rounding; every kernel then encodes
// identically.
template <int P>
__device__ __forceinline__ typename Codec<P>::T quantize(float x, float inv)
{
    if (!Codec<P>::scaled) return Codec<P>::enc(x);
    float y = x * inv;
    asm("" : "+v"(y));
    return Codec<P>::enc(y);
}

template <int P, int V>
__device__ __forceinline__ void load_row(const typename Codec<P>::T* p, float scale, float* x)
{
    using T = typename Codec<P>::T;
    Pack<T, V> q = *reinterpret_cast<const Pack<T, V>*>(p);
#pragma unroll
    for (int v = 0; v < V; ++v) x[v] = Codec<P>::scaled ? Codec<P>::dec(q.v[v]) * scale : Codec<P>::dec(q.v[v]);
}

template <int P, int V>
__device__ __forceinline__ void store_row(typename Codec<P>::T* p, const float* x, float inv)
{
    using T = typename Codec<P>::T;
    Pack<T, V> q;
#pragma unroll
    for (int v = 0; v < V; ++v) q.v[v] = quantize<P>(x[v], inv);
    *reinterpret_cast<Pack<T, V>*>(p) = q;
}

// ---------------------------------------------------------------------------
// Shift of one line: s = N + nu, N integer, nu in [0,1) for s >= 0 and in
// (-1,0] for s < 0 (Eqs. 3-4 give s; the integer part is an exact
// translation).  Everything after the split runs in the upwind frame, where
// the shift is non-negative: `neg` says the line is walked mirrored.
// ---------------------------------------------------------------------------
struct LineShift {
    int N;      // integer part in the upwind frame (>= 0), reduced mod M when periodic
    float mu;   // fractional part |nu| in [0,1)
    bool neg;   // s < 0: walk the line mirrored
    float w0, w1, w2, w3, w4;   // interface-value weights for cells j-2 .. j+2
};

// Interface value of the conservative SL flux: the mean over the departure
// interval of the quartic through the five cell averages j-2..j+2.  The flux
// is mu times this value; the weights are quartics in mu that tend to the
// fifth-order upwind point value (2,-13,47,27,-3)/60 as mu -> 0.
__device__ __forceinline__ void sl5_weights(float mu, LineShift& sh)
{
    const float m2 = mu * mu;
    const float k = 1.0f / 120.0f;
    sh.w0 = (m2 - 1.0f) * (m2 - 4.0f) * k;
    sh.w1 = -(m2 - 1.0f) * (mu + 2.0f) * (4.0f * mu - 13.0f) * k;
    sh.w2 = (mu + 1.0f) * (mu + 2.0f) * ((6.0f * mu - 33.0f) * mu + 47.0f) * k;
    sh.w3 = -(mu - 1.0f) * (mu - 2.0f) * (mu - 3.0f) * (4.0f * mu + 9.0f) * k;
    sh.w4 = (m2 - 1.0f) * (mu - 2.0f) * (mu - 3.0f) * k;
}

__device__ __forceinline__ LineShift split_shift(double s, int M, bool periodic)
{
    LineShift sh;
    const double n = (s >= 0.0) ? floor(s) : ceil(s);
    const double nu = s - n;                 // exact in FP64
    sh.neg = s < 0.0;
    double a = sh.neg ? -n : n;              // integer part in the upwind frame
    if (periodic) {
        a = fmod(a, (double)M);              // exact for |a| < 2^53
    } else if (a > (double)(M + 8)) {
        a = (double)(M + 8);                 // every cell already left the line
    }
    sh.N = (int)a;
    sh.mu = (float)fabs(nu);
    sl5_weights(sh.mu, sh);
    return sh;
}

// ---------------------------------------------------------------------------
// Suresh-Huynh monotonicity-preserving bounds (alpha = 4, epsilon = 0) and the
// positivity clamp, for one interface in its upwind frame.  a..e are the cell
// averages j-2..j+2 (j = upwind cell); Mp and Mm are the curvature minmods at
// j+1/2 and j-1/2.  Returns the flux magnitude through the interface.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float med3(float a, float b, float c)
{
    return __builtin_amdgcn_fmed3f(a, b, c);
}

// minmod(4Da-Db, 4Db-Da, Da, Db): least magnitude when all four share a
// strict sign, else 0 -- as med3(min, max, 0).
__device__ __forceinline__ float curv_minmod(float Da, float Db)
{
    const float p = fmaf(4.0f, Da, -Db);
    const float q = fmaf(4.0f, Db, -Da);
    const float mn = fminf(fminf(p, q), fminf(Da, Db));
    const float mx = fmaxf(fmaxf(p, q), fmaxf(Da, Db));
    return med3(mn, mx, 0.0f);
}

__device__ __forceinline__ float curvature(float l, float c, float r)
{
    return fmaf(-2.0f, c, l + r);
}

__device__ __forceinline__ float flux_mag(float a, float b, float c, float d, float e, float Mp,
                                          float Mm, const LineShift& sh)
{
    // unlimited SL interface value
    float fhat = sh.w0 * a;
    fhat = fmaf(sh.w1, b, fhat);
    fhat = fmaf(sh.w2, c, fhat);
    fhat = fmaf(sh.w3, d, fhat);
    fhat = fmaf(sh.w4, e, fhat);
    // bounds
    const float cb = c - b;
    const float fUL = fmaf(4.0f, cb, c);
    const float fMD = 0.5f * ((c + d) - Mp);
    const float fLC = fmaf(4.0f / 3.0f, Mm, fmaf(0.5f, cb, c));
    const float lo = fmaxf(fminf(fminf(c, d), fMD), fminf(fminf(c, fUL), fLC));
    const float hi = fminf(fmaxf(fmaxf(c, d), fMD), fmaxf(fmaxf(c, fUL), fLC));
    const float lim = med3(fhat, lo, hi);
    // positivity: what leaves the upwind cell lies between 0 and its content
    return med3(sh.mu * lim, 0.0f, c);
}

// ---------------------------------------------------------------------------
// Uniform walker: every lane of the wave moves in the same direction, so the
// line is walked in its upwind frame (mirrored when the shift is negative)
// with a 5-cell window.  Rows are requested in order from j0-3 = -N-3 to
// M-N+1; the reader turns a frame row into a value (wrap or zero ghost).
//   out_i = x_{i-N} - (Phi_{i-N+1/2} - Phi_{i-N-1/2})
// With zero ghosts the content leaving the upper face of the frame,
// sum_{r >= M-N} x_r + Phi_{M-N-1/2}, is returned in *ofl.
// MT > 0 fixes the line length at compile time (full unroll, and for
// periodic lines the first five rows are kept instead of re-read).
// ---------------------------------------------------------------------------
template <int V, int MT, class Reader, class Writer>
__device__ __forceinline__ void walk_uniform(Reader& rd, Writer& wr, const int Mrt,
                                             const LineShift& sh, const bool periodic,
                                             float* ofl)
{
    const int M = MT > 0 ? MT : Mrt;
    const int N = sh.N;
    float xm2[V], xm1[V], x0[V], xp1[V], xp2[V];
    float Dm1[V], D0[V], Dp1[V], Mm[V], phi_old[V];
    float head[5][V];
    float acc = 0.0f;
    int r = -N - 3;                       // frame row of the next value
    rd.seek(r);
    rd.next(xm2); rd.next(xm1); rd.next(x0); rd.next(xp1); rd.next(xp2);
    if (!periodic) {
        // rows already in the window that lie past the upper face
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const int row = r + q;
            if (row >= M - N && row < M) {
                const float* src = q == 0 ? xm2 : q == 1 ? xm1 : q == 2 ? x0 : q == 3 ? xp1 : xp2;
#pragma unroll
                for (int v = 0; v < V; ++v) acc += src[v];
            }
        }
    }
    if (MT > 0 && periodic) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            head[0][v] = xm2[v]; head[1][v] = xm1[v]; head[2][v] = x0[v];
            head[3][v] = xp1[v]; head[4][v] = xp2[v];
        }
    }
    r += 5;
    // state for the interface (j0-1)+1/2, j0 = -N
#pragma unroll
    for (int v = 0; v < V; ++v) {
        Dm1[v] = curvature(xm2[v], xm1[v], x0[v]);
        D0[v] = curvature(xm1[v], x0[v], xp1[v]);
        Dp1[v] = curvature(x0[v], xp1[v], xp2[v]);
        Mm[v] = curv_minmod(Dm1[v], D0[v]);
        const float Mp = curv_minmod(D0[v], Dp1[v]);
        phi_old[v] = flux_mag(xm2[v], xm1[v], x0[v], xp1[v], xp2[v], Mp, Mm[v], sh);
        Mm[v] = Mp;
        // slide by one: window for j0
        xm2[v] = xm1[v]; xm1[v] = x0[v]; x0[v] = xp1[v]; xp1[v] = xp2[v];
        Dm1[v] = D0[v]; D0[v] = Dp1[v];
    }
#pragma unroll(MT > 0 ? MT : 1)
    for (int i = 0; i < M; ++i) {
        // new row j+2 for j = i - N
        if (MT > 0 && periodic && i >= M - 5) {
#pragma unroll
            for (int v = 0; v < V; ++v) xp2[v] = head[i - (M - 5)][v];
        } else {
            rd.next(xp2);
        }
        if (!periodic) {
            if (r >= M - N && r < M) {
#pragma unroll
                for (int v = 0; v < V; ++v) acc += xp2[v];
            }
        }
        ++r;
        float res[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            Dp1[v] = curvature(x0[v], xp1[v], xp2[v]);
            const float Mp = curv_minmod(D0[v], Dp1[v]);
            const float phi = flux_mag(xm2[v], xm1[v], x0[v], xp1[v], xp2[v], Mp, Mm[v], sh);
            res[v] = x0[v] - (phi - phi_old[v]);
            phi_old[v] = phi;
            Mm[v] = Mp;
            xm2[v] = xm1[v]; xm1[v] = x0[v]; x0[v] = xp1[v]; xp1[v] = xp2[v];
            Dm1[v] = D0[v]; D0[v] = Dp1[v];
        }
        wr.put(i, res);
    }
    if (!periodic) {
        // phi_old now holds Phi_{M-N-1/2}; rows past the window are added below
#pragma unroll
        for (int v = 0; v < V; ++v) acc += phi_old[v];
        int row0 = r > M - N ? r : M - N;
        row0 = row0 > 0 ? row0 : 0;
        for (int row = row0; row < M; ++row) {
            float x[V];
            rd.seek(row);
            rd.next(x);
#pragma unroll
            for (int v = 0; v < V; ++v) acc += x[v];
        }
        *ofl = acc;
    }
}

// ---------------------------------------------------------------------------
// Mixed walker: lanes of one wave may move in opposite directions (the z
// sweep, where the shift follows the contiguous u_z index).  All lanes walk
// forward with a 6-cell window; each lane picks its upwind stencil and the
// matching curvature minmod by select.  Periodic lines only.
// ---------------------------------------------------------------------------
template <int V, int MT, class Reader, class Writer>
__device__ __forceinline__ void walk_mixed(Reader& rd, Writer& wr, const int Mrt, const int Nsgn,
                                           const LineShift& sh)
{
    const int M = MT > 0 ? MT : Mrt;
    const bool neg = sh.neg;
    // signed integer offset in the physical frame: out_i = x_{i-Ns} ...
    const int Ns = Nsgn;
    float xm2[V], xm1[V], x0[V], xp1[V], xp2[V], xp3[V];
    float Dm1[V], D0[V], Dp1[V], Dp2[V], Mm[V], M0[V], phi_old[V];
    float head[6][V];
    rd.seek(-Ns - 3);
    rd.next(xm2); rd.next(xm1); rd.next(x0); rd.next(xp1); rd.next(xp2); rd.next(xp3);
    if (MT > 0) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            head[0][v] = xm2[v]; head[1][v] = xm1[v]; head[2][v] = x0[v];
            head[3][v] = xp1[v]; head[4][v] = xp2[v]; head[5][v] = xp3[v];
        }
    }
    // state for j = j0 - 1
#pragma unroll
    for (int v = 0; v < V; ++v) {
        Dm1[v] = curvature(xm2[v], xm1[v], x0[v]);
        D0[v] = curvature(xm1[v], x0[v], xp1[v]);
        Dp1[v] = curvature(x0[v], xp1[v], xp2[v]);
        Dp2[v] = curvature(xp1[v], xp2[v], xp3[v]);
        Mm[v] = curv_minmod(Dm1[v], D0[v]);
        M0[v] = curv_minmod(D0[v], Dp1[v]);
        const float Mp = curv_minmod(Dp1[v], Dp2[v]);
        const float a = neg ? xp3[v] : xm2[v];
        const float b = neg ? xp2[v] : xm1[v];
        const float c = neg ? xp1[v] : x0[v];
        const float d = neg ? x0[v] : xp1[v];
        const float e = neg ? xm1[v] : xp2[v];
        phi_old[v] = flux_mag(a, b, c, d, e, M0[v], neg ? Mp : Mm[v], sh);
        Mm[v] = M0[v]; M0[v] = Mp;
        xm2[v] = xm1[v]; xm1[v] = x0[v]; x0[v] = xp1[v]; xp1[v] = xp2[v]; xp2[v] = xp3[v];
        Dm1[v] = D0[v]; D0[v] = Dp1[v]; Dp1[v] = Dp2[v];
    }
    const float sgn = neg ? -1.0f : 1.0f;
#pragma unroll(MT > 0 ? MT : 1)
    for (int i = 0; i < M; ++i) {
        if (MT > 0 && i >= M - 6) {
#pragma unroll
            for (int v = 0; v < V; ++v) xp3[v] = head[i - (M - 6)][v];
        } else {
            rd.next(xp3);
        }
        float res[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            Dp2[v] = curvature(xp1[v], xp2[v], xp3[v]);
            const float Mp = curv_minmod(Dp1[v], Dp2[v]);
            const float a = neg ? xp3[v] : xm2[v];
            const float b = neg ? xp2[v] : xm1[v];
            const float c = neg ? xp1[v] : x0[v];
            const float d = neg ? x0[v] : xp1[v];
            const float e = neg ? xm1[v] : xp2[v];
            const float phi = flux_mag(a, b, c, d, e, M0[v], neg ? Mp : Mm[v], sh);
            res[v] = fmaf(-sgn, phi - phi_old[v], x0[v]);
            phi_old[v] = phi;
            Mm[v] = M0[v]; M0[v] = Mp;
            xm2[v] = xm1[v]; xm1[v] = x0[v]; x0[v] = xp1[v]; xp1[v] = xp2[v]; xp2[v] = xp3[v];
            Dm1[v] = D0[v]; D0[v] = Dp1[v]; Dp1[v] = Dp2[v];
        }
        wr.put(i, res);
    }
}

}  // namespace vlasov
