// Device building blocks of the SL-MPP5 sweep (section 5.2): storage codecs,
// the per-line shift split, the conservative semi-Lagrangian weights, the
// Suresh-Huynh bounds and the two line walkers that every sweep kernel uses.
//
// All flux arithmetic is FP32 (section 5.1.1).  Each walker streams one line
// (or V lines side by side) through a register window, so every cell is
// loaded once and every interface flux is evaluated once.
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

// A wave-uniform value moved to a scalar register.  The empty asm hides
// the value's uniformity, so the optimiser keeps the readfirstlane (it drops
// one applied to a value it already knows to be uniform, which can leave the
// value in a vector register and the address arithmetic on the VALU).
__device__ __forceinline__ int uniform_sgpr(int v)
{
    asm volatile("" : "+v"(v));
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ long uniform_long(long v)
{
    const unsigned lo = (unsigned)uniform_sgpr((int)(unsigned)v);
    const unsigned hi = (unsigned)uniform_sgpr((int)(unsigned)((unsigned long)v >> 32));
    return (long)(((unsigned long)hi << 32) | lo);
}

__device__ __forceinline__ float uniform_f32(float v)
{
    return __builtin_bit_cast(float, uniform_sgpr(__builtin_bit_cast(int, v)));
}

// Inverse of a line scale: the hardware reciprocal, used by every kernel that
// encodes, so all of them produce the same codes.  A line whose largest
// |value| is below the smallest normal FP32 number (1.2e-38) is stored as
// zeros, as an all-zero line is: the reciprocal of such a scale overflows
// FP32 (a finite value times it would give an infinite code, a zero a NaN).
__device__ __forceinline__ float inv_scale(float m)
{
    return m >= 1.17549435e-38f ? __builtin_amdgcn_rcpf(m) : 0.0f;
}

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

// Value of code q with scale sc: the product code x scale, written as an FMA
// with -0 (which adds nothing, so the sign of a zero product survives) so
// that FP16 codes decode in one mixed-precision FMA (the FP16 operand is
// widened inside the instruction, exactly).  Every kernel decodes with it.
template <int P>
__device__ __forceinline__ float decode(typename Codec<P>::T q, float sc)
{
    if (!Codec<P>::scaled) return Codec<P>::dec(q);
    // (the -0 is hidden from the optimiser, which would otherwise turn the
    // FMA back into a widening and a multiply)
    float nz = -0.0f;
    asm("" : "+v"(nz));
    return fmaf(Codec<P>::dec(q), sc, nz);
}

template <int P, int V>
__device__ __forceinline__ void load_row(const typename Codec<P>::T* p, float scale, float* x)
{
    using T = typename Codec<P>::T;
    Pack<T, V> q = *reinterpret_cast<const Pack<T, V>*>(p);
#pragma unroll
    for (int v = 0; v < V; ++v) x[v] = decode<P>(q.v[v], scale);
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
//
// The limiter's reading splits the shift at the nearest integer instead, so
// that the fraction is at most half a cell either way and the Suresh-Huynh
// upper limit f_j + alpha (f_j - f_{j-1}) can use alpha = (1-|nu|)/|nu|, the
// largest value for which a single-stage update keeps monotone data
// monotone.  For a fraction mu >= 1/2 of the floor split that is the
// translation by N+1 followed by a move back by mu' = 1 - mu.  Both give the
// same unlimited flux through x_{j+1/2}: the quartic of cell j integrated
// over the last mu of the cell is the cell's content minus the quartic
// integrated over its first mu', so Phi = mu fhat = f_j - mu' ghat, where
// ghat is the mirrored interface value of the first mu' of cell j, and
// ghat - f_j = -(mu/mu') (fhat - f_j).  Such a line is flagged `comp`
// (complement): its bounds are those of ghat on the mirrored stencil with
// alpha' = alpha(mu'), and its flux is f_j - mu' ghat_lim.  The Suresh-Huynh
// early-out needs no change: with alpha = mu'/mu the interval test on
// fhat - f_j is the mirrored test on ghat - f_j with alpha' = mu/mu' (where
// alpha' is held at its cap the two tests differ, and such lines always
// evaluate the bounds).
// ---------------------------------------------------------------------------
struct LineShift {
    int N;      // integer part in the upwind frame (>= 0), reduced mod M when periodic
    float mu;   // fractional part |nu| in [0,1)
    bool neg;   // s < 0: walk the line mirrored
    bool comp;  // |nu| >= 1/2: the bounds act on the complement (see above)
    float alpha;                // upper-limit factor of the early-out test (and of the
                                // bounds of a line that is not comp), alpha(mu)
    float q, alpha_c, muc;      // comp lines: mu/mu', alpha(mu'), mu' = 1 - mu
    float w0, w1, w2, w3, w4;   // interface-value weights for cells j-2 .. j+2
    float v0, v1, v2, v3;       // the same in difference form (see sl5_weights)
};

// Largest upper-limit factor of a single-stage update with Courant number
// mu: (1-mu)/mu, held at 2^20 below mu = 1/(1+2^20) so that it stays finite
// at a whole-cell shift (a smaller factor keeps the property).
constexpr float kAlphaCap = 1048576.0f;
__device__ __forceinline__ float mp_alpha(float mu)
{
    return mu * (kAlphaCap + 1.0f) <= 1.0f ? kAlphaCap : (1.0f - mu) / mu;
}

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
    // The weights sum to one (a constant line is reproduced), so the
    // interface value is f_j plus a combination of the four differences
    // around it:  fhat - f_j = v0 (f_{j-1}-f_{j-2}) + v1 (f_j-f_{j-1})
    //                        + v2 (f_{j+1}-f_j) + v3 (f_{j+2}-f_{j+1}).
    sh.v0 = -sh.w0;
    sh.v1 = -(sh.w0 + sh.w1);
    sh.v2 = sh.w3 + sh.w4;
    sh.v3 = sh.w4;
}

// The limiter constants of the fraction nu (FP64; mu = |nu| in FP32).  For a
// comp line mu' is taken from FP64, where 1 - |nu| is exact and positive
// (mu itself may round to 1 in FP32).
__device__ __forceinline__ void mp_params(double nu, float mu, LineShift& sh)
{
    sh.comp = fabs(nu) >= 0.5;
    if (!sh.comp) {
        sh.alpha = mp_alpha(mu);
        sh.q = 0.0f;
        sh.alpha_c = 0.0f;
        sh.muc = 0.0f;
        return;
    }
    sh.muc = (float)(1.0 - fabs(nu));
    sh.q = mu / sh.muc;
    sh.alpha_c = mp_alpha(sh.muc);
    sh.alpha = sh.muc * (kAlphaCap + 1.0f) <= 1.0f ? 0.0f : sh.muc / mu;
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
    mp_params(nu, sh.mu, sh);
    return sh;
}

// ---------------------------------------------------------------------------
// Suresh-Huynh monotonicity-preserving bounds (epsilon = 0, upper-limit
// factor alpha) and the positivity clamp, for one interface in its upwind
// frame; a..e are the cell averages j-2..j+2 (j = upwind cell).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float med3(float a, float b, float c)
{
    return __builtin_amdgcn_fmed3f(a, b, c);
}

// minmod(4Da-Db, 4Db-Da, Da, Db): least magnitude when all four share a
// strict sign, else 0.  The two-argument minmod is med3(x, y, 0).  Let m =
// minmod(Da, Db) and o the other curvature.  When Da and Db share a strict
// sign, |4o - m| >= 3|o| >= |m| with the sign of o, so 4o - m never has the
// least magnitude, and the result is m or 4m - o, whichever is smaller in
// magnitude, or 0 where 4m - o has the other sign: med3(m, 4m - o, 0).
// Otherwise m = 0 and so is that median.  4m - o = 5m - (Da + Db): four
// operations instead of five, symmetric in Da and Db (as the carry between
// interfaces needs), and within one rounding of Da + Db of the four-way form.
__device__ __forceinline__ float curv_minmod(float Da, float Db)
{
    const float m = med3(Da, Db, 0.0f);
    return med3(m, fmaf(5.0f, m, -(Da + Db)), 0.0f);
}

__device__ __forceinline__ float curvature(float l, float c, float r)
{
    return fmaf(-2.0f, c, l + r);
}

// Upwind-frame stencil of one interface j+1/2: cell averages a..e =
// f_{j-2..j+2} and their differences b-a, c-b, d-c, e-d.  The walkers carry
// the differences from interface to interface, so each costs one subtraction.
struct Stencil {
    float a, b, c, d, e;
    float dm2, dm1, d0, dp1;
};

// The bounded value median(fhat, fmin, fmax) of the Suresh-Huynh constraint,
// given the curvature minmods d^M4 at j-1/2 (Mm) and j+1/2 (Mp).
__device__ __forceinline__ float mp_bounded_m(float fhat, const Stencil& s, float alpha, float Mm,
                                              float Mp)
{
    const float fUL = fmaf(alpha, s.dm1, s.c);
    // the mean of f_j and f_{j+1} as f_j + d0 / 2, minus half the minmod
    const float fMD = fmaf(-0.5f, Mp, fmaf(0.5f, s.d0, s.c));
    const float fLC = fmaf(4.0f / 3.0f, Mm, fmaf(0.5f, s.dm1, s.c));
    const float lo = fmaxf(fminf(fminf(s.c, s.d), fMD), fminf(fminf(s.c, fUL), fLC));
    const float hi = fminf(fmaxf(fmaxf(s.c, s.d), fMD), fmaxf(fmaxf(s.c, fUL), fLC));
    return med3(fhat, lo, hi);
}

__device__ __forceinline__ float mp_bounded(float fhat, const Stencil& s, float alpha)
{
    const float Dm = s.dm1 - s.dm2;                 // curvature at j-1
    const float D0 = s.d0 - s.dm1;                  // curvature at j
    const float Dp = s.dp1 - s.d0;                  // curvature at j+1
    const float Mp = curv_minmod(D0, Dp);           // d^M4 at j+1/2
    const float Mm = curv_minmod(Dm, D0);           // d^M4 at j-1/2
    return mp_bounded_m(fhat, s, alpha, Mm, Mp);
}

// Flux (before the positivity clamp) of an interface whose unlimited value
// fails the Suresh-Huynh test.  comp lines bound the complement ghat on the
// mirrored stencil (e, d, c, b, a) and return f_j - mu' ghat_lim (see
// LineShift).  UNI: branch on the line's flag -- one branch when the lanes of
// the wave agree, and a wave whose lanes all take the same side skips the
// other; otherwise each lane picks its stencil orientation and constants by
// select and one set of bounds is evaluated (for waves whose lanes mix both
// kinds of line throughout, as in the y sweep).  The same operations per lane
// either way.
template <bool UNI>
__device__ __forceinline__ float mp_flux(const Stencil& s, const LineShift& sh, float y)
{
    if (UNI) {
        if (!sh.comp) return sh.mu * mp_bounded(s.c + y, s, sh.alpha);
        const Stencil m{s.e, s.d, s.c, s.b, s.a, -s.dp1, -s.d0, -s.dm1, -s.dm2};
        const float ghat = fmaf(-sh.q, y, s.c);
        return fmaf(-sh.muc, mp_bounded(ghat, m, sh.alpha_c), s.c);
    }
    // (q and alpha_c are recomputed here, as split_shift computes them, so
    // that they hold no registers across the walk)
    const bool c = sh.comp;
    const float q = sh.mu / sh.muc;
    const float ac = mp_alpha(sh.muc);
    const Stencil t{c ? s.e : s.a, c ? s.d : s.b, s.c, c ? s.b : s.d, c ? s.a : s.e,
                    c ? -s.dp1 : s.dm2, c ? -s.d0 : s.dm1, c ? -s.dm1 : s.d0,
                    c ? -s.dm2 : s.dp1};
    const float fh = c ? fmaf(-q, y, s.c) : s.c + y;
    const float lim = mp_bounded(fh, t, c ? ac : sh.alpha);
    return c ? fmaf(-sh.muc, lim, s.c) : sh.mu * lim;
}

// Flux magnitude through the interface j+1/2 in its upwind frame: the SL
// interface value, limited, times mu, clamped to [0, c].
// Suresh & Huynh keep the unlimited value when it lies between f_j and
// f_MP = f_j + minmod(f_{j+1} - f_j, alpha (f_j - f_{j-1})); that interval
// lies inside [fmin, fmax], so with epsilon = 0 the test only skips work:
// the curvatures and bounds are evaluated for the (rarer, and in smooth data
// wave-coherent) interfaces that fail it.
// The unlimited value is formed as f_j + (fhat - f_j) from the carried
// differences (four products instead of five, and fhat - f_j is what the
// test needs).
template <bool UNI = true>
__device__ __forceinline__ float flux_mag(const Stencil& s, const LineShift& sh)
{
    float y = sh.v0 * s.dm2;                            // fhat - f_j
    y = fmaf(sh.v1, s.dm1, y);
    y = fmaf(sh.v2, s.d0, y);
    y = fmaf(sh.v3, s.dp1, y);
    const float m = med3(s.d0, sh.alpha * s.dm1, 0.0f); // f_MP - f_j
    float pre = sh.mu * (s.c + y);
    if (__builtin_expect(med3(y, 0.0f, m) != y, 0)) pre = mp_flux<UNI>(s, sh, y);
    // positivity: what leaves the upwind cell lies between 0 and its content
    return med3(pre, 0.0f, s.c);
}

// flux_mag with the curvature minmods d^M4 at j-1/2 (Mm) and j+1/2 (Mp)
// supplied by a walker that evaluates every interface of a line in order:
// d^M4 at j+1/2 is d^M4 at j-1/2 of the next interface (the minmod is
// symmetric in its two curvatures, so the values are the very bits
// mp_bounded would compute), so one minmod per interface is evaluated
// outside the test and the bounds left behind it cost ten operations.
// The mirrored stencil of a comp line swaps the two.  Same result as
// flux_mag, bit for bit.
// UNI: branch on the line's comp flag (as mp_flux<true>); otherwise each lane
// picks its orientation by select (as mp_flux<false>) -- mp_bounded_m reads
// only c, d, d0, dm1 and the two minmods of the stencil, so five selects
// orient it.
template <bool UNI = true>
__device__ __forceinline__ float flux_mag_mm(const Stencil& s, const LineShift& sh, float Mm,
                                             float Mp)
{
    float y = sh.v0 * s.dm2;                            // fhat - f_j
    y = fmaf(sh.v1, s.dm1, y);
    y = fmaf(sh.v2, s.d0, y);
    y = fmaf(sh.v3, s.dp1, y);
    const float m = med3(s.d0, sh.alpha * s.dm1, 0.0f); // f_MP - f_j
    float pre = sh.mu * (s.c + y);
    if (__builtin_expect(med3(y, 0.0f, m) != y, 0)) {
        if (UNI) {
            if (!sh.comp) {
                pre = sh.mu * mp_bounded_m(s.c + y, s, sh.alpha, Mm, Mp);
            } else {
                const Stencil r{s.e, s.d, s.c, s.b, s.a, -s.dp1, -s.d0, -s.dm1, -s.dm2};
                const float ghat = fmaf(-sh.q, y, s.c);
                pre = fmaf(-sh.muc, mp_bounded_m(ghat, r, sh.alpha_c, Mp, Mm), s.c);
            }
        } else {
            const bool c = sh.comp;
            const float q = sh.mu / sh.muc;
            const float ac = mp_alpha(sh.muc);
            Stencil t = s;
            t.d = c ? s.b : s.d;
            t.d0 = c ? -s.dm1 : s.d0;
            t.dm1 = c ? -s.d0 : s.dm1;
            const float fh = c ? fmaf(-q, y, s.c) : s.c + y;
            const float lim = mp_bounded_m(fh, t, c ? ac : sh.alpha, c ? Mp : Mm, c ? Mm : Mp);
            pre = c ? fmaf(-sh.muc, lim, s.c) : sh.mu * lim;
        }
    }
    return med3(pre, 0.0f, s.c);
}

// The constants of a line whose shift is the same in every lane of the wave,
// moved to scalar registers.
__device__ __forceinline__ LineShift uniform_shift(const LineShift& sh)
{
    LineShift u = sh;
    u.N = uniform_sgpr(sh.N);
    u.neg = uniform_sgpr(sh.neg ? 1 : 0) != 0;
    u.comp = uniform_sgpr(sh.comp ? 1 : 0) != 0;
    u.mu = uniform_f32(sh.mu);
    u.alpha = uniform_f32(sh.alpha);
    u.q = uniform_f32(sh.q);
    u.alpha_c = uniform_f32(sh.alpha_c);
    u.muc = uniform_f32(sh.muc);
    u.v0 = uniform_f32(sh.v0);
    u.v1 = uniform_f32(sh.v1);
    u.v2 = uniform_f32(sh.v2);
    u.v3 = uniform_f32(sh.v3);
    return u;
}

// ---------------------------------------------------------------------------
// Rows requested ahead of use.  With the line length known at compile time
// a walk is fully unrolled, so the ring slot of every row is a constant and
// the ring lives in registers: PD rows are in flight while the fluxes of
// earlier rows are computed (HBM needs many bytes in flight per CU, and one
// row of one wave is only 256 B-1 KiB).  The walks read rows strictly in
// order; take(i) hands out the i-th row of the walk's loop and requests row
// i + PD, never beyond the L rows the loop consumes.
// ---------------------------------------------------------------------------
template <int V, int MT>
struct RowPipeDepth {
    static constexpr int value = MT == 0 ? 1 : (V >= 2 ? 4 : 8);
};

template <int V, int PD, class Reader>
struct RowPipe {
    Reader& rd;
    float ring[PD][V];

    __device__ explicit RowPipe(Reader& r) : rd(r) {}
    __device__ void prime(int L)
    {
#pragma unroll
        for (int q = 0; q < PD; ++q)
            if (q < L) rd.next(ring[q]);
    }
    __device__ void take(int i, int L, float* x)
    {
        if (PD == 1) {
            rd.next(x);
            return;
        }
#pragma unroll
        for (int v = 0; v < V; ++v) x[v] = ring[i % PD][v];
        if (i + PD < L) rd.next(ring[i % PD]);
    }
};

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
template <int V, int MT, bool UNI, class Reader, class Writer>
__device__ __forceinline__ void walk_uniform(Reader& rd, Writer& wr, const int Mrt,
                                             const LineShift& sh, const bool periodic,
                                             float* ofl)
{
    const int M = MT > 0 ? MT : Mrt;
    const int N = sh.N;
    float xm2[V], xm1[V], x0[V], xp1[V], xp2[V], phi_old[V];
    float dm2[V], dm1[V], d0[V], dp1[V];    // x_{j-1}-x_{j-2}, ..., x_{j+2}-x_{j+1}
    // curvature at j and d^M4 at j-1/2, carried (flux_mag_mm).  Carrying
    // adds a minmod per interface outside the early-out test and saves two
    // behind it: it pays where the test fails often.  Not for waves of single
    // lines with per-lane shifts (one-direction waves of the z sweep), where
    // it was measured to cost time.
    constexpr bool CARRY = UNI || V > 1;
    float cj[V], kj[V];
    float head[5][V];
    float acc = 0.0f;
    int r = -N - 3;                       // frame row of the next value
    rd.seek(r);
    rd.next(xm2); rd.next(xm1); rd.next(x0); rd.next(xp1); rd.next(xp2);
    // rows the loop reads (a periodic line's last five come from head[])
    const int L = (MT > 0 && periodic) ? M - 5 : M;
    RowPipe<V, RowPipeDepth<V, MT>::value, Reader> pipe(rd);
    if (RowPipeDepth<V, MT>::value > 1) pipe.prime(L);
    if (!periodic) {
        // rows already in the window that lie past the upper face
        auto past = [&](int row) { return row >= M - N && row < M; };
#pragma unroll
        for (int v = 0; v < V; ++v) {
            acc += past(r) ? xm2[v] : 0.0f;
            acc += past(r + 1) ? xm1[v] : 0.0f;
            acc += past(r + 2) ? x0[v] : 0.0f;
            acc += past(r + 3) ? xp1[v] : 0.0f;
            acc += past(r + 4) ? xp2[v] : 0.0f;
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
    // flux through (j0-1)+1/2, j0 = -N; then slide the window to j0
#pragma unroll
    for (int v = 0; v < V; ++v) {
        dm2[v] = xm1[v] - xm2[v];
        dm1[v] = x0[v] - xm1[v];
        d0[v] = xp1[v] - x0[v];
        dp1[v] = xp2[v] - xp1[v];
        const Stencil st{xm2[v], xm1[v], x0[v], xp1[v], xp2[v], dm2[v], dm1[v], d0[v], dp1[v]};
        if constexpr (CARRY) {
            const float c0 = d0[v] - dm1[v], cp = dp1[v] - d0[v];
            const float Mp = curv_minmod(c0, cp);
            phi_old[v] = flux_mag_mm<UNI>(st, sh, curv_minmod(dm1[v] - dm2[v], c0), Mp);
            cj[v] = cp;
            kj[v] = Mp;
        } else {
            phi_old[v] = flux_mag<UNI>(st, sh);
        }
        xm2[v] = xm1[v]; xm1[v] = x0[v]; x0[v] = xp1[v]; xp1[v] = xp2[v];
        dm2[v] = dm1[v]; dm1[v] = d0[v]; d0[v] = dp1[v];
    }
    constexpr int UNR = MT > 0 ? MT : 1;
#pragma unroll UNR
    for (int i = 0; i < M; ++i) {
        // new row j+2 for j = i - N
        if (MT > 0 && periodic && i >= M - 5) {
#pragma unroll
            for (int v = 0; v < V; ++v) xp2[v] = head[i - (M - 5)][v];
        } else {
            pipe.take(i, L, xp2);
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
            dp1[v] = xp2[v] - xp1[v];
            const Stencil st{xm2[v], xm1[v], x0[v], xp1[v], xp2[v], dm2[v], dm1[v], d0[v], dp1[v]};
            float phi;
            if constexpr (CARRY) {
                const float cp = dp1[v] - d0[v];
                const float Mp = curv_minmod(cj[v], cp);
                phi = flux_mag_mm<UNI>(st, sh, kj[v], Mp);
                cj[v] = cp;
                kj[v] = Mp;
            } else {
                phi = flux_mag<UNI>(st, sh);
            }
            res[v] = x0[v] - (phi - phi_old[v]);
            phi_old[v] = phi;
            xm2[v] = xm1[v]; xm1[v] = x0[v]; x0[v] = xp1[v]; xp1[v] = xp2[v];
            dm2[v] = dm1[v]; dm1[v] = d0[v]; d0[v] = dp1[v];
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
// Whole-line update in registers: the line (compile-time length M) is already
// held in x[0..M-1] in its upwind frame, so every cell of every stencil is a
// fixed register and nothing waits on a load between interfaces.  Ghosts are
// zero (vacuum) or the wrapped cells (PER).  Hands each result
//   y_j = x_j - (Phi_{j+1/2} - Phi_{j-1/2}),   j = 0 .. M-1,
// to emit(j, y_j) as soon as it is known (for PER, y_0 comes last), with the
// same FP32 operations as walk_uniform; the integer translation
// out_{j+N} = y_j is the caller's.  Returns Phi_{M-1/2}, the flux through
// the upper face before the translation.
// ---------------------------------------------------------------------------
template <int M, bool PER>
__device__ __forceinline__ float line_cell(const float (&x)[M], int k)
{
    if (PER) return x[((k % M) + M) % M];
    return (k >= 0 && k < M) ? x[k] : 0.0f;
}

template <int M, bool PER, class Emit>
__device__ __forceinline__ float line_update_regs(const float (&x)[M], const LineShift& sh,
                                                  Emit&& emit)
{
    auto X = [&](int k) { return line_cell<M, PER>(x, k); };
    // curvature minmods carried from interface to interface (flux_mag_mm)
    const float e0 = X(-2) - X(-3), e1 = X(-1) - X(-2), e2 = X(0) - X(-1), e3 = X(1) - X(0);
    const float Dm1 = e2 - e1;                        // curvature at cell -1
    float D0 = e3 - e2;                               // curvature at cell 0
    float Mm = curv_minmod(e1 - e0, Dm1);             // d^M4 at -3/2
    // Phi_{-1/2}: the interface below cell 0 (for PER the one at the top)
    float phi_prev = 0.0f;
    {
        const float Mp = curv_minmod(Dm1, D0);        // d^M4 at -1/2
        if (!PER) phi_prev = flux_mag_mm(Stencil{X(-3), X(-2), X(-1), X(0), X(1), e0, e1, e2, e3},
                                         sh, Mm, Mp);
        Mm = Mp;
    }
    float dm2 = e1, dm1 = e2, d0 = e3;
    float phi_first = 0.0f;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const float dp1 = X(j + 2) - X(j + 1);
        const float Dp = dp1 - d0;                    // curvature at j+1
        const float Mp = curv_minmod(D0, Dp);         // d^M4 at j+1/2
        const float phi = flux_mag_mm(Stencil{X(j - 2), X(j - 1), X(j), X(j + 1), X(j + 2), dm2,
                                              dm1, d0, dp1}, sh, Mm, Mp);
        if (PER && j == 0) phi_first = phi;
        if (!PER || j > 0) emit(j, X(j) - (phi - phi_prev));
        phi_prev = phi;
        dm2 = dm1; dm1 = d0; d0 = dp1;
        D0 = Dp; Mm = Mp;
    }
    if (PER) emit(0, X(0) - (phi_first - phi_prev));   // Phi_{-1/2} = Phi_{M-1/2}
    return phi_prev;
}

// Upwind stencil of the interface j+1/2 from the window x_{j-2..j+3} and its
// differences: as is for a rightward shift, mirrored (x_{j+3..j-1}, negated
// differences in reverse order) for a leftward one.
__device__ __forceinline__ Stencil mixed_stencil(bool neg, float xm2, float xm1, float x0, float xp1,
                                                 float xp2, float xp3, float q0, float q1,
                                                 float q2, float q3, float q4)
{
    Stencil s;
    s.a = neg ? xp3 : xm2;
    s.b = neg ? xp2 : xm1;
    s.c = neg ? xp1 : x0;
    s.d = neg ? x0 : xp1;
    s.e = neg ? xm1 : xp2;
    s.dm2 = neg ? -q4 : q0;
    s.dm1 = neg ? -q3 : q1;
    s.d0 = neg ? -q2 : q2;
    s.dp1 = neg ? -q1 : q3;
    return s;
}

// ---------------------------------------------------------------------------
// Mixed walker: lanes of one wave may move in opposite directions (the z
// sweep, where the shift follows the contiguous u_z index).  All lanes walk
// forward with a 6-cell window; each lane picks its upwind stencil by select.
// Periodic lines only.
// ---------------------------------------------------------------------------
template <int V, int MT, class Reader, class Writer>
__device__ __forceinline__ void walk_mixed(Reader& rd, Writer& wr, const int Mrt, const int Nsgn,
                                           const LineShift& sh)
{
    const int M = MT > 0 ? MT : Mrt;
    const bool neg = sh.neg;
    const int Ns = Nsgn;                  // out_i = x_{i-Ns} - (Phi_{i-Ns+1/2} - Phi_{i-Ns-1/2})
    float xm2[V], xm1[V], x0[V], xp1[V], xp2[V], xp3[V], phi_old[V];
    float q0[V], q1[V], q2[V], q3[V], q4[V];   // x_{j-1}-x_{j-2}, ..., x_{j+3}-x_{j+2}
    // carried for flux_mag_mm: curvatures at j+1, j+2 and K_i = d^M4 at
    // i-1/2 (the minmod of the curvatures at i-1 and i) for i = j .. j+2.
    // The stencil of a lane moving up has d^M4 = K_j below and K_{j+1}
    // above; a mirrored lane's (upwind cell j+1) has K_{j+2} and K_{j+1}.
    float c1[V], c2[V], k0[V], k1[V], k2[V];
    float head[6][V];
    rd.seek(-Ns - 3);
    rd.next(xm2); rd.next(xm1); rd.next(x0); rd.next(xp1); rd.next(xp2); rd.next(xp3);
    const int L = MT > 0 ? M - 6 : M;           // rows the loop reads
    RowPipe<V, RowPipeDepth<V, MT>::value, Reader> pipe(rd);
    if (RowPipeDepth<V, MT>::value > 1) pipe.prime(L);
    if (MT > 0) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            head[0][v] = xm2[v]; head[1][v] = xm1[v]; head[2][v] = x0[v];
            head[3][v] = xp1[v]; head[4][v] = xp2[v]; head[5][v] = xp3[v];
        }
    }
    // flux through (j0-1)+1/2, then slide
#pragma unroll
    for (int v = 0; v < V; ++v) {
        q0[v] = xm1[v] - xm2[v];
        q1[v] = x0[v] - xm1[v];
        q2[v] = xp1[v] - x0[v];
        q3[v] = xp2[v] - xp1[v];
        q4[v] = xp3[v] - xp2[v];
        const float cm1 = q1[v] - q0[v], c0 = q2[v] - q1[v];
        c1[v] = q3[v] - q2[v];
        c2[v] = q4[v] - q3[v];
        k0[v] = curv_minmod(cm1, c0);
        k1[v] = curv_minmod(c0, c1[v]);
        k2[v] = curv_minmod(c1[v], c2[v]);
        phi_old[v] = flux_mag_mm(mixed_stencil(neg, xm2[v], xm1[v], x0[v], xp1[v], xp2[v], xp3[v],
                                               q0[v], q1[v], q2[v], q3[v], q4[v]),
                                 sh, neg ? k2[v] : k0[v], k1[v]);
        xm2[v] = xm1[v]; xm1[v] = x0[v]; x0[v] = xp1[v]; xp1[v] = xp2[v]; xp2[v] = xp3[v];
        q0[v] = q1[v]; q1[v] = q2[v]; q2[v] = q3[v]; q3[v] = q4[v];
    }
    const float sgn = neg ? -1.0f : 1.0f;
    constexpr int UNR = MT > 0 ? MT : 1;
#pragma unroll UNR
    for (int i = 0; i < M; ++i) {
        if (MT > 0 && i >= M - 6) {
#pragma unroll
            for (int v = 0; v < V; ++v) xp3[v] = head[i - (M - 6)][v];
        } else {
            pipe.take(i, L, xp3);
        }
        float res[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            q4[v] = xp3[v] - xp2[v];
            const float c3 = q4[v] - q3[v];
            const float k3 = curv_minmod(c2[v], c3);
            k0[v] = k1[v]; k1[v] = k2[v]; k2[v] = k3;
            c1[v] = c2[v]; c2[v] = c3;
            const float phi = flux_mag_mm(mixed_stencil(neg, xm2[v], xm1[v], x0[v], xp1[v], xp2[v],
                                                        xp3[v], q0[v], q1[v], q2[v], q3[v], q4[v]),
                                          sh, neg ? k2[v] : k0[v], k1[v]);
            res[v] = fmaf(-sgn, phi - phi_old[v], x0[v]);
            phi_old[v] = phi;
            xm2[v] = xm1[v]; xm1[v] = x0[v]; x0[v] = xp1[v]; xp1[v] = xp2[v]; xp2[v] = xp3[v];
            q0[v] = q1[v]; q1[v] = q2[v]; q2[v] = q3[v]; q3[v] = q4[v];
        }
        wr.put(i, res);
    }
}

// ---------------------------------------------------------------------------
// Paired walker: each lane updates two periodic lines whose rows it reads
// and writes together — line A moving up by less than one cell (shift in
// [0, 1)), line B moving down by less than one cell (shift in (-1, 0)) — so
// neither needs a per-lane select between upwind stencils.  The reader hands
// out each row's A and B values (x[0], x[1]); the writer takes both outputs.
//   A, upwind frame as is (walk_uniform's arithmetic, to the bit):
//     out_i = x_i - (Phi_i - Phi_{i-1}),  Phi_k = flux through k+1/2 from
//     cells k-2 .. k+2 (rows -3 .. 1 first, then row i+2 at step i).
//   B, upwind frame mirrored, walked forward: G_k = flux leaving cell k
//   through k-1/2, its stencil a..e being cells k+2 .. k-2 and its
//   differences x_{k+1}-x_{k+2}, x_k-x_{k+1}, x_{k-1}-x_k, x_{k-2}-x_{k-1}
//   (the subtractions walk_uniform does in the mirrored frame), and
//     out_i = x_i + (G_{i+1} - G_i)    (rows -2 .. 2 first, then row i+3),
//   the mirrored walk's x - (G_i - G_{i+1}) to the bit (a rounded difference
//   changes sign exactly).
// B needs each row one step before A, so a row is read once, at B's step,
// and A's value waits one step in a register.  MT (the line length) is
// fixed at compile time; rows 0..2, read first, serve again as rows M..M+2.
// ---------------------------------------------------------------------------
template <int MT, class Reader, class Writer>
__device__ __forceinline__ void walk_pair(Reader& rd, Writer& wr, const LineShift& sa,
                                          const LineShift& sb)
{
    constexpr int M = MT;
    constexpr int PD = 8;
    constexpr int L = M - 3;                      // rows the loop reads
    static_assert(MT > 3 + PD, "line too short for the paired walk");
    float a[5], da[4], phia;      // A: window x_{j-2..j+2}, forward differences
    float b[5], mb[4], gb;        // B: window x_{k-2..k+2}, md[q] = w[q] - w[q+1]
    float head[3][2];
    float carry;                  // A's value of the row read last
    rd.seek(-3);
    {
        float x[2];
        rd.next(x);                                // row -3 (A only)
        a[0] = x[0];
#pragma unroll
        for (int q = 1; q < 6; ++q) {              // rows -2 .. 2
            rd.next(x);
            if (q < 5) a[q] = x[0];
            else carry = x[0];
            b[q - 1] = x[1];
            if (q >= 3) {
                head[q - 3][0] = x[0];
                head[q - 3][1] = x[1];
            }
        }
    }
    RowPipe<2, PD, Reader> pipe(rd);
    pipe.prime(L);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        da[q] = a[q + 1] - a[q];
        mb[q] = b[q] - b[q + 1];
    }
    // carried for flux_mag_mm.  A: the newest curvature (da[3] - da[2]) and
    // d^M4 at the upper face (the next interface's lower one).  B (mirrored
    // stencil, differences mb[3..0]): the curvature mb[2] - mb[3] and d^M4
    // at the mirrored lower face (the next interface's upper one).
    float ca = da[3] - da[2];
    float ka = curv_minmod(da[2] - da[1], ca);
    float cb = mb[2] - mb[3];
    float kb = curv_minmod(cb, mb[1] - mb[2]);
    phia = flux_mag_mm(Stencil{a[0], a[1], a[2], a[3], a[4], da[0], da[1], da[2], da[3]}, sa,
                       curv_minmod(da[1] - da[0], da[2] - da[1]), ka);
    gb = flux_mag_mm(Stencil{b[4], b[3], b[2], b[1], b[0], mb[3], mb[2], mb[1], mb[0]}, sb, kb,
                     curv_minmod(mb[1] - mb[2], mb[0] - mb[1]));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        a[q] = a[q + 1];
        b[q] = b[q + 1];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        da[q] = da[q + 1];
        mb[q] = mb[q + 1];
    }
#pragma unroll MT
    for (int i = 0; i < M; ++i) {
        float x[2];                                // row i + 3
        if (i >= L) {
            x[0] = head[i - L][0];
            x[1] = head[i - L][1];
        } else {
            pipe.take(i, L, x);
        }
        a[4] = carry;                              // row i + 2
        carry = x[0];
        b[4] = x[1];
        da[3] = a[4] - a[3];
        mb[3] = b[3] - b[4];
        const float ca_new = da[3] - da[2];
        const float ka_new = curv_minmod(ca, ca_new);
        const float pa_new = flux_mag_mm(Stencil{a[0], a[1], a[2], a[3], a[4], da[0], da[1], da[2], da[3]},
                                         sa, ka, ka_new);
        ca = ca_new;
        ka = ka_new;
        const float cb_new = mb[2] - mb[3];
        const float kb_new = curv_minmod(cb_new, cb);
        const float gb_new = flux_mag_mm(Stencil{b[4], b[3], b[2], b[1], b[0], mb[3], mb[2], mb[1], mb[0]},
                                         sb, kb_new, kb);
        cb = cb_new;
        kb = kb_new;
        const float ra_out = a[2] - (pa_new - phia);
        const float rb_out = b[1] + (gb_new - gb);
        phia = pa_new;
        gb = gb_new;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a[q] = a[q + 1];
            b[q] = b[q + 1];
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            da[q] = da[q + 1];
            mb[q] = mb[q + 1];
        }
        wr.put(i, ra_out, rb_out);
    }
}

}  // namespace vlasov
