// Fused velocity kick: the three velocity sweeps D_uz D_uy D_ux of one half
// step (Eq. 5) applied to each spatial cell's velocity block inside LDS.
//
// Every velocity sweep is local to a spatial cell (the shift g(x) dt / du is
// the same for all lines of the cell, and velocity space is never split --
// section 5.1.3), so a work-group can hold the whole block (32^3 FP32 values
// = 128 KiB of MI355X's 160 KiB LDS), run ux, uy and uz on it, and touch HBM
// once for reading and once for writing instead of three times each.  Each
// sweep performs the same FP32 operations as the single-sweep kernels, so
// with FP32 storage the result is bitwise the one of the three separate
// sweeps.  With FP16/BF16 storage only the result is stored: the values
// between the three sweeps stay FP32 in LDS (the storage format is what
// lives in HBM), which saves the two intermediate roundings the separate
// sweeps make -- the fused result is the more accurate one.
//
// The work-groups are persistent (as many as fit on the chip, each walking
// cells blockIdx.x, blockIdx.x + gridDim.x, ...).  While one block is swept
// in LDS, the next one is already on its way from HBM into registers, and the
// finished block's stores drain behind the next block's arithmetic: the LDS
// holds one block, so this is the only way its HBM traffic overlaps compute.
//
// LDS layout: uz-lines of NU values padded to NU+1 floats, line index
// jx*NU + jy.  A thread owns one line per sweep; lanes of a wave read
// consecutive jz (ux, uy sweeps) or lines NU+1 floats apart (uz sweep), both
// free of bank conflicts.  Lines of one sweep are disjoint, so a thread may
// overwrite its own line as soon as it has read it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.hpp"
#include "rows.hpp"
#include "sl_mpp5.hpp"

namespace vlasov {

// One thread's share of a velocity block in flight from HBM: NS slots of 4
// consecutive values of one uz-line, with that line's scale.
template <int P, int NU>
struct BlockSlots {
    using T = typename Codec<P>::T;
    static constexpr int NT = NU * NU;
    static constexpr int NS = NU * NU * NU / (NT * 4);
    Pack<T, 4> q[NS];
    float sc[NS];
    float g[3];        // the cell's acceleration field (ux, uy, uz)

    // element index of slot s: consecutive threads take consecutive 4-value
    // groups, so every access is coalesced
    __device__ static int elem(int s, int t) { return (s * NT + t) * 4; }

    // (t arrives through fresh_tid() at every use: the slot offsets are
    // recomputed, a few integer operations, instead of occupying registers
    // for the whole sweep)
    __device__ void load(const T* __restrict__ fin, const float* __restrict__ sin,
                         const KickArgs& a, int cell, int t)
    {
        // the field first: the sweeps wait for it, not for the block behind it
#pragma unroll
        for (int k = 0; k < 3; ++k) g[k] = a.g[(long)k * a.cells + cell];
        const T* src = fin + (long)cell * (NT * NU);
        const float* ssrc = sin + (long)cell * NT;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int e = elem(s, t);
            q[s] = *reinterpret_cast<const Pack<T, 4>*>(src + e);
            sc[s] = Codec<P>::scaled ? ssrc[e / NU] : 1.0f;
        }
    }
    // decoded values into the padded LDS block
    __device__ void put(float* lds, int t) const
    {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int e = elem(s, t);
            float* dst = lds + (e / NU) * (NU + 1) + e % NU;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                dst[u] = decode<P>(q[s].v[u], sc[s]);
        }
    }
};

// threadIdx.x, opaque to the optimiser (see BlockSlots)
__device__ __forceinline__ int fresh_tid()
{
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

template <int M, int S, bool NEG>
__device__ __forceinline__ void read_line(const float* line, float (&x)[M])
{
#pragma unroll
    for (int k = 0; k < M; ++k) x[k] = line[(NEG ? M - 1 - k : k) * S];
}

// The integer part N > 0 of a line's shift, applied after the fractional
// update has left y_j at frame position j: out_{j+N} = y_j.  Vacuum lines
// return what passes the upper face, sum_{j >= M-N} y_j + Phi_{M-1/2};
// periodic lines rotate.  (Rare in practice -- a kick moves less than one
// cell per half step unless the field is strong -- so the addressing here is
// plain runtime arithmetic.)
template <int M, int S, bool NEG, bool PER>
__device__ __forceinline__ float translate_line(float* line, int N, float phi_top)
{
    auto at = [&](int p) -> float& { return line[(NEG ? M - 1 - p : p) * S]; };
    if (PER && M <= 32) {
        float z[M];
#pragma unroll
        for (int k = 0; k < M; ++k) z[k] = at(k);
#pragma unroll
        for (int k = 0; k < M; ++k) {
            int p = k + N;                     // N < M on periodic lines
            p = p >= M ? p - M : p;
            at(p) = z[k];
        }
        return 0.0f;
    }
    if (PER) {
        // 64-value lines: the rotation in place, as three reversals (all
        // positions, then 0..N-1 and N..M-1), so that no copy of the line
        // holds registers for the whole kernel (with one, the tiled uz
        // kernel needed 276 registers and spilled)
        auto rev = [&](int lo, int hi) {
            for (int i = lo, j = hi - 1; i < j; ++i, --j) {
                const float u = at(i);
                at(i) = at(j);
                at(j) = u;
            }
        };
        rev(0, M);
        rev(0, N);
        rev(N, M);
        return 0.0f;
    }
    float acc = 0.0f;
    for (int p = (M - N > 0 ? M - N : 0); p < M; ++p) acc += at(p);
    for (int p = M - 1; p >= N; --p) at(p) = at(p - N);
    const int nz = N < M ? N : M;
    for (int p = 0; p < nz; ++p) at(p) = 0.0f;
    return acc + phi_top;
}

// One velocity sweep of the block in LDS along AXIS (0: ux, 1: uy, 2: uz),
// for lines whose upwind direction is -u (NEG) or +u: frame position p of a
// line lies at line[(NEG ? M-1-p : p) * S], so every access of the common
// case (|shift| < 1 cell) has a fixed offset.  Returns this thread's line
// outflow (vacuum boundaries).  With scaled storage the uz sweep also finds
// the new scale of its uz-line (the largest |value| it keeps) and writes it to
// sout_line and lmax_line.
template <int P, int NU, bool PER, int AXIS, bool NEG>
__device__ __forceinline__ float kick_axis_dir(float* line, const LineShift& sh, int N,
                                               float* sout_line, float* lmax_line)
{
    constexpr int M = NU;
    constexpr int S = AXIS == 0 ? NU * (NU + 1) : (AXIS == 1 ? NU + 1 : 1);
    constexpr bool SCALE = Codec<P>::scaled && AXIS == 2;
    auto at = [&](int p) -> float& { return line[(NEG ? M - 1 - p : p) * S]; };
    float x[M];
#pragma unroll
    for (int k = 0; k < M; ++k) x[k] = at(k);
    float m = 0.0f;                              // largest |value| (uz sweep)
    const float phi_top = line_update_regs<M, PER>(x, sh, [&](int j, float v) {
        at(j) = v;                               // the line reads above came first
        if (SCALE) m = fmaxf(m, fabsf(v));
    });
    float ofl = PER ? 0.0f : phi_top;            // N = 0: Phi_{M-1/2} leaves
    if (N > 0) {
        ofl = translate_line<M, S, NEG, PER>(line, N, phi_top);
        if (SCALE && !PER) {
            m = 0.0f;                            // only what stayed
            for (int p = N; p < M; ++p) m = fmaxf(m, fabsf(at(p)));
        }
    }
    if (SCALE) {
        // the new scale of this uz-line; the store divides by it
        *sout_line = m;
        *lmax_line = m;
    }
    return ofl;
}

template <int P, int NU, bool PER, int AXIS>
__device__ __forceinline__ float kick_axis(float* lds, float* sout_line, float* lmax_line,
                                           const KickArgs& a, const KickShift* __restrict__ tab,
                                           int cell, float g, int t)
{
    constexpr int LS = NU + 1;
    const int base = AXIS == 0 ? (t / NU) * LS + (t % NU)
                   : AXIS == 1 ? (t / NU) * NU * LS + (t % NU)
                               : t * LS;
    LineShift sh;
    if (tab != nullptr) {
        // scalar loads of the precomputed split (uniform over the work-group)
        const KickShift e = tab[(long)cell * 3 + AXIS];
        sh.N = e.N;
        sh.neg = (e.flags & 1) != 0;
        sh.comp = (e.flags & 2) != 0;
        sh.mu = e.mu;
        sh.v0 = e.v0; sh.v1 = e.v1; sh.v2 = e.v2; sh.v3 = e.v3;
        sh.alpha = e.alpha; sh.q = e.q; sh.alpha_c = e.alpha_c; sh.muc = e.muc;
    } else {
        sh = split_shift((double)g * a.factor[AXIS], NU, PER);
    }
    const int N = uniform_sgpr(sh.N);
    if (uniform_sgpr(sh.neg ? 1 : 0))
        return kick_axis_dir<P, NU, PER, AXIS, true>(lds + base, sh, N, sout_line, lmax_line);
    return kick_axis_dir<P, NU, PER, AXIS, false>(lds + base, sh, N, sout_line, lmax_line);
}

// A double moved between lanes by a DPP control (each 32-bit half).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp((int)u, (int)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(u >> 32), (int)(u >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double read_lane_f64(double v, int lane)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = __builtin_amdgcn_readlane((int)u, lane);
    const unsigned hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// The sum of v over the wave, the same in every lane: a DPP tree within each
// 16-lane row (quad permutations, then half-row and row mirrors; partners
// add the same two partial sums, so every lane of a row holds the same bits),
// then the four row sums in row order.  Short VALU latencies: the sum sits
// right before a barrier.
__device__ __forceinline__ double wave_sum_f64(double v)
{
    v += dpp_f64<0xB1>(v);     // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);     // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);    // row_half_mirror
    v += dpp_f64<0x140>(v);    // row_mirror
    return ((read_lane_f64(v, 0) + read_lane_f64(v, 16)) + read_lane_f64(v, 32)) +
           read_lane_f64(v, 48);
}

// Outflow of one block, first half: the FP64 sums of the three per-thread
// line outflows over each wave, written by lane 0 to red[axis][wave].  The
// barrier that ends the last sweep publishes them.
template <int NT>
__device__ __forceinline__ void wave_sums3(const float (&o)[3], double* red)
{
    double v[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = wave_sum_f64((double)o[k]);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) red[k * (NT / 64) + (threadIdx.x >> 6)] = v[k];
    }
}

// Second half, in wave 0 after that barrier: lane k < 3 adds the wave sums of
// axis k in wave order, and lane 0 adds the three axes to the cell's total in
// sweep order (ux, uy, uz), as three separate sweeps would.  prev is the
// cell's total before this kick, loaded early by lane 0.
template <int NT>
__device__ __forceinline__ void outflow_total(const double* red, double prev, double du3,
                                              double* dst)
{
    const int lane = threadIdx.x;
    const int k = lane < 3 ? lane : 0;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) s += red[k * (NT / 64) + q];
    const double s0 = read_lane_f64(s, 0);
    const double s1 = read_lane_f64(s, 1);
    const double s2 = read_lane_f64(s, 2);
    if (lane == 0) {
        double acc = prev;
        acc += s0 * du3;
        acc += s1 * du3;
        acc += s2 * du3;
        *dst = acc;
    }
}

// Velocity moments of one stored block, second half: lane k < 4 of wave 0
// adds moment k's wave sums in wave order; lane 0 writes rho = sum f du^3
// and umean_a = sum u_a f / sum f (0 where the sum is 0), as vlasov_moments
// defines them.
template <int NT>
__device__ __forceinline__ void moments_total(const double* mred, const KickArgs& a, int cell)
{
    const int lane = threadIdx.x;
    const int k = lane < 4 ? lane : 0;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) s += mred[k * (NT / 64) + q];
    const double t0 = read_lane_f64(s, 0);
    const double t1 = read_lane_f64(s, 1);
    const double t2 = read_lane_f64(s, 2);
    const double t3 = read_lane_f64(s, 3);
    if (lane == 0) {
        a.rho[cell] = t0 * a.du3;
        if (a.umean != nullptr) {
            const double inv = t0 != 0.0 ? 1.0 / t0 : 0.0;
            a.umean[cell] = t1 * inv;
            a.umean[a.cells + cell] = t2 * inv;
            a.umean[2 * a.cells + cell] = t3 * inv;
        }
    }
}

template <int P, int NU, bool PER>
__global__ void __launch_bounds__(NU * NU) k_kick(const typename Codec<P>::T* __restrict__ fin,
                                                const float* __restrict__ sin,
                                                typename Codec<P>::T* __restrict__ fout,
                                                float* __restrict__ sout, KickArgs a,
                                                const KickShift* __restrict__ tab)
{
    using T = typename Codec<P>::T;
    using Slots = BlockSlots<P, NU>;
    constexpr int NT = NU * NU;
    constexpr int NL = NU * NU;                 // uz-lines per cell
    constexpr int NV = NU * NU * NU;
    extern __shared__ float lds[];
    __shared__ double red[3 * (NT / 64)];
    __shared__ double mred[4 * (NT / 64)];       // wave sums of the block's moments
    __shared__ float lmax[Codec<P>::scaled ? NL : 1];   // new uz-line scales
    const int t = threadIdx.x;
    const int ncell = (int)a.cells;             // the launcher checks the range
    int cell = blockIdx.x;
    if (cell >= ncell) return;                  // uniform over the work-group

    Slots R;
    R.load(fin, sin, a, cell, fresh_tid());
    R.put(lds, fresh_tid());
    float g[3];                                 // field of the cell in LDS (scalar)
#pragma unroll
    for (int k = 0; k < 3; ++k) g[k] = uniform_f32(R.g[k]);
    int next = uniform_sgpr(cell + (int)gridDim.x);
    if (next < ncell) R.load(fin, sin, a, next, fresh_tid());
    __syncthreads();

    const bool ofl = a.outflow != nullptr && !PER;
    const bool mom = a.rho != nullptr;
    int mcell = -1;                             // cell whose moment wave sums are in mred
    for (;;) {
        // moments of the block stored last round (published by the barrier
        // that ended it)
        if (mom && mcell >= 0 && t < 64) moments_total<NT>(mred, a, mcell);
        // the cell's outflow total so far, needed only after the sweeps
        double prev = 0.0;
        if (ofl && t == 0) prev = a.outflow[cell];
        float o[3];
        o[0] = kick_axis<P, NU, PER, 0>(lds, nullptr, nullptr, a, tab, cell, g[0], t);
        __syncthreads();
        o[1] = kick_axis<P, NU, PER, 1>(lds, nullptr, nullptr, a, tab, cell, g[1], t);
        __syncthreads();
        o[2] = kick_axis<P, NU, PER, 2>(lds, Codec<P>::scaled ? sout + (long)cell * NL + t : nullptr,
                                        lmax + t, a, tab, cell, g[2], t);
        if (ofl) wave_sums3<NT>(o, red);
        __syncthreads();
        if (ofl && t < 64) outflow_total<NT>(red, prev, a.du3, a.outflow + cell);

        // store the finished block; each slot is refilled with the next block
        // by the thread that stored it, so no barrier sits in between
        T* dst = fout + (long)cell * NV;
        const int ts = fresh_tid();
        // moments of what is stored (decoded codes for FP16/BF16), in FP64:
        // sum f, sum u_x f, sum u_y f, sum u_z f over this thread's slots
        double m[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < Slots::NS; ++s) {
            const int e = Slots::elem(s, ts);
            float* src = lds + (e / NU) * (NU + 1) + e % NU;
            const float inv = Codec<P>::scaled ? inv_scale(lmax[e / NU]) : 1.0f;
            Pack<T, 4> q;
#pragma unroll
            for (int u = 0; u < 4; ++u) q.v[u] = quantize<P>(src[u], inv);
            *reinterpret_cast<Pack<T, 4>*>(dst + e) = q;
            if (mom) {
                const float sc = Codec<P>::scaled ? lmax[e / NU] : 1.0f;
                const int jx = e / (NU * NU), jy = (e / NU) % NU, jz = e % NU;
                double s0 = 0.0, sz = 0.0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const double xv = (double)decode<P>(q.v[u], sc);
                    const double uz = a.umin[2] + ((double)(jz + u) + 0.5) * a.du[2];
                    s0 += xv;
                    sz = fma(uz, xv, sz);
                }
                const double ux = a.umin[0] + ((double)jx + 0.5) * a.du[0];
                const double uy = a.umin[1] + ((double)jy + 0.5) * a.du[1];
                m[0] += s0;
                m[1] = fma(ux, s0, m[1]);
                m[2] = fma(uy, s0, m[2]);
                m[3] += sz;
            }
        }
        if (mom) {
            double w[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) w[c] = wave_sum_f64(m[c]);
            if ((t & 63) == 0) {
#pragma unroll
                for (int c = 0; c < 4; ++c) mred[c * (NT / 64) + (t >> 6)] = w[c];
            }
            mcell = cell;
        }
        if (next >= ncell) break;
#pragma unroll
        for (int k = 0; k < 3; ++k) g[k] = uniform_f32(R.g[k]);
        R.put(lds, ts);
        cell = next;
        next = uniform_sgpr(cell + (int)gridDim.x);
        if (next < ncell) R.load(fin, sin, a, next, fresh_tid());
        __syncthreads();
    }
    if (mom) {
        __syncthreads();
        if (t < 64) moments_total<NT>(mred, a, mcell);
    }
}

// The split of every (cell, axis) shift of a kick, one thread each.
__global__ void __launch_bounds__(256) k_kick_shifts(KickArgs a, KickShift* __restrict__ tab)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * a.cells) return;
    const long cell = i / 3;
    const int axis = (int)(i - cell * 3);
    const LineShift sh = split_shift((double)a.g[(long)axis * a.cells + cell] * a.factor[axis],
                                     a.nu[axis], a.periodic);
    KickShift e;
    e.N = sh.N;
    e.flags = (sh.neg ? 1 : 0) | (sh.comp ? 2 : 0);
    e.mu = sh.mu;
    e.v0 = sh.v0; e.v1 = sh.v1; e.v2 = sh.v2; e.v3 = sh.v3;
    e.alpha = sh.alpha; e.q = sh.q; e.alpha_c = sh.alpha_c; e.muc = sh.muc;
    e.pad = 0.0f;
    tab[i] = e;
}

// ---------------------------------------------------------------------------
// uz sweep of long lines (nu_z = 64: a 64^3 FP32 block is 1 MiB, too large
// for the fused kick): a work-group of 256 threads walks one cell's 4096
// uz-lines in 16 tiles of 256 whole lines in LDS (padded to 65 floats), one
// line per thread with kick_axis_dir, while the tile after next is on its
// way from HBM into registers -- the kick's structure for one axis.  Loads
// and stores are 16-byte groups of consecutive values, so every access is
// coalesced; each thread owns a whole uz-line, so its new scale needs no
// reduction across lanes.  The line outflows are summed per thread over the
// cell's tiles, then over the work-group in a fixed order.
// ---------------------------------------------------------------------------
template <int P, int NU>
struct TileSlots {
    using T = typename Codec<P>::T;
    static constexpr int NT = 256;               // threads = lines per tile
    static constexpr int NS = NT * NU / (NT * 4); // 4-value groups per thread
    Pack<T, 4> q[NS];
    float sc[NS];
    __device__ static int elem(int s, int t) { return (s * NT + t) * 4; }
    __device__ void load(const T* __restrict__ src, const float* __restrict__ ssrc, int t)
    {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int e = elem(s, t);
            q[s] = *reinterpret_cast<const Pack<T, 4>*>(src + e);
            sc[s] = Codec<P>::scaled ? ssrc[e / NU] : 1.0f;
        }
    }
    __device__ void put(float* lds, int t) const
    {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int e = elem(s, t);
            float* dst = lds + (e / NU) * (NU + 1) + e % NU;
#pragma unroll
            for (int u = 0; u < 4; ++u) dst[u] = decode<P>(q[s].v[u], sc[s]);
        }
    }
};

template <int P, int NU, bool PER>
__global__ void __launch_bounds__(256) k_vel_uz_tiles(const typename Codec<P>::T* __restrict__ fin,
                                                     const float* __restrict__ sin,
                                                     typename Codec<P>::T* __restrict__ fout,
                                                     float* __restrict__ sout, VelArgs a)
{
    using T = typename Codec<P>::T;
    using Slots = TileSlots<P, NU>;
    constexpr int NT = Slots::NT;
    constexpr int NTILE = NU * NU / NT;          // tiles per cell
    constexpr int TE = NT * NU;                  // values per tile
    extern __shared__ float lds[];
    __shared__ float lmax[Codec<P>::scaled ? NT : 1];
    __shared__ double red[NT / 64];
    const int t = threadIdx.x;
    const long cell = blockIdx.x;
    const LineShift sh = split_shift((double)a.g[cell] * a.factor, NU, PER);
    const int N = uniform_sgpr(sh.N);
    const bool neg = uniform_sgpr(sh.neg ? 1 : 0) != 0;
    const T* src = fin + cell * (long)NU * NU * NU;
    const float* ssrc = sin + cell * (long)NU * NU;
    T* dst = fout + cell * (long)NU * NU * NU;
    float* sdst = sout + cell * (long)NU * NU;

    Slots R;
    R.load(src, ssrc, fresh_tid());
    R.put(lds, fresh_tid());
    R.load(src + TE, ssrc + NT, fresh_tid());
    __syncthreads();
    float ofl = 0.0f;
    for (int k = 0; k < NTILE; ++k) {
        float* line = lds + t * (NU + 1);
        float* sl = Codec<P>::scaled ? sdst + k * NT + t : nullptr;
        ofl += neg ? kick_axis_dir<P, NU, PER, 2, true>(line, sh, N, sl, lmax + t)
                   : kick_axis_dir<P, NU, PER, 2, false>(line, sh, N, sl, lmax + t);
        __syncthreads();
        const int ts = fresh_tid();
        T* out = dst + (long)k * TE;
#pragma unroll
        for (int s = 0; s < Slots::NS; ++s) {
            const int e = Slots::elem(s, ts);
            const float* v = lds + (e / NU) * (NU + 1) + e % NU;
            const float inv = Codec<P>::scaled ? inv_scale(lmax[e / NU]) : 1.0f;
            Pack<T, 4> q;
#pragma unroll
            for (int u = 0; u < 4; ++u) q.v[u] = quantize<P>(v[u], inv);
            *reinterpret_cast<Pack<T, 4>*>(out + e) = q;
        }
        __syncthreads();
        if (k + 1 < NTILE) {
            R.put(lds, ts);
            if (k + 2 < NTILE) R.load(src + (long)(k + 2) * TE, ssrc + (k + 2) * NT, fresh_tid());
        }
        __syncthreads();
    }
    if (a.outflow != nullptr && !PER) {
        const double tot = block_sum((double)ofl, red);
        if (t == 0) a.outflow[cell] += tot * a.du3;
    }
}

template <int P>
static hipError_t launch_vel_uz64_p(const void* fin, const float* sin, void* fout, float* sout,
                                    const VelArgs& a, hipStream_t st)
{
    using T = typename Codec<P>::T;
    constexpr int NU = 64;
    const size_t lds = (size_t)256 * (NU + 1) * sizeof(float);
    auto kern = a.periodic ? k_vel_uz_tiles<P, NU, true> : k_vel_uz_tiles<P, NU, false>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)a.cells), dim3(256), lds, st, (const T*)fin, sin,
                       (T*)fout, sout, a);
    return hipGetLastError();
}

hipError_t launch_vel_uz64(int prec, const void* fin, const float* sin, void* fout, float* sout,
                           const VelArgs& a, hipStream_t st)
{
    if (a.cells == 0) return hipSuccess;
    if (a.M != 64 || a.nsub != 64 * 64 || a.cells > 0x7fffffffL) return hipErrorInvalidValue;
    switch (prec) {
        case PREC_F16: return launch_vel_uz64_p<PREC_F16>(fin, sin, fout, sout, a, st);
        case PREC_BF16: return launch_vel_uz64_p<PREC_BF16>(fin, sin, fout, sout, a, st);
        default: return launch_vel_uz64_p<PREC_F32>(fin, sin, fout, sout, a, st);
    }
}

// ---------------------------------------------------------------------------
// uy and uz sweeps of 64^3 velocity blocks fused in LDS.  A 64^3 FP32 block
// (1 MiB) does not fit a work-group's LDS, but the eight u_x rows of a slab
// (jx0 .. jx0+7, all jy, all jz: 128 KiB, contiguous in HBM) hold whole
// u_y-lines and whole u_z-lines, so the last two sweeps of a half step run
// on it in LDS after the ux sweep (a separate launch).  Persistent
// work-groups of 512 threads walk cells blockIdx.x, +gridDim.x, ..., each
// cell's eight slabs in order, with the next slab on its way from HBM into
// registers while one is swept (the kick's structure); a thread owns one
// u_y-line and then one u_z-line of the slab.  The line outflows of a cell
// are summed per thread over its slabs and added to the cell's total, u_y
// before u_z, by wave 0 in a fixed order.
// ---------------------------------------------------------------------------
template <int P>
struct SlabSlots {
    using T = typename Codec<P>::T;
    static constexpr int NU = 64;
    static constexpr int NT = 512;                 // threads
    static constexpr int SX = 8;                   // u_x rows per slab
    static constexpr int SE = SX * NU * NU;        // values per slab
    static constexpr int NS = SE / (NT * 4);       // 4-value groups per thread
    Pack<T, 4> q[NS];
    float sc[NS];
    __device__ static int elem(int s, int t) { return (s * NT + t) * 4; }
    // slab k of a block: values k*SE .., uz-lines k*SX*NU ..
    __device__ void load(const T* src, const float* ssrc, int t)
    {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int e = elem(s, t);
            q[s] = *reinterpret_cast<const Pack<T, 4>*>(src + e);
            sc[s] = Codec<P>::scaled ? ssrc[e / NU] : 1.0f;
        }
    }
    __device__ void put(float* lds, int t) const
    {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int e = elem(s, t);
            float* dst = lds + (e / NU) * (NU + 1) + e % NU;
#pragma unroll
            for (int u = 0; u < 4; ++u) dst[u] = decode<P>(q[s].v[u], sc[s]);
        }
    }
};

// (fin may equal fout, and sin sout: every slab is read whole, by the one
// work-group that owns it, before that work-group writes it back, so the
// pointers carry no __restrict__)
template <int P, bool PER>
__global__ void __launch_bounds__(512) k_kick_yz64(const typename Codec<P>::T* fin,
                                                  const float* sin,
                                                  typename Codec<P>::T* fout,
                                                  float* sout, KickArgs a,
                                                  const KickShift* __restrict__ tab)
{
    using T = typename Codec<P>::T;
    using Slots = SlabSlots<P>;
    constexpr int NU = Slots::NU;
    constexpr int NT = Slots::NT;
    constexpr int SX = Slots::SX;
    constexpr int SE = Slots::SE;
    constexpr int NSLAB = NU / SX;
    constexpr long BLK = (long)NU * NU * NU;
    extern __shared__ float lds[];
    __shared__ float lmax[Codec<P>::scaled ? NT : 1];
    __shared__ double red[2 * (NT / 64)];
    const int t = threadIdx.x;
    const int ncell = (int)a.cells;            // the launcher checks the range
    int cell = blockIdx.x;
    if (cell >= ncell) return;                 // uniform over the work-group
    // thread t: u_y-line (jx = t / 64, jz = t % 64), then u_z-line (jx, jy = t % 64)
    const int ybase = (t / NU) * NU * (NU + 1) + (t % NU);
    const int zbase = t * (NU + 1);

    Slots R;
    R.load(fin + (long)cell * BLK, sin + (long)cell * NU * NU, fresh_tid());
    R.put(lds, fresh_tid());
    int slab = 0;
    // (cell, slab) of the slab in flight
    int ncl = NSLAB > 1 ? cell : cell + (int)gridDim.x;
    int nsl = NSLAB > 1 ? 1 : 0;
    if (ncl < ncell)
        R.load(fin + (long)ncl * BLK + (long)nsl * SE, sin + (long)ncl * NU * NU + nsl * SX * NU,
               fresh_tid());
    __syncthreads();
    float oy = 0.0f, oz = 0.0f;
    for (;;) {
        LineShift sy, sz;
        if (tab != nullptr) {
            const KickShift ey = tab[(long)cell * 3 + 1], ez = tab[(long)cell * 3 + 2];
            sy.N = ey.N; sy.neg = (ey.flags & 1) != 0; sy.comp = (ey.flags & 2) != 0;
            sy.mu = ey.mu; sy.v0 = ey.v0; sy.v1 = ey.v1; sy.v2 = ey.v2; sy.v3 = ey.v3;
            sy.alpha = ey.alpha; sy.q = ey.q; sy.alpha_c = ey.alpha_c; sy.muc = ey.muc;
            sz.N = ez.N; sz.neg = (ez.flags & 1) != 0; sz.comp = (ez.flags & 2) != 0;
            sz.mu = ez.mu; sz.v0 = ez.v0; sz.v1 = ez.v1; sz.v2 = ez.v2; sz.v3 = ez.v3;
            sz.alpha = ez.alpha; sz.q = ez.q; sz.alpha_c = ez.alpha_c; sz.muc = ez.muc;
        } else {
            sy = split_shift((double)a.g[a.cells + cell] * a.factor[1], NU, PER);
            sz = split_shift((double)a.g[2 * a.cells + cell] * a.factor[2], NU, PER);
        }
        const int Ny = uniform_sgpr(sy.N), Nz = uniform_sgpr(sz.N);
        oy += uniform_sgpr(sy.neg ? 1 : 0)
                  ? kick_axis_dir<P, NU, PER, 1, true>(lds + ybase, sy, Ny, nullptr, nullptr)
                  : kick_axis_dir<P, NU, PER, 1, false>(lds + ybase, sy, Ny, nullptr, nullptr);
        __syncthreads();
        float* sl = Codec<P>::scaled ? sout + (long)cell * NU * NU + slab * SX * NU + t : nullptr;
        oz += uniform_sgpr(sz.neg ? 1 : 0)
                  ? kick_axis_dir<P, NU, PER, 2, true>(lds + zbase, sz, Nz, sl, lmax + t)
                  : kick_axis_dir<P, NU, PER, 2, false>(lds + zbase, sz, Nz, sl, lmax + t);
        const bool last = slab == NSLAB - 1;
        const bool ofl = a.outflow != nullptr && !PER;
        if (ofl && last) {
            const double wy = wave_sum_f64((double)oy), wz = wave_sum_f64((double)oz);
            if ((t & 63) == 0) {
                red[t >> 6] = wy;
                red[NT / 64 + (t >> 6)] = wz;
            }
        }
        __syncthreads();
        if (ofl && last && t < 64) {
            const int k = t < 2 ? t : 0;
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) sum += red[k * (NT / 64) + w];
            const double ty = read_lane_f64(sum, 0), tz = read_lane_f64(sum, 1);
            if (t == 0) {
                double acc = a.outflow[cell];
                acc += ty * a.du3;
                acc += tz * a.du3;
                a.outflow[cell] = acc;
            }
        }
        if (last) {
            oy = 0.0f;
            oz = 0.0f;
        }
        // store the slab; each slot is refilled with the next slab by the
        // thread that stored it
        T* dst = fout + (long)cell * BLK + (long)slab * SE;
        const int ts = fresh_tid();
#pragma unroll
        for (int s = 0; s < Slots::NS; ++s) {
            const int e = Slots::elem(s, ts);
            const float* v = lds + (e / NU) * (NU + 1) + e % NU;
            const float inv = Codec<P>::scaled ? inv_scale(lmax[e / NU]) : 1.0f;
            Pack<T, 4> q;
#pragma unroll
            for (int u = 0; u < 4; ++u) q.v[u] = quantize<P>(v[u], inv);
            *reinterpret_cast<Pack<T, 4>*>(dst + e) = q;
        }
        if (ncl >= ncell) break;
        R.put(lds, ts);
        cell = ncl;
        slab = nsl;
        nsl = slab + 1;
        ncl = cell;
        if (nsl == NSLAB) {
            nsl = 0;
            ncl = cell + (int)gridDim.x;
        }
        ncl = uniform_sgpr(ncl);
        nsl = uniform_sgpr(nsl);
        if (ncl < ncell)
            R.load(fin + (long)ncl * BLK + (long)nsl * SE,
                   sin + (long)ncl * NU * NU + nsl * SX * NU, fresh_tid());
        __syncthreads();
    }
}

template <int P>
static hipError_t launch_kick_yz64_p(const void* fin, const float* sin, void* fout, float* sout,
                                     const KickArgs& a, const KickShift* tab, hipStream_t st)
{
    using T = typename Codec<P>::T;
    const size_t lds = (size_t)SlabSlots<P>::SX * 64 * 65 * sizeof(float);
    auto kern = a.periodic ? k_kick_yz64<P, true> : k_kick_yz64<P, false>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0, per_cu = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                          512, lds)) != hipSuccess)
        return e;
    long grid = (long)cus * (per_cu > 0 ? per_cu : 1);
    if (grid > a.cells) grid = a.cells;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(512), lds, st, (const T*)fin, sin, (T*)fout,
                       sout, a, tab);
    return hipGetLastError();
}

bool kick_yz64_supported(const int nu[3], size_t lds_limit)
{
    const size_t lds = (size_t)8 * 64 * 65 * sizeof(float) + 512 * sizeof(float) + 1024;
    return nu[0] == 64 && nu[1] == 64 && nu[2] == 64 && lds <= lds_limit;
}

hipError_t launch_kick_yz64(int prec, const void* fin, const float* sin, void* fout, float* sout,
                            const KickArgs& a, KickShift* shifts, hipStream_t st)
{
    if (a.cells == 0) return hipSuccess;
    if (a.cells > 0x7fffffffL) return hipErrorInvalidValue;   // cell indices are int
    if (shifts != nullptr) {
        const long n = 3 * a.cells;
        hipLaunchKernelGGL(k_kick_shifts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a,
                           shifts);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    switch (prec) {
        case PREC_F16: return launch_kick_yz64_p<PREC_F16>(fin, sin, fout, sout, a, shifts, st);
        case PREC_BF16: return launch_kick_yz64_p<PREC_BF16>(fin, sin, fout, sout, a, shifts, st);
        default: return launch_kick_yz64_p<PREC_F32>(fin, sin, fout, sout, a, shifts, st);
    }
}

template <int P, int N, bool PER>
static hipError_t launch_kick_t(const void* fin, const float* sin, void* fout, float* sout,
                                const KickArgs& a, const KickShift* tab, hipStream_t st)
{
    using T = typename Codec<P>::T;
    const size_t lds = (size_t)N * N * (N + 1) * sizeof(float);
    auto kern = k_kick<P, N, PER>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    // persistent grid: as many work-groups as are resident at once
    int dev = 0, cus = 0, per_cu = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                          N * N, lds)) != hipSuccess)
        return e;
    long grid = (long)cus * (per_cu > 0 ? per_cu : 1);
    if (grid > a.cells) grid = a.cells;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(N * N), lds, st, (const T*)fin, sin,
                       (T*)fout, sout, a, tab);
    return hipGetLastError();
}

template <int P>
static hipError_t launch_kick_p(const void* fin, const float* sin, void* fout, float* sout,
                                const KickArgs& a, const KickShift* tab, hipStream_t st)
{
    if (a.nu[0] == 32) {
        return a.periodic ? launch_kick_t<P, 32, true>(fin, sin, fout, sout, a, tab, st)
                          : launch_kick_t<P, 32, false>(fin, sin, fout, sout, a, tab, st);
    }
    return a.periodic ? launch_kick_t<P, 16, true>(fin, sin, fout, sout, a, tab, st)
                      : launch_kick_t<P, 16, false>(fin, sin, fout, sout, a, tab, st);
}

bool kick_supported(const int nu[3], size_t lds_limit)
{
    if (nu[0] != nu[1] || nu[1] != nu[2]) return false;
    if (nu[0] != 16 && nu[0] != 32) return false;
    const size_t lds = (size_t)nu[0] * nu[0] * (nu[0] + 1) * sizeof(float);
    return lds <= lds_limit;
}

hipError_t launch_kick(int prec, const void* fin, const float* sin, void* fout, float* sout,
                       const KickArgs& a, KickShift* shifts, hipStream_t st)
{
    if (a.cells == 0) return hipSuccess;
    if (a.cells > 0x7fffffffL) return hipErrorInvalidValue;   // cell indices are int
    if (shifts != nullptr) {
        const long n = 3 * a.cells;
        hipLaunchKernelGGL(k_kick_shifts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a,
                           shifts);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    switch (prec) {
        case PREC_F16: return launch_kick_p<PREC_F16>(fin, sin, fout, sout, a, shifts, st);
        case PREC_BF16: return launch_kick_p<PREC_BF16>(fin, sin, fout, sout, a, shifts, st);
        default: return launch_kick_p<PREC_F32>(fin, sin, fout, sout, a, shifts, st);
    }
}

}  // namespace vlasov
