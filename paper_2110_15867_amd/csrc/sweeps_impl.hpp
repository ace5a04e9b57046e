// Sweep kernels of the split SL-MPP5 Vlasov solver for gfx950 (templates;
// sweeps_f32/f16/bf16.hip instantiate one storage precision each, so the
// three compile in parallel).
//
// Layout f[ix][iy][iz][jx][jy][jz] (jz fastest).  A line along axis l is
// addressed as (o * M + i) * I + k: o runs over the axes before l, i along l,
// k over the axes after l ("inner", contiguous).  Three kernel families:
//
//  * k_position   x, y, z (Eq. 3).  One thread per V adjacent inner indices;
//                 neighbouring lanes read neighbouring addresses of the same
//                 row, so every row access is coalesced without a transpose.
//                 The shift follows the velocity index along l.  Waves whose
//                 lanes all move the same way use the mirrored 5-cell walker;
//                 waves with both signs (the z sweep, shift set by the
//                 contiguous u_z index) use the 6-cell walker with selects.
//  * k_vel_strided ux, uy (Eq. 4).  One work-group per spatial cell: the
//                 shift is g(x) dt / du, uniform over the velocity block, so
//                 the walk direction and row addresses are wave-uniform.
//                 The outflow through the velocity faces is reduced per cell
//                 in FP64 in a fixed order.
//  * k_vel_uz     uz.  The lines are contiguous (nu_z values), the case the
//                 paper solves with its load-and-transpose (section 5.3): a
//                 work-group loads a tile of whole lines with coalesced
//                 16-byte loads into LDS, each thread walks one line out of
//                 LDS, results go back through LDS and leave coalesced.
//
// Storage FP32, or FP16/BF16 codes with one FP32 scale per uz-line; the
// scale of an output line is the largest |value| of that line, reduced
// across the lanes that hold it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.hpp"
#include "rows.hpp"
#include "sl_mpp5.hpp"

namespace vlasov {

// ---------------------------------------------------------------------------
// Position sweeps
// ---------------------------------------------------------------------------
// (at least four work-groups of 256 per CU: the compiler keeps every variant
// within 128 VGPRs, four waves per SIMD -- the FP16/BF16 y walk with
// per-lane shifts would otherwise take 144 and run three)
template <int P, int V, int MT, int GC, bool US, bool MIX>
__global__ void __launch_bounds__(256, 4) k_position(const typename Codec<P>::T* __restrict__ fin,
                                                  const float* __restrict__ sin,
                                                  typename Codec<P>::T* __restrict__ fout,
                                                  float* __restrict__ sout, PosArgs a)
{
    const long IV = a.I / V;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = a.O * IV;
    if (t >= total) return;
    long o = t / IV;
    long k = (t - o * IV) * V;
    long k0w = 0;                                  // gathered mapping: lane 0's element
    const bool gathered = !Codec<P>::scaled && a.ug > 0;
    if constexpr (US) {
        if (gathered) {
            // Gathered mapping (y sweep).  A wave holds R = a.ug uz-lines,
            // one from each of R consecutive u_x rows, all at the same u_y:
            // lane l takes elements (l % G) V .. +V-1 of uz-line l / G
            // (G = nu_z / V lanes per line).  A unit (o, spatial cell of
            // the row, group of R u_x rows) has nu_y such waves, 4 to a
            // work-group, Q = nu_y / 4 work-groups.  Work-groups go to the
            // eight XCDs in turn, so the Q work-groups of a unit are taken
            // eight apart: they run on one XCD, whose L2 then holds the
            // 128-byte lines (scales, FP16 codes of neighbouring u_y) that
            // they share.  The host checks that the units fill whole
            // groups of eight.
            const long Q = a.nshift / 4;
            const long b = blockIdx.x;
            const long sup = b / (8 * Q);
            const long rem = b - sup * 8 * Q;
            const long unit = sup * 8 + rem % 8;
            const long jy = (rem / 8) * 4 + (threadIdx.x >> 6);
            const int lane = (int)(threadIdx.x & 63);
            const long ngx = a.nux / a.ug;              // u_x groups per block
            const long upr = (a.I / a.Nu) * ngx;        // units per row
            o = unit / upr;
            const long ur = unit - o * upr;
            const long blk = ur / ngx;
            const long jxg = ur - blk * ngx;
            const int G = (int)(a.nuz / V);
            const int rr = lane / G;
            k0w = blk * a.Nu + (jxg * a.ug * a.nshift + jy) * a.nuz;
            k = k0w + ((long)rr * a.nshift) * a.nuz + (long)(lane - rr * G) * V;
        }
    }
    const int M = MT > 0 ? MT : a.M;
    const int jl = (int)(((k % a.Nu) / a.pst) % a.nshift);
    const LineShift sh = split_shift(a.shift[jl], M, true);

    const long lbase = o * (long)M * a.I + k;
    const long sI = a.I / a.nuz;                 // uz-lines per row
    const long sb = o * (long)M * sI + k / a.nuz;

    if constexpr (US) {
        // The host guarantees that every lane of a wave has the same shift
        // (x sweeps: a wave's elements share u_x; gathered y sweeps: u_y)
        // and that rows hold whole waves: one direction, one integer shift,
        // wave-uniform row addresses and line constants in scalar registers.
        const LineShift shu = uniform_shift(sh);
        const long t0 = t - (threadIdx.x & 63);
        // the wave's row and first element (lane 0's)
        const long o0 = gathered ? o : t0 / IV;
        const long k0 = gathered ? uniform_long(k0w) : (t0 - o0 * IV) * V;
        const long ub = uniform_long(o0 * (long)M * a.I + k0);
        const long usb = uniform_long(o0 * (long)M * sI + k0 / a.nuz);
        const unsigned loff = (unsigned)((k - k0) * (long)sizeof(typename Codec<P>::T));
        const unsigned soff = (unsigned)((k / a.nuz - k0 / a.nuz) * (long)sizeof(float));
        const unsigned nb = (unsigned)uniform_sgpr(
            (int)row_span_bytes((a.I - k0) * (long)sizeof(typename Codec<P>::T)));
        const unsigned snb = (unsigned)uniform_sgpr((int)row_span_bytes((sI - k0 / a.nuz) * (long)sizeof(float)));
        const int r0 = a.skew ? uniform_sgpr((int)(((t0 >> 6) * 17) % M)) : 0;
        const int dir = shu.neg ? -1 : 1;
        URowReader<P, V> rd{fin + ub, sin + (Codec<P>::scaled ? usb : 0), loff, soff, nb, snb, a.I, sI, M, dir, r0, 0};
        URowWriter<P, V, GC> wr{fout + ub, sout + (Codec<P>::scaled ? usb : 0), loff, soff, nb, snb, a.I, sI, M, dir, r0, a.G};
        walk_uniform<V, MT, true>(rd, wr, M, shu, true, nullptr);
        return;
    }
    const unsigned long long neg_lanes = __ballot(sh.neg);
    const unsigned long long act = __ballot(1);
    const bool one_dir = neg_lanes == 0 || neg_lanes == act;
    // Every lane of the wave visits the same rows when the integer shift is
    // the same (for the mixed walker: the signed one).  Waves never straddle
    // two values of o (a.I / V is a multiple of the wave size), so the
    // lanes' elements then differ by a fixed in-row offset.
    const int Ns = sh.neg ? -sh.N : sh.N;
    const int key = one_dir ? sh.N : Ns;
    const int key0 = __builtin_amdgcn_readfirstlane(key);
    const bool full = act == ~0ull && (a.I / V) % 64 == 0;
    const bool urows = full && __ballot(key == key0) == act;
    if (urows) {
        const long t0 = t - (threadIdx.x & 63);          // lane 0 of this wave
        const long o0 = t0 / IV;
        const long k0 = (t0 - o0 * IV) * V;
        // (wave-uniform, kept in scalar registers: the row addresses are then
        // SGPR bases and each access adds only the lane's 32-bit offset)
        const long ub = uniform_long(o0 * (long)M * a.I + k0);
        const long usb = uniform_long(o0 * (long)M * sI + k0 / a.nuz);
        const unsigned loff = (unsigned)((k - k0) * (long)sizeof(typename Codec<P>::T));
        const unsigned soff = (unsigned)((k / a.nuz - k0 / a.nuz) * (long)sizeof(float));
        // bytes from the wave's first element (scale) to the end of its row
        const unsigned nb = (unsigned)uniform_sgpr(
            (int)row_span_bytes((a.I - k0) * (long)sizeof(typename Codec<P>::T)));
        const unsigned snb = (unsigned)uniform_sgpr((int)row_span_bytes((sI - k0 / a.nuz) * (long)sizeof(float)));
        LineShift shu = sh;
        shu.N = uniform_sgpr(sh.N);
        // x and y: each wave starts its walk at its own row (see URowWriter)
        const int r0 = a.skew ? uniform_sgpr((int)(((t0 >> 6) * 17) % M)) : 0;
        if (!MIX || one_dir) {
            const int dir = uniform_sgpr(sh.neg ? -1 : 1);
            URowReader<P, V> rd{fin + ub, sin + (Codec<P>::scaled ? usb : 0), loff, soff, nb, snb, a.I, sI, M, dir, r0, 0};
            URowWriter<P, V, GC> wr{fout + ub, sout + (Codec<P>::scaled ? usb : 0), loff, soff, nb, snb, a.I, sI, M, dir, r0, a.G};
            walk_uniform<V, MT, false>(rd, wr, M, shu, true, nullptr);
        } else if constexpr (MIX) {
            URowReader<P, V> rd{fin + ub, sin + (Codec<P>::scaled ? usb : 0), loff, soff, nb, snb, a.I, sI, M, 1, r0, 0};
            URowWriter<P, V, GC> wr{fout + ub, sout + (Codec<P>::scaled ? usb : 0), loff, soff, nb, snb, a.I, sI, M, 1, r0, a.G};
            walk_mixed<V, MT>(rd, wr, M, uniform_sgpr(Ns), shu);
        }
    } else if (!MIX || one_dir) {
        const int dir = sh.neg ? -1 : 1;
        GlobalReader<P, V> rd{fin + lbase, sin + (Codec<P>::scaled ? sb : 0), a.I, sI, M, dir, true, 0};
        GlobalWriter<P, V, GC> wr{fout + lbase, sout + (Codec<P>::scaled ? sb : 0), a.I, sI, M, dir, a.G};
        walk_uniform<V, MT, false>(rd, wr, M, sh, true, nullptr);
    } else if constexpr (MIX) {
        GlobalReader<P, V> rd{fin + lbase, sin + (Codec<P>::scaled ? sb : 0), a.I, sI, M, 1, true, 0};
        GlobalWriter<P, V, GC> wr{fout + lbase, sout + (Codec<P>::scaled ? sb : 0), a.I, sI, M, 1, a.G};
        walk_mixed<V, MT>(rd, wr, M, Ns, sh);
    }
}

// ---------------------------------------------------------------------------
// z sweep with paired lines.  The shift follows the contiguous u_z index;
// the host takes this path only when every line of the upper half of a
// uz-line (u_z > 0) moves up and every line of the lower half moves down,
// all by less than one cell, H = nu_z / 2 divides the wave and a row holds
// whole waves of lanes.  Each lane then owns one line of each half (see
// PairRowReader), every wave visits uniform rows (buffer addressing, one
// coalesced access per row) and runs two select-free walks.  Results are
// the bits of the per-lane mixed walk.
// ---------------------------------------------------------------------------
// (at least six work-groups per CU: 80 VGPRs, six waves per SIMD instead of
// five; the few values this spills cost less than the latency it hides)
template <int P, int MT, int H>
__global__ void __launch_bounds__(256, 6) k_position_pair(const typename Codec<P>::T* __restrict__ fin,
                                                       const float* __restrict__ sin,
                                                       typename Codec<P>::T* __restrict__ fout,
                                                       float* __restrict__ sout, PosArgs a)
{
    using T = typename Codec<P>::T;
    constexpr int NUZ = 2 * H;
    const long IP = a.I / 2;                      // lanes per row
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.O * IP) return;                    // whole waves (IP % 64 == 0)
    const long o = t / IP;
    const long kp = t - o * IP;
    const long q = kp / H;                        // uz-line within the row
    const int g = (int)(kp - q * H);              // lane within the uz-line
    const bool lo = g < H / 2;
    const int up = lo ? 2 * g + H : 2 * g + 1;    // velocity index of this lane's A line
    const int dn = lo ? 2 * g : 2 * g - H + 1;    // ... and of its B line
    const LineShift sa = split_shift(a.shift[up], MT, true);
    const LineShift sb = split_shift(a.shift[dn], MT, true);

    const long t0 = t - (threadIdx.x & 63);       // lane 0 of this wave
    const long o0 = t0 / IP;
    const long q0 = (t0 - o0 * IP) / H;
    const long sI = a.I / NUZ;
    const long ub = uniform_long(o0 * (long)MT * a.I + q0 * NUZ);
    const long usb = uniform_long(o0 * (long)MT * sI + q0);
    const unsigned off = (unsigned)(((q - q0) * NUZ + 2 * g) * (long)sizeof(T));
    const unsigned soff = (unsigned)((q - q0) * (long)sizeof(float));
    const unsigned nb = (unsigned)uniform_sgpr((int)row_span_bytes((a.I - q0 * NUZ) * (long)sizeof(T)));
    const unsigned snb = (unsigned)uniform_sgpr((int)row_span_bytes((sI - q0) * (long)sizeof(float)));
    PairRowReader<P, H> rd{fin + ub, Codec<P>::scaled ? sin + usb : nullptr, off, soff, nb, snb,
                           a.I, sI, MT, lo, 0};
    PairRowWriter<P, H> wr{fout + ub, Codec<P>::scaled ? sout + usb : nullptr, off, soff, nb, snb,
                           a.I, sI, lo};
    walk_pair<MT>(rd, wr, sa, sb);
}

// ---------------------------------------------------------------------------
// Velocity sweeps ux, uy: one work-group per spatial cell
// ---------------------------------------------------------------------------
template <int P, int V, int MT>
__global__ void __launch_bounds__(256) k_vel_strided(const typename Codec<P>::T* __restrict__ fin,
                                                     const float* __restrict__ sin,
                                                     typename Codec<P>::T* __restrict__ fout,
                                                     float* __restrict__ sout, VelArgs a)
{
    __shared__ double red[4];
    const long cell = blockIdx.x;
    const int M = MT > 0 ? MT : a.M;
    const double s = (double)a.g[cell] * a.factor;
    const LineShift sh = split_shift(s, M, a.periodic);
    const int dir = sh.neg ? -1 : 1;
    const long IV = a.I / V;
    const long lpc = (long)a.nsub * IV;
    const long sI = a.I / a.nuz;
    double mine = 0.0;
    for (long l = threadIdx.x; l < lpc; l += blockDim.x) {
        const long sub = l / IV;
        const long k = (l - sub * IV) * V;
        const long o = cell * a.nsub + sub;
        const long lbase = o * (long)M * a.I + k;
        const long sb = o * (long)M * sI + k / a.nuz;
        GlobalReader<P, V> rd{fin + lbase, sin + (Codec<P>::scaled ? sb : 0), a.I, sI, M, dir, a.periodic, 0};
        GlobalWriter<P, V> wr{fout + lbase, sout + (Codec<P>::scaled ? sb : 0), a.I, sI, M, dir, a.G};
        float ofl = 0.0f;
        walk_uniform<V, MT, true>(rd, wr, M, sh, a.periodic, &ofl);
        mine += (double)ofl;
    }
    if (a.outflow != nullptr && !a.periodic) {
        const double tot = block_sum(mine, red);
        if (threadIdx.x == 0) a.outflow[cell] += tot * a.du3;
    }
}

// ---------------------------------------------------------------------------
// Velocity sweep uz: contiguous lines staged through LDS
// ---------------------------------------------------------------------------
template <int P, int MT, int NT>
__global__ void __launch_bounds__(NT) k_vel_uz(const typename Codec<P>::T* __restrict__ fin,
                                              const float* __restrict__ sin,
                                              typename Codec<P>::T* __restrict__ fout,
                                              float* __restrict__ sout, VelArgs a)
{
    using T = typename Codec<P>::T;
    constexpr int LS = MT + 1;                  // padded line stride in LDS
    __shared__ float tile[NT * LS];
    __shared__ double red[NT / 64];
    const long cell = blockIdx.x;
    const double s = (double)a.g[cell] * a.factor;
    const LineShift sh = split_shift(s, MT, a.periodic);
    const int dir = sh.neg ? -1 : 1;
    const long lpc = a.nsub;                    // lines per cell = nux * nuy
    const long cbase = cell * lpc;              // first line of the cell
    double mine = 0.0;
    for (long l0 = 0; l0 < lpc; l0 += NT) {
        const int nl = (int)((lpc - l0) < NT ? (lpc - l0) : NT);
        const long gline = cbase + l0;
        // coalesced load of nl whole lines, 4 values per access
        const T* src = fin + gline * MT;
        for (int e = threadIdx.x * 4; e < nl * MT; e += NT * 4) {
            const int ln = e / MT;
            const int off = e - ln * MT;
            const float sc = Codec<P>::scaled ? sin[gline + ln] : 1.0f;
            float x[4];
            load_row<P, 4>(src + e, sc, x);
#pragma unroll
            for (int q = 0; q < 4; ++q) tile[ln * LS + off + q] = x[q];
        }
        __syncthreads();
        RegWriter<MT> wr;
        float ofl = 0.0f;
        if (threadIdx.x < nl) {
            LdsReader rd{tile + threadIdx.x * LS, 1, MT, dir, a.periodic, 0};
            walk_uniform<1, MT, true>(rd, wr, MT, sh, a.periodic, &ofl);
            mine += (double)ofl;
        }
        __syncthreads();
        if (threadIdx.x < nl) {
            float inv = 1.0f;
            if (Codec<P>::scaled) {
                float m = 0.0f;
#pragma unroll
                for (int i = 0; i < MT; ++i) m = fmaxf(m, fabsf(wr.out[i]));
                inv = inv_scale(m);
                sout[gline + threadIdx.x] = m;
            }
            float* line = tile + threadIdx.x * LS;
#pragma unroll
            for (int i = 0; i < MT; ++i) line[dir > 0 ? i : MT - 1 - i] = wr.out[i] * inv;
        }
        __syncthreads();
        T* dst = fout + gline * MT;
        for (int e = threadIdx.x * 4; e < nl * MT; e += NT * 4) {
            const int ln = e / MT;
            const int off = e - ln * MT;
            Pack<T, 4> q;
#pragma unroll
            for (int u = 0; u < 4; ++u) q.v[u] = Codec<P>::enc(tile[ln * LS + off + u]);
            *reinterpret_cast<Pack<T, 4>*>(dst + e) = q;
        }
        __syncthreads();
    }
    if (a.outflow != nullptr && !a.periodic) {
        const double tot = block_sum(mine, red);
        if (threadIdx.x == 0) a.outflow[cell] += tot * a.du3;
    }
}

// Fallback for line lengths without a tiled kernel: one thread per contiguous
// line straight from global memory (two passes for scaled storage).
template <int P>
__global__ void __launch_bounds__(256) k_vel_uz_generic(const typename Codec<P>::T* __restrict__ fin,
                                                       const float* __restrict__ sin,
                                                       typename Codec<P>::T* __restrict__ fout,
                                                       float* __restrict__ sout, VelArgs a)
{
    __shared__ double red[4];
    const long cell = blockIdx.x;
    const int M = a.M;
    const double s = (double)a.g[cell] * a.factor;
    const LineShift sh = split_shift(s, M, a.periodic);
    const int dir = sh.neg ? -1 : 1;
    double mine = 0.0;
    for (long l = threadIdx.x; l < a.nsub; l += blockDim.x) {
        const long line = cell * a.nsub + l;
        const float sc = Codec<P>::scaled ? sin[line] : 1.0f;
        GlobalReader<P, 1, false> rd{fin + line * M, nullptr, 1, 0, M, dir, a.periodic, 0};
        float ofl = 0.0f;
        float inv = 1.0f;
        if (Codec<P>::scaled) {
            // pass 1: the output scale
            struct ScaledReader {
                GlobalReader<P, 1, false> g;
                float sc;
                __device__ void seek(int r) { g.seek(r); }
                __device__ void next(float* x) { g.next(x); x[0] *= sc; }
            };
            ScaledReader srd{rd, sc};
            MaxWriter mw{0.0f};
            walk_uniform<1, 0, true>(srd, mw, M, sh, a.periodic, &ofl);
            inv = inv_scale(mw.m);
            sout[line] = mw.m;
            ScaledReader srd2{rd, sc};
            ContigWriter<P> cw{fout + line * M, M, dir, inv};
            walk_uniform<1, 0, true>(srd2, cw, M, sh, a.periodic, &ofl);
        } else {
            ContigWriter<P> cw{fout + line * M, M, dir, 1.0f};
            walk_uniform<1, 0, true>(rd, cw, M, sh, a.periodic, &ofl);
        }
        mine += (double)ofl;
    }
    if (a.outflow != nullptr && !a.periodic) {
        const double tot = block_sum(mine, red);
        if (threadIdx.x == 0) a.outflow[cell] += tot * a.du3;
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int P, int V>
inline hipError_t launch_position_v(const void* fin, const float* sin, void* fout, float* sout,
                                    const PosArgs& a, hipStream_t st)
{
    using T = typename Codec<P>::T;
    const long total = a.O * (a.I / V);
    const unsigned blocks = (unsigned)((total + 255) / 256);
    if (total == 0) return hipSuccess;
    // Paired z walks for FP16/BF16 storage, where the z sweep is bound by
    // its vector ALU work; with FP32 storage it is bound by memory and the
    // per-lane walk, with half the bytes per wave row, measured faster.
    if constexpr (V == 1 && Codec<P>::scaled) if (a.pair != 0) {
        // the host checked: nu_z in {16, 32, 64}, M in {16, 32, 64}
        const unsigned pblocks = (unsigned)((a.O * (a.I / 2) + 255) / 256);
#define VL_PAIR(MTV, HV) \
    hipLaunchKernelGGL((k_position_pair<P, MTV, HV>), dim3(pblocks), dim3(256), 0, st, (const T*)fin, sin, (T*)fout, sout, a)
#define VL_PAIR_M(HV) \
    switch (a.M) { case 16: VL_PAIR(16, HV); break; case 32: VL_PAIR(32, HV); break; default: VL_PAIR(64, HV); break; }
        if (a.nuz == 16) { VL_PAIR_M(8) }
        else if (a.nuz == 32) { VL_PAIR_M(16) }
        else { VL_PAIR_M(32) }
#undef VL_PAIR_M
#undef VL_PAIR
        return hipGetLastError();
    }
    // uz-lines of 32 values (the usual velocity block) get the compile-time
    // group size of the scale reduction
    constexpr int G32 = Codec<P>::scaled ? 32 / V : 0;
    const bool g32 = G32 > 0 && a.G == G32;
    // waves whose lanes all share the shift (x sweeps) get the variant with
    // the line constants in scalar registers; where no wave holds lanes of
    // both directions (y sweeps of the usual blocks) the mixed walk is left
    // out, which frees registers
    const bool us = (a.us != 0 || (a.ug > 0 && !Codec<P>::scaled)) && V == 4;
    const bool mix = a.mix != 0 || V != 4;
#define VL_POS(MTV) \
    if (us && g32) hipLaunchKernelGGL((k_position<P, V, MTV, G32, true, false>), dim3(blocks), dim3(256), 0, st, (const T*)fin, sin, (T*)fout, sout, a); \
    else if (us) hipLaunchKernelGGL((k_position<P, V, MTV, 0, true, false>), dim3(blocks), dim3(256), 0, st, (const T*)fin, sin, (T*)fout, sout, a); \
    else if (!mix && g32) hipLaunchKernelGGL((k_position<P, V, MTV, G32, false, false>), dim3(blocks), dim3(256), 0, st, (const T*)fin, sin, (T*)fout, sout, a); \
    else if (!mix) hipLaunchKernelGGL((k_position<P, V, MTV, 0, false, false>), dim3(blocks), dim3(256), 0, st, (const T*)fin, sin, (T*)fout, sout, a); \
    else if (g32) hipLaunchKernelGGL((k_position<P, V, MTV, G32, false, true>), dim3(blocks), dim3(256), 0, st, (const T*)fin, sin, (T*)fout, sout, a); \
    else hipLaunchKernelGGL((k_position<P, V, MTV, 0, false, true>), dim3(blocks), dim3(256), 0, st, (const T*)fin, sin, (T*)fout, sout, a)
    switch (a.M) {
        case 16: VL_POS(16); break;
        case 32: VL_POS(32); break;
        case 64: VL_POS(64); break;
        default: VL_POS(0); break;
    }
#undef VL_POS
    return hipGetLastError();
}

template <int P>
inline hipError_t launch_position_p(const void* fin, const float* sin, void* fout, float* sout,
                                    const PosArgs& a, hipStream_t st)
{
    switch (a.V) {
        case 4: return launch_position_v<P, 4>(fin, sin, fout, sout, a, st);
        case 2: return launch_position_v<P, 2>(fin, sin, fout, sout, a, st);
        default: return launch_position_v<P, 1>(fin, sin, fout, sout, a, st);
    }
}


template <int P, int V>
inline hipError_t launch_vel_strided_v(const void* fin, const float* sin, void* fout, float* sout,
                                       const VelArgs& a, hipStream_t st)
{
    using T = typename Codec<P>::T;
    if (a.cells == 0) return hipSuccess;
    const long lpc = (long)a.nsub * (a.I / V);
    long bs = ((lpc + 63) / 64) * 64;
    if (bs > 256) bs = 256;
#define VL_VEL(MTV) \
    hipLaunchKernelGGL((k_vel_strided<P, V, MTV>), dim3((unsigned)a.cells), dim3((unsigned)bs), 0, st, (const T*)fin, sin, (T*)fout, sout, a)
    switch (a.M) {
        case 16: VL_VEL(16); break;
        case 32: VL_VEL(32); break;
        case 64: VL_VEL(64); break;
        default: VL_VEL(0); break;
    }
#undef VL_VEL
    return hipGetLastError();
}

template <int P>
inline hipError_t launch_vel_strided_p(const void* fin, const float* sin, void* fout, float* sout,
                                       const VelArgs& a, hipStream_t st)
{
    switch (a.V) {
        case 4: return launch_vel_strided_v<P, 4>(fin, sin, fout, sout, a, st);
        case 2: return launch_vel_strided_v<P, 2>(fin, sin, fout, sout, a, st);
        default: return launch_vel_strided_v<P, 1>(fin, sin, fout, sout, a, st);
    }
}


template <int P>
inline hipError_t launch_vel_uz_p(const void* fin, const float* sin, void* fout, float* sout,
                                  const VelArgs& a, hipStream_t st)
{
    using T = typename Codec<P>::T;
    if (a.cells == 0) return hipSuccess;
    const dim3 grid((unsigned)a.cells);
    switch (a.M) {
        case 16:
            hipLaunchKernelGGL((k_vel_uz<P, 16, 256>), grid, dim3(256), 0, st, (const T*)fin, sin, (T*)fout, sout, a);
            break;
        case 32:
            hipLaunchKernelGGL((k_vel_uz<P, 32, 256>), grid, dim3(256), 0, st, (const T*)fin, sin, (T*)fout, sout, a);
            break;
        case 64:
            // cubic 64^3 blocks: double-buffered tiles (kick.hip)
            if (a.nsub == 64 * 64) return launch_vel_uz64(P, fin, sin, fout, sout, a, st);
            hipLaunchKernelGGL((k_vel_uz<P, 64, 128>), grid, dim3(128), 0, st, (const T*)fin, sin, (T*)fout, sout, a);
            break;
        default: {
            long bs = ((a.nsub + 63) / 64) * 64;
            if (bs > 256) bs = 256;
            hipLaunchKernelGGL((k_vel_uz_generic<P>), grid, dim3((unsigned)bs), 0, st, (const T*)fin, sin, (T*)fout, sout, a);
        }
    }
    return hipGetLastError();
}


}  // namespace vlasov
