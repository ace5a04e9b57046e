// Row readers and writers shared by the sweep kernels: they turn a frame row
// of one line into FP32 values (periodic wrap or zero ghosts, mirrored walk,
// decoding of FP16/BF16 codes) and store results (encoding with the per
// uz-line scale).  Also the fixed-order FP64 work-group sum.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sl_mpp5.hpp"

namespace vlasov {

// ---------------------------------------------------------------------------
// Row readers and writers
// ---------------------------------------------------------------------------

// Rows of a strided line in global memory.  Frame row r maps to physical row
// r (dir > 0) or M-1-r (mirrored); periodic lines wrap, others read zero
// outside [0, M).
template <int P, int V, bool SCALED = Codec<P>::scaled>
struct GlobalReader {
    using T = typename Codec<P>::T;
    const T* base;        // element (o, row 0, k)
    const float* sbase;   // scale of (o, row 0, k) (scaled storage)
    long stride;          // elements between rows
    long sstride;         // scales between rows
    int M;
    int dir;
    bool periodic;
    int phys;

    __device__ void seek(int r)
    {
        int q = dir > 0 ? r : M - 1 - r;
        if (periodic) {
            q %= M;
            if (q < 0) q += M;
        }
        phys = q;
    }
    // Each row address is computed from the row index (no running pointer):
    // the loads of an unrolled walk stay independent of each other and of
    // the wrap selects, so they can all be issued early.
    __device__ void next(float* x)
    {
        if (periodic || (phys >= 0 && phys < M)) {
            const float sc = SCALED ? sbase[(long)phys * sstride] : 1.0f;
            load_row<P, V>(base + (long)phys * stride, sc, x);
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) x[v] = 0.0f;
        }
        phys += dir;
        if (periodic) {
            if (phys == M) phys = 0;
            else if (phys < 0) phys = M - 1;
        }
    }
};

// Largest value over aligned groups of G lanes (G a power of two <= 64), in
// every lane of the group: DPP quad permutations and row mirrors within a
// 16-lane row, a swizzle across 32, a permute across 64.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
        __builtin_bit_cast(int, v), __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float group_max(float m, int G)
{
    // every step runs; the group size only selects whether the partner's
    // value counts (branch-free, so unrolled walks keep one basic block)
    float q;
    q = dpp_mov<0xB1>(m);                          // quad_perm [1,0,3,2]
    m = fmaxf(m, G >= 2 ? q : m);
    q = dpp_mov<0x4E>(m);                          // quad_perm [2,3,0,1]
    m = fmaxf(m, G >= 4 ? q : m);
    q = dpp_mov<0x141>(m);                         // row_half_mirror
    m = fmaxf(m, G >= 8 ? q : m);
    q = dpp_mov<0x140>(m);                         // row_mirror
    m = fmaxf(m, G >= 16 ? q : m);
    // swizzle, bit mode: lane ^ 16 within each half of the wave
    q = __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, m), 0x401F));
    m = fmaxf(m, G >= 32 ? q : m);
    q = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(
            (int)((threadIdx.x ^ 32) & 63) << 2, __builtin_bit_cast(int, m)));
    m = fmaxf(m, G >= 64 ? q : m);
    return m;
}

// The same for a group size fixed at compile time, on values >= 0: their
// IEEE bit patterns order like unsigned integers, so each step is a single
// v_max_u32 with a DPP operand (no canonicalising of DPP results, no select).
template <int CTRL>
__device__ __forceinline__ unsigned dpp_mov_u(unsigned v)
{
    // old = 0 (the identity of max) lets the move fold into v_max_u32_dpp
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, true);
}

template <int G>
__device__ __forceinline__ float group_max_nonneg(float m)
{
    unsigned u = __builtin_bit_cast(unsigned, m);
    if (G >= 2) u = max(u, dpp_mov_u<0xB1>(u));       // quad_perm [1,0,3,2]
    if (G >= 4) u = max(u, dpp_mov_u<0x4E>(u));       // quad_perm [2,3,0,1]
    if (G >= 8) u = max(u, dpp_mov_u<0x141>(u));      // row_half_mirror
    if (G >= 16) u = max(u, dpp_mov_u<0x140>(u));     // row_mirror
    if (G >= 32) u = max(u, (unsigned)__builtin_amdgcn_ds_swizzle((int)u, 0x401F));
    if (G >= 64)
        u = max(u, (unsigned)__builtin_amdgcn_ds_bpermute((int)((threadIdx.x ^ 32) & 63) << 2, (int)u));
    return __builtin_bit_cast(float, u);
}

// GC: lanes per uz-line when known at compile time (0: use the runtime G).
template <int P, int V, int GC = 0>
struct GlobalWriter {
    using T = typename Codec<P>::T;
    T* base;
    float* sbase;
    long stride;
    long sstride;
    int M;
    int dir;
    int G;                // lanes per uz-line (scaled storage), power of two

    __device__ void put(int i, const float* x)
    {
        const long p = dir > 0 ? i : M - 1 - i;
        if (Codec<P>::scaled) {
            float m = 0.0f;
#pragma unroll
            for (int v = 0; v < V; ++v) m = fmaxf(m, fabsf(x[v]));
            m = GC > 0 ? group_max_nonneg<GC>(m) : group_max(m, G);
            const float inv = inv_scale(m);
            store_row<P, V>(base + p * stride, x, inv);
            if ((threadIdx.x & (G - 1)) == 0) sbase[p * sstride] = m;
        } else {
            store_row<P, V>(base + p * stride, x, 1.0f);
        }
    }
};

// Raw buffer access for rows whose address is wave-uniform: the row's start
// goes into a buffer resource (scalar registers, rebuilt per row by a few
// scalar instructions) and each lane supplies only its fixed byte offset in a
// VGPR, so a row access costs no vector address arithmetic.  The resource
// covers exactly the bytes from the row start that the wave may touch; an
// access beyond them reads zero and writes nothing.
__device__ __forceinline__ unsigned row_span_bytes(long b)
{
    return b > 0xFFFFFFFFL ? 0xFFFFFFFFu : (unsigned)b;
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* p, unsigned bytes)
{
    // word 3 = 0x00020000: the gfx9 raw-buffer format (32-bit data format)
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <class T, int V>
__device__ __forceinline__ Pack<T, V> buffer_load_pack(__amdgpu_buffer_rsrc_t rs, unsigned off)
{
    constexpr int B = (int)sizeof(T) * V;
    static_assert(B == 2 || B == 4 || B == 8 || B == 16, "row piece of 2, 4, 8 or 16 bytes");
    if constexpr (B == 16) return __builtin_bit_cast(Pack<T, V>, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0));
    else if constexpr (B == 8) return __builtin_bit_cast(Pack<T, V>, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0));
    else if constexpr (B == 4) return __builtin_bit_cast(Pack<T, V>, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0));
    else return __builtin_bit_cast(Pack<T, V>, __builtin_amdgcn_raw_buffer_load_b16(rs, (int)off, 0, 0));
}

template <class T, int V>
__device__ __forceinline__ void buffer_store_pack(const Pack<T, V>& q, __amdgpu_buffer_rsrc_t rs, unsigned off)
{
    constexpr int B = (int)sizeof(T) * V;
    static_assert(B == 2 || B == 4 || B == 8 || B == 16, "row piece of 2, 4, 8 or 16 bytes");
    if constexpr (B == 16) {
        using W = __attribute__((ext_vector_type(4))) unsigned;
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(W, q), rs, (int)off, 0, 0);
    } else if constexpr (B == 8) {
        using W = __attribute__((ext_vector_type(2))) unsigned;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(W, q), rs, (int)off, 0, 0);
    } else if constexpr (B == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, q), rs, (int)off, 0, 0);
    } else {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, q), rs, (int)off, 0, 0);
    }
}

// Rows of the lines of one wave when every lane visits the same rows (one
// integer shift and one walk direction over the wave; periodic lines): the
// row index and the row's address are scalar work, and a lane only adds its
// fixed byte offset within the row (buffer addressing above).
template <int P, int V>
struct URowReader {
    using T = typename Codec<P>::T;
    const T* base;        // row 0 of the wave's first element (uniform)
    const float* sbase;   // its scale (uniform; scaled storage)
    unsigned loff;        // this lane's byte offset within a row
    unsigned soff;        // this lane's scale byte offset within a row
    unsigned nbytes;      // bytes from base to the end of its row
    unsigned sbytes;      // the same for the scales
    long stride;          // elements between rows
    long sstride;         // scales between rows
    int M;
    int dir;              // uniform
    int r0;               // frame rotation (uniform, 0 <= r0 < M; see URowWriter)
    int phys;             // uniform

    __device__ void seek(int r)
    {
        r += r0;
        int q = dir > 0 ? r : M - 1 - r;
        q %= M;
        if (q < 0) q += M;
        phys = q;
    }
    __device__ void next(float* x)
    {
        float sc = 1.0f;
        if (Codec<P>::scaled)
            sc = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                     row_rsrc(sbase + (long)phys * sstride, sbytes), (int)soff, 0, 0));
        const Pack<T, V> q = buffer_load_pack<T, V>(row_rsrc(base + (long)phys * stride, nbytes), loff);
#pragma unroll
        for (int v = 0; v < V; ++v)
            x[v] = decode<P>(q.v[v], sc);
        phys += dir;
        if (phys == M) phys = 0;
        else if (phys < 0) phys = M - 1;
    }
};

template <int P, int V, int GC = 0>
struct URowWriter {
    using T = typename Codec<P>::T;
    T* base;
    float* sbase;
    unsigned loff;
    unsigned soff;
    unsigned nbytes;
    unsigned sbytes;
    long stride;
    long sstride;
    int M;
    int dir;              // uniform
    int r0;               // frame rotation (uniform, 0 <= r0 < M)
    int G;                // lanes per uz-line (scaled storage)

    // A periodic line may be walked from any frame row: frame row i is row
    // i + r0 (mod M) of the unrotated frame, with the same arithmetic for
    // every output.  Waves that start at different rows spread their
    // concurrent accesses over more of the memory system.
    __device__ void put(int i, const float* x)
    {
        int f = i + r0;
        if (f >= M) f -= M;
        const long p = dir > 0 ? f : M - 1 - f;
        const __amdgpu_buffer_rsrc_t rs = row_rsrc(base + p * stride, nbytes);
        Pack<T, V> q;
        if (Codec<P>::scaled) {
            float m = 0.0f;
#pragma unroll
            for (int v = 0; v < V; ++v) m = fmaxf(m, fabsf(x[v]));
            m = GC > 0 ? group_max_nonneg<GC>(m) : group_max(m, G);
            const float inv = inv_scale(m);
#pragma unroll
            for (int v = 0; v < V; ++v) q.v[v] = quantize<P>(x[v], inv);
            buffer_store_pack<T, V>(q, rs, loff);
            if ((threadIdx.x & (G - 1)) == 0)
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, m),
                                                      row_rsrc(sbase + p * sstride, sbytes), (int)soff, 0, 0);
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) q.v[v] = Codec<P>::enc(x[v]);
            buffer_store_pack<T, V>(q, rs, loff);
        }
    }
};

// The value held by lane l ^ (H/2), for aligned groups of H lanes: a DPP
// row rotation by 8 for H = 16, an LDS-free swizzle otherwise.
template <int H>
__device__ __forceinline__ float xor_half(float v)
{
    static_assert(H == 8 || H == 16 || H == 32, "uz-line halves of 4, 8 or 16 lanes");
    if constexpr (H == 16)
        return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x128, 0xF, 0xF, true));
    else
        return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), ((H / 2) << 10) | 0x1F));
}

// Rows of the paired walk.  A uz-line of 2H values is held by H lanes; the
// wave reads (and writes) whole rows of 64/H uz-lines, two adjacent values
// per lane (coalesced, one access per row), and swaps values between lane g
// and g ^ (H/2) of each group so that lane g holds one value of each half:
//   g < H/2:  lower half value 2g,        upper half value 2g + H
//   g >= H/2: lower half value 2g - H + 1, upper half value 2g + 1.
// The upper half is line A (moving up), the lower half line B.
template <int P, int H>
struct PairRowReader {
    using T = typename Codec<P>::T;
    const T* base;        // row 0 of the wave's first uz-line (uniform)
    const float* sbase;   // its scale (uniform; scaled storage)
    unsigned off;         // this lane's byte offset within a row (two values)
    unsigned soff;        // byte offset of its uz-line's scale within a scale row
    unsigned nbytes;      // bytes from base to the end of its row
    unsigned sbytes;
    long stride;          // elements between rows
    long sstride;         // scales between rows
    int M;
    bool lo;              // lane g < H/2
    int phys;             // uniform

    __device__ void seek(int r)
    {
        int q = r % M;
        if (q < 0) q += M;
        phys = q;
    }
    __device__ void next(float* x)
    {
        float sc = 1.0f;
        if (Codec<P>::scaled)
            sc = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                     row_rsrc(sbase + (long)phys * sstride, sbytes), (int)soff, 0, 0));
        const Pack<T, 2> q = buffer_load_pack<T, 2>(row_rsrc(base + (long)phys * stride, nbytes), off);
        const float v0 = decode<P>(q.v[0], sc);
        const float v1 = decode<P>(q.v[1], sc);
        const float p0 = xor_half<H>(v0);
        const float p1 = xor_half<H>(v1);
        x[0] = lo ? p0 : v1;          // upper half: line A
        x[1] = lo ? v0 : p1;          // lower half: line B
        phys += 1;
        if (phys == M) phys = 0;
    }
};

// The inverse exchange, then one coalesced store per row; with scaled
// storage the uz-line's scale is the largest |value| over its H lanes (two
// values each).
template <int P, int H>
struct PairRowWriter {
    using T = typename Codec<P>::T;
    T* base;
    float* sbase;
    unsigned off;
    unsigned soff;
    unsigned nbytes;
    unsigned sbytes;
    long stride;
    long sstride;
    bool lo;

    __device__ void put(int i, float xa, float xb)
    {
        // xa: upper half value, xb: lower half value of this lane
        const float qa = xor_half<H>(xa);
        const float qb = xor_half<H>(xb);
        const float s0 = lo ? xb : qa;    // value 2g
        const float s1 = lo ? qb : xa;    // value 2g + 1
        const __amdgpu_buffer_rsrc_t rs = row_rsrc(base + (long)i * stride, nbytes);
        Pack<T, 2> q;
        if (Codec<P>::scaled) {
            float m = fmaxf(fabsf(xa), fabsf(xb));
            m = group_max_nonneg<H>(m);
            const float inv = inv_scale(m);
            q.v[0] = quantize<P>(s0, inv);
            q.v[1] = quantize<P>(s1, inv);
            if ((threadIdx.x & (H - 1)) == 0)
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, m),
                                                      row_rsrc(sbase + (long)i * sstride, sbytes),
                                                      (int)soff, 0, 0);
        } else {
            q.v[0] = Codec<P>::enc(s0);
            q.v[1] = Codec<P>::enc(s1);
        }
        buffer_store_pack<T, 2>(q, rs, off);
    }
};

// Rows of one line held in LDS (already decoded to FP32), `stride` floats
// apart.
struct LdsReader {
    const float* line;
    int stride;
    int M;
    int dir;
    bool periodic;
    int phys;

    __device__ void seek(int r)
    {
        int p = dir > 0 ? r : M - 1 - r;
        if (periodic) {
            p %= M;
            if (p < 0) p += M;
        }
        phys = p;
    }
    __device__ void next(float* x)
    {
        x[0] = (periodic || (phys >= 0 && phys < M)) ? line[phys * stride] : 0.0f;
        phys += dir;
        if (periodic) {
            if (phys == M) phys = 0;
            else if (phys < 0) phys = M - 1;
        }
    }
};

// Keeps the outputs of one line in registers, in frame order.
template <int MT>
struct RegWriter {
    float out[MT];
    __device__ void put(int i, const float* x) { out[i] = x[0]; }
};

// Tracks only the largest |output| (first pass of a scaled fallback line).
struct MaxWriter {
    float m;
    __device__ void put(int, const float* x) { m = fmaxf(m, fabsf(x[0])); }
};

// Writes a contiguous line with a known scale (second pass of the fallback).
template <int P>
struct ContigWriter {
    using T = typename Codec<P>::T;
    T* base;
    int M;
    int dir;
    float inv;
    __device__ void put(int i, const float* x)
    {
        const int p = dir > 0 ? i : M - 1 - i;
        base[p] = quantize<P>(x[0], inv);
    }
};

// ---------------------------------------------------------------------------
// FP64 reduction of one value per thread over the work-group, fixed order.
// Returns the total in thread 0.
// ---------------------------------------------------------------------------
__device__ inline double block_sum(double v, double* red)
{
    for (int w = 32; w >= 1; w >>= 1) v += __shfl_xor(v, w);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int q = 0; q < nw; ++q) t += red[q];
    }
    return t;
}

}  // namespace vlasov
