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
        int p = dir > 0 ? r : M - 1 - r;
        if (periodic) {
            p %= M;
            if (p < 0) p += M;
        }
        phys = p;
    }
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

// Writes frame row i of a strided line.  Scaled storage: the G lanes that
// hold one uz-line (aligned groups) agree on its largest |value|.
template <int P, int V>
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
        const int p = dir > 0 ? i : M - 1 - i;
        if (Codec<P>::scaled) {
            float m = 0.0f;
#pragma unroll
            for (int v = 0; v < V; ++v) m = fmaxf(m, fabsf(x[v]));
            for (int w = 1; w < G; w <<= 1) m = fmaxf(m, __shfl_xor(m, w));
            const float inv = m > 0.0f ? 1.0f / m : 0.0f;
            store_row<P, V>(base + (long)p * stride, x, inv);
            if ((threadIdx.x & (G - 1)) == 0) sbase[(long)p * sstride] = m;
        } else {
            store_row<P, V>(base + (long)p * stride, x, 1.0f);
        }
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
