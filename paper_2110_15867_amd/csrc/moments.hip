// Velocity moments per spatial cell (section 5.1.3) and a deterministic FP64
// sum.  Velocity space is whole inside each spatial cell, so every moment is a
// reduction over one contiguous block of nu_x*nu_y*nu_z values: one
// work-group per cell, coalesced loads, FP64 accumulation, wave shuffles and a
// fixed-order combine across waves.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.hpp"
#include "sl_mpp5.hpp"

namespace vlasov {

__device__ __forceinline__ double wave_sum(double v)
{
    for (int w = 32; w >= 1; w >>= 1) v += __shfl_xor(v, w);
    return v;
}

template <int P, int V>
__global__ void __launch_bounds__(256) k_moments(const typename Codec<P>::T* __restrict__ f,
                                                 const float* __restrict__ scale, MomArgs a)
{
    __shared__ double red[4][4];
    const long cell = blockIdx.x;
    const typename Codec<P>::T* blk = f + cell * a.Nu;
    const long nyz = (long)a.nu[1] * a.nu[2];
    double m0 = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
    for (long e = (long)threadIdx.x * V; e < a.Nu; e += (long)blockDim.x * V) {
        const long jx = e / nyz;
        const long jy = (e - jx * nyz) / a.nu[2];
        const long jz = e - jx * nyz - jy * a.nu[2];
        float sc = 1.0f;
        if (Codec<P>::scaled) sc = scale[cell * (a.Nu / a.nuz) + e / a.nuz];
        float x[V];
        load_row<P, V>(blk + e, sc, x);
        const double ux = a.umin[0] + ((double)jx + 0.5) * a.du[0];
        const double uy = a.umin[1] + ((double)jy + 0.5) * a.du[1];
        double s0 = 0.0, sz = 0.0;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const double xv = (double)x[v];
            const double uz = a.umin[2] + ((double)(jz + v) + 0.5) * a.du[2];
            s0 += xv;
            sz = fma(uz, xv, sz);
        }
        m0 += s0;
        mx = fma(ux, s0, mx);
        my = fma(uy, s0, my);
        mz += sz;
    }
    m0 = wave_sum(m0);
    mx = wave_sum(mx);
    my = wave_sum(my);
    mz = wave_sum(mz);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[wave][0] = m0; red[wave][1] = mx; red[wave][2] = my; red[wave][3] = mz;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[4] = {0.0, 0.0, 0.0, 0.0};
        const int nw = (blockDim.x + 63) >> 6;
        for (int q = 0; q < nw; ++q)
            for (int c = 0; c < 4; ++c) t[c] += red[q][c];
        a.rho[cell] = t[0] * a.du3;
        if (a.umean != nullptr) {
            const double inv = t[0] != 0.0 ? 1.0 / t[0] : 0.0;
            a.umean[cell] = t[1] * inv;
            a.umean[a.cells + cell] = t[2] * inv;
            a.umean[2 * a.cells + cell] = t[3] * inv;
        }
    }
}

template <int P>
static hipError_t launch_moments_p(const void* f, const float* scale, const MomArgs& a,
                                   hipStream_t st)
{
    using T = typename Codec<P>::T;
    if (a.cells == 0) return hipSuccess;
    if (a.nuz % 4 == 0) {
        hipLaunchKernelGGL((k_moments<P, 4>), dim3((unsigned)a.cells), dim3(256), 0, st,
                           (const T*)f, scale, a);
    } else {
        hipLaunchKernelGGL((k_moments<P, 1>), dim3((unsigned)a.cells), dim3(256), 0, st,
                           (const T*)f, scale, a);
    }
    return hipGetLastError();
}

hipError_t launch_moments(int prec, const void* f, const float* scale, const MomArgs& a,
                          hipStream_t st)
{
    switch (prec) {
        case PREC_F16: return launch_moments_p<PREC_F16>(f, scale, a, st);
        case PREC_BF16: return launch_moments_p<PREC_BF16>(f, scale, a, st);
        default: return launch_moments_p<PREC_F32>(f, scale, a, st);
    }
}

// Adjoint of the moments: lam_f[c][u] += du^3 (lam_rho[c] + sum_a
// lam_umean[a][c] (u_a - umean_a[c]) / rho[c]), the umean term only where
// rho[c] != 0.  One work-group per cell.
__global__ void __launch_bounds__(256) k_moments_adj(MomArgs a, const double* __restrict__ lam_rho,
                                                     const double* __restrict__ lam_umean,
                                                     float* __restrict__ lam_f)
{
    const long cell = blockIdx.x;
    const long nyz = (long)a.nu[1] * a.nu[2];
    const double base = a.du3 * lam_rho[cell];
    double lu[3] = {0.0, 0.0, 0.0}, um[3] = {0.0, 0.0, 0.0};
    if (lam_umean != nullptr && a.rho[cell] != 0.0) {
        for (int k = 0; k < 3; ++k) {
            lu[k] = a.du3 * lam_umean[k * a.cells + cell] / a.rho[cell];
            um[k] = a.umean[k * a.cells + cell];
        }
    }
    float* out = lam_f + cell * a.Nu;
    for (long e = threadIdx.x; e < a.Nu; e += blockDim.x) {
        const long jx = e / nyz;
        const long jy = (e - jx * nyz) / a.nu[2];
        const long jz = e - jx * nyz - jy * a.nu[2];
        const double u0 = a.umin[0] + ((double)jx + 0.5) * a.du[0];
        const double u1 = a.umin[1] + ((double)jy + 0.5) * a.du[1];
        const double u2 = a.umin[2] + ((double)jz + 0.5) * a.du[2];
        const double t = base + lu[0] * (u0 - um[0]) + lu[1] * (u1 - um[1]) + lu[2] * (u2 - um[2]);
        out[e] += (float)t;
    }
}

hipError_t launch_moments_adj(const MomArgs& a, const double* lam_rho, const double* lam_umean,
                              float* lam_f, hipStream_t st)
{
    if (a.cells == 0) return hipSuccess;
    hipLaunchKernelGGL(k_moments_adj, dim3((unsigned)a.cells), dim3(256), 0, st, a, lam_rho,
                       lam_umean, lam_f);
    return hipGetLastError();
}

// One work-group, fixed order: thread t sums x[t], x[t+1024], ..., then a
// fixed tree over the threads.
__global__ void __launch_bounds__(1024) k_sum(const double* __restrict__ x, long n, double scale,
                                              double* __restrict__ out)
{
    __shared__ double red[16];
    double s = 0.0;
    for (long i = threadIdx.x; i < n; i += blockDim.x) s += x[i];
    s = wave_sum(s);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < 16; ++q) t += red[q];
        *out = t * scale;
    }
}

hipError_t launch_sum(const double* x, long n, double scale, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, st, x, n, scale, out);
    return hipGetLastError();
}

}  // namespace vlasov
