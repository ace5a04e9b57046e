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

// With SIG, also the second moments about u = 0, from which the dispersion
// tensor of each cell follows as sum u_l u_m f / sum f - umean_l umean_m.  The
// sums are FP64 over FP32 (or decoded FP16/BF16) values, so the subtraction
// loses about log10(<u^2> / sigma) digits of the 16 FP64 carries.
// ZC: nu_z divides the trip stride 256 V, so every row a thread reads starts
// at the same jz and its V values of u_z are computed once.
template <int P, int V, bool SIG, bool ZC>
__global__ void __launch_bounds__(256) k_moments(const typename Codec<P>::T* __restrict__ f,
                                                 const float* __restrict__ scale, MomArgs a)
{
    constexpr int NS = SIG ? 10 : 4;
    __shared__ double red[4][NS];
    const long cell = blockIdx.x;
    const typename Codec<P>::T* blk = f + cell * a.Nu;
    // m[0] = sum f, m[1..3] = sum u f, m[4..9] = sum u_l u_m f (xx xy xz yy yz zz)
    double m[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) m[k] = 0.0;
    // U rows per thread and trip: their loads are issued before any of them
    // is summed, so each wave keeps U loads in flight.  Rows past the block
    // read nothing and add zeros.  Offsets inside a block fit 32 bits (the
    // library refuses larger velocity blocks), so the index arithmetic is
    // 32-bit; the trip counter is 64-bit so that it cannot wrap.
    constexpr int U = 4;
    const long nb = a.Nu, stride = (long)blockDim.x * V;
    const int nz = a.nu[2], ny = a.nu[1];
    double uzc[V];
    if (ZC) {
        const int jz0 = (int)((threadIdx.x * V) % nz);
#pragma unroll
        for (int v = 0; v < V; ++v) uzc[v] = a.umin[2] + ((double)(jz0 + v) + 0.5) * a.du[2];
    }
    for (long e0 = (long)threadIdx.x * V; e0 < nb; e0 += U * stride) {
        float x[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long e = e0 + u * stride;
            if (e < nb) {
                float sc = 1.0f;
                if (Codec<P>::scaled) sc = scale[cell * (a.Nu / a.nuz) + (int)e / nz];
                load_row<P, V>(blk + e, sc, x[u]);
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) x[u][v] = 0.0f;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long el = e0 + u * stride;
            const int e = el < nb ? (int)el : 0;         // rows past the block hold zeros
            const int row = e / nz;                      // jx * ny + jy
            const int jz = e - row * nz;
            const int jx = row / ny;
            const int jy = row - jx * ny;
            const double ux = a.umin[0] + ((double)jx + 0.5) * a.du[0];
            const double uy = a.umin[1] + ((double)jy + 0.5) * a.du[1];
            double s0 = 0.0, sz = 0.0, szz = 0.0;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const double xv = (double)x[u][v];
                const double uz =
                    ZC ? uzc[v] : a.umin[2] + ((double)(jz + v) + 0.5) * a.du[2];
                s0 += xv;
                sz = fma(uz, xv, sz);
                if (SIG) szz = fma(uz * uz, xv, szz);
            }
            m[0] += s0;
            m[1] = fma(ux, s0, m[1]);
            m[2] = fma(uy, s0, m[2]);
            m[3] += sz;
            if (SIG) {
                m[4] = fma(ux * ux, s0, m[4]);
                m[5] = fma(ux * uy, s0, m[5]);
                m[6] = fma(ux, sz, m[6]);
                m[7] = fma(uy * uy, s0, m[7]);
                m[8] = fma(uy, sz, m[8]);
                m[9] += szz;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) m[k] = wave_sum(m[k]);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NS; ++k) red[wave][k] = m[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[NS];
        for (int c = 0; c < NS; ++c) t[c] = 0.0;
        const int nw = (blockDim.x + 63) >> 6;
        for (int q = 0; q < nw; ++q)
            for (int c = 0; c < NS; ++c) t[c] += red[q][c];
        a.rho[cell] = t[0] * a.du3;
        const double inv = t[0] != 0.0 ? 1.0 / t[0] : 0.0;
        const double um[3] = {t[1] * inv, t[2] * inv, t[3] * inv};
        if (a.umean != nullptr) {
            a.umean[cell] = um[0];
            a.umean[a.cells + cell] = um[1];
            a.umean[2 * a.cells + cell] = um[2];
        }
        if (SIG) {
            const int l[6] = {0, 0, 0, 1, 1, 2}, r[6] = {0, 1, 2, 1, 2, 2};
            for (int k = 0; k < 6; ++k)
                a.sigma[(long)k * a.cells + cell] =
                    t[0] != 0.0 ? fma(t[4 + k], inv, -um[l[k]] * um[r[k]]) : 0.0;
        }
    }
}

template <int P, int V, bool SIG>
static void launch_moments_v(const typename Codec<P>::T* f, const float* scale, const MomArgs& a,
                             hipStream_t st)
{
    if ((256 * V) % a.nuz == 0)
        hipLaunchKernelGGL((k_moments<P, V, SIG, true>), dim3((unsigned)a.cells), dim3(256), 0,
                           st, f, scale, a);
    else
        hipLaunchKernelGGL((k_moments<P, V, SIG, false>), dim3((unsigned)a.cells), dim3(256), 0,
                           st, f, scale, a);
}

template <int P, bool SIG>
static void launch_moments_sig(const typename Codec<P>::T* f, const float* scale,
                               const MomArgs& a, hipStream_t st)
{
    // 16-byte loads: 4 FP32 or 8 FP16/BF16 values of one uz-line
    constexpr int V16 = 16 / sizeof(typename Codec<P>::T);
    if (a.nuz % V16 == 0)
        launch_moments_v<P, V16, SIG>(f, scale, a, st);
    else if (a.nuz % 4 == 0)
        launch_moments_v<P, 4, SIG>(f, scale, a, st);
    else
        launch_moments_v<P, 1, SIG>(f, scale, a, st);
}

template <int P>
static hipError_t launch_moments_p(const void* f, const float* scale, const MomArgs& a,
                                   hipStream_t st)
{
    using T = typename Codec<P>::T;
    if (a.cells == 0) return hipSuccess;
    if (a.sigma != nullptr)
        launch_moments_sig<P, true>((const T*)f, scale, a, st);
    else
        launch_moments_sig<P, false>((const T*)f, scale, a, st);
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
