// Acceleration field of a density on the periodic spatial mesh: the Poisson
// equation (Eq. 2), nabla^2 phi = c (rho - mean rho) with c = 4 pi G a^2,
// solved by the discrete Fourier transform as the convolution method the
// paper uses for its mesh part (section 3), and g = -grad phi, the speed of
// the velocity sweeps (Eq. 4).  In Fourier space, with k_a = 2 pi m_a / L_a
// and m_a the signed index:
//   phi_k = -c rho_k / |k|^2 (phi_0 = 0: the mean drops out),
//   g_a,k = -i k_a phi_k, with k_a = 0 on the Nyquist plane of an even
//   axis (the derivative of a real Nyquist mode has no real representation).
// The mesh is small next to phase space (n^3 against n^3 nu^3 cells), so the
// transforms are plain separable DFTs in FP64, one output element per
// thread and one axis per pass, with exact twiddle indices (k l mod n).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.hpp"

namespace vlasov {

// tw[m] = exp(-2 pi i m / n)
__global__ void __launch_bounds__(256) k_twiddles(double2* __restrict__ tw, int n)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    double s, c;
    sincospi(2.0 * (double)m / (double)n, &s, &c);
    tw[m] = make_double2(c, -s);
}

// One DFT pass along `axis` of a complex [n0][n1][n2] array (real input when
// `rin` is given).  Forward: sum_l x_l exp(-2 pi i k l / n); inverse: the
// conjugate twiddles (no 1/n).
__global__ void __launch_bounds__(256) k_dft_axis(const double2* __restrict__ in,
                                                  const double* __restrict__ rin,
                                                  double2* __restrict__ out,
                                                  const double2* __restrict__ tw, int n0, int n1,
                                                  int n2, int axis, int inverse)
{
    const long cells = (long)n0 * n1 * n2;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cells) return;
    const int i2 = (int)(t % n2);
    const int i1 = (int)((t / n2) % n1);
    const int i0 = (int)(t / ((long)n1 * n2));
    const int n = axis == 0 ? n0 : (axis == 1 ? n1 : n2);
    const long stride = axis == 0 ? (long)n1 * n2 : (axis == 1 ? n2 : 1);
    const int k = axis == 0 ? i0 : (axis == 1 ? i1 : i2);
    const long base = t - (long)k * stride;              // element l = 0 of this line
    double re = 0.0, im = 0.0;
    int m = 0;                                           // k * l mod n
    for (int l = 0; l < n; ++l) {
        const double2 w = tw[m];
        const double wi = inverse ? -w.y : w.y;
        if (rin != nullptr) {
            const double x = rin[base + (long)l * stride];
            re = fma(x, w.x, re);
            im = fma(x, wi, im);
        } else {
            const double2 x = in[base + (long)l * stride];
            re = fma(x.x, w.x, fma(-x.y, wi, re));
            im = fma(x.x, wi, fma(x.y, w.x, im));
        }
        m += k;
        if (m >= n) m -= n;
    }
    out[t] = make_double2(re, im);
}

__device__ __forceinline__ double wavenumber(int i, int n, double L)
{
    const int m = 2 * i < n ? i : i - n;                 // signed index (Nyquist: -n/2)
    return 2.0 * 3.141592653589793 * (double)m / L;
}

// phi_k and the three components g_a,k = -i k_a phi_k
__global__ void __launch_bounds__(256) k_poisson(const double2* __restrict__ R,
                                                 double2* __restrict__ G, FieldArgs a)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.cells) return;
    const int i2 = (int)(t % a.n[2]);
    const int i1 = (int)((t / a.n[2]) % a.n[1]);
    const int i0 = (int)(t / ((long)a.n[1] * a.n[2]));
    const int idx[3] = {i0, i1, i2};
    double k[3], k2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        k[d] = wavenumber(idx[d], a.n[d], a.L[d]);
        k2 = fma(k[d], k[d], k2);
    }
    double2 phi = make_double2(0.0, 0.0);
    if (t != 0) {
        const double s = -a.coupling / k2;
        phi = make_double2(s * R[t].x, s * R[t].y);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const bool nyq = (a.n[d] % 2 == 0) && (2 * idx[d] == a.n[d]);
        const double kd = nyq ? 0.0 : k[d];
        // -i kd (phi.x + i phi.y) = kd phi.y - i kd phi.x
        G[(long)d * a.cells + t] = make_double2(kd * phi.y, -kd * phi.x);
    }
}

__global__ void __launch_bounds__(256) k_field_store(const double2* __restrict__ X,
                                                     float* __restrict__ g, long cells,
                                                     double inv_n)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cells) return;
    g[t] = (float)(X[t].x * inv_n);
}

hipError_t launch_field(const double* rho, float* g, const FieldArgs& a, void* work,
                        hipStream_t st)
{
    const long cells = a.cells;
    if (cells == 0) return hipSuccess;
    const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
    double2* tw[3];
    char* p = (char*)work;
    for (int d = 0; d < 3; ++d) {
        tw[d] = (double2*)p;
        p += field_align((size_t)a.n[d] * sizeof(double2));
    }
    double2* A = (double2*)p;
    p += field_align((size_t)cells * sizeof(double2));
    double2* B = (double2*)p;
    p += field_align((size_t)cells * sizeof(double2));
    double2* G = (double2*)p;
    const unsigned blocks = (unsigned)((cells + 255) / 256);
    for (int d = 0; d < 3; ++d)
        hipLaunchKernelGGL(k_twiddles, dim3((a.n[d] + 255) / 256), dim3(256), 0, st, tw[d], a.n[d]);
    // forward: z (from the real density), y, x
    hipLaunchKernelGGL(k_dft_axis, dim3(blocks), dim3(256), 0, st, (const double2*)nullptr, rho, A,
                       tw[2], n0, n1, n2, 2, 0);
    hipLaunchKernelGGL(k_dft_axis, dim3(blocks), dim3(256), 0, st, A, (const double*)nullptr, B,
                       tw[1], n0, n1, n2, 1, 0);
    hipLaunchKernelGGL(k_dft_axis, dim3(blocks), dim3(256), 0, st, B, (const double*)nullptr, A,
                       tw[0], n0, n1, n2, 0, 0);
    hipLaunchKernelGGL(k_poisson, dim3(blocks), dim3(256), 0, st, A, G, a);
    const double inv_n = 1.0 / (double)cells;
    for (int d = 0; d < 3; ++d) {
        const double2* Gd = G + (long)d * cells;
        hipLaunchKernelGGL(k_dft_axis, dim3(blocks), dim3(256), 0, st, Gd, (const double*)nullptr,
                           B, tw[0], n0, n1, n2, 0, 1);
        hipLaunchKernelGGL(k_dft_axis, dim3(blocks), dim3(256), 0, st, B, (const double*)nullptr,
                           A, tw[1], n0, n1, n2, 1, 1);
        hipLaunchKernelGGL(k_dft_axis, dim3(blocks), dim3(256), 0, st, A, (const double*)nullptr,
                           B, tw[2], n0, n1, n2, 2, 1);
        hipLaunchKernelGGL(k_field_store, dim3(blocks), dim3(256), 0, st, B, g + (long)d * cells,
                           cells, inv_n);
    }
    return hipGetLastError();
}

}  // namespace vlasov
