// Storage codec of the reduced-precision forms: an FP32 array to FP16/BF16
// codes with one FP32 scale per uz-line, and back.  The scale of a line is
// its largest |value|; a code is the value times the hardware reciprocal of
// the scale (inv_scale), rounded once to FP32 and then to the storage type
// (quantize) -- the operations every sweep kernel uses when it stores, so a
// line encoded here carries the codes a sweep would write for the same FP32
// values.  Decoding is code times scale in FP32, as the kernels load.
//
// One thread per four consecutive values of a uz-line (16 bytes of FP32);
// the nu_z / 4 threads of a line share its maximum by lane exchanges.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.hpp"
#include "sl_mpp5.hpp"

namespace vlasov {

namespace {

template <int P>
__global__ void __launch_bounds__(256) k_encode(const float* __restrict__ f,
                                                typename Codec<P>::T* __restrict__ codes,
                                                float* __restrict__ scale, long nthreads, int G)
{
    using T = typename Codec<P>::T;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    // a line's G threads are consecutive and G divides the block, so a line
    // is either wholly inside the range or wholly outside
    if (t >= nthreads) return;
    float x[4];
    const Pack<float, 4> v = *reinterpret_cast<const Pack<float, 4>*>(f + 4 * t);
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = v.v[k];
    float m = fmaxf(fmaxf(fabsf(x[0]), fabsf(x[1])), fmaxf(fabsf(x[2]), fabsf(x[3])));
    for (int off = 1; off < G; off <<= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    const float inv = inv_scale(m);
    Pack<T, 4> q;
#pragma unroll
    for (int k = 0; k < 4; ++k) q.v[k] = quantize<P>(x[k], inv);
    *reinterpret_cast<Pack<T, 4>*>(codes + 4 * t) = q;
    if (t % G == 0) scale[t / G] = m;
}

template <int P>
__global__ void __launch_bounds__(256) k_decode(const typename Codec<P>::T* __restrict__ codes,
                                                const float* __restrict__ scale,
                                                float* __restrict__ f, long nthreads, int G)
{
    using T = typename Codec<P>::T;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nthreads) return;
    const Pack<T, 4> q = *reinterpret_cast<const Pack<T, 4>*>(codes + 4 * t);
    const float sc = scale[t / G];
    Pack<float, 4> v;
#pragma unroll
    for (int k = 0; k < 4; ++k) v.v[k] = decode<P>(q.v[k], sc);
    *reinterpret_cast<Pack<float, 4>*>(f + 4 * t) = v;
}

template <int P>
hipError_t launch_encode_p(const float* f, void* codes, float* scale, long total, long nuz,
                           hipStream_t st)
{
    const long nthreads = total / 4;
    const long blocks = (nthreads + 255) / 256;
    hipLaunchKernelGGL(k_encode<P>, dim3((unsigned)blocks), dim3(256), 0, st, f,
                       (typename Codec<P>::T*)codes, scale, nthreads, (int)(nuz / 4));
    return hipGetLastError();
}

template <int P>
hipError_t launch_decode_p(const void* codes, const float* scale, float* f, long total, long nuz,
                           hipStream_t st)
{
    const long nthreads = total / 4;
    const long blocks = (nthreads + 255) / 256;
    hipLaunchKernelGGL(k_decode<P>, dim3((unsigned)blocks), dim3(256), 0, st,
                       (const typename Codec<P>::T*)codes, scale, f, nthreads, (int)(nuz / 4));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_encode(int prec, const float* f, void* codes, float* scale, long total, long nuz,
                         hipStream_t st)
{
    if (total == 0) return hipSuccess;
    if ((total / 4 + 255) / 256 > 0x7fffffffL) return hipErrorInvalidValue;
    if (prec == PREC_BF16) return launch_encode_p<PREC_BF16>(f, codes, scale, total, nuz, st);
    return launch_encode_p<PREC_F16>(f, codes, scale, total, nuz, st);
}

hipError_t launch_decode(int prec, const void* codes, const float* scale, float* f, long total,
                         long nuz, hipStream_t st)
{
    if (total == 0) return hipSuccess;
    if ((total / 4 + 255) / 256 > 0x7fffffffL) return hipErrorInvalidValue;
    if (prec == PREC_BF16) return launch_decode_p<PREC_BF16>(codes, scale, f, total, nuz, st);
    return launch_decode_p<PREC_F16>(codes, scale, f, total, nuz, st);
}

}  // namespace vlasov
