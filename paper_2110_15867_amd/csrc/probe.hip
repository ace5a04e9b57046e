// Probes of the two ceilings of the sweeps, not part of the method: a plain
// device-to-device copy (the HBM rate a streaming kernel can reach, and the
// reference that scales the hardware traffic counters) and independent
// chains of FP32 vector operations (the VALU issue rate).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vlasov.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// One 16-byte element per thread and many short-lived work-groups: on
// MI355X this pattern streams faster than any per-thread loop over several
// elements, so it is the practical ceiling of a copy.
__global__ void __launch_bounds__(256) k_copy(const f4* __restrict__ src, f4* __restrict__ dst,
                                              long n)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// Independent chains of the FP32 operations the sweeps issue most (FMA,
// med3, min3, max3, add, mul), eight chains per thread so that no
// instruction waits on the one before it: the vector-ALU issue rate a sweep
// can reach.  64 lane-operations per thread and iteration.
__global__ void __launch_bounds__(256) k_valu(float* __restrict__ out, int iters, float s, float t)
{
    float a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = (float)threadIdx.x * 1e-3f + (float)i;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            a[i] = fmaf(a[i], s, t);
            a[i] = __builtin_amdgcn_fmed3f(a[i], s, t);
            a[i] = fminf(fminf(a[i], s), a[(i + 1) & 7]);
            a[i] = fmaxf(fmaxf(a[i], t), a[(i + 3) & 7]);
            a[i] = a[i] + s;
            a[i] = a[i] * s;
            a[i] = fmaf(a[i], t, s);
            a[i] = a[i] - t;
        }
    }
    float r = 0.0f;
#pragma unroll
    for (int i = 0; i < 8; ++i) r += a[i];
    out[(long)blockIdx.x * blockDim.x + threadIdx.x] = r;
}

}  // namespace

extern "C" int vlasov_valu_probe(float* out, int64_t n, int iters, double* lane_ops, void* stream)
{
    if (out == nullptr || lane_ops == nullptr) return VLASOV_ERR_NULL;
    if (n <= 0 || n % 256 != 0 || n / 256 > 0x7fffffffL || iters < 0) return VLASOV_ERR_SHAPE;
    *lane_ops = (double)n * (double)iters * 64.0;
    hipLaunchKernelGGL(k_valu, dim3((unsigned)(n / 256)), dim3(256), 0, (hipStream_t)stream, out,
                       iters, 1.0001f, 0.5f);
    return hipGetLastError() == hipSuccess ? VLASOV_OK : VLASOV_ERR_DEVICE;
}

extern "C" int vlasov_stream_copy(const void* src, void* dst, size_t bytes, void* stream)
{
    if (src == nullptr || dst == nullptr) return VLASOV_ERR_NULL;
    if ((bytes & 15u) != 0 || ((uintptr_t)src & 15u) != 0 || ((uintptr_t)dst & 15u) != 0)
        return VLASOV_ERR_SHAPE;
    const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
    if (a < b + bytes && b < a + bytes) return VLASOV_ERR_ALIAS;
    const long n = (long)(bytes / 16);
    if (n == 0) return VLASOV_OK;
    const long blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffL) return VLASOV_ERR_SHAPE;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (const f4*)src, (f4*)dst, n);
    return hipGetLastError() == hipSuccess ? VLASOV_OK : VLASOV_ERR_DEVICE;
}
