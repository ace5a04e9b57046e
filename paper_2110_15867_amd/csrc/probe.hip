// Plain device-to-device copy used as the HBM bandwidth probe: the practical
// ceiling a streaming kernel can reach, and the reference that scales the
// hardware traffic counters (bytes counted per byte really moved).
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

}  // namespace

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
