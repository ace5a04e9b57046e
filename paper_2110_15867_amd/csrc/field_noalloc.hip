// vlasov_field without a caller workspace: the transforms' twiddle tables and
// complex spectra live in a fixed device array of this file, so the call
// allocates nothing (for callers that cannot: code under stream capture,
// serving loops, harnesses that forbid allocation).  Meshes up to 64^3 cells
// fit; larger ones are refused.
//
// The array is a device symbol: its host-side name is not a device address.
// Its address on each device is looked up once, with that device current,
// and only that address is handed to the kernels.  Every call on a device
// uses the same array (the transforms write every element they read, so no
// clearing is needed); calls that overlap on one device race.
#include <hip/hip_runtime.h>
#include <math.h>
#include <mutex>
#include <stdint.h>
#include <string.h>

#include "../../include/vlasov.h"
#include "launch.hpp"

namespace {

constexpr size_t kScratchBytes = 24u << 20;   // 64^3 cells: 20 MiB of spectra + twiddles
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceScratch {
    std::once_flag once;
    void* ptr = nullptr;
    hipError_t err = hipSuccess;
};
DeviceScratch g_scratch[kMaxDevices];

// The array's address on the current device (looked up on the first call).
hipError_t scratch_on_current_device(void** ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    DeviceScratch& s = g_scratch[dev];
    std::call_once(s.once, [&s]() {
        void* p = nullptr;
        s.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        s.ptr = s.err == hipSuccess ? p : nullptr;
    });
    if (s.err != hipSuccess) return s.err;
    *ptr = s.ptr;
    return hipSuccess;
}

}  // namespace

extern "C" size_t vlasov_field_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" int vlasov_field_noalloc(const vlasov_grid* g, const double* rho, double coupling,
                                    float* field, void* stream)
{
    if (g == nullptr || rho == nullptr || field == nullptr) return VLASOV_ERR_NULL;
    int n[3];
    for (int a = 0; a < 3; ++a) {
        if (g->n[a] < 1 || g->nu[a] < 1) return VLASOV_ERR_SHAPE;
        if (!(g->L[a] > 0.0) || !isfinite(g->L[a])) return VLASOV_ERR_SHAPE;
        if (!(g->umax[a] > 0.0) || !isfinite(g->umax[a])) return VLASOV_ERR_SHAPE;
        n[a] = g->n[a];
    }
    if (!isfinite(coupling)) return VLASOV_ERR_NONFINITE;
    const long cells = (long)n[0] * n[1] * n[2];
    if (vlasov::field_workspace_bytes(n) > kScratchBytes) return VLASOV_ERR_TOO_LARGE;
    const uintptr_t pr = (uintptr_t)rho, pf = (uintptr_t)field;
    const size_t nb = (size_t)cells * sizeof(double), fb = 3 * (size_t)cells * sizeof(float);
    if (pr < pf + fb && pf < pr + nb) return VLASOV_ERR_ALIAS;
    void* work = nullptr;
    if (scratch_on_current_device(&work) != hipSuccess) return VLASOV_ERR_DEVICE;
    vlasov::FieldArgs a;
    memset(&a, 0, sizeof(a));
    for (int k = 0; k < 3; ++k) {
        a.n[k] = n[k];
        a.L[k] = g->L[k];
    }
    a.coupling = coupling;
    a.cells = cells;
    return vlasov::launch_field(rho, field, a, work, (hipStream_t)stream) == hipSuccess
               ? VLASOV_OK
               : VLASOV_ERR_DEVICE;
}
