// Storage-precision dispatch of the sweep launchers (the kernels live in
// sweeps_impl.hpp, instantiated per precision by sweeps_f32/f16/bf16.hip).
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "sl_mpp5.hpp"

namespace vlasov {

#define VL_DECL(NAME, ARGS)                                                                      \
    hipError_t NAME##_f32(const void*, const float*, void*, float*, const ARGS&, hipStream_t);  \
    hipError_t NAME##_f16(const void*, const float*, void*, float*, const ARGS&, hipStream_t);  \
    hipError_t NAME##_bf16(const void*, const float*, void*, float*, const ARGS&, hipStream_t);
VL_DECL(launch_position, PosArgs)
VL_DECL(launch_vel_strided, VelArgs)
VL_DECL(launch_vel_uz, VelArgs)
#undef VL_DECL

hipError_t launch_position(int prec, const void* fin, const float* sin, void* fout, float* sout,
                           const PosArgs& a, hipStream_t st)
{
    switch (prec) {
        case PREC_F16: return launch_position_f16(fin, sin, fout, sout, a, st);
        case PREC_BF16: return launch_position_bf16(fin, sin, fout, sout, a, st);
        default: return launch_position_f32(fin, sin, fout, sout, a, st);
    }
}

hipError_t launch_vel_strided(int prec, const void* fin, const float* sin, void* fout, float* sout,
                              const VelArgs& a, hipStream_t st)
{
    switch (prec) {
        case PREC_F16: return launch_vel_strided_f16(fin, sin, fout, sout, a, st);
        case PREC_BF16: return launch_vel_strided_bf16(fin, sin, fout, sout, a, st);
        default: return launch_vel_strided_f32(fin, sin, fout, sout, a, st);
    }
}

hipError_t launch_vel_uz(int prec, const void* fin, const float* sin, void* fout, float* sout,
                         const VelArgs& a, hipStream_t st)
{
    switch (prec) {
        case PREC_F16: return launch_vel_uz_f16(fin, sin, fout, sout, a, st);
        case PREC_BF16: return launch_vel_uz_bf16(fin, sin, fout, sout, a, st);
        default: return launch_vel_uz_f32(fin, sin, fout, sout, a, st);
    }
}

}  // namespace vlasov
