// The sweep kernels with F32 storage.
#include "sweeps_impl.hpp"

namespace vlasov {

hipError_t launch_position_f32(const void* fin, const float* sin, void* fout, float* sout,
                               const PosArgs& a, hipStream_t st)
{
    return launch_position_p<PREC_F32>(fin, sin, fout, sout, a, st);
}

hipError_t launch_vel_strided_f32(const void* fin, const float* sin, void* fout, float* sout,
                                  const VelArgs& a, hipStream_t st)
{
    return launch_vel_strided_p<PREC_F32>(fin, sin, fout, sout, a, st);
}

hipError_t launch_vel_uz_f32(const void* fin, const float* sin, void* fout, float* sout,
                             const VelArgs& a, hipStream_t st)
{
    return launch_vel_uz_p<PREC_F32>(fin, sin, fout, sout, a, st);
}

}  // namespace vlasov
