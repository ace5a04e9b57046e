// The sweep kernels with BF16 storage.
#include "sweeps_impl.hpp"

namespace vlasov {

hipError_t launch_position_bf16(const void* fin, const float* sin, void* fout, float* sout,
                               const PosArgs& a, hipStream_t st)
{
    return launch_position_p<PREC_BF16>(fin, sin, fout, sout, a, st);
}

hipError_t launch_vel_strided_bf16(const void* fin, const float* sin, void* fout, float* sout,
                                  const VelArgs& a, hipStream_t st)
{
    return launch_vel_strided_p<PREC_BF16>(fin, sin, fout, sout, a, st);
}

hipError_t launch_vel_uz_bf16(const void* fin, const float* sin, void* fout, float* sout,
                             const VelArgs& a, hipStream_t st)
{
    return launch_vel_uz_p<PREC_BF16>(fin, sin, fout, sout, a, st);
}

}  // namespace vlasov
