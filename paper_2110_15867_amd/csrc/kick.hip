// Fused velocity kick: the three velocity sweeps D_uz D_uy D_ux of one half
// step (Eq. 5) applied to each spatial cell's velocity block inside LDS.
//
// Every velocity sweep is local to a spatial cell (the shift g(x) dt / du is
// the same for all lines of the cell, and velocity space is never split --
// section 5.1.3), so a work-group can hold the whole block (32^3 FP32 values
// = 128 KiB of MI355X's 160 KiB LDS), run ux, uy and uz on it, and touch HBM
// once for reading and once for writing instead of three times each.  Each
// sweep runs the same line walker with the same FP32 operations as the
// single-sweep kernels, and with FP16/BF16 storage the intermediate results
// are rounded exactly as if they had been stored, so the result is bitwise
// the one of the three separate sweeps.
//
// LDS layout: uz-lines of NZ values padded to NZ+1 floats, line index
// jx*NY + jy.  A thread owns one line per sweep; lanes of a wave read
// consecutive jz (ux, uy sweeps) or lines 33 floats apart (uz sweep), both
// free of bank conflicts.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.hpp"
#include "rows.hpp"
#include "sl_mpp5.hpp"

namespace vlasov {

// Round the uz-line held by this thread in LDS as storage would: its scale
// is the largest |value|, each value becomes code * scale.
template <int P, int NZ>
__device__ __forceinline__ void storage_round_line(float* line)
{
    float x[NZ];
    float m = 0.0f;
#pragma unroll
    for (int i = 0; i < NZ; ++i) {
        x[i] = line[i];
        m = fmaxf(m, fabsf(x[i]));
    }
    const float inv = inv_scale(m);
#pragma unroll
    for (int i = 0; i < NZ; ++i) line[i] = Codec<P>::dec(quantize<P>(x[i], inv)) * m;
}

template <int P, int NX, int NY, int NZ>
__global__ void __launch_bounds__(NY * NZ) k_kick(const typename Codec<P>::T* __restrict__ fin,
                                                const float* __restrict__ sin,
                                                typename Codec<P>::T* __restrict__ fout,
                                                float* __restrict__ sout, KickArgs a)
{
    static_assert(NX * NZ == NY * NZ && NX * NY == NY * NZ, "cubic velocity blocks only");
    using T = typename Codec<P>::T;
    constexpr int NT = NY * NZ;
    constexpr int LS = NZ + 1;
    constexpr int NL = NX * NY;                 // uz-lines per cell
    constexpr int NU = NX * NY * NZ;
    extern __shared__ float lds[];
    __shared__ double red[NT / 64];
    const long cell = blockIdx.x;
    const int t = threadIdx.x;

    // ---- load the velocity block (coalesced 4-value accesses) ----
    const T* src = fin + cell * NU;
    for (int e = t * 4; e < NU; e += NT * 4) {
        const int ln = e / NZ;
        const int jz = e - ln * NZ;
        const float sc = Codec<P>::scaled ? sin[cell * NL + ln] : 1.0f;
        float x[4];
        load_row<P, 4>(src + e, sc, x);
#pragma unroll
        for (int q = 0; q < 4; ++q) lds[ln * LS + jz + q] = x[q];
    }
    __syncthreads();

    double tot[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int axis = 0; axis < 3; ++axis) {
        const int M = axis == 0 ? NX : (axis == 1 ? NY : NZ);
        const double s = (double)a.g[(long)axis * a.cells + cell] * a.factor[axis];
        const LineShift sh = split_shift(s, M, a.periodic);
        const int dir = sh.neg ? -1 : 1;
        // line of this thread and the LDS stride along the axis
        int base, stride;
        if (axis == 0) {            // lines (jy, jz) along jx
            base = (t / NZ) * LS + (t % NZ);
            stride = NY * LS;
        } else if (axis == 1) {     // lines (jx, jz) along jy
            base = (t / NZ) * NY * LS + (t % NZ);
            stride = LS;
        } else {                    // lines (jx, jy) along jz
            base = t * LS;
            stride = 1;
        }
        RegWriter<NX> wr;           // NX == NY == NZ
        float ofl = 0.0f;
        LdsReader rd{lds + base, stride, M, dir, a.periodic, 0};
        walk_uniform<1, NX>(rd, wr, M, sh, a.periodic, &ofl);
        tot[axis] = (double)ofl;
        __syncthreads();            // every line read before any is overwritten
        if (axis < 2) {
#pragma unroll
            for (int i = 0; i < NX; ++i) lds[base + (dir > 0 ? i : NX - 1 - i) * stride] = wr.out[i];
            if (Codec<P>::scaled) {
                __syncthreads();
                storage_round_line<P, NZ>(lds + t * LS);
            }
        } else {
            float inv = 1.0f;
            if (Codec<P>::scaled) {
                float m = 0.0f;
#pragma unroll
                for (int i = 0; i < NZ; ++i) m = fmaxf(m, fabsf(wr.out[i]));
                inv = inv_scale(m);
                sout[cell * NL + t] = m;
            }
#pragma unroll
            for (int i = 0; i < NZ; ++i) lds[base + (dir > 0 ? i : NZ - 1 - i)] = wr.out[i] * inv;
        }
        __syncthreads();
    }

    // ---- store (coalesced) ----
    T* dst = fout + cell * NU;
    for (int e = t * 4; e < NU; e += NT * 4) {
        const int ln = e / NZ;
        const int jz = e - ln * NZ;
        Pack<T, 4> q;
#pragma unroll
        for (int u = 0; u < 4; ++u) q.v[u] = Codec<P>::enc(lds[ln * LS + jz + u]);
        *reinterpret_cast<Pack<T, 4>*>(dst + e) = q;
    }
    if (a.outflow != nullptr && !a.periodic) {
        // same order as three separate sweeps: ux, then uy, then uz
        for (int axis = 0; axis < 3; ++axis) {
            const double s = block_sum(tot[axis], red);
            if (t == 0) a.outflow[cell] += s * a.du3;
        }
    }
}

template <int P, int N>
static hipError_t launch_kick_n(const void* fin, const float* sin, void* fout, float* sout,
                                const KickArgs& a, hipStream_t st)
{
    using T = typename Codec<P>::T;
    const size_t lds = (size_t)N * N * (N + 1) * sizeof(float);
    auto kern = k_kick<P, N, N, N>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)a.cells), dim3(N * N), lds, st, (const T*)fin, sin,
                       (T*)fout, sout, a);
    return hipGetLastError();
}

template <int P>
static hipError_t launch_kick_p(const void* fin, const float* sin, void* fout, float* sout,
                                const KickArgs& a, hipStream_t st)
{
    if (a.nu[0] == 32) return launch_kick_n<P, 32>(fin, sin, fout, sout, a, st);
    return launch_kick_n<P, 16>(fin, sin, fout, sout, a, st);
}

bool kick_supported(const int nu[3], size_t lds_limit)
{
    if (nu[0] != nu[1] || nu[1] != nu[2]) return false;
    if (nu[0] != 16 && nu[0] != 32) return false;
    const size_t lds = (size_t)nu[0] * nu[0] * (nu[0] + 1) * sizeof(float);
    return lds <= lds_limit;
}

hipError_t launch_kick(int prec, const void* fin, const float* sin, void* fout, float* sout,
                       const KickArgs& a, hipStream_t st)
{
    if (a.cells == 0) return hipSuccess;
    switch (prec) {
        case PREC_F16: return launch_kick_p<PREC_F16>(fin, sin, fout, sout, a, st);
        case PREC_BF16: return launch_kick_p<PREC_BF16>(fin, sin, fout, sout, a, st);
        default: return launch_kick_p<PREC_F32>(fin, sin, fout, sout, a, st);
    }
}

}  // namespace vlasov
