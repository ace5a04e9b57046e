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

// A work-group-uniform value moved to a scalar register.  The empty asm hides
// the value's uniformity, so the optimiser keeps the readfirstlane (it drops
// one applied to a value it already knows to be uniform, which can leave the
// value in a vector register and the address arithmetic on the VALU).
__device__ __forceinline__ int uniform_sgpr(int v)
{
    asm volatile("" : "+v"(v));
    return __builtin_amdgcn_readfirstlane(v);
}

// Writes the updated line y (frame order) at its translated positions
// out_{j+N} = y_j, frame position p at lds[b + p * st].  Vacuum lines: the
// cells the translation empties become zero and what passes the upper face
// is added to *acc; periodic lines wrap.
template <int M, bool PER>
__device__ __forceinline__ void put_translated(float* lds, int b, int st, const float (&y)[M],
                                               int N, float scale, float* acc)
{
    if (PER) {
#pragma unroll
        for (int j = 0; j < M; ++j) {
            int p = j + N;                          // N < M for periodic lines
            p = p >= M ? p - M : p;
            lds[b + p * st] = y[j] * scale;
        }
    } else {
        const int nz = N < M ? N : M;
        for (int i = 0; i < nz; ++i) lds[b + i * st] = 0.0f;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const int p = j + N;
            if (p < M) lds[b + p * st] = y[j] * scale;
            else *acc += y[j];
        }
    }
}

template <int M, bool PER>
__device__ __forceinline__ float kept_max(const float (&y)[M], int N)
{
    float m = 0.0f;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        if (PER || j + N < M) m = fmaxf(m, fabsf(y[j]));
    }
    return m;
}

template <int P, int NU, bool PER>
__global__ void __launch_bounds__(NU * NU) k_kick(const typename Codec<P>::T* __restrict__ fin,
                                                const float* __restrict__ sin,
                                                typename Codec<P>::T* __restrict__ fout,
                                                float* __restrict__ sout, KickArgs a)
{
    using T = typename Codec<P>::T;
    constexpr int M = NU;
    constexpr int NT = NU * NU;
    constexpr int LS = NU + 1;
    constexpr int NL = NU * NU;                 // uz-lines per cell
    constexpr int NV = NU * NU * NU;
    extern __shared__ float lds[];
    __shared__ double red[NT / 64];
    const long cell = blockIdx.x;
    const int t = threadIdx.x;

    // ---- load the velocity block (coalesced 4-value accesses) ----
    const T* src = fin + cell * NV;
    for (int e = t * 4; e < NV; e += NT * 4) {
        const int ln = e / NU;
        const int jz = e - ln * NU;
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
        const double s = (double)a.g[(long)axis * a.cells + cell] * a.factor[axis];
        const LineShift sh = split_shift(s, M, PER);
        // line of this thread and the LDS stride along the axis
        int base, stride;
        if (axis == 0) {            // lines (jy, jz) along jx
            base = (t / NU) * LS + (t % NU);
            stride = NU * LS;
        } else if (axis == 1) {     // lines (jx, jz) along jy
            base = (t / NU) * NU * LS + (t % NU);
            stride = LS;
        } else {                    // lines (jx, jy) along jz
            base = t * LS;
            stride = 1;
        }
        // upwind frame: frame position p sits at lds[b + p * st]
        // (the shift is uniform over the work-group: N and st live in SGPRs,
        // so the translated store addresses cost scalar arithmetic only)
        const int N = uniform_sgpr(sh.N);
        const int st = uniform_sgpr(sh.neg ? -stride : stride);
        const int b = sh.neg ? base + (M - 1) * stride : base;
        float x[M];
#pragma unroll
        for (int k = 0; k < M; ++k) x[k] = lds[b + k * st];
        __syncthreads();            // every line read before any is overwritten
        float y[M];
        float phi_top;
        line_update_regs<M, PER>(x, sh, y, &phi_top);
        float acc = 0.0f;
        if (axis < 2 || !Codec<P>::scaled) {
            put_translated<M, PER>(lds, b, st, y, N, 1.0f, &acc);
        } else {
            // the last sweep leaves the values divided by the new line scale
            const float m = kept_max<M, PER>(y, N);
            sout[cell * NL + t] = m;
            put_translated<M, PER>(lds, b, st, y, N, inv_scale(m), &acc);
        }
        if (!PER) tot[axis] = (double)(acc + phi_top);
        __syncthreads();
        if (Codec<P>::scaled && axis < 2) {
            storage_round_line<P, NU>(lds + t * LS);
            __syncthreads();
        }
    }

    // ---- store (coalesced) ----
    T* dst = fout + cell * NV;
    for (int e = t * 4; e < NV; e += NT * 4) {
        const int ln = e / NU;
        const int jz = e - ln * NU;
        Pack<T, 4> q;
#pragma unroll
        for (int u = 0; u < 4; ++u) q.v[u] = Codec<P>::enc(lds[ln * LS + jz + u]);
        *reinterpret_cast<Pack<T, 4>*>(dst + e) = q;
    }
    if (a.outflow != nullptr && !PER) {
        // same order as three separate sweeps: ux, then uy, then uz
        for (int axis = 0; axis < 3; ++axis) {
            const double sm = block_sum(tot[axis], red);
            if (t == 0) a.outflow[cell] += sm * a.du3;
        }
    }
}

template <int P, int N>
static hipError_t launch_kick_n(const void* fin, const float* sin, void* fout, float* sout,
                                const KickArgs& a, hipStream_t st)
{
    using T = typename Codec<P>::T;
    const size_t lds = (size_t)N * N * (N + 1) * sizeof(float);
    auto kern = a.periodic ? k_kick<P, N, true> : k_kick<P, N, false>;
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
