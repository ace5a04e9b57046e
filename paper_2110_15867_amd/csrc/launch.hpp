// Host-side launch descriptors shared by the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vlasov {

constexpr int kMaxShiftTable = 256;   // velocity cells per axis a position sweep supports

// Position sweep along one spatial axis (Eq. 3).
struct PosArgs {
    long O;          // lines before the axis (product of earlier spatial sizes)
    long I;          // inner elements after the axis
    int M;           // cells along the axis
    long Nu;         // velocity cells per spatial cell
    long pst;        // stride of the velocity index that sets the shift
    int nshift;      // velocity cells along the matching velocity axis
    long nuz;        // length of a uz-line (scale granularity)
    long nux;        // velocity cells along u_x
    int V;           // adjacent inner elements per thread
    int G;           // lanes per uz-line (scaled storage)
    int pair;        // z sweep with the halves of each uz-line paired per lane (0: no)
    int skew;        // waves start their walks at different rows (1) or all at row 0
    int us;          // every wave's lanes share one shift and rows hold whole waves (1)
    int ug;          // y sweep: waves can be gathered across u_x so that they share u_y
                     // (the number of uz-lines per wave, each from its own u_x row), or
                     // 0; used with FP32 storage
    int mix;         // some wave holds lanes that move in both directions (1)
    double shift[kMaxShiftTable];   // s_j = u_j dt a^-2 / dx per velocity index
};

// Velocity sweep along one velocity axis (Eq. 4).
struct VelArgs {
    const float* g;  // field component of this axis, [cells]
    double factor;   // dt / du
    int M;           // cells along the axis
    long I;          // inner elements after the axis (1 for uz)
    long nsub;       // ux: 1; uy: nux (sub-blocks per cell); uz: nux*nuy (lines per cell)
    long nuz;
    int V;
    int G;
    bool periodic;
    double* outflow; // per spatial cell, or nullptr
    double du3;
    long cells;
};

hipError_t launch_position(int prec, const void* fin, const float* sin, void* fout, float* sout,
                           const PosArgs& a, hipStream_t st);
hipError_t launch_vel_strided(int prec, const void* fin, const float* sin, void* fout, float* sout,
                              const VelArgs& a, hipStream_t st);
hipError_t launch_vel_uz(int prec, const void* fin, const float* sin, void* fout, float* sout,
                         const VelArgs& a, hipStream_t st);
// uz sweep of 64-cell lines through double-buffered LDS tiles (kick.hip)
hipError_t launch_vel_uz64(int prec, const void* fin, const float* sin, void* fout, float* sout,
                           const VelArgs& a, hipStream_t st);

// Split shift of one velocity line (uniform over a spatial cell's block):
// integer part, direction, the fractional part's interface weights in
// difference form and the limiter constants (LineShift); precomputed per
// cell and axis for the fused kick.
struct KickShift {
    int N;
    int flags;       // bit 0: walked mirrored (neg), bit 1: complement bounds (comp)
    float mu;
    float v0, v1, v2, v3;
    float alpha, q, alpha_c, muc;
    float pad;
};

// Fused kick: the three velocity sweeps of one half step (Eq. 5) in LDS.
struct KickArgs {
    const float* g;  // field [3][cells]
    double factor[3];// dt / du per axis
    bool periodic;
    double* outflow;
    double du3;
    long cells;
    int nu[3];
    double* rho;     // moments of the stored result per cell, or nullptr
    double* umean;   // [3][cells], or nullptr
    double umin[3];  // -umax (cell centres for the moments)
    double du[3];
};
bool kick_supported(const int nu[3], size_t lds_limit);
// shifts: [cells][3] table written by the kick's own pre-pass on the same
// stream when given, else each work-group splits its shifts itself
hipError_t launch_kick(int prec, const void* fin, const float* sin, void* fout, float* sout,
                       const KickArgs& a, KickShift* shifts, hipStream_t st);
// 64^3 blocks: uy and uz fused in LDS on slabs of eight u_x rows (the ux
// sweep is a separate launch before it); shifts as for launch_kick
bool kick_yz64_supported(const int nu[3], size_t lds_limit);
hipError_t launch_kick_yz64(int prec, const void* fin, const float* sin, void* fout, float* sout,
                            const KickArgs& a, KickShift* shifts, hipStream_t st);

struct MomArgs {
    long cells;
    long Nu;
    int nu[3];
    double umin[3];  // -umax
    double du[3];
    double du3;
    double* rho;
    double* umean;   // [3][cells] or nullptr
    long nuz;
    double* sigma;   // [6][cells] dispersion tensor (xx, xy, xz, yy, yz, zz) or nullptr
};
hipError_t launch_moments(int prec, const void* f, const float* scale, const MomArgs& a,
                          hipStream_t st);
hipError_t launch_sum(const double* x, long n, double scale, double* out, hipStream_t st);

// Storage codec (FP16/BF16 codes + per-uz-line scale); total values, uz-line
// length nuz (a power of two from 4 to 64)
hipError_t launch_encode(int prec, const float* f, void* codes, float* scale, long total, long nuz,
                         hipStream_t st);
hipError_t launch_decode(int prec, const void* codes, const float* scale, float* f, long total,
                         long nuz, hipStream_t st);

// Field of a density on the periodic mesh (Eq. 2), FP64 DFTs.
struct FieldArgs {
    int n[3];
    double L[3];
    double coupling; // 4 pi G a^2
    long cells;
};
inline size_t field_align(size_t b) { return (b + 255) & ~(size_t)255; }
// workspace: three twiddle tables, two complex [cells] buffers, three more
inline size_t field_workspace_bytes(const int n[3])
{
    const size_t cells = (size_t)n[0] * n[1] * n[2];
    size_t b = 0;
    for (int d = 0; d < 3; ++d) b += field_align((size_t)n[d] * 16);
    return b + 2 * field_align(cells * 16) + field_align(3 * cells * 16);
}
hipError_t launch_field(const double* rho, float* g, const FieldArgs& a, void* work,
                        hipStream_t st);
hipError_t launch_moments_adj(const MomArgs& a, const double* lam_rho, const double* lam_umean,
                              float* lam_f, hipStream_t st);

// tangents and adjoints (FP32 storage)
hipError_t launch_position_tan(const float* f, const float* v, float* out, const PosArgs& a,
                               hipStream_t st);
hipError_t launch_position_adj(const float* f, const float* lam, float* lam_in, const PosArgs& a,
                               hipStream_t st);
hipError_t launch_velocity_tan(const float* f, const float* v, float* out, const float* g_dot,
                               const VelArgs& a, hipStream_t st);
hipError_t launch_velocity_adj(const float* f, const float* lam, float* lam_in, float* lam_g,
                               const VelArgs& a, hipStream_t st);

}  // namespace vlasov
