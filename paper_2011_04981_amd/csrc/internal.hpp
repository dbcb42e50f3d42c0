// internal.hpp -- shared declarations of libnbx's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>

#include "../../include/nbx.h"

namespace nbx {

// Records the HIP error for nbx_last_hip_error() and returns NBX_EHIP.
int hip_fail(hipError_t e, const char *what);

#define NBX_HIP(call)                                              \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return ::nbx::hip_fail(e_, #call);   \
    } while (0)

#define NBX_LAUNCH_CHECK()                                         \
    do {                                                           \
        hipError_t e_ = hipGetLastError();                         \
        if (e_ != hipSuccess) return ::nbx::hip_fail(e_, "launch");\
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

constexpr int kMaxN = 16;

// Geometric factors.  Every G of the C ABI is [E][6][N^3], one plane per
// factor (gp_index).  Inside a problem the library keeps its own copy in
// three planes of factor pairs per element, (g1,g2), (g3,g4), (g5,g6), one
// pair per node, so that the solvers' fused operator fetches a pair with
// one 16-byte (FP64) or 8-byte (FP32) load (g_index); nbx_ax_paired takes
// that layout too.  Factor f of node p of element e:
__host__ __device__ inline int64_t gp_index(int64_t e, int f, int64_t p, int N3)
{
    return (e * 6 + f) * N3 + p;
}
__host__ __device__ inline int64_t g_index(int64_t e, int f, int64_t p, int N3)
{
    return ((e * 3 + (f >> 1)) * N3 + p) * 2 + (f & 1);
}
// [E][6][N^3] planes to factor pairs (dst must not overlap src); async.
int pair_factors_launch(const double *g6, double *g_pairs, int N, int64_t E, hipStream_t s);

// GLL nodes / weights / derivative matrix computed on the host.
int gll_host(int N, double *xi, double *w);
void deriv_host(int N, const double *xi, double *D);

// Gather-scatter plan (device arrays).
struct GsPlan {
    int64_t n_local = 0;
    int32_t n_groups = 0;       // shared groups (>= 2 copies)
    int32_t n_mask_only = 0;    // Dirichlet nodes with a single copy
    int32_t *off = nullptr;     // [n_groups+1]
    int32_t *idx = nullptr;     // [off[n_groups]] local indices
    uint8_t *gflag = nullptr;   // [n_groups] 1 = Dirichlet group
    int32_t *mask_idx = nullptr;// [n_mask_only]
    uint8_t *info = nullptr;    // [n_local] bits 0..6 multiplicity, bit 7 Dirichlet
};

// The exchange plan of the solvers' iterations, derived from a full plan:
// two-copy non-Dirichlet groups whose local indices are a and a + xd with
// xd = N^3 - N + 1 and a % N == N - 1 (the last x-face node of a row of an
// element and the first of the same row in the next element, the
// lexicographic element order's x neighbour) leave the plan, and the update
// kernel sums them from w instead, reading the pair's second value from a
// line that its neighbourhood streams anyway.  The derived plan's info byte
// carries the multiplicity in bits 0..4 (kXpMult), kXpNext at a, kXpPrev at
// a + xd, and the Dirichlet bit 7.  Synchronous (reads the full plan back);
// *found = 0, and nothing allocated, when no such pair exists or a
// multiplicity exceeds kXpMult.
constexpr uint8_t kXpMult = 0x1f, kXpNext = 0x20, kXpPrev = 0x40;
inline int64_t xpair_offset(int N) { return (int64_t)N * N * N - N + 1; }
int xpair_plan(const GsPlan &full, int N, GsPlan &out, int *found);
void free_plan(GsPlan &p);

// The step that forms alpha = rho / <p, A p> from the fused stage's nb
// per-workgroup partials (the solvers' one-block reduction R1), run by one
// more workgroup of the exchange launch: the partials are complete when
// the exchange starts, nothing in the exchange reads alpha, and the
// iteration saves a launch.
struct PapTask {
    int nb = 0;
    const double *part = nullptr;
    double *scal = nullptr;
};

// Enqueue dssum on a double or float vector.  With `flag` (device), the
// kernels do nothing once *flag != 0 (a finished solve).  With pap, the
// launch also performs that reduction (bit for bit the solvers' one-block
// kernel: same block size, same code).
template <typename T>
int dssum_launch(const GsPlan &gs, T *v, int apply_mask, hipStream_t s,
                 const double *flag = nullptr, const PapTask *pap = nullptr);

// AX launch (double / float) on factor pairs, the solvers' layout.
int ax_launch_f64(const double *u, const double *G, const double *D, int N, int64_t E,
                  double *w, hipStream_t s);
int ax_launch_f32(const float *u, const float *G, const double *D, int N, int64_t E,
                  float *w, hipStream_t s);

// Fused PCG first stage: p = z + beta p; w = AX(p); part[blk] = sum p*w.
// The number of partials written is ax_blocks(prec, N, E).
int ax_pcg_launch_f64(const double *G, const double *D, int N, int64_t E, const double *z,
                      double *p, double *w, double *part, const double *scal, hipStream_t s);
int ax_pcg_launch_f32(const float *G, const double *D, int N, int64_t E, const float *z,
                      float *p, float *w, double *part, const double *scal, hipStream_t s);
// AX with 16-bit geometric factors (gprec NBX_F16 or NBX_BF16; G16 holds
// G_e / gscale[e]) on FP32 vectors, plain and fused; tiles as for NBX_F32.
int ax_launch_g16(int gprec, const float *u, const void *G16, const float *gscale,
                  const double *D, int N, int64_t E, float *w, hipStream_t s);
int ax_pcg_launch_g16(int gprec, const void *G16, const float *gscale, const double *D, int N,
                      int64_t E, const float *z, float *p, float *w, double *part,
                      const double *scal, hipStream_t s);
// The FP32 operator on matrix cores (ax_mfma.hip): plain, on FP32 planes
// (gprec NBX_F32) or 16-bit words (NBX_F16 / NBX_BF16 with gscale); fused
// first stage on the problem's FP32 pairs or 16-bit words, one partial per
// element.
int ax_mfma_launch(int gprec, const float *u, const void *G, const float *gscale,
                   const double *D, int N, int64_t E, float *w, hipStream_t s);
int ax_mfma_pcg_launch(int gprec, const void *G, const float *gscale, const double *D, int N,
                       int64_t E, const float *z, float *p, float *w, double *part,
                       const double *scal, hipStream_t s);
// Packs G (FP64, planes != 0: [E][6][N^3], else factor pairs) into the
// 16-bit words and per-element scales of the reduced-storage operator.
int g16_pack_launch(int gprec, int planes, const double *G, int N, int64_t E, void *G16,
                    float *gscale, hipStream_t s);
// Elements per workgroup currently selected for (prec, N): ax_tile for the
// plain operator, pcg_tile for the fused first stage of the solvers; and
// the resulting number of fused-stage workgroups (partials) for E elements.
int ax_tile(int prec, int N);
int pcg_tile(int prec, int N);
int ax_blocks(int prec, int N, int64_t E);

// Jacobi diagonal of each element (unassembled).
int jacobi_diag_launch(const double *G, const double *D, int N, int64_t E, double *diag,
                       hipStream_t s);

}  // namespace nbx

struct nbx_gs {
    nbx::GsPlan plan;
};
