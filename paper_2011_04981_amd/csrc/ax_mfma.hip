// ax_mfma.hip -- the FP32 spectral-element operator on matrix cores, for
// the reduced-precision inner iterations (the paper names reduced precision
// as further work, Section V).
//
// The column-per-lane kernel of ax_kernel.hpp reads every u, wr and ws
// value N times from LDS for the r and s contractions (~257 B of LDS per
// node in FP32 with 16-bit factors), which, not HBM, sets its time.  Here
// the six length-N contractions of w_e = D^T G_e D u_e (Listing 1:
// local_grad3, the geometric step, local_grad3_t) become 16x16x4 FP32
// matrix-core products, D (or D^T) times the element's values arranged
// with the contracted index as the inner dimension:
//   r: UR[i][(j,k)] = sum_m D[i][m] u(m,j,k)    B[m][c] = u at m + N c
//   s: US[j][(i,k)] = sum_m D[j][m] u(i,m,k)    B[m][c] = u at c%N + N m + N^2 (c/N)
//   t: UT[k][(i,j)] = sum_m D[k][m] u(i,j,m)    B[m][c] = u at c + N^2 m
// so one A operand (D, N padded to 16 rows and to 4-wide k-steps) serves all
// three directions, and the transposed contractions take D^T the same way.
// One 64-lane wave owns one element:
//   1. u (or p = z + beta p) streamed into LDS, node per lane, coalesced;
//   2. the three forward products, results to three LDS slabs;
//   3. node per lane: the six factors (coalesced loads), wr, ws, wt written
//      over the slabs;
//   4. D^T products: the r result goes to the r slab, the s and t products
//      start their accumulators from it (each direction visits its own
//      node layout), so the last one holds w;
//   5. node per lane: w (and, fused, p and the <p, w> partial) to HBM.
// LDS per node is ~25 values read or written instead of ~64; the padding
// (N = 10 in 16-row tiles, 12-deep k-steps, 112 columns) costs matrix-core
// time, which the HBM stream hides.  Products are FP32 with FP32
// accumulation: the same precision class as the FP32 kernels, not their
// bits.
#include "ax_kernel.hpp"

namespace nbx {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int N>
struct MfmaShape {
    static constexpr int N2 = N * N, N3 = N2 * N;
    static constexpr int NT = (N2 + 15) / 16;     // 16-column tiles
    static constexpr int NK = (N + 3) / 4;        // 4-deep k-steps
    static constexpr int CMAX = 16 * NT - 1, MMAX = 4 * NK - 1;
    static constexpr int amax(int a, int b) { return a > b ? a : b; }
    // highest LDS address any B operand reads (padding rows and columns)
    static constexpr int HI = amax(amax(MMAX + N * CMAX, (N - 1) + N * MMAX + N2 * (CMAX / N)),
                                   CMAX + N2 * MMAX);
    static constexpr int SLAB = ((HI + 1) + 3) / 4 * 4;
    static constexpr size_t lds_bytes() { return 4 * SLAB * sizeof(float); }
};

// node of output row `row`, column `c` (and of B row `row`, column `c`)
template <int N, int DIR>
__device__ __forceinline__ int mf_node(int row, int c)
{
    if constexpr (DIR == 0) return row + N * c;
    else if constexpr (DIR == 1) return (c % N) + N * row + N * N * (c / N);
    else return c + N * N * row;
}

// acc[t] (+)= A * B over the k-steps for every column tile of direction DIR;
// a[s] is this lane's A operand of k-step s, B read from slab `src`.
template <int N, int DIR>
__device__ __forceinline__ void mf_products(const float *a, const float *src, f32x4 *acc,
                                            int lane)
{
    using S = MfmaShape<N>;
    const int cl = lane & 15, ml = lane >> 4;
#pragma unroll
    for (int t = 0; t < S::NT; ++t) {
        const int c = 16 * t + cl;
#pragma unroll
        for (int s = 0; s < S::NK; ++s) {
            const float b = src[mf_node<N, DIR>(4 * s + ml, c)];
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b, acc[t], 0, 0, 0);
        }
    }
}

// lane holds rows 4*(lane/16) + q, column 16 t + lane%16 of each tile
template <int N, int DIR>
__device__ __forceinline__ void mf_store(const f32x4 *acc, float *dst, int lane)
{
    using S = MfmaShape<N>;
#pragma unroll
    for (int t = 0; t < S::NT; ++t) {
        const int c = 16 * t + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = 4 * (lane >> 4) + q;
            if (row < N && c < S::N2) dst[mf_node<N, DIR>(row, c)] = acc[t][q];
        }
    }
}

template <int N, int DIR>
__device__ __forceinline__ void mf_load(f32x4 *acc, const float *src, int lane)
{
    using S = MfmaShape<N>;
#pragma unroll
    for (int t = 0; t < S::NT; ++t) {
        const int c = 16 * t + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = 4 * (lane >> 4) + q;
            acc[t][q] = (row < N && c < S::N2) ? src[mf_node<N, DIR>(row, c)] : 0.f;
        }
    }
}

template <int N>
__device__ __forceinline__ void mf_zero(f32x4 *acc)
{
#pragma unroll
    for (int t = 0; t < MfmaShape<N>::NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// PCG == false: w = AX(u).  PCG == true: uin is z; p <- z + beta p (stored);
// w = AX(p); part[element] = sum of p * w over the element (skipped once
// scal[FLAG] != 0).  G as in ax_body: factor pairs (T or 16-bit words with
// gscale) or, with PL, one plane per factor.
template <int N, bool PCG, typename GT, bool PL>
__global__ void __launch_bounds__(64)
ax_mfma_kernel(const float *__restrict__ uin, const GT *__restrict__ G,
               const double *__restrict__ Dg, float *__restrict__ w, float *__restrict__ pio,
               double *__restrict__ part, const double *__restrict__ scal, int64_t E,
               const float *__restrict__ gscale)
{
#pragma clang fp contract(off)
    using S = MfmaShape<N>;
    constexpr int N3 = S::N3, SL = S::SLAB;
    constexpr bool kHalfG = !std::is_same<GT, float>::value;
    __shared__ float su[SL], sr[SL], ss[SL], st[SL];
    if constexpr (PCG) {
        if (scal[NBX_S_FLAG] != 0.0) return;
    }
    const int lane = threadIdx.x;
    const int64_t e = blockIdx.x;
    const size_t base = (size_t)e * N3;
    const GT *Ge = G + (size_t)e * 6 * N3;

    // 1. u (or p = z + beta p) into LDS; the slabs' padding to zero, so that
    //    padded k-steps (A = 0) never meet a non-finite B
    const float beta = PCG ? (float)scal[NBX_S_BETA] : 0.f;
    for (int p = lane; p < N3; p += 64) {
        float v;
        if constexpr (PCG) {
            v = ax_fma(beta, pio[base + p], uin[base + p]);
            ax_st_nt(v, pio + base + p);
        } else {
            v = uin[base + p];
        }
        su[p] = v;
    }
    for (int p = N3 + lane; p < SL; p += 64) { su[p] = 0.f; sr[p] = 0.f; ss[p] = 0.f; st[p] = 0.f; }
    // A operands: D (rows i, k-step columns m) and D^T, zero outside N x N
    float aD[S::NK], aT[S::NK];
    {
        const int row = lane & 15;
#pragma unroll
        for (int s = 0; s < S::NK; ++s) {
            const int m = 4 * s + (lane >> 4);
            const bool in = row < N && m < N;
            aD[s] = in ? (float)Dg[row * N + m] : 0.f;
            aT[s] = in ? (float)Dg[m * N + row] : 0.f;
        }
    }
    __syncthreads();

    // 2. the forward products
    f32x4 acc[S::NT];
    mf_zero<N>(acc);
    mf_products<N, 0>(aD, su, acc, lane);
    mf_store<N, 0>(acc, sr, lane);
    mf_zero<N>(acc);
    mf_products<N, 1>(aD, su, acc, lane);
    mf_store<N, 1>(acc, ss, lane);
    mf_zero<N>(acc);
    mf_products<N, 2>(aD, su, acc, lane);
    mf_store<N, 2>(acc, st, lane);
    __syncthreads();

    // 3. the geometric step, node per lane
    for (int p = lane; p < N3; p += 64) {
        float g1, g2, g3, g4, g5, g6;
        ax_gpair<float, GT, PL, N3>(Ge, 0, p, g1, g2);
        ax_gpair<float, GT, PL, N3>(Ge, 1, p, g3, g4);
        ax_gpair<float, GT, PL, N3>(Ge, 2, p, g5, g6);
        const float ur = sr[p], us = ss[p], ut = st[p];
        sr[p] = ax_fma(g3, ut, ax_fma(g2, us, g1 * ur));
        ss[p] = ax_fma(g5, ut, ax_fma(g4, us, g2 * ur));
        st[p] = ax_fma(g6, ut, ax_fma(g5, us, g3 * ur));
    }
    __syncthreads();

    // 4. D^T products; the running sum lives in the r slab, which each
    //    direction reads and writes in its own node layout
    mf_zero<N>(acc);
    mf_products<N, 0>(aT, sr, acc, lane);
    mf_store<N, 0>(acc, sr, lane);
    __syncthreads();
    mf_load<N, 1>(acc, sr, lane);
    mf_products<N, 1>(aT, ss, acc, lane);
    mf_store<N, 1>(acc, sr, lane);
    __syncthreads();
    mf_load<N, 2>(acc, sr, lane);
    mf_products<N, 2>(aT, st, acc, lane);
    mf_store<N, 2>(acc, sr, lane);
    __syncthreads();

    // 5. w to HBM (scaled back for 16-bit factors), node per lane
    const float gsc = kHalfG ? gscale[e] : 1.f;
    double pw = 0.0;
    for (int p = lane; p < N3; p += 64) {
        float v = sr[p];
        if constexpr (kHalfG) v *= gsc;
        ax_st_nt(v, w + base + p);
        if constexpr (PCG) pw += (double)su[p] * (double)v;
    }
    if constexpr (PCG) {
        pw = ax_wave_sum(pw);
        if (lane == 0) part[e] = pw;
    }
    (void)E;
}

template <bool PCG, typename GT, bool PL>
int mfma_launch(int N, const float *u, const GT *G, const double *D, float *w, float *p,
                double *part, const double *scal, int64_t E, hipStream_t s, const float *gscale)
{
    if (E <= 0) return NBX_OK;
    if (E > 0x7fffffffLL) return NBX_EUNSUPPORTED;
#define NBX_MF_CASE(NN)                                                                      \
    case NN:                                                                                 \
        hipLaunchKernelGGL((ax_mfma_kernel<NN, PCG, GT, PL>), dim3((unsigned)E), dim3(64), 0, \
                           s, u, G, D, w, p, part, scal, E, gscale);                         \
        break;
    switch (N) {
        NBX_MF_CASE(2) NBX_MF_CASE(3) NBX_MF_CASE(4) NBX_MF_CASE(5) NBX_MF_CASE(6)
        NBX_MF_CASE(7) NBX_MF_CASE(8) NBX_MF_CASE(9) NBX_MF_CASE(10) NBX_MF_CASE(11)
        NBX_MF_CASE(12) NBX_MF_CASE(13) NBX_MF_CASE(14) NBX_MF_CASE(15) NBX_MF_CASE(16)
        default: return NBX_EINVAL;
    }
#undef NBX_MF_CASE
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

}  // namespace

// Plain operator on FP32 planes ([E][6][N^3], the C ABI's layout) or on
// 16-bit words (gprec NBX_F16 / NBX_BF16, with gscale).
int ax_mfma_launch(int gprec, const float *u, const void *G, const float *gscale,
                   const double *D, int N, int64_t E, float *w, hipStream_t s)
{
    if (gprec == NBX_F32)
        return mfma_launch<false, float, true>(N, u, (const float *)G, D, w, nullptr, nullptr,
                                               nullptr, E, s, nullptr);
    if (gprec == NBX_F16)
        return mfma_launch<false, g_f16, false>(N, u, (const g_f16 *)G, D, w, nullptr, nullptr,
                                                nullptr, E, s, gscale);
    if (gprec == NBX_BF16)
        return mfma_launch<false, g_bf16, false>(N, u, (const g_bf16 *)G, D, w, nullptr,
                                                 nullptr, nullptr, E, s, gscale);
    return NBX_EUNSUPPORTED;
}

// The solvers' fused first stage on the problem's FP32 factor pairs or
// 16-bit words; one partial per element.
int ax_mfma_pcg_launch(int gprec, const void *G, const float *gscale, const double *D, int N,
                       int64_t E, const float *z, float *p, float *w, double *part,
                       const double *scal, hipStream_t s)
{
    if (gprec == NBX_F32)
        return mfma_launch<true, float, false>(N, z, (const float *)G, D, w, p, part, scal, E, s,
                                               nullptr);
    if (gprec == NBX_F16)
        return mfma_launch<true, g_f16, false>(N, z, (const g_f16 *)G, D, w, p, part, scal, E,
                                               s, gscale);
    if (gprec == NBX_BF16)
        return mfma_launch<true, g_bf16, false>(N, z, (const g_bf16 *)G, D, w, p, part, scal, E,
                                                s, gscale);
    return NBX_EUNSUPPORTED;
}

}  // namespace nbx

using namespace nbx;

extern "C" int nbx_ax_mfma(int gprec, const float *u, const void *G, const float *gscale,
                           const double *D, int N, int64_t E, float *w, void *stream)
{
    if (N < 2 || N > kMaxN || E < 0) return NBX_EINVAL;
    if (gprec != NBX_F32 && gprec != NBX_F16 && gprec != NBX_BF16) return NBX_EUNSUPPORTED;
    if (E == 0) return NBX_OK;
    if (!u || !G || !D || !w || u == w) return NBX_EINVAL;
    if (gprec != NBX_F32 && !gscale) return NBX_EINVAL;
    return ax_mfma_launch(gprec, u, G, gscale, D, N, E, w, as_stream(stream));
}
