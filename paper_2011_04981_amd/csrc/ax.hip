// ax.hip -- the matrix-free spectral-element operator w_e = D^T G_e D u_e
// (Section II-B, Listing 1: local_grad3, the per-node geometric
// contraction, local_grad3_t) for gfx950.
//
// Mapping (one workgroup per element):
//   * thread (i,j) owns the k-column u(i,j,0..N-1) in registers, so the
//     t-direction contractions (ut forward, the wt term backward) never
//     leave the register file;
//   * the element's u slab is staged once in LDS and serves the r and s
//     contractions (thread (i,j) reads row u(:,j,k) and column u(i,:,k));
//   * wr and ws go to two more LDS slabs for the transposed contractions;
//   * the six geometric-factor planes of the thread's column (75% of the
//     element's HBM bytes, read exactly once) are all requested with
//     non-temporal loads before any arithmetic starts, so that each wave
//     keeps ~6N x 8 B per lane in flight while it waits for u;
//   * uniform entries D[k][m] are read through the scalar cache, per-thread
//     rows and columns of D sit in registers.
// The D operand of the r/s contractions is the paper's dxm1 / dxtm1.
#include "internal.hpp"

namespace nbx {
namespace {

template <int N>
struct Cfg {
    static constexpr int N2 = N * N;
    static constexpr int N3 = N2 * N;
    static constexpr int NT = ((N2 + 63) / 64) * 64;
    // Prefetching all 6N factors costs 12N VGPRs in FP64; beyond N = 12
    // they are loaded slab by slab instead.
    static constexpr bool kPrefetch = N <= 12;
};

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over the block in a fixed order (deterministic); valid in thread 0.
template <int NT>
__device__ inline double block_sum(double v, double *s_red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) s_red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NT / 64; ++q) s += s_red[q];
    }
    return s;
}

template <typename T>
__device__ inline T ld_nt(const T *p) { return __builtin_nontemporal_load(p); }

// PCG == false: w = AX(u).
// PCG == true : u is z; p <- z + beta p (stored); w = AX(p);
//               part[e] = sum over the element of p*w.
template <typename T, int N, bool PCG>
__global__ void __launch_bounds__(Cfg<N>::NT)
ax_col(const T *__restrict__ uin, const T *__restrict__ G, const double *__restrict__ Dg,
       T *__restrict__ w, T *__restrict__ pio, double *__restrict__ part,
       const double *__restrict__ scal)
{
    constexpr int N2 = Cfg<N>::N2, N3 = Cfg<N>::N3, NT = Cfg<N>::NT;
    __shared__ T s_u[N3];
    __shared__ T s_wr[N3];
    __shared__ T s_ws[N3];
    __shared__ T s_D[N2];
    __shared__ double s_red[NT / 64];

    if constexpr (PCG) {
        if (scal[NBX_S_FLAG] != 0.0) return;   // uniform: solve finished
    }
    const int t = threadIdx.x;
    const bool act = t < N2;
    const int tc = act ? t : N2 - 1;          // idle lanes shadow a real column
    const int i = tc % N, j = tc / N;
    const size_t base = (size_t)blockIdx.x * N3;
    const T *Ge = G + (size_t)blockIdx.x * 6 * N3;

    for (int q = t; q < N2; q += NT) s_D[q] = (T)Dg[q];

    T g[Cfg<N>::kPrefetch ? 6 : 1][Cfg<N>::kPrefetch ? N : 1];
    if constexpr (Cfg<N>::kPrefetch) {
#pragma unroll
        for (int k = 0; k < N; ++k)
#pragma unroll
            for (int f = 0; f < 6; ++f) g[f][k] = ld_nt(Ge + f * N3 + k * N2 + tc);
    }

    T uc[N];
    if constexpr (PCG) {
        const T beta = (T)scal[NBX_S_BETA];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const T zv = uin[base + k * N2 + tc];
            const T pv = pio[base + k * N2 + tc];
            uc[k] = zv + beta * pv;
        }
        if (act) {
#pragma unroll
            for (int k = 0; k < N; ++k) pio[base + k * N2 + t] = uc[k];
        }
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) uc[k] = uin[base + k * N2 + tc];
    }
    if (act) {
#pragma unroll
        for (int k = 0; k < N; ++k) s_u[k * N2 + t] = uc[k];
    }
    __syncthreads();

    // ---- local_grad3 + geometric contraction, slab by slab
    T wt[N];
    {
        T Di[N], Dj[N];
#pragma unroll
        for (int m = 0; m < N; ++m) { Di[m] = s_D[i * N + m]; Dj[m] = s_D[j * N + m]; }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            T ur = 0, us = 0, ut = 0;
#pragma unroll
            for (int m = 0; m < N; ++m) ur += Di[m] * s_u[k * N2 + j * N + m];
#pragma unroll
            for (int m = 0; m < N; ++m) us += Dj[m] * s_u[k * N2 + m * N + i];
#pragma unroll
            for (int m = 0; m < N; ++m) ut += (T)Dg[k * N + m] * uc[m];
            T g1, g2, g3, g4, g5, g6;
            if constexpr (Cfg<N>::kPrefetch) {
                g1 = g[0][k]; g2 = g[1][k]; g3 = g[2][k]; g4 = g[3][k]; g5 = g[4][k]; g6 = g[5][k];
            } else {
                const T *gp = Ge + k * N2 + tc;
                g1 = ld_nt(gp); g2 = ld_nt(gp + N3); g3 = ld_nt(gp + 2 * N3);
                g4 = ld_nt(gp + 3 * N3); g5 = ld_nt(gp + 4 * N3); g6 = ld_nt(gp + 5 * N3);
            }
            const T wr = g1 * ur + g2 * us + g3 * ut;
            const T ws = g2 * ur + g4 * us + g5 * ut;
            wt[k] = g3 * ur + g5 * us + g6 * ut;
            if (act) { s_wr[k * N2 + t] = wr; s_ws[k * N2 + t] = ws; }
        }
    }
    __syncthreads();

    // ---- local_grad3_t: w = D^T wr + (ws D per slab) + wt D
    double pw = 0.0;
    {
        T DTi[N], DTj[N];
#pragma unroll
        for (int m = 0; m < N; ++m) { DTi[m] = s_D[m * N + i]; DTj[m] = s_D[m * N + j]; }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            T acc = 0;
#pragma unroll
            for (int m = 0; m < N; ++m) acc += DTi[m] * s_wr[k * N2 + j * N + m];
#pragma unroll
            for (int m = 0; m < N; ++m) acc += DTj[m] * s_ws[k * N2 + m * N + i];
#pragma unroll
            for (int m = 0; m < N; ++m) acc += (T)Dg[m * N + k] * wt[m];
            if (act) w[base + k * N2 + t] = acc;
            if constexpr (PCG) pw += (double)uc[k] * (double)acc;
        }
    }
    if constexpr (PCG) {
        if (!act) pw = 0.0;
        const double s = block_sum<NT>(pw, s_red);
        if (t == 0) part[blockIdx.x] = s;
    }
}

template <typename T, bool PCG>
int launch_n(int N, const T *u, const T *G, const double *D, T *w, T *p, double *part,
             const double *scal, int64_t E, hipStream_t s)
{
    if (E == 0) return NBX_OK;
    if (E > 0x7fffffffLL) return NBX_EUNSUPPORTED;
    const dim3 grid((unsigned)E);
#define NBX_AX_CASE(NN)                                                              \
    case NN:                                                                         \
        hipLaunchKernelGGL((ax_col<T, NN, PCG>), grid, dim3(Cfg<NN>::NT), 0, s, u, G, \
                           D, w, p, part, scal);                                     \
        break;
    switch (N) {
        NBX_AX_CASE(2) NBX_AX_CASE(3) NBX_AX_CASE(4) NBX_AX_CASE(5) NBX_AX_CASE(6)
        NBX_AX_CASE(7) NBX_AX_CASE(8) NBX_AX_CASE(9) NBX_AX_CASE(10) NBX_AX_CASE(11)
        NBX_AX_CASE(12) NBX_AX_CASE(13) NBX_AX_CASE(14) NBX_AX_CASE(15) NBX_AX_CASE(16)
        default: return NBX_EINVAL;
    }
#undef NBX_AX_CASE
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

}  // namespace

int ax_launch_f64(const double *u, const double *G, const double *D, int N, int64_t E,
                  double *w, hipStream_t s)
{
    return launch_n<double, false>(N, u, G, D, w, nullptr, nullptr, nullptr, E, s);
}

int ax_launch_f32(const float *u, const float *G, const double *D, int N, int64_t E,
                  float *w, hipStream_t s)
{
    return launch_n<float, false>(N, u, G, D, w, nullptr, nullptr, nullptr, E, s);
}

int ax_pcg_launch_f64(const double *G, const double *D, int N, int64_t E, const double *z,
                      double *p, double *w, double *part, const double *scal, hipStream_t s)
{
    return launch_n<double, true>(N, z, G, D, w, p, part, scal, E, s);
}

}  // namespace nbx

extern "C" int nbx_ax(int prec, const void *u, const void *G, const double *D, int N,
                      int64_t E, void *w, void *stream)
{
    if (N < 2 || N > nbx::kMaxN || E < 0) return NBX_EINVAL;
    if (E == 0) return NBX_OK;
    if (!u || !G || !D || !w) return NBX_EINVAL;
    if (u == w) return NBX_EINVAL;
    hipStream_t s = nbx::as_stream(stream);
    switch (prec) {
        case NBX_F64:
            return nbx::ax_launch_f64((const double *)u, (const double *)G, D, N, E,
                                      (double *)w, s);
        case NBX_F32:
            return nbx::ax_launch_f32((const float *)u, (const float *)G, D, N, E,
                                      (float *)w, s);
        default:
            return NBX_EUNSUPPORTED;
    }
}
