// ax_kernel.hpp -- the matrix-free spectral-element operator
// w_e = D^T G_e D u_e (Section II-B, Listing 1: local_grad3, the per-node
// geometric contraction, local_grad3_t) as one gfx950 kernel template.
//
// Mapping: a workgroup takes EPB consecutive elements; element el's
// N^2 (i,j) columns occupy lanes el*N^2 .. el*N^2 + N^2-1 (packed, the last
// wave padded to 64 lanes).  Lane (i,j) of an element
//   * keeps the k-column u(i,j,0..N-1) in registers, so the t-direction
//     contractions never leave the register file;
//   * stages its column in the element's LDS slab, from which the r and s
//     contractions read row u(:,j,k) and column u(i,:,k);
//   * writes wr, ws to two more LDS slabs for the transposed contractions
//     and keeps wt in registers.
// Memory order matters on MI355X's HBM3E: the u column is requested first,
// then all 6N geometric factors of the column as 3N non-temporal pair loads
// (75% of the element's bytes, read exactly once), so that the first slab's
// contractions overlap the factor stream; w is written with non-temporal
// stores.  Measured on the 32^3 brick at N = 10 this order is worth ~20%
// over plain loads and stores.  Uniform entries D[k][m] come through the
// scalar cache (converted to FP32 by the VALU in the FP32 kernels, which
// are bound by LDS traffic: taking them from LDS as broadcasts made the
// FP16-G fused stage 7 % slower); per-lane rows and columns of D sit in
// registers.
#pragma once

#include "internal.hpp"

#include <type_traits>

namespace nbx {

template <int N, int EPB>
struct AxShape {
    static constexpr int N2 = N * N;
    static constexpr int N3 = N2 * N;
    static constexpr int NACT = EPB * N2;                 // active lanes
    static constexpr int NT = ((NACT + 63) / 64) * 64;   // threads per block
    // k-slabs of the column's six factors requested at entry and held in
    // registers (6 PF values); the remaining slabs are loaded in the k
    // loop.  The whole column fits up to N = 10 in FP64 (12N VGPRs) and
    // N = 12 in FP32; larger elements keep the register file under 256.
    // FP64 N = 12 takes 4 so that the kernel fits 168 VGPRs: three waves
    // per SIMD, i.e. all three 3-wave workgroups that its LDS allows on a CU
    // (6 slabs, 190 VGPRs, ran 19 % slower there); LDS holds the other
    // large sizes to two waves per SIMD (or one), so they take as many slabs
    // as fit without spilling (measured on 16-25 M nodes: 3-9 % faster than
    // with 4 slabs at N = 11 and 13-16).
    template <typename T>
    static constexpr int pf()
    {
        return sizeof(T) == sizeof(double)
                   ? (N <= 10 ? N : (N == 11 ? 10 : (N == 12 ? 4 : 8)))
                   : (N <= 12 ? N : 8);
    }
    // LDS of one block (three element slabs per element, D, reduction
    // slots) within the CU's 160 KB, and at most 1024 threads.
    template <typename T>
    static constexpr bool fits()
    {
        return NT <= 1024 &&
               (3 * EPB * N3 + N2) * sizeof(T) + (NT / 64) * sizeof(double) <= 160 * 1024;
    }
};

// Large elements take the uniform entries of D slab by slab (see ax_body):
// FP64 from N = 11, FP32 arithmetic from N = 13, where the factor loads are
// pinned too; smaller ones leave their order to the compiler.
template <typename T, int N>
constexpr bool ax_pin_d()
{
    return sizeof(T) == sizeof(double) ? N >= 11 : N >= 13;
}

__device__ inline double ax_wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

template <typename T>
__device__ inline T ax_ld_nt(const T *p) { return __builtin_nontemporal_load(p); }

// Half-precision storage of the geometric factors (16-bit words holding
// FP16 or BF16 bits), widened to FP32 on load.
struct g_f16 { uint16_t bits; };
struct g_bf16 { uint16_t bits; };

// Factor pair q of an element's pair planes (q = h N^3 + node: factors 2h
// and 2h+1 of the node), streamed once: one non-temporal 16-byte (FP64),
// 8-byte (FP32) or 4-byte (16-bit storage, widened to FP32) load.
template <typename T, typename GT>
__device__ inline void ax_pair(const GT *Ge, int q, T &lo, T &hi)
{
    if constexpr (std::is_same<GT, T>::value) {
        typedef T pair_t __attribute__((ext_vector_type(2)));
        const pair_t v = __builtin_nontemporal_load(reinterpret_cast<const pair_t *>(Ge) + q);
        lo = v.x;
        hi = v.y;
    } else {
        const uint32_t wd = __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(Ge) + q);
        if constexpr (std::is_same<GT, g_f16>::value) {
            lo = (float)__builtin_bit_cast(_Float16, (uint16_t)(wd & 0xffffu));
            hi = (float)__builtin_bit_cast(_Float16, (uint16_t)(wd >> 16));
        } else {
            lo = __uint_as_float(wd << 16);
            hi = __uint_as_float(wd & 0xffff0000u);
        }
    }
}

// Factors 2h and 2h+1 of node `node` of an element (Ge points at the
// element's 6 N^3 values): one pair load from the pair planes, or (PL, the
// C ABI's [E][6][N^3] layout) two loads from planes 2h and 2h+1.
template <typename T, typename GT, bool PL, int N3>
__device__ inline void ax_gpair(const GT *Ge, int h, int node, T &lo, T &hi)
{
    if constexpr (PL) {
        static_assert(std::is_same<GT, T>::value, "planes hold T");
        lo = __builtin_nontemporal_load(Ge + (2 * h) * N3 + node);
        hi = __builtin_nontemporal_load(Ge + (2 * h + 1) * N3 + node);
    } else {
        ax_pair<T>(Ge, h * N3 + node, lo, hi);
    }
}

template <typename T>
__device__ inline void ax_st_nt(T v, T *p) { __builtin_nontemporal_store(v, p); }
// Fused multiply-add written out: every instantiation (tile, fused or not)
// then performs the same operation sequence and produces the same bits.
__device__ inline double ax_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float ax_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// PCG == false: w = AX(u).
// PCG == true : uin is z; p <- z + beta p (stored); w = AX(p);
//               part[block] = sum over the block's elements of p*w
//               (skipped entirely once scal[FLAG] != 0).
// blk selects the block's elements [blk*EPB, blk*EPB + EPB) of this
// operator instance (blockIdx.x for a single operator; a table entry when
// one launch serves several independent problems).
// G is in planes of factor pairs (g_index), or with PL in one plane per
// factor (gp_index, T storage only).  GT is its storage type (T,
// or g_f16 / g_bf16 with T = float); for 16-bit storage G_e holds
// G_e / gscale[e] (gscale[e] a power of two), each pair in one 32-bit word
// (see ax_pair), and
// the element's result is multiplied by gscale[e], which in FP32 is exact
// and commutes with every rounding of the element's arithmetic.
template <typename T, int N, int EPB, bool PCG, typename GT = T, bool PL = false>
__device__ __forceinline__ void
ax_body(const T *__restrict__ uin, const GT *__restrict__ G, const double *__restrict__ Dg,
        T *__restrict__ w, T *__restrict__ pio, double *__restrict__ part,
        const double *__restrict__ scal, int64_t E, int64_t blk,
        const float *__restrict__ gscale = nullptr)
{
#pragma clang fp contract(off)
    using S = AxShape<N, EPB>;
    constexpr int N2 = S::N2, N3 = S::N3, NT = S::NT, NACT = S::NACT;
    __shared__ T s_u[EPB * N3];
    __shared__ T s_wr[EPB * N3];
    __shared__ T s_ws[EPB * N3];
    __shared__ T s_D[N2];
    __shared__ double s_red[NT / 64];

    if constexpr (PCG) {
        if (scal[NBX_S_FLAG] != 0.0) return;   // uniform: solve finished
    }
    const int t = threadIdx.x;
    const bool lane_act = t < NACT;
    const int tl = lane_act ? t : NACT - 1;    // idle lanes shadow a real column
    const int el = tl / N2, tc = tl - el * N2;
    const int i = tc % N, j = tc / N;
    const int64_t e_raw = blk * EPB + el;
    const bool valid = lane_act && e_raw < E;  // ragged last block
    const int64_t e = e_raw < E ? e_raw : E - 1;
    const size_t base = (size_t)e * N3;
    const GT *Ge = G + (size_t)e * 6 * N3;
    constexpr bool kHalfG = !std::is_same<GT, T>::value;
    constexpr bool kPinD = ax_pin_d<T, N>();
    T *su = s_u + el * N3, *swr = s_wr + el * N3, *sws = s_ws + el * N3;

    // 1. the column of u (or of z and the previous p) first ...
    T uc[N];
    if constexpr (PCG) {
        const T beta = (T)scal[NBX_S_BETA];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const T zv = uin[base + k * N2 + tc];
            const T pv = pio[base + k * N2 + tc];
            uc[k] = ax_fma(beta, pv, zv);
        }
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) uc[k] = uin[base + k * N2 + tc];
    }
    // 2. ... then every geometric factor of the column, streamed once, a
    // pair per load (pair planes halve the load count against one plane per
    // factor: 6.1 -> 6.5 TB/s at N = 10 in FP64)
    constexpr int PF = S::template pf<T>();
    // plane-major order: consecutive requests cover consecutive addresses,
    // so a line shared by two slabs is asked for twice in a row
    T g[6][PF];
#pragma unroll
    for (int h = 0; h < 3; ++h)
#pragma unroll
        for (int k = 0; k < PF; ++k)
            ax_gpair<T, GT, PL, N3>(Ge, h, k * N2 + tc, g[2 * h][k], g[2 * h + 1][k]);
    for (int q = t; q < N2; q += NT) s_D[q] = (T)Dg[q];
    if constexpr (PCG) {
        if (valid) {
#pragma unroll
            for (int k = 0; k < N; ++k) ax_st_nt(uc[k], pio + base + k * N2 + tc);
        }
    }
    if (lane_act) {
#pragma unroll
        for (int k = 0; k < N; ++k) su[k * N2 + tc] = uc[k];
    }
    __syncthreads();

    // 3. local_grad3 and the geometric contraction, slab by slab
    T wt[N];
    {
        T Di[N], Dj[N];
#pragma unroll
        for (int m = 0; m < N; ++m) { Di[m] = s_D[i * N + m]; Dj[m] = s_D[j * N + m]; }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            T ur = 0, us = 0, ut = 0;
#pragma unroll
            for (int m = 0; m < N; ++m) ur = ax_fma(Di[m], su[k * N2 + j * N + m], ur);
#pragma unroll
            for (int m = 0; m < N; ++m) us = ax_fma(Dj[m], su[k * N2 + m * N + i], us);
            // D[k][0..N-1] comes through the scalar cache; for large
            // elements the row's offset is tied to the previous slab's result,
            // as the factor loads below are, so that the compiler does not
            // hoist all N^2 uniform values to the top (more than the SGPR
            // file: 146-436 SGPRs spilled to VGPR lanes at N = 11-16 in FP64,
            // 13-16 in FP32)
            int dk = k * N;
            if constexpr (kPinD)
                if (k > 0) asm volatile("" : "+s"(dk) : "v"(wt[k - 1]));
#pragma unroll
            for (int m = 0; m < N; ++m)
                ut = ax_fma((T)Dg[dk + m], uc[m], ut);
            T g1, g2, g3, g4, g5, g6;
            if (k < PF) {
                g1 = g[0][k]; g2 = g[1][k]; g3 = g[2][k]; g4 = g[3][k]; g5 = g[4][k]; g6 = g[5][k];
            } else {
                // large FP64 elements: tie this slab's factor loads to the
                // previous slab's result so the scheduler cannot hoist all of
                // them to the top (6N live values spilled the register file;
                // measured 1.3-1.6x faster at N = 12-14; N = 15 runs faster
                // without)
                int off = k * N2 + tc;
                if constexpr ((sizeof(T) == sizeof(double) && N >= 11 && N != 15) ||
                              (sizeof(T) == sizeof(float) && N >= 13))
                    asm volatile("" : "+v"(off) : "v"(wt[k - 1]));
                ax_gpair<T, GT, PL, N3>(Ge, 0, off, g1, g2);
                ax_gpair<T, GT, PL, N3>(Ge, 1, off, g3, g4);
                ax_gpair<T, GT, PL, N3>(Ge, 2, off, g5, g6);
            }
            const T wr = ax_fma(g3, ut, ax_fma(g2, us, g1 * ur));
            const T ws = ax_fma(g5, ut, ax_fma(g4, us, g2 * ur));
            wt[k] = ax_fma(g6, ut, ax_fma(g5, us, g3 * ur));
            if (lane_act) { swr[k * N2 + tc] = wr; sws[k * N2 + tc] = ws; }
        }
    }
    __syncthreads();

    // 4. local_grad3_t: w = D^T wr + (ws D per slab) + wt D
    double pw = 0.0;
    T gsc = (T)1;
    [[maybe_unused]] T last = 0;   // the previous output, which the next column of D waits for
    if constexpr (kHalfG) gsc = (T)gscale[e];
    {
        T DTi[N], DTj[N];
#pragma unroll
        for (int m = 0; m < N; ++m) { DTi[m] = s_D[m * N + i]; DTj[m] = s_D[m * N + j]; }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            T acc = 0;
#pragma unroll
            for (int m = 0; m < N; ++m) acc = ax_fma(DTi[m], swr[k * N2 + j * N + m], acc);
#pragma unroll
            for (int m = 0; m < N; ++m) acc = ax_fma(DTj[m], sws[k * N2 + m * N + i], acc);
            int dc = k;
            if constexpr (kPinD)
                if (k > 0) asm volatile("" : "+s"(dc) : "v"(last));
#pragma unroll
            for (int m = 0; m < N; ++m)
                acc = ax_fma((T)Dg[m * N + dc], wt[m], acc);
            if constexpr (kHalfG) acc *= gsc;
            if (valid) ax_st_nt(acc, w + base + k * N2 + tc);
            last = acc;
            if constexpr (PCG) pw += (double)uc[k] * (double)acc;
        }
    }
    if constexpr (PCG) {
        if (!valid) pw = 0.0;
        pw = ax_wave_sum(pw);
        if ((t & 63) == 0) s_red[t >> 6] = pw;
        __syncthreads();
        if (t == 0) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < NT / 64; ++q) s += s_red[q];
            part[blk] = s;
        }
    }
}

template <typename T, int N, int EPB, bool PCG, typename GT = T, bool PL = false>
__global__ void __launch_bounds__((AxShape<N, EPB>::NT))
ax_kernel(const T *__restrict__ uin, const GT *__restrict__ G, const double *__restrict__ Dg,
          T *__restrict__ w, T *__restrict__ pio, double *__restrict__ part,
          const double *__restrict__ scal, int64_t E, const float *__restrict__ gscale)
{
    ax_body<T, N, EPB, PCG, GT, PL>(uin, G, Dg, w, pio, part, scal, E, (int64_t)blockIdx.x,
                                    gscale);
}

// Elements per workgroup the library may use (the autotuner's search space).
constexpr int kEpbChoices[] = {1, 2, 4, 8};

template <typename T, bool PCG, int N, typename GT = T, bool PL = false>
int ax_launch_epb(int epb, const T *u, const GT *G, const double *D, T *w, T *p, double *part,
                  const double *scal, int64_t E, hipStream_t s, const float *gscale = nullptr)
{
#define NBX_EPB_CASE(EE)                                                                     \
    case EE: {                                                                               \
        if constexpr (AxShape<N, EE>::template fits<T>()) {                                  \
            constexpr int NT_ = AxShape<N, EE>::NT;                                          \
            const int64_t nb = (E + EE - 1) / EE;                                            \
            hipLaunchKernelGGL((ax_kernel<T, N, EE, PCG, GT, PL>), dim3((unsigned)nb),    \
                               dim3(NT_),                                              \
                               0, s, u, G, D, w, p, part, scal, E, gscale);                  \
            return NBX_OK;                                                                   \
        } else {                                                                             \
            return NBX_EUNSUPPORTED;                                                         \
        }                                                                                    \
    }
    switch (epb) {
        NBX_EPB_CASE(1)
        NBX_EPB_CASE(2)
        NBX_EPB_CASE(4)
        NBX_EPB_CASE(8)
        default: return NBX_EINVAL;
    }
#undef NBX_EPB_CASE
}

template <typename T, bool PCG, typename GT = T, bool PL = false>
int ax_launch_any(int N, int epb, const T *u, const GT *G, const double *D, T *w, T *p,
                  double *part, const double *scal, int64_t E, hipStream_t s,
                  const float *gscale = nullptr)
{
    if (E <= 0) return NBX_OK;
    if ((E + epb - 1) / epb > 0x7fffffffLL) return NBX_EUNSUPPORTED;
    int st;
#define NBX_N_CASE(NN)                                                                     \
    case NN:                                                                               \
        st = ax_launch_epb<T, PCG, NN, GT, PL>(epb, u, G, D, w, p, part, scal, E, s,       \
                                               gscale);                                    \
        break;
    switch (N) {
        NBX_N_CASE(2) NBX_N_CASE(3) NBX_N_CASE(4) NBX_N_CASE(5) NBX_N_CASE(6)
        NBX_N_CASE(7) NBX_N_CASE(8) NBX_N_CASE(9) NBX_N_CASE(10) NBX_N_CASE(11)
        NBX_N_CASE(12) NBX_N_CASE(13) NBX_N_CASE(14) NBX_N_CASE(15) NBX_N_CASE(16)
        default: return NBX_EINVAL;
    }
#undef NBX_N_CASE
    if (st != NBX_OK) return st;
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

}  // namespace nbx
