// ax16_mfma.hpp -- the FP64 operator w_e = D^T G_e D u_e (Section II-B,
// Listing 1) at N = 16, the paper's large-element size (16^3 points per
// element, Table II), with the r and s contractions on the matrix cores.
//
// At N = 16 each r or s contraction of a k-slab is a whole 16x16x16 product,
// so FP64 16x16x4 matrix-core products (v_mfma_f64_16x16x4f64) carry them
// with no padding.  The column-per-lane kernel of ax_kernel.hpp reads ~64
// LDS values per node for those contractions and their transposes, and at
// N = 16 its 98 KB of LDS leaves one workgroup per CU, so that LDS time and
// the element's HBM stream do not overlap.  Here a node costs ~15 LDS
// accesses, and a workgroup needs 40 KB of LDS and 148 VGPRs: three
// workgroups per CU.
//
// Layout.  A workgroup of four waves owns one element; wave v owns the
// k-slabs 4v .. 4v+3.  Lane l = 16 g + c (g = l / 16, c = l % 16).  The
// product's result layout -- lane l, register r holds row g + 4 r, column c
// of the 16x16 result -- is the layout of every per-node value of a slab:
// register r of lane l holds node (i = c, j = 4 r + g), offset 64 r + l in
// the slab, so each u load, factor load and w store of a slab is one
// contiguous 512-byte request of the wave.  With U_k the slab as a matrix
// [j][i] and steps s = 0..3 of 4-deep k-steps over m = 4 s + g:
//   ws = D U_k        A = D[c][4s+g] (registers)     B = U_k[4s+g][c] (LDS)
//   wr = U_k D^T      A = U_k[c][4s+g] (LDS)         B = D[c][4s+g]   (registers)
//   wt = sum_m D[k][m] U_m             vector FMAs, U_m read from LDS
//   gr, gs, gt        the geometric step, per node (six factor planes)
//   w  = D^T gs       A = D[4s+g][c] (registers)     B = gs, register s (the
//                                                    result layout is the
//                                                    B layout of step s)
//      + gr D         A = gr[c][4s+g] (transposed through LDS)  B = D[4s+g][c]
//      + sum_m D[m][k] gt_m            vector FMAs, gt_m read from LDS
// LDS slabs are 16x16 with row j's entries permuted by i -> i ^ (j & 14):
// a half-wave's row reads (two whole rows) and column reads (two columns of
// all 16 rows) both touch 32 distinct 8-byte bank pairs.  In the plain
// operator gt of slab k is written over u's slab k once every wave has read
// u for its t contraction and the owning wave has taken slab k's r and s
// products; the fused stage keeps p in u's slabs for <p, w> and writes gt
// to slabs of its own (72 KB, two workgroups per CU).  Measured at E = 8000
// against a kernel with padded 17-double rows, separate gt slabs and the
// next slab's factors prefetched (76 KB, 209 VGPRs, two workgroups per
// CU): 306 against 310-317 us, same bits.
// Products accumulate in FP64; the results agree with the vector-unit
// kernel to rounding, not bit for bit (a different summation order).
// The body serves the plain operator (ax16_mfma.hip) and the solvers' fused
// first stage (PCG: p = z + beta p stored, w = AX(p), one <p, w> partial
// per element), standalone and batched.
#pragma once

#include "internal.hpp"

namespace nbx {
namespace ax16 {

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4 mf(double a, double b, f64x4 acc)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}

// LDS slot of entry (j, i) of a 16x16 slab
__device__ __forceinline__ int sw(int j, int i) { return j * 16 + (i ^ (j & 14)); }

// LDS values one lane wrote are read by other lanes of the same wave: LDS
// requests of a wave complete in order, so a wave-scope fence suffices.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The six factors of the lane's four nodes of slab k: from one plane per
// factor (PL, [6][4096] per element) or from the factor pairs ([3][4096][2]
// per element, one 16-byte load per pair).
template <bool PL>
__device__ __forceinline__ void factors(const double *Ge, int k, int l, double (&gv)[6][4])
{
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int node = k * 256 + 64 * r + l;
        if constexpr (PL) {
#pragma unroll
            for (int p = 0; p < 6; ++p)
                gv[p][r] = __builtin_nontemporal_load(Ge + p * 4096 + node);
        } else {
            typedef double pair_t __attribute__((ext_vector_type(2)));
#pragma unroll
            for (int h = 0; h < 3; ++h) {
                const pair_t v = __builtin_nontemporal_load(
                    reinterpret_cast<const pair_t *>(Ge) + h * 4096 + node);
                gv[2 * h][r] = v.x;
                gv[2 * h + 1][r] = v.y;
            }
        }
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// One element (blk) per 256-thread workgroup.
// PCG == false: w = AX(uin).
// PCG == true : uin is z; p <- z + beta p (pio, stored); w = AX(p);
//               part[blk] = sum over the element of p w (in the lane order
//               below, then the wave sum, then the four waves in order);
//               the whole block returns at once when scal[FLAG] != 0.
template <bool PL, bool PCG>
__device__ __forceinline__ void body(const double *__restrict__ uin, const double *__restrict__ G,
                                     const double *__restrict__ D, double *__restrict__ w,
                                     double *__restrict__ pio, double *__restrict__ part,
                                     const double *__restrict__ scal, int64_t blk)
{
#pragma clang fp contract(off)
    // u slabs (swizzled); the plain operator then writes gt (per-node
    // layout) over them, the fused stage keeps p there for <p, w> and puts
    // gt in slabs of its own (72 KB instead of 40: two workgroups per CU,
    // as its registers allow anyway)
    __shared__ double s_u[16 * 256];
    __shared__ double s_gt_own[PCG ? 16 * 256 : 1];
    __shared__ double s_gr[4 * 256];   // one slab of gr per wave (swizzled)
    __shared__ double s_red[4];
    double *const s_gt = PCG ? s_gt_own : s_u;

    if constexpr (PCG) {
        if (scal[NBX_S_FLAG] != 0.0) return;   // uniform: solve finished
    }
    const int l = threadIdx.x & 63;
    const int k0 = 4 * __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = l >> 4, c = l & 15;
    const size_t e = (size_t)blk;
    const double *ue = uin + e * 4096;
    const double *Ge = G + e * 6 * 4096;
    double *we = w + e * 4096;

    // 1. u (or p = z + beta p) of the wave's four slabs to LDS
    double uv[4][4];
    if constexpr (PCG) {
        const double beta = scal[NBX_S_BETA];
        double *pe = pio + e * 4096;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = (k0 + q) * 256 + 64 * r + l;
                uv[q][r] = __builtin_fma(beta, pe[o], ue[o]);
            }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                __builtin_nontemporal_store(uv[q][r], pe + (k0 + q) * 256 + 64 * r + l);
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) uv[q][r] = ue[(k0 + q) * 256 + 64 * r + l];
    }
    double Da[4], Db[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        Da[s] = D[c * 16 + 4 * s + g];
        Db[s] = D[(4 * s + g) * 16 + c];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) s_u[(k0 + q) * 256 + sw(4 * r + g, c)] = uv[q][r];
    __syncthreads();

    // 2. wt of the wave's four slabs: sum_m D[k][m] u(c, 4r+g, m)
    double wt[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) wt[q][r] = 0.0;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        double x[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = s_u[m * 256 + sw(4 * r + g, c)];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double d = D[(k0 + q) * 16 + m];
#pragma unroll
            for (int r = 0; r < 4; ++r) wt[q][r] = __builtin_fma(d, x[r], wt[q][r]);
        }
    }
    if constexpr (!PCG) __syncthreads();   // every wave's t reads of u done: gt may go over u

    // 3. slab by slab: ws and wr on the matrix cores, the geometric step,
    // then the r and s transposes into the slab's accumulator
    f64x4 W[4];
    double *sg = s_gr + (k0 / 4) * 256;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = k0 + q;
        const double *su = s_u + k * 256;
        f64x4 ws = {0.0, 0.0, 0.0, 0.0}, wr = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            ws = mf(Da[s], su[sw(4 * s + g, c)], ws);
            wr = mf(su[sw(c, 4 * s + g)], Da[s], wr);
        }
        double gv[6][4];
        factors<PL>(Ge, k, l, gv);
        if constexpr (!PCG) wave_lds_sync();   // the slab's u reads before its gt writes
        double gs[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double a = wr[r], b = ws[r], t = wt[q][r];
            const double gr =
                __builtin_fma(gv[2][r], t, __builtin_fma(gv[1][r], b, gv[0][r] * a));
            gs[r] = __builtin_fma(gv[4][r], t, __builtin_fma(gv[3][r], b, gv[1][r] * a));
            const double gt =
                __builtin_fma(gv[5][r], t, __builtin_fma(gv[4][r], b, gv[2][r] * a));
            s_gt[k * 256 + 64 * r + l] = gt;
            sg[sw(4 * r + g, c)] = gr;
        }
        wave_lds_sync();
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = mf(Db[s], gs[s], acc);
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = mf(sg[sw(c, 4 * s + g)], Db[s], acc);
        W[q] = acc;
        wave_lds_sync();   // this slab's gr reads before the next slab's writes
    }
    __syncthreads();

    // 4. the t transpose from every wave's gt, then w
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        double x[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = s_gt[m * 256 + 64 * r + l];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double d = D[m * 16 + k0 + q];
#pragma unroll
            for (int r = 0; r < 4; ++r) W[q][r] = __builtin_fma(d, x[r], W[q][r]);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            __builtin_nontemporal_store(W[q][r], we + (k0 + q) * 256 + 64 * r + l);
    if constexpr (PCG) {
        double pw = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                pw += s_u[(k0 + q) * 256 + sw(4 * r + g, c)] * W[q][r];
        pw = wave_sum(pw);
        if (l == 0) s_red[k0 / 4] = pw;
        __syncthreads();
        if (threadIdx.x == 0) part[blk] = ((s_red[0] + s_red[1]) + s_red[2]) + s_red[3];
    }
}

}  // namespace ax16
}  // namespace nbx
