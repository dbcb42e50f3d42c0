// solver_kernels.hpp -- vector updates and deterministic reductions of the
// CG iteration (Section II-B: vector operations and global reductions),
// templated on the vector type (FP64 solve, FP32 inner solve).  Scalars and
// all dot products stay in FP64; partial sums are combined in a fixed
// order, so reruns are bitwise identical.
#pragma once

#include "internal.hpp"

namespace nbx {
namespace sk {
namespace {   // internal linkage: each solver translation unit has its own copy

constexpr int kRedThreads = 256;
// Workgroups of a streaming vector kernel: one 16-byte vector per lane up
// to this many (more resident waves keep more HBM requests in flight: the
// FP64 update runs ~15 % faster than with 4096 grid-striding blocks).
constexpr int kMaxRedBlocks = 1 << 17;
constexpr double kFlagLimit = 3.0;

__device__ inline double wsum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// This thread's share of the per-workgroup partial pairs part[2q], part[2q+1]
// (q < nb, strided by the block size), in four independent accumulators so
// the loads overlap; fixed order, hence deterministic.
__device__ inline void partial_sums2(int nb, const double *__restrict__ part, double &a,
                                     double &b)
{
    const int st = blockDim.x;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0, b0 = 0, b1 = 0, b2 = 0, b3 = 0;
    int q = threadIdx.x;
    for (; q + 3 * st < nb; q += 4 * st) {
        a0 += part[2 * q];              b0 += part[2 * q + 1];
        a1 += part[2 * (q + st)];       b1 += part[2 * (q + st) + 1];
        a2 += part[2 * (q + 2 * st)];   b2 += part[2 * (q + 2 * st) + 1];
        a3 += part[2 * (q + 3 * st)];   b3 += part[2 * (q + 3 * st) + 1];
    }
    for (; q < nb; q += st) { a0 += part[2 * q]; b0 += part[2 * q + 1]; }
    a = (a0 + a1) + (a2 + a3);
    b = (b0 + b1) + (b2 + b3);
}

// Same for single partials part[q].
__device__ inline double partial_sum1(int nb, const double *__restrict__ part)
{
    const int st = blockDim.x;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    int q = threadIdx.x;
    for (; q + 3 * st < nb; q += 4 * st) {
        a0 += part[q]; a1 += part[q + st]; a2 += part[q + 2 * st]; a3 += part[q + 3 * st];
    }
    for (; q < nb; q += st) a0 += part[q];
    return (a0 + a1) + (a2 + a3);
}

// Two sums over a kRedThreads block, fixed order; valid in thread 0.
__device__ inline void block_sum2(double &a, double &b)
{
    __shared__ double s[2][kRedThreads / 64];
    a = wsum(a); b = wsum(b);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { s[0][wid] = a; s[1][wid] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0, y = 0;
        for (int q = 0; q < kRedThreads / 64; ++q) { x += s[0][q]; y += s[1][q]; }
        a = x; b = y;
    }
}

__device__ inline double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Per-node weight 1/multiplicity (info bits 0..6).
__device__ inline double cw(uint8_t info) { return 1.0 / (double)(info & 0x7f); }

// The same weight from the solvers' x-pair info byte (xpair_plan).
__device__ inline double cw_x(uint8_t info) { return 1.0 / (double)(info & kXpMult); }

// Workgroups for a vector kernel over n values, w values (one 16-byte
// vector) per lane.
inline int red_blocks(int64_t n, int w = 2)
{
    int64_t b = (n + (int64_t)w * kRedThreads - 1) / ((int64_t)w * kRedThreads);
    if (b > kMaxRedBlocks) b = kMaxRedBlocks;
    return (int)(b < 1 ? 1 : b);
}

// Start of a solve from x = 0 with right-hand side b (type TB, converted to
// T): x = 0, r = b, z = dinv r, p = 0; partials of c r r and c r z.
// Block blk of nblk (grid-stride within one vector).
template <typename T, typename TB>
__device__ __forceinline__ void
init_body(int64_t n, const TB *__restrict__ b, const T *__restrict__ dinv,
          const uint8_t *__restrict__ info, T *__restrict__ x, T *__restrict__ r,
          T *__restrict__ z, T *__restrict__ p, double *__restrict__ part, int64_t blk,
          int64_t nblk)
{
    double rr = 0, rz = 0;
    for (int64_t l = blk * blockDim.x + threadIdx.x; l < n; l += nblk * blockDim.x) {
        const T rv = (T)b[l], zv = dinv[l] * rv;
        const double c = cw(info[l]);
        x[l] = 0; r[l] = rv; z[l] = zv; p[l] = 0;
        rr += c * (double)rv * (double)rv;
        rz += c * (double)rv * (double)zv;
    }
    block_sum2(rr, rz);
    if (threadIdx.x == 0) { part[2 * blk] = rr; part[2 * blk + 1] = rz; }
}

template <typename T, typename TB>
__global__ void __launch_bounds__(kRedThreads)
init_kernel(int64_t n, const TB *__restrict__ b, const T *__restrict__ dinv,
            const uint8_t *__restrict__ info, T *__restrict__ x, T *__restrict__ r,
            T *__restrict__ z, T *__restrict__ p, double *__restrict__ part)
{
    init_body<T, TB>(n, b, dinv, info, x, r, z, p, part, blockIdx.x, gridDim.x);
}

// scal <- fresh state: RR = BB = sum of the first partials, RHO = second,
// STOP = rtol^2 BB (or -1), MAXIT, FLAG (converged at once if BB == 0).
__device__ __forceinline__ void
init_reduce_body(int nb, const double *__restrict__ part, double *__restrict__ scal,
                 double rtol, int fixed, int max_iter);

__global__ void __launch_bounds__(1024)
init_reduce_kernel(int nb, const double *__restrict__ part, double *__restrict__ scal,
                   double rtol, int fixed, int max_iter)
{
    init_reduce_body(nb, part, scal, rtol, fixed, max_iter);
}

__device__ __forceinline__ void
init_reduce_body(int nb, const double *__restrict__ part, double *__restrict__ scal,
                 double rtol, int fixed, int max_iter)
{
    __shared__ double s[2][16];
    double a, b;
    partial_sums2(nb, part, a, b);
    a = wsum(a); b = wsum(b);
    if ((threadIdx.x & 63) == 0) { s[0][threadIdx.x >> 6] = a; s[1][threadIdx.x >> 6] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double bb = 0, rho = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) { bb += s[0][q]; rho += s[1][q]; }
        for (int q = 0; q < NBX_SCAL_LEN; ++q) scal[q] = 0.0;
        scal[NBX_S_BB] = bb;
        scal[NBX_S_RHO] = rho;
        scal[NBX_S_RR] = bb;
        scal[NBX_S_STOP] = fixed ? -1.0 : rtol * rtol * bb;
        scal[NBX_S_MAXIT] = (double)max_iter;
        scal[NBX_S_FLAG] = (bb == 0.0) ? 1.0 : (max_iter <= 0 ? kFlagLimit : 0.0);
    }
}

// R1: pap from the AX partials; alpha; breakdown check.  One 1024-thread
// block per scalar block.
__device__ __forceinline__ void
pap_reduce_body(int nb, const double *__restrict__ part, double *__restrict__ scal)
{
    if (scal[NBX_S_FLAG] != 0.0) return;
    __shared__ double s[16];
    double a = partial_sum1(nb, part);
    a = wsum(a);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double pap = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) pap += s[q];
        scal[NBX_S_PAP] = pap;
        if (!(pap > 0.0) || !isfinite(pap)) scal[NBX_S_FLAG] = 2.0;
        else scal[NBX_S_ALPHA] = scal[NBX_S_RHO] / pap;
    }
}

__global__ void __launch_bounds__(1024)
pap_reduce_kernel(int nb, const double *__restrict__ part, double *__restrict__ scal)
{
    pap_reduce_body(nb, part, scal);
}

template <typename T> struct Vec;
template <> struct Vec<double> {
    typedef double v __attribute__((ext_vector_type(2)));
    typedef uint16_t iv;
    static constexpr int W = 2;
};
template <> struct Vec<float> {
    typedef float v __attribute__((ext_vector_type(4)));
    typedef uint32_t iv;
    static constexpr int W = 4;
};

// The exchange of an x-face pair done inside K3: the assembled value of a
// pair (a, a + xd) is the exchange's own sum, (0 + w[a]) + w[a + xd] with
// the lower local index first, so the result has the same bits.  wo is the
// partner's value (read by position, see update_body).
template <typename T>
__device__ __forceinline__ T xpair_w(T wl, T wo, uint8_t inf)
{
    T s = 0;
    if (inf & kXpNext) { s += wl; s += wo; return s; }
    if (inf & kXpPrev) { s += wo; s += wl; return s; }
    return wl;
}

// The partner value a node may need: x-pair nodes sit at the ends of the
// element rows (i = N - 1 pairs with l + xd, i = 0 with l - xd), so the
// load depends on the position only and is issued with the stream's own
// loads instead of after the info byte has arrived.
template <typename T>
__device__ __forceinline__ T xpair_partner(const T *__restrict__ w, int64_t l, uint32_t i,
                                           int xn, int64_t xd, int64_t n)
{
    if (i == (uint32_t)xn - 1 && l + xd < n) return w[l + xd];
    if (i == 0 && l >= xd) return w[l - xd];
    return 0;
}

// K3: x += alpha p; r -= alpha w; z = dinv r; partials of c r r and c r z.
// Vector accesses of 16 bytes per lane, scalar tail.  With XP, info is the
// solvers' xinfo and the x-face pairs are summed here (xpair_w).
template <typename T, bool XP = false>
__device__ __forceinline__ void
update_body(int64_t n, const T *__restrict__ p, const T *__restrict__ w,
            const T *__restrict__ dinv, const uint8_t *__restrict__ info, T *__restrict__ x,
            T *__restrict__ r, T *__restrict__ z, double *__restrict__ part,
            const double *__restrict__ scal, int64_t blk, int64_t nblk, int64_t xd = 0,
            int xn = 0)
{
    if (scal[NBX_S_FLAG] != 0.0) return;
    using V = Vec<T>;
    constexpr int W = V::W;
    const T alpha = (T)scal[NBX_S_ALPHA];
    double rr = 0, rz = 0;
    const int64_t nv = n / W;
    const typename V::v *pv = reinterpret_cast<const typename V::v *>(p);
    const typename V::v *wv = reinterpret_cast<const typename V::v *>(w);
    const typename V::v *dv = reinterpret_cast<const typename V::v *>(dinv);
    typename V::v *xv = reinterpret_cast<typename V::v *>(x);
    typename V::v *rv = reinterpret_cast<typename V::v *>(r);
    typename V::v *zv = reinterpret_cast<typename V::v *>(z);
    const typename V::iv *iv = reinterpret_cast<const typename V::iv *>(info);
    // every array is streamed once per iteration (and exceeds the caches at
    // benchmark sizes): non-temporal loads and stores throughout
    for (int64_t q = blk * blockDim.x + threadIdx.x; q < nv; q += nblk * blockDim.x) {
        const typename V::v pq = __builtin_nontemporal_load(pv + q);
        const typename V::v wq = __builtin_nontemporal_load(wv + q);
        const typename V::v dq = __builtin_nontemporal_load(dv + q);
        typename V::v xq = __builtin_nontemporal_load(xv + q);
        typename V::v rq = __builtin_nontemporal_load(rv + q);
        typename V::v zq;
        const typename V::iv inf = __builtin_nontemporal_load(iv + q);
        [[maybe_unused]] T wo[W];
        if constexpr (XP) {
            // n < 2^31 (the exchange plan's limit): 32-bit position arithmetic
            uint32_t i = (uint32_t)(q * W) % (uint32_t)xn;
#pragma unroll
            for (int c = 0; c < W; ++c) {
                wo[c] = xpair_partner<T>(w, q * W + c, i, xn, xd, n);
                i = i + 1 == (uint32_t)xn ? 0 : i + 1;
            }
        }
#pragma unroll
        for (int c = 0; c < W; ++c) {
            const uint8_t ic = (uint8_t)(inf >> (8 * c));
            T wc = wq[c];
            if constexpr (XP) wc = xpair_w<T>(wc, wo[c], ic);
            xq[c] = fmaT(alpha, pq[c], xq[c]);
            rq[c] = fmaT(-alpha, wc, rq[c]);
            zq[c] = dq[c] * rq[c];
            const double cc = XP ? cw_x(ic) : cw(ic);
            rr += cc * (double)rq[c] * (double)rq[c];
            rz += cc * (double)rq[c] * (double)zq[c];
        }
        __builtin_nontemporal_store(xq, xv + q);
        __builtin_nontemporal_store(rq, rv + q);
        __builtin_nontemporal_store(zq, zv + q);
    }
    if (blk == 0 && threadIdx.x == 0) {
        for (int64_t l = nv * W; l < n; ++l) {
            x[l] = fmaT(alpha, p[l], x[l]);
            T wl = w[l];
            if constexpr (XP)
                wl = xpair_w<T>(wl, xpair_partner<T>(w, l, (uint32_t)(l % xn), xn, xd, n),
                                info[l]);
            const T rl = fmaT(-alpha, wl, r[l]), zl = dinv[l] * rl;
            const double cc = XP ? cw_x(info[l]) : cw(info[l]);
            r[l] = rl; z[l] = zl;
            rr += cc * (double)rl * (double)rl;
            rz += cc * (double)rl * (double)zl;
        }
    }
    block_sum2(rr, rz);
    if (threadIdx.x == 0) { part[2 * blk] = rr; part[2 * blk + 1] = rz; }
}

// Workgroups are dealt to the 8 XCDs round-robin; renumbered so that each
// XCD takes one contiguous range of chunks, the neighbouring chunks (and
// an x-face pair's two values, N^3 - N + 1 apart) share its L2.  A
// bijection of [0, nblk) that keeps block 0 first, so the partial sums
// land in the same slots as without it.
__device__ __forceinline__ int64_t xcd_block(int64_t blk, int64_t nblk)
{
    const int64_t per = nblk / 8, rem = nblk % 8, x = blk % 8;
    return x * per + (x < rem ? x : rem) + blk / 8;
}

template <typename T>
__global__ void __launch_bounds__(kRedThreads)
update_kernel(int64_t n, const T *__restrict__ p, const T *__restrict__ w,
              const T *__restrict__ dinv, const uint8_t *__restrict__ info, T *__restrict__ x,
              T *__restrict__ r, T *__restrict__ z, double *__restrict__ part,
              const double *__restrict__ scal)
{
    update_body<T>(n, p, w, dinv, info, x, r, z, part, scal, xcd_block(blockIdx.x, gridDim.x),
                   gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(kRedThreads)
update_xp_kernel(int64_t n, const T *__restrict__ p, const T *__restrict__ w,
                 const T *__restrict__ dinv, const uint8_t *__restrict__ info,
                 T *__restrict__ x, T *__restrict__ r, T *__restrict__ z,
                 double *__restrict__ part, const double *__restrict__ scal, int64_t xd,
                 int xn)
{
    update_body<T, true>(n, p, w, dinv, info, x, r, z, part, scal,
                         xcd_block(blockIdx.x, gridDim.x), gridDim.x, xd, xn);
}

// R3: rr, rho'; convergence / breakdown / iteration limit; beta.  With
// stamp, the device wall clock at convergence is stored there.
__device__ __forceinline__ void
rr_reduce_body(int nb, const double *__restrict__ part, double *__restrict__ scal,
               double *__restrict__ stamp = nullptr)
{
    if (scal[NBX_S_FLAG] != 0.0) return;
    __shared__ double s[2][16];
    double a, b;
    partial_sums2(nb, part, a, b);
    a = wsum(a); b = wsum(b);
    if ((threadIdx.x & 63) == 0) { s[0][threadIdx.x >> 6] = a; s[1][threadIdx.x >> 6] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double rr = 0, rz = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) { rr += s[0][q]; rz += s[1][q]; }
        const double it = scal[NBX_S_ITER] + 1.0;
        scal[NBX_S_ITER] = it;
        scal[NBX_S_RR] = rr;
        if (rr <= scal[NBX_S_STOP]) {
            scal[NBX_S_FLAG] = 1.0;
        } else if (!(rz > 0.0) || !isfinite(rz) || !isfinite(rr)) {
            scal[NBX_S_FLAG] = 2.0;
        } else {
            scal[NBX_S_BETA] = rz / scal[NBX_S_RHO];
            scal[NBX_S_RHO] = rz;
            if (it >= scal[NBX_S_MAXIT]) scal[NBX_S_FLAG] = kFlagLimit;
        }
        if (stamp && scal[NBX_S_FLAG] != 0.0) *stamp = (double)wall_clock64();
    }
}

__global__ void __launch_bounds__(1024)
rr_reduce_kernel(int nb, const double *__restrict__ part, double *__restrict__ scal)
{
    rr_reduce_body(nb, part, scal);
}

// Partials of c (b - w)^2 and c b^2 (FP64 residual of a refinement step);
// optionally stores r = b - w.
__global__ void __launch_bounds__(kRedThreads)
resid_kernel(int64_t n, const double *__restrict__ b, const double *__restrict__ w,
             const uint8_t *__restrict__ info, double *__restrict__ r, double *__restrict__ part)
{
    double a = 0, c2 = 0;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (int64_t)gridDim.x * blockDim.x) {
        const double c = cw(info[l]), d = b[l] - w[l];
        if (r) r[l] = d;
        a += c * d * d; c2 += c * b[l] * b[l];
    }
    block_sum2(a, c2);
    if (threadIdx.x == 0) { part[2 * blockIdx.x] = a; part[2 * blockIdx.x + 1] = c2; }
}

__global__ void __launch_bounds__(1024)
sum2_kernel(int nb, const double *__restrict__ part, double *__restrict__ out)
{
    __shared__ double s[2][16];
    double a, b;
    partial_sums2(nb, part, a, b);
    a = wsum(a); b = wsum(b);
    if ((threadIdx.x & 63) == 0) { s[0][threadIdx.x >> 6] = a; s[1][threadIdx.x >> 6] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0, y = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) { x += s[0][q]; y += s[1][q]; }
        out[0] = x; out[1] = y;
    }
}

}  // namespace
}  // namespace sk
}  // namespace nbx
