// learned.hip -- the learned element-interior preconditioner bound to a
// problem, its training rows, and the flexible CG that uses it.
//
// The paper's CG uses a "simple preconditioner" (Section II-B, read as
// Jacobi).  The learned operator keeps Jacobi on every node except each
// element's learned interior nodes S (interior, one copy, off the Dirichlet
// set), where
//     z_S = (1/gd_e) L^T diag(gamma_e) L r_S
// with the model of lpi.hip: L shared by all elements, gamma_e from the
// perceptron on the element's normalised mean factors, computed once per
// binding.  The nodes in S belong to one element each, so the operator
// needs no exchange and is symmetric positive definite: a fixed SPD
// preconditioner.  Its BF16 products make it linear only to rounding, so
// the solve is flexible CG (Notay 2000, one stored direction:
// beta = -<z', A p> / <p, A p>), which tolerates that.
//
// Application per CG iteration: r_S gathered into BF16 rows [E][nIp] by
// the update step that produces r, one GEMM X L^T with the gains
// multiplied in its epilogue (BF16 out), one GEMM with L (FP32 out), and
// the kernel that forms z, <r, z>_c and <z, A p>_c.  The node-wise kernels
// are instantiated per N, so the node-to-interior-index arithmetic needs no
// run-time division.
//
// Training rows from a vector v the FP64 solver produced (an error x* - x,
// formed here as the difference of two vectors, or a residual r):
// X = A_SS v_S / (|v_S| gd_e), T = v_S / |v_S|, and the element's features;
// A_SS v_S is AX of v with every node outside S set to zero, read on S.
#include "solver.hpp"
#include "solver_kernels.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <new>

struct nbx_mlp;
struct nbx_lpi;

namespace nbx {

int gemm_bf16(int ta, int tb, int epi, int M, int N, int K, const uint16_t *A, int lda,
              const uint16_t *B, int ldb, float *C, int ldc, uint16_t *Cb, int ldcb,
              const float *bias, const uint16_t *act, int ldact, hipStream_t s,
              const float *mul);
int mlp_forward_rows(nbx_mlp *P, const uint16_t *X, int B, float *Y, hipStream_t s);
int lpi_dims(const nbx_lpi *M, int *N, int *nI, int *nIp);
const uint16_t *lpi_Lb(const nbx_lpi *M);
nbx_mlp *lpi_mlp(const nbx_lpi *M);
int lpi_max_batch(const nbx_lpi *M);

namespace {

constexpr int kEpiF32 = 0, kEpiMulBf16 = 5;   // GEMM epilogues of mlp.hip
constexpr int kFeat = 64;                     // feature row width (six used)
constexpr int64_t kGemmRows = 1 << 21;        // rows per GEMM launch (grid.y < 2^16)

__device__ __forceinline__ uint16_t lp_f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline double lp_block_sum(double v, double *s)
{
    v = sk::wsum(v);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += s[q];
    __syncthreads();
    return t;
}

// Local node number of interior node q (the interior's own order, i fastest).
__device__ __forceinline__ int lp_inode(int q, int N)
{
    const int m = N - 2;
    const int i = 1 + q % m, j = 1 + (q / m) % m, k = 1 + q / (m * m);
    return i + N * (j + N * k);
}

// A learned node: one copy and not Dirichlet (info = multiplicity | 0x80
// on the Dirichlet set).
__device__ __forceinline__ bool lp_learned(uint8_t info) { return info == 1; }

// gfeat[e][0..5] = element means of the six factors / gd, gfeat[e][6] = gd,
// igd[e] = 1 / gd; G in the problem's factor pairs.
__global__ void __launch_bounds__(256)
lp_geom_kernel(int N3, const double *__restrict__ G, float *__restrict__ gfeat,
               double *__restrict__ igd)
{
    __shared__ double s[4];
    const int64_t e = blockIdx.x;
    double m[6];
    for (int f = 0; f < 6; ++f) {
        double a = 0.0;
        for (int q = threadIdx.x; q < N3; q += blockDim.x) a += G[g_index(e, f, q, N3)];
        m[f] = lp_block_sum(a, s) / N3;
    }
    const double gd = (m[0] + m[3] + m[5]) / 3.0;
    if (threadIdx.x < 8) {
        const int f = threadIdx.x;
        gfeat[e * 8 + f] = f < 6 ? (float)(m[f] / gd) : (f == 6 ? (float)gd : 0.f);
    }
    if (threadIdx.x == 0) igd[e] = 1.0 / gd;
}

// F[e] = bf16 features (six, zeros to 64); rows e >= E zero.
__global__ void lp_feat_rows_kernel(int64_t E, int64_t Epad, const float *__restrict__ gfeat,
                                    uint16_t *__restrict__ F)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Epad * kFeat) return;
    const int64_t e = t / kFeat;
    const int c = (int)(t - e * kFeat);
    F[t] = (e < E && c < 6) ? lp_f2bf(gfeat[e * 8 + c]) : (uint16_t)0;
}

__global__ void lp_softplus_kernel(int64_t n, float *__restrict__ a)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const float v = a[q];
        a[q] = log1pf(expf(-fabsf(v))) + fmaxf(v, 0.f);
    }
}

// X[e][q] = bf16(r at interior node q) on learned nodes, 0 elsewhere and in
// the padding (q >= nI, e >= E).
__global__ void lp_gather_kernel(int N, int nI, int nIp, int64_t E, int64_t Epad,
                                 const double *__restrict__ r, const uint8_t *__restrict__ info,
                                 uint16_t *__restrict__ X, const double *__restrict__ flag)
{
    if (flag && *flag != 0.0) return;
    const int64_t N3 = (int64_t)N * N * N;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < Epad * nIp;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = t / nIp;
        const int q = (int)(t - e * nIp);
        uint16_t v = 0;
        if (e < E && q < nI) {
            const int64_t l = e * N3 + lp_inode(q, N);
            if (lp_learned(info[l])) v = lp_f2bf((float)r[l]);
        }
        X[t] = v;
    }
}

// z at local node l: the learned value on learned interior nodes, Jacobi
// elsewhere.
__device__ __forceinline__ double lp_z(int N, int64_t N3, int64_t l, double rl, double dl,
                                       uint8_t inf, const float *__restrict__ Zi, int nIp,
                                       const double *__restrict__ igd)
{
    const int64_t e = l / N3;
    const int p = (int)(l - e * N3);
    const int i = p % N, j = (p / N) % N, k = p / (N * N);
    if (i > 0 && i < N - 1 && j > 0 && j < N - 1 && k > 0 && k < N - 1 && lp_learned(inf)) {
        const int m = N - 2;
        const int q = (i - 1) + m * ((j - 1) + m * (k - 1));
        return (double)Zi[e * nIp + q] * igd[e];
    }
    return dl * rl;
}

// beta = -<z_new, w> / <p, w> (0 on the first application);
// rho = <r, z_new>; breakdown if it is not positive.
__global__ void __launch_bounds__(1024)
lp_beta_kernel(int nb, const double *__restrict__ part, double *__restrict__ scal, int first)
{
    if (scal[NBX_S_FLAG] != 0.0) return;
    __shared__ double s[2][16];
    double a, b;
    sk::partial_sums2(nb, part, a, b);
    a = sk::wsum(a); b = sk::wsum(b);
    if ((threadIdx.x & 63) == 0) { s[0][threadIdx.x >> 6] = a; s[1][threadIdx.x >> 6] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double rzn = 0, zw = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) { rzn += s[0][q]; zw += s[1][q]; }
        if (!(rzn > 0.0) || !isfinite(rzn) || !isfinite(zw)) {
            scal[NBX_S_FLAG] = 2.0;
            return;
        }
        scal[NBX_S_BETA] = first ? 0.0 : -zw / scal[NBX_S_PAP];
        scal[NBX_S_RHO] = rzn;
    }
}

// Interior index of node p of an element (N a compile-time constant, so
// the divisions become multiplications), -1 off the interior.
template <int N>
__device__ __forceinline__ int lp_iq(int p)
{
    const int i = p % N, j = (p / N) % N, k = p / (N * N);
    if (i == 0 || i == N - 1 || j == 0 || j == N - 1 || k == 0 || k == N - 1) return -1;
    constexpr int m = N - 2;
    return (i - 1) + m * ((j - 1) + m * (k - 1));
}

// The update step with the next application's gather fused in: x += alpha
// p; r -= alpha w; partials of c r r; and X[e][q] = bf16(r) on learned
// interior nodes, 0 on the other interior nodes (the padding of X stays as
// set at binding).  Two values per lane, the iteration's one pass over r.
template <int N>
__device__ __forceinline__ void lp_upd_node(int64_t l, double pl, double wl, uint8_t inf,
                                            double alpha, double &xl, double &rl, double &rr,
                                            int nIp, uint16_t *__restrict__ X)
{
    constexpr int64_t N3 = (int64_t)N * N * N;
    xl = __builtin_fma(alpha, pl, xl);
    rl = __builtin_fma(-alpha, wl, rl);
    rr += sk::cw(inf) * rl * rl;
    const int64_t e = l / N3;
    const int q = lp_iq<N>((int)(l - e * N3));
    if (q >= 0) X[e * nIp + q] = lp_learned(inf) ? lp_f2bf((float)rl) : (uint16_t)0;
}

template <int N>
__global__ void __launch_bounds__(sk::kRedThreads)
lp_update_gather_kernel(int64_t n, int nIp, const double *__restrict__ p,
                        const double *__restrict__ w, const uint8_t *__restrict__ info,
                        double *__restrict__ x, double *__restrict__ r,
                        uint16_t *__restrict__ X, double *__restrict__ part,
                        const double *__restrict__ scal)
{
    if (scal[NBX_S_FLAG] != 0.0) return;
    using V = sk::Vec<double>;
    const double alpha = scal[NBX_S_ALPHA];
    double rr = 0, one = 0;
    const int64_t nv = n / 2;
    const V::v *pv = reinterpret_cast<const V::v *>(p);
    const V::v *wv = reinterpret_cast<const V::v *>(w);
    V::v *xv = reinterpret_cast<V::v *>(x);
    V::v *rv = reinterpret_cast<V::v *>(r);
    const V::iv *iv = reinterpret_cast<const V::iv *>(info);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nv;
         q += (int64_t)gridDim.x * blockDim.x) {
        const V::v pq = __builtin_nontemporal_load(pv + q);
        const V::v wq = __builtin_nontemporal_load(wv + q);
        V::v xq = __builtin_nontemporal_load(xv + q);
        V::v rq = __builtin_nontemporal_load(rv + q);
        const V::iv inf = __builtin_nontemporal_load(iv + q);
        double x0 = xq[0], x1 = xq[1], r0 = rq[0], r1 = rq[1];
        lp_upd_node<N>(2 * q, pq[0], wq[0], (uint8_t)inf, alpha, x0, r0, rr, nIp, X);
        lp_upd_node<N>(2 * q + 1, pq[1], wq[1], (uint8_t)(inf >> 8), alpha, x1, r1, rr, nIp, X);
        xq[0] = x0; xq[1] = x1; rq[0] = r0; rq[1] = r1;
        __builtin_nontemporal_store(xq, xv + q);
        __builtin_nontemporal_store(rq, rv + q);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) {
        const int64_t l = n - 1;
        double xl = x[l], rl = r[l];
        lp_upd_node<N>(l, p[l], w[l], info[l], alpha, xl, rl, rr, nIp, X);
        x[l] = xl; r[l] = rl;
    }
    sk::block_sum2(rr, one);
    if (threadIdx.x == 0) { part[2 * blockIdx.x] = rr; part[2 * blockIdx.x + 1] = one; }
}

// z_new from r and the learned rows (Jacobi off the learned nodes);
// partials of <r, z_new>_c and <z_new, w>_c (w = A p of the step just
// taken; not read on the first application); z = z_new.  Two values per
// lane.
template <int N>
__device__ __forceinline__ double lp_zn(int64_t l, double rl, double dl, uint8_t inf,
                                        const float *__restrict__ Zi, int nIp,
                                        const double *__restrict__ igd)
{
    constexpr int64_t N3 = (int64_t)N * N * N;
    const int64_t e = l / N3;
    const int q = lp_iq<N>((int)(l - e * N3));
    if (q >= 0 && lp_learned(inf)) return (double)Zi[e * nIp + q] * igd[e];
    return dl * rl;
}

template <int N>
__global__ void __launch_bounds__(sk::kRedThreads)
lp_dots_n_kernel(int64_t n, const double *__restrict__ r, const double *__restrict__ dinv,
                 const uint8_t *__restrict__ info, const float *__restrict__ Zi, int nIp,
                 const double *__restrict__ igd, const double *__restrict__ w, int first,
                 double *__restrict__ z, double *__restrict__ part,
                 const double *__restrict__ scal)
{
    if (scal[NBX_S_FLAG] != 0.0) return;
    using V = sk::Vec<double>;
    double a = 0, b = 0;
    const int64_t nv = n / 2;
    const V::v *rv = reinterpret_cast<const V::v *>(r);
    const V::v *dv = reinterpret_cast<const V::v *>(dinv);
    const V::v *wv = reinterpret_cast<const V::v *>(w);
    V::v *zv = reinterpret_cast<V::v *>(z);
    const V::iv *iv = reinterpret_cast<const V::iv *>(info);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nv;
         q += (int64_t)gridDim.x * blockDim.x) {
        const V::v rq = __builtin_nontemporal_load(rv + q);
        const V::v dq = __builtin_nontemporal_load(dv + q);
        const V::iv inf = __builtin_nontemporal_load(iv + q);
        V::v zq;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const uint8_t ic = (uint8_t)(inf >> (8 * c));
            zq[c] = lp_zn<N>(2 * q + c, rq[c], dq[c], ic, Zi, nIp, igd);
            a += sk::cw(ic) * rq[c] * zq[c];
        }
        if (!first) {
            const V::v wq = __builtin_nontemporal_load(wv + q);
            b += sk::cw((uint8_t)inf) * zq[0] * wq[0];
            b += sk::cw((uint8_t)(inf >> 8)) * zq[1] * wq[1];
        }
        __builtin_nontemporal_store(zq, zv + q);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) {
        const int64_t l = n - 1;
        const double zn = lp_zn<N>(l, r[l], dinv[l], info[l], Zi, nIp, igd);
        a += sk::cw(info[l]) * r[l] * zn;
        if (!first) b += sk::cw(info[l]) * zn * w[l];
        z[l] = zn;
    }
    sk::block_sum2(a, b);
    if (threadIdx.x == 0) { part[2 * blockIdx.x] = a; part[2 * blockIdx.x + 1] = b; }
}

// ITER++, RR; FLAG = 1 when RR <= STOP, 3 at MAXIT.
__global__ void __launch_bounds__(1024)
lp_rr_kernel(int nb, const double *__restrict__ part, double *__restrict__ scal)
{
    if (scal[NBX_S_FLAG] != 0.0) return;
    __shared__ double s[16];
    double a, unused;
    sk::partial_sums2(nb, part, a, unused);
    a = sk::wsum(a);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double rr = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) rr += s[q];
        const double it = scal[NBX_S_ITER] + 1.0;
        scal[NBX_S_ITER] = it;
        scal[NBX_S_RR] = rr;
        if (rr <= scal[NBX_S_STOP]) scal[NBX_S_FLAG] = 1.0;
        else if (!isfinite(rr)) scal[NBX_S_FLAG] = 2.0;
        else if (it >= scal[NBX_S_MAXIT]) scal[NBX_S_FLAG] = sk::kFlagLimit;
    }
}

// z = M r (plain application, no dots)
__global__ void lp_out_kernel(int N, int64_t n, const double *__restrict__ r,
                              const double *__restrict__ dinv, const uint8_t *__restrict__ info,
                              const float *__restrict__ Zi, int nIp,
                              const double *__restrict__ igd, double *__restrict__ z)
{
    const int64_t N3 = (int64_t)N * N * N;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (int64_t)gridDim.x * blockDim.x)
        z[l] = lp_z(N, N3, l, r[l], dinv[l], info[l], Zi, nIp, igd);
}

// vm = v - v0 on learned interior nodes (v0 may be null), 0 elsewhere
__global__ void lp_mask_kernel(int N, int64_t n, const double *__restrict__ v,
                               const double *__restrict__ v0, const uint8_t *__restrict__ info,
                               double *__restrict__ vm)
{
    const int64_t N3 = (int64_t)N * N * N;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(l % N3);
        const int i = p % N, j = (p / N) % N, k = p / (N * N);
        const bool in = i > 0 && i < N - 1 && j > 0 && j < N - 1 && k > 0 && k < N - 1;
        vm[l] = (in && lp_learned(info[l])) ? (v0 ? v[l] - v0[l] : v[l]) : 0.0;
    }
}

// Training rows for the selected elements (one block per row), from the
// masked vector vm = v_S and y = A vm: with s = |v_S|, X = bf16(y_S / (s gd)),
// T = v_S / s, F = bf16 features; an element index outside [0, E) or
// v_S = 0 gives an all-zero row.
__global__ void __launch_bounds__(256)
lp_sample_kernel(int N, int nI, int nIp, int64_t E, const int32_t *__restrict__ elems,
                 const double *__restrict__ v, const double *__restrict__ y,
                 const uint8_t *__restrict__ info, const float *__restrict__ gfeat,
                 const double *__restrict__ igd, uint16_t *__restrict__ X,
                 float *__restrict__ T, uint16_t *__restrict__ F)
{
    __shared__ double s[4];
    const int row = blockIdx.x;
    const int64_t e = elems[row];
    uint16_t *xr = X + (size_t)row * nIp;
    float *tr = T + (size_t)row * nIp;
    uint16_t *fr = F + (size_t)row * kFeat;
    const int64_t N3 = (int64_t)N * N * N;
    const bool valid = e >= 0 && e < E;
    double ss = 0.0;
    if (valid) {
        for (int q = threadIdx.x; q < nI; q += blockDim.x) {
            const int64_t l = e * N3 + lp_inode(q, N);
            if (lp_learned(info[l])) ss += v[l] * v[l];
        }
    }
    const double nrm = sqrt(lp_block_sum(ss, s));
    if (!valid || !(nrm > 0.0)) {
        for (int q = threadIdx.x; q < nIp; q += blockDim.x) { xr[q] = 0; tr[q] = 0.f; }
        for (int c = threadIdx.x; c < kFeat; c += blockDim.x) fr[c] = 0;
        return;
    }
    const double inv = 1.0 / nrm, ig = igd[e];
    for (int q = threadIdx.x; q < nIp; q += blockDim.x) {
        uint16_t xv = 0;
        float tv = 0.f;
        if (q < nI) {
            const int64_t l = e * N3 + lp_inode(q, N);
            if (lp_learned(info[l])) {
                xv = lp_f2bf((float)(y[l] * inv * ig));
                tv = (float)(v[l] * inv);
            }
        }
        xr[q] = xv;
        tr[q] = tv;
    }
    for (int c = threadIdx.x; c < kFeat; c += blockDim.x)
        fr[c] = c < 6 ? lp_f2bf(gfeat[e * 8 + c]) : (uint16_t)0;
}

unsigned lp_grid(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    return (unsigned)(b < 1 ? 1 : b);
}

__global__ void lp_scale_kernel(int64_t n, double a, double *__restrict__ x)
{
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (int64_t)gridDim.x * blockDim.x)
        x[l] = a == 0.0 ? 0.0 : a * x[l];
}

__global__ void lp_add_kernel(int64_t n, const double *__restrict__ d, double *__restrict__ x)
{
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (int64_t)gridDim.x * blockDim.x)
        x[l] += d[l];
}

}  // namespace
}  // namespace nbx

using namespace nbx;

struct nbx_lp {
    nbx_problem *P = nullptr;
    nbx_lpi *M = nullptr;
    int N = 0, nI = 0, nIp = 0;
    int64_t E = 0, Epad = 0;
    float *gfeat = nullptr;     // [E][8]
    double *igd = nullptr;      // [E] 1 / gd
    uint16_t *F = nullptr;      // [Epad][64] BF16 features
    float *gam = nullptr;       // [Epad][nIp] gains
    uint16_t *X = nullptr, *Qb = nullptr;   // [Epad][nIp]
    float *Zi = nullptr;        // [Epad][nIp]
    double *part4 = nullptr;
    double *vm = nullptr, *ym = nullptr;    // sampling work vectors (first use)
    hipGraphExec_t gexec = nullptr;
    const double *g_x = nullptr;
    int g_iters = 0, g_tile = 0;
};

namespace nbx {
namespace {

// gamma for every element from the current model
int compute_gains(nbx_lp *L, hipStream_t s)
{
    nbx_mlp *mlp = lpi_mlp(L->M);
    const int mb = lpi_max_batch(L->M);
    for (int64_t r0 = 0; r0 < L->Epad; r0 += mb) {
        const int rows = (int)std::min<int64_t>(mb, L->Epad - r0);
        int st = mlp_forward_rows(mlp, L->F + (size_t)r0 * kFeat, rows,
                                  L->gam + (size_t)r0 * L->nIp, s);
        if (st != NBX_OK) return st;
    }
    const int64_t n = L->Epad * L->nIp;
    hipLaunchKernelGGL(lp_softplus_kernel, dim3(lp_grid(n)), dim3(256), 0, s, n, L->gam);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

// The two GEMMs of an application: Zi = ((X L^T) * gamma) L.
int enqueue_gemms(nbx_lp *L, hipStream_t s)
{
    const int n = L->nIp;
    const uint16_t *Lb = lpi_Lb(L->M);
    for (int64_t r0 = 0; r0 < L->Epad; r0 += kGemmRows) {
        const int rows = (int)std::min<int64_t>(kGemmRows, L->Epad - r0);
        const size_t o = (size_t)r0 * n;
        int st = gemm_bf16(0, 1, kEpiMulBf16, rows, n, n, L->X + o, n, Lb, n, nullptr, 0,
                           L->Qb + o, n, nullptr, nullptr, n, s, L->gam + o);
        if (st != NBX_OK) return st;
        st = gemm_bf16(0, 0, kEpiF32, rows, n, n, L->Qb + o, n, Lb, n, L->Zi + o, n, nullptr, 0,
                       nullptr, nullptr, 0, s, nullptr);
        if (st != NBX_OK) return st;
    }
    return NBX_OK;
}

// Zi = ((X L^T) * gamma) L for X = gather(r); flag may be null
int enqueue_rows(nbx_lp *L, const double *r, const double *flag, hipStream_t s)
{
    nbx_problem *P = L->P;
    const int n = L->nIp;
    hipLaunchKernelGGL(lp_gather_kernel, dim3(lp_grid(L->Epad * n)), dim3(256), 0, s, L->N,
                       L->nI, n, P->E, L->Epad, r, P->gs->plan.info, L->X, flag);
    NBX_LAUNCH_CHECK();
    return enqueue_gemms(L, s);
}

#define LP_FOR_EACH_N(C) C(3) C(4) C(5) C(6) C(7) C(8) C(9) C(10) C(11) C(12) C(13) C(14) C(15) C(16)

// The update step with the gather fused (lp_update_gather_kernel<N>).
int launch_update_gather(nbx_lp *L, double *x, hipStream_t s)
{
    nbx_problem *P = L->P;
    const int nb = sk::red_blocks(P->n);
    switch (L->N) {
#define LP_CASE(NN)                                                                             \
    case NN:                                                                                    \
        hipLaunchKernelGGL(lp_update_gather_kernel<NN>, dim3(nb), dim3(sk::kRedThreads), 0, s,  \
                           P->n, L->nIp, P->p, P->w, P->gs->plan.info, x, P->r, L->X, P->part3, \
                           P->scal);                                                            \
        break;
        LP_FOR_EACH_N(LP_CASE)
#undef LP_CASE
        default: return NBX_EUNSUPPORTED;
    }
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

// z_new, <r, z_new>_c and <z_new, w>_c from the learned rows (lp_dots_n_kernel<N>).
int launch_dots(nbx_lp *L, double *scal, int first, hipStream_t s)
{
    nbx_problem *P = L->P;
    const int nb = sk::red_blocks(P->n);
    switch (L->N) {
#define LP_CASE(NN)                                                                              \
    case NN:                                                                                     \
        hipLaunchKernelGGL(lp_dots_n_kernel<NN>, dim3(nb), dim3(sk::kRedThreads), 0, s, P->n,    \
                           P->r, P->dinv, P->gs->plan.info, L->Zi, L->nIp, L->igd, P->w, first, \
                           P->z, L->part4, scal);                                                \
        break;
        LP_FOR_EACH_N(LP_CASE)
#undef LP_CASE
        default: return NBX_EUNSUPPORTED;
    }
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

// z <- M(r) inside the flexible iteration, with the dots and beta.  With
// gathered != 0, X already holds r's rows (the update step wrote them).
int enqueue_precond(nbx_lp *L, double *scal, int first, int gathered, hipStream_t s)
{
    nbx_problem *P = L->P;
    int st = gathered ? enqueue_gemms(L, s) : enqueue_rows(L, P->r, scal + NBX_S_FLAG, s);
    if (st != NBX_OK) return st;
    st = launch_dots(L, scal, first, s);
    if (st != NBX_OK) return st;
    const int nb = sk::red_blocks(P->n);
    hipLaunchKernelGGL(lp_beta_kernel, dim3(1), dim3(1024), 0, s, nb, L->part4, scal, first);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

int enqueue_flex_iters(nbx_lp *L, double *x, int n_iter, hipStream_t s)
{
    nbx_problem *P = L->P;
    const GsPlan &gs = P->gs->plan;
    const int nb1 = ax_blocks(NBX_F64, P->N, P->E);
    const int nb3 = sk::red_blocks(P->n);
    for (int it = 0; it < n_iter; ++it) {
        int st = ax_pcg_launch_f64(P->G, P->D, P->N, P->E, P->z, P->p, P->w, P->part1, P->scal, s);
        if (st != NBX_OK) return st;
        const PapTask pap{nb1, P->part1, P->scal};   // R1 rides on the exchange launch
        st = dssum_launch<double>(gs, P->w, 1, s, P->scal + NBX_S_FLAG, &pap);
        if (st != NBX_OK) return st;
        st = launch_update_gather(L, x, s);
        if (st != NBX_OK) return st;
        hipLaunchKernelGGL(lp_rr_kernel, dim3(1), dim3(1024), 0, s, nb3, P->part3, P->scal);
        NBX_LAUNCH_CHECK();
        st = enqueue_precond(L, P->scal, 0, 1, s);
        if (st != NBX_OK) return st;
    }
    return NBX_OK;
}

}  // namespace
}  // namespace nbx

extern "C" int nbx_lp_destroy(nbx_lp *L)
{
    if (!L) return NBX_OK;
    if (L->gexec) hipGraphExecDestroy(L->gexec);
    hipFree(L->gfeat); hipFree(L->igd); hipFree(L->F); hipFree(L->gam); hipFree(L->X);
    hipFree(L->Qb); hipFree(L->Zi); hipFree(L->part4); hipFree(L->vm); hipFree(L->ym);
    delete L;
    return NBX_OK;
}

extern "C" int nbx_lp_refresh(nbx_lp *L, void *stream)
{
    if (!L) return NBX_EINVAL;
    hipStream_t s = as_stream(stream);
    int st = compute_gains(L, s);
    if (st != NBX_OK) return st;
    NBX_HIP(hipStreamSynchronize(s));
    return NBX_OK;
}

extern "C" int nbx_lp_create(nbx_problem *P, nbx_lpi *M, nbx_lp **out, void *stream)
{
    if (!out) return NBX_EINVAL;
    *out = nullptr;
    if (!P || !M) return NBX_EINVAL;
    int N, nI, nIp;
    lpi_dims(M, &N, &nI, &nIp);
    if (N != P->N) return NBX_EINVAL;
    nbx_lp *L = new (std::nothrow) nbx_lp;
    if (!L) return NBX_ENOMEM;
    L->P = P; L->M = M; L->N = N; L->nI = nI; L->nIp = nIp;
    L->E = P->E; L->Epad = (P->E + 63) / 64 * 64;
    const size_t Ep = (size_t)L->Epad, rows = Ep * nIp;
    if (hipMalloc(&L->gfeat, (size_t)P->E * 8 * sizeof(float)) != hipSuccess ||
        hipMalloc(&L->igd, (size_t)P->E * sizeof(double)) != hipSuccess ||
        hipMalloc(&L->F, Ep * kFeat * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc(&L->gam, rows * sizeof(float)) != hipSuccess ||
        hipMalloc(&L->X, rows * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc(&L->Qb, rows * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc(&L->Zi, rows * sizeof(float)) != hipSuccess ||
        hipMalloc(&L->part4, 2 * sk::kMaxRedBlocks * sizeof(double)) != hipSuccess) {
        nbx_lp_destroy(L);
        return NBX_ENOMEM;
    }
    hipStream_t s = as_stream(stream);
    // the padding of X (q >= nI, e >= E) stays zero: the fused update step
    // writes only the interior rows
    if (hipMemsetAsync(L->X, 0, rows * sizeof(uint16_t), s) != hipSuccess) {
        nbx_lp_destroy(L);
        return NBX_ENOMEM;
    }
    const int N3 = N * N * N;
    hipLaunchKernelGGL(lp_geom_kernel, dim3((unsigned)P->E), dim3(256), 0, s, N3, P->G, L->gfeat,
                       L->igd);
    hipLaunchKernelGGL(lp_feat_rows_kernel, dim3((unsigned)((Ep * kFeat + 255) / 256)), dim3(256),
                       0, s, P->E, L->Epad, L->gfeat, L->F);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { nbx_lp_destroy(L); return hip_fail(e, "lp_create"); }
    const int st = nbx_lp_refresh(L, stream);
    if (st != NBX_OK) { nbx_lp_destroy(L); return st; }
    *out = L;
    return NBX_OK;
}

extern "C" int nbx_lp_geom_features(nbx_lp *L, float *gfeat, void *stream)
{
    if (!L || !gfeat) return NBX_EINVAL;
    NBX_HIP(hipMemcpyAsync(gfeat, L->gfeat, (size_t)L->E * 8 * sizeof(float),
                           hipMemcpyDeviceToDevice, as_stream(stream)));
    return NBX_OK;
}

extern "C" int nbx_lp_apply(nbx_lp *L, const double *r, double *z, void *stream)
{
    if (!L || !r || !z || r == z) return NBX_EINVAL;
    hipStream_t s = as_stream(stream);
    int st = enqueue_rows(L, r, nullptr, s);
    if (st != NBX_OK) return st;
    nbx_problem *P = L->P;
    hipLaunchKernelGGL(lp_out_kernel, dim3(lp_grid(P->n)), dim3(256), 0, s, L->N, P->n, r,
                       P->dinv, P->gs->plan.info, L->Zi, L->nIp, L->igd, z);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

extern "C" int nbx_lp_samples(nbx_lp *L, const double *v, const double *v0,
                              const int32_t *elems, int nsel, void *X, float *T, void *F,
                              void *stream)
{
    if (!L || !v || !elems || !X || !T || !F || nsel < 0) return NBX_EINVAL;
    if (nsel == 0) return NBX_OK;
    nbx_problem *P = L->P;
    const size_t vb = sizeof(double) * (size_t)P->n;
    if (!L->vm && hipMalloc(&L->vm, vb) != hipSuccess) return NBX_ENOMEM;
    if (!L->ym && hipMalloc(&L->ym, vb) != hipSuccess) return NBX_ENOMEM;
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(lp_mask_kernel, dim3(lp_grid(P->n)), dim3(256), 0, s, L->N, P->n, v, v0,
                       P->gs->plan.info, L->vm);
    NBX_LAUNCH_CHECK();
    int st = ax_launch_f64(L->vm, P->G, P->D, P->N, P->E, L->ym, s);
    if (st != NBX_OK) return st;
    hipLaunchKernelGGL(lp_sample_kernel, dim3(nsel), dim3(256), 0, s, L->N, L->nI, L->nIp, P->E,
                       elems, L->vm, L->ym, P->gs->plan.info, L->gfeat, L->igd, (uint16_t *)X, T,
                       (uint16_t *)F);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

extern "C" int nbx_problem_residual(nbx_problem *P, double *r, void *stream)
{
    if (!P || !r) return NBX_EINVAL;
    NBX_HIP(hipMemcpyAsync(r, P->r, sizeof(double) * (size_t)P->n, hipMemcpyDeviceToDevice,
                           as_stream(stream)));
    return NBX_OK;
}

extern "C" int nbx_pcg_learned(nbx_lp *L, const double *b, double *x, const nbx_pcg_opts *opts,
                               nbx_pcg_result *res, void *stream)
{
    if (!L || !b || !x || !res) return NBX_EINVAL;
    nbx_pcg_opts o;
    if (opts) o = *opts; else nbx_pcg_default_opts(&o);
    if (o.max_iter < 0 || !(o.rtol >= 0)) return NBX_EINVAL;
    *res = nbx_pcg_result{};
    nbx_problem *P = L->P;
    hipStream_t cs = as_stream(stream), s = P->ws;
    NBX_HIP(hipEventRecord(P->ev, cs));
    NBX_HIP(hipStreamWaitEvent(s, P->ev, 0));
    const int chunk = o.check_every > 0 ? o.check_every : 10;
    const int tile = pcg_tile(NBX_F64, L->P->N);
    if (o.use_graph &&
        (L->gexec == nullptr || L->g_x != x || L->g_iters != chunk || L->g_tile != tile)) {
        if (L->gexec) { hipGraphExecDestroy(L->gexec); L->gexec = nullptr; }
        NBX_HIP(hipStreamSynchronize(s));
        NBX_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        int st = enqueue_flex_iters(L, x, chunk, s);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        if (st != NBX_OK) { if (g) hipGraphDestroy(g); return st; }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&L->gexec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) { L->gexec = nullptr; return hip_fail(e, "hipGraphInstantiate"); }
        L->g_x = x; L->g_iters = chunk; L->g_tile = tile;
    }
    NBX_HIP(hipStreamSynchronize(s));
    const auto t0 = std::chrono::steady_clock::now();
    const GsPlan &gs = P->gs->plan;
    const int nb = sk::red_blocks(P->n);
    // x = 0, r = b, p = 0, scalars; then z = M(b), rho = <b, z>, beta = 0
    hipLaunchKernelGGL((sk::init_kernel<double, double>), dim3(nb), dim3(sk::kRedThreads), 0, s,
                       P->n, b, P->dinv, gs.info, x, P->r, P->z, P->p, P->part3);
    hipLaunchKernelGGL(sk::init_reduce_kernel, dim3(1), dim3(1024), 0, s, nb, P->part3, P->scal,
                       o.rtol, o.fixed_iters, o.max_iter);
    NBX_LAUNCH_CHECK();
    int st = enqueue_precond(L, P->scal, 1, 0, s);
    if (st != NBX_OK) return st;
    int done = 0;
    double *h = P->h_scal;
    while (true) {
        if (o.use_graph) {
            NBX_HIP(hipGraphLaunch(L->gexec, s));
        } else {
            st = enqueue_flex_iters(L, x, chunk, s);
            if (st != NBX_OK) return st;
        }
        done += chunk;
        NBX_HIP(hipMemcpyAsync(h, P->scal, sizeof(double) * NBX_SCAL_LEN, hipMemcpyDeviceToHost, s));
        NBX_HIP(hipStreamSynchronize(s));
        if (h[NBX_S_FLAG] != 0.0) break;
        if (done >= o.max_iter + chunk) break;
    }
    res->iters = (int)h[NBX_S_ITER];
    res->outer_iters = res->iters;   // flexible iterations before any fallback
    const double fl = h[NBX_S_FLAG];
    res->flag = fl == 1.0 ? 1 : (fl == 2.0 ? 2 : 0);
    double rb[2];
    st = residual_f64(P, b, x, P->r, rb, s);
    if (st != NBX_OK) return st;
    double relres = rb[1] > 0 ? std::sqrt(rb[0] / rb[1]) : 0.0;
    const int left = o.max_iter - res->iters;
    if (res->flag == 2 && left > 0) {
        // breakdown: Jacobi-PCG on the residual equation from the current x
        // (from x = 0 if the flexible iterate diverged), within the
        // iterations the caller's budget has left
        res->fell_back = 1;
        const bool restart = !(relres < 1.0);
        double *rhs = nullptr, *d = nullptr;
        if (hipMalloc(&rhs, sizeof(double) * (size_t)P->n) != hipSuccess) return NBX_ENOMEM;
        if (hipMalloc(&d, sizeof(double) * (size_t)P->n) != hipSuccess) {
            hipFree(rhs);
            return NBX_ENOMEM;
        }
        NBX_HIP(hipMemcpyAsync(rhs, restart ? b : P->r, sizeof(double) * (size_t)P->n,
                               hipMemcpyDeviceToDevice, s));
        if (restart)
            hipLaunchKernelGGL(lp_scale_kernel, dim3(lp_grid(P->n)), dim3(256), 0, s, P->n, 0.0,
                               x);
        nbx_pcg_opts o64 = o;
        o64.prec = NBX_F64;
        o64.rtol = (relres > 0 && !restart) ? o.rtol / relres : o.rtol;
        o64.max_iter = left;
        nbx_pcg_result r64{};
        st = pcg_f64(P, rhs, d, o64, &r64);
        if (st == NBX_OK) {
            hipLaunchKernelGGL(lp_add_kernel, dim3(lp_grid(P->n)), dim3(256), 0, s, P->n, d, x);
            st = residual_f64(P, b, x, P->r, rb, s);
        }
        NBX_HIP(hipStreamSynchronize(s));
        hipFree(rhs);
        hipFree(d);
        if (st != NBX_OK) return st;
        res->iters += r64.iters;
        relres = rb[1] > 0 ? std::sqrt(rb[0] / rb[1]) : 0.0;
        res->flag = (relres <= o.rtol || r64.flag == 1) ? 1 : (r64.flag == 2 ? 2 : 0);
    }
    res->relres = relres;
    res->true_relres = relres;
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    NBX_HIP(hipEventRecord(P->ev, s));
    NBX_HIP(hipStreamWaitEvent(cs, P->ev, 0));
    if (res->flag == 2) return NBX_EBREAKDOWN;
    return res->flag == 1 ? NBX_OK : NBX_NOT_CONVERGED;
}
