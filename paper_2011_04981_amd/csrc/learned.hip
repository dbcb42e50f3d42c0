// learned.hip -- an element-local learned preconditioner for the CG solve
// and the flexible CG that uses it.
//
// The paper's CG uses a "simple preconditioner" (Section II-B); this adds a
// learned correction on top of Jacobi:
//   M(r) = dinv r + mask(dssum(c * s_e * f(x_e)))
// where, per element, x_e = [r_e / ||r_e||, the six element-mean geometric
// factors / gd_e] (BF16), s_e = ||r_e|| / gd_e, gd_e the element mean of the
// diagonal factors, and f the 3-layer network of mlp.hip (BF16 matrix-core
// products, FP32 accumulation).  c = 1/multiplicity averages the element
// outputs at shared nodes.  A network that outputs zero gives Jacobi back.
// M is nonlinear, so the outer iteration is flexible PCG (Notay 2000, one
// stored direction: beta = -<z_new, A p> / <p, A p> makes each new direction
// A-orthogonal to the previous one).  Training pairs come from
// the FP64 solver: T_e = (e_e - dinv r_e) / s_e with e = x* - x_k.
#include "solver.hpp"
#include "solver_kernels.hpp"

#include <chrono>
#include <cmath>
#include <new>

struct nbx_mlp;

namespace nbx {

int mlp_forward_rows(nbx_mlp *P, const uint16_t *X, int B, float *Y, hipStream_t s);
int mlp_dims(nbx_mlp *P, int *n_in, int *n_out, int *in_pad, int *out_pad, int *max_batch);

namespace {

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

// gfeat[e][0..5] = element means of the six factors / gd, gfeat[e][6] = gd.
__global__ void __launch_bounds__(256)
lp_geom_kernel(int N3, const double *__restrict__ G, float *__restrict__ gfeat)
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
}

// One block per padded row: X[e] = [bf16(r_e/||r_e||), gfeat[e][0..5], 0...],
// scale[e] = ||r_e|| / gd_e; rows e >= E are zero.
__global__ void __launch_bounds__(256)
lp_feat_kernel(int N3, int in_pad, int64_t E, const double *__restrict__ r,
               const float *__restrict__ gfeat, uint16_t *__restrict__ X,
               float *__restrict__ scale, const double *__restrict__ flag)
{
    if (flag && *flag != 0.0) return;
    __shared__ double s[4];
    const int64_t e = blockIdx.x;
    uint16_t *xr = X + (size_t)e * in_pad;
    if (e >= E) {
        for (int q = threadIdx.x; q < in_pad; q += blockDim.x) xr[q] = 0;
        if (threadIdx.x == 0) scale[e] = 0.f;
        return;
    }
    const double *re = r + (size_t)e * N3;
    double a = 0.0;
    for (int q = threadIdx.x; q < N3; q += blockDim.x) a += re[q] * re[q];
    const double nrm = sqrt(lp_block_sum(a, s));
    const double inv = nrm > 0 ? 1.0 / nrm : 0.0;
    for (int q = threadIdx.x; q < in_pad; q += blockDim.x) {
        float v = 0.f;
        if (q < N3) v = (float)(re[q] * inv);
        else if (q < N3 + 6) v = gfeat[e * 8 + (q - N3)];
        xr[q] = lp_f2bf(v);
    }
    if (threadIdx.x == 0) scale[e] = (float)(nrm / gfeat[e * 8 + 6]);
}

// zl[l] = c_l * scale[e] * Y[e][node]
__global__ void lp_combine_kernel(int N3, int out_pad, int64_t n, const float *__restrict__ Y,
                                  const float *__restrict__ scale,
                                  const uint8_t *__restrict__ info, double *__restrict__ zl,
                                  const double *__restrict__ flag)
{
    if (flag && *flag != 0.0) return;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = l / N3;
        const int q = (int)(l - e * N3);
        zl[l] = sk::cw(info[l]) * (double)scale[e] * (double)Y[(size_t)e * out_pad + q];
    }
}

// z_new = dinv r + zl; partials of <r, z_new>_c and <z_new, w>_c (w = A p
// of the step just taken; not read on the first application); z = z_new.
__global__ void __launch_bounds__(sk::kRedThreads)
lp_dots_kernel(int64_t n, const double *__restrict__ r, const double *__restrict__ dinv,
               const double *__restrict__ zl, const uint8_t *__restrict__ info,
               const double *__restrict__ w, int first, double *__restrict__ z,
               double *__restrict__ part, const double *__restrict__ scal)
{
    if (scal[NBX_S_FLAG] != 0.0) return;
    double a = 0, b = 0;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (int64_t)gridDim.x * blockDim.x) {
        const double c = sk::cw(info[l]), rl = r[l];
        const double zn = dinv[l] * rl + zl[l];
        a += c * rl * zn;
        if (!first) b += c * zn * w[l];
        z[l] = zn;
    }
    sk::block_sum2(a, b);
    if (threadIdx.x == 0) { part[2 * blockIdx.x] = a; part[2 * blockIdx.x + 1] = b; }
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

// x += alpha p; r -= alpha w; partials of c r r (and 1 in the second slot).
__global__ void __launch_bounds__(sk::kRedThreads)
lp_update_kernel(int64_t n, const double *__restrict__ p, const double *__restrict__ w,
                 const uint8_t *__restrict__ info, double *__restrict__ x,
                 double *__restrict__ r, double *__restrict__ part,
                 const double *__restrict__ scal)
{
    if (scal[NBX_S_FLAG] != 0.0) return;
    const double alpha = scal[NBX_S_ALPHA];
    double rr = 0, one = 0;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (int64_t)gridDim.x * blockDim.x) {
        x[l] = __builtin_fma(alpha, p[l], x[l]);
        const double rl = __builtin_fma(-alpha, w[l], r[l]);
        r[l] = rl;
        rr += sk::cw(info[l]) * rl * rl;
    }
    sk::block_sum2(rr, one);
    if (threadIdx.x == 0) { part[2 * blockIdx.x] = rr; part[2 * blockIdx.x + 1] = one; }
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

// z = dinv r + zl (plain application, no dots)
__global__ void lp_out_kernel(int64_t n, const double *__restrict__ r,
                              const double *__restrict__ dinv, const double *__restrict__ zl,
                              double *__restrict__ z)
{
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (int64_t)gridDim.x * blockDim.x)
        z[l] = dinv[l] * r[l] + zl[l];
}

// Training rows for selected elements: X as in lp_feat_kernel, T[j] =
// (e_j - dinv_j r_j) / s_e for the element's nodes (e = xs - x), 0 beyond.
__global__ void __launch_bounds__(256)
lp_sample_kernel(int N3, int in_pad, int out_pad, int64_t E, const int32_t *__restrict__ elems,
                 const double *__restrict__ r, const double *__restrict__ xs,
                 const double *__restrict__ x, const double *__restrict__ dinv,
                 const float *__restrict__ gfeat, uint16_t *__restrict__ X, float *__restrict__ T)
{
    __shared__ double s[4];
    const int row = blockIdx.x;
    const int64_t e = elems[row];
    uint16_t *xr = X + (size_t)row * in_pad;
    float *tr = T + (size_t)row * out_pad;
    if (e < 0 || e >= E) {  /* out-of-range index: an all-zero row */
        for (int q = threadIdx.x; q < in_pad; q += blockDim.x) xr[q] = 0;
        for (int q = threadIdx.x; q < out_pad; q += blockDim.x) tr[q] = 0.f;
        return;
    }
    const size_t base = (size_t)e * N3;
    double a = 0.0;
    for (int q = threadIdx.x; q < N3; q += blockDim.x) a += r[base + q] * r[base + q];
    const double nrm = sqrt(lp_block_sum(a, s));
    const double inv = nrm > 0 ? 1.0 / nrm : 0.0;
    const double sc = nrm / gfeat[e * 8 + 6];
    const double isc = sc > 0 ? 1.0 / sc : 0.0;
    for (int q = threadIdx.x; q < in_pad; q += blockDim.x) {
        float v = 0.f;
        if (q < N3) v = (float)(r[base + q] * inv);
        else if (q < N3 + 6) v = gfeat[e * 8 + (q - N3)];
        xr[q] = lp_f2bf(v);
    }
    for (int q = threadIdx.x; q < out_pad; q += blockDim.x) {
        double t = 0.0;
        if (q < N3) t = ((xs[base + q] - x[base + q]) - dinv[base + q] * r[base + q]) * isc;
        tr[q] = (float)t;
    }
}

unsigned lp_grid(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace
}  // namespace nbx

using namespace nbx;

struct nbx_lp {
    nbx_problem *P = nullptr;
    nbx_mlp *mlp = nullptr;
    int N3 = 0, in_pad = 0, out_pad = 0, max_batch = 0;
    int64_t E = 0, Epad = 0;
    float *gfeat = nullptr, *Y = nullptr, *scale = nullptr;
    uint16_t *X = nullptr;
    double *zl = nullptr, *part4 = nullptr;
    hipGraphExec_t gexec = nullptr;
    const double *g_x = nullptr;
    int g_iters = 0, g_tile = 0;
};

namespace nbx {
namespace {

// zl = mask(dssum(c * s * f(features(r)))) ; flag may be null
int enqueue_correction(nbx_lp *L, const double *r, const double *flag, hipStream_t s)
{
    nbx_problem *P = L->P;
    hipLaunchKernelGGL(lp_feat_kernel, dim3((unsigned)L->Epad), dim3(256), 0, s, L->N3,
                       L->in_pad, P->E, r, L->gfeat, L->X, L->scale, flag);
    NBX_LAUNCH_CHECK();
    for (int64_t r0 = 0; r0 < L->Epad; r0 += L->max_batch) {
        const int rows = (int)std::min<int64_t>(L->max_batch, L->Epad - r0);
        int st = mlp_forward_rows(L->mlp, L->X + (size_t)r0 * L->in_pad, rows,
                                  L->Y + (size_t)r0 * L->out_pad, s);
        if (st != NBX_OK) return st;
    }
    hipLaunchKernelGGL(lp_combine_kernel, dim3(lp_grid(P->n)), dim3(256), 0, s, L->N3,
                       L->out_pad, P->n, L->Y, L->scale, P->gs->plan.info, L->zl, flag);
    NBX_LAUNCH_CHECK();
    return dssum_launch<double>(P->gs->plan, L->zl, 1, s, flag);
}

// z <- M(r) inside the flexible iteration, with the dots and beta.
int enqueue_precond(nbx_lp *L, double *scal, int first, hipStream_t s)
{
    nbx_problem *P = L->P;
    int st = enqueue_correction(L, P->r, scal + NBX_S_FLAG, s);
    if (st != NBX_OK) return st;
    const int nb = sk::red_blocks(P->n);
    hipLaunchKernelGGL(lp_dots_kernel, dim3(nb), dim3(sk::kRedThreads), 0, s, P->n, P->r,
                       P->dinv, L->zl, P->gs->plan.info, P->w, first, P->z, L->part4, scal);
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
        hipLaunchKernelGGL(sk::pap_reduce_kernel, dim3(1), dim3(1024), 0, s, nb1, P->part1,
                           P->scal);
        st = dssum_launch<double>(gs, P->w, 1, s, P->scal + NBX_S_FLAG);
        if (st != NBX_OK) return st;
        hipLaunchKernelGGL(lp_update_kernel, dim3(nb3), dim3(sk::kRedThreads), 0, s, P->n, P->p,
                           P->w, gs.info, x, P->r, P->part3, P->scal);
        hipLaunchKernelGGL(lp_rr_kernel, dim3(1), dim3(1024), 0, s, nb3, P->part3, P->scal);
        NBX_LAUNCH_CHECK();
        st = enqueue_precond(L, P->scal, 0, s);
        if (st != NBX_OK) return st;
    }
    return NBX_OK;
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

extern "C" int nbx_lp_create(nbx_problem *P, nbx_mlp *mlp, nbx_lp **out, void *stream)
{
    if (!out) return NBX_EINVAL;
    *out = nullptr;
    if (!P || !mlp) return NBX_EINVAL;
    int n_in, n_out, in_pad, out_pad, max_batch;
    mlp_dims(mlp, &n_in, &n_out, &in_pad, &out_pad, &max_batch);
    const int N3 = P->N * P->N * P->N;
    if (n_in != N3 + 6 || n_out != N3) return NBX_EINVAL;
    nbx_lp *L = new (std::nothrow) nbx_lp;
    if (!L) return NBX_ENOMEM;
    L->P = P; L->mlp = mlp; L->N3 = N3; L->in_pad = in_pad; L->out_pad = out_pad;
    L->max_batch = max_batch; L->E = P->E; L->Epad = (P->E + 63) / 64 * 64;
    const size_t Ep = (size_t)L->Epad;
    if (hipMalloc(&L->gfeat, (size_t)P->E * 8 * sizeof(float)) != hipSuccess ||
        hipMalloc(&L->X, Ep * in_pad * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc(&L->Y, Ep * out_pad * sizeof(float)) != hipSuccess ||
        hipMalloc(&L->scale, Ep * sizeof(float)) != hipSuccess ||
        hipMalloc(&L->zl, (size_t)P->n * sizeof(double)) != hipSuccess ||
        hipMalloc(&L->part4, 2 * sk::kMaxRedBlocks * sizeof(double)) != hipSuccess) {
        nbx_lp_destroy(L);
        return NBX_ENOMEM;
    }
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(lp_geom_kernel, dim3((unsigned)P->E), dim3(256), 0, s, N3, P->G, L->gfeat);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { nbx_lp_destroy(L); return hip_fail(e, "lp_create"); }
    *out = L;
    return NBX_OK;
}

extern "C" int nbx_lp_destroy(nbx_lp *L)
{
    if (!L) return NBX_OK;
    if (L->gexec) hipGraphExecDestroy(L->gexec);
    hipFree(L->gfeat); hipFree(L->X); hipFree(L->Y); hipFree(L->scale); hipFree(L->zl);
    hipFree(L->part4);
    delete L;
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
    int st = enqueue_correction(L, r, nullptr, s);
    if (st != NBX_OK) return st;
    hipLaunchKernelGGL(lp_out_kernel, dim3(lp_grid(L->P->n)), dim3(256), 0, s, L->P->n, r,
                       L->P->dinv, L->zl, z);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

extern "C" int nbx_lp_samples(nbx_lp *L, const double *r, const double *xstar, const double *x,
                              const int32_t *elems, int nsel, void *X, float *T, void *stream)
{
    if (!L || !r || !xstar || !x || !elems || !X || !T || nsel < 0) return NBX_EINVAL;
    if (nsel == 0) return NBX_OK;
    hipLaunchKernelGGL(lp_sample_kernel, dim3(nsel), dim3(256), 0, as_stream(stream), L->N3,
                       L->in_pad, L->out_pad, L->P->E, elems, r, xstar, x, L->P->dinv, L->gfeat,
                       (uint16_t *)X, T);
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
    int st = enqueue_precond(L, P->scal, 1, s);
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
    if (res->flag != 1 && relres > o.rtol) {
        // fallback: Jacobi-PCG on the residual equation from the current x,
        // or on A x = b from x = 0 when the flexible iteration diverged
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
        o64.max_iter = std::max(2 * o.max_iter, 1000);
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
