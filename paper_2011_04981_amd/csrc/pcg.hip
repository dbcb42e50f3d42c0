// pcg.hip -- Jacobi-preconditioned conjugate gradients on the device
// (Section II-B: each CG iteration is vector operations, AX, the
// nearest-neighbour exchange and global reductions, with a simple
// preconditioner, read here as Jacobi).
//
// One iteration is five kernels, all scalars staying on the device:
//   K1  p = z + beta p, w = AX(p), per-element partials of p.w   (ax.hip)
//   R1  pap = sum of partials (fixed order), alpha = rho / pap
//   K2  w = mask(dssum(w))                                        (gs.hip)
//   K3  x += alpha p, r -= alpha w, z = dinv r, partials of c r r and c r z
//   R3  rr, rho' (fixed order), convergence / breakdown flag, beta
// <p,w>_c is taken before the exchange: p is continuous and zero on the
// Dirichlet set, so sum_l c_l p_l (dssum w)_l = sum_l p_l w_l.
// Every reduction is two-stage in a fixed order, so reruns are bitwise
// identical.  The host only launches (optionally a captured hipGraph of
// several iterations) and reads the flag between launches.
#include "internal.hpp"

#include <chrono>
#include <cmath>

namespace nbx {

int jacobi_setup_impl(const double *G, const double *D, int N, int64_t E, const GsPlan &gs,
                      double *dinv, hipStream_t s);

namespace {

constexpr int kRedThreads = 256;
constexpr int kMaxRedBlocks = 4096;
constexpr double kFlagLimit = 3.0;

__device__ inline double wsum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Two sums over a 256-thread block, fixed order; valid in thread 0.
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

__device__ inline double cw(uint8_t info) { return 1.0 / (double)(info & 0x7f); }

// x = 0, r = b, z = dinv b, p = 0; partials of c b b and c b z.
__global__ void __launch_bounds__(kRedThreads)
init_kernel(int64_t n, const double *__restrict__ b, const double *__restrict__ dinv,
            const uint8_t *__restrict__ info, double *__restrict__ x, double *__restrict__ r,
            double *__restrict__ z, double *__restrict__ p, double *__restrict__ part)
{
    double bb = 0, bz = 0;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (int64_t)gridDim.x * blockDim.x) {
        const double bv = b[l], zv = dinv[l] * bv, c = cw(info[l]);
        x[l] = 0.0; r[l] = bv; z[l] = zv; p[l] = 0.0;
        bb += c * bv * bv; bz += c * bv * zv;
    }
    block_sum2(bb, bz);
    if (threadIdx.x == 0) { part[2 * blockIdx.x] = bb; part[2 * blockIdx.x + 1] = bz; }
}

__global__ void __launch_bounds__(1024)
init_reduce_kernel(int nb, const double *__restrict__ part, double *__restrict__ scal,
                   double rtol, int fixed, int max_iter)
{
    __shared__ double s[2][16];
    double a = 0, b = 0;
    for (int q = threadIdx.x; q < nb; q += blockDim.x) { a += part[2 * q]; b += part[2 * q + 1]; }
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

// R1: pap from K1's per-element partials; alpha; breakdown check.
__global__ void __launch_bounds__(1024)
pap_reduce_kernel(int nb, const double *__restrict__ part, double *__restrict__ scal)
{
    if (scal[NBX_S_FLAG] != 0.0) return;
    __shared__ double s[16];
    double a = 0;
    for (int q = threadIdx.x; q < nb; q += blockDim.x) a += part[q];
    a = wsum(a);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double pap = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) pap += s[q];
        scal[NBX_S_PAP] = pap;
        if (!(pap > 0.0) || !isfinite(pap)) {
            scal[NBX_S_FLAG] = 2.0;
        } else {
            scal[NBX_S_ALPHA] = scal[NBX_S_RHO] / pap;
        }
    }
}

// K3: x += alpha p; r -= alpha w; z = dinv r; partials of c r r, c r z.
__global__ void __launch_bounds__(kRedThreads)
update_kernel(int64_t n, const double *__restrict__ p, const double *__restrict__ w,
              const double *__restrict__ dinv, const uint8_t *__restrict__ info,
              double *__restrict__ x, double *__restrict__ r, double *__restrict__ z,
              double *__restrict__ part, const double *__restrict__ scal)
{
    if (scal[NBX_S_FLAG] != 0.0) return;
    const double alpha = scal[NBX_S_ALPHA];
    double rr = 0, rz = 0;
    // two nodes per thread per step (16-byte accesses), then a scalar tail
    const int64_t n2 = n >> 1;
    const double2 *p2 = reinterpret_cast<const double2 *>(p);
    const double2 *w2 = reinterpret_cast<const double2 *>(w);
    const double2 *d2 = reinterpret_cast<const double2 *>(dinv);
    double2 *x2 = reinterpret_cast<double2 *>(x);
    double2 *r2 = reinterpret_cast<double2 *>(r);
    double2 *z2 = reinterpret_cast<double2 *>(z);
    const uint16_t *i2 = reinterpret_cast<const uint16_t *>(info);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n2;
         q += (int64_t)gridDim.x * blockDim.x) {
        const double2 pv = p2[q], wv = w2[q], dv = d2[q];
        double2 xv = x2[q], rv = r2[q];
        const uint16_t iv = i2[q];
        xv.x += alpha * pv.x; xv.y += alpha * pv.y;
        rv.x -= alpha * wv.x; rv.y -= alpha * wv.y;
        const double2 zv = make_double2(dv.x * rv.x, dv.y * rv.y);
        x2[q] = xv; r2[q] = rv; z2[q] = zv;
        const double c0 = cw((uint8_t)(iv & 0xff)), c1 = cw((uint8_t)(iv >> 8));
        rr += c0 * rv.x * rv.x + c1 * rv.y * rv.y;
        rz += c0 * rv.x * zv.x + c1 * rv.y * zv.y;
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const int64_t l = n - 1;
        x[l] += alpha * p[l];
        const double rv = r[l] - alpha * w[l], zv = dinv[l] * rv, c = cw(info[l]);
        r[l] = rv; z[l] = zv;
        rr += c * rv * rv; rz += c * rv * zv;
    }
    block_sum2(rr, rz);
    if (threadIdx.x == 0) { part[2 * blockIdx.x] = rr; part[2 * blockIdx.x + 1] = rz; }
}

// R3: rr, rho'; convergence / breakdown / iteration limit; beta.
__global__ void __launch_bounds__(1024)
rr_reduce_kernel(int nb, const double *__restrict__ part, double *__restrict__ scal)
{
    if (scal[NBX_S_FLAG] != 0.0) return;
    __shared__ double s[2][16];
    double a = 0, b = 0;
    for (int q = threadIdx.x; q < nb; q += blockDim.x) { a += part[2 * q]; b += part[2 * q + 1]; }
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
    }
}

// partials of c (b - w)^2 (true residual) and c b b.
__global__ void __launch_bounds__(kRedThreads)
resid_kernel(int64_t n, const double *__restrict__ b, const double *__restrict__ w,
             const uint8_t *__restrict__ info, double *__restrict__ part)
{
    double a = 0, c2 = 0;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (int64_t)gridDim.x * blockDim.x) {
        const double c = cw(info[l]), d = b[l] - w[l];
        a += c * d * d; c2 += c * b[l] * b[l];
    }
    block_sum2(a, c2);
    if (threadIdx.x == 0) { part[2 * blockIdx.x] = a; part[2 * blockIdx.x + 1] = c2; }
}

__global__ void __launch_bounds__(1024)
sum2_kernel(int nb, const double *__restrict__ part, double *__restrict__ out)
{
    __shared__ double s[2][16];
    double a = 0, b = 0;
    for (int q = threadIdx.x; q < nb; q += blockDim.x) { a += part[2 * q]; b += part[2 * q + 1]; }
    a = wsum(a); b = wsum(b);
    if ((threadIdx.x & 63) == 0) { s[0][threadIdx.x >> 6] = a; s[1][threadIdx.x >> 6] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0, y = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) { x += s[0][q]; y += s[1][q]; }
        out[0] = x; out[1] = y;
    }
}

inline int red_blocks(int64_t n)
{
    int64_t b = (n + 2 * kRedThreads - 1) / (2 * kRedThreads);
    if (b > kMaxRedBlocks) b = kMaxRedBlocks;
    return (int)(b < 1 ? 1 : b);
}

}  // namespace
}  // namespace nbx

using namespace nbx;

struct nbx_problem {
    const double *G = nullptr, *D = nullptr;
    int N = 0;
    int64_t E = 0, n = 0;
    nbx_gs *gs = nullptr;
    double *dinv = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *w = nullptr;
    double *part1 = nullptr, *part3 = nullptr, *scal = nullptr, *tmp2 = nullptr;
    double *h_scal = nullptr;   // pinned host mirror of scal
    int nb3 = 1;
    hipStream_t ws = nullptr;
    hipEvent_t ev = nullptr;
    hipGraphExec_t gexec = nullptr;
    const double *g_x = nullptr;
    int g_iters = 0;
};

namespace nbx {

// Enqueues n_iter fused iterations on s.
static int enqueue_iters(nbx_problem *P, double *x, double *r, double *z, double *p,
                         double *scal, int n_iter, hipStream_t s)
{
    const GsPlan &gs = P->gs->plan;
    for (int it = 0; it < n_iter; ++it) {
        int st = ax_pcg_launch_f64(P->G, P->D, P->N, P->E, z, p, P->w, P->part1, scal, s);
        if (st != NBX_OK) return st;
        hipLaunchKernelGGL(pap_reduce_kernel, dim3(1), dim3(1024), 0, s,
                           ax_blocks(NBX_F64, P->N, P->E), P->part1, scal);
        st = dssum_launch<double>(gs, P->w, 1, s, scal + NBX_S_FLAG);
        if (st != NBX_OK) return st;
        hipLaunchKernelGGL(update_kernel, dim3(P->nb3), dim3(kRedThreads), 0, s, P->n, p, P->w,
                           P->dinv, gs.info, x, r, z, P->part3, scal);
        hipLaunchKernelGGL(rr_reduce_kernel, dim3(1), dim3(1024), 0, s, P->nb3, P->part3, scal);
        NBX_LAUNCH_CHECK();
    }
    return NBX_OK;
}

}  // namespace nbx

extern "C" int nbx_problem_create(const double *G, const double *D, int N, int64_t E,
                                  nbx_gs *gs, nbx_problem **out, void *stream)
{
    if (!out) return NBX_EINVAL;
    *out = nullptr;
    if (!G || !D || !gs || N < 2 || N > kMaxN || E < 1) return NBX_EINVAL;
    if (E > 0x7fffffffLL) return NBX_EUNSUPPORTED;
    const int64_t n = E * (int64_t)N * N * N;
    if (gs->plan.n_local != n) return NBX_EINVAL;
    nbx_problem *P = new (std::nothrow) nbx_problem;
    if (!P) return NBX_ENOMEM;
    P->G = G; P->D = D; P->N = N; P->E = E; P->n = n; P->gs = gs;
    P->nb3 = red_blocks(n);
    auto fail = [&](int st) { nbx_problem_destroy(P); return st; };
    const size_t vb = sizeof(double) * (size_t)n;
    if (hipMalloc(&P->dinv, vb) != hipSuccess || hipMalloc(&P->r, vb) != hipSuccess ||
        hipMalloc(&P->z, vb) != hipSuccess || hipMalloc(&P->p, vb) != hipSuccess ||
        hipMalloc(&P->w, vb) != hipSuccess ||
        hipMalloc(&P->part1, sizeof(double) * (size_t)E) != hipSuccess ||
        hipMalloc(&P->part3, sizeof(double) * 2 * kMaxRedBlocks) != hipSuccess ||
        hipMalloc(&P->scal, sizeof(double) * NBX_SCAL_LEN) != hipSuccess ||
        hipMalloc(&P->tmp2, sizeof(double) * 2) != hipSuccess)
        return fail(NBX_ENOMEM);
    if (hipHostMalloc(&P->h_scal, sizeof(double) * NBX_SCAL_LEN, hipHostMallocDefault) !=
        hipSuccess)
        return fail(NBX_ENOMEM);
    hipError_t e = hipStreamCreateWithFlags(&P->ws, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(hip_fail(e, "hipStreamCreate"));
    e = hipEventCreateWithFlags(&P->ev, hipEventDisableTiming);
    if (e != hipSuccess) return fail(hip_fail(e, "hipEventCreate"));
    hipStream_t s = as_stream(stream);
    int st = jacobi_setup_impl(G, D, N, E, gs->plan, P->dinv, s);
    if (st != NBX_OK) return fail(st);
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(hip_fail(e, "hipStreamSynchronize"));
    *out = P;
    return NBX_OK;
}

extern "C" int nbx_problem_destroy(nbx_problem *P)
{
    if (!P) return NBX_OK;
    if (P->ws) hipStreamSynchronize(P->ws);
    if (P->gexec) hipGraphExecDestroy(P->gexec);
    hipFree(P->dinv); hipFree(P->r); hipFree(P->z); hipFree(P->p); hipFree(P->w);
    hipFree(P->part1); hipFree(P->part3); hipFree(P->scal); hipFree(P->tmp2);
    if (P->h_scal) hipHostFree(P->h_scal);
    if (P->ev) hipEventDestroy(P->ev);
    if (P->ws) hipStreamDestroy(P->ws);
    delete P;
    return NBX_OK;
}

extern "C" int nbx_problem_dinv(nbx_problem *P, double *out, void *stream)
{
    if (!P || !out) return NBX_EINVAL;
    NBX_HIP(hipMemcpyAsync(out, P->dinv, sizeof(double) * (size_t)P->n,
                           hipMemcpyDeviceToDevice, as_stream(stream)));
    return NBX_OK;
}

extern "C" int nbx_pcg_iterate(nbx_problem *P, double *x, double *r, double *z, double *pdir,
                               double *scal, int n_iter, void *stream)
{
    if (!P || !x || !r || !z || !pdir || !scal || n_iter < 0) return NBX_EINVAL;
    return enqueue_iters(P, x, r, z, pdir, scal, n_iter, as_stream(stream));
}

extern "C" void nbx_pcg_default_opts(nbx_pcg_opts *o)
{
    if (!o) return;
    o->max_iter = 1000;
    o->fixed_iters = 0;
    o->check_every = 10;
    o->use_graph = 1;
    o->rtol = 1e-10;
    o->prec = NBX_F64;
    o->inner_rtol = 1e-5;
    o->max_outer = 20;
}

namespace nbx {

// FP64 true residual ||b - mask(dssum(AX(x)))||_c / ||b||_c, synchronous on s.
int true_relres(nbx_problem *P, const double *b, const double *x, double *out, hipStream_t s)
{
    int st = ax_launch_f64(x, P->G, P->D, P->N, P->E, P->w, s);
    if (st != NBX_OK) return st;
    st = dssum_launch<double>(P->gs->plan, P->w, 1, s);
    if (st != NBX_OK) return st;
    const int nb = red_blocks(P->n);
    hipLaunchKernelGGL(resid_kernel, dim3(nb), dim3(kRedThreads), 0, s, P->n, b, P->w,
                       P->gs->plan.info, P->part3);
    hipLaunchKernelGGL(sum2_kernel, dim3(1), dim3(1024), 0, s, nb, P->part3, P->tmp2);
    NBX_LAUNCH_CHECK();
    double h[2];
    NBX_HIP(hipMemcpyAsync(h, P->tmp2, sizeof(h), hipMemcpyDeviceToHost, s));
    NBX_HIP(hipStreamSynchronize(s));
    *out = h[1] > 0 ? std::sqrt(h[0] / h[1]) : 0.0;
    return NBX_OK;
}

// Plain FP64 Jacobi-PCG from x = 0 on the problem's own stream.
int pcg_f64(nbx_problem *P, const double *b, double *x, const nbx_pcg_opts &o,
            nbx_pcg_result *res)
{
    hipStream_t s = P->ws;
    const GsPlan &gs = P->gs->plan;
    const int nb = red_blocks(P->n);
    hipLaunchKernelGGL(init_kernel, dim3(nb), dim3(kRedThreads), 0, s, P->n, b, P->dinv,
                       gs.info, x, P->r, P->z, P->p, P->part3);
    hipLaunchKernelGGL(init_reduce_kernel, dim3(1), dim3(1024), 0, s, nb, P->part3, P->scal,
                       o.rtol, o.fixed_iters, o.max_iter);
    NBX_LAUNCH_CHECK();
    const int chunk = o.check_every > 0 ? o.check_every : 10;
    if (o.use_graph && (P->gexec == nullptr || P->g_x != x || P->g_iters != chunk)) {
        if (P->gexec) { hipGraphExecDestroy(P->gexec); P->gexec = nullptr; }
        NBX_HIP(hipStreamSynchronize(s));
        NBX_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        int st = enqueue_iters(P, x, P->r, P->z, P->p, P->scal, chunk, s);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        if (st != NBX_OK) { if (g) hipGraphDestroy(g); return st; }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) { P->gexec = nullptr; return hip_fail(e, "hipGraphInstantiate"); }
        P->g_x = x; P->g_iters = chunk;
    }
    NBX_HIP(hipStreamSynchronize(s));
    const auto t0 = std::chrono::steady_clock::now();
    int done = 0;
    while (true) {
        if (o.use_graph) {
            NBX_HIP(hipGraphLaunch(P->gexec, s));
        } else {
            int st = enqueue_iters(P, x, P->r, P->z, P->p, P->scal, chunk, s);
            if (st != NBX_OK) return st;
        }
        done += chunk;
        NBX_HIP(hipMemcpyAsync(P->h_scal, P->scal, sizeof(double) * NBX_SCAL_LEN,
                               hipMemcpyDeviceToHost, s));
        NBX_HIP(hipStreamSynchronize(s));
        if (P->h_scal[NBX_S_FLAG] != 0.0) break;
        if (done >= o.max_iter + chunk) break;   // defensive; the device limit stops first
    }
    const auto t1 = std::chrono::steady_clock::now();
    res->seconds = std::chrono::duration<double>(t1 - t0).count();
    res->iters = (int)P->h_scal[NBX_S_ITER];
    res->outer_iters = 1;
    const double bb = P->h_scal[NBX_S_BB];
    res->relres = bb > 0 ? std::sqrt(P->h_scal[NBX_S_RR] / bb) : 0.0;
    const double fl = P->h_scal[NBX_S_FLAG];
    res->flag = fl == 1.0 ? 1 : (fl == 2.0 ? 2 : 0);
    res->fell_back = 0;
    return true_relres(P, b, x, &res->true_relres, s);
}

int pcg_mixed(nbx_problem *P, const double *b, double *x, const nbx_pcg_opts &o,
              nbx_pcg_result *res);

}  // namespace nbx

extern "C" int nbx_pcg(nbx_problem *P, const double *b, double *x, const nbx_pcg_opts *opts,
                       nbx_pcg_result *res, void *stream)
{
    if (!P || !b || !x || !res) return NBX_EINVAL;
    nbx_pcg_opts o;
    if (opts) o = *opts; else nbx_pcg_default_opts(&o);
    if (o.max_iter < 0 || !(o.rtol >= 0)) return NBX_EINVAL;
    *res = nbx_pcg_result{};
    hipStream_t cs = as_stream(stream);
    // order the solve after the caller's pending work on its stream
    NBX_HIP(hipEventRecord(P->ev, cs));
    NBX_HIP(hipStreamWaitEvent(P->ws, P->ev, 0));
    int st;
    if (o.prec == NBX_F64) st = pcg_f64(P, b, x, o, res);
    else if (o.prec == NBX_F32) st = pcg_mixed(P, b, x, o, res);
    else return NBX_EUNSUPPORTED;
    if (st != NBX_OK) return st;
    NBX_HIP(hipEventRecord(P->ev, P->ws));
    NBX_HIP(hipStreamWaitEvent(cs, P->ev, 0));
    if (res->flag == 2) return NBX_EBREAKDOWN;
    return res->flag == 1 ? NBX_OK : NBX_NOT_CONVERGED;
}
