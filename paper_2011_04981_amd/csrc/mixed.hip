// mixed.hip -- FP32 inner Jacobi-PCG inside FP64 iterative refinement.
//
// The paper keeps every real in double and names reduced precision (single,
// half, fixed point) as further work (Section V).  This driver takes that
// step for the solve: the outer loop is classical iterative refinement
// (residual and correction in FP64), the inner loop is the same fused PCG
// iteration as pcg.hip but on FP32 vectors and FP32 geometric factors
// (half the HBM bytes per iteration), with dot products, alpha and beta in
// FP64:
//   x = 0, r = b
//   repeat: solve A d = r to inner_rtol in FP32;  x += d (FP64);
//           r = b - A x (FP64 AX, dssum, mask);   stop when ||r||_c <= rtol ||b||_c
// If an inner solve breaks down, or an outer step fails to reduce the
// residual tenfold, the remaining reduction is done by the FP64 PCG on the
// residual equation (fell_back = 1).
#include "solver.hpp"
#include "solver_kernels.hpp"

#include <chrono>
#include <cmath>

namespace nbx {
namespace {

__global__ void f64_to_f32_kernel(int64_t n, const double *__restrict__ a, float *__restrict__ b)
{
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (int64_t)gridDim.x * blockDim.x)
        b[l] = (float)a[l];
}

// x += d (FP32 correction accumulated in FP64)
__global__ void add_f32_to_f64_kernel(int64_t n, const float *__restrict__ d, double *__restrict__ x)
{
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (int64_t)gridDim.x * blockDim.x)
        x[l] += (double)d[l];
}

__global__ void add_f64_kernel(int64_t n, const double *__restrict__ d, double *__restrict__ x)
{
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (int64_t)gridDim.x * blockDim.x)
        x[l] += d[l];
}

unsigned grid_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    return (unsigned)(b < 1 ? 1 : b);
}

// The inner operator's kernel choice as the captured graphs record it: the
// fused-stage tile, or -1 for the matrix-core kernel.
int inner_tile(const nbx_problem *P)
{
    return P->inner_mfma ? -1 : pcg_tile(P->inner_fmt, P->N);
}

int enqueue_iters32(nbx_problem *P, int n_iter, hipStream_t s)
{
    const GsPlan &gs = iter_plan(P);
    // one partial per workgroup of the fused stage: per element on matrix cores
    const int nb1 = P->inner_mfma ? (int)P->E : ax_blocks(P->inner_fmt, P->N, P->E);
    const int nb3 = sk::red_blocks(P->n, sk::Vec<float>::W);
    for (int it = 0; it < n_iter; ++it) {
        int st;
        if (P->inner_mfma)
            st = ax_mfma_pcg_launch(P->inner_fmt,
                                    P->inner_fmt == NBX_F32 ? (const void *)P->G32
                                                            : (const void *)P->G16,
                                    P->gscale, P->D, P->N, P->E, P->z32, P->p32, P->w32,
                                    P->part1, P->scal32, s);
        else
            st = P->inner_fmt == NBX_F32
                     ? ax_pcg_launch_f32(P->G32, P->D, P->N, P->E, P->z32, P->p32, P->w32,
                                         P->part1, P->scal32, s)
                     : ax_pcg_launch_g16(P->inner_fmt, P->G16, P->gscale, P->D, P->N, P->E,
                                         P->z32, P->p32, P->w32, P->part1, P->scal32, s);
        if (st != NBX_OK) return st;
        const PapTask pap{nb1, P->part1, P->scal32};   // R1 rides on the exchange launch
        st = dssum_launch<float>(gs, P->w32, 1, s, P->scal32 + NBX_S_FLAG, &pap);
        if (st != NBX_OK) return st;
        if (P->xd)
            hipLaunchKernelGGL(sk::update_xp_kernel<float>, dim3(nb3), dim3(sk::kRedThreads), 0,
                               s, P->n, P->p32, P->w32, P->dinv32, gs.info, P->d32, P->r32,
                               P->z32, P->part3, P->scal32, P->xd, P->N);
        else
            hipLaunchKernelGGL(sk::update_kernel<float>, dim3(nb3), dim3(sk::kRedThreads), 0, s,
                               P->n, P->p32, P->w32, P->dinv32, gs.info, P->d32, P->r32,
                               P->z32, P->part3, P->scal32);
        hipLaunchKernelGGL(sk::rr_reduce_kernel, dim3(1), dim3(1024), 0, s, nb3, P->part3,
                           P->scal32);
        NBX_LAUNCH_CHECK();
    }
    return NBX_OK;
}

}  // namespace

int prepare_inner(nbx_problem *P, int fmt, hipStream_t s)
{
    if (fmt != NBX_F32 && fmt != NBX_F16 && fmt != NBX_BF16) return NBX_EUNSUPPORTED;
    const size_t n = (size_t)P->n;
    if (!P->dinv32) {
        if (hipMalloc(&P->dinv32, n * sizeof(float)) != hipSuccess ||
            hipMalloc(&P->r32, n * sizeof(float)) != hipSuccess ||
            hipMalloc(&P->z32, n * sizeof(float)) != hipSuccess ||
            hipMalloc(&P->p32, n * sizeof(float)) != hipSuccess ||
            hipMalloc(&P->w32, n * sizeof(float)) != hipSuccess ||
            hipMalloc(&P->d32, n * sizeof(float)) != hipSuccess ||
            hipMalloc(&P->scal32, NBX_SCAL_LEN * sizeof(double)) != hipSuccess) {
            hipFree(P->dinv32); hipFree(P->r32); hipFree(P->z32); hipFree(P->p32);
            hipFree(P->w32); hipFree(P->d32); hipFree(P->scal32);
            P->dinv32 = P->r32 = P->z32 = P->p32 = P->w32 = P->d32 = nullptr;
            P->scal32 = nullptr;
            return NBX_ENOMEM;
        }
        hipLaunchKernelGGL(f64_to_f32_kernel, dim3(grid_for(P->n)), dim3(256), 0, s, P->n,
                           P->dinv, P->dinv32);
        NBX_LAUNCH_CHECK();
    }
    if (fmt == NBX_F32 && !P->G32) {
        if (hipMalloc(&P->G32, 6 * n * sizeof(float)) != hipSuccess) return NBX_ENOMEM;
        hipLaunchKernelGGL(f64_to_f32_kernel, dim3(grid_for(6 * P->n)), dim3(256), 0, s,
                           6 * P->n, P->G, P->G32);
        NBX_LAUNCH_CHECK();
    }
    if (fmt != NBX_F32 && P->g16_fmt != fmt) {
        if (!P->G16) {
            if (hipMalloc(&P->G16, 6 * n * sizeof(uint16_t)) != hipSuccess) return NBX_ENOMEM;
            if (hipMalloc(&P->gscale, (size_t)P->E * sizeof(float)) != hipSuccess) {
                hipFree(P->G16);
                P->G16 = nullptr;
                return NBX_ENOMEM;
            }
        }
        int st = g16_pack_launch(fmt, 0, P->G, P->N, P->E, P->G16, P->gscale, s);
        if (st != NBX_OK) return st;
        P->g16_fmt = fmt;
    }
    P->inner_fmt = fmt;
    NBX_HIP(hipStreamSynchronize(s));
    return NBX_OK;
}

// One FP32 inner solve of A d = r64 to inner_rtol; returns the iterations
// done and the final flag through the pointers.
static int inner_solve(nbx_problem *P, const nbx_pcg_opts &o, int max_iter, int *iters,
                       int *flag)
{
    hipStream_t s = P->ws;
    const GsPlan &gs = P->gs->plan;
    const int nb = sk::red_blocks(P->n);
    hipLaunchKernelGGL((sk::init_kernel<float, double>), dim3(nb), dim3(sk::kRedThreads), 0, s,
                       P->n, P->r, P->dinv32, gs.info, P->d32, P->r32, P->z32, P->p32, P->part3);
    hipLaunchKernelGGL(sk::init_reduce_kernel, dim3(1), dim3(1024), 0, s, nb, P->part3,
                       P->scal32, o.inner_rtol, 0, max_iter);
    NBX_LAUNCH_CHECK();
    const int chunk = o.check_every > 0 ? o.check_every : 10;
    if (o.use_graph && (P->gexec32 == nullptr || P->g32_iters != chunk ||
                        P->g32_fmt != P->inner_fmt || P->g32_tile != inner_tile(P))) {
        if (P->gexec32) { hipGraphExecDestroy(P->gexec32); P->gexec32 = nullptr; }
        NBX_HIP(hipStreamSynchronize(s));
        NBX_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        int st = enqueue_iters32(P, chunk, s);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        if (st != NBX_OK) { if (g) hipGraphDestroy(g); return st; }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&P->gexec32, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) { P->gexec32 = nullptr; return hip_fail(e, "hipGraphInstantiate"); }
        P->g32_iters = chunk;
        P->g32_fmt = P->inner_fmt;
        P->g32_tile = inner_tile(P);
    }
    int done = 0;
    while (true) {
        if (o.use_graph) {
            NBX_HIP(hipGraphLaunch(P->gexec32, s));
        } else {
            int st = enqueue_iters32(P, chunk, s);
            if (st != NBX_OK) return st;
        }
        done += chunk;
        NBX_HIP(hipMemcpyAsync(P->h_scal, P->scal32, sizeof(double) * NBX_SCAL_LEN,
                               hipMemcpyDeviceToHost, s));
        NBX_HIP(hipStreamSynchronize(s));
        if (P->h_scal[NBX_S_FLAG] != 0.0) break;
        if (done >= max_iter + chunk) break;
    }
    *iters = (int)P->h_scal[NBX_S_ITER];
    const double fl = P->h_scal[NBX_S_FLAG];
    *flag = fl == 1.0 ? 1 : (fl == 2.0 ? 2 : 0);
    return NBX_OK;
}

static int pcg_mixed_restart(nbx_problem *P, const double *b, double *x,
                             const nbx_pcg_opts &o, nbx_pcg_result *res);
static int pcg_mixed_reliable(nbx_problem *P, const double *b, double *x,
                              const nbx_pcg_opts &o, nbx_pcg_result *res);

int pcg_mixed(nbx_problem *P, const double *b, double *x, const nbx_pcg_opts &o,
              nbx_pcg_result *res)
{
    P->inner_mfma = o.inner_mfma ? 1 : 0;
    return o.mixed_mode == 1 ? pcg_mixed_restart(P, b, x, o, res)
                             : pcg_mixed_reliable(P, b, x, o, res);
}

// ------------------------------------------------------ reliable updates
// One FP32 Krylov sequence (van der Vorst & Ye's reliable updating): the
// FP32 iteration accumulates its correction in d32; whenever its recurrence
// residual has fallen by a factor inner_rtol since the last update, the
// correction is folded into the FP64 solution, the true residual
// r = b - A x is recomputed in FP64 and replaces the FP32 one, and the
// iteration continues along the same search direction (beta taken from the
// true residual).  Convergence is judged on the FP64 true residual only.

namespace {

// internal slots of the FP32 scalar block beyond the documented ones
constexpr int kSlotBB = 10;      // <b,b>_c in FP64
constexpr int kSlotTol = 11;     // rtol^2 <b,b>_c
constexpr int kSlotD2 = 12;      // inner_rtol^2
constexpr int kSlotFinal = 13;   // 1 once the FP64 true residual meets rtol
constexpr int kSlotTrue = 14;    // last FP64 true <r,r>_c

__global__ void mixed_setup_kernel(double *__restrict__ scal, const double *__restrict__ bb2,
                                   double rtol, double delta)
{
    const double bb = bb2[1];
    scal[kSlotBB] = bb;
    scal[kSlotTol] = rtol * rtol * bb;
    scal[kSlotD2] = delta * delta;
    scal[kSlotTrue] = bb;
    scal[kSlotFinal] = (bb == 0.0) ? 1.0 : 0.0;
    if (bb == 0.0) scal[NBX_S_FLAG] = 1.0;
}

// x += d; d = 0
__global__ void fold_kernel(int64_t n, float *__restrict__ d, double *__restrict__ x)
{
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (int64_t)gridDim.x * blockDim.x) {
        x[l] += (double)d[l];
        d[l] = 0.0f;
    }
}

// r64 = b - w; r32 = r64; z32 = dinv32 r32; partials of c r64^2, c r32 z32.
__global__ void __launch_bounds__(sk::kRedThreads)
replace_kernel(int64_t n, const double *__restrict__ b, const double *__restrict__ w,
               const float *__restrict__ dinv, const uint8_t *__restrict__ info,
               float *__restrict__ r32, float *__restrict__ z32, double *__restrict__ part)
{
    double rr = 0, rz = 0;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (int64_t)gridDim.x * blockDim.x) {
        const double r = b[l] - w[l], c = sk::cw(info[l]);
        const float rf = (float)r, zf = dinv[l] * rf;
        r32[l] = rf; z32[l] = zf;
        rr += c * r * r;
        rz += c * (double)rf * (double)zf;
    }
    sk::block_sum2(rr, rz);
    if (threadIdx.x == 0) { part[2 * blockIdx.x] = rr; part[2 * blockIdx.x + 1] = rz; }
}

__global__ void __launch_bounds__(1024)
reliable_reduce_kernel(int nb, const double *__restrict__ part, double *__restrict__ scal)
{
    __shared__ double s[2][16];
    double a, b;
    sk::partial_sums2(nb, part, a, b);
    a = sk::wsum(a); b = sk::wsum(b);
    if ((threadIdx.x & 63) == 0) { s[0][threadIdx.x >> 6] = a; s[1][threadIdx.x >> 6] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double rr = 0, rz = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) { rr += s[0][q]; rz += s[1][q]; }
        scal[kSlotTrue] = rr;
        scal[NBX_S_RR] = rr;
        if (rr <= scal[kSlotTol]) {
            scal[kSlotFinal] = 1.0;
            scal[NBX_S_FLAG] = 1.0;
        } else if (!(rz > 0.0) || !isfinite(rz) || !isfinite(rr)) {
            scal[NBX_S_FLAG] = 2.0;
        } else {
            scal[NBX_S_BETA] = rz / scal[NBX_S_RHO];
            scal[NBX_S_RHO] = rz;
            scal[NBX_S_STOP] = scal[kSlotD2] * rr;
            scal[NBX_S_FLAG] = scal[NBX_S_ITER] >= scal[NBX_S_MAXIT] ? sk::kFlagLimit : 0.0;
        }
    }
}

}  // namespace

int reliable_start(nbx_problem *P, const double *b, double *x, const nbx_pcg_opts &o,
                   hipStream_t s)
{
    const GsPlan &gs = P->gs->plan;
    const int nb = sk::red_blocks(P->n);
    const double delta = (o.inner_rtol > 0 && o.inner_rtol < 1) ? o.inner_rtol : 0.1;
    // x = 0; r64 = b; <b,b>_c; FP32 state from b
    NBX_HIP(hipMemsetAsync(x, 0, sizeof(double) * (size_t)P->n, s));
    hipLaunchKernelGGL(sk::resid_kernel, dim3(nb), dim3(sk::kRedThreads), 0, s, P->n, b, x,
                       gs.info, P->r, P->part3);
    hipLaunchKernelGGL(sk::sum2_kernel, dim3(1), dim3(1024), 0, s, nb, P->part3, P->tmp2);
    hipLaunchKernelGGL((sk::init_kernel<float, double>), dim3(nb), dim3(sk::kRedThreads), 0, s,
                       P->n, P->r, P->dinv32, gs.info, P->d32, P->r32, P->z32, P->p32, P->part3);
    hipLaunchKernelGGL(sk::init_reduce_kernel, dim3(1), dim3(1024), 0, s, nb, P->part3,
                       P->scal32, delta, 0, o.max_iter);
    hipLaunchKernelGGL(mixed_setup_kernel, dim3(1), dim3(1), 0, s, P->scal32, P->tmp2, o.rtol,
                       delta);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

namespace {

// Ends a problem's FP32 iterations on the device: every later launch of its
// stages (a batch keeps replaying all problems) returns at once, so ITER
// and the state stay as the host's decision left them.
__global__ void stop_kernel(double *scal) { scal[NBX_S_FLAG] = sk::kFlagLimit; }

}  // namespace

int reliable_step(nbx_problem *P, const double *b, double *x, const nbx_pcg_opts &o,
                  const double *h, ReliableState &rs, hipStream_t s)
{
    if (h[kSlotFinal] == 1.0) { rs.done = 1; return NBX_OK; }     // zero right-hand side
    if (h[NBX_S_FLAG] == 2.0) { rs.fell_back = rs.done = 1; return NBX_OK; }
    const GsPlan &gs = P->gs->plan;
    const int nb = sk::red_blocks(P->n);
    // reliable update (also after the iteration limit, to report x)
    hipLaunchKernelGGL(fold_kernel, dim3(grid_for(P->n)), dim3(256), 0, s, P->n, P->d32, x);
    NBX_LAUNCH_CHECK();
    int st = ax_launch_f64(x, P->G, P->D, P->N, P->E, P->w, s);
    if (st != NBX_OK) return st;
    st = dssum_launch<double>(gs, P->w, 1, s);
    if (st != NBX_OK) return st;
    const bool at_limit = h[NBX_S_FLAG] == sk::kFlagLimit;
    hipLaunchKernelGGL(replace_kernel, dim3(nb), dim3(sk::kRedThreads), 0, s, P->n, b, P->w,
                       P->dinv32, gs.info, P->r32, P->z32, P->part3);
    hipLaunchKernelGGL(reliable_reduce_kernel, dim3(1), dim3(1024), 0, s, nb, P->part3,
                       P->scal32);
    NBX_LAUNCH_CHECK();
    double *g = P->h_scal;
    NBX_HIP(hipMemcpyAsync(g, P->scal32, sizeof(double) * NBX_SCAL_LEN, hipMemcpyDeviceToHost,
                           s));
    NBX_HIP(hipStreamSynchronize(s));
    ++rs.updates;
    if (g[kSlotFinal] == 1.0 || at_limit || g[NBX_S_FLAG] == sk::kFlagLimit) {
        rs.done = 1;
        return NBX_OK;
    }
    if (g[NBX_S_FLAG] == 2.0) { rs.fell_back = rs.done = 1; return NBX_OK; }
    // stagnation: two updates in a row without a twofold reduction
    if (rs.last_true >= 0 && !(g[kSlotTrue] < 0.25 * rs.last_true)) ++rs.stalls;
    else rs.stalls = 0;
    rs.last_true = g[kSlotTrue];
    if (rs.stalls >= 2 || rs.updates >= o.max_outer) {
        // the device flag reads 0 (continue) here: make it terminal
        rs.fell_back = rs.stalls >= 2;
        rs.done = 1;
        hipLaunchKernelGGL(stop_kernel, dim3(1), dim3(1), 0, s, P->scal32);
        NBX_LAUNCH_CHECK();
    }
    return NBX_OK;
}

int reliable_finish(nbx_problem *P, const double *b, double *x, const nbx_pcg_opts &o,
                    const ReliableState &rs, nbx_pcg_result *res, hipStream_t s)
{
    double *h = P->h_scal;
    NBX_HIP(hipMemcpyAsync(h, P->scal32, sizeof(double) * NBX_SCAL_LEN, hipMemcpyDeviceToHost,
                           s));
    NBX_HIP(hipStreamSynchronize(s));
    int total = (int)h[NBX_S_ITER];
    const double bb = h[kSlotBB];
    double relres = bb > 0 ? std::sqrt(h[kSlotTrue] / bb) : 0.0;
    int flag = h[kSlotFinal] == 1.0 ? 1 : 0;
    if (rs.fell_back && !flag) {
        // the FP32 sequence broke down or stalled: FP64 PCG from the current x
        double rb[2];
        int st = residual_f64(P, b, x, P->r, rb, s);
        if (st != NBX_OK) return st;
        const double rel0 = rb[1] > 0 ? std::sqrt(rb[0] / rb[1]) : 0.0;
        double *rhs = nullptr, *d = nullptr;
        if (hipMalloc(&rhs, sizeof(double) * (size_t)P->n) != hipSuccess) return NBX_ENOMEM;
        if (hipMalloc(&d, sizeof(double) * (size_t)P->n) != hipSuccess) {
            hipFree(rhs);
            return NBX_ENOMEM;
        }
        NBX_HIP(hipMemcpyAsync(rhs, P->r, sizeof(double) * (size_t)P->n,
                               hipMemcpyDeviceToDevice, s));
        NBX_HIP(hipStreamSynchronize(s));   // pcg_f64 runs on the problem's own stream
        nbx_pcg_opts o64 = o;
        o64.prec = NBX_F64;
        o64.rtol = rel0 > 0 ? o.rtol / rel0 : o.rtol;
        o64.max_iter = o.max_iter - total;
        nbx_pcg_result r64{};
        st = pcg_f64(P, rhs, d, o64, &r64);
        if (st == NBX_OK) {
            hipLaunchKernelGGL(add_f64_kernel, dim3(grid_for(P->n)), dim3(256), 0, s, P->n, d, x);
            st = residual_f64(P, b, x, P->r, rb, s);
        }
        NBX_HIP(hipStreamSynchronize(s));
        hipFree(rhs);
        hipFree(d);
        if (st != NBX_OK) return st;
        total += r64.iters;
        relres = rb[1] > 0 ? std::sqrt(rb[0] / rb[1]) : 0.0;
        flag = relres <= o.rtol ? 1 : (r64.flag == 2 ? 2 : 0);
    }
    res->iters = total;
    res->outer_iters = rs.updates;
    res->relres = relres;
    res->true_relres = relres;
    res->fell_back = rs.fell_back;
    res->flag = flag;
    return NBX_OK;
}

static int pcg_mixed_reliable(nbx_problem *P, const double *b, double *x,
                              const nbx_pcg_opts &o, nbx_pcg_result *res)
{
    hipStream_t s = P->ws;
    int st = prepare_inner(P, o.prec, s);
    if (st != NBX_OK) return st;
    const int chunk = o.check_every > 0 ? o.check_every : 10;
    if (o.use_graph && (P->gexec32 == nullptr || P->g32_iters != chunk ||
                        P->g32_fmt != P->inner_fmt || P->g32_tile != inner_tile(P))) {
        if (P->gexec32) { hipGraphExecDestroy(P->gexec32); P->gexec32 = nullptr; }
        NBX_HIP(hipStreamSynchronize(s));
        NBX_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        st = enqueue_iters32(P, chunk, s);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        if (st != NBX_OK) { if (g) hipGraphDestroy(g); return st; }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&P->gexec32, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) { P->gexec32 = nullptr; return hip_fail(e, "hipGraphInstantiate"); }
        P->g32_iters = chunk;
        P->g32_fmt = P->inner_fmt;
        P->g32_tile = inner_tile(P);
    }
    NBX_HIP(hipStreamSynchronize(s));
    const auto t0 = std::chrono::steady_clock::now();
    st = reliable_start(P, b, x, o, s);
    if (st != NBX_OK) return st;
    ReliableState rs;
    double *h = P->h_scal;
    while (!rs.done) {
        // FP32 iterations until the segment's reduction, breakdown or limit
        while (true) {
            if (o.use_graph) {
                NBX_HIP(hipGraphLaunch(P->gexec32, s));
            } else {
                st = enqueue_iters32(P, chunk, s);
                if (st != NBX_OK) return st;
            }
            NBX_HIP(hipMemcpyAsync(h, P->scal32, sizeof(double) * NBX_SCAL_LEN,
                                   hipMemcpyDeviceToHost, s));
            NBX_HIP(hipStreamSynchronize(s));
            if (h[NBX_S_FLAG] != 0.0) break;
        }
        st = reliable_step(P, b, x, o, h, rs, s);
        if (st != NBX_OK) return st;
    }
    st = reliable_finish(P, b, x, o, rs, res, s);
    if (st != NBX_OK) return st;
    const auto t1 = std::chrono::steady_clock::now();
    res->seconds = std::chrono::duration<double>(t1 - t0).count();
    return NBX_OK;
}

// ------------------------------------------------- restarted refinement

static int pcg_mixed_restart(nbx_problem *P, const double *b, double *x,
                             const nbx_pcg_opts &o, nbx_pcg_result *res)
{
    hipStream_t s = P->ws;
    int st = prepare_inner(P, o.prec, s);
    if (st != NBX_OK) return st;
    const auto t0 = std::chrono::steady_clock::now();
    // x = 0, r = b, ||b||_c
    NBX_HIP(hipMemsetAsync(x, 0, sizeof(double) * (size_t)P->n, s));
    const int nb = sk::red_blocks(P->n);
    hipLaunchKernelGGL(sk::resid_kernel, dim3(nb), dim3(sk::kRedThreads), 0, s, P->n, b, x,
                       P->gs->plan.info, P->r, P->part3);
    hipLaunchKernelGGL(sk::sum2_kernel, dim3(1), dim3(1024), 0, s, nb, P->part3, P->tmp2);
    NBX_LAUNCH_CHECK();
    double rb[2];
    NBX_HIP(hipMemcpyAsync(rb, P->tmp2, sizeof(rb), hipMemcpyDeviceToHost, s));
    NBX_HIP(hipStreamSynchronize(s));
    const double bb = rb[1];
    double relres = bb > 0 ? std::sqrt(rb[0] / bb) : 0.0;
    int total = 0, outer = 0, fell_back = 0, flag = relres <= o.rtol ? 1 : 0;
    double prev = relres;
    while (!flag && outer < o.max_outer && total < o.max_iter) {
        int it = 0, iflag = 0;
        st = inner_solve(P, o, o.max_iter - total, &it, &iflag);
        if (st != NBX_OK) return st;
        total += it;
        ++outer;
        if (iflag == 2 && it == 0) { fell_back = 1; break; }
        hipLaunchKernelGGL(add_f32_to_f64_kernel, dim3(grid_for(P->n)), dim3(256), 0, s, P->n,
                           P->d32, x);
        NBX_LAUNCH_CHECK();
        st = residual_f64(P, b, x, P->r, rb, s);
        if (st != NBX_OK) return st;
        relres = bb > 0 ? std::sqrt(rb[0] / bb) : 0.0;
        if (relres <= o.rtol) { flag = 1; break; }
        if (!std::isfinite(relres) || relres > 0.1 * prev) { fell_back = 1; break; }
        prev = relres;
    }
    if (fell_back && !flag) {
        // finish with FP64 PCG on A d = r (r = b - A x from the last outer step)
        double *rhs = nullptr, *d = nullptr;
        if (hipMalloc(&rhs, sizeof(double) * (size_t)P->n) != hipSuccess) return NBX_ENOMEM;
        if (hipMalloc(&d, sizeof(double) * (size_t)P->n) != hipSuccess) {
            hipFree(rhs);
            return NBX_ENOMEM;
        }
        NBX_HIP(hipMemcpyAsync(rhs, P->r, sizeof(double) * (size_t)P->n,
                               hipMemcpyDeviceToDevice, s));
        nbx_pcg_opts o64 = o;
        o64.prec = NBX_F64;
        o64.rtol = relres > 0 ? o.rtol / relres : o.rtol;
        o64.max_iter = o.max_iter - total;
        nbx_pcg_result r64{};
        st = pcg_f64(P, rhs, d, o64, &r64);
        if (st == NBX_OK) {
            hipLaunchKernelGGL(add_f64_kernel, dim3(grid_for(P->n)), dim3(256), 0, s, P->n, d, x);
            st = residual_f64(P, b, x, P->r, rb, s);
        }
        NBX_HIP(hipStreamSynchronize(s));
        hipFree(rhs);
        hipFree(d);
        if (st != NBX_OK) return st;
        total += r64.iters;
        ++outer;
        relres = bb > 0 ? std::sqrt(rb[0] / bb) : 0.0;
        flag = relres <= o.rtol ? 1 : (r64.flag == 2 ? 2 : 0);
    }
    const auto t1 = std::chrono::steady_clock::now();
    res->seconds = std::chrono::duration<double>(t1 - t0).count();
    res->iters = total;
    res->outer_iters = outer;
    res->relres = relres;
    res->true_relres = relres;
    res->fell_back = fell_back;
    res->flag = flag;
    return NBX_OK;
}

}  // namespace nbx
