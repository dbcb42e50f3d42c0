// pcg.hip -- Jacobi-preconditioned conjugate gradients on the device
// (Section II-B: each CG iteration is vector operations, AX, the
// nearest-neighbour exchange and global reductions, with a simple
// preconditioner, read here as Jacobi).
//
// One iteration is four kernels, all scalars staying on the device:
//   K1  p = z + beta p, w = AX(p), per-block partials of p.w   (ax_kernel.hpp)
//   K2  w = mask(dssum(w))                                      (gs.hip)
//       + R1 in one more workgroup of the same launch: pap = sum of the
//       partials (fixed order), alpha = rho / pap
//   K3  x += alpha p, r -= alpha w, z = dinv r, partials of c r r and c r z
//   R3  rr, rho' (fixed order), convergence / breakdown flag, beta
// <p,w>_c is taken before the exchange: p is continuous and zero on the
// Dirichlet set, so sum_l c_l p_l (dssum w)_l = sum_l p_l w_l.
// The host only launches (optionally a captured hipGraph of several
// iterations) and reads the flag between launches.
#include "solver.hpp"
#include "solver_kernels.hpp"

#include <chrono>
#include <cmath>
#include <mutex>
#include <new>

namespace nbx {

int jacobi_setup_impl(const double *G, const double *D, int N, int64_t E, const GsPlan &gs,
                      double *dinv, hipStream_t s);

// What one fused FP64 iteration reads and writes: the operator (factor
// pairs Gp, D, N, E), the exchange plan, dinv, the state vectors, w (A p of
// the last step) and the two partial-sum buffers (part1: one double per
// fused-stage workgroup, ax_blocks(); part3: 2 * red_blocks(n) doubles).
// xd != 0: gs is an x-pair plan (xpair_plan) and K3 sums its pairs.
struct IterArgs {
    const double *Gp, *D, *dinv;
    int N;
    int64_t E, n;
    const GsPlan *gs;
    double *w, *part1, *part3;
    int64_t xd = 0;
};

// Enqueues n_iter fused FP64 iterations on s.
static int enqueue_iters_on(const IterArgs &a, double *x, double *r, double *z, double *p,
                            double *scal, int n_iter, hipStream_t s)
{
    const GsPlan &gs = *a.gs;
    const int nb1 = ax_blocks(NBX_F64, a.N, a.E);
    const int nb3 = sk::red_blocks(a.n);
    for (int it = 0; it < n_iter; ++it) {
        int st = ax_pcg_launch_f64(a.Gp, a.D, a.N, a.E, z, p, a.w, a.part1, scal, s);
        if (st != NBX_OK) return st;
        const PapTask pap{nb1, a.part1, scal};   // R1 rides on the exchange launch
        st = dssum_launch<double>(gs, a.w, 1, s, scal + NBX_S_FLAG, &pap);
        if (st != NBX_OK) return st;
        if (a.xd)
            hipLaunchKernelGGL(sk::update_xp_kernel<double>, dim3(nb3), dim3(sk::kRedThreads), 0,
                               s, a.n, p, a.w, a.dinv, gs.info, x, r, z, a.part3, scal, a.xd,
                               a.N);
        else
            hipLaunchKernelGGL(sk::update_kernel<double>, dim3(nb3), dim3(sk::kRedThreads), 0, s,
                               a.n, p, a.w, a.dinv, gs.info, x, r, z, a.part3, scal);
        hipLaunchKernelGGL(sk::rr_reduce_kernel, dim3(1), dim3(1024), 0, s, nb3, a.part3,
                           scal);
        NBX_LAUNCH_CHECK();
    }
    return NBX_OK;
}

static int enqueue_iters(nbx_problem *P, double *x, double *r, double *z, double *p,
                         double *scal, int n_iter, hipStream_t s)
{
    const IterArgs a{P->G, P->D, P->dinv, P->N, P->E, P->n, &iter_plan(P),
                     P->w, P->part1, P->part3, P->xd};
    return enqueue_iters_on(a, x, r, z, p, scal, n_iter, s);
}

int residual_f64(nbx_problem *P, const double *b, const double *x, double *r, double out[2],
                 hipStream_t s)
{
    int st = ax_launch_f64(x, P->G, P->D, P->N, P->E, P->w, s);
    if (st != NBX_OK) return st;
    st = dssum_launch<double>(P->gs->plan, P->w, 1, s);
    if (st != NBX_OK) return st;
    const int nb = sk::red_blocks(P->n);
    hipLaunchKernelGGL(sk::resid_kernel, dim3(nb), dim3(sk::kRedThreads), 0, s, P->n, b, P->w,
                       P->gs->plan.info, r, P->part3);
    hipLaunchKernelGGL(sk::sum2_kernel, dim3(1), dim3(1024), 0, s, nb, P->part3, P->tmp2);
    NBX_LAUNCH_CHECK();
    NBX_HIP(hipMemcpyAsync(P->h_scal, P->tmp2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    NBX_HIP(hipStreamSynchronize(s));
    out[0] = P->h_scal[0];
    out[1] = P->h_scal[1];
    return NBX_OK;
}

// Plain FP64 Jacobi-PCG from x = 0 on the problem's own stream.
int pcg_f64(nbx_problem *P, const double *b, double *x, const nbx_pcg_opts &o,
            nbx_pcg_result *res)
{
    hipStream_t s = P->ws;
    const GsPlan &gs = P->gs->plan;
    const int nb = sk::red_blocks(P->n);
    hipLaunchKernelGGL((sk::init_kernel<double, double>), dim3(nb), dim3(sk::kRedThreads), 0, s,
                       P->n, b, P->dinv, gs.info, x, P->r, P->z, P->p, P->part3);
    hipLaunchKernelGGL(sk::init_reduce_kernel, dim3(1), dim3(1024), 0, s, nb, P->part3, P->scal,
                       o.rtol, o.fixed_iters, o.max_iter);
    NBX_LAUNCH_CHECK();
    const int chunk = o.check_every > 0 ? o.check_every : 10;
    const int tile = pcg_tile(NBX_F64, P->N);   // the captured launches bake it in
    if (o.use_graph &&
        (P->gexec == nullptr || P->g_x != x || P->g_iters != chunk || P->g_tile != tile)) {
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
        P->g_x = x; P->g_iters = chunk; P->g_tile = tile;
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
    double rb[2];
    int st = residual_f64(P, b, x, nullptr, rb, s);
    if (st != NBX_OK) return st;
    res->true_relres = rb[1] > 0 ? std::sqrt(rb[0] / rb[1]) : 0.0;
    return NBX_OK;
}

}  // namespace nbx

using namespace nbx;

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
    P->D = D; P->N = N; P->E = E; P->n = n; P->gs = gs;
    auto fail = [&](int st) { nbx_problem_destroy(P); return st; };
    const size_t vb = sizeof(double) * (size_t)n;
    if (hipMalloc(&P->Gown, 6 * vb) != hipSuccess) return fail(NBX_ENOMEM);
    P->G = P->Gown;
    if (hipMalloc(&P->dinv, vb) != hipSuccess || hipMalloc(&P->r, vb) != hipSuccess ||
        hipMalloc(&P->z, vb) != hipSuccess || hipMalloc(&P->p, vb) != hipSuccess ||
        hipMalloc(&P->w, vb) != hipSuccess ||
        hipMalloc(&P->part1, sizeof(double) * (size_t)E) != hipSuccess ||
        hipMalloc(&P->part3, sizeof(double) * 2 * sk::kMaxRedBlocks) != hipSuccess ||
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
    int st = pair_factors_launch(G, P->Gown, N, E, s);
    if (st != NBX_OK) return fail(st);
    st = jacobi_setup_impl(G, D, N, E, gs->plan, P->dinv, s);
    if (st != NBX_OK) return fail(st);
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(hip_fail(e, "hipStreamSynchronize"));
    int found = 0;
    st = xpair_plan(gs->plan, N, P->xplan, &found);
    if (st != NBX_OK) return fail(st);
    if (found) P->xd = xpair_offset(N);
    *out = P;
    return NBX_OK;
}

extern "C" int nbx_problem_destroy(nbx_problem *P)
{
    if (!P) return NBX_OK;
    if (P->ws) hipStreamSynchronize(P->ws);
    if (P->gexec) hipGraphExecDestroy(P->gexec);
    if (P->gexec32) hipGraphExecDestroy(P->gexec32);
    free_plan(P->xplan);
    hipFree(P->Gown);
    hipFree(P->dinv); hipFree(P->r); hipFree(P->z); hipFree(P->p); hipFree(P->w);
    hipFree(P->part1); hipFree(P->part3); hipFree(P->scal); hipFree(P->tmp2);
    hipFree(P->G32); hipFree(P->dinv32); hipFree(P->r32); hipFree(P->z32); hipFree(P->p32);
    hipFree(P->w32); hipFree(P->d32); hipFree(P->scal32); hipFree(P->G16); hipFree(P->gscale);
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

extern "C" int nbx_problem_exchange_info(nbx_problem *P, int64_t out[5])
{
    if (!P || !out) return NBX_EINVAL;
    out[0] = P->gs->plan.n_groups;
    out[1] = iter_plan(P).n_groups;
    out[2] = P->xd;   // x-face pairs only
    out[3] = out[4] = 0;
    return NBX_OK;
}

extern "C" int nbx_pcg_iterate(nbx_problem *P, double *x, double *r, double *z, double *pdir,
                               double *scal, int n_iter, void *stream)
{
    if (!P || !x || !r || !z || !pdir || !scal || n_iter < 0) return NBX_EINVAL;
    return enqueue_iters(P, x, r, z, pdir, scal, n_iter, as_stream(stream));
}

// ------------------------------------------ the allocation-free variant
//
// For callers that cannot allocate (code under stream capture, serving
// loops): the reduction partials of nbx_pcg_iterate_noalloc live in one
// file-scope device array per GPU, reached through the address that
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in in host code).  Every call on a GPU shares that GPU's
// array, so calls that overlap on one GPU race.  Each launch writes every
// partial it later reads, so nothing needs clearing between calls.
namespace {

constexpr int64_t kNoallocPart3 = 2 * (int64_t)sk::kMaxRedBlocks;   // 2 MB
constexpr int64_t kNoallocPart1 = NBX_NOALLOC_MAX_BLOCKS;           // 2 MB
__device__ __align__(256) double scratch[kNoallocPart3 + kNoallocPart1];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch` (looked up once per device).
int scratch_for_current_device(double **out)
{
    int dev = 0;
    NBX_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return NBX_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        NBX_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return NBX_OK;
}

}  // namespace

extern "C" int nbx_pcg_iterate_noalloc(const double *Gp, const double *D, int N, int64_t E,
                                       nbx_gs *gs, const double *dinv, double *x, double *r,
                                       double *z, double *pdir, double *w, double *scal,
                                       int n_iter, void *stream)
{
    if (!Gp || !D || !gs || !dinv || !x || !r || !z || !pdir || !w || !scal || n_iter < 0)
        return NBX_EINVAL;
    if (N < 2 || N > kMaxN || E < 1) return NBX_EINVAL;
    const int64_t n = E * (int64_t)N * N * N;
    if (gs->plan.n_local != n) return NBX_EINVAL;
    if (ax_blocks(NBX_F64, N, E) > kNoallocPart1) return NBX_EUNSUPPORTED;   // scratch too small
    double *sc = nullptr;
    const int st = scratch_for_current_device(&sc);
    if (st != NBX_OK) return st;
    const IterArgs a{Gp, D, dinv, N, E, n, &gs->plan, w, sc + kNoallocPart3, sc};
    return enqueue_iters_on(a, x, r, z, pdir, scal, n_iter, as_stream(stream));
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
    o->inner_rtol = 0.1;
    o->max_outer = 200;
    o->mixed_mode = 0;
    o->inner_mfma = 0;
}

extern "C" int nbx_pcg(nbx_problem *P, const double *b, double *x, const nbx_pcg_opts *opts,
                       nbx_pcg_result *res, void *stream)
{
    if (!P || !b || !x || !res) return NBX_EINVAL;
    nbx_pcg_opts o;
    if (opts) o = *opts; else nbx_pcg_default_opts(&o);
    if (o.max_iter < 0 || !(o.rtol >= 0) || o.max_outer < 1) return NBX_EINVAL;
    *res = nbx_pcg_result{};
    hipStream_t cs = as_stream(stream);
    // order the solve after the caller's pending work on its stream
    NBX_HIP(hipEventRecord(P->ev, cs));
    NBX_HIP(hipStreamWaitEvent(P->ws, P->ev, 0));
    int st;
    if (o.prec == NBX_F64) st = pcg_f64(P, b, x, o, res);
    else if (o.prec == NBX_F32 || o.prec == NBX_F16 || o.prec == NBX_BF16)
        st = pcg_mixed(P, b, x, o, res);
    else return NBX_EUNSUPPORTED;
    if (st != NBX_OK) return st;
    NBX_HIP(hipEventRecord(P->ev, P->ws));
    NBX_HIP(hipStreamWaitEvent(cs, P->ev, 0));
    if (res->flag == 2) return NBX_EBREAKDOWN;
    return res->flag == 1 ? NBX_OK : NBX_NOT_CONVERGED;
}
