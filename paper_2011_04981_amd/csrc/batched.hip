// batched.hip -- many independent Jacobi-PCG solves of uneven size and
// polynomial order advanced together.
//
// Each problem keeps its own workspace (nbx_problem).  A device table of
// per-problem descriptors plus, for every fused step of the iteration, a
// table of (problem, block) entries lets ONE launch of that step serve every
// problem: the AX step is launched once per polynomial size present (its
// kernel is specialised on N, with the tile the autotuner chose), the
// reductions once with one workgroup per problem, dssum and the vector
// update once over all problems' blocks.  Blocks of a converged problem
// return at once, so the batch shrinks as problems finish.  The host replays
// a captured hipGraph of `check_every` iterations until every problem's
// flag is set.  The per-problem arithmetic is exactly the standalone
// solver's (same bodies, same block counts, same reduction order): batched
// results are bit-identical to solving each problem alone.
//
// Mixed-precision batches (prec NBX_F32 / NBX_F16 / NBX_BF16, reliable
// updates) run the FP32 iterations of all problems the same way, from a
// second descriptor table, and do each problem's FP64 residual replacement
// between replays with the standalone solver's own steps (reliable_step), so
// those results are bit-identical to standalone mixed solves too.
//
// The paper distributes independent elements across kernels (Section IV);
// here independent problems share launches for the same reason: the GPU is
// only full when small problems are processed together.
#include "solver.hpp"
#include "solver_kernels.hpp"
#include "ax_kernel.hpp"
#include "ax16_mfma.hpp"
#include "gs_kernels.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

namespace nbx {
namespace {

struct BDesc {
    const double *G, *D, *dinv, *b;
    const uint8_t *info;
    double *x, *r, *z, *p, *w, *part1, *part3, *scal, *stamp;
    const int32_t *off, *idx, *mask_idx;
    const uint8_t *gflag;
    int32_t n_groups, n_mask_only;
    int64_t E, n;
    int32_t N, nb1, nb3, pad;
};

struct BEntry {
    int32_t pid, blk;
};

// Pointers read from a descriptor carry no address space, so every access
// through them would compile to a flat one (flat loads count against both
// the memory and the LDS wait counters, and uniform ones cannot use scalar
// loads).  These casts restore what they are: global memory (rebuilt from
// the integer value: a cast straight from the generic pointer and back is
// folded away before address spaces are inferred).  Measured on the batched
// N = 12 fused AX stage: 279 flat loads and 432 waits became the standalone
// kernel's global and scalar loads and 249 waits.
template <typename T>
__device__ inline T *gp(T *p)
{
    return (T *)(__attribute__((address_space(1))) T *)(uintptr_t)p;
}
// D for an AX stage.  Where the kernel takes D slab by slab (ax_pin_d), its
// uniform loads stay scalar only from constant memory (the ordering asm
// would count as a possible store to global memory); elsewhere constant
// memory would let the compiler hoist all N^2 values to the top (SGPR
// spills in FP64, 214-256 VGPRs in FP32), so D stays global there.
template <typename T, int N>
__device__ inline const double *dp(const double *p)
{
    if constexpr (ax_pin_d<T, N>())
        return (const double *)(const __attribute__((address_space(4))) double *)(uintptr_t)p;
    else
        return gp(p);
}

__global__ void __launch_bounds__(sk::kRedThreads)
b_init_kernel(const BDesc *__restrict__ desc, const BEntry *__restrict__ tab)
{
    const BEntry en = tab[blockIdx.x];
    const BDesc &d = desc[en.pid];
    sk::init_body<double, double>(d.n, gp(d.b), gp(d.dinv), gp(d.info), gp(d.x), gp(d.r),
                                  gp(d.z), gp(d.p), gp(d.part3), en.blk, d.nb3);
}

__global__ void __launch_bounds__(1024)
b_init_reduce_kernel(const BDesc *__restrict__ desc, double rtol, int fixed, int max_iter)
{
    const BDesc &d = desc[blockIdx.x];
    sk::init_reduce_body(d.nb3, gp(d.part3), gp(d.scal), rtol, fixed, max_iter);
}

template <int N, int EPB>
__global__ void __launch_bounds__((AxShape<N, EPB>::NT))
b_ax_kernel(const BDesc *__restrict__ desc, const BEntry *__restrict__ tab)
{
    const BEntry en = tab[blockIdx.x];
    const BDesc &d = desc[en.pid];
    ax_body<double, N, EPB, true>(gp(d.z), gp(d.G), dp<double, N>(d.D), gp(d.w), gp(d.p),
                                  gp(d.part1), gp(d.scal), d.E, en.blk);
}

// N = 16: the standalone solver's matrix-core body, so a batched problem
// computes the standalone solve's bits
__global__ void __launch_bounds__(256, 2)
b_ax16_kernel(const BDesc *__restrict__ desc, const BEntry *__restrict__ tab)
{
    const BEntry en = tab[blockIdx.x];
    const BDesc &d = desc[en.pid];
    ax16::body<false, true>(gp(d.z), gp(d.G), gp(d.D), gp(d.w), gp(d.p), gp(d.part1),
                            gp(d.scal), en.blk);
}

__global__ void __launch_bounds__(1024) b_pap_kernel(const BDesc *__restrict__ desc)
{
    const BDesc &d = desc[blockIdx.x];
    sk::pap_reduce_body(d.nb1, gp(d.part1), gp(d.scal));
}

__global__ void __launch_bounds__(kGsThreads)
b_dssum_kernel(const BDesc *__restrict__ desc, const BEntry *__restrict__ tab)
{
    const BEntry en = tab[blockIdx.x];
    const BDesc &d = desc[en.pid];
    if (gp(d.scal)[NBX_S_FLAG] != 0.0) return;
    const int32_t g = en.blk * kGsThreads + threadIdx.x;
    if (g < d.n_groups) dssum_group<double>(g, gp(d.off), gp(d.idx), gp(d.gflag), gp(d.w), 1);
}

__global__ void __launch_bounds__(256)
b_mask_kernel(const BDesc *__restrict__ desc, const BEntry *__restrict__ tab)
{
    const BEntry en = tab[blockIdx.x];
    const BDesc &d = desc[en.pid];
    if (gp(d.scal)[NBX_S_FLAG] != 0.0) return;
    const int32_t q = en.blk * 256 + threadIdx.x;
    if (q < d.n_mask_only) gp(d.w)[gp(d.mask_idx)[q]] = 0.0;
}

__global__ void __launch_bounds__(sk::kRedThreads)
b_update_kernel(const BDesc *__restrict__ desc, const BEntry *__restrict__ tab)
{
    const BEntry en = tab[blockIdx.x];
    const BDesc &d = desc[en.pid];
    sk::update_body<double>(d.n, gp(d.p), gp(d.w), gp(d.dinv), gp(d.info), gp(d.x), gp(d.r),
                            gp(d.z), gp(d.part3), gp(d.scal), en.blk, d.nb3);
}

__global__ void __launch_bounds__(1024) b_rr_kernel(const BDesc *__restrict__ desc)
{
    const BDesc &d = desc[blockIdx.x];
    sk::rr_reduce_body(d.nb3, gp(d.part3), gp(d.scal), gp(d.stamp));
}

__global__ void b_clock_kernel(double *t0) { *t0 = (double)wall_clock64(); }

// ---- the FP32 iterations of a mixed-precision batch (enqueue_iters32's
// stages, one launch each for every problem)
struct BDesc32 {
    const void *G;             // FP32 pair planes or 16-bit words
    const float *gscale;
    const double *D;
    const float *dinv;
    const uint8_t *info;
    float *z, *p, *w, *d, *r;
    double *part1, *part3, *scal;
    const int32_t *off, *idx, *mask_idx;
    const uint8_t *gflag;
    int32_t n_groups, n_mask_only;
    int64_t E, n;
    int32_t N, nb1, nb3, pad;
};

template <int N, int EPB, typename GT>
__global__ void __launch_bounds__((AxShape<N, EPB>::NT))
b_ax32_kernel(const BDesc32 *__restrict__ desc, const BEntry *__restrict__ tab)
{
    const BEntry en = tab[blockIdx.x];
    const BDesc32 &d = desc[en.pid];
    ax_body<float, N, EPB, true, GT>(gp(d.z), gp(reinterpret_cast<const GT *>(d.G)),
                                     dp<float, N>(d.D), gp(d.w), gp(d.p), gp(d.part1),
                                     gp(d.scal), d.E, en.blk, gp(d.gscale));
}

__global__ void __launch_bounds__(1024) b_pap32_kernel(const BDesc32 *__restrict__ desc)
{
    const BDesc32 &d = desc[blockIdx.x];
    sk::pap_reduce_body(d.nb1, gp(d.part1), gp(d.scal));
}

__global__ void __launch_bounds__(kGsThreads)
b_dssum32_kernel(const BDesc32 *__restrict__ desc, const BEntry *__restrict__ tab)
{
    const BEntry en = tab[blockIdx.x];
    const BDesc32 &d = desc[en.pid];
    if (gp(d.scal)[NBX_S_FLAG] != 0.0) return;
    const int32_t g = en.blk * kGsThreads + threadIdx.x;
    if (g < d.n_groups) dssum_group<float>(g, gp(d.off), gp(d.idx), gp(d.gflag), gp(d.w), 1);
}

__global__ void __launch_bounds__(256)
b_mask32_kernel(const BDesc32 *__restrict__ desc, const BEntry *__restrict__ tab)
{
    const BEntry en = tab[blockIdx.x];
    const BDesc32 &d = desc[en.pid];
    if (gp(d.scal)[NBX_S_FLAG] != 0.0) return;
    const int32_t q = en.blk * 256 + threadIdx.x;
    if (q < d.n_mask_only) gp(d.w)[gp(d.mask_idx)[q]] = 0.0f;
}

__global__ void __launch_bounds__(sk::kRedThreads)
b_update32_kernel(const BDesc32 *__restrict__ desc, const BEntry *__restrict__ tab)
{
    const BEntry en = tab[blockIdx.x];
    const BDesc32 &d = desc[en.pid];
    sk::update_body<float>(d.n, gp(d.p), gp(d.w), gp(d.dinv), gp(d.info), gp(d.d), gp(d.r),
                           gp(d.z), gp(d.part3), gp(d.scal), en.blk, d.nb3);
}

__global__ void __launch_bounds__(1024) b_rr32_kernel(const BDesc32 *__restrict__ desc)
{
    const BDesc32 &d = desc[blockIdx.x];
    sk::rr_reduce_body(d.nb3, gp(d.part3), gp(d.scal));
}

template <int N, typename GT>
int launch_b_ax32(int epb, const BDesc32 *desc, const BEntry *tab, int nblk, hipStream_t s)
{
    switch (epb) {
#define NBX_BAX32(EE)                                                                        \
    case EE:                                                                                 \
        if constexpr (AxShape<N, EE>::template fits<float>()) {                              \
            hipLaunchKernelGGL((b_ax32_kernel<N, EE, GT>), dim3(nblk),                       \
                               dim3(AxShape<N, EE>::NT), 0, s, desc, tab);                   \
            return NBX_OK;                                                                   \
        } else {                                                                             \
            return NBX_EUNSUPPORTED;                                                         \
        }
        NBX_BAX32(1) NBX_BAX32(2) NBX_BAX32(4) NBX_BAX32(8)
#undef NBX_BAX32
        default: return NBX_EINVAL;
    }
}

template <typename GT>
int launch_b_ax32_n(int N, int epb, const BDesc32 *desc, const BEntry *tab, int nblk,
                    hipStream_t s)
{
    switch (N) {
#define NBX_BAX32N(NN) case NN: return launch_b_ax32<NN, GT>(epb, desc, tab, nblk, s);
        NBX_BAX32N(2) NBX_BAX32N(3) NBX_BAX32N(4) NBX_BAX32N(5) NBX_BAX32N(6) NBX_BAX32N(7)
        NBX_BAX32N(8) NBX_BAX32N(9) NBX_BAX32N(10) NBX_BAX32N(11) NBX_BAX32N(12)
        NBX_BAX32N(13) NBX_BAX32N(14) NBX_BAX32N(15) NBX_BAX32N(16)
#undef NBX_BAX32N
        default: return NBX_EINVAL;
    }
}

template <int N>
int launch_b_ax(int epb, const BDesc *desc, const BEntry *tab, int nblk, hipStream_t s)
{
    switch (epb) {
#define NBX_BAX(EE)                                                                          \
    case EE:                                                                                 \
        if constexpr (AxShape<N, EE>::template fits<double>()) {                             \
            hipLaunchKernelGGL((b_ax_kernel<N, EE>), dim3(nblk), dim3(AxShape<N, EE>::NT),   \
                               0, s, desc, tab);                                             \
            return NBX_OK;                                                                   \
        } else {                                                                             \
            return NBX_EUNSUPPORTED;                                                         \
        }
        NBX_BAX(1) NBX_BAX(2) NBX_BAX(4) NBX_BAX(8)
#undef NBX_BAX
        default: return NBX_EINVAL;
    }
}

int launch_b_ax_n(int N, int epb, const BDesc *desc, const BEntry *tab, int nblk, hipStream_t s)
{
    if (N == 16) {
        if (epb != 1) return NBX_EUNSUPPORTED;
        hipLaunchKernelGGL(b_ax16_kernel, dim3(nblk), dim3(256), 0, s, desc, tab);
        return NBX_OK;
    }
    switch (N) {
#define NBX_BAXN(NN) case NN: return launch_b_ax<NN>(epb, desc, tab, nblk, s);
        NBX_BAXN(2) NBX_BAXN(3) NBX_BAXN(4) NBX_BAXN(5) NBX_BAXN(6) NBX_BAXN(7) NBX_BAXN(8)
        NBX_BAXN(9) NBX_BAXN(10) NBX_BAXN(11) NBX_BAXN(12) NBX_BAXN(13) NBX_BAXN(14)
        NBX_BAXN(15) NBX_BAXN(16)
#undef NBX_BAXN
        default: return NBX_EINVAL;
    }
}

// Device copies of the batch's tables, freed by the destructor.
struct BatchPlan {
    int nprob = 0;
    BDesc *desc = nullptr;
    double *stamps = nullptr, *t0 = nullptr;
    BEntry *t_vec = nullptr, *t_gs = nullptr, *t_mask = nullptr;
    int n_vec = 0, n_gs = 0, n_mask = 0;
    struct AxClass { int N, epb, nblk; BEntry *tab; };
    std::vector<AxClass> ax;
    ~BatchPlan()
    {
        hipFree(desc); hipFree(stamps); hipFree(t0);
        hipFree(t_vec); hipFree(t_gs); hipFree(t_mask);
        for (auto &c : ax) hipFree(c.tab);
    }
};

template <typename T>
int upload(T **dst, const std::vector<T> &h)
{
    if (hipMalloc(dst, std::max<size_t>(h.size(), 1) * sizeof(T)) != hipSuccess) return NBX_ENOMEM;
    if (!h.empty())
        NBX_HIP(hipMemcpy(*dst, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return NBX_OK;
}

int enqueue_batch_iters(const BatchPlan &B, int n_iter, hipStream_t s)
{
    for (int it = 0; it < n_iter; ++it) {
        for (const auto &c : B.ax) {
            int st = launch_b_ax_n(c.N, c.epb, B.desc, c.tab, c.nblk, s);
            if (st != NBX_OK) return st;
        }
        hipLaunchKernelGGL(b_pap_kernel, dim3(B.nprob), dim3(1024), 0, s, B.desc);
        if (B.n_gs > 0)
            hipLaunchKernelGGL(b_dssum_kernel, dim3(B.n_gs), dim3(kGsThreads), 0, s, B.desc,
                               B.t_gs);
        if (B.n_mask > 0)
            hipLaunchKernelGGL(b_mask_kernel, dim3(B.n_mask), dim3(256), 0, s, B.desc, B.t_mask);
        hipLaunchKernelGGL(b_update_kernel, dim3(B.n_vec), dim3(sk::kRedThreads), 0, s, B.desc,
                           B.t_vec);
        hipLaunchKernelGGL(b_rr_kernel, dim3(B.nprob), dim3(1024), 0, s, B.desc);
        NBX_LAUNCH_CHECK();
    }
    return NBX_OK;
}

// The FP32 tables of a mixed-precision batch, freed by the destructor.
struct BatchPlan32 {
    int nprob = 0, fmt = NBX_F32;
    BDesc32 *desc = nullptr;
    BEntry *t_vec = nullptr, *t_gs = nullptr, *t_mask = nullptr;
    int n_vec = 0, n_gs = 0, n_mask = 0;
    struct AxClass { int N, epb, nblk; BEntry *tab; };
    std::vector<AxClass> ax;
    ~BatchPlan32()
    {
        hipFree(desc); hipFree(t_vec); hipFree(t_gs); hipFree(t_mask);
        for (auto &c : ax) hipFree(c.tab);
    }
};

int enqueue_batch32_iters(const BatchPlan32 &B, int n_iter, hipStream_t s)
{
    for (int it = 0; it < n_iter; ++it) {
        for (const auto &c : B.ax) {
            int st = B.fmt == NBX_F32
                         ? launch_b_ax32_n<float>(c.N, c.epb, B.desc, c.tab, c.nblk, s)
                         : (B.fmt == NBX_F16
                                ? launch_b_ax32_n<g_f16>(c.N, c.epb, B.desc, c.tab, c.nblk, s)
                                : launch_b_ax32_n<g_bf16>(c.N, c.epb, B.desc, c.tab, c.nblk, s));
            if (st != NBX_OK) return st;
        }
        hipLaunchKernelGGL(b_pap32_kernel, dim3(B.nprob), dim3(1024), 0, s, B.desc);
        if (B.n_gs > 0)
            hipLaunchKernelGGL(b_dssum32_kernel, dim3(B.n_gs), dim3(kGsThreads), 0, s, B.desc,
                               B.t_gs);
        if (B.n_mask > 0)
            hipLaunchKernelGGL(b_mask32_kernel, dim3(B.n_mask), dim3(256), 0, s, B.desc,
                               B.t_mask);
        hipLaunchKernelGGL(b_update32_kernel, dim3(B.n_vec), dim3(sk::kRedThreads), 0, s, B.desc,
                           B.t_vec);
        hipLaunchKernelGGL(b_rr32_kernel, dim3(B.nprob), dim3(1024), 0, s, B.desc);
        NBX_LAUNCH_CHECK();
    }
    return NBX_OK;
}

// A mixed-precision batch (reliable updates): the FP32 iterations of every
// unfinished problem replayed together, each problem's FP64 residual
// replacement done between replays by the standalone steps.  Per-solve
// latency is taken on the host when a problem's last step ends.
int pcg_batched_mixed(nbx_problem *const *probs, const double *const *b, double *const *x,
                      int nprob, const nbx_pcg_opts &o, nbx_pcg_result *results,
                      double *solve_seconds, hipStream_t cs)
{
    if (o.mixed_mode != 0) return NBX_EUNSUPPORTED;
    for (int p = 0; p < nprob; ++p) {
        int st = prepare_inner(probs[p], o.prec, probs[p]->ws);
        if (st != NBX_OK) return st;
    }
    BatchPlan32 B;
    B.nprob = nprob;
    B.fmt = o.prec;
    std::vector<BDesc32> hd(nprob);
    std::vector<BEntry> tv, tg, tm;
    for (int p = 0; p < nprob; ++p) {
        nbx_problem *P = probs[p];
        const GsPlan &g = P->gs->plan;
        BDesc32 &d = hd[p];
        d.G = o.prec == NBX_F32 ? (const void *)P->G32 : (const void *)P->G16;
        d.gscale = P->gscale;
        d.D = P->D; d.dinv = P->dinv32; d.info = g.info;
        d.z = P->z32; d.p = P->p32; d.w = P->w32; d.d = P->d32; d.r = P->r32;
        d.part1 = P->part1; d.part3 = P->part3; d.scal = P->scal32;
        d.off = g.off; d.idx = g.idx; d.mask_idx = g.mask_idx; d.gflag = g.gflag;
        d.n_groups = g.n_groups; d.n_mask_only = g.n_mask_only;
        d.E = P->E; d.n = P->n; d.N = P->N;
        d.nb1 = ax_blocks(o.prec, P->N, P->E);
        d.nb3 = sk::red_blocks(P->n, sk::Vec<float>::W);
        d.pad = 0;
        for (int q = 0; q < d.nb3; ++q) tv.push_back({p, q});
        for (int q = 0; q < (g.n_groups + kGsThreads - 1) / kGsThreads; ++q) tg.push_back({p, q});
        for (int q = 0; q < (g.n_mask_only + 255) / 256; ++q) tm.push_back({p, q});
    }
    int st;
    if ((st = upload(&B.desc, hd)) != NBX_OK) return st;
    if ((st = upload(&B.t_vec, tv)) != NBX_OK) return st;
    if ((st = upload(&B.t_gs, tg)) != NBX_OK) return st;
    if ((st = upload(&B.t_mask, tm)) != NBX_OK) return st;
    B.n_vec = (int)tv.size(); B.n_gs = (int)tg.size(); B.n_mask = (int)tm.size();
    std::vector<int> Ns;
    for (int p = 0; p < nprob; ++p) Ns.push_back(probs[p]->N);
    std::sort(Ns.begin(), Ns.end());
    Ns.erase(std::unique(Ns.begin(), Ns.end()), Ns.end());
    for (int N : Ns) {
        std::vector<BEntry> ta;
        for (int p = 0; p < nprob; ++p)
            if (probs[p]->N == N)
                for (int q = 0; q < hd[p].nb1; ++q) ta.push_back({p, q});
        BatchPlan32::AxClass c{N, pcg_tile(o.prec, N), (int)ta.size(), nullptr};
        if ((st = upload(&c.tab, ta)) != NBX_OK) return st;
        B.ax.push_back(c);
    }

    hipStream_t s = nullptr;
    NBX_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipEvent_t ev = nullptr;
    NBX_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    double *h = nullptr;
    NBX_HIP(hipHostMalloc(&h, sizeof(double) * NBX_SCAL_LEN * nprob, hipHostMallocDefault));
    hipGraphExec_t gexec = nullptr;
    auto cleanup = [&]() {
        if (gexec) hipGraphExecDestroy(gexec);
        if (s) { hipStreamSynchronize(s); hipStreamDestroy(s); }
        if (ev) hipEventDestroy(ev);
        if (h) hipHostFree(h);
    };
    auto fail = [&](int code) { cleanup(); return code; };

    // after the caller's pending work and each problem's set-up
    if (hipEventRecord(ev, cs) != hipSuccess || hipStreamWaitEvent(s, ev, 0) != hipSuccess)
        return fail(NBX_EHIP);
    for (int p = 0; p < nprob; ++p)
        if (hipStreamSynchronize(probs[p]->ws) != hipSuccess) return fail(NBX_EHIP);
    const int chunk = o.check_every > 0 ? o.check_every : 10;
    if (o.use_graph) {
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(NBX_EHIP);
        st = enqueue_batch32_iters(B, chunk, s);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        if (st != NBX_OK) { if (g) hipGraphDestroy(g); return fail(st); }
        if (e != hipSuccess) return fail(hip_fail(e, "hipStreamEndCapture"));
        e = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) { gexec = nullptr; return fail(hip_fail(e, "hipGraphInstantiate")); }
    }

    const auto t0 = std::chrono::steady_clock::now();
    for (int p = 0; p < nprob; ++p) {
        st = reliable_start(probs[p], b[p], x[p], o, s);
        if (st != NBX_OK) return fail(st);
    }
    std::vector<ReliableState> rs(nprob);
    std::vector<double> finished(nprob, 0.0);
    // every replay advances each unfinished problem by up to chunk FP32
    // iterations or ends a segment; the bound only guards the host loop
    const int64_t max_replays = (int64_t)o.max_iter / chunk + 2 * (int64_t)o.max_outer + 16;
    int left = nprob;
    for (int64_t rep = 0; left > 0 && rep < max_replays; ++rep) {
        if (o.use_graph) {
            if (hipGraphLaunch(gexec, s) != hipSuccess) return fail(NBX_EHIP);
        } else {
            st = enqueue_batch32_iters(B, chunk, s);
            if (st != NBX_OK) return fail(st);
        }
        for (int p = 0; p < nprob; ++p)
            if (hipMemcpyAsync(h + p * NBX_SCAL_LEN, probs[p]->scal32,
                               sizeof(double) * NBX_SCAL_LEN, hipMemcpyDeviceToHost,
                               s) != hipSuccess)
                return fail(NBX_EHIP);
        if (hipStreamSynchronize(s) != hipSuccess) return fail(NBX_EHIP);
        for (int p = 0; p < nprob; ++p) {
            if (rs[p].done || h[p * NBX_SCAL_LEN + NBX_S_FLAG] == 0.0) continue;
            st = reliable_step(probs[p], b[p], x[p], o, h + p * NBX_SCAL_LEN, rs[p], s);
            if (st != NBX_OK) return fail(st);
            if (rs[p].done) {
                finished[p] =
                    std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                --left;
            }
        }
    }
    const double wall =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int worst = NBX_OK;
    for (int p = 0; p < nprob; ++p) {
        nbx_pcg_result &r = results[p];
        r = nbx_pcg_result{};
        st = reliable_finish(probs[p], b[p], x[p], o, rs[p], &r, s);
        if (st != NBX_OK) return fail(st);
        r.seconds = wall;
        if (solve_seconds) solve_seconds[p] = rs[p].done ? finished[p] : wall;
        if (r.flag == 2) worst = NBX_EBREAKDOWN;
        else if (r.flag != 1 && worst == NBX_OK) worst = NBX_NOT_CONVERGED;
    }
    if (hipEventRecord(ev, s) != hipSuccess || hipStreamWaitEvent(cs, ev, 0) != hipSuccess)
        return fail(NBX_EHIP);
    cleanup();
    return worst;
}

}  // namespace
}  // namespace nbx

using namespace nbx;

extern "C" int nbx_pcg_batched(nbx_problem *const *probs, const double *const *b,
                               double *const *x, int nprob, const nbx_pcg_opts *opts,
                               nbx_pcg_result *results, double *solve_seconds, void *stream)
{
    if (nprob < 0 || (nprob > 0 && (!probs || !b || !x || !results))) return NBX_EINVAL;
    if (nprob == 0) return NBX_OK;
    nbx_pcg_opts o;
    if (opts) o = *opts; else nbx_pcg_default_opts(&o);
    if (o.max_iter < 0 || !(o.rtol >= 0) || o.max_outer < 1) return NBX_EINVAL;
    for (int p = 0; p < nprob; ++p)
        if (!probs[p] || !b[p] || !x[p]) return NBX_EINVAL;
    if (o.inner_mfma) return NBX_EUNSUPPORTED;
    if (o.prec == NBX_F32 || o.prec == NBX_F16 || o.prec == NBX_BF16)
        return pcg_batched_mixed(probs, b, x, nprob, o, results, solve_seconds,
                                 as_stream(stream));
    if (o.prec != NBX_F64) return NBX_EUNSUPPORTED;

    BatchPlan B;
    B.nprob = nprob;
    std::vector<BDesc> hd(nprob);
    std::vector<BEntry> tv, tg, tm;
    for (int p = 0; p < nprob; ++p) {
        nbx_problem *P = probs[p];
        const GsPlan &g = P->gs->plan;
        BDesc &d = hd[p];
        d.G = P->G; d.D = P->D; d.dinv = P->dinv; d.b = b[p]; d.info = g.info;
        d.x = x[p]; d.r = P->r; d.z = P->z; d.p = P->p; d.w = P->w;
        d.part1 = P->part1; d.part3 = P->part3; d.scal = P->scal; d.stamp = nullptr;
        d.off = g.off; d.idx = g.idx; d.mask_idx = g.mask_idx; d.gflag = g.gflag;
        d.n_groups = g.n_groups; d.n_mask_only = g.n_mask_only;
        d.E = P->E; d.n = P->n; d.N = P->N;
        d.nb1 = ax_blocks(NBX_F64, P->N, P->E);
        d.nb3 = sk::red_blocks(P->n);
        d.pad = 0;
        for (int q = 0; q < d.nb3; ++q) tv.push_back({p, q});
        for (int q = 0; q < (g.n_groups + kGsThreads - 1) / kGsThreads; ++q) tg.push_back({p, q});
        for (int q = 0; q < (g.n_mask_only + 255) / 256; ++q) tm.push_back({p, q});
    }
    int st;
    if (hipMalloc(&B.stamps, sizeof(double) * nprob) != hipSuccess ||
        hipMalloc(&B.t0, sizeof(double)) != hipSuccess)
        return NBX_ENOMEM;
    NBX_HIP(hipMemset(B.stamps, 0, sizeof(double) * nprob));
    for (int p = 0; p < nprob; ++p) hd[p].stamp = B.stamps + p;
    if ((st = upload(&B.desc, hd)) != NBX_OK) return st;
    if ((st = upload(&B.t_vec, tv)) != NBX_OK) return st;
    if ((st = upload(&B.t_gs, tg)) != NBX_OK) return st;
    if ((st = upload(&B.t_mask, tm)) != NBX_OK) return st;
    B.n_vec = (int)tv.size(); B.n_gs = (int)tg.size(); B.n_mask = (int)tm.size();
    // one AX table per polynomial size present, with that size's tile
    std::vector<int> Ns;
    for (int p = 0; p < nprob; ++p) Ns.push_back(probs[p]->N);
    std::sort(Ns.begin(), Ns.end());
    Ns.erase(std::unique(Ns.begin(), Ns.end()), Ns.end());
    for (int N : Ns) {
        std::vector<BEntry> ta;
        for (int p = 0; p < nprob; ++p)
            if (probs[p]->N == N)
                for (int q = 0; q < hd[p].nb1; ++q) ta.push_back({p, q});
        BatchPlan::AxClass c{N, pcg_tile(NBX_F64, N), (int)ta.size(), nullptr};
        if ((st = upload(&c.tab, ta)) != NBX_OK) return st;
        B.ax.push_back(c);
    }

    hipStream_t cs = as_stream(stream);
    hipStream_t s = nullptr;
    NBX_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipEvent_t ev = nullptr;
    NBX_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    double *h = nullptr;
    NBX_HIP(hipHostMalloc(&h, sizeof(double) * NBX_SCAL_LEN * nprob, hipHostMallocDefault));
    hipGraphExec_t gexec = nullptr;
    auto cleanup = [&]() {
        if (gexec) hipGraphExecDestroy(gexec);
        if (s) { hipStreamSynchronize(s); hipStreamDestroy(s); }
        if (ev) hipEventDestroy(ev);
        if (h) hipHostFree(h);
    };
    auto fail = [&](int code) { cleanup(); return code; };

    if (hipEventRecord(ev, cs) != hipSuccess || hipStreamWaitEvent(s, ev, 0) != hipSuccess)
        return fail(NBX_EHIP);
    const int chunk = o.check_every > 0 ? o.check_every : 10;
    if (o.use_graph) {
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(NBX_EHIP);
        st = enqueue_batch_iters(B, chunk, s);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        if (st != NBX_OK) { if (g) hipGraphDestroy(g); return fail(st); }
        if (e != hipSuccess) return fail(hip_fail(e, "hipStreamEndCapture"));
        e = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) { gexec = nullptr; return fail(hip_fail(e, "hipGraphInstantiate")); }
    }
    int dev = 0, rate_khz = 0;
    NBX_HIP(hipGetDevice(&dev));
    NBX_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));

    const auto t0 = std::chrono::steady_clock::now();
    hipLaunchKernelGGL(b_init_kernel, dim3(B.n_vec), dim3(sk::kRedThreads), 0, s, B.desc, B.t_vec);
    hipLaunchKernelGGL(b_init_reduce_kernel, dim3(nprob), dim3(1024), 0, s, B.desc, o.rtol,
                       o.fixed_iters, o.max_iter);
    hipLaunchKernelGGL(b_clock_kernel, dim3(1), dim3(1), 0, s, B.t0);
    if (hipGetLastError() != hipSuccess) return fail(NBX_EHIP);
    int done = 0;
    std::vector<double> host_scal(NBX_SCAL_LEN);
    while (true) {
        if (o.use_graph) {
            if (hipGraphLaunch(gexec, s) != hipSuccess) return fail(NBX_EHIP);
        } else {
            st = enqueue_batch_iters(B, chunk, s);
            if (st != NBX_OK) return fail(st);
        }
        done += chunk;
        bool all = true;
        for (int p = 0; p < nprob; ++p)
            if (hipMemcpyAsync(h + p * NBX_SCAL_LEN, probs[p]->scal, sizeof(double) * NBX_SCAL_LEN,
                               hipMemcpyDeviceToHost, s) != hipSuccess)
                return fail(NBX_EHIP);
        if (hipStreamSynchronize(s) != hipSuccess) return fail(NBX_EHIP);
        for (int p = 0; p < nprob; ++p)
            if (h[p * NBX_SCAL_LEN + NBX_S_FLAG] == 0.0) { all = false; break; }
        if (all || done >= o.max_iter + chunk) break;
    }
    const auto t1 = std::chrono::steady_clock::now();
    const double wall = std::chrono::duration<double>(t1 - t0).count();
    std::vector<double> stamps(nprob);
    double t0d = 0.0;
    if (hipMemcpy(stamps.data(), B.stamps, sizeof(double) * nprob, hipMemcpyDeviceToHost) !=
            hipSuccess ||
        hipMemcpy(&t0d, B.t0, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(NBX_EHIP);
    int worst = NBX_OK;
    for (int p = 0; p < nprob; ++p) {
        const double *hs = h + p * NBX_SCAL_LEN;
        nbx_pcg_result &r = results[p];
        r = nbx_pcg_result{};
        r.iters = (int)hs[NBX_S_ITER];
        r.outer_iters = 1;
        r.relres = hs[NBX_S_BB] > 0 ? std::sqrt(hs[NBX_S_RR] / hs[NBX_S_BB]) : 0.0;
        const double fl = hs[NBX_S_FLAG];
        r.flag = fl == 1.0 ? 1 : (fl == 2.0 ? 2 : 0);
        r.seconds = wall;
        double rb[2];
        st = residual_f64(probs[p], b[p], x[p], nullptr, rb, s);
        if (st != NBX_OK) return fail(st);
        r.true_relres = rb[1] > 0 ? std::sqrt(rb[0] / rb[1]) : 0.0;
        if (solve_seconds)
            solve_seconds[p] = rate_khz > 0 && stamps[p] > t0d
                                   ? (stamps[p] - t0d) / (rate_khz * 1e3) : 0.0;
        if (r.flag == 2) worst = NBX_EBREAKDOWN;
        else if (r.flag != 1 && worst == NBX_OK) worst = NBX_NOT_CONVERGED;
    }
    if (hipEventRecord(ev, s) != hipSuccess || hipStreamWaitEvent(cs, ev, 0) != hipSuccess)
        return fail(NBX_EHIP);
    cleanup();
    return worst;
}
