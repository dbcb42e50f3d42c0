// gs.hip -- direct stiffness summation (dssum) and the Dirichlet mask.
//
// The paper's CG iteration includes a nearest-neighbour exchange (Section
// II-B) that makes the element-local copies of every shared node agree; on
// one GPU that is this gather-scatter.  The plan lists only nodes with
// more than one copy (a brick at N = 10 shares under half of its local
// nodes), grouped by global node with local indices ascending, so every
// group sums in a fixed order and writes identical bits to all copies:
// no atomics, deterministic, and bit-identical to a sequential sum in
// ascending local order.
#include "gs_kernels.hpp"
#include "solver_kernels.hpp"

#include <algorithm>
#include <numeric>
#include <vector>

namespace nbx {
namespace {

// Threads [0, n_groups) sum one shared group each; with apply_mask the
// threads after them zero the unshared Dirichlet nodes (one launch for
// both steps).
// With pap_part, the last workgroup performs the alpha step (PapTask) and
// the others the exchange.
template <typename T>
__global__ void __launch_bounds__(kGsThreads)
dssum_kernel(int32_t n_groups, const int32_t *__restrict__ off, const int32_t *__restrict__ idx,
             const uint8_t *__restrict__ gflag, T *__restrict__ v, int apply_mask,
             int32_t n_mask, const int32_t *__restrict__ mask_idx,
             const double *__restrict__ flag, int pap_nb, const double *__restrict__ pap_part,
             double *__restrict__ pap_scal)
{
    unsigned nblk = gridDim.x;
    if (pap_part) {
        if (blockIdx.x == gridDim.x - 1) {
            sk::pap_reduce_body(pap_nb, pap_part, pap_scal);
            return;
        }
        --nblk;
    }
    if (flag && *flag != 0.0) return;   // uniform: solve already finished
    // XCD-aware mapping: workgroups are dealt to the 8 XCDs round-robin, so
    // give each XCD a contiguous range of groups (neighbouring groups share
    // cache lines; each XCD has its own L2)
    const int32_t per = (int32_t)(nblk / 8);
    const int32_t vb = (int32_t)(blockIdx.x % 8) * per + (int32_t)(blockIdx.x / 8);
    const int32_t g = vb * blockDim.x + threadIdx.x;
    if (g < n_groups) {
        dssum_group<T>(g, off, idx, gflag, v, apply_mask);
    } else if (apply_mask && g - n_groups < n_mask) {
        v[mask_idx[g - n_groups]] = 0;
    }
}

__global__ void multiplicity_kernel(int64_t n, const uint8_t *__restrict__ info,
                                    double *__restrict__ out)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l < n) out[l] = (double)(info[l] & 0x7f);
}

// Device copy of h (the copy is issued on s; the caller synchronises s
// before h goes out of scope).
template <typename T>
void *dev_upload(const std::vector<T> &h, int &st, hipStream_t s = nullptr)
{
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(h.size(), 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) { st = NBX_ENOMEM; return nullptr; }
    if (!h.empty()) {
        e = hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) { st = hip_fail(e, "hipMemcpyAsync"); hipFree(p); return nullptr; }
    }
    return p;
}

template <typename T>
int dev_download(const T *d, size_t count, std::vector<T> &h)
{
    h.resize(count);
    if (count == 0) return NBX_OK;
    NBX_HIP(hipMemcpy(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost));
    return NBX_OK;
}

}  // namespace

void free_plan(GsPlan &p)
{
    hipFree(p.off); hipFree(p.idx); hipFree(p.gflag); hipFree(p.mask_idx); hipFree(p.info);
    p = GsPlan{};
}

int xpair_plan(const GsPlan &full, int N, GsPlan &out, int *found)
{
    *found = 0;
    out = GsPlan{};
    if (N < 2 || full.n_groups == 0) return NBX_OK;
    const int64_t xd = xpair_offset(N);
    std::vector<int32_t> off, idx, mask_idx;
    std::vector<uint8_t> gflag, info;
    int st = dev_download(full.off, (size_t)full.n_groups + 1, off);
    if (st == NBX_OK) st = dev_download(full.idx, (size_t)off.back(), idx);
    if (st == NBX_OK) st = dev_download(full.gflag, (size_t)full.n_groups, gflag);
    if (st == NBX_OK) st = dev_download(full.mask_idx, (size_t)full.n_mask_only, mask_idx);
    if (st == NBX_OK) st = dev_download(full.info, (size_t)full.n_local, info);
    if (st != NBX_OK) return st;
    for (uint8_t v : info)
        if ((v & 0x7f) > kXpMult) return NBX_OK;   // the bits are needed for multiplicity
    std::vector<int32_t> roff{0}, ridx;
    std::vector<uint8_t> rflag;
    int64_t pairs = 0;
    for (int32_t g = 0; g < full.n_groups; ++g) {
        const int32_t b = off[g], e = off[g + 1];
        if (e - b == 2 && !gflag[g] && (int64_t)idx[b + 1] - idx[b] == xd &&
            idx[b] % N == N - 1) {
            info[idx[b]] = (uint8_t)((info[idx[b]] & kXpMult) | kXpNext);
            info[idx[b + 1]] = (uint8_t)((info[idx[b + 1]] & kXpMult) | kXpPrev);
            ++pairs;
            continue;
        }
        ridx.insert(ridx.end(), idx.begin() + b, idx.begin() + e);
        roff.push_back((int32_t)ridx.size());
        rflag.push_back(gflag[g]);
    }
    if (pairs == 0) return NBX_OK;
    out.n_local = full.n_local;
    out.n_groups = (int32_t)rflag.size();
    out.n_mask_only = full.n_mask_only;
    out.off = (int32_t *)dev_upload(roff, st);
    if (st == NBX_OK) out.idx = (int32_t *)dev_upload(ridx, st);
    if (st == NBX_OK) out.gflag = (uint8_t *)dev_upload(rflag, st);
    if (st == NBX_OK) out.mask_idx = (int32_t *)dev_upload(mask_idx, st);
    if (st == NBX_OK) out.info = (uint8_t *)dev_upload(info, st);
    const hipError_t e = hipStreamSynchronize(nullptr);   // the host vectors die here
    if (st == NBX_OK && e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    if (st != NBX_OK) { free_plan(out); return st; }
    *found = 1;
    return NBX_OK;
}

template <typename T>
int dssum_launch(const GsPlan &gs, T *v, int apply_mask, hipStream_t s, const double *flag,
                 const PapTask *pap)
{
    const int64_t nt = (int64_t)gs.n_groups + (apply_mask ? gs.n_mask_only : 0);
    if (nt > 0 || pap) {
        const int64_t nb = ((nt + kGsThreads - 1) / kGsThreads + 7) / 8 * 8;   // 8 XCDs
        hipLaunchKernelGGL(dssum_kernel<T>, dim3((unsigned)(nb + (pap ? 1 : 0))),
                           dim3(kGsThreads), 0, s, gs.n_groups, gs.off, gs.idx, gs.gflag, v,
                           apply_mask, gs.n_mask_only, gs.mask_idx, flag, pap ? pap->nb : 0,
                           pap ? pap->part : nullptr, pap ? pap->scal : nullptr);
        NBX_LAUNCH_CHECK();
    }
    return NBX_OK;
}

template int dssum_launch<double>(const GsPlan &, double *, int, hipStream_t, const double *,
                                  const PapTask *);
template int dssum_launch<float>(const GsPlan &, float *, int, hipStream_t, const double *,
                                 const PapTask *);

}  // namespace nbx

using namespace nbx;

extern "C" int nbx_gs_create(const int64_t *gid_host, int64_t n_local,
                             const uint8_t *bnd_host, nbx_gs **out, void *stream)
{
    if (!out || n_local < 0 || (n_local > 0 && !gid_host)) return NBX_EINVAL;
    *out = nullptr;
    if (n_local >= 0x7fffffffLL) return NBX_EUNSUPPORTED;
    const int32_t n = (int32_t)n_local;
    // order local nodes by (global id, local index)
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return gid_host[a] < gid_host[b]; });
    std::vector<int32_t> off{0}, idx, mask_idx;
    std::vector<uint8_t> gflag, info(n, 0);
    for (int32_t q = 0; q < n;) {
        int32_t r = q;
        uint8_t bnd = 0;
        while (r < n && gid_host[order[r]] == gid_host[order[q]]) {
            if (bnd_host && bnd_host[order[r]]) bnd = 1;
            ++r;
        }
        const int32_t m = r - q;
        if (m > 127) return NBX_EUNSUPPORTED;
        for (int32_t t = q; t < r; ++t) info[order[t]] = (uint8_t)(m | (bnd ? 0x80 : 0));
        if (m >= 2) {
            for (int32_t t = q; t < r; ++t) idx.push_back(order[t]);
            off.push_back((int32_t)idx.size());
            gflag.push_back(bnd);
        } else if (bnd) {
            mask_idx.push_back(order[q]);
        }
        q = r;
    }
    nbx_gs *gs = new (std::nothrow) nbx_gs;
    if (!gs) return NBX_ENOMEM;
    GsPlan &p = gs->plan;
    p.n_local = n_local;
    p.n_groups = (int32_t)gflag.size();
    p.n_mask_only = (int32_t)mask_idx.size();
    int st = NBX_OK;
    hipStream_t s = as_stream(stream);
    p.off = (int32_t *)dev_upload(off, st, s);
    if (st == NBX_OK) p.idx = (int32_t *)dev_upload(idx, st, s);
    if (st == NBX_OK) p.gflag = (uint8_t *)dev_upload(gflag, st, s);
    if (st == NBX_OK) p.mask_idx = (int32_t *)dev_upload(mask_idx, st, s);
    if (st == NBX_OK) p.info = (uint8_t *)dev_upload(info, st, s);
    const hipError_t e = hipStreamSynchronize(s);   // the host vectors die here
    if (st == NBX_OK && e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    if (st != NBX_OK) { free_plan(p); delete gs; return st; }
    *out = gs;
    return NBX_OK;
}

extern "C" int nbx_gs_destroy(nbx_gs *gs)
{
    if (!gs) return NBX_OK;
    free_plan(gs->plan);
    delete gs;
    return NBX_OK;
}

extern "C" int nbx_dssum(nbx_gs *gs, int prec, void *v, int apply_mask, void *stream)
{
    if (!gs || (!v && gs->plan.n_local > 0)) return NBX_EINVAL;
    hipStream_t s = as_stream(stream);
    switch (prec) {
        case NBX_F64: return dssum_launch<double>(gs->plan, (double *)v, apply_mask, s);
        case NBX_F32: return dssum_launch<float>(gs->plan, (float *)v, apply_mask, s);
        default: return NBX_EUNSUPPORTED;
    }
}

extern "C" int nbx_gs_multiplicity(nbx_gs *gs, double *out, void *stream)
{
    if (!gs || (!out && gs->plan.n_local > 0)) return NBX_EINVAL;
    const int64_t n = gs->plan.n_local;
    if (n == 0) return NBX_OK;
    hipLaunchKernelGGL(multiplicity_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       as_stream(stream), n, gs->plan.info, out);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}
