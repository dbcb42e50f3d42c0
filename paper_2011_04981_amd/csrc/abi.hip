// abi.hip -- status codes, error capture and version of the C ABI.
#include "internal.hpp"

namespace nbx {

static thread_local int g_last_hip_error = 0;

int hip_fail(hipError_t e, const char *what)
{
    g_last_hip_error = (int)e;
    (void)what;
    return NBX_EHIP;
}

}  // namespace nbx

extern "C" const char *nbx_status_str(int st)
{
    switch (st) {
        case NBX_OK: return "ok";
        case NBX_NOT_CONVERGED: return "not converged (iteration limit)";
        case NBX_EINVAL: return "invalid argument";
        case NBX_EUNSUPPORTED: return "unsupported configuration";
        case NBX_EHIP: return "HIP runtime error";
        case NBX_ENOMEM: return "out of device memory";
        case NBX_EBREAKDOWN: return "CG breakdown";
        default: return "unknown status";
    }
}

extern "C" int nbx_last_hip_error(void) { return nbx::g_last_hip_error; }

extern "C" int nbx_version(void) { return 100; }

namespace {

typedef double dbl2 __attribute__((ext_vector_type(2)));

// One 16-byte element per thread, non-temporal store (the fastest plain
// copy measured on MI355X: ~6.4 TB/s for 0.8 GB each way).
__global__ void __launch_bounds__(256)
copy_kernel(const dbl2 *__restrict__ src, dbl2 *__restrict__ dst, int64_t n2)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n2) __builtin_nontemporal_store(src[q], dst + q);
}

__global__ void copy_tail_kernel(const double *__restrict__ src, double *__restrict__ dst,
                                 int64_t n)
{
    if (threadIdx.x == 0 && (n & 1)) dst[n - 1] = src[n - 1];
}

// Bandwidth references: a copy with non-temporal loads and stores, and a
// read-only stream (the loads feed a sum that is written only if it equals
// an impossible value, so nothing is stored and nothing is optimised away).
__global__ void __launch_bounds__(256)
copy_nt_kernel(const dbl2 *__restrict__ src, dbl2 *__restrict__ dst, int64_t n2)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n2) __builtin_nontemporal_store(__builtin_nontemporal_load(src + q), dst + q);
}

__global__ void __launch_bounds__(256)
read_kernel(const dbl2 *__restrict__ src, int64_t n2, double *__restrict__ sink)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n2) {
        const dbl2 v = __builtin_nontemporal_load(src + q);
        if (v.x + v.y == -1.2345e300) sink[0] = v.x;
    }
}

}  // namespace

extern "C" int nbx_stream_f64(int mode, const double *src, double *dst, int64_t n,
                              double *sink, void *stream)
{
    if (n < 0 || (mode != 0 && mode != 1)) return NBX_EINVAL;
    if (n == 0) return NBX_OK;
    if (!src || (mode == 0 && !dst) || (mode == 1 && !sink)) return NBX_EINVAL;
    if (n & 1) return NBX_EINVAL;
    const int64_t n2 = n >> 1;
    const int64_t blocks = (n2 + 255) / 256;
    if (blocks > 0x7fffffffLL) return NBX_EUNSUPPORTED;
    hipStream_t s = nbx::as_stream(stream);
    if (mode == 0)
        hipLaunchKernelGGL(copy_nt_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                           reinterpret_cast<const dbl2 *>(src), reinterpret_cast<dbl2 *>(dst), n2);
    else
        hipLaunchKernelGGL(read_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                           reinterpret_cast<const dbl2 *>(src), n2, sink);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

extern "C" int nbx_copy_f64(const double *src, double *dst, int64_t n, void *stream)
{
    if (n < 0 || (n > 0 && (!src || !dst))) return NBX_EINVAL;
    if (n == 0) return NBX_OK;
    hipStream_t s = nbx::as_stream(stream);
    const int64_t n2 = n >> 1;
    if (n2 > 0) {
        const int64_t blocks = (n2 + 255) / 256;
        if (blocks > 0x7fffffffLL) return NBX_EUNSUPPORTED;
        hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                           reinterpret_cast<const dbl2 *>(src), reinterpret_cast<dbl2 *>(dst),
                           n2);
    }
    if (n & 1) hipLaunchKernelGGL(copy_tail_kernel, dim3(1), dim3(64), 0, s, src, dst, n);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}
