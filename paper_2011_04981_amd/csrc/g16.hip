// g16.hip -- 16-bit storage of the geometric factors for the reduced-
// precision inner operator.
//
// The paper keeps G in double and names half precision and fixed point as
// further work (Section V); G is 48 of AX's 64 bytes per node, so halving
// its width is the largest bandwidth lever after FP32.  Per element e the
// factors are divided by a power of two, gscale[e] = 2^(floor(log2 m) - 14)
// with m = max |G_e|, which puts the largest into [2^14, 2^15): FP16 then
// never overflows and its subnormal range only holds factors below 2^-24 m.
// Each value is rounded to nearest-even twice, FP64 -> FP32 -> 16 bits
// (IEEE binary16 or bfloat16).  AX multiplies the element's FP32 result by
// gscale[e]; a power-of-two scale is exact, so this equals AX with the
// dequantised factors.  Storage: per element three planes of 32-bit words,
// plane h holding factors 2h and 2h+1 of each node in its low and high half
// ([E][3][N^3][2] 16-bit words), so that AX fetches a node's six factors
// with three 4-byte loads instead of six 2-byte ones.
#include "internal.hpp"

#include <cmath>

namespace nbx {
namespace {

__device__ inline uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline uint16_t to16(int bf16, double v)
{
    const float f = (float)v;
    return bf16 ? f32_to_bf16_rne(f) : __builtin_bit_cast(uint16_t, (_Float16)f);
}

// one block per element: max |G_e|, the scale, then the packed words.
// G is [E][6][N^3] (planes != 0, the C ABI's layout) or factor pairs.
__global__ void __launch_bounds__(256)
g16_pack_kernel(int bf16, int planes, int N3, const double *__restrict__ G,
                uint32_t *__restrict__ G16, float *__restrict__ gscale)
{
    const int n6 = 6 * N3;
    __shared__ double s_max[4];
    const int64_t e = blockIdx.x;
    const double *Ge = G + (size_t)e * n6;
    double m = 0.0;
    for (int q = threadIdx.x; q < n6; q += blockDim.x) m = fmax(m, fabs(Ge[q]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = m;
    __syncthreads();
    m = fmax(fmax(s_max[0], s_max[1]), fmax(s_max[2], s_max[3]));
    int ex = 0;
    if (m > 0.0 && isfinite(m)) { frexp(m, &ex); ex -= 15; }   // m = f 2^ex', f in [0.5,1)
    const double inv = ldexp(1.0, -ex);
    if (threadIdx.x == 0) gscale[e] = ldexpf(1.0f, ex);
    uint32_t *out = G16 + (size_t)e * 3 * N3;
    for (int q = threadIdx.x; q < 3 * N3; q += blockDim.x) {
        // word q = h N^3 + node holds factors 2h (low half) and 2h + 1
        const int h = q / N3, node = q - h * N3;
        const double glo = planes ? Ge[(2 * h) * N3 + node] : Ge[2 * q];
        const double ghi = planes ? Ge[(2 * h + 1) * N3 + node] : Ge[2 * q + 1];
        const uint32_t lo = to16(bf16, glo * inv);
        const uint32_t hi = to16(bf16, ghi * inv);
        out[q] = lo | (hi << 16);
    }
}

}  // namespace

int g16_pack_launch(int gprec, int planes, const double *G, int N, int64_t E, void *G16,
                    float *gscale, hipStream_t s)
{
    if (N < 2 || N > kMaxN || E < 0) return NBX_EINVAL;
    if (gprec != NBX_F16 && gprec != NBX_BF16) return NBX_EUNSUPPORTED;
    if (E == 0) return NBX_OK;
    if (!G || !G16 || !gscale) return NBX_EINVAL;
    if (E > 0x7fffffffLL) return NBX_EUNSUPPORTED;
    hipLaunchKernelGGL(g16_pack_kernel, dim3((unsigned)E), dim3(256), 0, s,
                       gprec == NBX_BF16 ? 1 : 0, planes, N * N * N, G, (uint32_t *)G16, gscale);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

}  // namespace nbx

using namespace nbx;

extern "C" int nbx_g16_pack(int gprec, const double *G, int N, int64_t E, void *G16,
                            float *gscale, void *stream)
{
    return g16_pack_launch(gprec, 1, G, N, E, G16, gscale, as_stream(stream));
}

extern "C" int nbx_ax_g16(int gprec, const float *u, const void *G16, const float *gscale,
                          const double *D, int N, int64_t E, float *w, void *stream)
{
    if (N < 2 || N > kMaxN || E < 0) return NBX_EINVAL;
    if (gprec != NBX_F16 && gprec != NBX_BF16) return NBX_EUNSUPPORTED;
    if (E == 0) return NBX_OK;
    if (!u || !G16 || !gscale || !D || !w || u == w) return NBX_EINVAL;
    return ax_launch_g16(gprec, u, G16, gscale, D, N, E, w, as_stream(stream));
}
