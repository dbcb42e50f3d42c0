// ax_bf16.hip -- AX with geometric factors stored in 16 bits (g_bf16 words,
// per-element power-of-two scale), FP32 arithmetic: plain and fused-PCG
// instantiations (see ax_kernel.hpp).
#include "ax_kernel.hpp"

namespace nbx {

int ax_launch_g_bf16(int N, int epb, const float *u, const void *G, const float *gscale,
                    const double *D, float *w, int64_t E, hipStream_t s)
{
    return ax_launch_any<float, false, g_bf16>(N, epb, u, (const g_bf16 *)G, D, w, nullptr, nullptr,
                                             nullptr, E, s, gscale);
}

int ax_pcg_launch_g_bf16(int N, int epb, const void *G, const float *gscale, const double *D,
                        int64_t E, const float *z, float *p, float *w, double *part,
                        const double *scal, hipStream_t s)
{
    return ax_launch_any<float, true, g_bf16>(N, epb, z, (const g_bf16 *)G, D, w, p, part, scal, E,
                                            s, gscale);
}

}  // namespace nbx
