// ax_pcg.hip -- the fused first stage of a CG iteration, p = z + beta p and
// w = AX(p) with per-block partials of p.w, in FP64 and FP32 (see
// ax_kernel.hpp).
#include "ax_kernel.hpp"

namespace nbx {

int ax_pcg_launch_f64_tiled(int N, int epb, const double *G, const double *D, int64_t E,
                            const double *z, double *p, double *w, double *part,
                            const double *scal, hipStream_t s)
{
    return ax_launch_any<double, true>(N, epb, z, G, D, w, p, part, scal, E, s);
}

int ax_pcg_launch_f32_tiled(int N, int epb, const float *G, const double *D, int64_t E,
                            const float *z, float *p, float *w, double *part,
                            const double *scal, hipStream_t s)
{
    return ax_launch_any<float, true>(N, epb, z, G, D, w, p, part, scal, E, s);
}

}  // namespace nbx
