// ax_planes.hip -- instantiations of the AX kernel (see ax_kernel.hpp) on
// geometric factors in the C ABI's layout, one plane per factor
// ([E][6][N^3]): FP64 and FP32.
#include "ax_kernel.hpp"

namespace nbx {

int ax_launch_f64_planes_tiled(int N, int epb, const double *u, const double *G,
                               const double *D, double *w, int64_t E, hipStream_t s)
{
    return ax_launch_any<double, false, double, true>(N, epb, u, G, D, w, nullptr, nullptr,
                                                      nullptr, E, s);
}

int ax_launch_f32_planes_tiled(int N, int epb, const float *u, const float *G, const double *D,
                               float *w, int64_t E, hipStream_t s)
{
    return ax_launch_any<float, false, float, true>(N, epb, u, G, D, w, nullptr, nullptr,
                                                    nullptr, E, s);
}

}  // namespace nbx
