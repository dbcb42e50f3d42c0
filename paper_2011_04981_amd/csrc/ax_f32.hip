// ax_f32.hip -- FP32 instantiations of the AX kernel (see ax_kernel.hpp).
#include "ax_kernel.hpp"

namespace nbx {

int ax_launch_f32_tiled(int N, int epb, const float *u, const float *G, const double *D,
                        float *w, int64_t E, hipStream_t s)
{
    return ax_launch_any<float, false>(N, epb, u, G, D, w, nullptr, nullptr, nullptr, E, s);
}

}  // namespace nbx
