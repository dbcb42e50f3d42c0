// ax_f64.hip -- FP64 instantiations of the AX kernel (see ax_kernel.hpp).
#include "ax_kernel.hpp"

namespace nbx {

int ax_launch_f64_tiled(int N, int epb, const double *u, const double *G, const double *D,
                        double *w, int64_t E, hipStream_t s)
{
    return ax_launch_any<double, false>(N, epb, u, G, D, w, nullptr, nullptr, nullptr, E, s);
}

}  // namespace nbx
