// mixed.hip -- FP32 inner PCG inside FP64 iterative refinement.
#include "internal.hpp"

struct nbx_problem;

namespace nbx {

int pcg_mixed(nbx_problem *, const double *, double *, const nbx_pcg_opts &, nbx_pcg_result *)
{
    return NBX_EUNSUPPORTED;
}

}  // namespace nbx
