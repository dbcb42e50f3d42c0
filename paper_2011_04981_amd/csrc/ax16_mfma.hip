// ax16_mfma.hip -- kernels and launchers of the FP64 operator at N = 16 on
// the matrix cores (the body and its design: ax16_mfma.hpp): the plain
// operator on factor planes or pairs, and the solvers' fused first stage on
// factor pairs.
#include "ax16_mfma.hpp"

namespace nbx {
namespace {

// Three workgroups per CU on factor planes (148 VGPRs); on factor pairs the
// compiler needs more registers (34 spilled at the three-workgroup bound), so
// that layout runs two per CU, as does the fused stage (p stays live for the
// <p, w> partial).
template <bool PL, bool PCG>
__global__ void __launch_bounds__(256, (PL && !PCG) ? 3 : 2)
ax16_mfma_kernel(const double *__restrict__ u, const double *__restrict__ G,
                 const double *__restrict__ D, double *__restrict__ w, double *__restrict__ p,
                 double *__restrict__ part, const double *__restrict__ scal)
{
    ax16::body<PL, PCG>(u, G, D, w, p, part, scal, (int64_t)blockIdx.x);
}

}  // namespace

// Plain operator at N = 16 on FP64 factors, one plane per factor
// ([E][6][4096], planes != 0) or factor pairs ([E][3][4096][2]); one
// workgroup per element.  Both layouts give the same bits.
int ax16_mfma_launch(int planes, const double *u, const double *G, const double *D, double *w,
                     int64_t E, hipStream_t s)
{
    if (E <= 0) return NBX_OK;
    if (E > 0x7fffffffLL) return NBX_EUNSUPPORTED;
    if (planes)
        hipLaunchKernelGGL((ax16_mfma_kernel<true, false>), dim3((unsigned)E), dim3(256), 0, s,
                           u, G, D, w, nullptr, nullptr, nullptr);
    else
        hipLaunchKernelGGL((ax16_mfma_kernel<false, false>), dim3((unsigned)E), dim3(256), 0, s,
                           u, G, D, w, nullptr, nullptr, nullptr);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

// The solvers' fused first stage at N = 16 on factor pairs: p = z + beta p,
// w = AX(p), part[e] = <p, w> over element e (E partials).
int ax16_mfma_pcg_launch(const double *Gp, const double *D, int64_t E, const double *z,
                         double *p, double *w, double *part, const double *scal, hipStream_t s)
{
    if (E <= 0) return NBX_OK;
    if (E > 0x7fffffffLL) return NBX_EUNSUPPORTED;
    hipLaunchKernelGGL((ax16_mfma_kernel<false, true>), dim3((unsigned)E), dim3(256), 0, s, z,
                       Gp, D, w, p, part, scal);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

}  // namespace nbx
