// lpi.hip -- the model of the learned element-interior preconditioner and
// its training step (the learned part is not in the paper).
//
// Per element e, on the interior nodes S that have one copy and are off
// the Dirichlet set (nI = (N-2)^3 of them at most):
//     z_S = (1/gd_e) L^T diag(gamma_e) L r_S,   gamma_e = softplus(f(g_e)),
// L a shared nI x nI matrix and f a 3-layer perceptron (mlp.hip) on the six
// element-mean geometric factors over gd_e (the mean of the diagonal
// factors).  L^T diag(gamma) L is symmetric positive semidefinite whatever
// L and gamma > 0 are, so the preconditioner stays SPD by construction.
//
// Storage: L as [nIp][nIp] FP32 master weights (zero beyond nI; nIp = nI
// rounded up to 64) with a BF16 copy for the matrix-core products; the
// perceptron's arena as in mlp.hip (6 inputs padded to 64, n_hid hidden,
// nI outputs padded to nIp).  The parameter arena of nbx_lpi_set_params /
// get_params is [L | perceptron].
//
// Training rows (B of them): X [B][nIp] BF16, T [B][nIp] FP32, F [B][64]
// BF16; loss = mean over rows and the nI outputs of (Z - T)^2 with
// Z = ((X L^T) * gamma) L.  Gradient by the chain rule:
//   Hx = X L^T, Q = Hx * gamma, Z = Q L, dZ = 2 (Z - T) / (B nI),
//   Pm = dZ L^T, dL = Q^T dZ + (gamma * Pm)^T X,
//   dA = Hx * Pm * sigmoid(A) (A the perceptron's output), then the
//   perceptron's own backward pass.
// Every product is the BF16 GEMM of mlp.hip (FP32 accumulation).
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <new>

struct nbx_mlp;
extern "C" int nbx_mlp_create(int n_in, int n_hidden, int n_out, int max_batch, nbx_mlp **out);
extern "C" int nbx_mlp_destroy(nbx_mlp *P);

namespace nbx {

int gemm_bf16(int ta, int tb, int epi, int M, int N, int K, const uint16_t *A, int lda,
              const uint16_t *B, int ldb, float *C, int ldc, uint16_t *Cb, int ldcb,
              const float *bias, const uint16_t *act, int ldact, hipStream_t s,
              const float *mul);
int mse_grad(int B, int n_pad, int n_out, const float *Y, const float *T, float *dY,
             uint16_t *dYb, double *part, double *loss, hipStream_t s);
int adam_update(int64_t n, float *w, uint16_t *wb, float *m, float *v, const float *g, float lr,
                int step, hipStream_t s);
int to_bf16(int64_t n, const float *a, uint16_t *b, hipStream_t s);
int mlp_forward_rows(nbx_mlp *P, const uint16_t *X, int B, float *Y, hipStream_t s);
int mlp_grad_buffers(nbx_mlp *P, float **dY, uint16_t **dYb);
int mlp_backprop_rows(nbx_mlp *P, const uint16_t *X, int B, hipStream_t s);
int mlp_adam(nbx_mlp *P, float lr, hipStream_t s);
int64_t mlp_nparams(nbx_mlp *P);
int64_t mlp_last_bias(nbx_mlp *P, int *n);
int mlp_set_params(nbx_mlp *P, const float *params, hipStream_t s);
float *mlp_weights(nbx_mlp *P);
float *mlp_grads(nbx_mlp *P);

namespace {

// GEMM epilogue ids of mlp.hip
constexpr int kEpiF32 = 0, kEpiAcc = 4;
constexpr int kLossParts = 1024;

__device__ __forceinline__ uint16_t lpi_f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float lpi_softplus(float a)
{
    return log1pf(expf(-fabsf(a))) + fmaxf(a, 0.f);
}

__device__ __forceinline__ float lpi_sigmoid(float a) { return 1.f / (1.f + expf(-a)); }

unsigned lpi_grid(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    return (unsigned)(b < 1 ? 1 : b);
}

// Qb = bf16(Hx * softplus(A))
__global__ void lpi_q_kernel(int64_t n, const float *__restrict__ Hx, const float *__restrict__ A,
                             uint16_t *__restrict__ Qb)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        Qb[q] = lpi_f2bf(Hx[q] * lpi_softplus(A[q]));
}

// dA = Hx * Pm * sigmoid(A) (FP32 and BF16, the perceptron's output
// gradient); G2b = bf16(softplus(A) * Pm)
__global__ void lpi_back_kernel(int64_t n, const float *__restrict__ Hx,
                                const float *__restrict__ Pm, const float *__restrict__ A,
                                float *__restrict__ dA, uint16_t *__restrict__ dAb,
                                uint16_t *__restrict__ G2b)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const float a = A[q], pm = Pm[q];
        const float d = Hx[q] * pm * lpi_sigmoid(a);
        dA[q] = d;
        dAb[q] = lpi_f2bf(d);
        G2b[q] = lpi_f2bf(lpi_softplus(a) * pm);
    }
}

// partials of <X, T> and <X, X> over n entries (X BF16, T FP32)
__global__ void __launch_bounds__(256)
lpi_xt_kernel(int64_t n, const uint16_t *__restrict__ X, const float *__restrict__ T,
              double *__restrict__ part)
{
    __shared__ double s[2][4];
    double xt = 0.0, xx = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const double x = (double)__uint_as_float((uint32_t)X[q] << 16);
        xt += x * (double)T[q];
        xx += x * x;
    }
    for (int off = 32; off > 0; off >>= 1) {
        xt += __shfl_down(xt, off, 64);
        xx += __shfl_down(xx, off, 64);
    }
    if ((threadIdx.x & 63) == 0) { s[0][threadIdx.x >> 6] = xt; s[1][threadIdx.x >> 6] = xx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ((s[0][0] + s[0][1]) + s[0][2]) + s[0][3];
        part[2 * blockIdx.x + 1] = ((s[1][0] + s[1][1]) + s[1][2]) + s[1][3];
    }
}

// b[0..nb) = softplus^-1(s0), s0 = <X,T> / <X,X> from the partials (in order)
__global__ void lpi_bias_kernel(int np, const double *__restrict__ part, int nb,
                                float *__restrict__ b)
{
    __shared__ float val;
    if (threadIdx.x == 0) {
        double xt = 0.0, xx = 0.0;
        for (int q = 0; q < np; ++q) { xt += part[2 * q]; xx += part[2 * q + 1]; }
        const double s0 = (xt > 0.0 && xx > 0.0) ? xt / xx : 1.0;
        val = (float)(s0 + log(-expm1(-s0)));   // softplus^-1
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nb; q += blockDim.x) b[q] = val;
}

}  // namespace
}  // namespace nbx

using namespace nbx;

struct nbx_lpi {
    int N = 0, nI = 0, nIp = 0, n_hid = 0, max_batch = 0;
    nbx_mlp *mlp = nullptr;
    float *L = nullptr, *gL = nullptr, *mL = nullptr, *vL = nullptr;
    uint16_t *Lb = nullptr;
    int step = 0;
    // training buffers, max_batch rows
    float *A = nullptr, *Hx = nullptr, *Z = nullptr, *dZ = nullptr, *Pm = nullptr;
    uint16_t *Qb = nullptr, *dZb = nullptr, *G2b = nullptr;
    double *part = nullptr, *loss = nullptr;
    int64_t nL() const { return (int64_t)nIp * nIp; }
};

namespace nbx {

// Accessors for the bound preconditioner (learned.hip).
int lpi_dims(const nbx_lpi *M, int *N, int *nI, int *nIp)
{
    if (!M) return NBX_EINVAL;
    *N = M->N; *nI = M->nI; *nIp = M->nIp;
    return NBX_OK;
}
const uint16_t *lpi_Lb(const nbx_lpi *M) { return M->Lb; }
nbx_mlp *lpi_mlp(const nbx_lpi *M) { return M->mlp; }
int lpi_max_batch(const nbx_lpi *M) { return M->max_batch; }

}  // namespace nbx

extern "C" int nbx_lpi_destroy(nbx_lpi *M)
{
    if (!M) return NBX_OK;
    nbx_mlp_destroy(M->mlp);
    hipFree(M->L); hipFree(M->gL); hipFree(M->mL); hipFree(M->vL); hipFree(M->Lb);
    hipFree(M->A); hipFree(M->Hx); hipFree(M->Z); hipFree(M->dZ); hipFree(M->Pm);
    hipFree(M->Qb); hipFree(M->dZb); hipFree(M->G2b); hipFree(M->part); hipFree(M->loss);
    delete M;
    return NBX_OK;
}

extern "C" int nbx_lpi_create(int N, int n_hidden, int max_batch, nbx_lpi **out)
{
    if (!out) return NBX_EINVAL;
    *out = nullptr;
    if (N < 3 || N > kMaxN || n_hidden < 64 || n_hidden % 64 || max_batch < 64 ||
        max_batch % 64)
        return NBX_EINVAL;
    nbx_lpi *M = new (std::nothrow) nbx_lpi;
    if (!M) return NBX_ENOMEM;
    M->N = N;
    M->nI = (N - 2) * (N - 2) * (N - 2);
    M->nIp = (M->nI + 63) / 64 * 64;
    M->n_hid = n_hidden;
    M->max_batch = max_batch;
    int st = nbx_mlp_create(6, n_hidden, M->nI, max_batch, &M->mlp);
    if (st != NBX_OK) { nbx_lpi_destroy(M); return st; }
    const size_t nL = (size_t)M->nL(), rows = (size_t)max_batch * M->nIp;
    bool ok = hipMalloc(&M->L, nL * 4) == hipSuccess && hipMalloc(&M->gL, nL * 4) == hipSuccess &&
              hipMalloc(&M->mL, nL * 4) == hipSuccess && hipMalloc(&M->vL, nL * 4) == hipSuccess &&
              hipMalloc(&M->Lb, nL * 2) == hipSuccess &&
              hipMalloc(&M->A, rows * 4) == hipSuccess && hipMalloc(&M->Hx, rows * 4) == hipSuccess &&
              hipMalloc(&M->Z, rows * 4) == hipSuccess && hipMalloc(&M->dZ, rows * 4) == hipSuccess &&
              hipMalloc(&M->Pm, rows * 4) == hipSuccess && hipMalloc(&M->Qb, rows * 2) == hipSuccess &&
              hipMalloc(&M->dZb, rows * 2) == hipSuccess && hipMalloc(&M->G2b, rows * 2) == hipSuccess &&
              hipMalloc(&M->part, kLossParts * sizeof(double)) == hipSuccess &&
              hipMalloc(&M->loss, sizeof(double)) == hipSuccess;
    if (!ok) { nbx_lpi_destroy(M); return NBX_ENOMEM; }
    ok = hipMemset(M->L, 0, nL * 4) == hipSuccess && hipMemset(M->Lb, 0, nL * 2) == hipSuccess &&
         hipMemset(M->mL, 0, nL * 4) == hipSuccess && hipMemset(M->vL, 0, nL * 4) == hipSuccess &&
         hipMemset(M->gL, 0, nL * 4) == hipSuccess;
    if (!ok) { nbx_lpi_destroy(M); return NBX_EHIP; }
    *out = M;
    return NBX_OK;
}

extern "C" int nbx_lpi_shape(nbx_lpi *M, int *nI, int *nIp, int64_t *n_params)
{
    if (!M) return NBX_EINVAL;
    if (nI) *nI = M->nI;
    if (nIp) *nIp = M->nIp;
    if (n_params) *n_params = M->nL() + mlp_nparams(M->mlp);
    return NBX_OK;
}

extern "C" int nbx_lpi_set_params(nbx_lpi *M, const float *params, void *stream)
{
    if (!M || !params) return NBX_EINVAL;
    hipStream_t s = as_stream(stream);
    const int64_t nL = M->nL();
    NBX_HIP(hipMemcpyAsync(M->L, params, nL * 4, hipMemcpyDeviceToDevice, s));
    int st = to_bf16(nL, M->L, M->Lb, s);
    if (st != NBX_OK) return st;
    NBX_HIP(hipMemsetAsync(M->mL, 0, nL * 4, s));
    NBX_HIP(hipMemsetAsync(M->vL, 0, nL * 4, s));
    M->step = 0;
    return mlp_set_params(M->mlp, params + nL, s);
}

extern "C" int nbx_lpi_get_params(nbx_lpi *M, float *params, float *grads, void *stream)
{
    if (!M) return NBX_EINVAL;
    hipStream_t s = as_stream(stream);
    const int64_t nL = M->nL(), nP = mlp_nparams(M->mlp);
    if (params) {
        NBX_HIP(hipMemcpyAsync(params, M->L, nL * 4, hipMemcpyDeviceToDevice, s));
        NBX_HIP(hipMemcpyAsync(params + nL, mlp_weights(M->mlp), nP * 4, hipMemcpyDeviceToDevice,
                               s));
    }
    if (grads) {
        NBX_HIP(hipMemcpyAsync(grads, M->gL, nL * 4, hipMemcpyDeviceToDevice, s));
        NBX_HIP(hipMemcpyAsync(grads + nL, mlp_grads(M->mlp), nP * 4, hipMemcpyDeviceToDevice,
                               s));
    }
    return NBX_OK;
}

static int lpi_grad(nbx_lpi *M, const uint16_t *X, const float *T, const uint16_t *F, int B,
                    hipStream_t s)
{
    const int n = M->nIp;
    const int64_t cnt = (int64_t)B * n;
    int st = mlp_forward_rows(M->mlp, F, B, M->A, s);
    if (st != NBX_OK) return st;
    // Hx = X L^T
    if ((st = gemm_bf16(0, 1, kEpiF32, B, n, n, X, n, M->Lb, n, M->Hx, n, nullptr, 0, nullptr,
                        nullptr, 0, s, nullptr)) != NBX_OK)
        return st;
    hipLaunchKernelGGL(lpi_q_kernel, dim3(lpi_grid(cnt)), dim3(256), 0, s, cnt, M->Hx, M->A,
                       M->Qb);
    NBX_LAUNCH_CHECK();
    // Z = Q L; dZ, loss
    if ((st = gemm_bf16(0, 0, kEpiF32, B, n, n, M->Qb, n, M->Lb, n, M->Z, n, nullptr, 0, nullptr,
                        nullptr, 0, s, nullptr)) != NBX_OK)
        return st;
    if ((st = mse_grad(B, n, M->nI, M->Z, T, M->dZ, M->dZb, M->part, M->loss, s)) != NBX_OK)
        return st;
    // Pm = dZ L^T
    if ((st = gemm_bf16(0, 1, kEpiF32, B, n, n, M->dZb, n, M->Lb, n, M->Pm, n, nullptr, 0,
                        nullptr, nullptr, 0, s, nullptr)) != NBX_OK)
        return st;
    float *dA = nullptr;
    uint16_t *dAb = nullptr;
    mlp_grad_buffers(M->mlp, &dA, &dAb);
    hipLaunchKernelGGL(lpi_back_kernel, dim3(lpi_grid(cnt)), dim3(256), 0, s, cnt, M->Hx, M->Pm,
                       M->A, dA, dAb, M->G2b);
    NBX_LAUNCH_CHECK();
    // dL = Q^T dZ + (gamma Pm)^T X
    if ((st = gemm_bf16(1, 0, kEpiF32, n, n, B, M->Qb, n, M->dZb, n, M->gL, n, nullptr, 0,
                        nullptr, nullptr, 0, s, nullptr)) != NBX_OK)
        return st;
    if ((st = gemm_bf16(1, 0, kEpiAcc, n, n, B, M->G2b, n, X, n, M->gL, n, nullptr, 0, nullptr,
                        nullptr, 0, s, nullptr)) != NBX_OK)
        return st;
    return mlp_backprop_rows(M->mlp, F, B, s);
}

extern "C" int nbx_lpi_grad(nbx_lpi *M, const void *X, const float *T, const void *F, int B,
                            double *loss, void *stream)
{
    if (!M || !X || !T || !F || B < 64 || B % 64 || B > M->max_batch) return NBX_EINVAL;
    hipStream_t s = as_stream(stream);
    int st = lpi_grad(M, (const uint16_t *)X, T, (const uint16_t *)F, B, s);
    if (st != NBX_OK) return st;
    if (loss) NBX_HIP(hipMemcpyAsync(loss, M->loss, sizeof(double), hipMemcpyDeviceToDevice, s));
    return NBX_OK;
}

extern "C" int nbx_lpi_init_scale(nbx_lpi *M, const void *X, const float *T, int B,
                                  void *stream)
{
    if (!M || !X || !T || B < 1) return NBX_EINVAL;
    hipStream_t s = as_stream(stream);
    const int64_t n = (int64_t)B * M->nIp;
    const int np = (int)std::min<int64_t>((n + 255) / 256, kLossParts / 2);
    hipLaunchKernelGGL(lpi_xt_kernel, dim3(np), dim3(256), 0, s, n, (const uint16_t *)X, T,
                       M->part);
    int nb = 0;
    const int64_t ob = mlp_last_bias(M->mlp, &nb);
    hipLaunchKernelGGL(lpi_bias_kernel, dim3(1), dim3(256), 0, s, np, M->part, nb,
                       mlp_weights(M->mlp) + ob);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

extern "C" int nbx_lpi_train_step(nbx_lpi *M, const void *X, const float *T, const void *F,
                                  int B, float lr, double *loss, void *stream)
{
    if (!(lr > 0)) return NBX_EINVAL;
    int st = nbx_lpi_grad(M, X, T, F, B, loss, stream);
    if (st != NBX_OK) return st;
    hipStream_t s = as_stream(stream);
    M->step += 1;
    st = adam_update(M->nL(), M->L, M->Lb, M->mL, M->vL, M->gL, lr, M->step, s);
    if (st != NBX_OK) return st;
    return mlp_adam(M->mlp, lr, s);
}
