// mlp.hip -- BF16 matrix-core kernels for the element-local network of the
// learned preconditioner: a tiled GEMM on gfx950's v_mfma_f32_16x16x32_bf16
// with fused epilogues, and the training steps built on it (loss gradient,
// bias gradients, Adam).  This is the one dense contraction of the hot path:
// a batch of elements times the weight matrices, [B x 1024] x [1024 x 128]
// and back, which fills matrix-core tiles; FP32 accumulation throughout,
// FP32 master weights with BF16 copies for the products.
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <new>

namespace nbx {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// float -> bfloat16, round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

enum Epi { EPI_F32 = 0, EPI_BIAS_RELU_BF16 = 1, EPI_BIAS_F32 = 2, EPI_RELU_GRAD_BF16 = 3,
           EPI_ACC_F32 = 4, EPI_MUL_BF16 = 5 };

constexpr int TM = 64, TN = 64, TK = 32, LDS_PAD = 8;
constexpr int kLossBlocks = 1024;   // partial sums of the squared-error loss

// C[M x N] = op(A)[M x K] op(B)[K x N], BF16 operands, FP32 accumulation.
//   A element (m,k): TA ? A[k*lda + m] : A[m*lda + k]
//   B element (k,n): TB ? B[n*ldb + k] : B[k*ldb + n]
// M, N multiples of 64, K a multiple of 32, leading dimensions multiples of
// 8 (16-byte rows).  A 256-thread block computes a 64x64 tile; each wave a
// 32x32 quarter as 2x2 16x16x32 MFMA tiles.  Operand tiles are staged in
// LDS K-contiguous ([m][k] and [n][k]) so every lane's 8-element MFMA
// operand is one 16-byte LDS read.
// Epilogues: EPI_F32 C = v; EPI_ACC_F32 C += v; EPI_BIAS_F32 C = v + bias[n];
// EPI_BIAS_RELU_BF16 Cb = bf16(relu(v + bias[n])); EPI_RELU_GRAD_BF16
// Cb = bf16(v) where the BF16 activation act[m][n] is positive, else 0;
// EPI_MUL_BF16 Cb = bf16(v * mul[m][n]) (mul FP32, leading dimension ldact).
template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256)
gemm_bf16_kernel(int M, int N, int K, const uint16_t *__restrict__ A, int lda,
                 const uint16_t *__restrict__ B, int ldb, float *__restrict__ C, int ldc,
                 uint16_t *__restrict__ Cb, int ldcb, const float *__restrict__ bias,
                 const uint16_t *__restrict__ act, int ldact, const float *__restrict__ mul)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[TM][TK + LDS_PAD];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[TN][TK + LDS_PAD];
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < K; k0 += TK) {
        if (!TA) {   // 64 rows x 4 chunks of 8 along k
            const int r = t >> 2, c = (t & 3) * 8;
            *reinterpret_cast<uint4 *>(&As[r][c]) =
                *reinterpret_cast<const uint4 *>(A + (size_t)(m0 + r) * lda + k0 + c);
        } else {     // 32 k x 8 chunks of 8 along m, transposed into [m][k]
            const int kk = t >> 3, mc = (t & 7) * 8;
            const uint4 v = *reinterpret_cast<const uint4 *>(A + (size_t)(k0 + kk) * lda + m0 + mc);
            const uint16_t *e = reinterpret_cast<const uint16_t *>(&v);
#pragma unroll
            for (int i = 0; i < 8; ++i) As[mc + i][kk] = e[i];
        }
        if (TB) {    // 64 n x 4 chunks of 8 along k
            const int r = t >> 2, c = (t & 3) * 8;
            *reinterpret_cast<uint4 *>(&Bs[r][c]) =
                *reinterpret_cast<const uint4 *>(B + (size_t)(n0 + r) * ldb + k0 + c);
        } else {     // 32 k x 8 chunks of 8 along n, transposed into [n][k]
            const int kk = t >> 3, nc = (t & 7) * 8;
            const uint4 v = *reinterpret_cast<const uint4 *>(B + (size_t)(k0 + kk) * ldb + n0 + nc);
            const uint16_t *e = reinterpret_cast<const uint16_t *>(&v);
#pragma unroll
            for (int i = 0; i < 8; ++i) Bs[nc + i][kk] = e[i];
        }
        __syncthreads();
        const int row = lane & 15, kq = 8 * (lane >> 4);
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const bf16x8 av = *reinterpret_cast<const bf16x8 *>(&As[wm + 16 * a + row][kq]);
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(&Bs[wn + 16 * b + row][kq]);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[a][b], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // lane holds C[4*(lane/16) + i][lane%16] of each 16x16 tile
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = m0 + wm + 16 * a + 4 * (lane >> 4) + i;
                const int n = n0 + wn + 16 * b + (lane & 15);
                float v = acc[a][b][i];
                if (EPI == EPI_F32) {
                    C[(size_t)m * ldc + n] = v;
                } else if (EPI == EPI_ACC_F32) {
                    C[(size_t)m * ldc + n] += v;
                } else if (EPI == EPI_MUL_BF16) {
                    Cb[(size_t)m * ldcb + n] = f2bf(v * mul[(size_t)m * ldact + n]);
                } else if (EPI == EPI_BIAS_F32) {
                    C[(size_t)m * ldc + n] = v + bias[n];
                } else if (EPI == EPI_BIAS_RELU_BF16) {
                    v += bias[n];
                    Cb[(size_t)m * ldcb + n] = f2bf(v > 0.f ? v : 0.f);
                } else {   // EPI_RELU_GRAD_BF16: gradient through relu(H)
                    const uint16_t h = act[(size_t)m * ldact + n];
                    const bool pos = (h & 0x8000u) == 0 && (h & 0x7fffu) != 0;
                    Cb[(size_t)m * ldcb + n] = f2bf(pos ? v : 0.f);
                }
            }
}

template <bool TA, bool TB, int EPI>
void launch_gemm(int M, int N, int K, const uint16_t *A, int lda, const uint16_t *B, int ldb,
                 float *C, int ldc, uint16_t *Cb, int ldcb, const float *bias,
                 const uint16_t *act, int ldact, const float *mul, hipStream_t s)
{
    hipLaunchKernelGGL((gemm_bf16_kernel<TA, TB, EPI>), dim3(N / TN, M / TM), dim3(256), 0, s, M,
                       N, K, A, lda, B, ldb, C, ldc, Cb, ldcb, bias, act, ldact, mul);
}

int gemm(int ta, int tb, int epi, int M, int N, int K, const uint16_t *A, int lda,
         const uint16_t *B, int ldb, float *C, int ldc, uint16_t *Cb, int ldcb, const float *bias,
         const uint16_t *act, int ldact, hipStream_t s, const float *mul = nullptr)
{
    if (M <= 0 || N <= 0 || K <= 0 || M % TM || N % TN || K % TK) return NBX_EINVAL;
    if (lda % 8 || ldb % 8) return NBX_EINVAL;
    if (!A || !B) return NBX_EINVAL;
    if ((epi == EPI_F32 || epi == EPI_BIAS_F32 || epi == EPI_ACC_F32) && !C) return NBX_EINVAL;
    if ((epi == EPI_BIAS_RELU_BF16 || epi == EPI_RELU_GRAD_BF16 || epi == EPI_MUL_BF16) && !Cb)
        return NBX_EINVAL;
    if ((epi == EPI_BIAS_F32 || epi == EPI_BIAS_RELU_BF16) && !bias) return NBX_EINVAL;
    if (epi == EPI_RELU_GRAD_BF16 && !act) return NBX_EINVAL;
    if (epi == EPI_MUL_BF16 && !mul) return NBX_EINVAL;
#define NBX_G(TA_, TB_, E_)                                                                 \
    if (ta == TA_ && tb == TB_ && epi == E_) {                                              \
        launch_gemm<TA_, TB_, E_>(M, N, K, A, lda, B, ldb, C, ldc, Cb, ldcb, bias, act, ldact, \
                                  mul, s);                                                  \
        NBX_LAUNCH_CHECK();                                                                 \
        return NBX_OK;                                                                      \
    }
    NBX_G(0, 0, 0) NBX_G(0, 1, 0) NBX_G(1, 0, 0) NBX_G(1, 1, 0)
    NBX_G(0, 1, 1) NBX_G(0, 1, 2) NBX_G(0, 0, 3) NBX_G(1, 0, 4) NBX_G(0, 1, 5)
#undef NBX_G
    return NBX_EUNSUPPORTED;
}

// dY = 2 (Y - T) / (B * n_out) on the first n_out columns, 0 elsewhere (FP32
// and BF16 copies); per-block partial sums of (Y - T)^2.
__global__ void __launch_bounds__(256)
loss_grad_kernel(int B, int n_pad, int n_out, const float *__restrict__ Y,
                 const float *__restrict__ T, float *__restrict__ dY, uint16_t *__restrict__ dYb,
                 double *__restrict__ part)
{
    __shared__ double s[4];
    const float scale = 2.0f / ((float)B * (float)n_out);
    double acc = 0.0;
    const int64_t total = (int64_t)B * n_pad;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int col = (int)(q % n_pad);
        float g = 0.f;
        if (col < n_out) {
            const float d = Y[q] - T[q];
            acc += (double)d * (double)d;
            g = scale * d;
        }
        dY[q] = g;
        dYb[q] = f2bf(g);
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

__global__ void __launch_bounds__(256)
sum_partials_kernel(int nb, const double *__restrict__ part, double scale, double *__restrict__ out)
{
    __shared__ double s[4];
    double a = 0.0;
    for (int q = threadIdx.x; q < nb; q += blockDim.x) a += part[q];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) *out = (s[0] + s[1] + s[2] + s[3]) * scale;
}

// Column sums of X [M x N] (FP32 or BF16; M, N multiples of 64), deterministic, in two
// launches: colsum_part_kernel sums 64 consecutive columns over a chunk of
// 64 rows per workgroup (four row strides per column, coalesced across the
// columns, then added in a fixed order) into part[M/64][N];
// colsum_fin_kernel adds the chunks in order.  (One thread per column over
// all rows left a batch of 1024 rows to one or two workgroups: 160-220 us a
// call.)
template <bool BF>
__global__ void __launch_bounds__(256)
colsum_part_kernel(int N, const void *__restrict__ X, int ldx, float *__restrict__ part)
{
    __shared__ float s_red[4][64];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + tx;
    const int r0 = blockIdx.y * 64;
    float s = 0.f;
    for (int r = ty; r < 64; r += 4) {
        const size_t q = (size_t)(r0 + r) * ldx + n;
        s += BF ? bf2f(reinterpret_cast<const uint16_t *>(X)[q])
                : reinterpret_cast<const float *>(X)[q];
    }
    s_red[ty][tx] = s;
    __syncthreads();
    if (ty == 0)
        part[(size_t)blockIdx.y * N + n] = ((s_red[0][tx] + s_red[1][tx]) + s_red[2][tx]) +
                                           s_red[3][tx];
}

__global__ void colsum_fin_kernel(int R, int N, const float *__restrict__ part,
                                  float *__restrict__ out)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int c = 0; c < R; ++c) s += part[(size_t)c * N + n];
    out[n] = s;
}

// Adam (Kingma & Ba 2015) on FP32 master weights; refreshes the BF16 copy.
__global__ void adam_kernel(int64_t n, float *__restrict__ w, uint16_t *__restrict__ wb,
                            float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, float lr, float b1, float b2, float eps,
                            float c1, float c2)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const float gq = g[q];
        const float mq = b1 * m[q] + (1.f - b1) * gq;
        const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
        m[q] = mq; v[q] = vq;
        const float mh = mq / c1, vh = vq / c2;
        const float wq = w[q] - lr * mh / (sqrtf(vh) + eps);
        w[q] = wq;
        if (wb) wb[q] = f2bf(wq);
    }
}

__global__ void to_bf16_kernel(int64_t n, const float *__restrict__ a, uint16_t *__restrict__ b)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        b[q] = f2bf(a[q]);
}

unsigned grid_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b > 16384) b = 16384;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

int gemm_bf16(int ta, int tb, int epi, int M, int N, int K, const uint16_t *A, int lda,
              const uint16_t *B, int ldb, float *C, int ldc, uint16_t *Cb, int ldcb,
              const float *bias, const uint16_t *act, int ldact, hipStream_t s,
              const float *mul)
{
    return gemm(ta, tb, epi, M, N, K, A, lda, B, ldb, C, ldc, Cb, ldcb, bias, act, ldact, s,
                mul);
}

int mse_grad(int B, int n_pad, int n_out, const float *Y, const float *T, float *dY,
             uint16_t *dYb, double *part, double *loss, hipStream_t s)
{
    hipLaunchKernelGGL(loss_grad_kernel, dim3(kLossBlocks), dim3(256), 0, s, B, n_pad, n_out, Y,
                       T, dY, dYb, part);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, kLossBlocks, part,
                       1.0 / ((double)B * n_out), loss);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

int adam_update(int64_t n, float *w, uint16_t *wb, float *m, float *v, const float *g, float lr,
                int step, hipStream_t s)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, w, wb, m, v, g, lr,
                       b1, b2, eps, c1, c2);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

int to_bf16(int64_t n, const float *a, uint16_t *b, hipStream_t s)
{
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, a, b);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

int mlp_forward_rows(nbx_mlp *P, const uint16_t *X, int B, float *Y, hipStream_t s);

}  // namespace nbx

// ----------------------------------------------------------------- handle

struct nbx_mlp {
    int n_in = 0, n_hid = 0, n_out = 0, in_pad = 0, out_pad = 0, max_batch = 0;
    // FP32 master parameters, gradients, Adam moments: one arena each,
    // laid out W1 [hid x in_pad], b1 [hid], W2 [hid x hid], b2 [hid],
    // W3 [out_pad x hid], b3 [out_pad].
    int64_t n_par = 0;
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    uint16_t *wb = nullptr;   // BF16 copy of w (biases unused)
    // activations for max_batch rows
    uint16_t *H1 = nullptr, *H2 = nullptr, *dYb = nullptr, *dH1 = nullptr, *dH2 = nullptr;
    float *Y = nullptr, *dY = nullptr;
    double *part = nullptr, *loss = nullptr;
    float *cpart = nullptr;   // column-sum chunks [max_batch/64][max(n_hid, out_pad)]
    int step = 0;
    int64_t oW1() const { return 0; }
    int64_t ob1() const { return (int64_t)n_hid * in_pad; }
    int64_t oW2() const { return ob1() + n_hid; }
    int64_t ob2() const { return oW2() + (int64_t)n_hid * n_hid; }
    int64_t oW3() const { return ob2() + n_hid; }
    int64_t ob3() const { return oW3() + (int64_t)out_pad * n_hid; }
    int64_t total() const { return ob3() + out_pad; }
};

namespace nbx {
namespace {

// out[N] = column sums of X [M x N] (M, N multiples of 64; part holds
// M/64 x N floats).
template <bool BF>
void colsum(int M, int N, const void *X, int ldx, float *part, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(colsum_part_kernel<BF>, dim3(N / 64, M / 64), dim3(256), 0, s, N, X, ldx,
                       part);
    hipLaunchKernelGGL(colsum_fin_kernel, dim3((N + 255) / 256), dim3(256), 0, s, M / 64, N, part,
                       out);
}

// Forward pass for B rows of X [B x in_pad] (BF16): H1, H2 (BF16) and
// Y [B x out_pad] (FP32, biases added).
int mlp_forward(nbx_mlp *P, const uint16_t *X, int B, float *Y, hipStream_t s)
{
    int st;
    const uint16_t *wb = P->wb;
    const float *w = P->w;
    if ((st = gemm(0, 1, EPI_BIAS_RELU_BF16, B, P->n_hid, P->in_pad, X, P->in_pad,
                   wb + P->oW1(), P->in_pad, nullptr, 0, P->H1, P->n_hid, w + P->ob1(), nullptr,
                   0, s)) != NBX_OK)
        return st;
    if ((st = gemm(0, 1, EPI_BIAS_RELU_BF16, B, P->n_hid, P->n_hid, P->H1, P->n_hid,
                   wb + P->oW2(), P->n_hid, nullptr, 0, P->H2, P->n_hid, w + P->ob2(), nullptr,
                   0, s)) != NBX_OK)
        return st;
    return gemm(0, 1, EPI_BIAS_F32, B, P->out_pad, P->n_hid, P->H2, P->n_hid, wb + P->oW3(),
                P->n_hid, Y, P->out_pad, nullptr, 0, w + P->ob3(), nullptr, 0, s);
}

// Gradients of every parameter into P->g from the output gradient already in
// P->dY (FP32) and P->dYb (BF16), for the B rows of X whose forward pass
// left H1, H2 in the activation buffers.
int mlp_backprop(nbx_mlp *P, const uint16_t *X, int B, hipStream_t s)
{
    int st;
    const uint16_t *wb = P->wb;
    float *g = P->g;
    // layer 3: dW3 = dY^T H2, db3 = colsum dY, dH2 = (dY W3) * relu'(H2)
    if ((st = gemm(1, 0, EPI_F32, P->out_pad, P->n_hid, B, P->dYb, P->out_pad, P->H2, P->n_hid,
                   g + P->oW3(), P->n_hid, nullptr, 0, nullptr, nullptr, 0, s)) != NBX_OK)
        return st;
    colsum<false>(B, P->out_pad, P->dY, P->out_pad, P->cpart, g + P->ob3(), s);
    if ((st = gemm(0, 0, EPI_RELU_GRAD_BF16, B, P->n_hid, P->out_pad, P->dYb, P->out_pad,
                   wb + P->oW3(), P->n_hid, nullptr, 0, P->dH2, P->n_hid, nullptr, P->H2,
                   P->n_hid, s)) != NBX_OK)
        return st;
    // layer 2
    if ((st = gemm(1, 0, EPI_F32, P->n_hid, P->n_hid, B, P->dH2, P->n_hid, P->H1, P->n_hid,
                   g + P->oW2(), P->n_hid, nullptr, 0, nullptr, nullptr, 0, s)) != NBX_OK)
        return st;
    colsum<true>(B, P->n_hid, P->dH2, P->n_hid, P->cpart, g + P->ob2(), s);
    if ((st = gemm(0, 0, EPI_RELU_GRAD_BF16, B, P->n_hid, P->n_hid, P->dH2, P->n_hid,
                   wb + P->oW2(), P->n_hid, nullptr, 0, P->dH1, P->n_hid, nullptr, P->H1,
                   P->n_hid, s)) != NBX_OK)
        return st;
    // layer 1
    if ((st = gemm(1, 0, EPI_F32, P->n_hid, P->in_pad, B, P->dH1, P->n_hid, X, P->in_pad,
                   g + P->oW1(), P->in_pad, nullptr, 0, nullptr, nullptr, 0, s)) != NBX_OK)
        return st;
    colsum<true>(B, P->n_hid, P->dH1, P->n_hid, P->cpart, g + P->ob1(), s);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

// Gradients of the mean squared error over the first n_out outputs into
// P->g, loss into P->loss (device).
int mlp_backward(nbx_mlp *P, const uint16_t *X, const float *T, int B, hipStream_t s)
{
    int st = mlp_forward(P, X, B, P->Y, s);
    if (st != NBX_OK) return st;
    hipLaunchKernelGGL(loss_grad_kernel, dim3(kLossBlocks), dim3(256), 0, s, B, P->out_pad,
                       P->n_out, P->Y, T, P->dY, P->dYb, P->part);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, kLossBlocks, P->part,
                       1.0 / ((double)B * P->n_out), P->loss);
    NBX_LAUNCH_CHECK();
    return mlp_backprop(P, X, B, s);
}

}  // namespace

int mlp_forward_rows(nbx_mlp *P, const uint16_t *X, int B, float *Y, hipStream_t s)
{
    if (B < 64 || B % 64 || B > P->max_batch) return NBX_EINVAL;
    return mlp_forward(P, X, B, Y, s);
}

int mlp_dims(nbx_mlp *P, int *n_in, int *n_out, int *in_pad, int *out_pad, int *max_batch)
{
    if (!P) return NBX_EINVAL;
    *n_in = P->n_in; *n_out = P->n_out; *in_pad = P->in_pad; *out_pad = P->out_pad;
    *max_batch = P->max_batch;
    return NBX_OK;
}

// For a composite model: the output-gradient buffers (FP32 and BF16,
// [max_batch][out_pad]) to fill before mlp_backprop_rows, which then forms
// every parameter's gradient for the B rows of X last run forward with
// mlp_forward_rows; mlp_adam applies one Adam step to all parameters.
int mlp_grad_buffers(nbx_mlp *P, float **dY, uint16_t **dYb)
{
    if (!P) return NBX_EINVAL;
    *dY = P->dY; *dYb = P->dYb;
    return NBX_OK;
}

int mlp_backprop_rows(nbx_mlp *P, const uint16_t *X, int B, hipStream_t s)
{
    if (!P || B < 64 || B % 64 || B > P->max_batch) return NBX_EINVAL;
    return mlp_backprop(P, X, B, s);
}

int mlp_adam(nbx_mlp *P, float lr, hipStream_t s)
{
    P->step += 1;
    return adam_update(P->n_par, P->w, P->wb, P->m, P->v, P->g, lr, P->step, s);
}

int64_t mlp_nparams(nbx_mlp *P) { return P ? P->n_par : 0; }
int64_t mlp_last_bias(nbx_mlp *P, int *n) { *n = P->out_pad; return P->ob3(); }
float *mlp_weights(nbx_mlp *P) { return P ? P->w : nullptr; }
float *mlp_grads(nbx_mlp *P) { return P ? P->g : nullptr; }

}  // namespace nbx

using namespace nbx;

extern "C" int nbx_gemm_bf16(int trans_a, int trans_b, int M, int N, int K, const void *A,
                             int lda, const void *B, int ldb, float *C, int ldc, void *stream)
{
    return gemm(trans_a ? 1 : 0, trans_b ? 1 : 0, EPI_F32, M, N, K, (const uint16_t *)A, lda,
                (const uint16_t *)B, ldb, C, ldc, nullptr, 0, nullptr, nullptr, 0,
                as_stream(stream));
}

extern "C" int nbx_mlp_create(int n_in, int n_hidden, int n_out, int max_batch, nbx_mlp **out)
{
    if (!out) return NBX_EINVAL;
    *out = nullptr;
    if (n_in < 1 || n_out < 1 || n_hidden < 64 || n_hidden % 64 || max_batch < 64 ||
        max_batch % 64)
        return NBX_EINVAL;
    nbx_mlp *P = new (std::nothrow) nbx_mlp;
    if (!P) return NBX_ENOMEM;
    P->n_in = n_in; P->n_hid = n_hidden; P->n_out = n_out; P->max_batch = max_batch;
    P->in_pad = (n_in + 63) / 64 * 64;
    P->out_pad = (n_out + 63) / 64 * 64;
    P->n_par = P->total();
    const size_t np = (size_t)P->n_par, B = (size_t)max_batch;
    bool ok = hipMalloc(&P->w, np * 4) == hipSuccess && hipMalloc(&P->g, np * 4) == hipSuccess &&
              hipMalloc(&P->m, np * 4) == hipSuccess && hipMalloc(&P->v, np * 4) == hipSuccess &&
              hipMalloc(&P->wb, np * 2) == hipSuccess &&
              hipMalloc(&P->H1, B * P->n_hid * 2) == hipSuccess &&
              hipMalloc(&P->H2, B * P->n_hid * 2) == hipSuccess &&
              hipMalloc(&P->dH1, B * P->n_hid * 2) == hipSuccess &&
              hipMalloc(&P->dH2, B * P->n_hid * 2) == hipSuccess &&
              hipMalloc(&P->dYb, B * P->out_pad * 2) == hipSuccess &&
              hipMalloc(&P->Y, B * P->out_pad * 4) == hipSuccess &&
              hipMalloc(&P->dY, B * P->out_pad * 4) == hipSuccess &&
              hipMalloc(&P->part, kLossBlocks * sizeof(double)) == hipSuccess &&
              hipMalloc(&P->loss, sizeof(double)) == hipSuccess &&
              hipMalloc(&P->cpart, B / 64 * std::max(P->n_hid, P->out_pad) * 4) == hipSuccess;
    if (!ok) { nbx_mlp_destroy(P); return NBX_ENOMEM; }
    hipMemset(P->w, 0, np * 4); hipMemset(P->g, 0, np * 4);
    hipMemset(P->m, 0, np * 4); hipMemset(P->v, 0, np * 4); hipMemset(P->wb, 0, np * 2);
    *out = P;
    return NBX_OK;
}

extern "C" int nbx_mlp_destroy(nbx_mlp *P)
{
    if (!P) return NBX_OK;
    hipFree(P->w); hipFree(P->g); hipFree(P->m); hipFree(P->v); hipFree(P->wb);
    hipFree(P->H1); hipFree(P->H2); hipFree(P->dH1); hipFree(P->dH2); hipFree(P->dYb);
    hipFree(P->Y); hipFree(P->dY); hipFree(P->part); hipFree(P->loss); hipFree(P->cpart);
    delete P;
    return NBX_OK;
}

extern "C" int nbx_mlp_shape(nbx_mlp *P, int *in_pad, int *out_pad, int64_t *n_params)
{
    if (!P) return NBX_EINVAL;
    if (in_pad) *in_pad = P->in_pad;
    if (out_pad) *out_pad = P->out_pad;
    if (n_params) *n_params = P->n_par;
    return NBX_OK;
}

namespace nbx {

int mlp_set_params(nbx_mlp *P, const float *params, hipStream_t s)
{
    if (!P || !params) return NBX_EINVAL;
    NBX_HIP(hipMemcpyAsync(P->w, params, (size_t)P->n_par * 4, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(P->n_par)), dim3(256), 0, s, P->n_par, P->w,
                       P->wb);
    NBX_LAUNCH_CHECK();
    NBX_HIP(hipMemsetAsync(P->m, 0, (size_t)P->n_par * 4, s));
    NBX_HIP(hipMemsetAsync(P->v, 0, (size_t)P->n_par * 4, s));
    P->step = 0;
    return NBX_OK;
}

}  // namespace nbx

extern "C" int nbx_mlp_set_params(nbx_mlp *P, const float *params, void *stream)
{
    return mlp_set_params(P, params, as_stream(stream));
}

extern "C" int nbx_mlp_get_params(nbx_mlp *P, float *params, float *grads, void *stream)
{
    if (!P) return NBX_EINVAL;
    hipStream_t s = as_stream(stream);
    if (params)
        NBX_HIP(hipMemcpyAsync(params, P->w, (size_t)P->n_par * 4, hipMemcpyDeviceToDevice, s));
    if (grads)
        NBX_HIP(hipMemcpyAsync(grads, P->g, (size_t)P->n_par * 4, hipMemcpyDeviceToDevice, s));
    return NBX_OK;
}

extern "C" int nbx_mlp_forward(nbx_mlp *P, const void *X, int B, float *Y, void *stream)
{
    if (!P || !X || !Y || B < 64 || B % 64 || B > P->max_batch) return NBX_EINVAL;
    return mlp_forward(P, (const uint16_t *)X, B, Y, as_stream(stream));
}

extern "C" int nbx_mlp_grad(nbx_mlp *P, const void *X, const float *T, int B, double *loss,
                            void *stream)
{
    if (!P || !X || !T || B < 64 || B % 64 || B > P->max_batch) return NBX_EINVAL;
    hipStream_t s = as_stream(stream);
    int st = mlp_backward(P, (const uint16_t *)X, T, B, s);
    if (st != NBX_OK) return st;
    if (loss) NBX_HIP(hipMemcpyAsync(loss, P->loss, sizeof(double), hipMemcpyDeviceToDevice, s));
    return NBX_OK;
}

extern "C" int nbx_mlp_train_step(nbx_mlp *P, const void *X, const float *T, int B, float lr,
                                  double *loss, void *stream)
{
    if (!(lr > 0)) return NBX_EINVAL;
    int st = nbx_mlp_grad(P, X, T, B, loss, stream);
    if (st != NBX_OK) return st;
    return mlp_adam(P, lr, as_stream(stream));
}
