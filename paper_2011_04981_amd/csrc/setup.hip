// setup.hip -- discretisation set-up for the Poisson problem: GLL rule,
// derivative matrix, brick geometry and its isoparametric factors, global
// numbering, the Jacobi diagonal and the assembled load vector.
//
// The paper names the problem (Poisson by CG on a "block or linear
// geometry", Section II-B) and the layout of the factors (Listing 1:
// g(1..6) = the symmetric 3x3 matrix), not the discretisation; this file
// uses the standard spectral-element definitions.
#include "internal.hpp"

#include <cmath>
#include <vector>

namespace nbx {

// GLL nodes by Newton's method on  q(x) = x P_p(x) - P_{p-1}(x), whose
// interior roots are the roots of P'_p (from (1-x^2) P'_p = p (P_{p-1} -
// x P_p)), with the update dx = q / ((p+1) P_p) started from
// Chebyshev-Gauss-Lobatto points; weights 2 / (p (p+1) P_p(x)^2).
int gll_host(int N, double *xi, double *w)
{
    if (N < 2 || N > kMaxN) return NBX_EINVAL;
    const int p = N - 1;
    std::vector<double> x(N), Pp(N), Pm(N);
    for (int q = 0; q < N; ++q) x[q] = -std::cos(M_PI * q / p);
    for (int it = 0; it < 100; ++it) {
        double dmax = 0.0;
        for (int q = 0; q < N; ++q) {
            double a = 1.0, b = x[q];       // P_0, P_1
            for (int n = 2; n <= p; ++n) {
                const double c = ((2 * n - 1) * x[q] * b - (n - 1) * a) / n;
                a = b; b = c;
            }
            Pp[q] = b; Pm[q] = a;           // P_p, P_{p-1}
            if (q == 0 || q == p) continue;
            const double dx = (x[q] * b - a) / (N * b);
            x[q] -= dx;
            dmax = std::fmax(dmax, std::fabs(dx));
        }
        if (dmax < 1e-17) break;
    }
    x[0] = -1.0; x[p] = 1.0;
    for (int q = 0; q < N; ++q) {
        double a = 1.0, b = x[q];
        for (int n = 2; n <= p; ++n) {
            const double c = ((2 * n - 1) * x[q] * b - (n - 1) * a) / n;
            a = b; b = c;
        }
        xi[q] = x[q];
        w[q] = 2.0 / (p * (p + 1.0) * b * b);
    }
    return NBX_OK;
}

// Derivative matrix from barycentric weights lambda_b = 1/prod(xi_b-xi_k):
// D[a][b] = (lambda_b/lambda_a) / (xi_a - xi_b) for a != b and the
// diagonal as minus the row sum (the derivative of a constant is zero).
void deriv_host(int N, const double *xi, double *D)
{
    std::vector<double> lam(N);
    for (int b = 0; b < N; ++b) {
        double prod = 1.0;
        for (int k = 0; k < N; ++k)
            if (k != b) prod *= (xi[b] - xi[k]);
        lam[b] = 1.0 / prod;
    }
    for (int a = 0; a < N; ++a) {
        double row = 0.0;
        for (int b = 0; b < N; ++b) {
            if (a == b) continue;
            const double v = (lam[b] / lam[a]) / (xi[a] - xi[b]);
            D[a * N + b] = v;
            row += v;
        }
        D[a * N + a] = -row;
    }
}

namespace {

struct GllTab {
    double xi[kMaxN];
    double w[kMaxN];
    double D[kMaxN * kMaxN];
};

struct BrickDesc {
    int ex, ey, ez;
    double def[12];
};

// One workgroup per element: node coordinates into LDS (from the brick
// mapping or from xyz_in), then the isoparametric Jacobian at each node,
// its inverse by cofactors, and the six weighted factors.
__global__ void geom_kernel(int N, int64_t E, GllTab tab, BrickDesc brick,
                            const double *__restrict__ xyz_in, double *__restrict__ G,
                            double *__restrict__ bm, double *__restrict__ xyz_out)
{
    extern __shared__ double s_xyz[];
    const int64_t e = blockIdx.x;
    const int N3 = N * N * N, N2 = N * N;
    double *sx = s_xyz, *sy = s_xyz + N3, *sz = s_xyz + 2 * N3;
    const size_t n_tot = (size_t)E * N3;
    for (int n = threadIdx.x; n < N3; n += blockDim.x) {
        const int i = n % N, j = (n / N) % N, k = n / N2;
        double c[3];
        if (xyz_in) {
            for (int q = 0; q < 3; ++q) c[q] = xyz_in[q * n_tot + e * N3 + n];
        } else {
            const int a = (int)(e % brick.ex), b = (int)((e / brick.ex) % brick.ey),
                      cc = (int)(e / ((int64_t)brick.ex * brick.ey));
            const double X = (a + 0.5 * (tab.xi[i] + 1.0)) / brick.ex;
            const double Y = (b + 0.5 * (tab.xi[j] + 1.0)) / brick.ey;
            const double Z = (cc + 0.5 * (tab.xi[k] + 1.0)) / brick.ez;
            const double ref[3] = {X, Y, Z};
            for (int q = 0; q < 3; ++q) {
                const double *d = brick.def + 4 * q;
                c[q] = ref[q] + d[0] * sin(d[1] * M_PI * X) * sin(d[2] * M_PI * Y) *
                                    sin(d[3] * M_PI * Z);
            }
        }
        sx[n] = c[0]; sy[n] = c[1]; sz[n] = c[2];
        if (xyz_out)
            for (int q = 0; q < 3; ++q) xyz_out[q * n_tot + e * N3 + n] = c[q];
    }
    __syncthreads();
    for (int n = threadIdx.x; n < N3; n += blockDim.x) {
        const int i = n % N, j = (n / N) % N, k = n / N2;
        const double *S[3] = {sx, sy, sz};
        double J[3][3];
        for (int q = 0; q < 3; ++q) {
            double dr = 0, ds = 0, dt = 0;
            for (int m = 0; m < N; ++m) {
                dr += tab.D[i * N + m] * S[q][m + N * (j + N * k)];
                ds += tab.D[j * N + m] * S[q][i + N * (m + N * k)];
                dt += tab.D[k * N + m] * S[q][i + N * (j + N * m)];
            }
            J[q][0] = dr; J[q][1] = ds; J[q][2] = dt;
        }
        // cofactor matrix C[a][b]; inverse(J)[a][b] = C[b][a] / det
        double Cf[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const int a1 = (a + 1) % 3, a2 = (a + 2) % 3, b1 = (b + 1) % 3, b2 = (b + 2) % 3;
                Cf[a][b] = J[a1][b1] * J[a2][b2] - J[a1][b2] * J[a2][b1];
            }
        const double det = J[0][0] * Cf[0][0] + J[0][1] * Cf[0][1] + J[0][2] * Cf[0][2];
        // grad r_a = row a of inv(J) = column a of C / det;
        // W det (grad r_a . grad r_b) = W (C[:,a] . C[:,b]) / det
        const double W = tab.w[i] * tab.w[j] * tab.w[k];
        const int fa[6] = {0, 0, 0, 1, 1, 2}, fb[6] = {0, 1, 2, 1, 2, 2};
        for (int f = 0; f < 6; ++f) {
            const int a = fa[f], b = fb[f];
            const double dot = Cf[0][a] * Cf[0][b] + Cf[1][a] * Cf[1][b] + Cf[2][a] * Cf[2][b];
            G[gp_index(e, f, n, N3)] = W * dot / det;
        }
        if (bm) bm[(size_t)e * N3 + n] = W * det;
    }
}

// diag(A_e) at node p = (i,j,k):  sum_m D[m][i]^2 g1(m,j,k)
//   + sum_m D[m][j]^2 g4(i,m,k) + sum_m D[m][k]^2 g6(i,j,m)
//   + 2 D[i][i] D[j][j] g2 + 2 D[i][i] D[k][k] g3 + 2 D[j][j] D[k][k] g5.
// (Only the r-r, s-s, t-t products reach other nodes of the same line;
// the mixed products touch the diagonal only through D's own diagonal.)
__global__ void jacobi_diag_kernel(int N, int64_t E, const double *__restrict__ G,
                                   const double *__restrict__ D, double *__restrict__ diag)
{
    const int N3 = N * N * N;
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= E * N3) return;
    const int64_t e = l / N3;
    const int n = (int)(l - e * N3);
    const int i = n % N, j = (n / N) % N, k = n / (N * N);
    double s = 0.0;
    for (int m = 0; m < N; ++m) {
        const double a = D[m * N + i], b = D[m * N + j], c = D[m * N + k];
        s += a * a * G[gp_index(e, 0, m + N * (j + N * k), N3)];
        s += b * b * G[gp_index(e, 3, i + N * (m + N * k), N3)];
        s += c * c * G[gp_index(e, 5, i + N * (j + N * m), N3)];
    }
    const double di = D[i * N + i], dj = D[j * N + j], dk = D[k * N + k];
    s += 2.0 * (di * dj * G[gp_index(e, 1, n, N3)] + di * dk * G[gp_index(e, 2, n, N3)] +
                dj * dk * G[gp_index(e, 4, n, N3)]);
    diag[l] = s;
}

// dinv = 1/d off the Dirichlet set, 0 on it (info bit 7).
__global__ void invert_masked_kernel(int64_t n, const uint8_t *__restrict__ info,
                                     double *__restrict__ d)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    d[l] = (info[l] & 0x80) ? 0.0 : 1.0 / d[l];
}

__global__ void mul_kernel(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                           double *__restrict__ out)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l < n) out[l] = a[l] * b[l];
}

__global__ void sine_source_kernel(int64_t n, const double *__restrict__ xyz,
                                   double *__restrict__ f)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    f[l] = 3.0 * M_PI * M_PI * sin(M_PI * xyz[l]) * sin(M_PI * xyz[n + l]) *
           sin(M_PI * xyz[2 * n + l]);
}

// g(6, N^3, E) with the factor index fastest (the layout of the operator's
// g argument in Section II-B) to one plane per factor, [E][6][N^3]: a block
// stages 256 nodes' six factors, contiguous in the source, in LDS and
// writes them plane by plane, consecutive nodes of a plane being
// contiguous in the target.
constexpr int kRepackNodes = 256;
typedef double dpair __attribute__((ext_vector_type(2)));

__global__ void __launch_bounds__(kRepackNodes)
repack_g_kernel(int64_t n, int N3, const double *__restrict__ src, double *__restrict__ dst)
{
    __shared__ double s[6 * kRepackNodes + 6];
    const int64_t l0 = (int64_t)blockIdx.x * kRepackNodes;
    const int64_t left = n - l0;
    const int cnt = left < kRepackNodes ? (int)left : kRepackNodes;
    for (int q = threadIdx.x; q < 6 * cnt; q += kRepackNodes)
        s[q] = __builtin_nontemporal_load(src + 6 * l0 + q);
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
        const int64_t l = l0 + threadIdx.x;
        const int64_t e = l / N3, p = l - e * N3;
#pragma unroll
        for (int f = 0; f < 6; ++f)
            __builtin_nontemporal_store(s[6 * threadIdx.x + f], dst + gp_index(e, f, p, N3));
    }
}

// [E][6][N^3] planes to planes of factor pairs: thread (e, h, p) joins
// factors 2h and 2h+1 of node p (both reads and the write coalesce).
__global__ void __launch_bounds__(256)
pair_factors_kernel(int64_t n3e, int N3, const double *__restrict__ src, double *__restrict__ dst)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (e*3 + h)*N3 + p
    if (q >= n3e) return;
    const int64_t eh = q / N3, p = q - eh * N3;
    dpair v;
    v.x = __builtin_nontemporal_load(src + (2 * eh) * N3 + p);
    v.y = __builtin_nontemporal_load(src + (2 * eh + 1) * N3 + p);
    __builtin_nontemporal_store(v, reinterpret_cast<dpair *>(dst) + q);
}

int make_tab(int N, GllTab &tab)
{
    int st = gll_host(N, tab.xi, tab.w);
    if (st != NBX_OK) return st;
    double D[kMaxN * kMaxN];
    deriv_host(N, tab.xi, D);
    for (int q = 0; q < N * N; ++q) tab.D[q] = D[q];
    return NBX_OK;
}

int geom_launch(int N, int64_t E, const BrickDesc &brick, const double *xyz_in, double *G,
                double *bm, double *xyz_out, hipStream_t s)
{
    GllTab tab{};
    int st = make_tab(N, tab);
    if (st != NBX_OK) return st;
    if (E == 0) return NBX_OK;
    if (E > 0x7fffffffLL) return NBX_EUNSUPPORTED;
    const size_t shm = 3 * sizeof(double) * N * N * N;
    NBX_HIP(hipFuncSetAttribute((const void *)geom_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    hipLaunchKernelGGL(geom_kernel, dim3((unsigned)E), dim3(256), shm, s, N, E, tab, brick,
                       xyz_in, G, bm, xyz_out);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

int jacobi_diag_launch(const double *G, const double *D, int N, int64_t E, double *diag,
                       hipStream_t s)
{
    const int64_t n = E * (int64_t)N * N * N;
    if (n == 0) return NBX_OK;
    hipLaunchKernelGGL(jacobi_diag_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, N, E,
                       G, D, diag);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

int jacobi_setup_impl(const double *G, const double *D, int N, int64_t E, const GsPlan &gs,
                      double *dinv, hipStream_t s)
{
    int st = jacobi_diag_launch(G, D, N, E, dinv, s);
    if (st != NBX_OK) return st;
    st = dssum_launch<double>(gs, dinv, 0, s);
    if (st != NBX_OK) return st;
    const int64_t n = gs.n_local;
    if (n == 0) return NBX_OK;
    hipLaunchKernelGGL(invert_masked_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, n,
                       gs.info, dinv);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

}  // namespace nbx

using namespace nbx;

extern "C" int nbx_gll(int N, double *xi_host, double *w_host)
{
    if (!xi_host || !w_host) return NBX_EINVAL;
    return gll_host(N, xi_host, w_host);
}

extern "C" int nbx_deriv(int N, double *D_host)
{
    if (!D_host || N < 2 || N > kMaxN) return NBX_EINVAL;
    double xi[kMaxN], w[kMaxN];
    int st = gll_host(N, xi, w);
    if (st != NBX_OK) return st;
    deriv_host(N, xi, D_host);
    return NBX_OK;
}

extern "C" int nbx_geom_brick(int ex, int ey, int ez, int N, const double *deform_host,
                              double *G, double *bm, double *xyz, void *stream)
{
    if (ex < 1 || ey < 1 || ez < 1 || N < 2 || N > kMaxN || !G) return NBX_EINVAL;
    BrickDesc b{};
    b.ex = ex; b.ey = ey; b.ez = ez;
    for (int q = 0; q < 12; ++q) b.def[q] = deform_host ? deform_host[q] : (q % 4 ? 1.0 : 0.0);
    const int64_t E = (int64_t)ex * ey * ez;
    return geom_launch(N, E, b, nullptr, G, bm, xyz, as_stream(stream));
}

extern "C" int nbx_geom(const double *xyz, int N, int64_t E, double *G, double *bm,
                        void *stream)
{
    if (!xyz || !G || N < 2 || N > kMaxN || E < 0) return NBX_EINVAL;
    BrickDesc b{};
    b.ex = b.ey = b.ez = 1;
    return geom_launch(N, E, b, xyz, G, bm, nullptr, as_stream(stream));
}

extern "C" int nbx_repack_g_aos_to_soa(const double *g_aos, double *g_soa, int N, int64_t E,
                                       void *stream)
{
    if (N < 2 || N > kMaxN || E < 0) return NBX_EINVAL;
    if (E == 0) return NBX_OK;
    if (!g_aos || !g_soa) return NBX_EINVAL;
    const int N3 = N * N * N;
    const int64_t n = E * N3;
    if ((n + kRepackNodes - 1) / kRepackNodes > 0x7fffffffLL) return NBX_EUNSUPPORTED;
    // the two arrays must not overlap
    const uintptr_t a = (uintptr_t)g_aos, b = (uintptr_t)g_soa,
                    bytes = (uintptr_t)(6 * n) * sizeof(double);
    if (a < b + bytes && b < a + bytes) return NBX_EINVAL;
    hipLaunchKernelGGL(repack_g_kernel, dim3((unsigned)((n + kRepackNodes - 1) / kRepackNodes)),
                       dim3(kRepackNodes), 0, as_stream(stream), n, N3, g_aos, g_soa);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

namespace nbx {

int pair_factors_launch(const double *g6, double *g_pairs, int N, int64_t E, hipStream_t s)
{
    const int N3 = N * N * N;
    const int64_t n3e = 3 * E * N3;
    if (n3e == 0) return NBX_OK;
    if ((n3e + 255) / 256 > 0x7fffffffLL) return NBX_EUNSUPPORTED;
    hipLaunchKernelGGL(pair_factors_kernel, dim3((unsigned)((n3e + 255) / 256)), dim3(256), 0, s,
                       n3e, N3, g6, g_pairs);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}

}  // namespace nbx

extern "C" int nbx_pair_factors(const double *g6, double *g_pairs, int N, int64_t E,
                                void *stream)
{
    if (N < 2 || N > kMaxN || E < 0) return NBX_EINVAL;
    if (E == 0) return NBX_OK;
    if (!g6 || !g_pairs) return NBX_EINVAL;
    const uintptr_t a = (uintptr_t)g6, b = (uintptr_t)g_pairs,
                    bytes = (uintptr_t)(6 * E * (int64_t)N * N * N) * sizeof(double);
    if (a < b + bytes && b < a + bytes) return NBX_EINVAL;
    return pair_factors_launch(g6, g_pairs, N, E, as_stream(stream));
}

extern "C" int nbx_brick_ids(int ex, int ey, int ez, int N, int64_t *gid_host,
                             uint8_t *bnd_host)
{
    if (ex < 1 || ey < 1 || ez < 1 || N < 2 || N > kMaxN || !gid_host) return NBX_EINVAL;
    const int64_t Gx = (int64_t)ex * (N - 1) + 1, Gy = (int64_t)ey * (N - 1) + 1,
                  Gz = (int64_t)ez * (N - 1) + 1;
    int64_t l = 0;
    for (int c = 0; c < ez; ++c)
        for (int b = 0; b < ey; ++b)
            for (int a = 0; a < ex; ++a)
                for (int k = 0; k < N; ++k)
                    for (int j = 0; j < N; ++j)
                        for (int i = 0; i < N; ++i, ++l) {
                            const int64_t I = (int64_t)a * (N - 1) + i;
                            const int64_t J = (int64_t)b * (N - 1) + j;
                            const int64_t K = (int64_t)c * (N - 1) + k;
                            gid_host[l] = (K * Gy + J) * Gx + I;
                            if (bnd_host)
                                bnd_host[l] = (I == 0 || J == 0 || K == 0 || I == Gx - 1 ||
                                               J == Gy - 1 || K == Gz - 1) ? 1 : 0;
                        }
    return NBX_OK;
}

extern "C" int nbx_jacobi_setup(const double *G, const double *D, int N, int64_t E,
                                nbx_gs *gs, double *dinv, void *stream)
{
    if (!G || !D || !gs || !dinv || N < 2 || N > kMaxN || E < 0) return NBX_EINVAL;
    if (gs->plan.n_local != E * (int64_t)N * N * N) return NBX_EINVAL;
    return jacobi_setup_impl(G, D, N, E, gs->plan, dinv, as_stream(stream));
}

extern "C" int nbx_rhs(nbx_gs *gs, const double *bm, const double *f, int64_t n_local,
                       double *b, void *stream)
{
    if (!gs || !bm || !f || !b || n_local != gs->plan.n_local) return NBX_EINVAL;
    hipStream_t s = as_stream(stream);
    if (n_local == 0) return NBX_OK;
    hipLaunchKernelGGL(mul_kernel, dim3(blocks_for(n_local, 256)), dim3(256), 0, s, n_local,
                       bm, f, b);
    NBX_LAUNCH_CHECK();
    return dssum_launch<double>(gs->plan, b, 1, s);
}

extern "C" int nbx_sine_source(const double *xyz, int64_t n, double *f, void *stream)
{
    if (n < 0 || (n > 0 && (!xyz || !f))) return NBX_EINVAL;
    if (n == 0) return NBX_OK;
    hipLaunchKernelGGL(sine_source_kernel, dim3(blocks_for(n, 256)), dim3(256), 0,
                       as_stream(stream), n, xyz, f);
    NBX_LAUNCH_CHECK();
    return NBX_OK;
}
