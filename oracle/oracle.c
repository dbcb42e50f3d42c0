/*
 * oracle.c -- plain FP64 CPU oracle for the spectral-element Poisson path
 * (matrix-free AX operator, direct stiffness summation, Jacobi-PCG).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP path.
 *
 * Everything is IEEE double, built with -O2 -ffp-contract=off so that no
 * multiply-add is fused behind the reader's back.  OpenMP is used only
 * across independent elements (AX, geometry, diagonal) or across fixed
 * element blocks whose partial sums are combined in block order, so every
 * result is independent of the thread count.
 *
 * Sources, by function:
 *   ora_ax ........ the operator's definition w_e = D^T G_e D u_e
 *                   (Section II-B): gradient by the collocation derivative
 *                   along each direction, contraction with the symmetric
 *                   six-factor matrix, transposed gradient; written as
 *                   explicit index sums.
 *   ora_gll, ora_deriv, ora_geom, ora_brick_*, ora_gs_*, ora_jacobi_diag,
 *   ora_pcg_* ..... the paper names these (Section II-B: CG with a simple
 *                   preconditioner on a block geometry, nearest-neighbour
 *                   exchange, global reductions) without defining them;
 *                   they follow the standard spectral-element definitions
 *                   (Gauss-Lobatto-Legendre collocation, isoparametric
 *                   geometric factors, Jacobi-preconditioned CG).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX3(i, j, k, N) ((i) + (N) * ((j) + (N) * (k)))

/* ------------------------------------------------------------------ GLL */

/* Legendre polynomial P_p and its derivative at x by the three-term
 * recurrence (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1} and
 * P'_{n+1} = P'_{n-1} + (2n+1) P_n. */
static void legendre(int p, double x, double *P, double *dP)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (p == 0) { *P = 1.0; *dP = 0.0; return; }
    for (int n = 1; n < p; ++n) {
        double p2 = ((2.0 * n + 1.0) * x * p1 - n * p0) / (n + 1.0);
        double d2 = d0 + (2.0 * n + 1.0) * p1;
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    *P = p1; *dP = d1;
}

/* Gauss-Lobatto-Legendre nodes and weights for N points (degree p=N-1):
 * the end points -1, +1 and the roots of P'_p, found by Newton's method
 * on P'_p (P''_p from Legendre's equation) from Chebyshev-Gauss-Lobatto
 * starting guesses; weights w_i = 2 / (p (p+1) P_p(xi_i)^2).
 * Returns 0, or -1 if N < 2 or Newton fails to converge. */
int ora_gll(int N, double *xi, double *w)
{
    if (N < 2) return -1;
    int p = N - 1;
    xi[0] = -1.0; xi[p] = 1.0;
    for (int i = 1; i < p; ++i) {
        double x = -cos(M_PI * (double)i / (double)p);
        int ok = 0;
        for (int it = 0; it < 200; ++it) {
            double P, dP;
            legendre(p, x, &P, &dP);
            double d2P = (2.0 * x * dP - p * (p + 1.0) * P) / (1.0 - x * x);
            double dx = dP / d2P;
            x -= dx;
            if (fabs(dx) <= 1e-16 * (1.0 + fabs(x))) { ok = 1; break; }
        }
        if (!ok) return -1;
        xi[i] = x;
    }
    for (int i = 0; i < N; ++i) {
        double P, dP;
        legendre(p, xi[i], &P, &dP);
        w[i] = 2.0 / (p * (p + 1.0) * P * P);
    }
    return 0;
}

/* Collocation derivative matrix, row-major: D[a*N+b] = l_b'(xi_a), where
 * l_b is the Lagrange polynomial through the GLL nodes that is 1 at xi_b.
 * Closed form: P_p(xi_a) / (P_p(xi_b) (xi_a - xi_b)) off the diagonal,
 * -p(p+1)/4 and +p(p+1)/4 at the two end points, 0 elsewhere on the
 * diagonal. */
void ora_deriv(int N, const double *xi, double *D)
{
    int p = N - 1;
    double *Pv = (double *)malloc(sizeof(double) * N);
    for (int a = 0; a < N; ++a) { double dP; legendre(p, xi[a], &Pv[a], &dP); }
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            double v;
            if (a != b) v = Pv[a] / (Pv[b] * (xi[a] - xi[b]));
            else if (a == 0) v = -p * (p + 1.0) / 4.0;
            else if (a == p) v = p * (p + 1.0) / 4.0;
            else v = 0.0;
            D[a * N + b] = v;
        }
    free(Pv);
}

/* ----------------------------------------------------------------- mesh */

/* Physical node coordinates of an ex*ey*ez brick on [0,1]^3.  Element
 * (a,b,c) is e = a + ex*(b + ey*c); its node (i,j,k) sits at the reference
 * position X = (a + (xi_i+1)/2)/ex (likewise Y, Z) and is moved by
 * c = C + A_c sin(k1 pi X) sin(k2 pi Y) sin(k3 pi Z) for each coordinate,
 * deform[c*4 + {0,1,2,3}] = {A_c, k1, k2, k3}. */
void ora_brick_coords(int ex, int ey, int ez, int N, const double *xi,
                      const double *deform, double *x, double *y, double *z)
{
    int64_t E = (int64_t)ex * ey * ez, N3 = (int64_t)N * N * N;
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        int a = (int)(e % ex), b = (int)((e / ex) % ey), c = (int)(e / ((int64_t)ex * ey));
        for (int k = 0; k < N; ++k)
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i) {
                    double X = (a + 0.5 * (xi[i] + 1.0)) / ex;
                    double Y = (b + 0.5 * (xi[j] + 1.0)) / ey;
                    double Z = (c + 0.5 * (xi[k] + 1.0)) / ez;
                    double ref[3] = {X, Y, Z}, out[3];
                    for (int q = 0; q < 3; ++q) {
                        const double *t = deform + 4 * q;
                        out[q] = ref[q] + t[0] * sin(t[1] * M_PI * X) *
                                 sin(t[2] * M_PI * Y) * sin(t[3] * M_PI * Z);
                    }
                    int64_t l = e * N3 + IDX3(i, j, k, N);
                    x[l] = out[0]; y[l] = out[1]; z[l] = out[2];
                }
    }
}

/* Isoparametric geometric factors.  The reference derivatives of the
 * nodal coordinates are taken with D (x_r = sum_m D[i][m] x(m,j,k), etc.),
 * J = d(x,y,z)/d(r,s,t), and with W = w_i w_j w_k the six stored factors
 * are W det(J) (grad r_a . grad r_b) in the order rr, rs, rt, ss, st, tt
 * (Listing 1: g(1..6) = G_11, G_12, G_13, G_22, G_23, G_33).  Layout
 * G[e][f][node].  bm[e][node] = W det(J) (the diagonal mass).  Returns
 * the minimum det(J) seen (negative means a folded element). */
double ora_geom(int N, int64_t E, const double *D, const double *wts,
                const double *x, const double *y, const double *z,
                double *G, double *bm)
{
    int64_t N3 = (int64_t)N * N * N;
    double jmin = INFINITY;
    #pragma omp parallel for schedule(static) reduction(min : jmin)
    for (int64_t e = 0; e < E; ++e) {
        const double *X[3] = {x + e * N3, y + e * N3, z + e * N3};
        for (int k = 0; k < N; ++k)
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i) {
                    double J[3][3];   /* J[q][a] = d x_q / d r_a */
                    for (int q = 0; q < 3; ++q) {
                        double dr = 0, ds = 0, dt = 0;
                        for (int m = 0; m < N; ++m) {
                            dr += D[i * N + m] * X[q][IDX3(m, j, k, N)];
                            ds += D[j * N + m] * X[q][IDX3(i, m, k, N)];
                            dt += D[k * N + m] * X[q][IDX3(i, j, m, N)];
                        }
                        J[q][0] = dr; J[q][1] = ds; J[q][2] = dt;
                    }
                    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
                               - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
                               + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                    /* rows of inv(J) are grad r, grad s, grad t */
                    double Ji[3][3];
                    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
                    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
                    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
                    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
                    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
                    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
                    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
                    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
                    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
                    double W = wts[i] * wts[j] * wts[k];
                    double s = W * det;
                    static const int fa[6] = {0, 0, 0, 1, 1, 2};
                    static const int fb[6] = {0, 1, 2, 1, 2, 2};
                    int64_t n = IDX3(i, j, k, N);
                    for (int f = 0; f < 6; ++f) {
                        double dot = Ji[fa[f]][0] * Ji[fb[f]][0] + Ji[fa[f]][1] * Ji[fb[f]][1]
                                   + Ji[fa[f]][2] * Ji[fb[f]][2];
                        G[(e * 6 + f) * N3 + n] = s * dot;
                    }
                    if (bm) bm[e * N3 + n] = s;
                    if (det < jmin) jmin = det;
                }
    }
    return jmin;
}

/* Global node numbering of the brick: node (i,j,k) of element (a,b,c) is
 * global grid point (I,J,K) = (a(N-1)+i, b(N-1)+j, c(N-1)+k) of a
 * Gx x Gy x Gz grid, Gx = ex(N-1)+1, id = I + Gx (J + Gy K).  bnd = 1 for
 * points on the boundary of the unit cube (homogeneous Dirichlet). */
void ora_brick_ids(int ex, int ey, int ez, int N, int64_t *gid, uint8_t *bnd)
{
    int64_t E = (int64_t)ex * ey * ez, N3 = (int64_t)N * N * N;
    int64_t Gx = (int64_t)ex * (N - 1) + 1, Gy = (int64_t)ey * (N - 1) + 1,
            Gz = (int64_t)ez * (N - 1) + 1;
    for (int64_t e = 0; e < E; ++e) {
        int64_t a = e % ex, b = (e / ex) % ey, c = e / ((int64_t)ex * ey);
        for (int k = 0; k < N; ++k)
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i) {
                    int64_t I = a * (N - 1) + i, J = b * (N - 1) + j, K = c * (N - 1) + k;
                    int64_t l = e * N3 + IDX3(i, j, k, N);
                    gid[l] = I + Gx * (J + Gy * K);
                    bnd[l] = (I == 0 || I == Gx - 1 || J == 0 || J == Gy - 1 ||
                              K == 0 || K == Gz - 1);
                }
    }
}

/* ------------------------------------------------------------------- AX */

/* One element of the operator, written out from its definition
 * w_e = D^T G_e D u_e (Section II-B): the reference-space gradient of u
 * (the collocation derivative D applied along r, s and t), the symmetric
 * contraction with the node's factor matrix [[g1,g2,g3],[g2,g4,g5],
 * [g3,g5,g6]], and the transposed gradient
 *   w(i,j,k) = sum_m D[m][i] vr(m,j,k) + D[m][j] vs(i,m,k) + D[m][k] vt(i,j,m).
 * D is row-major, D[a*N+b] = l_b'(xi_a).  Every sum runs over m in
 * ascending order.  v holds 3 N^3 doubles of scratch. */
static void ax_elem(double *w, const double *u, const double *g, int N, const double *D,
                    double *v)
{
    const int64_t N3 = (int64_t)N * N * N;
    double *vr = v, *vs = v + N3, *vt = v + 2 * N3;
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                double ur = 0.0, us = 0.0, ut = 0.0;
                for (int m = 0; m < N; ++m) ur += D[i * N + m] * u[IDX3(m, j, k, N)];
                for (int m = 0; m < N; ++m) us += D[j * N + m] * u[IDX3(i, m, k, N)];
                for (int m = 0; m < N; ++m) ut += D[k * N + m] * u[IDX3(i, j, m, N)];
                const int64_t q = IDX3(i, j, k, N);
                const double g1 = g[q], g2 = g[N3 + q], g3 = g[2 * N3 + q];
                const double g4 = g[3 * N3 + q], g5 = g[4 * N3 + q], g6 = g[5 * N3 + q];
                vr[q] = g1 * ur + g2 * us + g3 * ut;
                vs[q] = g2 * ur + g4 * us + g5 * ut;
                vt[q] = g3 * ur + g5 * us + g6 * ut;
            }
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                double acc = 0.0;
                for (int m = 0; m < N; ++m) acc += D[m * N + i] * vr[IDX3(m, j, k, N)];
                for (int m = 0; m < N; ++m) acc += D[m * N + j] * vs[IDX3(i, m, k, N)];
                for (int m = 0; m < N; ++m) acc += D[m * N + k] * vt[IDX3(i, j, m, N)];
                w[IDX3(i, j, k, N)] = acc;
            }
}

/* ax: w(:,e) = A_e u(:,e) for every element; G is [E][6][N^3]. */
void ora_ax(int N, int64_t E, const double *u, const double *G, const double *D, double *w)
{
    const int64_t N3 = (int64_t)N * N * N;
    #pragma omp parallel
    {
        double *v = (double *)malloc(sizeof(double) * 3 * N3);
        #pragma omp for schedule(static)
        for (int64_t e = 0; e < E; ++e)
            ax_elem(w + e * N3, u + e * N3, G + e * 6 * N3, N, D, v);
        free(v);
    }
}

/* ---------------------------------------------------- gather-scatter */

typedef struct {
    int64_t n_local, n_groups;
    int64_t *off;      /* [n_groups+1] */
    int64_t *idx;      /* [n_local] local indices, grouped by global id,
                          ascending within a group */
} ora_gs;

/* Groups every local node with the other copies of its global node (a
 * counting sort on the global id, stable, so each group lists its local
 * indices in ascending order). */
ora_gs *ora_gs_create(const int64_t *gid, int64_t n_local)
{
    int64_t gmax = -1;
    for (int64_t l = 0; l < n_local; ++l) if (gid[l] > gmax) gmax = gid[l];
    int64_t ng = gmax + 1;
    int64_t *cnt = (int64_t *)calloc((size_t)ng + 1, sizeof(int64_t));
    for (int64_t l = 0; l < n_local; ++l) cnt[gid[l] + 1]++;
    for (int64_t g = 0; g < ng; ++g) cnt[g + 1] += cnt[g];
    ora_gs *gs = (ora_gs *)malloc(sizeof(ora_gs));
    gs->n_local = n_local; gs->n_groups = ng;
    gs->off = cnt;
    gs->idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_local > 0 ? n_local : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ng > 0 ? ng : 1));
    for (int64_t g = 0; g < ng; ++g) fill[g] = cnt[g];
    for (int64_t l = 0; l < n_local; ++l) gs->idx[fill[gid[l]]++] = l;
    free(fill);
    return gs;
}

void ora_gs_free(ora_gs *gs)
{
    if (!gs) return;
    free(gs->off); free(gs->idx); free(gs);
}

/* dssum: for every global node, s = sum of its local copies in ascending
 * local index, then every copy <- s. */
void ora_dssum(const ora_gs *gs, double *v)
{
    for (int64_t g = 0; g < gs->n_groups; ++g) {
        int64_t b = gs->off[g], e = gs->off[g + 1];
        if (e - b < 2) continue;
        double s = 0.0;
        for (int64_t q = b; q < e; ++q) s += v[gs->idx[q]];
        for (int64_t q = b; q < e; ++q) v[gs->idx[q]] = s;
    }
}

/* Homogeneous Dirichlet mask: zero every local node whose global node
 * lies on the boundary. */
void ora_mask(const uint8_t *bnd, int64_t n_local, double *v)
{
    for (int64_t l = 0; l < n_local; ++l) if (bnd[l]) v[l] = 0.0;
}

/* Multiplicity m_l (number of local copies of l's global node). */
void ora_multiplicity(const ora_gs *gs, double *m)
{
    for (int64_t g = 0; g < gs->n_groups; ++g) {
        int64_t b = gs->off[g], e = gs->off[g + 1];
        for (int64_t q = b; q < e; ++q) m[gs->idx[q]] = (double)(e - b);
    }
}

/* ----------------------------------------------------------- Jacobi */

/* Diagonal of each element matrix A_e = sum_{a,b} D_a^T diag(G_ab) D_b,
 * D_r = I x I x D, D_s = I x D x I, D_t = D x I x I (i fastest):
 *   diag_p = sum_m D[m][i]^2 g1(m,j,k) + sum_m D[m][j]^2 g4(i,m,k)
 *          + sum_m D[m][k]^2 g6(i,j,m) + 2 D[i][i] D[j][j] g2(p)
 *          + 2 D[i][i] D[k][k] g3(p) + 2 D[j][j] D[k][k] g5(p). */
void ora_jacobi_diag(int N, int64_t E, const double *G, const double *D, double *diag)
{
    int64_t N3 = (int64_t)N * N * N;
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        const double *g = G + e * 6 * N3;
        for (int k = 0; k < N; ++k)
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i) {
                    double s = 0.0;
                    for (int m = 0; m < N; ++m) s += D[m * N + i] * D[m * N + i] * g[IDX3(m, j, k, N)];
                    for (int m = 0; m < N; ++m) s += D[m * N + j] * D[m * N + j] * g[3 * N3 + IDX3(i, m, k, N)];
                    for (int m = 0; m < N; ++m) s += D[m * N + k] * D[m * N + k] * g[5 * N3 + IDX3(i, j, m, N)];
                    int64_t p = IDX3(i, j, k, N);
                    s += 2.0 * D[i * N + i] * D[j * N + j] * g[N3 + p];
                    s += 2.0 * D[i * N + i] * D[k * N + k] * g[2 * N3 + p];
                    s += 2.0 * D[j * N + j] * D[k * N + k] * g[4 * N3 + p];
                    diag[e * N3 + p] = s;
                }
    }
}

/* --------------------------------------------------------------- PCG */

/* Weighted dot <a,b>_c = sum_l c_l a_l b_l (c = 1/multiplicity counts every
 * global node once).  Neumaier-compensated sums over fixed blocks of
 * ORA_BLOCK local nodes, then over the block results in block order:
 * deterministic for any thread count. */
#define ORA_BLOCK 65536
static double neumaier_add(double s, double x, double *comp)
{
    double t = s + x;
    if (fabs(s) >= fabs(x)) *comp += (s - t) + x;
    else *comp += (x - t) + s;
    return t;
}

double ora_wdot(int64_t n, const double *c, const double *a, const double *b)
{
    int64_t nb = (n + ORA_BLOCK - 1) / ORA_BLOCK;
    double *part = (double *)malloc(sizeof(double) * (size_t)(nb > 0 ? nb : 1));
    #pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < nb; ++q) {
        int64_t lo = q * ORA_BLOCK, hi = lo + ORA_BLOCK < n ? lo + ORA_BLOCK : n;
        double s = 0.0, comp = 0.0;
        for (int64_t l = lo; l < hi; ++l) s = neumaier_add(s, c[l] * a[l] * b[l], &comp);
        part[q] = s + comp;
    }
    double s = 0.0, comp = 0.0;
    for (int64_t q = 0; q < nb; ++q) s = neumaier_add(s, part[q], &comp);
    free(part);
    return s + comp;
}

typedef struct {
    int N; int64_t E;
    const double *G, *D;
    const ora_gs *gs;
    const uint8_t *bnd;
    const double *dinv, *c;
} ora_problem;

/* w = mask(dssum(AX(p))) */
static void apply_A(const ora_problem *P, const double *p, double *w)
{
    int64_t n = P->E * (int64_t)P->N * P->N * P->N;
    ora_ax(P->N, P->E, p, P->G, P->D, w);
    ora_dssum(P->gs, w);
    ora_mask(P->bnd, n, w);
}

/* One or more iterations of Jacobi-preconditioned CG from the state
 * (x, r, z, p, rho) where p is the next search direction and
 * rho = <r,z>_c.  Per iteration:
 *   w = mask(dssum(AX(p)));  pap = <p,w>_c;  alpha = rho/pap;
 *   x += alpha p;  r -= alpha w;  (stop if <r,r>_c <= rtol^2 <b,b>_c)
 *   z = dinv r;  rho' = <r,z>_c;  beta = rho'/rho;  p = z + beta p.
 * w is caller scratch.  hist (optional) receives sqrt(<r,r>_c) after each
 * iteration.  Returns the number of iterations done; *state is 0 if the
 * iteration limit was reached, 1 on convergence, 2 on breakdown
 * (pap <= 0, rho <= 0 or a non-finite scalar). */
int ora_pcg_iterate(int N, int64_t E, const double *G, const double *D,
                    const ora_gs *gs, const uint8_t *bnd, const double *dinv,
                    const double *c, double *x, double *r, double *z, double *p,
                    double *w, double *rho_io, int max_iter, double stop_rr,
                    double *hist, int *state)
{
    ora_problem P = {N, E, G, D, gs, bnd, dinv, c};
    int64_t n = E * (int64_t)N * N * N;
    double rho = *rho_io;
    int k;
    *state = 0;
    for (k = 0; k < max_iter; ++k) {
        apply_A(&P, p, w);
        double pap = ora_wdot(n, c, p, w);
        if (!(pap > 0.0) || !isfinite(pap)) { *state = 2; break; }
        double alpha = rho / pap;
        #pragma omp parallel for schedule(static)
        for (int64_t l = 0; l < n; ++l) { x[l] += alpha * p[l]; r[l] -= alpha * w[l]; }
        double rr = ora_wdot(n, c, r, r);
        if (hist) hist[k] = sqrt(rr);
        if (rr <= stop_rr) { *state = 1; ++k; break; }
        #pragma omp parallel for schedule(static)
        for (int64_t l = 0; l < n; ++l) z[l] = dinv[l] * r[l];
        double rho2 = ora_wdot(n, c, r, z);
        if (!(rho2 > 0.0) || !isfinite(rho2)) { *state = 2; ++k; break; }
        double beta = rho2 / rho;
        rho = rho2;
        #pragma omp parallel for schedule(static)
        for (int64_t l = 0; l < n; ++l) p[l] = z[l] + beta * p[l];
    }
    *rho_io = rho;
    return k;
}

/* Full solve from x = 0: r = b, z = dinv r, p = z, rho = <r,z>_c, then
 * ora_pcg_iterate until <r,r>_c <= rtol^2 <b,b>_c or max_iter.  x, r, z,
 * p, w are caller-owned arrays of n_local doubles. */
int ora_pcg(int N, int64_t E, const double *G, const double *D,
            const ora_gs *gs, const uint8_t *bnd, const double *dinv,
            const double *c, const double *b, double *x, double *r, double *z,
            double *p, double *w, int max_iter, double rtol, double *hist,
            int *state, double *relres)
{
    int64_t n = E * (int64_t)N * N * N;
    for (int64_t l = 0; l < n; ++l) { x[l] = 0.0; r[l] = b[l]; z[l] = dinv[l] * r[l]; p[l] = z[l]; }
    double bb = ora_wdot(n, c, b, b);
    double rho = ora_wdot(n, c, r, z);
    int it = ora_pcg_iterate(N, E, G, D, gs, bnd, dinv, c, x, r, z, p, w, &rho,
                             max_iter, rtol * rtol * bb, hist, state);
    double rr = ora_wdot(n, c, r, r);
    if (relres) *relres = bb > 0 ? sqrt(rr / bb) : 0.0;
    return it;
}

/* Thread count OpenMP would use (for reporting). */
int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------- single precision --
 * The same operator and exchange in IEEE single arithmetic, for the
 * iterative-refinement oracle (reduced precision is the paper's stated
 * further work, Section V): ax_elem's sums in float, D rounded to float. */

static void ax_elem_f(float *w, const float *u, const float *g, int N, const float *D,
                      float *v)
{
    const int64_t N3 = (int64_t)N * N * N;
    float *vr = v, *vs = v + N3, *vt = v + 2 * N3;
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                float ur = 0.0f, us = 0.0f, ut = 0.0f;
                for (int m = 0; m < N; ++m) ur += D[i * N + m] * u[IDX3(m, j, k, N)];
                for (int m = 0; m < N; ++m) us += D[j * N + m] * u[IDX3(i, m, k, N)];
                for (int m = 0; m < N; ++m) ut += D[k * N + m] * u[IDX3(i, j, m, N)];
                const int64_t q = IDX3(i, j, k, N);
                const float g1 = g[q], g2 = g[N3 + q], g3 = g[2 * N3 + q];
                const float g4 = g[3 * N3 + q], g5 = g[4 * N3 + q], g6 = g[5 * N3 + q];
                vr[q] = g1 * ur + g2 * us + g3 * ut;
                vs[q] = g2 * ur + g4 * us + g5 * ut;
                vt[q] = g3 * ur + g5 * us + g6 * ut;
            }
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                float acc = 0.0f;
                for (int m = 0; m < N; ++m) acc += D[m * N + i] * vr[IDX3(m, j, k, N)];
                for (int m = 0; m < N; ++m) acc += D[m * N + j] * vs[IDX3(i, m, k, N)];
                for (int m = 0; m < N; ++m) acc += D[m * N + k] * vt[IDX3(i, j, m, N)];
                w[IDX3(i, j, k, N)] = acc;
            }
}

/* w = AX(u) in single precision; D is the double matrix rounded to float. */
void ora_ax_f32(int N, int64_t E, const float *u, const float *G, const double *D, float *w)
{
    const int64_t N3 = (int64_t)N * N * N;
    float *Df = (float *)malloc(sizeof(float) * N * N);
    for (int q = 0; q < N * N; ++q) Df[q] = (float)D[q];
    #pragma omp parallel
    {
        float *v = (float *)malloc(sizeof(float) * 3 * N3);
        #pragma omp for schedule(static)
        for (int64_t e = 0; e < E; ++e)
            ax_elem_f(w + e * N3, u + e * N3, G + e * 6 * N3, N, Df, v);
        free(v);
    }
    free(Df);
}

/* dssum in single precision, ascending local index. */
void ora_dssum_f32(const ora_gs *gs, float *v)
{
    for (int64_t g = 0; g < gs->n_groups; ++g) {
        int64_t b = gs->off[g], e = gs->off[g + 1];
        if (e - b < 2) continue;
        float s = 0.0f;
        for (int64_t q = b; q < e; ++q) s += v[gs->idx[q]];
        for (int64_t q = b; q < e; ++q) v[gs->idx[q]] = s;
    }
}
