/*
 * nbx.h -- C ABI of libnbx, the MI355X (gfx950) library for the
 * spectral-element Poisson hot path studied in N. Brown, "Exploring the
 * acceleration of Nekbone on reconfigurable architectures" (arXiv
 * 2011.04981): the matrix-free operator AX (Section II-B, Listing 1),
 * direct stiffness summation, and the Jacobi-preconditioned conjugate
 * gradient solve built on them (Section II-B: CG with a simple
 * preconditioner, nearest-neighbour exchange and global reductions).
 *
 * General conventions (every entry point):
 *   - Return value: an nbx_status (0 = NBX_OK).  No C++ exception crosses
 *     this boundary.  After NBX_EHIP, nbx_last_hip_error() gives the raw
 *     hipError_t.
 *   - Pointers named *_host are host memory; every other array pointer is
 *     device memory (hipMalloc / torch CUDA tensors), 16-byte aligned.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Calls documented "async" only enqueue work on `stream` and return;
 *     they never allocate or synchronise.
 *   - The caller owns every array it passes.  The library owns only what a
 *     *_create call allocates, released by the matching *_destroy.
 *   - A handle must not be used from two host threads at once.
 *
 * Layouts (Section II-B, Listing 1, column-major u(i,j,k,e)):
 *   u, w, vectors : [E][N][N][N], i fastest: u[((e*N + k)*N + j)*N + i]
 *   G             : [E][6][N^3], one plane per factor: factor f (0-based,
 *                   g_(f+1) of the listing, the symmetric matrix
 *                   [[g1,g2,g3],[g2,g4,g5],[g3,g5,g6]]) of node q of
 *                   element e at G[(e*6 + f)*N^3 + q] (6*E*N^3 values).
 *                   nbx_repack_g_aos_to_soa converts from the listing's
 *                   g(6,N^3,E), the six factors of a node contiguous.
 *   Gp            : the same factors as three planes of factor pairs per
 *                   element, (g1,g2), (g3,g4), (g5,g6), one pair per node,
 *                   at Gp[((e*3 + f/2)*N^3 + q)*2 + f%2], written
 *                   [E][3][N^3][2]: the layout inside a problem, where a
 *                   lane of the fused operator fetches a pair with one
 *                   16-byte load.  Only nbx_ax_paired / nbx_ax_paired_tiled
 *                   take it; nbx_pair_factors converts G to it.
 *   D             : N x N row-major, D[a*N + b] = l_b'(xi_a) (the
 *                   listing's dxm1; its transpose dxtm1 is derived inside)
 *   N             : Gauss-Lobatto-Legendre nodes per direction (degree N-1),
 *                   2 <= N <= 16.
 *   Brick meshes  : element (a,b,c) of an ex x ey x ez brick on [0,1]^3 is
 *                   e = a + ex*(b + ey*c).
 */
#ifndef NBX_H
#define NBX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { NBX_F64 = 0, NBX_F32 = 1, NBX_BF16 = 2, NBX_F16 = 3 } nbx_prec;

typedef enum {
    NBX_OK = 0,
    NBX_NOT_CONVERGED = 1,   /* solve hit max_iter before rtol */
    NBX_EINVAL = -1,         /* bad argument (null pointer, N out of range, E < 0) */
    NBX_EUNSUPPORTED = -2,   /* valid but not implemented (precision, size) */
    NBX_EHIP = -3,           /* a HIP runtime call failed */
    NBX_ENOMEM = -4,         /* a *_create allocation failed */
    NBX_EBREAKDOWN = -5      /* CG breakdown: <p,Ap> <= 0, <r,z> <= 0 or non-finite */
} nbx_status;

/* Text for a status code (static storage). */
const char *nbx_status_str(int status);
/* Raw hipError_t of the most recent NBX_EHIP on this thread. */
int nbx_last_hip_error(void);
/* Library version, 100*major + minor. */
int nbx_version(void);

/* dst[0..n) = src[0..n) with 16-byte accesses (a plain streaming copy of
 * known size: the reference point for achievable HBM bandwidth and for
 * calibrating hardware byte counters).  Async.  src, dst device, no
 * overlap. */
int nbx_copy_f64(const double *src, double *dst, int64_t n, void *stream);

/* Further achievable-bandwidth references over n doubles (n even), one
 * 16-byte vector per lane with non-temporal accesses: mode 0 copies src to
 * dst; mode 1 only reads src (sink, one device double, is written only in
 * an impossible case, so no bytes are stored).  Async.  NBX_EINVAL for odd
 * n, another mode or null pointers. */
int nbx_stream_f64(int mode, const double *src, double *dst, int64_t n, double *sink,
                   void *stream);

/* ------------------------------------------------------------ set-up --
 * The paper names the geometry ("block or linear geometry", Section II-B)
 * but not its discretisation; these calls build it with the standard
 * spectral-element definitions. */

/* Gauss-Lobatto-Legendre nodes xi_host[N] (ascending, -1..1) and weights
 * w_host[N].  Host only.  NBX_EINVAL if N < 2 or N > 16. */
int nbx_gll(int N, double *xi_host, double *w_host);

/* Derivative matrix D_host[N*N] (row-major, D[a*N+b] = l_b'(xi_a)) for the
 * GLL nodes.  Host only. */
int nbx_deriv(int N, double *D_host);

/* Geometric factors of a deformed brick, computed on the device (async).
 * deform_host[12] = {A_x,k1,k2,k3, A_y,k1,k2,k3, A_z,k1,k2,k3}: coordinate
 * c of the node at undeformed position (X,Y,Z) is
 * C + A_c sin(k1 pi X) sin(k2 pi Y) sin(k3 pi Z).  Outputs (device):
 * G[E][6][N^3] = w_i w_j w_k det(J) (grad r_a . grad r_b) from
 * isoparametric derivatives, in the [E][6][N^3] layout above,
 * bm[E][N^3] = w_i w_j w_k det(J) (may be NULL), xyz[3][E][N^3] node
 * coordinates (may be NULL). */
int nbx_geom_brick(int ex, int ey, int ez, int N, const double *deform_host,
                   double *G, double *bm, double *xyz, void *stream);

/* Same factors from arbitrary node coordinates xyz[3][E][N^3] (device,
 * async).  bm may be NULL. */
int nbx_geom(const double *xyz, int N, int64_t E, double *G, double *bm, void *stream);

/* Repacks geometric factors given in the layout of the operator's g
 * argument (Section II-B: g(6, N^3, E), the six factors of a node
 * contiguous, g_aos[(e*N^3 + p)*6 + f]) into the layout every other call
 * takes, one plane per factor (g_soa[(e*6 + f)*N^3 + p]).
 * nbx_pair_factors turns such planes, g6 = G[E][6][N^3], into the factor
 * pairs of nbx_ax_paired (g_pairs[((e*3 + f/2)*N^3 + p)*2 + f%2]).
 * f = 0..5 for g1..g6.  Device arrays of 6*E*N^3 doubles each,
 * caller-owned; they must not overlap (NBX_EINVAL).  Async on stream, no
 * allocation; E = 0 is a no-op.  NBX_EINVAL for N outside [2, 16], E < 0 or
 * a null pointer. */
int nbx_repack_g_aos_to_soa(const double *g_aos, double *g_soa, int N, int64_t E,
                            void *stream);
int nbx_pair_factors(const double *g6, double *g_pairs, int N, int64_t E, void *stream);

/* Global node ids of the brick's local nodes (gid_host[E*N^3]) and the
 * homogeneous Dirichlet flags (bnd_host[E*N^3] = 1 on the cube's
 * boundary).  Host only. */
int nbx_brick_ids(int ex, int ey, int ez, int N, int64_t *gid_host, uint8_t *bnd_host);

/* ---------------------------------------------------------------- AX --
 * w_e = D^T G_e D u_e for every element e in [0,E) (Section II-B,
 * Listing 1: local_grad3, the geometric contraction, local_grad3_t).
 * G is [E][6][N^3] (the listing's g with the element and node indices
 * outermost, see Layouts).  Async; no allocation.  prec selects the storage
 * and arithmetic type of u, G, w: NBX_F64 (double), NBX_F32 (float, FP32
 * arithmetic).  D is always double (converted inside).  u and w must not
 * overlap.  E == 0 is a no-op.  NBX_EINVAL for null pointers, N outside
 * [2,16] or E < 0; NBX_EUNSUPPORTED for other precisions.
 * FP64 at N = 16 (the paper's element size, Table II) runs the r and s
 * contractions on the matrix cores (FP64 products, one workgroup per
 * element); its results agree with the vector-unit kernel (nbx_ax_tiled) to
 * FP64 rounding, not bit for bit.  Every other (prec, N) runs the vector-unit
 * kernel with the tile table's tile. */
int nbx_ax(int prec, const void *u, const void *G, const double *D, int N, int64_t E,
           void *w, void *stream);

/* nbx_ax with an explicit tile: epb elements per workgroup (1, 2, 4 or 8)
 * of the vector-unit kernel, at every N (FP64 N = 16 included).
 * Every tile computes bit-identical results; tiles differ only in speed.
 * NBX_EINVAL for another epb, NBX_EUNSUPPORTED if the tile's LDS would
 * exceed 160 KB or its workgroup 1024 threads. */
int nbx_ax_tiled(int prec, const void *u, const void *G, const double *D, int N, int64_t E,
                 void *w, int epb, void *stream);

/* The same operator on factor pairs Gp[E][3][N^3][2] (see Layouts): three
 * 16-byte factor loads per node instead of six 8-byte ones, the form the
 * solvers use inside a problem.  Results are bit-identical to nbx_ax /
 * nbx_ax_tiled on the same factors (FP64 at N = 16 runs nbx_ax's
 * matrix-core kernel here too).  Arguments and errors as there. */
int nbx_ax_paired(int prec, const void *u, const void *Gp, const double *D, int N, int64_t E,
                  void *w, void *stream);
int nbx_ax_paired_tiled(int prec, const void *u, const void *Gp, const double *D, int N,
                        int64_t E, void *w, int epb, void *stream);

/* The tile nbx_ax and nbx_ax_paired use for (prec, N) (process-wide; set by the
 * autotuner).  get returns epb or a negative status; set refuses a tile
 * that does not fit (NBX_EUNSUPPORTED, as nbx_ax_tiled).  prec NBX_F64,
 * NBX_F32, or NBX_F16 / NBX_BF16 for the one table of the 16-bit-G kernels
 * (nbx_ax_g16 and the inner iterations of NBX_F16 / NBX_BF16 solves). */
int nbx_ax_set_tile(int prec, int N, int epb);
int nbx_ax_get_tile(int prec, int N);
/* The tile of the solvers' fused first stage (p = z + beta p, w = AX(p),
 * per-workgroup <p,w> partials) for (prec, N): nbx_pcg, nbx_pcg_iterate,
 * nbx_pcg_batched, nbx_pcg_learned.  The partials follow the workgroups, so
 * a solve's rounding (not its correctness) depends on this tile; standalone
 * and batched solves share it and agree bit for bit. */
int nbx_pcg_set_tile(int prec, int N, int epb);
int nbx_pcg_get_tile(int prec, int N);

/* The reduced-storage operator for the inner iterations of a mixed-
 * precision solve.  Half precision and fixed point are the paper's further
 * work (Section V); G is 48 of AX's 64 bytes per node in FP64.
 *
 * nbx_g16_pack: per element e, gscale[e] = 2^(floor(log2 m_e) - 14) with
 * m_e = max |G_e| (1 if G_e is zero), and the 16-bit word of factor f at
 * node q, round(round32(G[e][f][q] / gscale[e])) with both roundings to
 * nearest-even, first to FP32, then to gprec = NBX_F16 (IEEE binary16) or
 * NBX_BF16 (bfloat16), stored at G16[((e*3 + f/2)*N^3 + q)*2 + f%2]: three
 * planes per element of 32-bit words holding the factor pairs (g1,g2),
 * (g3,g4), (g5,g6) of a node, low half first.  G (FP64, [E][6][N^3]), G16
 * (6*E*N^3 16-bit words, 4-byte aligned) and gscale ([E] float) are device
 * arrays.  Async.
 *
 * nbx_ax_g16: w = AX(u) in FP32 arithmetic with the factors
 * gscale[e] * G16_e (u, w float [E][N^3]); bit-identical to FP32 AX with
 * those dequantised factors.  Async; tiles as nbx_ax with NBX_F32.
 * Both: NBX_EINVAL for null pointers, N outside [2,16], E < 0, u == w;
 * NBX_EUNSUPPORTED for another gprec. */
int nbx_g16_pack(int gprec, const double *G, int N, int64_t E, void *G16, float *gscale,
                 void *stream);
int nbx_ax_g16(int gprec, const float *u, const void *G16, const float *gscale,
               const double *D, int N, int64_t E, float *w, void *stream);

/* The FP32 operator on matrix cores, the reduced-precision option of the
 * inner iterations: per element, the six length-N contractions are
 * 16x16x4 FP32 matrix-core products of D (or D^T, N padded to 16) with the
 * element's values arranged with the contracted index inside; one 64-lane
 * workgroup per element, values staged in LDS.  gprec NBX_F32: G is FP32
 * [E][6][N^3] (gscale unused, may be NULL); NBX_F16 / NBX_BF16: G16 and
 * gscale from nbx_g16_pack.  u, w float [E][N^3].  FP32 products, FP32
 * accumulation: the FP32 kernels' accuracy, not their bits.  Async; no
 * allocation.  NBX_EINVAL for null pointers, N outside [2,16], E < 0,
 * u == w; NBX_EUNSUPPORTED for another gprec. */
int nbx_ax_mfma(int gprec, const float *u, const void *G, const float *gscale, const double *D,
                int N, int64_t E, float *w, void *stream);

/* ------------------------------------------------ gather-scatter (dssum) --
 * The "nearest-neighbour communication" step of a CG iteration (Section
 * II-B), on one GPU: local copies of a global node are summed and the sum
 * written back to every copy. */
typedef struct nbx_gs nbx_gs;

/* Builds the gather-scatter plan from host global ids (gid_host[n_local],
 * equal ids = same global node) and Dirichlet flags (dirichlet_host[n_local],
 * nonzero = on the Dirichlet boundary; may be NULL for none).  Allocates
 * device arrays and uploads them on `stream`; returns once the plan is on
 * the device (synchronous).  NBX_EINVAL for a null gid_host with
 * n_local > 0, n_local < 0 or a null out; NBX_EUNSUPPORTED if
 * n_local >= 2^31 or a node has more than 127 copies. */
int nbx_gs_create(const int64_t *gid_host, int64_t n_local, const uint8_t *dirichlet_host,
                  nbx_gs **out, void *stream);
int nbx_gs_destroy(nbx_gs *gs);

/* In place: v_l <- sum of v over l's global node, summed in ascending local
 * index (every copy gets identical bits).  apply_mask != 0 then zeroes
 * Dirichlet nodes.  Async; prec NBX_F64 or NBX_F32. */
int nbx_dssum(nbx_gs *gs, int prec, void *v, int apply_mask, void *stream);

/* Multiplicity (number of copies) of every local node as double, device
 * out[n_local].  Async. */
int nbx_gs_multiplicity(nbx_gs *gs, double *out, void *stream);

/* ------------------------------------------------------------ Jacobi --
 * The "simple preconditioner" (Section II-B) read as Jacobi: dinv =
 * 1 / dssum(diag(A_e)), 0 on Dirichlet nodes.  Async. */
int nbx_jacobi_setup(const double *G, const double *D, int N, int64_t E, nbx_gs *gs,
                     double *dinv, void *stream);

/* Manufactured source f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z) at the nodes
 * xyz[3][n] (device), for which u* = sin(pi x) sin(pi y) sin(pi z) solves
 * -lap u = f with u = 0 on the unit cube's boundary.  Async. */
int nbx_sine_source(const double *xyz, int64_t n, double *f, void *stream);

/* Assembled load vector b = mask(dssum(bm * f)) for nodal source values f
 * (device, [E][N^3]).  Async. */
int nbx_rhs(nbx_gs *gs, const double *bm, const double *f, int64_t n_local, double *b,
            void *stream);

/* --------------------------------------------------------------- PCG -- */
typedef struct nbx_problem nbx_problem;

/* Binds D, N, E and a gather-scatter plan (caller-owned; they must outlive
 * the problem), copies G ([E][6][N^3]) into the problem's own factor-pair
 * layout (6*E*N^3 doubles; G itself may be freed afterwards), computes dinv
 * on the device and allocates the solver workspace (four vectors,
 * reduction partials, scalars).  Synchronous.  NBX_ENOMEM if device memory
 * runs out. */
int nbx_problem_create(const double *G, const double *D, int N, int64_t E, nbx_gs *gs,
                       nbx_problem **out, void *stream);
int nbx_problem_destroy(nbx_problem *p);
/* Copies the problem's dinv into out[n_local] (device).  Async. */
int nbx_problem_dinv(nbx_problem *p, double *out, void *stream);
/* The exchange of the solvers' iterations (Section II-B's nearest-neighbour
 * exchange): at nbx_problem_create the two-copy, non-Dirichlet groups of
 * x faces (node a with a % N == N-1, the last node of an element row, and
 * node a + d, d = N^3 - N + 1, the first node of the same row in the next
 * element) leave the gather-scatter plan, and the solvers' update step
 * sums them in the exchange's own order, so results are bit-identical to
 * the full exchange.  out[0] = groups of the full plan, out[1] = groups the
 * solvers' exchange keeps, out[2] = d (0 when no pair was taken and the
 * solvers use the full plan), out[3] = out[4] = 0 (y and z face pairs stay
 * in the exchange).  Host memory; synchronous, no GPU work.  NBX_EINVAL for
 * null arguments. */
int nbx_problem_exchange_info(nbx_problem *p, int64_t out[5]);

/* Length of the device scalar block used by nbx_pcg_iterate. */
#define NBX_SCAL_LEN 16
/* scal[] slots: */
#define NBX_S_RHO 0      /* <r,z>_c */
#define NBX_S_BETA 1     /* beta applied at the start of the next iteration */
#define NBX_S_ALPHA 2
#define NBX_S_PAP 3      /* <p,Ap>_c */
#define NBX_S_RR 4       /* <r,r>_c after the last iteration */
#define NBX_S_BB 5       /* <b,b>_c */
#define NBX_S_STOP 6     /* stop when RR <= STOP (negative: never) */
#define NBX_S_FLAG 7     /* 0 running, 1 converged, 2 breakdown, 3 MAXIT reached */
#define NBX_S_ITER 8     /* iterations completed */
#define NBX_S_MAXIT 9    /* FLAG becomes 3 when ITER reaches this */

/* Advances a Jacobi-PCG state by up to n_iter iterations (async; no
 * allocation).  State on entry: x, r, z (= dinv r), p (previous search
 * direction; finite), scal[RHO] = <r,z>_c, scal[BETA], scal[STOP],
 * scal[FLAG] = 0.  Each iteration:
 *   p = z + beta p;  w = mask(dssum(AX(p)));  alpha = rho / <p,w>_c;
 *   x += alpha p;  r -= alpha w;  stop if <r,r>_c <= STOP;
 *   z = dinv r;  rho' = <r,z>_c;  beta = rho'/rho.
 * <a,b>_c weights each local node by 1/multiplicity.  Once FLAG != 0 the
 * remaining iterations do nothing (FLAG = 3 when ITER reaches MAXIT).
 * Vectors are [E][N^3] doubles; every vector and scal must be distinct
 * from the problem's own workspace. */
int nbx_pcg_iterate(nbx_problem *p, double *x, double *r, double *z, double *pdir,
                    double *scal, int n_iter, void *stream);

/* Partial sums that nbx_pcg_iterate_noalloc can hold: one per workgroup
 * of the fused first stage, ceil(E / tile) with the FP64 tile of
 * nbx_pcg_get_tile (4 MB of device memory per GPU in all). */
#define NBX_NOALLOC_MAX_BLOCKS 262144

/* nbx_pcg_iterate without a problem handle and without any allocation, for
 * callers that cannot allocate device memory: code under stream capture,
 * tight serving loops, harnesses that forbid it.  The caller passes
 * everything the iterations read and write: the factors as factor pairs
 * Gp[E][3][N^3][2] (nbx_pair_factors), D, a plan gs for E N^3 local nodes,
 * dinv (e.g. from nbx_jacobi_setup), the state x, r, z, pdir and scal as
 * for nbx_pcg_iterate, and w[E][N^3], which receives A p of the last step
 * (unspecified after a step that breaks down).
 * The reduction partials live in a fixed device array per GPU (looked up on
 * the first call on each device): every call on one GPU shares it, so calls
 * that overlap on one GPU race; nothing needs clearing between calls.
 * Same kernels, order and results as nbx_pcg_iterate.  Async; allocates
 * nothing and calls no allocating routine.  NBX_EINVAL for null pointers,
 * N outside [2, 16], E < 1 or a plan of another size; NBX_EUNSUPPORTED if
 * ceil(E / tile) exceeds NBX_NOALLOC_MAX_BLOCKS. */
int nbx_pcg_iterate_noalloc(const double *Gp, const double *D, int N, int64_t E, nbx_gs *gs,
                            const double *dinv, double *x, double *r, double *z, double *pdir,
                            double *w, double *scal, int n_iter, void *stream);

typedef struct {
    int max_iter;        /* iteration cap (default 1000) */
    int fixed_iters;     /* nonzero: run exactly max_iter iterations, no test */
    int check_every;     /* iterations per graph launch between host checks */
    int use_graph;       /* nonzero: replay iterations from a captured hipGraph */
    double rtol;         /* stop when ||r||_c <= rtol ||b||_c */
    int prec;            /* NBX_F64: plain FP64 PCG; NBX_F32: FP32 iteration
                            with FP64 residuals (see mixed_mode);
                            NBX_F16 / NBX_BF16: the same with the inner
                            operator's G in 16 bits (nbx_g16_pack) */
    double inner_rtol;   /* mixed_mode 0: residual reduction per reliable
                            update (e.g. 0.1); mixed_mode 1: relative
                            tolerance of each inner solve (e.g. 1e-5) */
    int max_outer;       /* cap on reliable updates / refinement steps */
    int mixed_mode;      /* 0: one FP32 Krylov sequence with FP64 reliable
                            updates; 1: restarted iterative refinement */
    int inner_mfma;      /* nonzero: the FP32 iterations' operator on matrix
                            cores (nbx_ax_mfma's kernel) instead of the
                            vector-unit kernel; standalone solves only
                            (nbx_pcg_batched returns NBX_EUNSUPPORTED) */
} nbx_pcg_opts;

typedef struct {
    int iters;           /* total (inner) CG iterations */
    int outer_iters;     /* refinement steps (1 for plain PCG) */
    double relres;       /* ||r||_c / ||b||_c of the recurrence residual */
    double true_relres;  /* ||b - A x||_c / ||b||_c recomputed in FP64 */
    int fell_back;       /* a fallback solver was used */
    int flag;            /* 0 limit, 1 converged, 2 breakdown */
    double seconds;      /* wall time of the iteration loop */
} nbx_pcg_result;

/* Fills opts with defaults. */
void nbx_pcg_default_opts(nbx_pcg_opts *opts);

/* Solves A x = b from x = 0 (b, x device [E][N^3] doubles).  Synchronous:
 * returns after convergence, breakdown or max_iter, with res filled.
 * Returns NBX_OK, NBX_NOT_CONVERGED or NBX_EBREAKDOWN. */
int nbx_pcg(nbx_problem *p, const double *b, double *x, const nbx_pcg_opts *opts,
            nbx_pcg_result *res, void *stream);

/* Solves nprob independent problems (each with its own N, E, G, plan and
 * workspace) together: every fused step of the FP64 Jacobi-PCG iteration is
 * one launch serving all unconverged problems, replayed from a captured
 * hipGraph of check_every iterations (the elements of independent problems
 * are independent work, as the paper distributes independent elements over
 * kernels, Section IV).  probs, b and x are host arrays of nprob handles /
 * device pointers; results[nprob] is filled per problem (seconds = the whole
 * batch); solve_seconds[nprob] (may be NULL) receives each problem's time
 * from the batch start to its convergence on the device clock.  With
 * opts->prec NBX_F32, NBX_F16 or NBX_BF16 (mixed_mode 0, reliable updates;
 * mixed_mode 1 gives NBX_EUNSUPPORTED) the FP32 iterations of all problems
 * run together the same way and each problem's FP64 residual replacement
 * follows between replays; solve_seconds is then taken on the host when a
 * problem's last step ends.  Results are bit-identical to nbx_pcg with the
 * same options on each problem alone.  Synchronous.  Returns NBX_OK if
 * every problem converged, else NBX_NOT_CONVERGED or NBX_EBREAKDOWN.  A
 * problem must not appear twice. */
int nbx_pcg_batched(nbx_problem *const *probs, const double *const *b, double *const *x,
                    int nprob, const nbx_pcg_opts *opts, nbx_pcg_result *results,
                    double *solve_seconds, void *stream);

/* ------------------------------------------- element-local network (BF16) --
 * Matrix-core kernels for the learned preconditioner's network (reduced
 * precision is the paper's further work, Section V; the network itself is
 * not in the paper).  BF16 values are passed as raw 16-bit words
 * (uint16_t arrays); accumulation is FP32. */

/* C[M x N] (FP32, row-major, ldc) = op(A)[M x K] op(B)[K x N] with BF16
 * operands: A(m,k) = trans_a ? A[k*lda + m] : A[m*lda + k], B(k,n) =
 * trans_b ? B[n*ldb + k] : B[k*ldb + n].  M, N multiples of 64, K a
 * multiple of 32, lda and ldb multiples of 8, otherwise NBX_EINVAL.
 * Async. */
int nbx_gemm_bf16(int trans_a, int trans_b, int M, int N, int K, const void *A, int lda,
                  const void *B, int ldb, float *C, int ldc, void *stream);

typedef struct nbx_mlp nbx_mlp;

/* A 3-layer perceptron n_in -> n_hidden -> n_hidden -> n_out with ReLU,
 * for batches of up to max_batch rows (multiple of 64; n_hidden a multiple
 * of 64).  Inputs and outputs are padded to in_pad / out_pad (multiples of
 * 64).  Parameters live in one FP32 arena of n_params floats:
 * W1[n_hidden][in_pad], b1[n_hidden], W2[n_hidden][n_hidden], b2[n_hidden],
 * W3[out_pad][n_hidden], b3[out_pad] (row-major, W[out][in]); a BF16 copy
 * feeds the products.  Allocates; synchronous.  All parameters start at 0. */
int nbx_mlp_create(int n_in, int n_hidden, int n_out, int max_batch, nbx_mlp **out);
int nbx_mlp_destroy(nbx_mlp *mlp);
int nbx_mlp_shape(nbx_mlp *mlp, int *in_pad, int *out_pad, int64_t *n_params);
/* Copies a parameter arena (device FP32) in, refreshes the BF16 copy and
 * resets the optimiser state.  Async. */
int nbx_mlp_set_params(nbx_mlp *mlp, const float *params, void *stream);
/* Copies the parameters and/or the last gradients out (device, may be
 * NULL).  Async. */
int nbx_mlp_get_params(nbx_mlp *mlp, float *params, float *grads, void *stream);
/* Y[B][out_pad] (FP32) = network(X[B][in_pad] BF16); B a multiple of 64,
 * at most max_batch.  Async. */
int nbx_mlp_forward(nbx_mlp *mlp, const void *X, int B, float *Y, void *stream);
/* Gradients of the mean squared error sum_{b, j < n_out} (Y - T)^2 / (B n_out)
 * for targets T[B][out_pad] (FP32) into the gradient arena; *loss (device,
 * may be NULL) receives the loss.  Async. */
int nbx_mlp_grad(nbx_mlp *mlp, const void *X, const float *T, int B, double *loss,
                 void *stream);
/* nbx_mlp_grad, then one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with
 * learning rate lr on the FP32 master parameters.  Async. */
int nbx_mlp_train_step(nbx_mlp *mlp, const void *X, const float *T, int B, float lr,
                       double *loss, void *stream);

/* ------------------------------- learned element-interior preconditioner --
 * Not in the paper, which uses a "simple preconditioner" (Section II-B,
 * read as Jacobi).  The learned operator keeps Jacobi on every node except
 * each element's learned nodes S: its interior nodes (1 <= i,j,k <= N-2)
 * with a single copy, off the Dirichlet set.  On them
 *     z_S = (1/gd_e) L^T diag(gamma_e) L r_S,  gamma_e = softplus(f(g_e)),
 * with L an nI x nI matrix shared by all elements (nI = (N-2)^3, interior
 * nodes in their own i-fastest order), f a 3-layer perceptron
 * (6 -> n_hidden -> n_hidden -> nI, ReLU) on the element's six mean
 * geometric factors divided by gd_e, the element mean of g1, g4, g6.
 * L^T diag(gamma) L is symmetric positive semidefinite for any L, and the
 * learned nodes of different elements are disjoint, so the operator is a
 * fixed symmetric positive (semi)definite preconditioner that needs no
 * exchange. */
typedef struct nbx_lpi nbx_lpi;

/* The model: L ([nIp][nIp] FP32, nIp = nI rounded up to 64, zero beyond nI)
 * and the perceptron (an nbx_mlp arena with n_in 6, n_out nI), for training
 * batches of up to max_batch rows (a multiple of 64; n_hidden a multiple of
 * 64).  All parameters start at 0.  Allocates; synchronous.  NBX_EINVAL for
 * N outside [3, 16] or other sizes. */
int nbx_lpi_create(int N, int n_hidden, int max_batch, nbx_lpi **out);
int nbx_lpi_destroy(nbx_lpi *m);
/* nI, nIp and the length of the parameter arena [L | perceptron]. */
int nbx_lpi_shape(nbx_lpi *m, int *nI, int *nIp, int64_t *n_params);
/* Copies a parameter arena (device FP32) in, refreshes the BF16 copies and
 * resets the optimiser state / copies parameters and gradients out (device,
 * either may be NULL).  Async. */
int nbx_lpi_set_params(nbx_lpi *m, const float *params, void *stream);
int nbx_lpi_get_params(nbx_lpi *m, float *params, float *grads, void *stream);
/* Gradient of the mean squared error, over B rows (a multiple of 64, at
 * most max_batch) and the nI outputs, of Z = ((X L^T) * gamma(F)) L against
 * T: X [B][nIp] BF16, T [B][nIp] FP32, F [B][64] BF16 (six features, then
 * zeros).  *loss (device, may be NULL) receives the loss.  BF16 operands,
 * FP32 accumulation.  Async. */
int nbx_lpi_grad(nbx_lpi *m, const void *X, const float *T, const void *F, int B, double *loss,
                 void *stream);
/* Sets every gain bias (the perceptron's last bias) so that a model whose
 * L is the identity and whose last layer is zero is the least-squares
 * scalar map of the B rows (X, T as for nbx_lpi_grad): gamma = s0 with
 * s0 = <X, T> / <X, X> (sums over all entries; 1 if <X, T> <= 0).  The
 * usual start of training.  Async. */
int nbx_lpi_init_scale(nbx_lpi *m, const void *X, const float *T, int B, void *stream);
/* nbx_lpi_grad, then one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with
 * learning rate lr on every FP32 master parameter.  Async. */
int nbx_lpi_train_step(nbx_lpi *m, const void *X, const float *T, const void *F, int B,
                       float lr, double *loss, void *stream);

typedef struct nbx_lp nbx_lp;

/* Binds a problem and a model of the same N (both must outlive the
 * handle): computes each element's features and gd, and gamma for every
 * element from the model's current parameters.  Allocates; synchronous.
 * NBX_EINVAL if the sizes do not match. */
int nbx_lp_create(nbx_problem *p, nbx_lpi *m, nbx_lp **out, void *stream);
int nbx_lp_destroy(nbx_lp *lp);
/* Recomputes gamma after the model's parameters changed.  Synchronous. */
int nbx_lp_refresh(nbx_lp *lp, void *stream);
/* gfeat[E][8]: six normalised factors, gd, 0.  Async. */
int nbx_lp_geom_features(nbx_lp *lp, float *gfeat, void *stream);
/* z = M r (device FP64 vectors, r != z).  Async. */
int nbx_lp_apply(nbx_lp *lp, const double *r, double *z, void *stream);
/* Training rows from the vector v - v0 (device FP64, [E][N^3]; v0 may be
 * NULL for v alone) that the FP64 solver produced, an error x* - x_k or a
 * residual r_k: for the nsel elements in elems (device int32), with
 * s = |v_S| and y_S = A_SS v_S (the element operator on v with every node
 * outside S set to zero, read on S):  X[row] = bf16(y_S / (s gd)),
 * T[row] = v_S / s (0 beyond S and nI), F[row] = bf16 features.  A model
 * with L^T diag(gamma) L = gd A_SS^-1 fits such rows exactly.  An index
 * outside [0, E) or v_S = 0 gives an all-zero row.  Allocates two work
 * vectors on the first call; async after that. */
int nbx_lp_samples(nbx_lp *lp, const double *v, const double *v0, const int32_t *elems,
                   int nsel, void *X, float *T, void *F, void *stream);
/* Copies the recurrence residual of the problem's last solve. Async. */
int nbx_problem_residual(nbx_problem *p, double *r, void *stream);
/* Flexible PCG (Notay 2000, one stored direction: beta = -<z', A p> / <p, A p>,
 * each new direction A-orthogonal to the last; the BF16 products make M
 * linear only to rounding) from x = 0, for at most opts->max_iter
 * iterations.  If it breaks down (<r, M r> or <p, A p> not positive),
 * Jacobi-PCG continues from the current x (from x = 0 if the flexible
 * iterate diverged) for the iterations the budget has left, and
 * res->fell_back = 1; res->iters counts all iterations, res->outer_iters
 * those of the flexible phase.  Synchronous; returns like nbx_pcg. */
int nbx_pcg_learned(nbx_lp *lp, const double *b, double *x, const nbx_pcg_opts *opts,
                    nbx_pcg_result *res, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* NBX_H */
