// ax.hip -- C-ABI front end of the AX operator (Section II-B, Listing 1):
// argument checks, the per-(precision, N) tile table that the autotuner
// fills, and the launch wrappers the solvers use.  The kernel itself is in
// ax_kernel.hpp; its instantiations are in ax_f64.hip, ax_f32.hip,
// ax_pcg.hip, ax_f16.hip and ax_bf16.hip so that they compile in parallel.
#include "internal.hpp"

#include <atomic>

namespace nbx {

int ax_launch_f64_tiled(int N, int epb, const double *u, const double *G, const double *D,
                        double *w, int64_t E, hipStream_t s);
int ax_launch_f32_tiled(int N, int epb, const float *u, const float *G, const double *D,
                        float *w, int64_t E, hipStream_t s);
int ax_launch_f64_planes_tiled(int N, int epb, const double *u, const double *G,
                               const double *D, double *w, int64_t E, hipStream_t s);
int ax_launch_f32_planes_tiled(int N, int epb, const float *u, const float *G, const double *D,
                               float *w, int64_t E, hipStream_t s);
int ax_pcg_launch_f64_tiled(int N, int epb, const double *G, const double *D, int64_t E,
                            const double *z, double *p, double *w, double *part,
                            const double *scal, hipStream_t s);
int ax_pcg_launch_f32_tiled(int N, int epb, const float *G, const double *D, int64_t E,
                            const float *z, float *p, float *w, double *part,
                            const double *scal, hipStream_t s);
int ax16_mfma_launch(int planes, const double *u, const double *G, const double *D, double *w,
                     int64_t E, hipStream_t s);
int ax16_mfma_pcg_launch(const double *Gp, const double *D, int64_t E, const double *z,
                         double *p, double *w, double *part, const double *scal, hipStream_t s);
int ax_launch_g_f16(int N, int epb, const float *u, const void *G, const float *gscale,
                    const double *D, float *w, int64_t E, hipStream_t s);
int ax_launch_g_bf16(int N, int epb, const float *u, const void *G, const float *gscale,
                     const double *D, float *w, int64_t E, hipStream_t s);
int ax_pcg_launch_g_f16(int N, int epb, const void *G, const float *gscale, const double *D,
                        int64_t E, const float *z, float *p, float *w, double *part,
                        const double *scal, hipStream_t s);
int ax_pcg_launch_g_bf16(int N, int epb, const void *G, const float *gscale, const double *D,
                         int64_t E, const float *z, float *p, float *w, double *part,
                         const double *scal, hipStream_t s);

namespace {

// Elements per workgroup by [kind][operator][N]; kind 0 is the plain
// operator (nbx_ax), kind 1 the solvers' fused first stage (p update, AX,
// <p,w> partials), whose register and LDS use differ; operator 0 FP64, 1
// FP32, 2 FP32 arithmetic on 16-bit G (FP16 and BF16 storage share it).
// Defaults: two elements per block where a block's three LDS slabs stay
// small (measured best at N = 10 in FP64), one for the large elements.
std::atomic<int> g_tile[2][3][kMaxN + 1];
std::atomic<bool> g_tile_init{false};

void init_tiles()
{
    if (g_tile_init.load()) return;
    for (int k = 0; k < 2; ++k)
        for (int p = 0; p < 3; ++p)
            for (int n = 0; n <= kMaxN; ++n) {
                int e = n <= 6 ? 4 : (n <= 12 ? 2 : 1);
                g_tile[k][p][n].store(e);
            }
    g_tile_init.store(true);
}

int prec_slot(int prec) { return prec == NBX_F64 ? 0 : (prec == NBX_F32 ? 1 : 2); }

bool valid_epb(int epb) { return epb == 1 || epb == 2 || epb == 4 || epb == 8; }

// The host side of AxShape::fits: LDS and thread count of a tile.
bool tile_fits(int prec, int N, int epb)
{
    const int64_t N2 = N * N, N3 = N2 * N, nt = (epb * N2 + 63) / 64 * 64;
    const int64_t word = prec == NBX_F64 ? 8 : 4;
    return nt <= 1024 && (3 * epb * N3 + N2) * word + (nt / 64) * 8 <= 160 * 1024;
}

}  // namespace

int ax_tile(int prec, int N)
{
    init_tiles();
    return g_tile[0][prec_slot(prec)][N].load();
}

int pcg_tile(int prec, int N)
{
    init_tiles();
    return g_tile[1][prec_slot(prec)][N].load();
}

int ax_blocks(int prec, int N, int64_t E)
{
    const int epb = pcg_tile(prec, N);
    return (int)((E + epb - 1) / epb);
}

int ax_launch_f64(const double *u, const double *G, const double *D, int N, int64_t E,
                  double *w, hipStream_t s)
{
    return ax_launch_f64_tiled(N, ax_tile(NBX_F64, N), u, G, D, w, E, s);
}

int ax_launch_f32(const float *u, const float *G, const double *D, int N, int64_t E,
                  float *w, hipStream_t s)
{
    return ax_launch_f32_tiled(N, ax_tile(NBX_F32, N), u, G, D, w, E, s);
}

int ax_pcg_launch_f64(const double *G, const double *D, int N, int64_t E, const double *z,
                      double *p, double *w, double *part, const double *scal, hipStream_t s)
{
    // N = 16: the matrix-core body, one element and one partial per
    // workgroup (the only tile that fits there, so ax_blocks agrees)
    if (N == 16) return ax16_mfma_pcg_launch(G, D, E, z, p, w, part, scal, s);
    return ax_pcg_launch_f64_tiled(N, pcg_tile(NBX_F64, N), G, D, E, z, p, w, part, scal, s);
}

int ax_pcg_launch_f32(const float *G, const double *D, int N, int64_t E, const float *z,
                      float *p, float *w, double *part, const double *scal, hipStream_t s)
{
    return ax_pcg_launch_f32_tiled(N, pcg_tile(NBX_F32, N), G, D, E, z, p, w, part, scal, s);
}

int ax_launch_g16(int gprec, const float *u, const void *G16, const float *gscale,
                  const double *D, int N, int64_t E, float *w, hipStream_t s)
{
    const int epb = ax_tile(NBX_F16, N);
    return gprec == NBX_F16 ? ax_launch_g_f16(N, epb, u, G16, gscale, D, w, E, s)
                            : ax_launch_g_bf16(N, epb, u, G16, gscale, D, w, E, s);
}

int ax_pcg_launch_g16(int gprec, const void *G16, const float *gscale, const double *D, int N,
                      int64_t E, const float *z, float *p, float *w, double *part,
                      const double *scal, hipStream_t s)
{
    const int epb = pcg_tile(NBX_F16, N);
    return gprec == NBX_F16
               ? ax_pcg_launch_g_f16(N, epb, G16, gscale, D, E, z, p, w, part, scal, s)
               : ax_pcg_launch_g_bf16(N, epb, G16, gscale, D, E, z, p, w, part, scal, s);
}

}  // namespace nbx

using namespace nbx;

static int ax_check(int prec, const void *u, const void *G, const double *D, int N, int64_t E,
                    void *w)
{
    if (N < 2 || N > kMaxN || E < 0) return NBX_EINVAL;
    if (E == 0) return NBX_OK;
    if (!u || !G || !D || !w || u == w) return NBX_EINVAL;
    if (prec != NBX_F64 && prec != NBX_F32) return NBX_EUNSUPPORTED;
    return 1;   // proceed
}

// The C ABI's operator: G in one plane per factor, [E][6][N^3].
static int ax_planes(int prec, const void *u, const void *G, const double *D, int N, int64_t E,
                     void *w, int epb, hipStream_t s)
{
    if (prec == NBX_F64)
        return ax_launch_f64_planes_tiled(N, epb, (const double *)u, (const double *)G, D,
                                          (double *)w, E, s);
    return ax_launch_f32_planes_tiled(N, epb, (const float *)u, (const float *)G, D,
                                      (float *)w, E, s);
}

// The same operator on factor pairs, [E][3][N^3][2] (the solvers' layout).
static int ax_pairs(int prec, const void *u, const void *G, const double *D, int N, int64_t E,
                    void *w, int epb, hipStream_t s)
{
    if (prec == NBX_F64)
        return ax_launch_f64_tiled(N, epb, (const double *)u, (const double *)G, D, (double *)w,
                                   E, s);
    return ax_launch_f32_tiled(N, epb, (const float *)u, (const float *)G, D, (float *)w, E, s);
}

extern "C" int nbx_ax(int prec, const void *u, const void *G, const double *D, int N,
                      int64_t E, void *w, void *stream)
{
    const int c = ax_check(prec, u, G, D, N, E, w);
    if (c != 1) return c;
    // FP64 at N = 16: the r and s contractions on the matrix cores
    if (prec == NBX_F64 && N == 16)
        return ax16_mfma_launch(1, (const double *)u, (const double *)G, D, (double *)w, E,
                                as_stream(stream));
    return ax_planes(prec, u, G, D, N, E, w, ax_tile(prec, N), as_stream(stream));
}

extern "C" int nbx_ax_tiled(int prec, const void *u, const void *G, const double *D, int N,
                            int64_t E, void *w, int epb, void *stream)
{
    if (!valid_epb(epb)) return NBX_EINVAL;
    const int c = ax_check(prec, u, G, D, N, E, w);
    if (c != 1) return c;
    return ax_planes(prec, u, G, D, N, E, w, epb, as_stream(stream));
}

extern "C" int nbx_ax_paired(int prec, const void *u, const void *Gp, const double *D, int N,
                             int64_t E, void *w, void *stream)
{
    const int c = ax_check(prec, u, Gp, D, N, E, w);
    if (c != 1) return c;
    if (prec == NBX_F64 && N == 16)
        return ax16_mfma_launch(0, (const double *)u, (const double *)Gp, D, (double *)w, E,
                                as_stream(stream));
    return ax_pairs(prec, u, Gp, D, N, E, w, ax_tile(prec, N), as_stream(stream));
}

extern "C" int nbx_ax_paired_tiled(int prec, const void *u, const void *Gp, const double *D,
                                   int N, int64_t E, void *w, int epb, void *stream)
{
    if (!valid_epb(epb)) return NBX_EINVAL;
    const int c = ax_check(prec, u, Gp, D, N, E, w);
    if (c != 1) return c;
    return ax_pairs(prec, u, Gp, D, N, E, w, epb, as_stream(stream));
}

static int set_tile(int kind, int prec, int N, int epb)
{
    if (N < 2 || N > kMaxN || !valid_epb(epb)) return NBX_EINVAL;
    if (prec != NBX_F64 && prec != NBX_F32 && prec != NBX_F16 && prec != NBX_BF16)
        return NBX_EUNSUPPORTED;
    if (!tile_fits(prec, N, epb)) return NBX_EUNSUPPORTED;
    init_tiles();
    g_tile[kind][prec_slot(prec)][N].store(epb);
    return NBX_OK;
}

static int get_tile(int kind, int prec, int N)
{
    if (N < 2 || N > kMaxN) return NBX_EINVAL;
    if (prec != NBX_F64 && prec != NBX_F32 && prec != NBX_F16 && prec != NBX_BF16)
        return NBX_EUNSUPPORTED;
    return kind == 0 ? ax_tile(prec, N) : pcg_tile(prec, N);
}

extern "C" int nbx_ax_set_tile(int prec, int N, int epb) { return set_tile(0, prec, N, epb); }
extern "C" int nbx_ax_get_tile(int prec, int N) { return get_tile(0, prec, N); }
extern "C" int nbx_pcg_set_tile(int prec, int N, int epb) { return set_tile(1, prec, N, epb); }
extern "C" int nbx_pcg_get_tile(int prec, int N) { return get_tile(1, prec, N); }
