// solver.hpp -- the solver handle shared by the FP64 PCG driver (pcg.hip)
// and the mixed-precision refinement driver (mixed.hip).
#pragma once

#include "internal.hpp"

struct nbx_problem {
    // G: the problem's own copy of the caller's factors in factor pairs
    // (g_index), the layout of the fused operator; D stays caller-owned.
    const double *G = nullptr, *D = nullptr;
    double *Gown = nullptr;
    int N = 0;
    int64_t E = 0, n = 0;
    nbx_gs *gs = nullptr;
    // FP64 workspace
    double *dinv = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *w = nullptr;
    double *part1 = nullptr, *part3 = nullptr, *scal = nullptr, *tmp2 = nullptr;
    double *h_scal = nullptr;   // pinned host mirror of a scalar block
    hipStream_t ws = nullptr;   // the problem's own stream (default priority)
    hipEvent_t ev = nullptr;
    hipGraphExec_t gexec = nullptr;   // FP64 iterations, captured per (x, chunk, tile)
    const double *g_x = nullptr;
    int g_iters = 0, g_tile = 0;
    // FP32 inner-solve workspace (allocated by the first mixed solve)
    float *G32 = nullptr, *dinv32 = nullptr, *r32 = nullptr, *z32 = nullptr, *p32 = nullptr,
          *w32 = nullptr, *d32 = nullptr;
    double *scal32 = nullptr;
    hipGraphExec_t gexec32 = nullptr;
    int g32_iters = 0, g32_fmt = -1, g32_tile = 0;   // chunk, format, tile of the capture
    // 16-bit factors for the reduced-storage inner operator (NBX_F16 / NBX_BF16)
    uint16_t *G16 = nullptr;
    float *gscale = nullptr;
    int g16_fmt = -1;                  // format G16 currently holds
    int inner_fmt = NBX_F32;           // operator the FP32 iterations use
    int inner_mfma = 0;                // 1: the inner operator on matrix cores
    // The solvers' exchange: the plan without the two-copy x-face groups,
    // whose sums the update kernel forms from w, with their own info bytes
    // (xplan.info, bits as sk::kXpNext / kXpPrev); xd = N^3 - N + 1, the
    // local offset of an x-face pair; xd = 0 when the plan has no such
    // pairs and the solvers use the full plan.
    nbx::GsPlan xplan;
    int64_t xd = 0;
};

namespace nbx {

// The exchange plan of the solvers' iterations: xplan (with the x-face
// pairs summed in the update kernel) when there is one, else the full plan.
inline const GsPlan &iter_plan(const nbx_problem *P) { return P->xd ? P->xplan : P->gs->plan; }

// FP64 residual r = b - mask(dssum(AX(x))) (r may be null) and
// out[0] = <r,r>_c, out[1] = <b,b>_c; synchronous on s.
int residual_f64(nbx_problem *P, const double *b, const double *x, double *r, double out[2],
                 hipStream_t s);

int pcg_f64(nbx_problem *P, const double *b, double *x, const nbx_pcg_opts &o,
            nbx_pcg_result *res);
int pcg_mixed(nbx_problem *P, const double *b, double *x, const nbx_pcg_opts &o,
              nbx_pcg_result *res);
// FP32 inner workspace and the inner operator's factors in format fmt
// (NBX_F32: FP32 copy of G; NBX_F16 / NBX_BF16: 16-bit packed G); sets
// P->inner_fmt.  Synchronous.
int prepare_inner(nbx_problem *P, int fmt, hipStream_t s);

// The mixed solver's reliable-update scheme (mixed_mode 0), in three steps
// so that a batch can run the FP32 iterations of many problems together:
// reliable_start sets x = 0 and the FP32 state from b (async on s); after
// the FP32 iterations of a problem have stopped (h = its FP32 scalar block
// as read on the host), reliable_step folds the correction into x, replaces
// the residual by the FP64 one and applies the stop tests (synchronous on
// s; rs.done once the solve is over); reliable_finish runs the FP64
// fallback if the FP32 sequence broke down or stalled and fills res (all
// but seconds).
struct ReliableState {
    int updates = 0, stalls = 0, fell_back = 0, done = 0;
    double last_true = -1.0;
};
int reliable_start(nbx_problem *P, const double *b, double *x, const nbx_pcg_opts &o,
                   hipStream_t s);
int reliable_step(nbx_problem *P, const double *b, double *x, const nbx_pcg_opts &o,
                  const double *h, ReliableState &rs, hipStream_t s);
int reliable_finish(nbx_problem *P, const double *b, double *x, const nbx_pcg_opts &o,
                    const ReliableState &rs, nbx_pcg_result *res, hipStream_t s);

}  // namespace nbx
