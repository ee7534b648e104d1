// bmg_model.h -- the alpha-beta-gamma performance model of a V-cycle (section 3)
// in its single-GPU form, used to pick the collapse level l* (the analogue of
// the redistribution choice of section 4).
#pragma once

#include "hipbmg.h"

#include <vector>

namespace hbmg {

// One streaming kernel as the model sees it: the row-pair steps one wave
// walks, the residency rounds of the launch, and the bytes it loads per
// algorithmic byte (halo lanes shared with neighbouring strips and prologue
// rows shared with the block below are loaded twice).
struct ModelKernel {
    int steps, rounds;
    double reread;
};

// One level as the model sees it.  The host fills in the launch geometry the
// streaming kernels will use: the down (pre-relaxation) and up
// (interpolation) kernels, and for a pipelined finest level the single pass
// that replaces both; in_lds says whether the level is staged in LDS when it
// is collapsed.
struct ModelLevel {
    int nx, ny, npt;
    ModelKernel dn, up, pipe;
    int pipelined;
    int in_lds;
    // where a leg finds the level's data: 1 in HBM (evicted since its last
    // use), 0 in the last-level cache
    int dn_cold, up_cold;
    // the up leg forms r/C from the rows it loads (no q plane written or read)
    int rc;
    // the pipelined pass forms the diagonal from the connections (zero-excess
    // operator) instead of loading it
    int zexc;
    // the r/C level's two kernels form the diagonal of its deep vertices
    int zc9;
};

// Machine parameters.  Paper -> GPU correspondence:
//   alpha (message latency)  -> alpha_launch: one dependent kernel boundary on a
//                               grid-wide level; alpha_bar: one barrier phase of
//                               the collapsed workgroup (level in LDS or in
//                               global memory)
//   beta (inverse bandwidth) -> beta_hbm / beta_cache for grid-wide levels (by
//                               working set), beta_wg for the collapsed workgroup
//   gamma (per flop)         -> gamma_wg, single-thread FP64 work of the coarse solve
// plus step_dn / step_up, the latency of one row-pair step of a streaming wave
// (pre-relaxation and interpolation kernels), and t0_dn / t0_up, a kernel's
// fixed cost after the previous one (launch gap, wave start, first loads),
// which bound a grid-wide kernel on a level too small to fill the GPU; and
// t_base, the collapsed launch holding only the coarsest level.
// Per-precision entries are indexed [0] FP64, [1] FP32; alpha_bar and beta_wg
// also by [0] LDS, [1] global.  An agglomeration stage of 2^(k+1) workgroups
// (k < MODEL_STAGE_SIZES) costs alpha_stage per barrier phase plus bytes x
// beta_stage per level.
constexpr int MODEL_STAGE_SIZES = 8;   // 2, 4, ..., 256 workgroups
struct ModelParams {
    double alpha_launch_us;
    double beta_hbm_us_per_B;
    double beta_cache_us_per_B;
    double cache_bytes;
    double step_dn_us[2];
    double step_up_us[2];
    double t0_dn_us[2];
    double t0_up_us[2];
    double t_base_us[2];
    double alpha_bar_us[2][2];
    double beta_wg_us_per_B[2][2];
    double gamma_wg_us_per_flop;
    double lds_budget_bytes;    // LDS available for staged collapsed levels
    double alpha_stage_us[2][MODEL_STAGE_SIZES];
    double beta_stage_us_per_B[2][MODEL_STAGE_SIZES];
    int stages_calibrated;      // 1 once the stage terms are measured
    int calibrated;             // 1 once measured on the device
};

// process-wide parameters: defaults until hipbmg_calibrate replaces them
ModelParams &model_params();

// Fit the step latencies and the collapsed-level terms of p by timing the
// solver's own kernels on a synthetic hierarchy (alpha_launch and the
// bandwidths must already be measured).  stream is a hipStream_t.
hipbmg_status calibrate_on_kernels(void *stream, ModelParams &p);

// barrier phases and algorithmic bytes of one visit of a collapsed level per
// V(nu1,nu2)-cycle (zeroing, 4 colours per relaxation, residual, restriction,
// interpolation; 9-point operator, word bytes per value)
double model_wg_phases(int nu1, int nu2);
double model_wg_bytes(int nx, int ny, int nu1, int nu2, int word);

// Predicted time (microseconds) of one V(nu1,nu2)-cycle for every collapse
// level l* in [0, L-1] into t_us[l*]; returns the argmin.  word = bytes per value.
int model_choose(const ModelLevel *lv, int L, int nu1, int nu2, int nc, int word,
                 const ModelParams &p, double *t_us);

// the collapsed launch holding only the coarsest level (nc unknowns):
// launch gap, base cost and coarse solve
double model_base_us(int nc, int word, const ModelParams &p);

// The redistribution search of section 4 on one GPU.  A state is (level l,
// processors m): m = 0 all processors (grid-wide kernels), m = 1..8 a stage
// of 256, 128, ..., 2 workgroups (the factor-2 enumeration), m = 9 one
// workgroup.  From (l, m) the solve either runs level l there and moves to
// (l-1, m), or agglomerates onto fewer processors, (l, m') with m' > m.  The
// start is (L-1, 0), the goal (0, 9): level 0 is the coarse solve.  g is the
// model time so far; the heuristic h is the sum over the levels left of
// their cheapest cost on the processors still reachable, plus the cheapest
// hand-off to one workgroup, which never overestimates.
constexpr int MODEL_MODES = MODEL_STAGE_SIZES + 2;
struct ModelPath {
    int lstar;        // levels 0..lstar in one workgroup
    int nstage;       // stages on several workgroups, above it
    int wg[4], hi[4]; // workgroups and highest level of each stage, decreasing
    double t_us;      // model time of one cycle along the path
    int expanded;     // states expanded by the search
};
// workgroups of mode m (0 for all processors)
int model_mode_wg(int m);
// cost of level l in mode m (infinite where not allowed); max_wg: largest
// stage that fits on the device; lcap: highest level one workgroup (or a
// stage) can address
double model_level_cost(const ModelLevel *lv, int L, int l, int m, int nu1, int nu2, int word,
                        const ModelParams &p, int max_wg, int lcap);
ModelPath model_search(const ModelLevel *lv, int L, int nu1, int nu2, int nc, int word, const ModelParams &p,
                       int max_wg, int lcap);
// every path enumerated (the cost A* avoids), for checking the search
ModelPath model_search_exhaustive(const ModelLevel *lv, int L, int nu1, int nu2, int nc, int word,
                                  const ModelParams &p, int max_wg, int lcap);
// model time of one cycle with the given stages above collapse level lstar
double model_path_us(const ModelLevel *lv, int L, int nu1, int nu2, int nc, int word, const ModelParams &p,
                     int lstar, int nstage, const int *wg, const int *hi);

// the two parts of the model for one level (exposed for reporting)
double model_grid_level_us(const ModelLevel &lv, bool finest, int nu1, int nu2, int word,
                           const ModelParams &p);
double model_wg_level_us(const ModelLevel &lv, int nu1, int nu2, int word, const ModelParams &p);

// The same model for 3D hierarchies (section 3's terms with 3D counts).  A
// grid-wide level launches one kernel per colour and relaxation (four per
// relaxation on a 7-point level, whose colours fall into four uncoupled
// groups), the residual, the restriction, the zeroing of the coarse iterate
// and the interpolation; each kernel costs its fixed cost t0 plus its loaded
// bytes at the level's bandwidth (cache or HBM by working set).  A collapsed
// level costs one barrier phase per kernel plus its bytes at the one-workgroup
// bandwidth from global memory.  The collapse launch adds model_base_us.
struct ModelLevel3 {
    int nx, ny, nz, npt;
};
double model3_grid_level_us(const ModelLevel3 &lv, int nu1, int nu2, const ModelParams &p);
double model3_wg_level_us(const ModelLevel3 &lv, int nu1, int nu2, const ModelParams &p);
// t_us[l*] for l* in [0, min(L-1, lcap)]; returns the argmin
int model3_choose(const ModelLevel3 *lv, int L, int nu1, int nu2, int nc, const ModelParams &p, int lcap,
                  double *t_us);

// ---------------------------------------------------------------------------
// The paper's distributed model in its own form (section 3) and its processor
// grid enumeration (section 4): what the redistribution search runs over when
// the levels are spread over processors (here: GPUs), written out from the
// equations.  Levels are numbered as in the paper, 0 coarsest.
// ---------------------------------------------------------------------------
struct PaperMachine {
    double alpha, beta, gamma;   // seconds, seconds per byte, seconds per flop
};
// halo exchange of width 1 in D dimensions over the local sizes n[0..D-1]
double paper_exchange(int D, const int *n, const PaperMachine &m);
double paper_smooth(int D, const int *n, int ns, int ncolors, int nu1, int nu2, const PaperMachine &m);
double paper_residual(int D, const int *n, int ns, const PaperMachine &m);
double paper_restrict(int D, const int *n, int ns, const PaperMachine &m);
// interpolation and correction from the coarse local sizes nc to the fine
// local sizes n (D = 2 or 3: the two interpolation cost equations)
double paper_interp(int D, const int *n, const int *nc, const PaperMachine &m);
// gather of the right-hand side (and scatter of the solution unless
// redundant) when the processor grid shrinks from pf to pc with the coarse
// global sizes N (0 if it does not shrink)
double paper_agglomerate(int D, const int *N, const int *pf, const int *pc, int redundant, const PaperMachine &m);
// Coarse processor grids for a global coarse grid N on processor grid P:
// start from 1 x ... x 1 and double, one dimension at a time, the dimension
// whose agglomerated local size ceil(N_d / p_d) is largest among those below
// P_d, stopping before P itself.  Returns the count (at most max).
int paper_enumerate(int D, const int *N, const int *P, int max, int *grids);

// The redistribution search of section 4 over the paper's model.  A state is
// (global grid N, processor grid p).  A level on p coarsens N to ceil(N/2)
// while every local side ceil(N_d/p_d) exceeds `limit` (the coarsening
// limit) and N exceeds `coarsest`; at the limit the solve agglomerates onto
// one of the enumerated coarser grids of (N, p).  On 1 x ... x 1 the levels
// continue down to `coarsest` and end in the Cholesky solve.  The search
// returns the cheapest path (the grids after the first, up to 1 x ... x 1)
// and its model time; path_cost prices a given sequence of grids.
struct PaperSetup {
    int D, limit, coarsest, ns, ncolors, nu1, nu2, redundant;
    PaperMachine m;
};
double paper_search(const PaperSetup &s, const int *N, const int *P, std::vector<std::vector<int>> *path);
// The same search by A* (section 4): f = g + h with h the remaining levels
// priced on the current processor grid plus the coarse solve (a grid only
// shrinks along a path and a level costs no less on fewer processors, so h
// never overestimates).  *expanded = states taken off the open list.
double paper_astar(const PaperSetup &s, const int *N, const int *P, std::vector<std::vector<int>> *path,
                   int *expanded);
double paper_path_cost(const PaperSetup &s, const int *N, const int *P, const std::vector<std::vector<int>> &seq);

}  // namespace hbmg
