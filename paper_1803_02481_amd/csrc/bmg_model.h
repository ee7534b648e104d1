// bmg_model.h -- the alpha-beta-gamma performance model of a V-cycle (section 3)
// in its single-GPU form, used to pick the collapse level l* (the analogue of
// the redistribution choice of section 4).
#pragma once

namespace hbmg {

struct ModelLevel {
    int nx, ny, npt, rb;
};

// Machine parameters.  Paper -> GPU correspondence:
//   alpha (message latency)  -> alpha_launch: one dependent kernel boundary for
//                               grid-wide levels; alpha_bar: one workgroup barrier
//                               plus an L2 round trip inside the collapsed workgroup
//   beta (inverse bandwidth) -> beta_hbm / beta_cache (grid-wide, by working set)
//                               and beta_wg (one workgroup)
//   gamma (per flop)         -> gamma_wg (single-thread FP64 work of the coarse solve)
// plus step_us, the latency of one row-pair step of a streaming wave, which
// bounds a grid-wide kernel on a level too small to fill the GPU.
struct ModelParams {
    double alpha_launch_us;
    double step_us;
    double beta_hbm_us_per_B;
    double beta_cache_us_per_B;
    double cache_bytes;
    double alpha_bar_us;        // barrier after a dependent L2 access (level in global memory)
    double alpha_bar_lds_us;    // barrier after a dependent LDS access (level staged in LDS)
    double beta_wg_us_per_B;
    double gamma_wg_us_per_flop;
    double lds_budget_bytes;    // LDS available for staged collapsed levels
    int calibrated;             // 1 once measured on the device
};

// process-wide parameters (defaults, replaced by calibrate or the
// HIPBMG_MODEL_PARAMS environment variable: "alpha_launch_us,step_us,
// hbm_GBps,cache_GBps,alpha_bar_us,wg_GBps")
ModelParams &model_params();

// Predicted time (microseconds) of one V(nu1,nu2)-cycle for every collapse
// level l* in [0, L-1] into t_us[l*]; returns the argmin.  word = bytes per value.
int model_choose(const ModelLevel *lv, int L, int nu1, int nu2, int nc, int word,
                 const ModelParams &p, double *t_us);

// the two parts of the model for one level (exposed for reporting)
double model_grid_level_us(const ModelLevel &lv, bool finest, int nu1, int nu2, int word,
                           const ModelParams &p);
double model_wg_level_us(const ModelLevel &lv, int nu1, int nu2, int word, bool in_lds,
                         const ModelParams &p);

}  // namespace hbmg
