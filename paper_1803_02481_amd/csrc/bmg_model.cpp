// bmg_model.cpp -- performance model of the V-cycle with collapsed coarse levels.
//
// The paper models a V-cycle as the coarse solve plus, per level, smoothing,
// residual, restriction, interpolation and agglomeration, each a computation
// term (flops x gamma) plus a communication term (halo exchanges, each
// alpha + bytes x beta) (section 3, V-cycle model and its component
// equations).  On one GPU the computation is memory-bound, so the work term of
// a stage is its algorithmic bytes times an inverse bandwidth, and the
// synchronisation term is the cost of the point where the paper exchanges
// halos: a kernel boundary on grid-wide levels, a workgroup barrier on
// collapsed levels.  Agglomeration onto the collapsed workgroup costs one
// kernel boundary (one launch for all collapsed levels).
#include "bmg_model.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

namespace hbmg {

ModelParams &model_params()
{
    static ModelParams p = [] {
        ModelParams d;
        d.alpha_launch_us = 6.0;
        d.step_us = 1.2;
        d.beta_hbm_us_per_B = 1.0 / 5.0e6;     // 5 TB/s achieved from HBM
        d.beta_cache_us_per_B = 1.0 / 10.0e6;  // 10 TB/s from cache-resident levels
        d.cache_bytes = 256.0e6;
        d.alpha_bar_us = 1.0;
        d.alpha_bar_lds_us = 0.1;
        d.beta_wg_us_per_B = 1.0 / 1.0e5;      // 100 GB/s for one workgroup
        d.gamma_wg_us_per_flop = 1.0e-3;
        d.lds_budget_bytes = 150.0 * 1024.0;
        d.calibrated = 0;
        if (const char *env = std::getenv("HIPBMG_MODEL_PARAMS")) {
            double a, st, hb, cb, ab, wb;
            if (std::sscanf(env, "%lf,%lf,%lf,%lf,%lf,%lf", &a, &st, &hb, &cb, &ab, &wb) == 6) {
                d.alpha_launch_us = a;
                d.step_us = st;
                d.beta_hbm_us_per_B = 1.0 / (hb * 1e3);
                d.beta_cache_us_per_B = 1.0 / (cb * 1e3);
                d.alpha_bar_us = ab;
                d.beta_wg_us_per_B = 1.0 / (wb * 1e3);
            }
        }
        return d;
    }();
    return p;
}

// planes read by a relaxation: b, x and the stencil (3 planes 5-point, 5 planes 9-point)
static double planes(int npt) { return npt == 5 ? 3.0 : 5.0; }

double model_grid_level_us(const ModelLevel &lv, bool finest, int nu1, int nu2, int word,
                           const ModelParams &p)
{
    const double n = (double)lv.nx * lv.ny, s = planes(lv.npt), w = word;
    const double level_bytes = n * w * (s + 4.0) + n * w * 2.0 / 4.0 * 8.0 / 4.0;
    const double beta = level_bytes < p.cache_bytes ? p.beta_cache_us_per_B : p.beta_hbm_us_per_B;
    const int nsteps = (lv.ny - 1) / 2;
    double t = 0.0;
    // down: nu1 relaxations; the last two run as one pass fused with residual,
    // r/C and restriction (the last one alone if nu1 = 1)
    const int nk = nu1 >= 2 ? nu1 - 1 : nu1;
    for (int k = 1; k <= nk; ++k) {
        double bytes = n * w * (s + 3.0);
        if (k == 1 && !finest) bytes -= n * w;               // iterate starts at zero
        int pro = 1;
        if (k == nk) {
            bytes += n * w * (1.0 + 2.0 + 0.25);             // q, weights, coarse rhs
            pro = nk < nu1 ? 5 : 2;
        }
        const double steps = std::min(lv.rb, nsteps) + pro;
        t += p.alpha_launch_us + std::max(steps * p.step_us, bytes * beta);
    }
    // up: interpolation fused with the first post-relaxation
    for (int k = 1; k <= nu2; ++k) {
        double bytes = n * w * (s + 3.0);
        if (k == 1) bytes += n * w * (0.25 + 2.0 + 1.0);     // coarse x, weights, q
        const double steps = std::min(lv.rb, nsteps) + 2;
        t += p.alpha_launch_us + std::max(steps * p.step_us, bytes * beta);
    }
    return t;
}

double model_wg_level_us(const ModelLevel &lv, int nu1, int nu2, int word, bool in_lds,
                         const ModelParams &p)
{
    const double n = (double)lv.nx * lv.ny, s = 5.0, w = word;
    // barriers: zeroing, 4 colours per relaxation, residual, restriction, interpolation
    const double phases = 1.0 + 4.0 * (nu1 + nu2) + 3.0;
    const double bytes = n * w * ((nu1 + nu2) * (s + 3.0) + (s + 3.0) + 3.25 + 6.25);
    if (in_lds)   // staged once per launch from global memory, then LDS speed
        return phases * p.alpha_bar_lds_us + n * w * 10.0 * p.beta_wg_us_per_B +
               0.25 * bytes * p.beta_wg_us_per_B;
    return phases * p.alpha_bar_us + bytes * p.beta_wg_us_per_B;
}

int model_choose(const ModelLevel *lv, int L, int nu1, int nu2, int nc, int word,
                 const ModelParams &p, double *t_us)
{
    // coarse solve: two triangular substitutions, 2 barriers per unknown
    const double t_cg = (nc > 1 ? 4.0 * nc * p.alpha_bar_lds_us : p.alpha_bar_lds_us) +
                        2.0 * (double)nc * nc * p.gamma_wg_us_per_flop;
    // levels staged in LDS: from the coarsest up while their footprint fits
    bool in_lds[64] = {};
    double used = 0.0;
    for (int l = 0; l < L && l < 64; ++l) {
        const double cn = l ? (double)lv[l - 1].nx * lv[l - 1].ny : 0.0;
        used += (8.0 * lv[l].nx * lv[l].ny + 8.0 * cn) * word;
        if (used > p.lds_budget_bytes) break;
        in_lds[l] = true;
    }
    int best = 0;
    for (int ls = 0; ls < L; ++ls) {
        double t = p.alpha_launch_us + t_cg;                   // the collapsed launch
        for (int l = ls + 1; l < L; ++l) t += model_grid_level_us(lv[l], l == L - 1, nu1, nu2, word, p);
        for (int l = 1; l <= ls; ++l) t += model_wg_level_us(lv[l], nu1, nu2, word, in_lds[l], p);
        t += p.alpha_launch_us;                                // norm finalisation
        t_us[ls] = t;
        if (t < t_us[best]) best = ls;
    }
    return best;
}

}  // namespace hbmg
