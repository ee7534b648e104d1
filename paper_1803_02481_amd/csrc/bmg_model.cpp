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

namespace hbmg {

ModelParams &model_params()
{
    // defaults of the order measured on an MI355X; hipbmg_calibrate replaces them
    static ModelParams p = [] {
        ModelParams d{};
        d.alpha_launch_us = 2.5;
        d.beta_hbm_us_per_B = 1.0 / 5.0e6;     // 5 TB/s from HBM
        d.beta_cache_us_per_B = 1.0 / 10.0e6;  // 10 TB/s from cache-resident levels
        d.cache_bytes = 256.0e6;
        for (int q = 0; q < 2; ++q) {
            d.step_dn_us[q] = 1.4;
            d.step_up_us[q] = 1.2;
            d.t0_dn_us[q] = 5.0;
            d.t0_up_us[q] = 4.0;
            d.t_base_us[q] = 10.0;
            d.alpha_bar_us[q][0] = 0.15;
            d.alpha_bar_us[q][1] = 1.5;
            d.beta_wg_us_per_B[q][0] = 1.0 / 4.0e5;   // 400 GB/s, one workgroup on LDS
            d.beta_wg_us_per_B[q][1] = 1.0 / 5.0e4;   // 50 GB/s, one workgroup on L2
        }
        d.gamma_wg_us_per_flop = 1.0e-3;
        d.lds_budget_bytes = 150.0 * 1024.0;
        d.calibrated = 0;
        return d;
    }();
    return p;
}

// planes read by a relaxation: b, x and the stencil (3 planes 5-point, 5 planes 9-point)
static double planes(int npt) { return npt == 5 ? 3.0 : 5.0; }

// one streaming kernel: the longer of its waves' sequential steps (after its
// fixed cost) and the bytes it loads at the level's bandwidth (after a launch gap)
static double kernel_us(const ModelKernel &k, double step_us, double t0_us, double bytes, double beta,
                        const ModelParams &p)
{
    const double lat = t0_us + (double)k.rounds * k.steps * step_us;
    return std::max(lat, p.alpha_launch_us + bytes * k.reread * beta);
}

double model_grid_level_us(const ModelLevel &lv, bool finest, int nu1, int nu2, int word,
                           const ModelParams &p)
{
    const int q = word == 4 ? 1 : 0;
    const double n = (double)lv.nx * lv.ny, s = planes(lv.npt), w = word;
    const double bdn = lv.dn_cold ? p.beta_hbm_us_per_B : p.beta_cache_us_per_B;
    const double bup = lv.up_cold ? p.beta_hbm_us_per_B : p.beta_cache_us_per_B;
    if (finest && lv.pipelined) {
        // one pass per cycle: interpolate + relax + norm of this cycle, two
        // relaxations + residual + restriction of the next (68 B per vertex in
        // FP64); its waves do the work of a down and an up step per row pair
        const double bytes = n * w * (s + 3.0 + 0.25 + 2.0 + 0.25);
        return kernel_us(lv.pipe, p.step_dn_us[q] + p.step_up_us[q], p.t0_dn_us[q], bytes, bdn, p);
    }
    double t = 0.0;
    // down: nu1 relaxations; the last two run as one pass fused with residual,
    // r/C and restriction (the last one alone if nu1 = 1)
    const int nk = nu1 >= 2 ? nu1 - 1 : nu1;
    for (int k = 1; k <= nk; ++k) {
        double bytes = n * w * (s + 3.0);                    // one pass, however many sweeps it fuses
        if (k == 1 && !finest) bytes -= n * w;               // iterate starts at zero
        if (k == nk) bytes += n * w * (1.0 + 2.0 + 0.25);    // q, weights, coarse rhs
        t += kernel_us(lv.dn, p.step_dn_us[q], p.t0_dn_us[q], bytes, bdn, p);
    }
    // up: interpolation fused with the first post-relaxation
    for (int k = 1; k <= nu2; ++k) {
        double bytes = n * w * (s + 3.0);
        if (k == 1) bytes += n * w * (0.25 + 2.0 + 1.0);     // coarse x, weights, q
        t += kernel_us(lv.up, p.step_up_us[q], p.t0_up_us[q], bytes, bup, p);
    }
    return t;
}

double model_wg_phases(int nu1, int nu2) { return 4.0 * (nu1 + nu2) + 4.0; }

double model_wg_bytes(int nx, int ny, int nu1, int nu2, int word)
{
    // per relaxation x, b and the 9-point operator read, x written; the
    // residual once more; restriction and interpolation read the weights
    const double n = (double)nx * ny, s = 5.0, w = word;
    return n * w * ((nu1 + nu2) * (s + 3.0) + (s + 3.0) + 3.25 + 6.25);
}

double model_wg_level_us(const ModelLevel &lv, int nu1, int nu2, int word, const ModelParams &p)
{
    const int q = word == 4 ? 1 : 0, g = lv.in_lds ? 0 : 1;
    return model_wg_phases(nu1, nu2) * p.alpha_bar_us[q][g] +
           model_wg_bytes(lv.nx, lv.ny, nu1, nu2, word) * p.beta_wg_us_per_B[q][g];
}

double model_base_us(int nc, int word, const ModelParams &p)
{
    const int q = word == 4 ? 1 : 0;
    // coarse solve beyond the one-unknown base: two triangular substitutions,
    // 2 barriers per unknown, nc^2 multiply-adds each
    const double t_cg = (nc > 1 ? 4.0 * (nc - 1) * p.alpha_bar_us[q][0] : 0.0) +
                        2.0 * (double)nc * nc * p.gamma_wg_us_per_flop;
    return p.alpha_launch_us + p.t_base_us[q] + t_cg;
}

int model_choose(const ModelLevel *lv, int L, int nu1, int nu2, int nc, int word,
                 const ModelParams &p, double *t_us)
{
    const double base = model_base_us(nc, word, p);
    int best = 0;
    for (int ls = 0; ls < L; ++ls) {
        double t = base;                                         // the collapsed launch
        for (int l = ls + 1; l < L; ++l) t += model_grid_level_us(lv[l], l == L - 1, nu1, nu2, word, p);
        for (int l = 1; l <= ls; ++l) t += model_wg_level_us(lv[l], nu1, nu2, word, p);
        t += p.alpha_launch_us;                                  // norm finalisation
        t_us[ls] = t;
        if (t < t_us[best]) best = ls;
    }
    return best;
}

}  // namespace hbmg
