// Checks of the redistribution search of the performance model (section 4),
// compiled on the host against the library's model source.  For random model
// parameters on a 4097^2-like hierarchy:
//   - the A* path costs the same as the cheapest path found by enumerating
//     every path, and A* expands fewer states than the enumeration visits;
//   - the cost the search reports equals the model's cost of the path it
//     returns, recomputed level by level;
//   - with stages far too expensive to use, the search returns the plain
//     collapse level that the one-dimensional argmin over l* chooses.
#include "bmg_model.h"

#include <cmath>
#include <cstdio>
#include <random>

using namespace hbmg;

int main()
{
    const int L = 12;
    ModelLevel lv[HIPBMG_MAX_LEVELS] = {};
    for (int l = 0; l < L; ++l) {
        const int n = (1 << (l + 1)) + 1;
        lv[l].nx = lv[l].ny = n;
        lv[l].npt = l == L - 1 ? 5 : 9;
        const int steps = std::max(1, (n - 1) / 2);
        lv[l].dn = ModelKernel{l > 8 ? 24 : 5, 1, 1.3};
        lv[l].up = ModelKernel{l > 8 ? 11 : 2, 1, 1.2};
        lv[l].pipe = ModelKernel{std::min(85, steps), 1, 1.25};
        lv[l].pipelined = l == L - 1;
        lv[l].in_lds = l <= 4;
        lv[l].dn_cold = 1;
        lv[l].up_cold = l >= 10;
    }
    std::mt19937_64 rng(12345);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    int fails = 0, trials = 0, with_stages = 0, multi = 0;
    long long exp_astar = 0, exp_all = 0;
    for (int t = 0; t < 60; ++t) {
        ModelParams p = model_params();
        p.alpha_launch_us = 1.0 + 3.0 * u(rng);
        p.beta_hbm_us_per_B = 1.0 / (3.0e6 + 3.0e6 * u(rng));
        p.beta_cache_us_per_B = 1.0 / (1.0e7 + 1.0e7 * u(rng));
        for (int q = 0; q < 2; ++q) {
            p.step_dn_us[q] = 0.5 + 2.0 * u(rng);
            p.step_up_us[q] = 0.3 + 1.0 * u(rng);
            p.t0_dn_us[q] = 5.0 * u(rng);
            p.t0_up_us[q] = 5.0 * u(rng);
            p.t_base_us[q] = 2.0 + 8.0 * u(rng);
            for (int g = 0; g < 2; ++g) {
                p.alpha_bar_us[q][g] = 0.05 + 0.8 * u(rng);
                p.beta_wg_us_per_B[q][g] = 1.0 / (1.0e4 + 1.0e5 * u(rng));
            }
            for (int k = 0; k < MODEL_STAGE_SIZES; ++k) {
                // some trials make stages attractive, some not
                p.alpha_stage_us[q][k] = (t % 3 == 0 ? 0.05 : 0.5) + 3.0 * u(rng);
                p.beta_stage_us_per_B[q][k] = 1.0 / ((1.0e4 + 1.0e5 * u(rng)) * (2 << k));
            }
        }
        const int word = t % 2 ? 4 : 8, max_wg = 256 >> (t % 4), lcap = L - 1;
        const ModelPath a = model_search(lv, L, 2, 1, 1, word, p, max_wg, lcap);
        const ModelPath e = model_search_exhaustive(lv, L, 2, 1, 1, word, p, max_wg, lcap);
        const double again = model_path_us(lv, L, 2, 1, 1, word, p, a.lstar, a.nstage, a.wg, a.hi);
        ++trials;
        with_stages += a.nstage > 0;
        multi += a.nstage > 1;
        exp_astar += a.expanded;
        exp_all += e.expanded;
        const bool same = std::fabs(a.t_us - e.t_us) <= 1e-9 * e.t_us;
        const bool cost = std::fabs(again - a.t_us) <= 1e-9 * a.t_us;
        bool wg_ok = true;
        for (int k = 0; k < a.nstage; ++k) wg_ok = wg_ok && a.wg[k] <= max_wg && a.wg[k] >= 2 &&
                                                  (k == 0 || a.wg[k] < a.wg[k - 1]) && a.hi[k] > a.lstar &&
                                                  a.hi[k] <= L - 2 && (k == 0 || a.hi[k] < a.hi[k - 1]);
        if (!same || !cost || !wg_ok || a.expanded >= e.expanded) {
            ++fails;
            std::printf("trial %d: astar %.6f (lstar %d, %d stages, %d expanded) exhaustive %.6f (%d visited) "
                        "recomputed %.6f\n", t, a.t_us, a.lstar, a.nstage, a.expanded, e.t_us, e.expanded, again);
        }
        // stages priced out: the search reduces to the argmin over l*
        ModelParams p2 = p;
        for (int q = 0; q < 2; ++q)
            for (int k = 0; k < MODEL_STAGE_SIZES; ++k) p2.alpha_stage_us[q][k] = 1e6;
        double tl[HIPBMG_MAX_LEVELS];
        const int best = model_choose(lv, L, 2, 1, 1, word, p2, tl);
        const ModelPath b = model_search(lv, L, 2, 1, 1, word, p2, max_wg, lcap);
        if (b.nstage != 0 || std::fabs(b.t_us - tl[best]) > 1e-9 * tl[best] ||
            std::fabs(tl[b.lstar] - tl[best]) > 1e-9 * tl[best]) {
            ++fails;
            std::printf("trial %d: no-stage search lstar %d (%.6f) vs argmin %d (%.6f)\n", t, b.lstar, b.t_us, best,
                        tl[best]);
        }
    }
    std::printf("trials %d fails %d with stages %d (several %d) mean expanded astar %.1f exhaustive %.1f\n",
                trials, fails, with_stages, multi, (double)exp_astar / trials, (double)exp_all / trials);
    // the random draws must exercise paths with stages, not only plain collapses
    return fails || with_stages < 5 ? 1 : 0;
}
