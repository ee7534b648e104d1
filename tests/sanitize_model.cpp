// Driver that calls the host-only performance-model code (the single-GPU
// model, its redistribution search and the paper's distributed model with its
// enumeration and searches) on the paper's own problems and on random ones,
// built with AddressSanitizer and UndefinedBehaviorSanitizer by the CPU test
// suite.  Numerical checks live in the model tests; a run that ends with status
// 0 and no sanitizer report means no out-of-bounds access, leak or undefined
// operation on these paths.
#include "bmg_model.h"

#include <cstdio>
#include <random>
#include <vector>

using namespace hbmg;

int main()
{
    double sink = 0.0;
    // the single-GPU model on a 4097^2-like hierarchy and a 3D one
    const int L = 12;
    ModelLevel lv[HIPBMG_MAX_LEVELS] = {};
    for (int l = 0; l < L; ++l) {
        const int n = (1 << (l + 1)) + 1;
        lv[l].nx = lv[l].ny = n;
        lv[l].npt = l == L - 1 ? 5 : 9;
        lv[l].dn = ModelKernel{l > 8 ? 24 : 5, 1, 1.3};
        lv[l].up = ModelKernel{l > 8 ? 11 : 2, 1, 1.2};
        lv[l].pipe = ModelKernel{85, 1, 1.25};
        lv[l].pipelined = l == L - 1;
        lv[l].in_lds = l <= 4;
        lv[l].dn_cold = 1;
    }
    const ModelParams &p = model_params();
    double t[HIPBMG_MAX_LEVELS] = {};
    sink += model_choose(lv, L, 2, 1, 1, 8, p, t);
    const ModelPath path = model_search(lv, L, 2, 1, 1, 8, p, 256, L - 1);
    sink += path.t_us + model_path_us(lv, L, 2, 1, 1, 8, p, path.lstar, path.nstage, path.wg, path.hi);
    const ModelPath all = model_search_exhaustive(lv, 8, 2, 1, 1, 4, p, 64, 7);
    sink += all.t_us + model_base_us(1, 8, p);
    ModelLevel3 l3[6];
    for (int l = 0; l < 6; ++l) l3[l] = ModelLevel3{(1 << (l + 1)) + 1, (1 << (l + 1)) + 1, (1 << (l + 1)) + 1,
                                                     l == 5 ? 7 : 27};
    double t3[6] = {};
    sink += model3_choose(l3, 6, 2, 1, 1, p, 5, t3);

    // the paper's model with the Blue Waters parameters: the enumeration
    // example, the weak-scaling problem's search, and random setups
    const PaperMachine bw{0.65e-6, 5.65e-9, 0.44e-9};
    int grids[64 * 3];
    const int Ne[2] = {1136, 71}, Pe[2] = {16, 8};
    sink += paper_enumerate(2, Ne, Pe, 64, grids);
    PaperSetup s{2, 9, 3, 9, 4, 2, 1, 0, bw};
    const int N[2] = {36352, 2272}, P[2] = {64, 32};
    std::vector<std::vector<int>> pa, pb;
    int expanded = 0;
    sink += paper_search(s, N, P, &pa) + paper_astar(s, N, P, &pb, &expanded) + paper_path_cost(s, N, P, pb);
    const int n3[3] = {64, 32, 32}, c3[3] = {32, 16, 16};
    sink += paper_exchange(3, n3, bw) + paper_smooth(3, n3, 27, 8, 2, 1, bw) + paper_residual(3, n3, 27, bw) +
            paper_restrict(3, n3, 27, bw) + paper_interp(3, n3, c3, bw);
    const int N3[3] = {256, 128, 128}, pf[3] = {8, 4, 4}, pc[3] = {2, 1, 1};
    sink += paper_agglomerate(3, N3, pf, pc, 1, bw);
    std::mt19937 rng(7);
    for (int k = 0; k < 200; ++k) {
        const int D = 2 + (int)(rng() % 2);
        int Nr[3], Pr[3];
        for (int d = 0; d < D; ++d) {
            Pr[d] = 1 + (int)(rng() % 24);
            Nr[d] = Pr[d] * (4 + (int)(rng() % 200));
        }
        PaperSetup r{D, 5 + (int)(rng() % 12), 2 + (int)(rng() % 6), D == 2 ? 9 : 27, D == 2 ? 4 : 8, 2, 1,
                     (int)(rng() % 2), PaperMachine{1e-6 * (1 + rng() % 10), 1e-9 * (1 + rng() % 10), 1e-10}};
        std::vector<std::vector<int>> q1, q2;
        int ex = 0;
        sink += paper_search(r, Nr, Pr, &q1) + paper_astar(r, Nr, Pr, &q2, &ex) + paper_path_cost(r, Nr, Pr, q1);
    }
    std::printf("model driver done (%d states expanded on the weak-scaling problem), sink %.6e\n", expanded, sink);
    return 0;
}
