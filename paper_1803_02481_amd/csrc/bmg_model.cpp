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
#include <limits>
#include <map>
#include <queue>
#include <vector>

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
        // until measured, stages cost far more than either alternative
        for (int q = 0; q < 2; ++q)
            for (int k = 0; k < MODEL_STAGE_SIZES; ++k) {
                d.alpha_stage_us[q][k] = 50.0;
                d.beta_stage_us_per_B[q][k] = 1.0 / 1.0e4;
            }
        d.stages_calibrated = 0;
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
        // FP64, 60 B when the diagonal is formed instead of loaded); its waves
        // do the work of a down and an up step per row pair
        const double bytes = n * w * (s + 3.0 + 0.25 + 2.0 + 0.25 - (lv.zexc ? 1.0 : 0.0));
        return kernel_us(lv.pipe, p.step_dn_us[q] + p.step_up_us[q], p.t0_dn_us[q], bytes, bdn, p);
    }
    double t = 0.0;
    // down: nu1 relaxations; the last two run as one pass fused with residual,
    // r/C and restriction (the last one alone if nu1 = 1)
    const int nk = nu1 >= 2 ? nu1 - 1 : nu1;
    for (int k = 1; k <= nk; ++k) {
        double bytes = n * w * (s + 3.0);                    // one pass, however many sweeps it fuses
        if (k == 1 && !finest) bytes -= n * w;               // iterate starts at zero
        if (k == nk) bytes += n * w * ((lv.rc ? 0.0 : 1.0) + 2.0 + 0.25);   // q, weights, coarse rhs
        if (k == nk && lv.rc && lv.zc9) bytes -= n * w;                      // diagonal formed
        t += kernel_us(lv.dn, p.step_dn_us[q], p.t0_dn_us[q], bytes, bdn, p);
    }
    // up: interpolation fused with the first post-relaxation
    for (int k = 1; k <= nu2; ++k) {
        double bytes = n * w * (s + 3.0);
        if (k == 1) bytes += n * w * (0.25 + 2.0 + (lv.rc ? 0.0 : 1.0));   // coarse x, weights, q
        if (k == 1 && lv.rc && lv.zc9) bytes -= n * w;                      // diagonal formed
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

static const double kInf = std::numeric_limits<double>::infinity();
constexpr int kSingle = MODEL_MODES - 1;
constexpr int kMaxStages = 4;

int model_mode_wg(int m)
{
    if (m <= 0) return 0;
    if (m >= kSingle) return 1;
    return 256 >> (m - 1);
}

// stage parameters of mode m: index k with 2^(k+1) workgroups
static int stage_index(int m) { return MODEL_STAGE_SIZES - m; }

double model_level_cost(const ModelLevel *lv, int L, int l, int m, int nu1, int nu2, int word,
                        const ModelParams &p, int max_wg, int lcap)
{
    if (l < 1 || l >= L) return kInf;   // level 0 is the coarse solve, inside the hand-off
    if (m == 0) return model_grid_level_us(lv[l], l == L - 1, nu1, nu2, word, p);
    if (l > lcap) return kInf;
    if (m == kSingle) return model_wg_level_us(lv[l], nu1, nu2, word, p);
    if (l >= L - 1 || model_mode_wg(m) > max_wg) return kInf;
    const int q = word == 4 ? 1 : 0, k = stage_index(m);
    return model_wg_phases(nu1, nu2) * p.alpha_stage_us[q][k] +
           model_wg_bytes(lv[l].nx, lv[l].ny, nu1, nu2, word) * p.beta_stage_us_per_B[q][k];
}

// agglomeration at level l from mode m onto mode m2: the launch that starts
// the several-workgroup part (its coarsest-level part inside it), or the
// collapse launch
static double handoff_us(int l, int L, int m, int m2, int nc, int word, const ModelParams &p, int max_wg,
                         int lcap)
{
    if (m2 <= m || l > lcap) return kInf;
    if (m2 == kSingle) return m == 0 ? model_base_us(nc, word, p) : model_base_us(nc, word, p) - p.alpha_launch_us;
    if (l >= L - 1 || model_mode_wg(m2) > max_wg) return kInf;
    return m == 0 ? p.alpha_launch_us : 0.0;
}

namespace {
struct SearchCtx {
    const ModelLevel *lv;
    int L, nu1, nu2, nc, word, max_wg, lcap;
    const ModelParams *p;
    double level(int l, int m) const { return model_level_cost(lv, L, l, m, nu1, nu2, word, *p, max_wg, lcap); }
    double handoff(int l, int m, int m2) const { return handoff_us(l, L, m, m2, nc, word, *p, max_wg, lcap); }
    int id(int l, int m, int n) const { return (l * MODEL_MODES + m) * (kMaxStages + 1) + n; }
};

// a path as the list of (level, mode) states it passes, start to goal
ModelPath path_from_states(const SearchCtx &c, const std::vector<std::pair<int, int>> &st, double g, int expanded)
{
    ModelPath r{};
    r.t_us = g + c.p->alpha_launch_us;   // norm finalisation after the cycle
    r.expanded = expanded;
    r.lstar = 0;
    // levels run in each mode: a move (l, m) -> (l-1, m) runs level l in m
    int cur_m = -1;
    for (size_t i = 1; i < st.size(); ++i) {
        const int l0 = st[i - 1].first, m0 = st[i - 1].second, l1 = st[i].first;
        if (l1 == l0 - 1 && m0 > 0 && m0 < kSingle) {
            if (m0 != cur_m) {
                if (r.nstage < 4) {
                    r.wg[r.nstage] = model_mode_wg(m0);
                    r.hi[r.nstage] = l0;
                    ++r.nstage;
                }
                cur_m = m0;
            }
        }
        if (st[i].second == kSingle && m0 != kSingle) r.lstar = l0;
    }
    return r;
}
}  // namespace

ModelPath model_search(const ModelLevel *lv, int L, int nu1, int nu2, int nc, int word, const ModelParams &p,
                       int max_wg, int lcap)
{
    const SearchCtx c{lv, L, nu1, nu2, nc, word, max_wg, lcap, &p};
    // heuristic: cheapest cost of each level left over the modes still
    // reachable, plus the cheapest hand-off into one workgroup
    std::vector<double> hs((size_t)L * MODEL_MODES, 0.0);
    const double base = model_base_us(nc, word, p);
    for (int m = 0; m < MODEL_MODES; ++m) {
        double acc = m == kSingle ? 0.0 : (m == 0 ? base : base - p.alpha_launch_us);
        hs[m] = acc;
        for (int l = 1; l < L; ++l) {
            double mn = kInf;
            for (int m2 = m; m2 < MODEL_MODES; ++m2) mn = std::min(mn, c.level(l, m2));
            if (std::isfinite(mn)) acc += mn;
            hs[(size_t)l * MODEL_MODES + m] = acc;
        }
    }
    const int nstates = L * MODEL_MODES * (kMaxStages + 1);
    std::vector<double> g(nstates, kInf);
    std::vector<int> parent(nstates, -1);
    std::vector<char> closed(nstates, 0);
    struct Node {
        double f;
        int id, l, m, n;
        bool operator<(const Node &o) const { return f > o.f || (f == o.f && id > o.id); }
    };
    std::priority_queue<Node> open;
    const int s0 = c.id(L - 1, 0, 0);
    g[s0] = 0.0;
    open.push({hs[(size_t)(L - 1) * MODEL_MODES], s0, L - 1, 0, 0});
    int expanded = 0, goal = -1;
    auto relax = [&](int from, int l, int m, int n, double cost) {
        if (!std::isfinite(cost)) return;
        const int to = c.id(l, m, n);
        const double gn = g[from] + cost;
        if (gn < g[to] && !closed[to]) {
            g[to] = gn;
            parent[to] = from;
            open.push({gn + hs[(size_t)l * MODEL_MODES + m], to, l, m, n});
        }
    };
    while (!open.empty()) {
        const Node nd = open.top();
        open.pop();
        if (closed[nd.id]) continue;
        closed[nd.id] = 1;
        ++expanded;
        if (nd.l == 0 && nd.m == kSingle) {
            goal = nd.id;
            break;
        }
        if (nd.l >= 1) relax(nd.id, nd.l - 1, nd.m, nd.n, c.level(nd.l, nd.m));
        for (int m2 = nd.m + 1; m2 < MODEL_MODES; ++m2) {
            const int n2 = nd.n + (m2 != kSingle ? 1 : 0);
            if (n2 > kMaxStages) continue;
            relax(nd.id, nd.l, m2, n2, c.handoff(nd.l, nd.m, m2));
        }
    }
    ModelPath r{};
    if (goal < 0) {
        r.t_us = kInf;
        r.expanded = expanded;
        return r;
    }
    std::vector<std::pair<int, int>> st;
    for (int v = goal; v >= 0; v = parent[v]) {
        const int n = v % (kMaxStages + 1), lm = v / (kMaxStages + 1);
        (void)n;
        st.push_back({lm / MODEL_MODES, lm % MODEL_MODES});
    }
    std::reverse(st.begin(), st.end());
    return path_from_states(c, st, g[goal], expanded);
}

ModelPath model_search_exhaustive(const ModelLevel *lv, int L, int nu1, int nu2, int nc, int word,
                                  const ModelParams &p, int max_wg, int lcap)
{
    const SearchCtx c{lv, L, nu1, nu2, nc, word, max_wg, lcap, &p};
    double best = kInf;
    std::vector<std::pair<int, int>> cur, best_st;
    int visited = 0;
    // depth-first over every path from (L-1, 0) to (0, one workgroup)
    struct Rec {
        const SearchCtx &c;
        double &best;
        std::vector<std::pair<int, int>> &cur, &best_st;
        int &visited;
        void go(int l, int m, int n, double g)
        {
            ++visited;
            cur.push_back({l, m});
            if (l == 0 && m == kSingle) {
                if (g < best) {
                    best = g;
                    best_st = cur;
                }
            } else {
                const double cl = l >= 1 ? c.level(l, m) : kInf;
                if (std::isfinite(cl)) go(l - 1, m, n, g + cl);
                for (int m2 = m + 1; m2 < MODEL_MODES; ++m2) {
                    const int n2 = n + (m2 != kSingle ? 1 : 0);
                    const double h = c.handoff(l, m, m2);
                    if (n2 <= kMaxStages && std::isfinite(h)) go(l, m2, n2, g + h);
                }
            }
            cur.pop_back();
        }
    } rec{c, best, cur, best_st, visited};
    rec.go(L - 1, 0, 0, 0.0);
    if (!std::isfinite(best)) {
        ModelPath r{};
        r.t_us = kInf;
        r.expanded = visited;
        return r;
    }
    return path_from_states(c, best_st, best, visited);
}

double model_path_us(const ModelLevel *lv, int L, int nu1, int nu2, int nc, int word, const ModelParams &p,
                     int lstar, int nstage, const int *wg, const int *hi)
{
    const SearchCtx c{lv, L, nu1, nu2, nc, word, 256, L - 1, &p};
    const int top = nstage > 0 ? hi[0] : lstar;
    double t = 0.0;
    for (int l = L - 1; l > top; --l) t += c.level(l, 0);
    for (int s = 0; s < nstage; ++s) {
        const int lo = s + 1 < nstage ? hi[s + 1] : lstar;
        int m = 1;
        while (m < kSingle && model_mode_wg(m) != wg[s]) ++m;
        for (int l = hi[s]; l > lo; --l) t += c.level(l, m);
    }
    for (int l = lstar; l >= 1; --l) t += c.level(l, kSingle);
    // the collapse launch, or the stages' launch with the collapse inside it
    // (its launch gap, then the collapse without one): the same total
    t += model_base_us(nc, word, p);
    return t + p.alpha_launch_us;
}

// ---------------------------------------------------------------------------
// 3D levels
// ---------------------------------------------------------------------------
namespace {

// loaded FP64 words per vertex of one relaxation or residual (stencil entries,
// the iterate at every stencil point, b, one store)
double words3_sweep(int npt) { return npt == 7 ? 16.0 : 56.0; }

struct Kernels3 {
    int n;             // launches
    double bytes[4];   // relaxation launch, residual, restriction + zeroing, interpolation
    int nrelax;
};

Kernels3 kernels3(const ModelLevel3 &lv, int nu1, int nu2)
{
    const double nv = (double)lv.nx * lv.ny * lv.nz;
    Kernels3 k;
    const int per = lv.npt == 7 ? 4 : 8;
    k.nrelax = (nu1 + nu2) * per;
    k.n = k.nrelax + 4;
    k.bytes[0] = nv * words3_sweep(lv.npt) * 8.0 / per;
    k.bytes[1] = nv * words3_sweep(lv.npt) * 8.0;
    k.bytes[2] = nv * (54.0 / 8.0 + 1.0 / 8.0) * 8.0;   // 27 (r, weight) pairs per coarse vertex; zeroing
    k.bytes[3] = nv * 8.25 * 8.0;                       // x in and out, r, C, 3.25 weights, x_c
    return k;
}

}  // namespace

double model3_grid_level_us(const ModelLevel3 &lv, int nu1, int nu2, const ModelParams &p)
{
    const Kernels3 k = kernels3(lv, nu1, nu2);
    // the level's working set: stencil planes, x, b, r and the weights onto it
    const double ws = (double)lv.nx * lv.ny * lv.nz * ((lv.npt == 7 ? 4.0 : 14.0) + 3.0 + 3.25) * 8.0;
    const double beta = ws > p.cache_bytes ? p.beta_hbm_us_per_B : p.beta_cache_us_per_B;
    const double t0 = p.t0_dn_us[0];
    // the zeroing launch moves little; count it as its fixed cost
    return k.nrelax * (t0 + k.bytes[0] * beta) + (t0 + k.bytes[1] * beta) + (2.0 * t0 + k.bytes[2] * beta) +
           (t0 + k.bytes[3] * beta);
}

double model3_wg_level_us(const ModelLevel3 &lv, int nu1, int nu2, const ModelParams &p)
{
    const Kernels3 k = kernels3(lv, nu1, nu2);
    const int phases = (nu1 + nu2) * 8 + 4;
    const double bytes = (nu1 + nu2) * 8 * (k.bytes[1] / 8.0) + k.bytes[1] + k.bytes[2] + k.bytes[3];
    return phases * p.alpha_bar_us[0][1] + bytes * p.beta_wg_us_per_B[0][1];
}

int model3_choose(const ModelLevel3 *lv, int L, int nu1, int nu2, int nc, const ModelParams &p, int lcap,
                  double *t_us)
{
    int best = 0;
    const int top = L - 1 < lcap ? L - 1 : lcap;
    for (int ls = 0; ls <= top; ++ls) {
        double t = model_base_us(nc, 8, p);
        for (int l = 1; l < L; ++l)
            t += l > ls ? model3_grid_level_us(lv[l], nu1, nu2, p) : model3_wg_level_us(lv[l], nu1, nu2, p);
        t_us[ls] = t;
        if (t < t_us[best]) best = ls;
    }
    return best;
}

// ---------------------------------------------------------------------------
// the paper's distributed model (section 3) and grid enumeration (section 4)
// ---------------------------------------------------------------------------
namespace {
double prod(int D, const int *n)
{
    double p = 1.0;
    for (int d = 0; d < D; ++d) p *= n[d];
    return p;
}
int ceil_div(int a, int b) { return (a + b - 1) / b; }
}  // namespace

// 2 D messages of alpha and, per dimension, two faces of n_d doubles
double paper_exchange(int D, const int *n, const PaperMachine &m)
{
    double faces = 0.0;
    for (int d = 0; d < D; ++d) faces += n[d];
    return 2.0 * D * m.alpha + 2.0 * faces * 8.0 * m.beta;
}

// 2 ns flops per point and relaxation; one exchange per colour and relaxation
double paper_smooth(int D, const int *n, int ns, int ncolors, int nu1, int nu2, const PaperMachine &m)
{
    return 2.0 * ns * prod(D, n) * (nu1 + nu2) * m.gamma + ncolors * (nu1 + nu2) * paper_exchange(D, n, m);
}

double paper_residual(int D, const int *n, int ns, const PaperMachine &m)
{
    return 2.0 * ns * prod(D, n) * m.gamma + paper_exchange(D, n, m);
}

// restriction needs no halo
double paper_restrict(int D, const int *n, int ns, const PaperMachine &m)
{
    return 2.0 * ns * prod(D, n) * m.gamma;
}

// injection at every fine point, then per coarse point the edge, face and
// cell formulas (5 and 9 flops in 2D), and the boundary lines and planes of
// the coarse block; one exchange
double paper_interp(int D, const int *n, const int *nc, const PaperMachine &m)
{
    double flops;
    if (D == 2) {
        flops = prod(2, n) + 20.0 * prod(2, nc) + 6.0 * ((double)nc[0] + nc[1]);
    } else {
        flops = prod(3, n) + 60.0 * prod(3, nc) + 15.0 * (double)nc[0] * nc[2] + 6.0 * (double)nc[1] * nc[2] +
                (double)nc[2];
    }
    return flops * m.gamma + paper_exchange(D, n, m);
}

// a processor block of the finer grid sends its pieces to one coarse
// processor: a binomial gather of log2 p_block messages and the block's data
double paper_agglomerate(int D, const int *N, const int *pf, const int *pc, int redundant, const PaperMachine &m)
{
    bool shrinks = false;
    for (int d = 0; d < D; ++d) shrinks = shrinks || pf[d] > pc[d];
    if (!shrinks) return 0.0;
    double pblock = 1.0, nblock = 1.0;
    for (int d = 0; d < D; ++d) {
        pblock *= ceil_div(pf[d], pc[d]);
        nblock *= ceil_div(N[d], pc[d]);
    }
    const double gather = std::ceil(std::log2(pblock)) * m.alpha + nblock * (pblock - 1.0) / pblock * 8.0 * m.beta;
    return gather + (redundant ? 0.0 : gather);
}

int paper_enumerate(int D, const int *N, const int *P, int max, int *grids)
{
    int p[4] = {1, 1, 1, 1};
    int count = 0;
    for (;;) {
        bool full = true;
        for (int d = 0; d < D; ++d) full = full && p[d] >= P[d];
        if (full || count >= max) break;
        for (int d = 0; d < D; ++d) grids[count * D + d] = p[d];
        ++count;
        // refine the dimension with the largest agglomerated local size that can still grow
        int best = -1;
        for (int d = 0; d < D; ++d)
            if (p[d] < P[d] && (best < 0 || ceil_div(N[d], p[d]) > ceil_div(N[best], p[best]))) best = d;
        p[best] = std::min(2 * p[best], P[best]);
    }
    return count;
}

namespace {

using Grid = std::vector<int>;

// one level on p from global N to its coarsening Nn (the coarse level on the same grid)
double paper_level(const PaperSetup &s, const Grid &N, const Grid &Nn, const Grid &p)
{
    int n[3], nc[3];
    for (int d = 0; d < s.D; ++d) {
        n[d] = ceil_div(N[d], p[d]);
        nc[d] = ceil_div(Nn[d], p[d]);
    }
    return paper_smooth(s.D, n, s.ns, s.ncolors, s.nu1, s.nu2, s.m) + paper_residual(s.D, n, s.ns, s.m) +
           paper_restrict(s.D, n, s.ns, s.m) + paper_interp(s.D, n, nc, s.m);
}

bool at_one(const Grid &p)
{
    for (int v : p)
        if (v != 1) return false;
    return true;
}

// true while the level on p may coarsen once more
bool coarsens(const PaperSetup &s, const Grid &N, const Grid &p, bool anywhere)
{
    for (int d = 0; d < s.D; ++d) {
        if (N[d] <= s.coarsest) return false;
        if (!anywhere && ceil_div(N[d], p[d]) <= s.limit) return false;
    }
    return true;
}

Grid halve(const Grid &N)
{
    Grid r(N.size());
    for (size_t d = 0; d < N.size(); ++d) r[d] = ceil_div(N[d], 2);
    return r;
}

// the levels on 1 x ... x 1 down to the coarsest and the Cholesky solve
double paper_tail(const PaperSetup &s, Grid N)
{
    const Grid one(s.D, 1);
    double t = 0.0;
    while (coarsens(s, N, one, true)) {
        const Grid Nn = halve(N);
        t += paper_level(s, N, Nn, one);
        N = Nn;
    }
    double nn = 1.0;
    for (int v : N) nn *= v;
    return t + nn * nn * s.m.gamma;
}

double paper_agg(const PaperSetup &s, const Grid &N, const Grid &pf, const Grid &pc)
{
    return paper_agglomerate(s.D, N.data(), pf.data(), pc.data(), s.redundant, s.m);
}

struct Searcher {
    const PaperSetup &s;
    std::map<std::pair<Grid, Grid>, std::pair<double, std::vector<Grid>>> memo;
    // cheapest continuation from (N, p)
    std::pair<double, std::vector<Grid>> go(Grid N, const Grid &p)
    {
        if (at_one(p)) return {paper_tail(s, N), {}};
        double run = 0.0;
        while (coarsens(s, N, p, false)) {
            const Grid Nn = halve(N);
            run += paper_level(s, N, Nn, p);
            N = Nn;
        }
        const auto key = std::make_pair(N, p);
        auto it = memo.find(key);
        if (it == memo.end()) {
            int grids[64 * 3];
            const int cnt = paper_enumerate(s.D, N.data(), p.data(), 64, grids);
            std::pair<double, std::vector<Grid>> best{std::numeric_limits<double>::infinity(), {}};
            for (int k = 0; k < cnt; ++k) {
                const Grid q(grids + k * s.D, grids + (k + 1) * s.D);
                auto sub = go(N, q);
                const double t = paper_agg(s, N, p, q) + sub.first;
                if (t < best.first) {
                    best.first = t;
                    best.second.assign(1, q);
                    best.second.insert(best.second.end(), sub.second.begin(), sub.second.end());
                }
            }
            it = memo.emplace(key, best).first;
        }
        return {run + it->second.first, it->second.second};
    }
};

}  // namespace

double paper_search(const PaperSetup &s, const int *N, const int *P, std::vector<std::vector<int>> *path)
{
    Searcher se{s, {}};
    auto r = se.go(Grid(N, N + s.D), Grid(P, P + s.D));
    if (path) *path = r.second;
    return r.first;
}

double paper_path_cost(const PaperSetup &s, const int *N0, const int *P, const std::vector<std::vector<int>> &seq)
{
    Grid N(N0, N0 + s.D), p(P, P + s.D);
    double t = 0.0;
    size_t k = 0;
    for (;;) {
        if (at_one(p)) return t + paper_tail(s, N);
        while (coarsens(s, N, p, false)) {
            const Grid Nn = halve(N);
            t += paper_level(s, N, Nn, p);
            N = Nn;
        }
        if (k >= seq.size()) return std::numeric_limits<double>::infinity();
        t += paper_agg(s, N, p, seq[k]);
        p = seq[k++];
    }
}

// remaining levels from N priced on p down to the coarsest, plus the coarse solve
static double paper_h(const PaperSetup &s, Grid N, const Grid &p)
{
    double t = 0.0;
    while (coarsens(s, N, p, true)) {
        const Grid Nn = halve(N);
        t += paper_level(s, N, Nn, p);
        N = Nn;
    }
    double nn = 1.0;
    for (int v : N) nn *= v;
    return t + nn * nn * s.m.gamma;
}

double paper_astar(const PaperSetup &s, const int *N0, const int *P, std::vector<std::vector<int>> *path,
                   int *expanded)
{
    struct Node {
        double f, g;
        Grid N, p;
        int parent;
        bool goal;
    };
    std::vector<Node> nodes;
    auto cmp = [&](int a, int b) { return nodes[a].f > nodes[b].f; };
    std::priority_queue<int, std::vector<int>, decltype(cmp)> open(cmp);
    // the start: coarsen on P to its limit
    Grid N(N0, N0 + s.D), p(P, P + s.D);
    double g0 = 0.0;
    if (at_one(p)) {
        if (path) path->clear();
        if (expanded) *expanded = 1;
        return paper_tail(s, N);
    }
    while (coarsens(s, N, p, false)) {
        const Grid Nn = halve(N);
        g0 += paper_level(s, N, Nn, p);
        N = Nn;
    }
    nodes.push_back({g0 + paper_h(s, N, p), g0, N, p, -1, false});
    open.push(0);
    int exp = 0;
    std::map<std::pair<Grid, Grid>, double> best_g;
    while (!open.empty()) {
        const int id = open.top();
        open.pop();
        if (nodes[id].goal) {
            if (path) {
                path->clear();
                for (int k = id; nodes[k].parent >= 0; k = nodes[k].parent) path->insert(path->begin(), nodes[k].p);
            }
            if (expanded) *expanded = exp;
            return nodes[id].g;
        }
        const auto key = std::make_pair(nodes[id].N, nodes[id].p);
        auto it = best_g.find(key);
        if (it != best_g.end() && it->second <= nodes[id].g) continue;
        best_g[key] = nodes[id].g;
        ++exp;
        const Grid Nc = nodes[id].N, pc = nodes[id].p;
        const double gc = nodes[id].g;
        int grids[64 * 3];
        const int cnt = paper_enumerate(s.D, Nc.data(), pc.data(), 64, grids);
        for (int k = 0; k < cnt; ++k) {
            const Grid q(grids + k * s.D, grids + (k + 1) * s.D);
            double g = gc + paper_agg(s, Nc, pc, q);
            if (at_one(q)) {
                g += paper_tail(s, Nc);
                nodes.push_back({g, g, Nc, q, id, true});
            } else {
                Grid Nq = Nc;
                while (coarsens(s, Nq, q, false)) {
                    const Grid Nn = halve(Nq);
                    g += paper_level(s, Nq, Nn, q);
                    Nq = Nn;
                }
                nodes.push_back({g + paper_h(s, Nq, q), g, Nq, q, id, false});
            }
            open.push((int)nodes.size() - 1);
        }
    }
    if (expanded) *expanded = exp;
    return std::numeric_limits<double>::infinity();
}

}  // namespace hbmg
