// bmg_internal.h -- shared declarations of the hipbmg device code and host runtime.
//
// Storage of one level (all planes pitched, row j starts at j*pitch, pitch even
// and rows 256-byte aligned, padding columns hold 0):
//   coef planes C, W, S, SW, SE   (positive connections; SW = SE = 0 for a
//                                  5-point finest level)
//   x0, x1                        ping-pong iterates (streaming kernels read one
//                                 and write the other)
//   b                             right-hand side (restricted residual below the finest)
//   q                             r/C at fine-only vertices after pre-relaxation
//   wt                            8 interpolation weight planes from level l-1,
//                                 at coarse resolution (plane order as in hipbmg.h)
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <vector>

namespace hbmg {

// Set the message hipbmg_last_error() returns on the calling thread.
void set_last_error(const char *msg);

// Device memory owned by a handle: from the allocator registered with
// hipbmg_set_allocator, else hipMalloc.  dev_free_all returns every block of
// v to whichever allocator made it (waiting for the device first when a
// registered allocator is involved, since such memory may be handed out again
// at once) and clears v.
hipError_t dev_malloc(void **p, size_t bytes);
void dev_free_all(std::vector<void *> &v);
// a zeroed pinned host buffer of at most 512 bytes, mapped (dev, if not null,
// gets its device address) and coherent, from a pool kept for the process;
// pinned_small_free returns it to the pool (null is accepted)
hipError_t pinned_small(void **host, void **dev, size_t bytes);
void pinned_small_free(void *host);
// a zeroed pinned host block of at least `bytes` (its size, a power of two of
// at least 4 KiB, in *cap) from a per-size pool kept for the process;
// pinned_block_free returns it (null is accepted)
hipError_t pinned_block(void **host, size_t bytes, size_t *cap);
void pinned_block_free(void *host, size_t cap);

// Weight plane indices (fine vertex of coarse cell (I,J) -> coarse corner).
enum { WXL = 0, WXR = 1, WYB = 2, WYT = 3, WCSW = 4, WCSE = 5, WCNW = 6, WCNE = 7 };

template <typename T>
struct LevelDev {
    int nx, ny, pitch, npt;
    size_t plane;          // elements per plane (ny * pitch)
    T *C, *W, *S, *SW, *SE;
    T *x[2];
    T *b, *q;
    T *wt;                 // weights from the next-coarser level onto this one (null on level 0)
    int cpitch;            // pitch of the coarser level
    size_t cplane;         // plane size of the coarser level
};

// Arguments of the streaming relaxation kernel.
template <typename T>
struct StreamArgs {
    int nx, ny, pitch;
    const T *C, *W, *S, *SW, *SE, *b;
    const T *x_in;
    T *x_out;
    T *x_out2;           // SV_FUSED3: the iterate after the next pre-relaxations
    // interpolate-and-correct on load (up-leg)
    const T *xc, *wt, *q_in;
    int cnx, cny, cpitch;
    long long cplane;
    int rescorr;
    // residual -> q, restriction -> bc (down-leg)
    T *q_out, *bc;
    // norm partial sums, one per tile
    double *partials;
    int nstrips, nblocks, rb, ntiles;
    // the solve's run flag (null: always run); a launch whose flag reads 0
    // returns at once (the convergence test of an earlier cycle was met)
    const int *active;
    // SV_FUSED3*: the level's diagonal is the sum of its four connections
    // (FP64, checked bitwise at setup) or its FP32 excess is zero: the pass
    // forms the diagonal itself instead of loading the C plane
    int zexc;
    // SV_FUSED3* on an FP64 level: the pass forms the interpolation weights
    // from the rows it loads instead of reading the stored ones (bitwise equal)
    int wform;
};

enum StreamVariant {
    SV_SWEEP = 0,        // one relaxation
    SV_SWEEP_ZX = 1,     // one relaxation from x = 0 (x not read)
    SV_SWEEP_RQ = 2,     // relaxation, residual -> q, restriction -> bc
    SV_SWEEP_RQ_ZX = 3,
    SV_INTERP = 4,       // interpolate-and-correct on load, then relaxation
    SV_INTERP_NORM = 5,  // ... plus residual norm partials
    SV_SWEEP_NORM = 6,   // relaxation plus residual norm partials
    SV_SWEEP2_RQ = 7,    // two relaxations, residual -> q, restriction -> bc
    SV_SWEEP2_RQ_ZX = 8, // the same from x = 0
    SV_FUSED3 = 9,       // 5-point finest level: interpolate (r/C formed from the loaded
                         // iterate) + relax (norm), then two relaxations (-> x_out2),
                         // residual, restriction -> bc
    SV_FUSED3_P = 10,    // the interpolate + relax stage of SV_FUSED3 alone (-> x_out)
    SV_SWEEP2_R = 11,    // SV_SWEEP2_RQ without storing q (the up leg forms r/C itself)
    SV_SWEEP2_R_ZX = 12, // the same from x = 0
    SV_INTERP_RC = 13,   // interpolate-and-correct with r/C formed from the loaded rows, relaxation
    SV_FUSED3_PN = 14,   // SV_FUSED3_P plus the residual norm: a capped solve's last cycle
    SV_COUNT = 15
};

// Owned column pairs per strip for a variant (64 lanes minus halo lanes).
int stream_owned_pairs(int npt, int variant);
// Launch geometry for a level.
void stream_geometry(int nx, int ny, int npt, int variant, int rb, int *nstrips, int *nblocks,
                     int *ntiles, int *grid);
// workgroups of a single-problem streaming kernel (one 64-lane wave each) that
// the device holds at once (compute units x occupancy); 0 if unknown
int stream_resident(int npt, int variant, int fp32);
// row-pair steps one tile of the variant walks for a row block of rb steps
// (its own rb plus the prologue that rebuilds the state below the block)
int stream_steps_per_tile(int variant, int rb);
template <typename T>
hipError_t launch_stream(int npt, int variant, const StreamArgs<T> &a, int grid, hipStream_t s);
// one launch over many problems: map[w] = (problem, tile) of wave w,
// args[problem]; wpg waves (strips) per workgroup, 1, 2 or 4
template <typename T>
hipError_t launch_stream_batched(int npt, int variant, const StreamArgs<T> *args, const int2 *map,
                                 int nmap, const int *active, int wpg, hipStream_t s);

// the pipelined finest pass (SV_FUSED3, or SV_FUSED3_P for the rebuild of a
// stopped cycle's iterate) over many problems: map[w] = (problem, tile) of
// wave w, args[problem]; zc: every problem's pass forms its diagonal; active
// may be null (every problem in the map runs)
template <typename T>
hipError_t launch_stream3_batched(int variant, int zc, const StreamArgs<T> *args, const int2 *map, int nmap,
                                  const int *active, int wpg, hipStream_t s);

// ZC9 (9-point levels whose rows at least two vertices from the boundary have
// zero row sums): set = 0 sets *flag (device int) to 1 if every such vertex's
// diagonal is within 1e-12 of the ordered sum of its eight connections, else
// 0; set = 1 stores that sum as their diagonal if *flag is 1 (read on the
// device, so no host round trip between the two).  The FP32 check sets *flag to
// 1 if the edge-form excess is exactly zero there.  The streaming kernels of
// SV_SWEEP2_R_ZX and SV_INTERP_RC take a.zexc = 1 on such a level.
hipError_t launch_rowsum_diag(const LevelDev<double> &A, int *flag, int set, hipStream_t s);
hipError_t launch_zero_excess9(const LevelDev<float> &A, int *flag, hipStream_t s);

// Tile kernels of the small 9-point coarse levels (V(2,1)): a workgroup of nw
// waves (4 or 8) owns a strip by tile_steps(nw, down) row-pair steps.  down:
// two relaxations from zero, residual, r/C and restriction (the work of
// SV_SWEEP2_RQ_ZX); up: interpolate and correct, one relaxation (SV_INTERP).
// a.nstrips / a.ntiles come from tile_geometry; one workgroup per tile.
int tile_steps(int nw, int down);
void tile_geometry(int nx, int ny, int npt, int nw, int down, int *nstrips, int *nblocks, int *ntiles);
template <typename T>
hipError_t launch_tile(int down, int nw, const StreamArgs<T> &a, hipStream_t s);

// 1 if every interior vertex of a 5-point level has C exactly equal to
// ((W_p + W_e) + S_p) + S_n (FP64), or an FP32 edge-form excess of exactly 0;
// the result goes to *flag (device int, written by the check)
hipError_t launch_zero_excess_check(const LevelDev<double> &A, int *flag, hipStream_t s);
hipError_t launch_zero_excess_check(const LevelDev<float> &A, int *flag, hipStream_t s);

// Setup kernels.
// nprob problems of one size (cells one after another; problem k's planes
// k * ostride elements after the first's)
hipError_t launch_fv5(int nx, int ny, const double *cell, int is_log, double *C, double *W,
                      double *S, int pitch, hipStream_t s, int nprob = 1, size_t ostride = 0);
hipError_t launch_fv5_aniso(int nx, int ny, const double *dx_cell, const double *dy_cell, double hx, double hy,
                            double *C, double *W, double *S, int pitch, hipStream_t s);
hipError_t launch_grad_logD(int nx, int ny, const double *theta, const double *u,
                            const double *lam, double *g, hipStream_t s, int nprob = 1);
hipError_t launch_interp_weights(const LevelDev<double> &f, int cnx, int cny, double *wt,
                                 int cpitch, size_t cplane, hipStream_t s);
hipError_t launch_rap(const LevelDev<double> &f, const LevelDev<double> &c, hipStream_t s);
// weights and Galerkin products of levels l_top .. 1 (each coarse level of at
// most SETUP_TAIL_POINTS vertices, l_top <= SETUP_TAIL_MAX) in one launch of
// one workgroup, the same values as launch_interp_weights and launch_rap
// level by level
constexpr int SETUP_TAIL_MAX = 6, SETUP_TAIL_POINTS = 512;
hipError_t launch_setup_tail(const LevelDev<double> *lv, int l_top, hipStream_t s);

// Collapsed coarse levels: one persistent workgroup runs levels top..0 of the
// V-cycle.  The iterate of a collapsed level below `top` is x[1] and x[0] holds
// its residual; at `top` the iterate is x[xb_top] and the residual x[1 - xb_top].
// Levels 0..lds_top are staged in LDS for the whole launch.
constexpr int COLLAPSE_MAX_LEVELS = 24;
constexpr int COLLAPSE_LDS_BUDGET = 150 * 1024;   // dynamic LDS bytes for staged levels
template <typename T>
struct CollapseArgs {
    const LevelDev<T> *levels;   // device array, index = level
    int top, xb_top, zero_top;   // zero_top: start level `top` from x = 0
    int nu1, nu2, rescorr;
    const double *chol;          // coarsest Cholesky factor (nc x nc, lower, row-major), FP64
    const int *cidx;             // coarsest vertex (row-major [ny0][nx0]) -> unknown or -1
    int nc;
    double *work;                // nc doubles
    double *partials;            // want_norm: partials[0] = ||b - A x||^2 at level top
    int want_norm;
    int lds_top;                 // highest level staged in LDS (-1: none)
    int lds_bytes;               // dynamic LDS of the launch
    int lds_off[COLLAPSE_MAX_LEVELS];   // byte offset of each staged level
    const int *active;                  // run flag as in StreamArgs (null: always run)
};
template <typename T>
hipError_t launch_collapse(const CollapseArgs<T> &a, hipStream_t s);

// Agglomeration stages between the grid-wide kernels and the collapsed
// workgroup (section 4: the coarse grid moves onto fewer and fewer
// processors).  One launch of wg[0] workgroups: stage s runs levels
// hi[s] down to hi[s+1]+1 on its first wg[s] workgroups, with a grid barrier
// where the single workgroup has a workgroup barrier; workgroup 0 then runs
// the collapse of levels 0..col.top (= hi[nstage]); the up legs follow in
// reverse order.  The stages' workgroup counts decrease.
constexpr int CLUSTER_MAX_STAGES = 4;
template <typename T>
struct ClusterArgs {
    CollapseArgs<T> col;                 // levels 0..col.top on workgroup 0 (from zero, no norm)
    int nstage;
    int wg[CLUSTER_MAX_STAGES];
    int hi[CLUSTER_MAX_STAGES + 1];
    int xb_top;                          // iterate buffer of level hi[0] (its residual: the other)
    unsigned *bar;                       // per stage: arrival count, generation
    int *err;                            // set when a barrier wait gives up
    const int *active;                   // run flag as in StreamArgs
};
template <typename T>
hipError_t launch_cluster(const ClusterArgs<T> &a, hipStream_t s);
// workgroups of the cluster kernel that fit on the device at once with
// `lds_bytes` of dynamic LDS each (0 on error)
template <typename T>
int cluster_max_resident(int lds_bytes);
template <typename T>
size_t collapse_lds_bytes(int nx, int ny, int cnx, int cny);
hipError_t collapse_set_attributes();
template <typename T>
hipError_t launch_collapse_batched(const CollapseArgs<T> *args, int nprob, int lds_bytes,
                                   const int *active, hipStream_t s);

// batched norm helpers (see bmg_collapse.hip)
hipError_t launch_sumsq_batched(const double *const *v, const int4 *dims, int nprob, double *partials,
                                int nparts, hipStream_t s);
// out[p] = sqrt(sum of problem p's partials) (/ denom[p]); an active problem
// whose value is <= the tolerance (or not finite) is retired.  The tolerance
// is tol_dev[tol_stride * p] when tol_dev is not null (read when the kernel
// runs, so a captured graph sees the values written before each replay; one
// for all problems with stride 0, one per problem with stride 1), else tol.
hipError_t launch_finalize_batched(const double *partials, const int *off, const int *cnt,
                                   const double *denom, double *out, int *active, double tol,
                                   const double *tol_dev, int nprob, hipStream_t s, int tol_stride = 0);
hipError_t launch_count_active(const int *active, int n, int *count, hipStream_t s);

// Sum of squares of interior entries of a pitched field -> partials.
hipError_t launch_sumsq(const double *v, int nx, int ny, int pitch, double *partials, int nparts,
                        hipStream_t s);
// out[0] = sqrt(sum(partials)) / denom_src[0] (denom_src may be null -> plain norm).
hipError_t launch_finalize_norm(const double *partials, int n, const double *denom, double *out,
                                hipStream_t s);
// Convergence test after cycle k of a solve: ||r|| / denom[0] from the norm
// partials (the same fixed-order reduction as launch_finalize_norm) goes to
// last[0], to hist[k-1] (if k <= hist_cap) and, with the flag state, to the four doubles
// at slot {relres, run flag, stopping cycle, k} (host-mapped memory read by
// the host a few cycles later).  When relres <= tol, or is not finite, the run
// flag flags[0] is cleared and flags[1] = k, flags[2] = 1 (met) or 2 (not
// finite).  Nothing is written once the flag is clear.
hipError_t launch_finalize_check(const double *partials, int n, const double *denom, double tol, int k,
                                 double *hist, int hist_cap, double *last, int *flags, double *slot,
                                 hipStream_t s);
// flags[0] = 1 (run), flags[1] = flags[2] = 0: the start of a solve
hipError_t launch_flags_reset(int *flags, hipStream_t s);

}  // namespace hbmg
