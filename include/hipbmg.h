/*
 * hipbmg.h -- C interface of hipbmg, a structured variational multigrid solver
 * for 2D heterogeneous diffusion on AMD MI355X (gfx950).
 *
 * Method: Reisner, Olson, Moulton, "Scaling Structured Multigrid to 500K+
 * Cores through Coarse-Grid Redistribution" (arXiv 1803.02481):
 *   - section 2: operator-induced interpolation, Galerkin coarse operators
 *     A_{l-1} = P_l^T A_l P_l on a fixed 9-point pattern, standard coarsening
 *     by two, four-colour Gauss-Seidel relaxation, the V-cycle of Algorithm 1;
 *   - section 3: the interpolate-and-correct step u += P u_c + r/C, the
 *     Cholesky coarse-grid solve factored at setup, and the alpha-beta-gamma
 *     performance model (equations for T_smooth, T_residual, T_restrict,
 *     T_interp, T_agglomerate, T_cgsolve, summed as T_V-cycle);
 *   - sections 2.2 and 4: coarse-grid redistribution chosen by that model.  On
 *     one GPU the redistribution becomes the choice of the level l* below which
 *     grid-wide kernel launches stop and all coarser levels run inside one
 *     persistent workgroup.
 *
 * Conventions shared by every entry point:
 *   - Grids are vertex grids of nx x ny points including the boundary ring;
 *     nx and ny are odd and >= 3.  Unknowns are the interior vertices; the
 *     boundary carries the homogeneous Dirichlet value 0.
 *   - Every array argument is a DEVICE pointer (hipMalloc / torch CUDA tensor
 *     memory) unless the name ends in _host.  Arrays are row-major, x fastest,
 *     contiguous: a vertex field is [ny][nx]; a cell field is [ny-1][nx-1]
 *     with cell (i,j) = [x_i, x_i+1] x [y_j, y_j+1]; a stencil is a stack of
 *     planes [nplanes][ny][nx].
 *   - Stencil planes: 5-point {C, W, S}; 9-point {C, W, S, SW, SE}.  C is the
 *     diagonal entry, the others are positive connection values: the matrix
 *     entry between p=(i,j) and its west neighbour is -W(i,j), east -W(i+1,j),
 *     south -S(i,j), north -S(i,j+1), south-west -SW(i,j), north-east
 *     -SW(i+1,j+1), south-east -SE(i,j), north-west -SE(i-1,j+1).  Values that
 *     couple to boundary vertices may be present; they multiply u = 0.
 *   - stream is a hipStream_t (NULL = the null stream).  All device work of a
 *     call is ordered on it.  Calls that return convergence information
 *     synchronise the stream before returning.
 *   - Every call returns a hipbmg_status and never throws; hipbmg_last_error()
 *     gives a message for the calling thread's last failure.
 *   - The caller owns every array it passes.  A handle owns all device memory
 *     of its hierarchy.  Setup takes it from the allocator registered with
 *     hipbmg_set_allocator, or from hipMalloc if none is registered; solves
 *     allocate nothing.  hipbmg_destroy returns every block to the allocator
 *     that made it, and the handle's small pinned host buffers to a pool the
 *     library keeps for the process.  Destroy first synchronises the whole
 *     device (hipDeviceSynchronize), because a registered allocator may hand a
 *     block out again at once and the next handle may take the pinned
 *     buffers; it therefore waits for work on every stream, not only the
 *     caller's.  A handle serves one stream at a time; calls on one handle
 *     must not overlap.
 */
#ifndef HIPBMG_H
#define HIPBMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hipbmg_hier *hipbmg_handle;

typedef enum {
    HIPBMG_OK = 0,
    HIPBMG_EINVAL = 1,   /* bad size, null pointer, bad parameter          */
    HIPBMG_ENOMEM = 2,   /* device allocation failed                       */
    HIPBMG_EHIP = 3,     /* a HIP runtime call failed                      */
    HIPBMG_ENOTSPD = 4,  /* coarsest operator not positive definite        */
    HIPBMG_ENOCONV = 5,  /* max_cycles reached before tol; u = last iterate */
    HIPBMG_ENAN = 6      /* residual norm is not finite                    */
} hipbmg_status;

typedef enum { HIPBMG_FP64 = 0, HIPBMG_MIXED = 1 } hipbmg_precision;

#define HIPBMG_MAX_LEVELS 24
#define HIPBMG_MAX_HIST 1024

typedef struct {
    int nu1;                 /* pre-relaxations per level (Algorithm 1), default 2          */
    int nu2;                 /* post-relaxations per level, default 1                       */
    int coarsest_n;          /* coarsen while both sides are odd and exceed this, default 3 */
    int collapse_level;      /* -1: chosen by the performance model; k >= 0: levels 0..k    */
                             /* run in one persistent workgroup (0 = coarsest solve only)   */
    int residual_correction; /* 1: add r/C at fine-only vertices after interpolation (sec 3) */
    int max_cycles;          /* FP64: V-cycles; mixed: total inner cycles cap, default 500  */
    int precision;           /* hipbmg_precision, default HIPBMG_FP64                       */
    int inner_max_cycles;    /* mixed: FP32 cycles per refinement step, default 32          */
    double inner_tol;        /* mixed: inner relative residual target, default 1e-4; a step */
                             /* stops its inner solve already at tol / (2 relres) when that */
                             /* is looser (what the outer tolerance still needs)            */
    int use_graph;           /* 1: replay the V-cycle as a captured hipGraph, default 1     */
    int cluster_wg;          /* agglomeration stages on several workgroups between the      */
                             /* grid-wide kernels and the collapsed workgroup (section 4):  */
                             /* -1 chosen with l* by the model's A* search (default; needs  */
                             /* collapse_level = -1), 0 none, K = 2, 4, ..., 256 one stage   */
                             /* of K workgroups forced (with collapse_level and cluster_top) */
    int cluster_top;         /* forced stage: its highest level, collapse_level < cluster_top */
                             /* <= L - 2                                                      */
} hipbmg_params;

typedef struct {
    int cycles;              /* V-cycles run (mixed: FP32 inner cycles, all steps)          */
    int outer_steps;         /* mixed: refinement steps; FP64: equals cycles                */
    double relres;           /* final ||b - A u||_2 / ||b||_2, FP64, interior vertices      */
    int levels;              /* number of levels L                                          */
    int collapse_level;      /* l* in use                                                   */
    double model_us[HIPBMG_MAX_LEVELS]; /* model time of one cycle for each l*, microseconds */
    double setup_ms;         /* wall time of hipbmg_setup                                   */
    double solve_ms;         /* wall time of the solve call                                 */
    double relres_hist[HIPBMG_MAX_HIST]; /* relres after each cycle (mixed: each step)     */
    int rb_down[HIPBMG_MAX_LEVELS]; /* row-pair steps per tile, pre-relaxation kernels, level l */
    int rb_up[HIPBMG_MAX_LEVELS];   /* row-pair steps per tile, interpolation kernels, level l  */
    int rb_pipelined;        /* row-pair steps per tile of the pipelined finest kernel, 0 if */
                             /* the finest level is not pipelined                            */
    int cluster_stages;      /* agglomeration stages in use above l* (0: grid-wide kernels   */
                             /* down to l*, then one workgroup)                               */
    int cluster_wg[4];       /* workgroups of each stage, decreasing                         */
    int cluster_hi[4];       /* highest level of each stage                                  */
    double search_us;        /* model time of one cycle along the path the search found     */
    int search_expanded;     /* states the A* search expanded                                */
    double path_us;          /* model time of one cycle of the configuration in use (l* and */
                             /* stages, searched or forced)                                   */
} hipbmg_info;

/* Fill *p with the defaults above. */
void hipbmg_default_params(hipbmg_params *p);

/* Device memory of the handles (the 2D, batched and 3D hierarchies: level
 * planes, weights, factors, launch tables) comes from this allocator, for
 * callers that pool device memory themselves (PyTorch's caching allocator,
 * for one).  alloc_fn(bytes, ctx) returns a device pointer on the current
 * device, 256-byte aligned, or NULL on failure (the call then fails with
 * HIPBMG_ENOMEM; a misaligned block is handed back and the call fails).
 * free_fn(ptr, ctx) releases it.  Both NULL restores hipMalloc/hipFree;
 * exactly one NULL is HIPBMG_EINVAL.  The setting is process-wide and applies
 * to allocations made after the call; each block is returned to the
 * allocator that made it, whenever its handle is destroyed.  Before handing
 * such blocks back the library waits for the device, so memory the allocator
 * gives out again is no longer in use by the library's streams.  The
 * callbacks may be called from any library call that builds or destroys a
 * handle (the solves allocate nothing), and from the worker threads of
 * hipbmg_setup_batched, so they must be thread-safe.  A 2D hierarchy asks for
 * one block sized for all its levels (and a little more) at setup and cuts its
 * arrays from it; only arrays that no longer fit ask for more (blocks of 1, 2,
 * 4, 8, then 16 MiB, or one block per array larger than 8 MiB).  The one-time
 * machine calibration keeps its scratch on hipMalloc.  Host only; thread-safe. */
typedef void *(*hipbmg_alloc_fn)(size_t bytes, void *ctx);
typedef void (*hipbmg_free_fn)(void *ptr, void *ctx);
hipbmg_status hipbmg_set_allocator(hipbmg_alloc_fn alloc_fn, hipbmg_free_fn free_fn, void *ctx);

/* Build the multigrid hierarchy for the operator given by `coeffs`
 * ([3][ny][nx] if npt == 5, [5][ny][nx] if npt == 9; see the plane convention
 * above).  On the GPU: operator-induced interpolation weights and the Galerkin
 * product for every level (section 2), the Cholesky factor of the coarsest
 * operator (section 3, coarse-solve cost), and the collapse level l* from the
 * performance model (sections 3 and 4) unless params->collapse_level >= 0.  With
 * cluster_wg = -1 (the default) and collapse_level = -1, l* and any
 * agglomeration stages above it come from the model's A* search over
 * (level, workgroups) states (section 4); info reports the path.
 * coeffs is copied and may be freed after return.  params may be NULL for the
 * defaults.  Returns HIPBMG_ENOTSPD if the coarsest factorisation fails. */
hipbmg_status hipbmg_setup(int nx, int ny, int npt, const double *coeffs,
                           const hipbmg_params *params, void *stream, hipbmg_handle *out);

/* Solve A u = b by V(nu1,nu2)-cycles (Algorithm 1) until
 * ||b - A u||_2 / ||b||_2 <= tol over interior vertices, or max_cycles.
 * b: [ny][nx] right-hand side (boundary entries ignored).  u: [ny][nx], the
 * initial guess on entry (boundary entries ignored), the iterate on return
 * (boundary entries set to 0).  precision HIPBMG_MIXED runs FP32 V-cycles as
 * the inner solver of FP64 iterative refinement; the outer residual, the norms
 * and the coarsest solve stay FP64.  info may be NULL.  If ||b|| = 0 then u = 0.
 * Returns HIPBMG_ENOCONV if tol was not reached (u holds the last iterate). */
hipbmg_status hipbmg_solve(hipbmg_handle h, const double *b, double *u, double tol, void *stream,
                           hipbmg_info *info);

/* Release every device buffer of the handle. NULL is accepted. */
hipbmg_status hipbmg_destroy(hipbmg_handle h);

/* Number of levels and the size of level l (0 = coarsest). */
hipbmg_status hipbmg_level_size(hipbmg_handle h, int l, int *nx_host, int *ny_host);

/* Copy level l's stencil planes {C, W, S, SW, SE} into out ([5][ny][nx],
 * device).  The finest level is stored as given (SW = SE = 0 for npt 5). */
hipbmg_status hipbmg_get_stencil(hipbmg_handle h, int l, double *out, void *stream);

/* Copy the interpolation weights from level l-1 to level l (l >= 1) into out
 * ([8][cny][cnx], device, coarse size).  For coarse vertex (I,J) the planes
 * hold the weights of the fine vertices of the coarse cell [I,I+1]x[J,J+1]:
 *   0: (2I+1,2J)   on (I,J)      1: (2I+1,2J)   on (I+1,J)
 *   2: (2I,2J+1)   on (I,J)      3: (2I,2J+1)   on (I,J+1)
 *   4: (2I+1,2J+1) on (I,J)      5: (2I+1,2J+1) on (I+1,J)
 *   6: (2I+1,2J+1) on (I,J+1)    7: (2I+1,2J+1) on (I+1,J+1)
 * Weights on boundary coarse vertices and rows of boundary fine vertices are 0. */
hipbmg_status hipbmg_get_interp(hipbmg_handle h, int l, double *out, void *stream);

/* Single solve-phase operations on level l, in the plain [ny][nx] layout,
 * exposed for checking the fused kernels one by one (they overwrite level l's
 * internal right-hand side and iterate buffers; a later hipbmg_solve is not
 * affected):
 *   op_smooth: `sweeps` four-colour Gauss-Seidel relaxations of A_l x = b,
 *     x updated in place (section 2).
 *   op_smooth_restrict (l >= 1): `sweeps` (1 or 2, the latter as one fused pass)
 *     relaxations, then the residual r = b - A_l x,
 *     q = r / C at vertices that are not coarse points (q = 0 elsewhere), and
 *     bc = P_l^T r ([cny][cnx]) (Algorithm 1, residual and restriction).
 *   op_interp_smooth (l >= 1): x += P_l xc (plus q at vertices that are not
 *     coarse points if rescorr), then one relaxation (Algorithm 1, interpolate
 *     and correct; section 3, the r/C term); if sumsq_host is not NULL it
 *     receives ||b - A_l x||^2 after the relaxation. */
hipbmg_status hipbmg_op_smooth(hipbmg_handle h, int l, const double *b, double *x, int sweeps,
                               void *stream);
hipbmg_status hipbmg_op_smooth_restrict(hipbmg_handle h, int l, const double *b, double *x,
                                        int sweeps, double *q, double *bc, void *stream);
hipbmg_status hipbmg_op_interp_smooth(hipbmg_handle h, int l, const double *b, double *x,
                                      const double *q, const double *xc, int rescorr,
                                      double *sumsq_host, void *stream);

/* The FP32 levels of a mixed-precision handle (precision HIPBMG_MIXED; any
 * other handle gives HIPBMG_EINVAL).  Mixed precision keeps setup in FP64 and
 * demotes every level once to an edge form: the connections W, S, SW, SE
 * rounded to float, and in place of C the excess E = C - (sum of the eight
 * connections of the vertex, including those that couple to boundary
 * vertices), formed in FP64 and rounded.  The FP32 kernels apply
 *   (A x)_p = sum_q conn_pq (x_p - x_q) + E_p x_p,  diagonal sum_q conn_pq + E_p,
 * so rows of pure diffusion keep a zero row sum after rounding.  The inner
 * FP32 V-cycles of iterative refinement run on these levels; the coarsest
 * level is solved with the FP64 Cholesky factor.
 *   get_level32: level l's planes {E, W, S, SW, SE} into stencil_out
 *     ([5][ny][nx], float, device) and, if interp_out is not NULL (l >= 1),
 *     the FP32 weights into interp_out ([8][cny][cnx], plane order as in
 *     hipbmg_get_interp).
 *   op32_smooth, op32_smooth_restrict, op32_interp_smooth: the FP32 forms of
 *     the three single operations above, on float arrays; q holds r / diag.
 *   op32_inner: the inner solve of one refinement step: up to `cycles` FP32
 *     V-cycles (Algorithm 1, the finest level's passes as in a solve) on
 *     A e = r from e = 0, each followed by the test
 *     ||r - A e||_2 / rnorm <= inner_tol (norm accumulated in FP64 over
 *     interior vertices; inner_tol 0 runs every cycle).  r: [ny][nx] float
 *     (the demoted outer residual), e: [ny][nx] float output, rnorm > 0 the
 *     FP64 norm of the outer residual.  hist_host (NULL or [cycles]) receives
 *     the inner relative residual after each cycle run, cycles_host (NULL or
 *     one int) their number. */
hipbmg_status hipbmg_get_level32(hipbmg_handle h, int l, float *stencil_out, float *interp_out, void *stream);
hipbmg_status hipbmg_op32_smooth(hipbmg_handle h, int l, const float *b, float *x, int sweeps, void *stream);
hipbmg_status hipbmg_op32_smooth_restrict(hipbmg_handle h, int l, const float *b, float *x, int sweeps,
                                          float *q, float *bc, void *stream);
hipbmg_status hipbmg_op32_interp_smooth(hipbmg_handle h, int l, const float *b, float *x, const float *q,
                                        const float *xc, int rescorr, double *sumsq_host, void *stream);
hipbmg_status hipbmg_op32_inner(hipbmg_handle h, const float *r, float *e, int cycles, double rnorm,
                                double inner_tol, double *hist_host, int *cycles_host, void *stream);

/* The quantity of the convergence test (relative residual, the stopping
 * criterion of every solve) for any operator and iterate:
 * out_host[0] = ||b - A u||_2 and out_host[1] = ||b||_2, both over interior
 * vertices, with A given by coeffs ([3 or 5][ny][nx] planes, npt 5 or 9, the
 * plane format above) and b, u [ny][nx] (device).  Entries of u on the
 * boundary ring are read as 0.  Any nx, ny >= 3.  The sums of squares are
 * reduced in a fixed order, so equal inputs give equal bits.  Per-workgroup
 * partial sums go to scratch device memory taken for the call from the
 * registered allocator (or hipMalloc) and returned before the call returns.
 * Synchronises the stream.  EINVAL on a null pointer or bad sizes, ENOMEM if
 * the scratch cannot be had, EHIP on a launch or copy failure. */
hipbmg_status hipbmg_residual_norm(int nx, int ny, int npt, const double *coeffs, const double *b,
                                   const double *u, double *out_host, void *stream);

/* hipbmg_residual_norm for callers that cannot allocate device memory (code
 * under stream capture, serving loops, harnesses that forbid hipMalloc): the
 * same arguments, kernels and results (bitwise), but the partial sums live in
 * a fixed 512 KiB array of each device's global memory that the library holds
 * until the process ends.  No hipMalloc, hipFree or other allocating call is
 * made.  Grids whose partials exceed the array (more than 32767 workgroups of
 * 256 columns x 64 rows; every grid up to 16385 x 16385 fits) give EINVAL
 * before any device work.  All calls on one device share its array: calls that
 * overlap on one device race and must be serialised by the caller. */
hipbmg_status hipbmg_residual_norm_noalloc(int nx, int ny, int npt, const double *coeffs, const double *b,
                                           const double *u, double *out_host, void *stream);

/* Batched solves of many independent problems of different sizes (each with
 * its own hierarchy, built as by hipbmg_setup, and its own collapse level).
 * One launch runs the same V-cycle stage (Algorithm 1) of all problems; the
 * collapsed levels run one workgroup per problem; converged problems are
 * retired on the device and skipped by later launches; with use_graph one
 * cycle is captured as a hipGraph and replayed.  precision HIPBMG_MIXED runs
 * the FP32 V-cycles of all problems inside FP64 iterative refinement.
 * nx, ny: host arrays [nprob]; coeffs: host array of nprob device pointers to
 * [3 or 5][ny][nx] planes (npt 5 or 9 for every problem).  b, u: host arrays
 * of nprob device pointers to [ny][nx]; u holds the initial guesses on entry.
 * infos: NULL or a host array [nprob].  Returns HIPBMG_ENOCONV if any problem
 * did not reach tol (every u holds its last iterate).  hipbmg_setup_batched
 * builds the first problem's hierarchy on `stream` and the others on up to 8
 * host threads of its own, each with its own stream (HIPBMG_SETUP_THREADS
 * sets the count; 1 builds them all on `stream`), and returns when all are
 * built; a registered allocator's callbacks may therefore be called from
 * those threads. */
typedef struct hipbmg_batch *hipbmg_batch_handle;
hipbmg_status hipbmg_setup_batched(int nprob, const int *nx_host, const int *ny_host, int npt,
                                   const double *const *coeffs_host, const hipbmg_params *params,
                                   void *stream, hipbmg_batch_handle *out);
hipbmg_status hipbmg_solve_batched(hipbmg_batch_handle h, const double *const *b_host,
                                   double *const *u_host, double tol, void *stream,
                                   hipbmg_info *infos_host);
hipbmg_status hipbmg_destroy_batched(hipbmg_batch_handle h);
/* The tile shape the batch's autotuner chose at setup (row-block length of a
 * tile, as for a single problem, and the number of neighbouring strips, one
 * wave each, that share a workgroup): strips_per_group (1, 2 or 4), rb_cap
 * (the cap on row-pair steps per tile, 0 for the single-problem rule) and rb,
 * the row-pair steps per tile that level `level` (0 = coarsest) of problem
 * `problem` uses (0 for a level inside the collapse).  Any output may be
 * NULL.  EINVAL for a NULL handle or an index out of range. */
hipbmg_status hipbmg_batch_tile_shape(hipbmg_batch_handle h, int problem, int level, int *strips_per_group,
                                      int *rb_cap, int *rb);

/* Vertex-centred 5-point finite-volume stencil of -div(D grad u) (section 5):
 * the face between vertices p and q takes the mean of the two cells it cuts,
 * C is the sum of the four connections.  cell: [ny-1][nx-1] holding D, or
 * theta = ln D if is_log.  coeffs_out: [3][ny][nx] planes {C, W, S}. */
hipbmg_status hipbmg_fv5_from_cells(int nx, int ny, const double *cell, int is_log,
                                    double *coeffs_out, void *stream);

/* hipbmg_fv5_from_cells for nprob problems of one size in one launch, the
 * same values problem by problem: cell [nprob][ny-1][nx-1], coeffs_out
 * [nprob][3][ny][nx] (device).  EINVAL for null pointers, nprob outside
 * 1..65535 or nx, ny < 3. */
hipbmg_status hipbmg_fv5_from_cells_batched(int nprob, int nx, int ny, const double *cell, int is_log,
                                            double *coeffs_out, void *stream);

/* The same stencil for a diagonal diffusion tensor D = diag(Dx, Dy) per cell
 * on a grid of spacings hx, hy (section 5: the stretched grids with
 * compensating anisotropy D = diag(1/r, r)).  The dual face of an x-edge has
 * length hy across a distance hx and takes (hy/hx) times the mean Dx of the two
 * cells it cuts; a y-edge takes (hx/hy) times the mean Dy.  dx_cell, dy_cell:
 * [ny-1][nx-1] device arrays; coeffs_out: [3][ny][nx] planes {C, W, S}.
 * EINVAL for null pointers, nx or ny < 3, or a spacing that is not positive. */
hipbmg_status hipbmg_fv5_aniso(int nx, int ny, const double *dx_cell, const double *dy_cell, double hx,
                               double hy, double *coeffs_out, void *stream);

/* Gradient of a scalar loss with respect to theta = ln D per cell, given the
 * solution u and the adjoint lam = A^{-1} dL/du:
 *   g_c = -(D_c/2) * sum over the four edges (p,q) of cell c of
 *         (lam_p - lam_q)(u_p - u_q)          (boundary values 0).
 * theta: [ny-1][nx-1]; u, lam: [ny][nx]; grad_out: [ny-1][nx-1]. */
hipbmg_status hipbmg_grad_logD(int nx, int ny, const double *theta, const double *u,
                               const double *lam, double *grad_out, void *stream);

/* hipbmg_grad_logD for nprob problems of one size in one launch, the same
 * values problem by problem: theta, grad_out [nprob][ny-1][nx-1]; u, lam
 * [nprob][ny][nx] (device).  EINVAL for null pointers, nprob outside
 * 1..65535 or nx, ny < 3. */
hipbmg_status hipbmg_grad_logD_batched(int nprob, int nx, int ny, const double *theta, const double *u,
                                       const double *lam, double *grad_out, void *stream);

/* Live timing of the relaxation kernels, the per-component timers of the
 * paper's experiments (section 5) for one GPU.  While enabled, every solve
 * records HIP events on the solve stream around each finest-level streaming
 * kernel (enable = 1), or around every streaming kernel of every level and
 * the collapse launch (enable = 2; more events, so slightly slower solves).
 * enable = 0 stops and keeps the totals; enable = 1 or 2 clears them.
 * profile_read returns, for one precision (0 FP64, 1 FP32 inner) and
 * one kernel index (0 relax, 1 relax from zero, 2 relax + residual +
 * restriction, 3 the same from zero, 4 interpolate + relax, 5 the same + norm,
 * 6 relax + norm, 7 two relaxations + residual + restriction in one pass,
 * 8 the same from zero, 9 interpolate + relax + norm followed by the next
 * cycle's two relaxations + residual + restriction in one pass, 10 its
 * interpolate + relax stage alone, which rebuilds the stopping cycle's
 * iterate, 11 and 12 kernels 7 and 8 without storing r/C, 13 interpolate
 * with r/C formed from the loaded rows + relax, 14 kernel 10 with the norm,
 * the last cycle of a solve that reaches max_cycles), the summed
 * duration, the number of launches and the
 * algorithmic bytes one launch moves.  Any output pointer may be NULL. */
hipbmg_status hipbmg_profile(hipbmg_handle h, int enable);
hipbmg_status hipbmg_profile_read(hipbmg_handle h, int precision, int kernel,
                                  double *total_ms_host, long long *launches_host,
                                  double *bytes_per_launch_host);

/* Per-level totals recorded with enable = 2, for one precision: for level l,
 * ms_host[3l] the down leg (pre-relaxations, residual, restriction),
 * ms_host[3l+1] the up leg (interpolation and post-relaxations), ms_host[3l+2]
 * the collapse launch whose top level is l; n_host the matching launch
 * counts.  Both arrays hold 3 * HIPBMG_MAX_LEVELS entries (n_host may be
 * NULL).  For the pipelined finest level the single pass is counted in its
 * up leg. */
hipbmg_status hipbmg_profile_levels(hipbmg_handle h, int precision, double *ms_host, long long *n_host);

/* The performance model's terms for this hierarchy, in microseconds per
 * V-cycle (section 3 model; parameters as at setup): grid_us_host[l] the
 * level's grid-wide kernels, wg_us_host[l] the level inside the collapse
 * workgroup, base_us_host[0] the collapse launch holding only the coarsest
 * level (launch gap and coarse solve included).  Arrays of HIPBMG_MAX_LEVELS
 * entries; entries past the number of levels are 0. */
hipbmg_status hipbmg_model_levels(hipbmg_handle h, double *grid_us_host, double *wg_us_host,
                                  double *base_us_host);

/* Measure the machine parameters of the collapse-level performance model on
 * the current device, as the paper measures its alpha, beta and gamma
 * (section 3, postal model; section 5, machine parameters from benchmarks):
 * the gap between dependent kernel launches and the streaming bandwidth of the
 * relaxation's access mix out of HBM and out of cache, with micro-kernels;
 * then, on a synthetic 257 x 257 hierarchy built and destroyed inside the
 * call, the solver's own kernels: the row-pair step latency and fixed cost of the
 * down and up streaming kernels, and per collapsed level the cost of a barrier phase and
 * the workgroup's inverse bandwidth, fitted separately for levels staged in
 * LDS and levels left in global memory, in FP64 and FP32.  The values replace
 * the process-wide model parameters used by later hipbmg_setup calls.
 * out_host (may be NULL) receives 64 doubles:
 *   [0] alpha_launch_us  [1] hbm_GBps  [2] cache_GBps
 *   [3] step_dn_us FP64  [4] step_up_us FP64  [5] step_dn_us FP32  [6] step_up_us FP32
 *   [7] t_base_us FP64 (collapsed launch holding only the coarsest level)  [8] t_base_us FP32
 *   [9] alpha_bar_us FP64 LDS  [10] alpha_bar_us FP64 global
 *   [11] alpha_bar_us FP32 LDS  [12] alpha_bar_us FP32 global
 *   [13] wg_GBps FP64 LDS  [14] wg_GBps FP64 global  [15] wg_GBps FP32 LDS  [16] wg_GBps FP32 global
 *   [17] bare LDS barrier us  [18] bare barrier after an L2 access us
 *   [19] one workgroup's L2 bandwidth GBps  [20] step of a plain relaxation sweep us
 *   [21] t0_dn_us FP64  [22] t0_up_us FP64  [23] t0_dn_us FP32  [24] t0_up_us FP32 (fixed cost of
 *        a down / up streaming kernel after the previous kernel)
 *   [25..32] alpha_stage_us FP64 and [33..40] stage GBps FP64 of an agglomeration
 *        stage of 2, 4, ..., 256 workgroups (barrier phase cost; bytes of a level
 *        per second), [41..48] and [49..56] the same for FP32 (sizes the
 *        device cannot hold at once keep the uncalibrated defaults)
 *   [57..63] 0.
 * Every timing of the solver's kernels is taken cold (after a 512 MB write
 * has evicted the caches), as the kernels run inside a solve.
 * Allocates about 1 GB of device memory for the duration of the call (with
 * hipMalloc; its internal hierarchy takes the registered allocator, if any).
 * The parameters are process-wide and replaced at the end of the call: do not
 * run it while another thread builds a hierarchy. */
hipbmg_status hipbmg_calibrate(void *stream, double *out_host);

/* Message for the calling thread's most recent failure ("" if none). */
/* The paper's distributed V-cycle model in its own form (section 3), host
 * only, no device calls.  D = 2 or 3 dimensions, L levels (0 coarsest),
 * N_host [L][D] global grid points per level, P_host [L][D] processor grid
 * per level (local sizes ceil(N/P)), ns stencil points, ncolors smoother
 * colours, V(nu1,nu2), redundant = 1 if the coarse solution is not scattered
 * back, alpha (s), beta (s/B), gamma (s/flop).  terms_host [L][6] (may be
 * NULL): per level smoothing, residual, restriction, interpolation (the 2D
 * and 3D interpolation cost equations), agglomeration (gather of level l-1's
 * right-hand side, and scatter, when P shrinks from level l to l-1), and at
 * level 0 the coarse solve (agglomeration onto one processor plus the
 * Cholesky substitutions, (prod N^0)^2 gamma).  total_host: their sum,
 * T_V-cycle. */
hipbmg_status hipbmg_paper_model(int D, int L, const int *N_host, const int *P_host, int ns, int ncolors,
                                 int nu1, int nu2, int redundant, double alpha, double beta, double gamma,
                                 double *terms_host, double *total_host);

/* The coarse processor grids the paper's redistribution search runs over
 * (section 4, coarse processor grid enumeration): for a global coarse grid
 * N_host [D] on processor grid P_host [D], start from 1 x ... x 1 and double
 * one dimension at a time, the one whose agglomerated local size
 * ceil(N_d / p_d) is largest among those still below P_d, stopping before P.
 * grids_host [max][D]; *count_host = number written.  Host only. */
hipbmg_status hipbmg_paper_enumerate(int D, const int *N_host, const int *P_host, int max, int *grids_host,
                                     int *count_host);

/* The redistribution search of section 4 over that model.  A state is a
 * global grid and a processor grid.  Levels coarsen (N -> ceil(N/2)) while
 * every local side ceil(N_d/p_d) exceeds `limit` (the coarsening limit) and
 * every global side exceeds `coarsest`; at the limit the solve agglomerates
 * onto one of the enumerated coarser processor grids; on 1 x ... x 1 the
 * levels continue to `coarsest` and end in the Cholesky solve. */
typedef struct {
    int D, limit, coarsest, ns, ncolors, nu1, nu2, redundant;
    double alpha, beta, gamma;
} hipbmg_paper_setup;

/* Cheapest redistribution path from fine global grid N_host [D] on processor
 * grid P_host [D]: path_host [max_path][D] the grids after the first, ending
 * with 1 x ... x 1, *len_host their number, *t_host the model time of one
 * V-cycle along it (seconds).  Host only. */
hipbmg_status hipbmg_paper_search(const hipbmg_paper_setup *setup, const int *N_host, const int *P_host,
                                  int max_path, int *path_host, int *len_host, double *t_host);

/* The same search by A* (section 4, f(s) = g(s) + h(s)): g is the model time
 * down to state s, h the remaining levels priced on s's processor grid plus
 * the Cholesky solve.  A grid only shrinks along a path and no level is
 * cheaper on fewer processors, so h never overestimates and the path found
 * is a cheapest one (its time equals hipbmg_paper_search's up to summation
 * order; among equally cheap paths either may be returned).  Outputs as
 * there, plus *expanded_host = states taken off the open list.  Host only. */
hipbmg_status hipbmg_paper_astar(const hipbmg_paper_setup *setup, const int *N_host, const int *P_host,
                                 int max_path, int *path_host, int *len_host, double *t_host, int *expanded_host);

/* Model time of one V-cycle along the given sequence of processor grids
 * (path_host [len][D], the grids after the first); infinite if the sequence
 * ends before 1 x ... x 1. */
hipbmg_status hipbmg_paper_path_cost(const hipbmg_paper_setup *setup, const int *N_host, const int *P_host,
                                     const int *path_host, int len, double *t_host);

const char *hipbmg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HIPBMG_H */
