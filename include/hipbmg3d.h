/*
 * hipbmg3d.h -- C interface of hipbmg's 3D path: the structured variational
 * multigrid solver for 3D heterogeneous diffusion on AMD MI355X (gfx950).
 *
 * Method: Reisner, Olson, Moulton, "Scaling Structured Multigrid to 500K+
 * Cores through Coarse-Grid Redistribution" (arXiv 1803.02481), in three
 * dimensions:
 *   - section 2: operator-induced interpolation, Galerkin coarse operators
 *     A_{l-1} = P_l^T A_l P_l on a fixed 27-point pattern, standard coarsening
 *     by two in every direction, the V-cycle of Algorithm 1;
 *   - section 3: the 3D interpolation (its cost equation counts the coarse
 *     lines, faces and cells that the three passes of the construction visit),
 *     the interpolate-and-correct step u += P u_c + r/C, and the Cholesky
 *     coarse-grid solve factored at setup.
 * The relaxation is eight-colour Gauss-Seidel, colour (i mod 2) + 2 (j mod 2)
 * + 4 (k mod 2), colours 0..7 in turn.
 *
 * Interpolation (the paper prints no formulas; this is the 3D form of the
 * operator-induced reading used in 2D).  A fine vertex with no odd index is a
 * coarse point (weight 1).  One odd index: the stencil is summed over the
 * plane normal to that direction, giving a three-point relation along the
 * coarse line.  Two odd indices: the stencil is summed along the normal of
 * the coarse face and the vertex is eliminated against its eight in-face
 * neighbours.  Three odd indices: the vertex is eliminated against all 26
 * neighbours.  Weights on boundary coarse vertices are 0.
 *
 * Conventions (those of hipbmg.h, plus):
 *   - Grids are vertex grids of nx x ny x nz points including the boundary;
 *     every side odd and >= 3.  Levels coarsen while all three sides are odd
 *     and exceed params->coarsest_n; the coarsest level may hold at most 4096
 *     unknowns.
 *   - Arrays are DEVICE pointers, [nz][ny][nx] with x fastest (cells
 *     [nz-1][ny-1][nx-1], cell (i,j,k) = [x_i,x_i+1] x [y_j,y_j+1] x [z_k,z_k+1]).
 *   - Stencil planes, npt = 7: {C, W, S, B}: the diagonal and the positive
 *     connections to the west, south and lower neighbour (matrix entries
 *     -W(i,j,k) to (i-1,j,k), -W(i+1,j,k) to (i+1,j,k), likewise S along y and
 *     B along z).  npt = 27: 14 planes, C then -A(p, p+d) for the 13 offsets d
 *     whose linear index (dz+1)*9 + (dy+1)*3 + (dx+1) is 0..12; the entry for
 *     -d is the one stored at p-d (symmetry).
 *   - Only FP64 is provided in 3D (params->precision must be HIPBMG_FP64);
 *     cluster_wg and cluster_top are ignored.  collapse_level works as in 2D:
 *     levels 0..l* run inside one persistent workgroup (the one-GPU form of
 *     the paper's coarse-grid redistribution, sections 2.2 and 4), l* forced
 *     (0 .. min(L-1, 7)) or, with -1, the argmin of the section 3 model with 3D
 *     counts on the calibrated machine parameters.  The iteration does not
 *     depend on l*.  With use_graph
 *     (the default) each V-cycle and its residual norm are replayed from a
 *     hipGraph captured on the first solve on the caller's stream.
 *   - Inside a handle every field is held in an octant layout: eight
 *     sub-grids by index parity, so that each colour of the relaxation and
 *     each kind of interpolated vertex is one contiguous array.  The calls
 *     below take and return the plain [nz][ny][nx] layout.
 */
#ifndef HIPBMG3D_H
#define HIPBMG3D_H

#include "hipbmg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hipbmg3d_hier *hipbmg3d_handle;

/* 7-point vertex-centred finite volumes for -div(D grad u) with zero
 * Dirichlet data (section 5's problem in 3D): the connection of an edge is
 * the mean of the four cell values around it (the common factor h of a
 * uniform grid is left out), C the sum of the six connections of an interior
 * vertex.  cell: [nz-1][ny-1][nx-1] diffusivities.  planes_out: [4][nz][ny][nx]
 * {C, W, S, B}, fully written (0 where undefined). */
hipbmg_status hipbmg3d_fv7_from_cells(int nx, int ny, int nz, const double *cell, double *planes_out,
                                      void *stream);

/* Build the hierarchy for the operator `planes` (npt 7 or 27, see above):
 * interpolation weights and Galerkin products on the GPU for every level, the
 * Cholesky factor of the coarsest operator on the host (its planes are copied
 * back once).  planes is copied and may be freed after return.  params may be
 * NULL for the defaults.  HIPBMG_ENOTSPD if the coarsest factorisation meets a
 * pivot <= 0; HIPBMG_EINVAL for bad sizes or parameters. */
hipbmg_status hipbmg3d_setup(int nx, int ny, int nz, int npt, const double *planes, const hipbmg_params *params,
                             void *stream, hipbmg3d_handle *out);

/* V(nu1,nu2)-cycles until ||b - A u||_2 / ||b||_2 <= tol over the interior
 * vertices or params->max_cycles.  b, u: [nz][ny][nx]; u is the initial guess
 * on entry and the iterate on return (boundary entries set to 0).  The
 * residual norm is read back after every cycle.  info (may be NULL) gets
 * cycles, relres, relres_hist, levels, collapse_level and model_us (the
 * model's time of one cycle for each l*).  HIPBMG_ENOCONV if tol was not
 * reached, HIPBMG_ENAN on a non-finite residual. */
hipbmg_status hipbmg3d_solve(hipbmg3d_handle h, const double *b, double *u, double tol, void *stream,
                             hipbmg_info *info);

/* Release the handle's device memory.  NULL is accepted. */
hipbmg_status hipbmg3d_destroy(hipbmg3d_handle h);

/* Number of levels, and the size of level l (0 = coarsest). */
hipbmg_status hipbmg3d_num_levels(hipbmg3d_handle h, int *levels_host);
hipbmg_status hipbmg3d_level_size(hipbmg3d_handle h, int l, int *nx_host, int *ny_host, int *nz_host);

/* Level l's matrix entries: out [27][nz][ny][nx], out[o] = A(p, p+d) with
 * o = (dz+1)*9 + (dy+1)*3 + (dx+1); 0 at boundary vertices and for
 * neighbours on the boundary. */
hipbmg_status hipbmg3d_get_stencil(hipbmg3d_handle h, int l, double *out, void *stream);

/* Interpolation rows of level l (l >= 1) onto level l-1: out [8][nz][ny][nx],
 * out[4c+2b+a] at fine vertex (i,j,k) = weight on coarse vertex
 * ((i>>1)+a, (j>>1)+b, (k>>1)+c); 0 at boundary fine vertices. */
hipbmg_status hipbmg3d_get_interp(hipbmg3d_handle h, int l, double *out, void *stream);

/* Single solve-phase operations on level l in the plain layout, for checking
 * the kernels one by one (they use level l's internal buffers; a later solve
 * is not affected):
 *   op_smooth: `sweeps` eight-colour Gauss-Seidel relaxations, x in place;
 *   op_residual: r = b - A_l x at interior vertices, 0 elsewhere;
 *   op_restrict (l >= 1): bc = P_l^T r, bc of level l-1's size;
 *   op_interp_correct (l >= 1): x += P_l xc, plus r/C at vertices that are
 *     not coarse points if rescorr;
 *   op_coarse_solve: x = A_0^{-1} b on the coarsest level by the Cholesky
 *     factor. */
hipbmg_status hipbmg3d_op_smooth(hipbmg3d_handle h, int l, const double *b, double *x, int sweeps, void *stream);
hipbmg_status hipbmg3d_op_residual(hipbmg3d_handle h, int l, const double *b, const double *x, double *r,
                                   void *stream);
hipbmg_status hipbmg3d_op_restrict(hipbmg3d_handle h, int l, const double *r, double *bc, void *stream);
hipbmg_status hipbmg3d_op_interp_correct(hipbmg3d_handle h, int l, double *x, const double *r, const double *xc,
                                         int rescorr, void *stream);
hipbmg_status hipbmg3d_op_coarse_solve(hipbmg3d_handle h, const double *b, double *x, void *stream);

/* Kernel timing of the solve phase: with enable = 1 every later solve
 * brackets its finest-level relaxation, residual, restriction and
 * interpolation launches with HIP events and accumulates their durations;
 * profile_read returns, for kernel class k (0 relaxation colours of the
 * finest level, 1 finest residual, with or without the norm, 2
 * finest-to-next restriction, 3 next-to-finest interpolation, 4 everything
 * below the finest level), the summed duration in ms, the number of launches
 * and the mean algorithmic bytes of one launch (FP64 values read and written
 * once each; 0 for class 4).  A 7-point finest level whose every interior
 * diagonal is bitwise the sum of its six connections (finite volumes of pure
 * diffusion, hipbmg3d_fv7_from_cells) has that sum formed in its relaxation
 * and residual kernels instead of the C plane loaded, which shows as 8 bytes
 * per vertex fewer in classes 0 and 1.  Any output pointer may be NULL. */
hipbmg_status hipbmg3d_profile(hipbmg3d_handle h, int enable);
hipbmg_status hipbmg3d_profile_read(hipbmg3d_handle h, int k, double *ms_host, long long *launches_host,
                                    double *bytes_per_launch_host);

#ifdef __cplusplus
}
#endif

#endif
