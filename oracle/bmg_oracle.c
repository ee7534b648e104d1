/*
 * bmg_oracle.c -- plain, slow, FP64 reference implementation of the structured
 * variational multigrid V-cycle for 2D diffusion (Reisner, Olson, Moulton,
 * "Scaling Structured Multigrid to 500K+ Cores through Coarse-Grid
 * Redistribution", arXiv 1803.02481).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg load it.  It shares no code, header, table or helper with
 * the GPU path, and the GPU path never calls it.
 *
 * Everything is written out from the definitions, with no blocking, fusion or
 * reordering:
 *   - the operator is held as an explicit 3x3 matrix-entry stencil per vertex,
 *     A(p, p+d), with entries towards boundary vertices set to zero (the
 *     boundary is not an unknown; the diagonal keeps the Dirichlet part);
 *   - interpolation P is held as explicit rows: each fine vertex carries four
 *     weights on the corners of the coarse cell that contains it;
 *   - the Galerkin product is the triple sum A_c(I,J) = sum_p sum_q
 *     P(p,I) A(p,q) P(q,J) scattered over all fine couplings (section 2);
 *   - the smoother is four-colour Gauss-Seidel, one colour at a time;
 *   - the V-cycle follows Algorithm 1 (section 2) with the residual term r/C
 *     added at fine-only points after interpolation (section 3, interpolation
 *     cost paragraph, following Dendy 2010);
 *   - the coarsest problem is solved by a dense Cholesky factorisation
 *     computed once at setup (section 3, coarse-solve cost equation).
 *
 * Parity unpinned: the exact BoxMG interpolation heuristics are not printed in
 * the paper.  The collapse formulas below are the reading used throughout
 * (operator-induced, motivated by continuity of the normal flux, section 2);
 * the tests pin them by closed forms (bilinear for D=1, flux-weighted for
 * coefficients that vary in one direction only) rather than by BoxMG itself.
 *
 * Threads: the loops over rows of one colour, of the residual and of the
 * interpolation run in parallel (OpenMP).  Their points are independent (no
 * two points of one colour couple), so the results are bitwise those of one
 * thread; restriction (a scatter), norms and setup stay sequential.
 *
 * Floating point: double throughout, built with -ffp-contract=off, except the
 * FP32 edge-form section at the end, which emulates the inner solver of mixed
 * precision with float arithmetic on a once-demoted copy of every level.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define MAXLEV 32

typedef struct {
    int nx, ny;
    double *A;  /* [ny][nx][9]: A(p, p+(dx,dy)) at index (dy+1)*3+(dx+1)  */
    double *P;  /* [ny][nx][4]: interpolation row of fine vertex (i,j) onto the
                   corners ((i>>1)+a, (j>>1)+b) of level l-1, index 2*b+a.
                   Unused on the coarsest level.                              */
    double *x, *b, *r;
    /* FP32 edge form (mixed precision), built by oracle32_demote:
     * A32[..][k] for k != 4 is the connection -A(p, p+d) rounded to float,
     * A32[..][4] the excess A(p,p) - (sum of the connections) computed in
     * double and rounded to float; P32 is P rounded to float. */
    float *A32, *P32, *x32, *b32, *r32;
} olevel;

typedef struct {
    int L;
    olevel lev[MAXLEV];   /* lev[0] coarsest ... lev[L-1] finest */
    int nc;               /* unknowns on the coarsest level */
    int *cidx;            /* [ny0][nx0] -> unknown number or -1 */
    double *chol;         /* nc x nc lower factor, row-major */
    int nu1, nu2, rescorr;
} ohier;

static int interior(const olevel *lv, int i, int j)
{
    return i >= 1 && i <= lv->nx - 2 && j >= 1 && j <= lv->ny - 2;
}

static double *Aent(const olevel *lv, int i, int j, int dx, int dy)
{
    return &lv->A[((size_t)j * lv->nx + i) * 9 + (dy + 1) * 3 + (dx + 1)];
}

/* ---------------------------------------------------------------------------
 * Vertex-centred 5-point finite volume discretisation of -div(D grad u)
 * (section 5, diffusion equation with homogeneous Dirichlet data).
 * cellD[(ny-1)][(nx-1)] holds a constant diffusivity per cell
 * [x_i, x_i+1] x [y_j, y_j+1].  The flux through the dual-cell face crossing
 * edge (i,j)-(i+1,j) is the mean of the two cells that the face cuts.
 * Output in the library's plane format: C, W, S as [ny][nx], W and S being
 * positive connection values (matrix entry = -W).  The connection of the
 * east-most / north-most interior vertex to the boundary is stored at the
 * boundary column / row.
 * ------------------------------------------------------------------------- */
static double cellv(const double *D, int nx, int ny, int ci, int cj)
{
    if (ci < 0 || cj < 0 || ci >= nx - 1 || cj >= ny - 1) return 0.0;
    return D[(size_t)cj * (nx - 1) + ci];
}

void oracle_fv5(int nx, int ny, const double *cellD, double *C, double *W, double *S)
{
    size_t n = (size_t)nx * ny;
    memset(C, 0, n * sizeof(double));
    memset(W, 0, n * sizeof(double));
    memset(S, 0, n * sizeof(double));
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            /* edge (i-1,j)-(i,j): face cuts cells (i-1,j-1) and (i-1,j) */
            if (i >= 1 && j >= 1 && j <= ny - 2)
                W[(size_t)j * nx + i] = 0.5 * (cellv(cellD, nx, ny, i - 1, j - 1) +
                                              cellv(cellD, nx, ny, i - 1, j));
            /* edge (i,j-1)-(i,j): face cuts cells (i-1,j-1) and (i,j-1) */
            if (j >= 1 && i >= 1 && i <= nx - 2)
                S[(size_t)j * nx + i] = 0.5 * (cellv(cellD, nx, ny, i - 1, j - 1) +
                                              cellv(cellD, nx, ny, i, j - 1));
        }
    for (int j = 1; j <= ny - 2; ++j)
        for (int i = 1; i <= nx - 2; ++i) {
            size_t p = (size_t)j * nx + i;
            C[p] = W[p] + W[p + 1] + S[p] + S[p + nx];
        }
}

/* Section 5, the paper's own workload: a diagonal diffusion tensor
 * D = diag(Dx, Dy) per cell on a grid of spacings hx, hy.  The flux through
 * the dual face of an x-edge is the integral of Dx du/dx over the face: the
 * face has length hy, half of it in each of the two cells it cuts, and
 * du/dx = (u_q - u_p) / hx, so the connection is
 *   (hy/2 * Dx(cell below) + hy/2 * Dx(cell above)) / hx;
 * a y-edge likewise with Dy, hx and hy exchanged.  C is the sum of the four
 * connections of the vertex. */
void oracle_fv5_aniso(int nx, int ny, const double *Dx, const double *Dy, double hx, double hy, double *C,
                      double *W, double *S)
{
    size_t n = (size_t)nx * ny;
    memset(C, 0, n * sizeof(double));
    memset(W, 0, n * sizeof(double));
    memset(S, 0, n * sizeof(double));
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            /* x-edge (i-1,j)-(i,j): face x = x_{i-1/2}, cells (i-1,j-1) and (i-1,j) */
            if (i >= 1 && j >= 1 && j <= ny - 2) {
                double flux = 0.5 * hy * cellv(Dx, nx, ny, i - 1, j - 1) + 0.5 * hy * cellv(Dx, nx, ny, i - 1, j);
                W[(size_t)j * nx + i] = flux / hx;
            }
            /* y-edge (i,j-1)-(i,j): face y = y_{j-1/2}, cells (i-1,j-1) and (i,j-1) */
            if (j >= 1 && i >= 1 && i <= nx - 2) {
                double flux = 0.5 * hx * cellv(Dy, nx, ny, i - 1, j - 1) + 0.5 * hx * cellv(Dy, nx, ny, i, j - 1);
                S[(size_t)j * nx + i] = flux / hy;
            }
        }
    for (int j = 1; j <= ny - 2; ++j)
        for (int i = 1; i <= nx - 2; ++i) {
            size_t p = (size_t)j * nx + i;
            C[p] = W[p] + W[p + 1] + S[p] + S[p + nx];
        }
}

/* ---------------------------------------------------------------------------
 * Hierarchy construction.
 * ------------------------------------------------------------------------- */
static void level_alloc(olevel *lv, int nx, int ny)
{
    size_t n = (size_t)nx * ny;
    lv->nx = nx;
    lv->ny = ny;
    lv->A = calloc(n * 9, sizeof(double));
    lv->P = calloc(n * 4, sizeof(double));
    lv->x = calloc(n, sizeof(double));
    lv->b = calloc(n, sizeof(double));
    lv->r = calloc(n, sizeof(double));
}

/* Import the finest operator from the plane format {C,W,S[,SW,SE]}. */
static void import_stencil(olevel *lv, int npt, const double *planes)
{
    int nx = lv->nx, ny = lv->ny;
    size_t n = (size_t)nx * ny;
    const double *C = planes, *W = planes + n, *S = planes + 2 * n;
    const double *SW = npt == 9 ? planes + 3 * n : NULL;
    const double *SE = npt == 9 ? planes + 4 * n : NULL;
    for (int j = 1; j <= ny - 2; ++j)
        for (int i = 1; i <= nx - 2; ++i) {
            size_t p = (size_t)j * nx + i;
            double e[9] = {0};
            e[4] = C[p];
            e[3] = -W[p];                    /* west  */
            e[5] = -W[p + 1];                /* east  */
            e[1] = -S[p];                    /* south */
            e[7] = -S[p + nx];               /* north */
            if (npt == 9) {
                e[0] = -SW[p];               /* south-west */
                e[8] = -SW[p + nx + 1];      /* north-east */
                e[2] = -SE[p];               /* south-east */
                e[6] = -SE[p + nx - 1];      /* north-west */
            }
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int k = (dy + 1) * 3 + (dx + 1);
                    if (k != 4 && !interior(lv, i + dx, j + dy)) e[k] = 0.0;
                    *Aent(lv, i, j, dx, dy) = e[k];
                }
        }
}

/* Operator-induced interpolation from level l-1 (coarse) to level l (fine),
 * section 2.  Rows are built in two passes: coarse-aligned vertices first
 * (injection, or a one-dimensional collapse along the coarse line), then the
 * cell centres, which eliminate their eight neighbours using the rows of the
 * first pass. */
static void prow_add(const olevel *f, int pi, int pj, double *dst, int qi, int qj, double s)
{
    const double *q = &f->P[((size_t)qj * f->nx + qi) * 4];
    for (int b = 0; b <= 1; ++b)
        for (int a = 0; a <= 1; ++a) {
            double w = q[2 * b + a];
            if (w == 0.0) continue;
            int ci = (qi >> 1) + a - (pi >> 1);
            int cj = (qj >> 1) + b - (pj >> 1);
            if (ci < 0 || ci > 1 || cj < 0 || cj > 1) abort();
            dst[2 * cj + ci] += s * w;
        }
}

static void build_interp(olevel *f, const olevel *c)
{
    int nx = f->nx, ny = f->ny;
    memset(f->P, 0, (size_t)nx * ny * 4 * sizeof(double));
    /* pass 1: vertices on coarse lines */
    for (int j = 1; j <= ny - 2; ++j)
        for (int i = 1; i <= nx - 2; ++i) {
            double *pr = &f->P[((size_t)j * nx + i) * 4];
            if (i % 2 == 0 && j % 2 == 0) {
                pr[0] = 1.0;
            } else if (i % 2 == 1 && j % 2 == 0) {
                /* on a coarse x-line: sum the stencil over each column */
                double den = *Aent(f, i, j, 0, 0) + *Aent(f, i, j, 0, 1) + *Aent(f, i, j, 0, -1);
                double aw = *Aent(f, i, j, -1, 0) + *Aent(f, i, j, -1, 1) + *Aent(f, i, j, -1, -1);
                double ae = *Aent(f, i, j, 1, 0) + *Aent(f, i, j, 1, 1) + *Aent(f, i, j, 1, -1);
                pr[0] = -aw / den;
                pr[1] = -ae / den;
            } else if (i % 2 == 0 && j % 2 == 1) {
                /* on a coarse y-line: sum the stencil over each row */
                double den = *Aent(f, i, j, 0, 0) + *Aent(f, i, j, 1, 0) + *Aent(f, i, j, -1, 0);
                double as = *Aent(f, i, j, 0, -1) + *Aent(f, i, j, 1, -1) + *Aent(f, i, j, -1, -1);
                double an = *Aent(f, i, j, 0, 1) + *Aent(f, i, j, 1, 1) + *Aent(f, i, j, -1, 1);
                pr[0] = -as / den;
                pr[2] = -an / den;
            }
        }
    /* pass 2: cell centres, e_p = -sum_{q != p} A(p,q) e_q / A(p,p) */
    for (int j = 1; j <= ny - 2; ++j)
        for (int i = 1; i <= nx - 2; ++i) {
            if (!(i % 2 == 1 && j % 2 == 1)) continue;
            double *pr = &f->P[((size_t)j * nx + i) * 4];
            double diag = *Aent(f, i, j, 0, 0);
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    double a = *Aent(f, i, j, dx, dy);
                    if (a == 0.0) continue;
                    prow_add(f, i, j, pr, i + dx, j + dy, -a / diag);
                }
        }
    /* coarse boundary vertices are not unknowns: no weight on them */
    for (int j = 1; j <= ny - 2; ++j)
        for (int i = 1; i <= nx - 2; ++i)
            for (int b = 0; b <= 1; ++b)
                for (int a = 0; a <= 1; ++a)
                    if (!interior(c, (i >> 1) + a, (j >> 1) + b))
                        f->P[((size_t)j * nx + i) * 4 + 2 * b + a] = 0.0;
}

/* Galerkin coarse operator A_c = P^T A P (section 2), as the triple sum over
 * every fine coupling (p,q) and every pair of coarse columns. */
static void build_galerkin(const olevel *f, olevel *c)
{
    memset(c->A, 0, (size_t)c->nx * c->ny * 9 * sizeof(double));
    for (int pj = 1; pj <= f->ny - 2; ++pj)
        for (int pi = 1; pi <= f->nx - 2; ++pi) {
            const double *Pp = &f->P[((size_t)pj * f->nx + pi) * 4];
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int qi = pi + dx, qj = pj + dy;
                    double a = *Aent(f, pi, pj, dx, dy);
                    if (a == 0.0 || !interior(f, qi, qj)) continue;
                    const double *Pq = &f->P[((size_t)qj * f->nx + qi) * 4];
                    for (int k = 0; k < 4; ++k) {
                        if (Pp[k] == 0.0) continue;
                        int Ii = (pi >> 1) + (k & 1), Ij = (pj >> 1) + (k >> 1);
                        for (int m = 0; m < 4; ++m) {
                            if (Pq[m] == 0.0) continue;
                            int Ji = (qi >> 1) + (m & 1), Jj = (qj >> 1) + (m >> 1);
                            int ex = Ji - Ii, ey = Jj - Ij;
                            if (ex < -1 || ex > 1 || ey < -1 || ey > 1) abort();
                            *Aent(c, Ii, Ij, ex, ey) += Pp[k] * a * Pq[m];
                        }
                    }
                }
        }
}

/* Dense Cholesky factorisation of the coarsest operator (interior unknowns). */
static int factor_coarsest(ohier *h)
{
    olevel *c = &h->lev[0];
    int nx = c->nx, ny = c->ny;
    h->cidx = malloc((size_t)nx * ny * sizeof(int));
    int n = 0;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            h->cidx[j * nx + i] = interior(c, i, j) ? n++ : -1;
    h->nc = n;
    double *M = calloc((size_t)n * n, sizeof(double));
    for (int j = 1; j <= ny - 2; ++j)
        for (int i = 1; i <= nx - 2; ++i)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (!interior(c, i + dx, j + dy)) continue;
                    M[(size_t)h->cidx[j * nx + i] * n + h->cidx[(j + dy) * nx + i + dx]] =
                        *Aent(c, i, j, dx, dy);
                }
    for (int k = 0; k < n; ++k) {
        double d = M[(size_t)k * n + k];
        for (int m = 0; m < k; ++m) d -= M[(size_t)k * n + m] * M[(size_t)k * n + m];
        if (!(d > 0.0)) { free(M); return -1; }
        d = sqrt(d);
        M[(size_t)k * n + k] = d;
        for (int r = k + 1; r < n; ++r) {
            double s = M[(size_t)r * n + k];
            for (int m = 0; m < k; ++m) s -= M[(size_t)r * n + m] * M[(size_t)k * n + m];
            M[(size_t)r * n + k] = s / d;
        }
    }
    h->chol = M;
    return 0;
}

void *oracle_setup(int nx, int ny, int npt, const double *planes, int coarsest_n,
                   int nu1, int nu2, int rescorr, int *status)
{
    *status = 0;
    if (nx < 3 || ny < 3 || nx % 2 == 0 || ny % 2 == 0 || (npt != 5 && npt != 9) ||
        coarsest_n < 3) {
        *status = 1;
        return NULL;
    }
    int sx[MAXLEV], sy[MAXLEV], L = 1;
    sx[0] = nx;
    sy[0] = ny;
    /* standard coarsening keeps the even-indexed vertices; a level with an even
     * number of vertices on a side has its last (boundary) vertex at an odd
     * index, so it cannot be coarsened again and becomes the coarsest level */
    while (sx[L - 1] > coarsest_n && sy[L - 1] > coarsest_n && (sx[L - 1] & 1) && (sy[L - 1] & 1) &&
           L < MAXLEV) {
        sx[L] = (sx[L - 1] + 1) / 2;
        sy[L] = (sy[L - 1] + 1) / 2;
        ++L;
    }
    ohier *h = calloc(1, sizeof(ohier));
    h->L = L;
    h->nu1 = nu1;
    h->nu2 = nu2;
    h->rescorr = rescorr;
    for (int l = 0; l < L; ++l) level_alloc(&h->lev[l], sx[L - 1 - l], sy[L - 1 - l]);
    import_stencil(&h->lev[L - 1], npt, planes);
    for (int l = L - 1; l >= 1; --l) {
        build_interp(&h->lev[l], &h->lev[l - 1]);
        build_galerkin(&h->lev[l], &h->lev[l - 1]);
    }
    if (factor_coarsest(h) != 0) *status = 4;
    return h;
}

void oracle_free(void *hv)
{
    ohier *h = hv;
    if (!h) return;
    for (int l = 0; l < h->L; ++l) {
        free(h->lev[l].A);
        free(h->lev[l].P);
        free(h->lev[l].x);
        free(h->lev[l].b);
        free(h->lev[l].r);
        free(h->lev[l].A32);
        free(h->lev[l].P32);
        free(h->lev[l].x32);
        free(h->lev[l].b32);
        free(h->lev[l].r32);
    }
    free(h->cidx);
    free(h->chol);
    free(h);
}

int oracle_num_levels(void *hv) { return ((ohier *)hv)->L; }

/* Threads of the parallel loops from now on (n >= 1); returns the previous
 * count.  Results do not depend on it. */
int oracle_set_threads(int n)
{
    int prev = omp_get_max_threads();
    if (n >= 1) omp_set_num_threads(n);
    return prev;
}

void oracle_level_size(void *hv, int l, int *nx, int *ny)
{
    ohier *h = hv;
    *nx = h->lev[l].nx;
    *ny = h->lev[l].ny;
}

void oracle_get_stencil(void *hv, int l, double *out)
{
    ohier *h = hv;
    memcpy(out, h->lev[l].A, (size_t)h->lev[l].nx * h->lev[l].ny * 9 * sizeof(double));
}

void oracle_get_interp(void *hv, int l, double *out)
{
    ohier *h = hv;
    memcpy(out, h->lev[l].P, (size_t)h->lev[l].nx * h->lev[l].ny * 4 * sizeof(double));
}

/* ---------------------------------------------------------------------------
 * Solve-phase operations on level l (Algorithm 1).
 * ------------------------------------------------------------------------- */
static double apply_row(const olevel *lv, const double *x, int i, int j)
{
    double s = 0.0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx)
            s += *Aent(lv, i, j, dx, dy) * x[(size_t)(j + dy) * lv->nx + (i + dx)];
    return s;
}

/* One relaxation: four-colour Gauss-Seidel, colour k = (i mod 2) + 2 (j mod 2),
 * colours 0,1,2,3 in turn; within a colour the points are independent. */
static void gs_sweep(const olevel *lv, double *x, const double *b)
{
    for (int colour = 0; colour < 4; ++colour)
#pragma omp parallel for schedule(static)
        for (int j = 1; j <= lv->ny - 2; ++j)
            for (int i = 1; i <= lv->nx - 2; ++i) {
                if ((i % 2) + 2 * (j % 2) != colour) continue;
                size_t p = (size_t)j * lv->nx + i;
                double r = b[p] - apply_row(lv, x, i, j);
                x[p] += r / *Aent(lv, i, j, 0, 0);
            }
}

static void residual(const olevel *lv, const double *x, const double *b, double *r)
{
    memset(r, 0, (size_t)lv->nx * lv->ny * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int j = 1; j <= lv->ny - 2; ++j)
        for (int i = 1; i <= lv->nx - 2; ++i) {
            size_t p = (size_t)j * lv->nx + i;
            r[p] = b[p] - apply_row(lv, x, i, j);
        }
}

/* b_c = P^T r: every fine vertex scatters its residual to its coarse corners */
static void restrict_pt(const olevel *f, const double *r, const olevel *c, double *bc)
{
    memset(bc, 0, (size_t)c->nx * c->ny * sizeof(double));
    for (int j = 1; j <= f->ny - 2; ++j)
        for (int i = 1; i <= f->nx - 2; ++i) {
            const double *pr = &f->P[((size_t)j * f->nx + i) * 4];
            for (int k = 0; k < 4; ++k)
                if (pr[k] != 0.0)
                    bc[(size_t)((j >> 1) + (k >> 1)) * c->nx + (i >> 1) + (k & 1)] +=
                        pr[k] * r[(size_t)j * f->nx + i];
        }
}

/* x += P x_c, plus r/C at vertices that are not coarse points */
static void interp_correct(const olevel *f, double *x, const double *r, const olevel *c,
                           const double *xc, int rescorr)
{
#pragma omp parallel for schedule(static)
    for (int j = 1; j <= f->ny - 2; ++j)
        for (int i = 1; i <= f->nx - 2; ++i) {
            const double *pr = &f->P[((size_t)j * f->nx + i) * 4];
            double s = 0.0;
            for (int k = 0; k < 4; ++k)
                s += pr[k] * xc[(size_t)((j >> 1) + (k >> 1)) * c->nx + (i >> 1) + (k & 1)];
            size_t p = (size_t)j * f->nx + i;
            x[p] += s;
            if (rescorr && !(i % 2 == 0 && j % 2 == 0)) x[p] += r[p] / *Aent(f, i, j, 0, 0);
        }
}

static void coarse_solve(const ohier *h, double *x, const double *b)
{
    const olevel *c = &h->lev[0];
    int n = h->nc;
    double *y = calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (int j = 0; j < c->ny; ++j)
        for (int i = 0; i < c->nx; ++i) {
            int k = h->cidx[j * c->nx + i];
            if (k >= 0) y[k] = b[(size_t)j * c->nx + i];
        }
    for (int k = 0; k < n; ++k) {        /* L y = b */
        double s = y[k];
        for (int m = 0; m < k; ++m) s -= h->chol[(size_t)k * n + m] * y[m];
        y[k] = s / h->chol[(size_t)k * n + k];
    }
    for (int k = n - 1; k >= 0; --k) {   /* L^T x = y */
        double s = y[k];
        for (int m = k + 1; m < n; ++m) s -= h->chol[(size_t)m * n + k] * y[m];
        y[k] = s / h->chol[(size_t)k * n + k];
    }
    memset(x, 0, (size_t)c->nx * c->ny * sizeof(double));
    for (int j = 0; j < c->ny; ++j)
        for (int i = 0; i < c->nx; ++i) {
            int k = h->cidx[j * c->nx + i];
            if (k >= 0) x[(size_t)j * c->nx + i] = y[k];
        }
    free(y);
}

/* Algorithm 1, recursive form; x and b of level l are the level's own buffers
 * except on the finest level. */
static void vcycle(ohier *h, int l, double *x, const double *b)
{
    olevel *f = &h->lev[l];
    if (l == 0) {
        coarse_solve(h, x, b);
        return;
    }
    olevel *c = &h->lev[l - 1];
    for (int k = 0; k < h->nu1; ++k) gs_sweep(f, x, b);
    residual(f, x, b, f->r);
    restrict_pt(f, f->r, c, c->b);
    memset(c->x, 0, (size_t)c->nx * c->ny * sizeof(double));
    vcycle(h, l - 1, c->x, c->b);
    interp_correct(f, x, f->r, c, c->x, h->rescorr);
    for (int k = 0; k < h->nu2; ++k) gs_sweep(f, x, b);
}

static double norm_interior(const olevel *lv, const double *v)
{
    double s = 0.0;
    for (int j = 1; j <= lv->ny - 2; ++j)
        for (int i = 1; i <= lv->nx - 2; ++i) {
            double a = v[(size_t)j * lv->nx + i];
            s += a * a;
        }
    return sqrt(s);
}

/* Outer iteration: V-cycles until ||b - A u|| / ||b|| <= tol.  Returns the
 * number of cycles run; hist[k] is the relative residual after cycle k+1.
 * u is the initial guess on entry (boundary entries are forced to zero). */
int oracle_solve(void *hv, const double *bin, double *u, double tol, int max_cycles,
                 double *hist)
{
    ohier *h = hv;
    olevel *f = &h->lev[h->L - 1];
    size_t n = (size_t)f->nx * f->ny;
    double *b = calloc(n, sizeof(double));
    for (int j = 1; j <= f->ny - 2; ++j)
        for (int i = 1; i <= f->nx - 2; ++i) b[(size_t)j * f->nx + i] = bin[(size_t)j * f->nx + i];
    for (int j = 0; j < f->ny; ++j)
        for (int i = 0; i < f->nx; ++i)
            if (!interior(f, i, j)) u[(size_t)j * f->nx + i] = 0.0;
    double bn = norm_interior(f, b);
    int cycles = 0;
    if (bn == 0.0) {
        memset(u, 0, n * sizeof(double));
        free(b);
        return 0;
    }
    double *r = calloc(n, sizeof(double));
    while (cycles < max_cycles) {
        vcycle(h, h->L - 1, u, b);
        residual(f, u, b, r);
        double rel = norm_interior(f, r) / bn;
        if (hist) hist[cycles] = rel;
        ++cycles;
        if (rel <= tol) break;
    }
    free(r);
    free(b);
    return cycles;
}

/* Single operations, exposed for kernel-by-kernel comparisons. */
void oracle_smooth(void *hv, int l, const double *b, double *x, int sweeps)
{
    ohier *h = hv;
    for (int k = 0; k < sweeps; ++k) gs_sweep(&h->lev[l], x, b);
}

void oracle_residual(void *hv, int l, const double *b, const double *x, double *r)
{
    ohier *h = hv;
    residual(&h->lev[l], x, b, r);
}

void oracle_restrict(void *hv, int l, const double *r, double *bc)
{
    ohier *h = hv;
    restrict_pt(&h->lev[l], r, &h->lev[l - 1], bc);
}

void oracle_interp_correct(void *hv, int l, double *x, const double *r, const double *xc,
                           int rescorr)
{
    ohier *h = hv;
    interp_correct(&h->lev[l], x, r, &h->lev[l - 1], xc, rescorr);
}

void oracle_coarse_solve(void *hv, const double *b, double *x)
{
    coarse_solve((ohier *)hv, x, b);
}

void oracle_vcycle(void *hv, const double *b, double *u)
{
    ohier *h = hv;
    vcycle(h, h->L - 1, u, b);
}

/* ---------------------------------------------------------------------------
 * Adjoint of the discrete solve with respect to theta = log D per cell.
 * With u^T A v = sum over edges e of a_e (u_p - u_q)(v_p - v_q) (boundary
 * values zero) and every edge coefficient taking D_c / 2 from each of the two
 * cells its dual face cuts, dL/dtheta_c = -lam^T (dA/dtheta_c) u
 *   = -(D_c / 2) sum over the four edges of cell c of (lam_p - lam_q)(u_p - u_q).
 * ------------------------------------------------------------------------- */
static double vat(const double *v, int nx, int ny, int i, int j)
{
    if (i <= 0 || j <= 0 || i >= nx - 1 || j >= ny - 1) return 0.0;
    return v[(size_t)j * nx + i];
}

void oracle_grad_logD(int nx, int ny, const double *cellD, const double *u, const double *lam,
                      double *g)
{
    for (int cj = 0; cj < ny - 1; ++cj)
        for (int ci = 0; ci < nx - 1; ++ci) {
            double s = 0.0;
            /* bottom and top edges (x direction) */
            for (int t = 0; t <= 1; ++t) {
                int j = cj + t;
                s += (vat(lam, nx, ny, ci, j) - vat(lam, nx, ny, ci + 1, j)) *
                     (vat(u, nx, ny, ci, j) - vat(u, nx, ny, ci + 1, j));
            }
            /* left and right edges (y direction) */
            for (int t = 0; t <= 1; ++t) {
                int i = ci + t;
                s += (vat(lam, nx, ny, i, cj) - vat(lam, nx, ny, i, cj + 1)) *
                     (vat(u, nx, ny, i, cj) - vat(u, nx, ny, i, cj + 1));
            }
            g[(size_t)cj * (nx - 1) + ci] = -0.5 * cellD[(size_t)cj * (nx - 1) + ci] * s;
        }
}

/* ---------------------------------------------------------------------------
 * FP32 edge form: the inner solver of mixed-precision iterative refinement.
 *
 * Setup stays FP64; every level is demoted once.  Rounding the matrix entries
 * of a pure-diffusion row to float would break its zero row sum by about one
 * float ulp of the diagonal, which makes the FP32 operator a much worse model
 * of the FP64 one as the grid grows.  The edge form keeps the connections
 * c_pq = -A(p,q) (rounded to float) and the excess E_p = A(p,p) - sum_q c_pq
 * (formed in double, then rounded), and applies the operator as
 *     (A x)_p = sum_q c_pq (x_p - x_q) + E_p x_p ,
 * whose diagonal is sum_q c_pq + E_p.  A row whose FP64 sum is zero keeps an
 * excess of FP64 rounding size, so constants stay in the near null space.
 * All arithmetic of the relaxation, residual, restriction and interpolation is
 * float; residual norms are accumulated in double; the coarsest level is
 * solved with the FP64 Cholesky factor (its right-hand side widened to double,
 * the solution rounded to float).
 * ------------------------------------------------------------------------- */
void oracle32_demote(void *hv)
{
    ohier *h = hv;
    for (int l = 0; l < h->L; ++l) {
        olevel *lv = &h->lev[l];
        size_t n = (size_t)lv->nx * lv->ny;
        if (!lv->A32) {
            lv->A32 = calloc(n * 9, sizeof(float));
            lv->P32 = calloc(n * 4, sizeof(float));
            lv->x32 = calloc(n, sizeof(float));
            lv->b32 = calloc(n, sizeof(float));
            lv->r32 = calloc(n, sizeof(float));
        }
        for (int j = 1; j <= lv->ny - 2; ++j)
            for (int i = 1; i <= lv->nx - 2; ++i) {
                float *e = &lv->A32[((size_t)j * lv->nx + i) * 9];
                double conn_sum = 0.0;
                for (int k = 0; k < 9; ++k) {
                    if (k == 4) continue;
                    double c = -lv->A[((size_t)j * lv->nx + i) * 9 + k];
                    e[k] = (float)c;
                    conn_sum += c;
                }
                e[4] = (float)(*Aent(lv, i, j, 0, 0) - conn_sum);
            }
        for (size_t k = 0; k < n * 4; ++k) lv->P32[k] = (float)lv->P[k];
    }
}

/* every FP32 entry point works on the demoted levels: built on first use */
static ohier *with32(void *hv)
{
    ohier *h = hv;
    if (!h->lev[0].A32) oracle32_demote(h);
    return h;
}

void oracle32_get_level(void *hv, int l, float *A32, float *P32)
{
    ohier *h = with32(hv);
    const olevel *lv = &h->lev[l];
    size_t n = (size_t)lv->nx * lv->ny;
    memcpy(A32, lv->A32, n * 9 * sizeof(float));
    if (P32) memcpy(P32, lv->P32, n * 4 * sizeof(float));
}

/* (A x)_p in edge form, and the diagonal sum_q c_pq + E_p */
static float apply_row32(const olevel *lv, const float *x, int i, int j, float *diag)
{
    const float *e = &lv->A32[((size_t)j * lv->nx + i) * 9];
    float xp = x[(size_t)j * lv->nx + i];
    float s = 0.0f, d = 0.0f;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            int k = (dy + 1) * 3 + (dx + 1);
            if (k == 4) continue;
            float xq = x[(size_t)(j + dy) * lv->nx + (i + dx)];
            s += e[k] * (xp - xq);
            d += e[k];
        }
    s += e[4] * xp;
    *diag = d + e[4];
    return s;
}

static float diag32(const olevel *lv, int i, int j)
{
    const float *e = &lv->A32[((size_t)j * lv->nx + i) * 9];
    float d = 0.0f;
    for (int k = 0; k < 9; ++k)
        if (k != 4) d += e[k];
    return d + e[4];
}

static void gs_sweep32(const olevel *lv, float *x, const float *b)
{
    for (int colour = 0; colour < 4; ++colour)
#pragma omp parallel for schedule(static)
        for (int j = 1; j <= lv->ny - 2; ++j)
            for (int i = 1; i <= lv->nx - 2; ++i) {
                if ((i % 2) + 2 * (j % 2) != colour) continue;
                size_t p = (size_t)j * lv->nx + i;
                float d;
                float r = b[p] - apply_row32(lv, x, i, j, &d);
                x[p] += r / d;
            }
}

static void residual32(const olevel *lv, const float *x, const float *b, float *r)
{
    memset(r, 0, (size_t)lv->nx * lv->ny * sizeof(float));
#pragma omp parallel for schedule(static)
    for (int j = 1; j <= lv->ny - 2; ++j)
        for (int i = 1; i <= lv->nx - 2; ++i) {
            size_t p = (size_t)j * lv->nx + i;
            float d;
            r[p] = b[p] - apply_row32(lv, x, i, j, &d);
        }
}

static void restrict32(const olevel *f, const float *r, const olevel *c, float *bc)
{
    memset(bc, 0, (size_t)c->nx * c->ny * sizeof(float));
    for (int j = 1; j <= f->ny - 2; ++j)
        for (int i = 1; i <= f->nx - 2; ++i) {
            const float *pr = &f->P32[((size_t)j * f->nx + i) * 4];
            for (int k = 0; k < 4; ++k)
                if (pr[k] != 0.0f)
                    bc[(size_t)((j >> 1) + (k >> 1)) * c->nx + (i >> 1) + (k & 1)] +=
                        pr[k] * r[(size_t)j * f->nx + i];
        }
}

/* x += P x_c, plus r / diag at vertices that are not coarse points */
static void interp_correct32(const olevel *f, float *x, const float *r, const olevel *c, const float *xc,
                             int rescorr)
{
#pragma omp parallel for schedule(static)
    for (int j = 1; j <= f->ny - 2; ++j)
        for (int i = 1; i <= f->nx - 2; ++i) {
            const float *pr = &f->P32[((size_t)j * f->nx + i) * 4];
            float s = 0.0f;
            for (int k = 0; k < 4; ++k)
                s += pr[k] * xc[(size_t)((j >> 1) + (k >> 1)) * c->nx + (i >> 1) + (k & 1)];
            size_t p = (size_t)j * f->nx + i;
            x[p] += s;
            if (rescorr && !(i % 2 == 0 && j % 2 == 0)) x[p] += r[p] / diag32(f, i, j);
        }
}

static void coarse_solve32(const ohier *h, float *x, const float *b)
{
    const olevel *c = &h->lev[0];
    size_t n = (size_t)c->nx * c->ny;
    double *bd = calloc(n, sizeof(double)), *xd = calloc(n, sizeof(double));
    for (size_t k = 0; k < n; ++k) bd[k] = (double)b[k];
    coarse_solve(h, xd, bd);
    for (size_t k = 0; k < n; ++k) x[k] = (float)xd[k];
    free(bd);
    free(xd);
}

static void vcycle32(ohier *h, int l, float *x, const float *b)
{
    olevel *f = &h->lev[l];
    if (l == 0) {
        coarse_solve32(h, x, b);
        return;
    }
    olevel *c = &h->lev[l - 1];
    for (int k = 0; k < h->nu1; ++k) gs_sweep32(f, x, b);
    residual32(f, x, b, f->r32);
    restrict32(f, f->r32, c, c->b32);
    memset(c->x32, 0, (size_t)c->nx * c->ny * sizeof(float));
    vcycle32(h, l - 1, c->x32, c->b32);
    interp_correct32(f, x, f->r32, c, c->x32, h->rescorr);
    for (int k = 0; k < h->nu2; ++k) gs_sweep32(f, x, b);
}

static double norm32_interior(const olevel *lv, const float *v)
{
    double s = 0.0;
    for (int j = 1; j <= lv->ny - 2; ++j)
        for (int i = 1; i <= lv->nx - 2; ++i) {
            double a = (double)v[(size_t)j * lv->nx + i];
            s += a * a;
        }
    return sqrt(s);
}

void oracle32_smooth(void *hv, int l, const float *b, float *x, int sweeps)
{
    ohier *h = with32(hv);
    for (int k = 0; k < sweeps; ++k) gs_sweep32(&h->lev[l], x, b);
}

void oracle32_residual(void *hv, int l, const float *b, const float *x, float *r)
{
    ohier *h = with32(hv);
    residual32(&h->lev[l], x, b, r);
}

void oracle32_restrict(void *hv, int l, const float *r, float *bc)
{
    ohier *h = with32(hv);
    restrict32(&h->lev[l], r, &h->lev[l - 1], bc);
}

void oracle32_interp_correct(void *hv, int l, float *x, const float *r, const float *xc, int rescorr)
{
    ohier *h = with32(hv);
    interp_correct32(&h->lev[l], x, r, &h->lev[l - 1], xc, rescorr);
}

void oracle32_vcycle(void *hv, const float *b, float *x)
{
    ohier *h = with32(hv);
    vcycle32(h, h->L - 1, x, b);
}

/* The inner solve of one refinement step: V-cycles on A e = r from e = 0,
 * each followed by the inner relative residual ||r - A e|| / rnorm (rnorm the
 * FP64 norm of the outer residual), until it is <= inner_tol or `cycles`
 * cycles have run.  Returns the number of cycles; hist[k] is the inner
 * relative residual after cycle k+1. */
int oracle32_inner(void *hv, const float *r, float *e, int cycles, double rnorm, double inner_tol, double *hist)
{
    ohier *h = with32(hv);
    olevel *f = &h->lev[h->L - 1];
    size_t n = (size_t)f->nx * f->ny;
    float *rr = calloc(n, sizeof(float));
    memset(e, 0, n * sizeof(float));
    int k = 0;
    while (k < cycles) {
        vcycle32(h, h->L - 1, e, r);
        residual32(f, e, r, rr);
        double rel = norm32_interior(f, rr) / rnorm;
        if (hist) hist[k] = rel;
        ++k;
        if (rel <= inner_tol) break;
    }
    free(rr);
    return k;
}

/* Mixed precision: FP64 iterative refinement around FP32 inner solves.  Each
 * step forms the outer residual r = b - A u in FP64 and its relative norm
 * rel (hist[step]); it stops when that is <= tol or when the cycle budget is
 * spent, else demotes r to float, runs an inner solve of at most
 * min(inner_max, max_cycles - cycles done) cycles to an inner relative
 * residual of max(inner_tol, tol / (2 rel)) (inner_tol alone if !adapt) and
 * adds the widened correction to u.  Returns the FP32 cycles run; *steps is the number
 * of inner solves. */
int oracle_solve_mixed(void *hv, const double *bin, double *u, double tol, int max_cycles, int inner_max,
                       double inner_tol, int adapt, double *hist, int *steps)
{
    ohier *h = with32(hv);
    olevel *f = &h->lev[h->L - 1];
    size_t n = (size_t)f->nx * f->ny;
    double *b = calloc(n, sizeof(double)), *r = calloc(n, sizeof(double));
    float *r32 = calloc(n, sizeof(float)), *e32 = calloc(n, sizeof(float));
    for (int j = 1; j <= f->ny - 2; ++j)
        for (int i = 1; i <= f->nx - 2; ++i) b[(size_t)j * f->nx + i] = bin[(size_t)j * f->nx + i];
    for (int j = 0; j < f->ny; ++j)
        for (int i = 0; i < f->nx; ++i)
            if (!interior(f, i, j)) u[(size_t)j * f->nx + i] = 0.0;
    double bn = norm_interior(f, b);
    int cycles = 0, st = 0;
    if (bn == 0.0) {
        memset(u, 0, n * sizeof(double));
    } else {
        for (;;) {
            residual(f, u, b, r);
            double rn = norm_interior(f, r);
            double rel = rn / bn;
            if (hist) hist[st] = rel;
            if (rel <= tol || cycles >= max_cycles) break;
            for (size_t k = 0; k < n; ++k) r32[k] = (float)r[k];
            int cap = inner_max < max_cycles - cycles ? inner_max : max_cycles - cycles;
            /* the inner solve stops at inner_tol, or (adapt) as soon as its
             * residual is below half of what the outer tolerance still asks
             * for (tol / rel), whichever comes first */
            double itol = 0.5 * tol / rel;
            if (!adapt || itol < inner_tol) itol = inner_tol;
            cycles += oracle32_inner(h, r32, e32, cap, rn, itol, NULL);
            for (int j = 1; j <= f->ny - 2; ++j)
                for (int i = 1; i <= f->nx - 2; ++i) u[(size_t)j * f->nx + i] += (double)e32[(size_t)j * f->nx + i];
            ++st;
        }
    }
    if (steps) *steps = st;
    free(b);
    free(r);
    free(r32);
    free(e32);
    return cycles;
}
