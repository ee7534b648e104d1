/*
 * bmg_oracle3d.c -- plain, slow, FP64 reference implementation of the
 * structured variational multigrid V-cycle for 3D diffusion: the
 * three-dimensional form of the method of Reisner, Olson, Moulton, "Scaling
 * Structured Multigrid to 500K+ Cores through Coarse-Grid Redistribution"
 * (arXiv 1803.02481), whose section 3 gives the 3D interpolation cost and
 * whose section 2 defines the method by its operator-induced interpolation
 * and Galerkin coarse operators.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library's
 * 3D path is checked against.  Only the test-suite and the benchmark's
 * CPU-baseline leg load it.  It shares no code, header, table or helper with
 * the GPU path (nor with the 2D oracle), and the GPU path never calls it.
 *
 * Everything is written out from the definitions, with no blocking, fusion or
 * reordering:
 *   - the operator is held as an explicit 3x3x3 matrix-entry stencil per
 *     vertex, A(p, p+d), with entries towards boundary vertices set to zero;
 *   - interpolation P is held as explicit rows: each fine vertex carries eight
 *     weights on the corners of the coarse cell that contains it;
 *   - interpolation is operator-induced (section 2): vertices on a coarse line
 *     collapse the stencil onto the line, vertices on a coarse face collapse it
 *     onto the face and eliminate their in-face neighbours, and cell centres
 *     eliminate all 26 neighbours;
 *   - the Galerkin product is the triple sum A_c(I,J) = sum_p sum_q
 *     P(p,I) A(p,q) P(q,J) over all fine couplings (section 2);
 *   - the smoother is eight-colour Gauss-Seidel, one colour at a time;
 *   - the V-cycle follows Algorithm 1 (section 2) with the residual term r/C
 *     added at vertices that are not coarse points after interpolation
 *     (section 3, interpolation cost paragraph);
 *   - the coarsest problem is solved by a dense Cholesky factorisation
 *     computed once at setup (section 3, coarse-solve cost equation).
 *
 * Parity unpinned against BoxMG itself: the paper prints neither the 2D nor
 * the 3D interpolation formulas.  The collapses below extend the 2D reading
 * one dimension up; the tests pin them by closed forms (trilinear weights and
 * a Kronecker-product coarse operator for D=1, products of one-dimensional
 * flux weights for coefficients that vary along x only).
 *
 * Threads: the loops over planes of one colour, of the residual and of the
 * interpolation run in parallel (OpenMP); their points are independent, so
 * the results are bitwise those of one thread.  Restriction (a scatter),
 * norms and setup stay sequential.
 *
 * Floating point: double throughout, built with -ffp-contract=off.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXLEV3 24

typedef struct {
    int nx, ny, nz;
    double *A;  /* [nz][ny][nx][27]: A(p, p+(dx,dy,dz)) at (dz+1)*9+(dy+1)*3+(dx+1) */
    double *P;  /* [nz][ny][nx][8]: interpolation row of fine vertex (i,j,k) onto
                   the corners ((i>>1)+a, (j>>1)+b, (k>>1)+c) of the next
                   coarser level, index 4c+2b+a.  Unused on the coarsest.      */
    double *x, *b, *r;
} olev3;

typedef struct {
    int L;
    olev3 lev[MAXLEV3];   /* lev[0] coarsest ... lev[L-1] finest */
    int nc;
    int *cidx;
    double *chol;
    int nu1, nu2, rescorr;
} ohier3;

static size_t vid(const olev3 *lv, int i, int j, int k)
{
    return ((size_t)k * lv->ny + j) * lv->nx + i;
}

static int inside(const olev3 *lv, int i, int j, int k)
{
    return i >= 1 && i <= lv->nx - 2 && j >= 1 && j <= lv->ny - 2 && k >= 1 && k <= lv->nz - 2;
}

static double *A3(const olev3 *lv, int i, int j, int k, int dx, int dy, int dz)
{
    return &lv->A[vid(lv, i, j, k) * 27 + (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)];
}

/* ---------------------------------------------------------------------------
 * Vertex-centred 7-point finite volume discretisation of -div(D grad u) with
 * homogeneous Dirichlet data (section 5's diffusion problem, in 3D).
 * cellD[(nz-1)][(ny-1)][(nx-1)] holds a constant diffusivity per cell
 * [x_i,x_i+1] x [y_j,y_j+1] x [z_k,z_k+1].  The dual face crossing an edge
 * cuts the four cells around the edge, a quarter of its area in each, so the
 * connection of the edge is the mean of those four diffusivities (the common
 * factor h of a uniform grid is left out: it scales A and b alike).
 * Output: C, W, S, B as [nz][ny][nx]; W, S and B are positive connection
 * values towards the west, south and lower neighbour (matrix entry = -W).
 * ------------------------------------------------------------------------- */
static double cell3(const double *D, int nx, int ny, int nz, int ci, int cj, int ck)
{
    if (ci < 0 || cj < 0 || ck < 0 || ci >= nx - 1 || cj >= ny - 1 || ck >= nz - 1) return 0.0;
    return D[((size_t)ck * (ny - 1) + cj) * (nx - 1) + ci];
}

void oracle3_fv7(int nx, int ny, int nz, const double *cellD, double *C, double *W, double *S, double *B)
{
    size_t n = (size_t)nx * ny * nz;
    memset(C, 0, n * sizeof(double));
    memset(W, 0, n * sizeof(double));
    memset(S, 0, n * sizeof(double));
    memset(B, 0, n * sizeof(double));
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t p = ((size_t)k * ny + j) * nx + i;
                /* x-edge (i-1,j,k)-(i,j,k): cells (i-1, j-1..j, k-1..k) */
                if (i >= 1 && j >= 1 && j <= ny - 2 && k >= 1 && k <= nz - 2)
                    W[p] = 0.25 * (cell3(cellD, nx, ny, nz, i - 1, j - 1, k - 1) +
                                   cell3(cellD, nx, ny, nz, i - 1, j, k - 1) +
                                   cell3(cellD, nx, ny, nz, i - 1, j - 1, k) +
                                   cell3(cellD, nx, ny, nz, i - 1, j, k));
                /* y-edge (i,j-1,k)-(i,j,k): cells (i-1..i, j-1, k-1..k) */
                if (j >= 1 && i >= 1 && i <= nx - 2 && k >= 1 && k <= nz - 2)
                    S[p] = 0.25 * (cell3(cellD, nx, ny, nz, i - 1, j - 1, k - 1) +
                                   cell3(cellD, nx, ny, nz, i, j - 1, k - 1) +
                                   cell3(cellD, nx, ny, nz, i - 1, j - 1, k) +
                                   cell3(cellD, nx, ny, nz, i, j - 1, k));
                /* z-edge (i,j,k-1)-(i,j,k): cells (i-1..i, j-1..j, k-1) */
                if (k >= 1 && i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2)
                    B[p] = 0.25 * (cell3(cellD, nx, ny, nz, i - 1, j - 1, k - 1) +
                                   cell3(cellD, nx, ny, nz, i, j - 1, k - 1) +
                                   cell3(cellD, nx, ny, nz, i - 1, j, k - 1) +
                                   cell3(cellD, nx, ny, nz, i, j, k - 1));
            }
    for (int k = 1; k <= nz - 2; ++k)
        for (int j = 1; j <= ny - 2; ++j)
            for (int i = 1; i <= nx - 2; ++i) {
                size_t p = ((size_t)k * ny + j) * nx + i;
                C[p] = W[p] + W[p + 1] + S[p] + S[p + nx] + B[p] + B[p + (size_t)nx * ny];
            }
}

/* ---------------------------------------------------------------------------
 * Hierarchy construction.
 * ------------------------------------------------------------------------- */
static void lev3_alloc(olev3 *lv, int nx, int ny, int nz)
{
    size_t n = (size_t)nx * ny * nz;
    lv->nx = nx;
    lv->ny = ny;
    lv->nz = nz;
    lv->A = calloc(n * 27, sizeof(double));
    lv->P = calloc(n * 8, sizeof(double));
    lv->x = calloc(n, sizeof(double));
    lv->b = calloc(n, sizeof(double));
    lv->r = calloc(n, sizeof(double));
}

/* Import the finest operator.  npt = 7: planes {C, W, S, B}.  npt = 27: 14
 * planes, the diagonal C then the positive connection values -A(p, p+d) for
 * the 13 offsets d whose linear index (dz+1)*9+(dy+1)*3+(dx+1) is 0..12 (the
 * lower half); the upper half follows from symmetry, A(p, p+d) = A(p+d, p). */
static void import3(olev3 *lv, int npt, const double *planes)
{
    int nx = lv->nx, ny = lv->ny, nz = lv->nz;
    size_t n = (size_t)nx * ny * nz;
    for (int k = 1; k <= nz - 2; ++k)
        for (int j = 1; j <= ny - 2; ++j)
            for (int i = 1; i <= nx - 2; ++i) {
                size_t p = vid(lv, i, j, k);
                double e[27] = {0};
                if (npt == 7) {
                    const double *C = planes, *W = planes + n, *S = planes + 2 * n, *B = planes + 3 * n;
                    e[13] = C[p];
                    e[12] = -W[p];
                    e[14] = -W[p + 1];
                    e[10] = -S[p];
                    e[16] = -S[p + nx];
                    e[4] = -B[p];
                    e[22] = -B[p + (size_t)nx * ny];
                } else {
                    e[13] = planes[p];
                    for (int o = 0; o < 13; ++o) {
                        int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
                        e[o] = -planes[(size_t)(1 + o) * n + p];
                        /* the mirror entry: stored at the neighbour p - d */
                        int qi = i - dx, qj = j - dy, qk = k - dz;
                        if (qi >= 0 && qi < nx && qj >= 0 && qj < ny && qk >= 0 && qk < nz)
                            e[26 - o] = -planes[(size_t)(1 + o) * n + vid(lv, qi, qj, qk)];
                    }
                }
                for (int o = 0; o < 27; ++o) {
                    int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
                    if (o != 13 && !inside(lv, i + dx, j + dy, k + dz)) e[o] = 0.0;
                    lv->A[p * 27 + o] = e[o];
                }
            }
}

/* add s * (interpolation row of q) to the row dst of p; both rows refer to
 * corners of their own coarse cells, which overlap because q is a neighbour
 * of p */
static void prow3_add(const olev3 *f, int pi, int pj, int pk, double *dst, int qi, int qj, int qk, double s)
{
    const double *q = &f->P[vid(f, qi, qj, qk) * 8];
    for (int c = 0; c <= 1; ++c)
        for (int b = 0; b <= 1; ++b)
            for (int a = 0; a <= 1; ++a) {
                double w = q[4 * c + 2 * b + a];
                if (w == 0.0) continue;
                int ci = (qi >> 1) + a - (pi >> 1);
                int cj = (qj >> 1) + b - (pj >> 1);
                int ck = (qk >> 1) + c - (pk >> 1);
                if (ci < 0 || ci > 1 || cj < 0 || cj > 1 || ck < 0 || ck > 1) abort();
                dst[4 * ck + 2 * cj + ci] += s * w;
            }
}

/* Operator-induced interpolation from level l-1 (coarse) to level l (fine).
 * A fine vertex is classified by how many of its indices are odd:
 *   0: a coarse point, injected;
 *   1: on a coarse line along the odd direction: the stencil is summed over
 *      the plane normal to the line (the other two directions), leaving a
 *      three-point relation along the line whose end points are coarse;
 *   2: on a coarse face spanned by the two odd directions: the stencil is
 *      summed along the face normal, leaving a nine-point relation in the
 *      face; the point is eliminated against its eight in-face neighbours,
 *      which are line points (rows of the first pass) and coarse points;
 *   3: a coarse cell centre: eliminated against its 26 neighbours, whose
 *      rows come from the first two passes.
 * Passes run in that order. */
static void build_interp3(olev3 *f, const olev3 *c)
{
    int nx = f->nx, ny = f->ny, nz = f->nz;
    memset(f->P, 0, (size_t)nx * ny * nz * 8 * sizeof(double));
    for (int pass = 0; pass <= 3; ++pass)
        for (int k = 1; k <= nz - 2; ++k)
            for (int j = 1; j <= ny - 2; ++j)
                for (int i = 1; i <= nx - 2; ++i) {
                    int oi = i & 1, oj = j & 1, ok = k & 1;
                    if (oi + oj + ok != pass) continue;
                    double *pr = &f->P[vid(f, i, j, k) * 8];
                    if (pass == 0) {
                        pr[0] = 1.0;
                    } else if (pass == 1) {
                        /* the odd direction t; sum over the other two */
                        double den = 0.0, am = 0.0, ap = 0.0;
                        for (int u = -1; u <= 1; ++u)
                            for (int v = -1; v <= 1; ++v) {
                                int d0[3], dm[3], dp[3];
                                /* offsets with component t = 0, -1, +1 and (u, v) in the others */
                                int t = oi ? 0 : (oj ? 1 : 2);
                                int o1 = t == 0 ? 1 : 0, o2 = t == 2 ? 1 : 2;
                                d0[t] = 0;  dm[t] = -1;  dp[t] = 1;
                                d0[o1] = dm[o1] = dp[o1] = u;
                                d0[o2] = dm[o2] = dp[o2] = v;
                                den += *A3(f, i, j, k, d0[0], d0[1], d0[2]);
                                am += *A3(f, i, j, k, dm[0], dm[1], dm[2]);
                                ap += *A3(f, i, j, k, dp[0], dp[1], dp[2]);
                            }
                        int im = oi ? 1 : 0, jm = oj ? 2 : 0, km = ok ? 4 : 0;
                        pr[0] = -am / den;                 /* corner at the lower end */
                        pr[im + jm + km] = -ap / den;      /* corner at the upper end */
                    } else if (pass == 2) {
                        /* the even direction n is the face normal: sum along it */
                        int n = !oi ? 0 : (!oj ? 1 : 2);
                        double at[3][3] = {{0}};   /* collapsed in-face stencil, [s][r] */
                        int o1 = n == 0 ? 1 : 0, o2 = n == 2 ? 1 : 2;
                        for (int s = -1; s <= 1; ++s)
                            for (int r = -1; r <= 1; ++r)
                                for (int m = -1; m <= 1; ++m) {
                                    int d[3];
                                    d[o1] = r;
                                    d[o2] = s;
                                    d[n] = m;
                                    at[s + 1][r + 1] += *A3(f, i, j, k, d[0], d[1], d[2]);
                                }
                        double diag = at[1][1];
                        for (int s = -1; s <= 1; ++s)
                            for (int r = -1; r <= 1; ++r) {
                                if (r == 0 && s == 0) continue;
                                double a = at[s + 1][r + 1];
                                if (a == 0.0) continue;
                                int d[3];
                                d[o1] = r;
                                d[o2] = s;
                                d[n] = 0;
                                prow3_add(f, i, j, k, pr, i + d[0], j + d[1], k + d[2], -a / diag);
                            }
                    } else {
                        double diag = *A3(f, i, j, k, 0, 0, 0);
                        for (int dz = -1; dz <= 1; ++dz)
                            for (int dy = -1; dy <= 1; ++dy)
                                for (int dx = -1; dx <= 1; ++dx) {
                                    if (dx == 0 && dy == 0 && dz == 0) continue;
                                    double a = *A3(f, i, j, k, dx, dy, dz);
                                    if (a == 0.0) continue;
                                    prow3_add(f, i, j, k, pr, i + dx, j + dy, k + dz, -a / diag);
                                }
                    }
                }
    /* coarse boundary vertices are not unknowns: no weight on them */
    for (int k = 1; k <= nz - 2; ++k)
        for (int j = 1; j <= ny - 2; ++j)
            for (int i = 1; i <= nx - 2; ++i)
                for (int m = 0; m < 8; ++m)
                    if (!inside(c, (i >> 1) + (m & 1), (j >> 1) + ((m >> 1) & 1), (k >> 1) + (m >> 2)))
                        f->P[vid(f, i, j, k) * 8 + m] = 0.0;
}

/* Galerkin coarse operator A_c = P^T A P (section 2) as the triple sum over
 * every fine coupling (p,q) and every pair of coarse columns. */
static void build_galerkin3(const olev3 *f, olev3 *c)
{
    memset(c->A, 0, (size_t)c->nx * c->ny * c->nz * 27 * sizeof(double));
    for (int pk = 1; pk <= f->nz - 2; ++pk)
        for (int pj = 1; pj <= f->ny - 2; ++pj)
            for (int pi = 1; pi <= f->nx - 2; ++pi) {
                const double *Pp = &f->P[vid(f, pi, pj, pk) * 8];
                for (int o = 0; o < 27; ++o) {
                    int qi = pi + o % 3 - 1, qj = pj + (o / 3) % 3 - 1, qk = pk + o / 9 - 1;
                    double a = f->A[vid(f, pi, pj, pk) * 27 + o];
                    if (a == 0.0 || !inside(f, qi, qj, qk)) continue;
                    const double *Pq = &f->P[vid(f, qi, qj, qk) * 8];
                    for (int s = 0; s < 8; ++s) {
                        if (Pp[s] == 0.0) continue;
                        int Ii = (pi >> 1) + (s & 1), Ij = (pj >> 1) + ((s >> 1) & 1), Ik = (pk >> 1) + (s >> 2);
                        for (int m = 0; m < 8; ++m) {
                            if (Pq[m] == 0.0) continue;
                            int Ji = (qi >> 1) + (m & 1), Jj = (qj >> 1) + ((m >> 1) & 1), Jk = (qk >> 1) + (m >> 2);
                            int ex = Ji - Ii, ey = Jj - Ij, ez = Jk - Ik;
                            if (ex < -1 || ex > 1 || ey < -1 || ey > 1 || ez < -1 || ez > 1) abort();
                            *A3(c, Ii, Ij, Ik, ex, ey, ez) += Pp[s] * a * Pq[m];
                        }
                    }
                }
            }
}

static int factor3(ohier3 *h)
{
    olev3 *c = &h->lev[0];
    size_t nv = (size_t)c->nx * c->ny * c->nz;
    h->cidx = malloc(nv * sizeof(int));
    int n = 0;
    for (int k = 0; k < c->nz; ++k)
        for (int j = 0; j < c->ny; ++j)
            for (int i = 0; i < c->nx; ++i) h->cidx[vid(c, i, j, k)] = inside(c, i, j, k) ? n++ : -1;
    h->nc = n;
    double *M = calloc((size_t)(n > 0 ? n : 1) * (n > 0 ? n : 1), sizeof(double));
    for (int k = 1; k <= c->nz - 2; ++k)
        for (int j = 1; j <= c->ny - 2; ++j)
            for (int i = 1; i <= c->nx - 2; ++i)
                for (int o = 0; o < 27; ++o) {
                    int qi = i + o % 3 - 1, qj = j + (o / 3) % 3 - 1, qk = k + o / 9 - 1;
                    if (!inside(c, qi, qj, qk)) continue;
                    M[(size_t)h->cidx[vid(c, i, j, k)] * n + h->cidx[vid(c, qi, qj, qk)]] =
                        c->A[vid(c, i, j, k) * 27 + o];
                }
    for (int k = 0; k < n; ++k) {
        double d = M[(size_t)k * n + k];
        for (int m = 0; m < k; ++m) d -= M[(size_t)k * n + m] * M[(size_t)k * n + m];
        if (!(d > 0.0)) {
            free(M);
            return -1;
        }
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

void *oracle3_setup(int nx, int ny, int nz, int npt, const double *planes, int coarsest_n, int nu1, int nu2,
                    int rescorr, int *status)
{
    *status = 0;
    if (nx < 3 || ny < 3 || nz < 3 || !(nx & 1) || !(ny & 1) || !(nz & 1) || (npt != 7 && npt != 27) ||
        coarsest_n < 3) {
        *status = 1;
        return NULL;
    }
    int sx[MAXLEV3], sy[MAXLEV3], sz[MAXLEV3], L = 1;
    sx[0] = nx;
    sy[0] = ny;
    sz[0] = nz;
    /* standard coarsening keeps the even-indexed vertices; a level with an even
     * number of vertices on a side cannot be coarsened again */
    while (sx[L - 1] > coarsest_n && sy[L - 1] > coarsest_n && sz[L - 1] > coarsest_n && (sx[L - 1] & 1) &&
           (sy[L - 1] & 1) && (sz[L - 1] & 1) && L < MAXLEV3) {
        sx[L] = (sx[L - 1] + 1) / 2;
        sy[L] = (sy[L - 1] + 1) / 2;
        sz[L] = (sz[L - 1] + 1) / 2;
        ++L;
    }
    ohier3 *h = calloc(1, sizeof(ohier3));
    h->L = L;
    h->nu1 = nu1;
    h->nu2 = nu2;
    h->rescorr = rescorr;
    for (int l = 0; l < L; ++l) lev3_alloc(&h->lev[l], sx[L - 1 - l], sy[L - 1 - l], sz[L - 1 - l]);
    import3(&h->lev[L - 1], npt, planes);
    for (int l = L - 1; l >= 1; --l) {
        build_interp3(&h->lev[l], &h->lev[l - 1]);
        build_galerkin3(&h->lev[l], &h->lev[l - 1]);
    }
    if (factor3(h) != 0) *status = 4;
    return h;
}

void oracle3_free(void *hv)
{
    ohier3 *h = hv;
    if (!h) return;
    for (int l = 0; l < h->L; ++l) {
        free(h->lev[l].A);
        free(h->lev[l].P);
        free(h->lev[l].x);
        free(h->lev[l].b);
        free(h->lev[l].r);
    }
    free(h->cidx);
    free(h->chol);
    free(h);
}

int oracle3_num_levels(void *hv) { return ((ohier3 *)hv)->L; }

void oracle3_level_size(void *hv, int l, int *nx, int *ny, int *nz)
{
    ohier3 *h = hv;
    *nx = h->lev[l].nx;
    *ny = h->lev[l].ny;
    *nz = h->lev[l].nz;
}

void oracle3_get_stencil(void *hv, int l, double *out)
{
    ohier3 *h = hv;
    const olev3 *lv = &h->lev[l];
    memcpy(out, lv->A, (size_t)lv->nx * lv->ny * lv->nz * 27 * sizeof(double));
}

void oracle3_get_interp(void *hv, int l, double *out)
{
    ohier3 *h = hv;
    const olev3 *lv = &h->lev[l];
    memcpy(out, lv->P, (size_t)lv->nx * lv->ny * lv->nz * 8 * sizeof(double));
}

/* ---------------------------------------------------------------------------
 * Solve-phase operations on one level (Algorithm 1).
 * ------------------------------------------------------------------------- */
static double apply3(const olev3 *lv, const double *x, int i, int j, int k)
{
    double s = 0.0;
    for (int o = 0; o < 27; ++o)
        s += lv->A[vid(lv, i, j, k) * 27 + o] * x[vid(lv, i + o % 3 - 1, j + (o / 3) % 3 - 1, k + o / 9 - 1)];
    return s;
}

/* One relaxation: eight-colour Gauss-Seidel, colour (i mod 2) + 2 (j mod 2)
 * + 4 (k mod 2), colours 0..7 in turn.  Points of one colour differ by even
 * amounts in every index, so no two of them couple in a 27-point stencil and
 * the order within a colour does not matter. */
static void gs3(const olev3 *lv, double *x, const double *b)
{
    for (int colour = 0; colour < 8; ++colour)
#pragma omp parallel for schedule(static)
        for (int k = 1; k <= lv->nz - 2; ++k)
            for (int j = 1; j <= lv->ny - 2; ++j)
                for (int i = 1; i <= lv->nx - 2; ++i) {
                    if ((i & 1) + 2 * (j & 1) + 4 * (k & 1) != colour) continue;
                    size_t p = vid(lv, i, j, k);
                    double r = b[p] - apply3(lv, x, i, j, k);
                    x[p] += r / lv->A[p * 27 + 13];
                }
}

static void residual3(const olev3 *lv, const double *x, const double *b, double *r)
{
    memset(r, 0, (size_t)lv->nx * lv->ny * lv->nz * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int k = 1; k <= lv->nz - 2; ++k)
        for (int j = 1; j <= lv->ny - 2; ++j)
            for (int i = 1; i <= lv->nx - 2; ++i) {
                size_t p = vid(lv, i, j, k);
                r[p] = b[p] - apply3(lv, x, i, j, k);
            }
}

/* b_c = P^T r: every fine vertex scatters its residual to its coarse corners */
static void restrict3(const olev3 *f, const double *r, const olev3 *c, double *bc)
{
    memset(bc, 0, (size_t)c->nx * c->ny * c->nz * sizeof(double));
    for (int k = 1; k <= f->nz - 2; ++k)
        for (int j = 1; j <= f->ny - 2; ++j)
            for (int i = 1; i <= f->nx - 2; ++i) {
                const double *pr = &f->P[vid(f, i, j, k) * 8];
                for (int m = 0; m < 8; ++m)
                    if (pr[m] != 0.0)
                        bc[vid(c, (i >> 1) + (m & 1), (j >> 1) + ((m >> 1) & 1), (k >> 1) + (m >> 2))] +=
                            pr[m] * r[vid(f, i, j, k)];
            }
}

/* x += P x_c, plus r/C at vertices that are not coarse points */
static void interp3(const olev3 *f, double *x, const double *r, const olev3 *c, const double *xc, int rescorr)
{
#pragma omp parallel for schedule(static)
    for (int k = 1; k <= f->nz - 2; ++k)
        for (int j = 1; j <= f->ny - 2; ++j)
            for (int i = 1; i <= f->nx - 2; ++i) {
                const double *pr = &f->P[vid(f, i, j, k) * 8];
                double s = 0.0;
                for (int m = 0; m < 8; ++m)
                    s += pr[m] * xc[vid(c, (i >> 1) + (m & 1), (j >> 1) + ((m >> 1) & 1), (k >> 1) + (m >> 2))];
                size_t p = vid(f, i, j, k);
                x[p] += s;
                if (rescorr && ((i & 1) || (j & 1) || (k & 1))) x[p] += r[p] / f->A[p * 27 + 13];
            }
}

static void coarse3(const ohier3 *h, double *x, const double *b)
{
    const olev3 *c = &h->lev[0];
    int n = h->nc;
    size_t nv = (size_t)c->nx * c->ny * c->nz;
    double *y = calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (size_t v = 0; v < nv; ++v)
        if (h->cidx[v] >= 0) y[h->cidx[v]] = b[v];
    for (int k = 0; k < n; ++k) {
        double s = y[k];
        for (int m = 0; m < k; ++m) s -= h->chol[(size_t)k * n + m] * y[m];
        y[k] = s / h->chol[(size_t)k * n + k];
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = y[k];
        for (int m = k + 1; m < n; ++m) s -= h->chol[(size_t)m * n + k] * y[m];
        y[k] = s / h->chol[(size_t)k * n + k];
    }
    memset(x, 0, nv * sizeof(double));
    for (size_t v = 0; v < nv; ++v)
        if (h->cidx[v] >= 0) x[v] = y[h->cidx[v]];
    free(y);
}

static void vcycle3(ohier3 *h, int l, double *x, const double *b)
{
    olev3 *f = &h->lev[l];
    if (l == 0) {
        coarse3(h, x, b);
        return;
    }
    olev3 *c = &h->lev[l - 1];
    for (int s = 0; s < h->nu1; ++s) gs3(f, x, b);
    residual3(f, x, b, f->r);
    restrict3(f, f->r, c, c->b);
    memset(c->x, 0, (size_t)c->nx * c->ny * c->nz * sizeof(double));
    vcycle3(h, l - 1, c->x, c->b);
    interp3(f, x, f->r, c, c->x, h->rescorr);
    for (int s = 0; s < h->nu2; ++s) gs3(f, x, b);
}

static double norm3(const olev3 *lv, const double *v)
{
    double s = 0.0;
    for (int k = 1; k <= lv->nz - 2; ++k)
        for (int j = 1; j <= lv->ny - 2; ++j)
            for (int i = 1; i <= lv->nx - 2; ++i) {
                double a = v[vid(lv, i, j, k)];
                s += a * a;
            }
    return sqrt(s);
}

/* V-cycles until ||b - A u|| / ||b|| <= tol over the interior unknowns, at
 * most max_cycles.  hist[c] is the relative residual after cycle c+1.  u is
 * the initial guess on entry (boundary entries are forced to zero). */
int oracle3_solve(void *hv, const double *bin, double *u, double tol, int max_cycles, double *hist)
{
    ohier3 *h = hv;
    olev3 *f = &h->lev[h->L - 1];
    size_t n = (size_t)f->nx * f->ny * f->nz;
    double *b = calloc(n, sizeof(double));
    for (int k = 0; k < f->nz; ++k)
        for (int j = 0; j < f->ny; ++j)
            for (int i = 0; i < f->nx; ++i) {
                size_t p = vid(f, i, j, k);
                if (inside(f, i, j, k)) b[p] = bin[p];
                else u[p] = 0.0;
            }
    double bn = norm3(f, b);
    int cycles = 0;
    if (bn == 0.0) {
        memset(u, 0, n * sizeof(double));
        free(b);
        return 0;
    }
    double *r = calloc(n, sizeof(double));
    while (cycles < max_cycles) {
        vcycle3(h, h->L - 1, u, b);
        residual3(f, u, b, r);
        double rel = norm3(f, r) / bn;
        if (hist) hist[cycles] = rel;
        ++cycles;
        if (rel <= tol) break;
    }
    free(r);
    free(b);
    return cycles;
}

void oracle3_smooth(void *hv, int l, const double *b, double *x, int sweeps)
{
    ohier3 *h = hv;
    for (int s = 0; s < sweeps; ++s) gs3(&h->lev[l], x, b);
}

void oracle3_residual(void *hv, int l, const double *b, const double *x, double *r)
{
    ohier3 *h = hv;
    residual3(&h->lev[l], x, b, r);
}

void oracle3_restrict(void *hv, int l, const double *r, double *bc)
{
    ohier3 *h = hv;
    restrict3(&h->lev[l], r, &h->lev[l - 1], bc);
}

void oracle3_interp_correct(void *hv, int l, double *x, const double *r, const double *xc, int rescorr)
{
    ohier3 *h = hv;
    interp3(&h->lev[l], x, r, &h->lev[l - 1], xc, rescorr);
}

void oracle3_coarse_solve(void *hv, const double *b, double *x) { coarse3((ohier3 *)hv, x, b); }

void oracle3_vcycle(void *hv, const double *b, double *u)
{
    ohier3 *h = hv;
    vcycle3(h, h->L - 1, u, b);
}
