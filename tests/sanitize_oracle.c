/* Driver that calls every entry point of the 2D and 3D oracles on small,
 * ragged problems, built with AddressSanitizer and UndefinedBehaviorSanitizer
 * by the CPU test suite.  It checks nothing numerically (the pins do): a run
 * that ends with status 0 and no sanitizer report means no out-of-bounds
 * access, use after free, leak or undefined operation on these paths. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* 2D oracle */
void oracle_fv5(int nx, int ny, const double *cellD, double *C, double *W, double *S);
void oracle_fv5_aniso(int nx, int ny, const double *Dx, const double *Dy, double hx, double hy, double *C,
                      double *W, double *S);
void *oracle_setup(int nx, int ny, int npt, const double *planes, int coarsest_n, int nu1, int nu2, int rescorr,
                   int *status);
void oracle_free(void *h);
int oracle_num_levels(void *h);
void oracle_level_size(void *h, int l, int *nx, int *ny);
void oracle_get_stencil(void *h, int l, double *out);
void oracle_get_interp(void *h, int l, double *out);
int oracle_solve(void *h, const double *b, double *u, double tol, int max_cycles, double *hist);
void oracle_smooth(void *h, int l, const double *b, double *x, int sweeps);
void oracle_residual(void *h, int l, const double *b, const double *x, double *r);
void oracle_restrict(void *h, int l, const double *r, double *bc);
void oracle_interp_correct(void *h, int l, double *x, const double *r, const double *xc, int rescorr);
void oracle_coarse_solve(void *h, const double *b, double *x);
void oracle_vcycle(void *h, const double *b, double *u);
void oracle_grad_logD(int nx, int ny, const double *cellD, const double *u, const double *lam, double *g);
int oracle_set_threads(int n);
void oracle32_demote(void *h);
void oracle32_get_level(void *h, int l, float *A32, float *P32);
void oracle32_smooth(void *h, int l, const float *b, float *x, int sweeps);
void oracle32_residual(void *h, int l, const float *b, const float *x, float *r);
void oracle32_restrict(void *h, int l, const float *r, float *bc);
void oracle32_interp_correct(void *h, int l, float *x, const float *r, const float *xc, int rescorr);
void oracle32_vcycle(void *h, const float *b, float *x);
int oracle32_inner(void *h, const float *r, float *e, int cycles, double rnorm, double inner_tol, double *hist);
int oracle_solve_mixed(void *h, const double *b, double *u, double tol, int max_cycles, int inner_max,
                       double inner_tol, int adapt, double *hist, int *steps);
/* 3D oracle */
void oracle3_fv7(int nx, int ny, int nz, const double *cellD, double *C, double *W, double *S, double *B);
void *oracle3_setup(int nx, int ny, int nz, int npt, const double *planes, int coarsest_n, int nu1, int nu2,
                    int rescorr, int *status);
void oracle3_free(void *h);
int oracle3_num_levels(void *h);
void oracle3_level_size(void *h, int l, int *nx, int *ny, int *nz);
void oracle3_get_stencil(void *h, int l, double *out);
void oracle3_get_interp(void *h, int l, double *out);
int oracle3_solve(void *h, const double *b, double *u, double tol, int max_cycles, double *hist);
void oracle3_smooth(void *h, int l, const double *b, double *x, int sweeps);
void oracle3_residual(void *h, int l, const double *b, const double *x, double *r);
void oracle3_restrict(void *h, int l, const double *r, double *bc);
void oracle3_interp_correct(void *h, int l, double *x, const double *r, const double *xc, int rescorr);
void oracle3_coarse_solve(void *h, const double *b, double *x);
void oracle3_vcycle(void *h, const double *b, double *u);

static unsigned long long rng_state = 88172645463325252ULL;
static double urand(void)   /* xorshift64, uniform in [0, 1) */
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) / 9007199254740992.0;
}

static double *vec(size_t n, double lo, double hi)
{
    double *v = malloc(n * sizeof(double));
    for (size_t k = 0; k < n; ++k) v[k] = lo + (hi - lo) * urand();
    return v;
}

static float *vec32(size_t n)
{
    float *v = malloc(n * sizeof(float));
    for (size_t k = 0; k < n; ++k) v[k] = (float)(2.0 * urand() - 1.0);
    return v;
}

static double checksum = 0.0;
static void acc(const double *v, size_t n)
{
    for (size_t k = 0; k < n; ++k) checksum += fabs(v[k]);
}

/* every solve-phase operation on every level, FP64 and FP32 */
static void exercise2(void *h, int nx, int ny)
{
    int L = oracle_num_levels(h);
    for (int l = 0; l < L; ++l) {
        int lx, ly;
        oracle_level_size(h, l, &lx, &ly);
        size_t n = (size_t)lx * ly;
        double *st = malloc(n * 9 * sizeof(double)), *P = malloc(n * 4 * sizeof(double));
        oracle_get_stencil(h, l, st);
        acc(st, n * 9);
        double *b = vec(n, -1, 1), *x = vec(n, -1, 1), *r = calloc(n, sizeof(double));
        oracle_smooth(h, l, b, x, 2);
        oracle_residual(h, l, b, x, r);
        acc(r, n);
        if (l >= 1) {
            oracle_get_interp(h, l, P);
            int cx, cy;
            oracle_level_size(h, l - 1, &cx, &cy);
            double *bc = calloc((size_t)cx * cy, sizeof(double)), *xc = vec((size_t)cx * cy, -1, 1);
            oracle_restrict(h, l, r, bc);
            oracle_interp_correct(h, l, x, r, xc, 1);
            oracle_interp_correct(h, l, x, r, xc, 0);
            acc(bc, (size_t)cx * cy);
            float *r32 = vec32(n), *x32 = vec32(n), *b32 = vec32(n), *bc32 = calloc((size_t)cx * cy, sizeof(float));
            float *xc32 = vec32((size_t)cx * cy);
            oracle32_smooth(h, l, b32, x32, 2);
            oracle32_residual(h, l, b32, x32, r32);
            oracle32_restrict(h, l, r32, bc32);
            oracle32_interp_correct(h, l, x32, r32, xc32, 1);
            free(r32), free(x32), free(b32), free(bc32), free(xc32), free(bc), free(xc);
        } else {
            oracle_coarse_solve(h, b, x);
        }
        float *A32 = malloc(n * 9 * sizeof(float)), *P32 = malloc(n * 4 * sizeof(float));
        oracle32_get_level(h, l, A32, P32);
        free(A32), free(P32), free(st), free(P), free(b), free(x), free(r);
    }
    size_t n = (size_t)nx * ny;
    double *b = vec(n, -1, 1), *u = calloc(n, sizeof(double)), hist[200];
    int cyc = oracle_solve(h, b, u, 1e-10, 200, hist);
    oracle_vcycle(h, b, u);
    acc(u, n);
    int steps = 0;
    memset(u, 0, n * sizeof(double));
    int cyc32 = oracle_solve_mixed(h, b, u, 1e-10, 200, 32, 1e-4, 1, hist, &steps);
    float *r32 = vec32(n), *e32 = calloc(n, sizeof(float));
    double ih[4];
    oracle32_inner(h, r32, e32, 4, 1.0, 0.0, ih);
    oracle32_vcycle(h, r32, e32);
    printf("2D %dx%d: %d levels, %d cycles, mixed %d cycles in %d steps\n", nx, ny, L, cyc, cyc32, steps);
    free(b), free(u), free(r32), free(e32);
}

static void run2d(int nx, int ny, int npt)
{
    size_t n = (size_t)nx * ny, nc = (size_t)(nx - 1) * (ny - 1);
    double *D = vec(nc, 0.01, 100.0);
    double *planes = calloc(5 * n, sizeof(double));
    oracle_fv5(nx, ny, D, planes, planes + n, planes + 2 * n);
    if (npt == 9)
        for (size_t k = 0; k < n; ++k) {   /* small extra diagonal couplings */
            planes[3 * n + k] = 0.05 * planes[n + k];
            planes[4 * n + k] = 0.05 * planes[2 * n + k];
            planes[k] += 0.4 * (planes[n + k] + planes[2 * n + k]);
        }
    int st = 0;
    void *h = oracle_setup(nx, ny, npt, planes, 3, 2, 1, 1, &st);
    if (!h || st) {
        fprintf(stderr, "setup failed (%d)\n", st);
        exit(1);
    }
    oracle32_demote(h);
    exercise2(h, nx, ny);
    double *u = vec(n, -1, 1), *lam = vec(n, -1, 1), *g = malloc(nc * sizeof(double));
    oracle_grad_logD(nx, ny, D, u, lam, g);
    acc(g, nc);
    oracle_free(h);
    double *Dy = vec(nc, 0.01, 100.0);
    oracle_fv5_aniso(nx, ny, D, Dy, 1.0 / (nx - 1), 16.0 / (ny - 1), planes, planes + n, planes + 2 * n);
    h = oracle_setup(nx, ny, 5, planes, 5, 1, 1, 0, &st);
    exercise2(h, nx, ny);
    oracle_free(h);
    free(D), free(Dy), free(planes), free(u), free(lam), free(g);
}

static void run3d(int nx, int ny, int nz, int npt)
{
    size_t n = (size_t)nx * ny * nz, nc = (size_t)(nx - 1) * (ny - 1) * (nz - 1);
    double *D = vec(nc, 0.01, 100.0);
    double *planes = calloc(14 * n, sizeof(double));
    oracle3_fv7(nx, ny, nz, D, planes, planes + n, planes + 2 * n, planes + 3 * n);
    if (npt == 27) {
        /* a 27-point operator: the first Galerkin level of a finer 7-point grid */
        int fx = 2 * nx - 1, fy = 2 * ny - 1, fz = 2 * nz - 1, st = 0;
        size_t fn = (size_t)fx * fy * fz, fc = (size_t)(fx - 1) * (fy - 1) * (fz - 1);
        double *fD = vec(fc, 0.01, 100.0), *fp = calloc(4 * fn, sizeof(double));
        oracle3_fv7(fx, fy, fz, fD, fp, fp + fn, fp + 2 * fn, fp + 3 * fn);
        void *fh = oracle3_setup(fx, fy, fz, 7, fp, 3, 2, 1, 1, &st);
        double *A = malloc(n * 27 * sizeof(double));
        oracle3_get_stencil(fh, oracle3_num_levels(fh) - 2, A);
        for (size_t p = 0; p < n; ++p) {
            planes[p] = A[p * 27 + 13];
            for (int o = 0; o < 13; ++o) planes[(size_t)(1 + o) * n + p] = -A[p * 27 + o];
        }
        oracle3_free(fh);
        free(fD), free(fp), free(A);
    }
    int st = 0;
    void *h = oracle3_setup(nx, ny, nz, npt, planes, 3, 2, 1, 1, &st);
    if (!h || st) {
        fprintf(stderr, "3D setup failed (%d)\n", st);
        exit(1);
    }
    int L = oracle3_num_levels(h);
    for (int l = 0; l < L; ++l) {
        int lx, ly, lz;
        oracle3_level_size(h, l, &lx, &ly, &lz);
        size_t m = (size_t)lx * ly * lz;
        double *A = malloc(m * 27 * sizeof(double)), *P = malloc(m * 8 * sizeof(double));
        oracle3_get_stencil(h, l, A);
        double *b = vec(m, -1, 1), *x = vec(m, -1, 1), *r = calloc(m, sizeof(double));
        oracle3_smooth(h, l, b, x, 2);
        oracle3_residual(h, l, b, x, r);
        if (l >= 1) {
            oracle3_get_interp(h, l, P);
            int cx, cy, cz;
            oracle3_level_size(h, l - 1, &cx, &cy, &cz);
            size_t mc = (size_t)cx * cy * cz;
            double *bc = calloc(mc, sizeof(double)), *xc = vec(mc, -1, 1);
            oracle3_restrict(h, l, r, bc);
            oracle3_interp_correct(h, l, x, r, xc, 1);
            acc(bc, mc);
            free(bc), free(xc);
        } else {
            oracle3_coarse_solve(h, b, x);
        }
        acc(x, m);
        free(A), free(P), free(b), free(x), free(r);
    }
    double *b = vec(n, -1, 1), *u = calloc(n, sizeof(double)), hist[200];
    int cyc = oracle3_solve(h, b, u, 1e-10, 200, hist);
    oracle3_vcycle(h, b, u);
    printf("3D %dx%dx%d (%d-point): %d levels, %d cycles\n", nx, ny, nz, npt, L, cyc);
    oracle3_free(h);
    free(D), free(planes), free(b), free(u);
}

int main(void)
{
    oracle_set_threads(2);
    run2d(33, 17, 5);
    run2d(25, 41, 9);
    run2d(3, 3, 5);
    run3d(9, 17, 13, 7);
    run3d(9, 5, 9, 27);
    run3d(3, 3, 3, 7);
    /* rejected arguments leave nothing behind */
    int st = 0;
    double z[64] = {0};
    if (oracle_setup(4, 5, 5, z, 3, 2, 1, 1, &st) != NULL || st == 0) return 2;
    if (oracle3_setup(4, 3, 3, 7, z, 3, 2, 1, 1, &st) != NULL || st == 0) return 3;
    printf("checksum %.6e\n", checksum);
    return 0;
}
