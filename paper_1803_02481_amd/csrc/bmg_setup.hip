// bmg_setup.hip -- setup-phase kernels: finite-volume operator, operator-induced
// interpolation, Galerkin coarse operator, and the adjoint gradient kernel.
// One thread per output vertex (or cell); these run once per hierarchy and are
// not part of the solve-phase time the paper reports.
#include "bmg_internal.h"
#include "bmg_weights.h"

namespace hbmg {

// ---------------------------------------------------------------------------
// Vertex-centred 5-point finite volume (section 5): connection across the dual
// face of edge p-q is the mean of the two cells the face cuts; C = sum of the
// four connections.  cell is D, or theta = ln D when is_log.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double cell_at(const double *cell, int nx, int ny, int ci, int cj,
                                          int is_log)
{
    if (ci < 0 || cj < 0 || ci >= nx - 1 || cj >= ny - 1) return 0.0;
    double v = cell[(size_t)cj * (nx - 1) + ci];
    return is_log ? exp(v) : v;
}

// Diagonal tensor D = diag(Dx, Dy) per cell on a grid of spacings hx, hy
// (section 5, the stretched grids with compensating anisotropy): the dual face
// of an x-edge has length hy across a distance hx, so it takes sx = hy/hx times
// the mean Dx of the two cells it cuts; a y-edge takes sy = hx/hy times the
// mean Dy.  The isotropic form passes the same cells twice and sx = sy = 1.
// (blockIdx.z: problem of a batch, its cells cstride and its planes ostride
// elements after the previous problem's)
__global__ void k_fv5(int nx, int ny, const double *__restrict__ cx, const double *__restrict__ cy, int is_log,
                      double sx, double sy, double *__restrict__ C, double *__restrict__ W,
                      double *__restrict__ S, int pitch, size_t cstride, size_t ostride)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    if (i >= nx) return;
    cx += blockIdx.z * cstride;
    cy += blockIdx.z * cstride;
    C += blockIdx.z * ostride;
    W += blockIdx.z * ostride;
    S += blockIdx.z * ostride;
    size_t p = (size_t)j * pitch + i;
    // W(i,j): edge (i-1,j)-(i,j), cells (i-1,j-1) and (i-1,j)
    double w = 0.0, s = 0.0;
    if (i >= 1 && j >= 1 && j <= ny - 2)
        w = sx * (0.5 * (cell_at(cx, nx, ny, i - 1, j - 1, is_log) + cell_at(cx, nx, ny, i - 1, j, is_log)));
    // S(i,j): edge (i,j-1)-(i,j), cells (i-1,j-1) and (i,j-1)
    if (j >= 1 && i >= 1 && i <= nx - 2)
        s = sy * (0.5 * (cell_at(cy, nx, ny, i - 1, j - 1, is_log) + cell_at(cy, nx, ny, i, j - 1, is_log)));
    W[p] = w;
    S[p] = s;
    double c = 0.0;
    if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2) {
        double we = sx * (0.5 * (cell_at(cx, nx, ny, i, j - 1, is_log) + cell_at(cx, nx, ny, i, j, is_log)));
        double sn = sy * (0.5 * (cell_at(cy, nx, ny, i - 1, j, is_log) + cell_at(cy, nx, ny, i, j, is_log)));
        c = w + we + s + sn;
    }
    C[p] = c;
}

hipError_t launch_fv5(int nx, int ny, const double *cell, int is_log, double *C, double *W,
                      double *S, int pitch, hipStream_t s, int nprob, size_t ostride)
{
    dim3 b(256), g((nx + 255) / 256, ny, nprob);
    hipLaunchKernelGGL(k_fv5, g, b, 0, s, nx, ny, cell, cell, is_log, 1.0, 1.0, C, W, S, pitch,
                       (size_t)(nx - 1) * (ny - 1), ostride);
    return hipGetLastError();
}

hipError_t launch_fv5_aniso(int nx, int ny, const double *dx_cell, const double *dy_cell, double hx, double hy,
                            double *C, double *W, double *S, int pitch, hipStream_t s)
{
    dim3 b(256), g((nx + 255) / 256, ny);
    hipLaunchKernelGGL(k_fv5, g, b, 0, s, nx, ny, dx_cell, dy_cell, 0, hy / hx, hx / hy, C, W, S, pitch, 0, 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adjoint gradient with respect to theta = ln D per cell: with
// u^T A v = sum_edges a_e (u_p - u_q)(v_p - v_q) and each edge taking D_c/2
// from each cell its dual face cuts,
//   g_c = -(D_c/2) sum_{4 edges of c} (lam_p - lam_q)(u_p - u_q).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double vtx(const double *v, int nx, int ny, int i, int j)
{
    if (i <= 0 || j <= 0 || i >= nx - 1 || j >= ny - 1) return 0.0;
    return v[(size_t)j * nx + i];
}

// (blockIdx.z: problem of a batch of one size, arrays stored one after another)
__global__ void k_grad_logD(int nx, int ny, const double *__restrict__ theta,
                            const double *__restrict__ u, const double *__restrict__ lam,
                            double *__restrict__ g)
{
    int ci = blockIdx.x * blockDim.x + threadIdx.x;
    int cj = blockIdx.y;
    if (ci >= nx - 1) return;
    const size_t vs = (size_t)blockIdx.z * nx * ny, cs = (size_t)blockIdx.z * (nx - 1) * (ny - 1);
    theta += cs;
    g += cs;
    u += vs;
    lam += vs;
    double u00 = vtx(u, nx, ny, ci, cj), u10 = vtx(u, nx, ny, ci + 1, cj);
    double u01 = vtx(u, nx, ny, ci, cj + 1), u11 = vtx(u, nx, ny, ci + 1, cj + 1);
    double l00 = vtx(lam, nx, ny, ci, cj), l10 = vtx(lam, nx, ny, ci + 1, cj);
    double l01 = vtx(lam, nx, ny, ci, cj + 1), l11 = vtx(lam, nx, ny, ci + 1, cj + 1);
    double s = (l00 - l10) * (u00 - u10) + (l01 - l11) * (u01 - u11) + (l00 - l01) * (u00 - u01) +
               (l10 - l11) * (u10 - u11);
    size_t c = (size_t)cj * (nx - 1) + ci;
    g[c] = -0.5 * exp(theta[c]) * s;
}

hipError_t launch_grad_logD(int nx, int ny, const double *theta, const double *u,
                            const double *lam, double *g, hipStream_t s, int nprob)
{
    dim3 b(256), g2((nx - 1 + 255) / 256, ny - 1, nprob);
    hipLaunchKernelGGL(k_grad_logD, g2, b, 0, s, nx, ny, theta, u, lam, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Operator-induced interpolation (section 2).  For coarse cell (I,J) one
// thread builds the weights of its three fine-only vertices:
//   x-line vertex p=(2I+1,2J): collapse the stencil onto the coarse line,
//     w = (sum of connections towards that coarse column) / (C - S_p - N_p);
//   y-line vertex p=(2I,2J+1): the same with rows;
//   cell centre p=(2I+1,2J+1): e_p = sum_q conn_pq e_q / C_p over its eight
//     neighbours, the four edge neighbours replaced by their line weights.
// Weights on boundary coarse vertices are zero; boundary fine vertices carry
// no row.
// ---------------------------------------------------------------------------
struct StView {
    int nx, ny, pitch;
    const double *C, *W, *S, *SW, *SE;
    int npt;
    __device__ double c(int i, int j) const { return C[(size_t)j * pitch + i]; }
    __device__ double w(int i, int j) const { return W[(size_t)j * pitch + i]; }
    __device__ double s(int i, int j) const { return S[(size_t)j * pitch + i]; }
    __device__ double sw(int i, int j) const { return npt == 9 ? SW[(size_t)j * pitch + i] : 0.0; }
    __device__ double se(int i, int j) const { return npt == 9 ? SE[(size_t)j * pitch + i] : 0.0; }
    __device__ bool inner(int i, int j) const { return i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2; }
};

// weights of the x-line vertex (i odd, j even) on its west and east coarse vertices
__device__ void xline_w(const StView &A, int i, int j, double &ww, double &we)
{
    xline_weights(A.c(i, j), A.s(i, j + 1), A.s(i, j), A.w(i, j), A.se(i - 1, j + 1), A.sw(i, j), A.w(i + 1, j),
                  A.sw(i + 1, j + 1), A.se(i, j), ww, we);
}

// weights of the y-line vertex (i even, j odd) on its south and north coarse vertices
__device__ void yline_w(const StView &A, int i, int j, double &ws, double &wn)
{
    yline_weights(A.c(i, j), A.w(i + 1, j), A.w(i, j), A.s(i, j), A.se(i, j), A.sw(i, j), A.s(i, j + 1),
                  A.sw(i + 1, j + 1), A.se(i - 1, j + 1), ws, wn);
}

// the 8 weights stored at coarse vertex (I, J)
__device__ __forceinline__ void interp_weights_at(const StView &A, int cnx, int cny, double *__restrict__ wt,
                                                  int cpitch, size_t cplane, int I, int J)
{
    auto cin = [&](int a, int b) { return a >= 1 && a <= cnx - 2 && b >= 1 && b <= cny - 2; };
    double w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // x-line vertex (2I+1, 2J)
    int i = 2 * I + 1, j = 2 * J;
    if (A.inner(i, j)) xline_w(A, i, j, w[WXL], w[WXR]);
    // y-line vertex (2I, 2J+1)
    i = 2 * I;
    j = 2 * J + 1;
    if (A.inner(i, j)) yline_w(A, i, j, w[WYB], w[WYT]);
    // cell centre (2I+1, 2J+1)
    i = 2 * I + 1;
    j = 2 * J + 1;
    if (A.inner(i, j)) {
        double sl = 0, sr = 0, nl = 0, nr = 0, wb = 0, wtp = 0, eb = 0, etp = 0;
        if (A.inner(i, j - 1)) xline_w(A, i, j - 1, sl, sr);      // south edge neighbour
        if (A.inner(i, j + 1)) xline_w(A, i, j + 1, nl, nr);      // north edge neighbour
        if (A.inner(i - 1, j)) yline_w(A, i - 1, j, wb, wtp);     // west edge neighbour
        if (A.inner(i + 1, j)) yline_w(A, i + 1, j, eb, etp);     // east edge neighbour
        // e_p = -sum_q A(p,q) e_q / A(p,p); a boundary edge neighbour holds e = 0,
        // which its zero line weights express
        double cw = A.w(i, j), ce = A.w(i + 1, j), cs = A.s(i, j), cn = A.s(i, j + 1);
        double csw = A.sw(i, j), cne = A.sw(i + 1, j + 1), cse = A.se(i, j), cnw = A.se(i - 1, j + 1);
        double d = A.c(i, j);
        w[WCSW] = centre_weight(csw, cs, sl, cw, wb, d);
        w[WCSE] = centre_weight(cse, cs, sr, ce, eb, d);
        w[WCNW] = centre_weight(cnw, cn, nl, cw, wtp, d);
        w[WCNE] = centre_weight(cne, cn, nr, ce, etp, d);
    }
    // no weight on boundary coarse vertices
    if (!cin(I, J)) w[WXL] = w[WYB] = w[WCSW] = 0.0;
    if (!cin(I + 1, J)) w[WXR] = w[WCSE] = 0.0;
    if (!cin(I, J + 1)) w[WYT] = w[WCNW] = 0.0;
    if (!cin(I + 1, J + 1)) w[WCNE] = 0.0;
    size_t o = (size_t)J * cpitch + I;
    for (int k = 0; k < 8; ++k) wt[k * cplane + o] = w[k];
}

__global__ void k_interp_weights(StView A, int cnx, int cny, double *__restrict__ wt, int cpitch,
                                 size_t cplane)
{
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    int J = blockIdx.y;
    if (I >= cnx) return;
    interp_weights_at(A, cnx, cny, wt, cpitch, cplane, I, J);
}

hipError_t launch_interp_weights(const LevelDev<double> &f, int cnx, int cny, double *wt,
                                 int cpitch, size_t cplane, hipStream_t s)
{
    StView A{f.nx, f.ny, f.pitch, f.C, f.W, f.S, f.SW, f.SE, f.npt};
    dim3 b(128), g((cnx + 127) / 128, cny);
    hipLaunchKernelGGL(k_interp_weights, g, b, 0, s, A, cnx, cny, wt, cpitch, cplane);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Galerkin coarse operator A_c = P^T A P (section 2), one thread per coarse
// vertex I computing A_c(I, J) for J in {I, W, S, SW, SE}:
//   A_c(I,J) = sum_{p in supp P(.,I)} P(p,I) sum_{q ~ p, q in supp P(.,J)} A(p,q) P(q,J),
// with p, q interior fine vertices and I, J interior coarse vertices.
// ---------------------------------------------------------------------------
struct WView {
    const double *wt;
    int cnx, cny, cpitch;
    size_t cplane;
    __device__ double at(int k, int I, int J) const
    {
        if (I < 0 || J < 0 || I >= cnx || J >= cny) return 0.0;
        return wt[k * cplane + (size_t)J * cpitch + I];
    }
    // P(2I+dx, 2J+dy ; I,J) for dx, dy in {-1,0,1}
    __device__ double col(int I, int J, int dx, int dy) const
    {
        if (dx == 0 && dy == 0) return 1.0;
        if (dy == 0) return dx > 0 ? at(WXL, I, J) : at(WXR, I - 1, J);
        if (dx == 0) return dy > 0 ? at(WYB, I, J) : at(WYT, I, J - 1);
        if (dx > 0 && dy > 0) return at(WCSW, I, J);
        if (dx < 0 && dy > 0) return at(WCSE, I - 1, J);
        if (dx > 0 && dy < 0) return at(WCNW, I, J - 1);
        return at(WCNE, I - 1, J - 1);
    }
};

// matrix entry A(p, p + (sx, sy)) from the planes
__device__ __forceinline__ double Aent(const StView &A, int i, int j, int sx, int sy)
{
    if (sx == 0 && sy == 0) return A.c(i, j);
    if (sy == 0) return -(sx < 0 ? A.w(i, j) : A.w(i + 1, j));
    if (sx == 0) return -(sy < 0 ? A.s(i, j) : A.s(i, j + 1));
    if (sx < 0 && sy < 0) return -A.sw(i, j);
    if (sx > 0 && sy > 0) return -A.sw(i + 1, j + 1);
    if (sx > 0 && sy < 0) return -A.se(i, j);
    return -A.se(i - 1, j + 1);
}

// the five stored entries of A_c at coarse vertex (I, J)
__device__ __forceinline__ void rap_at(const StView &A, const WView &P, double *__restrict__ Cc,
                                       double *__restrict__ Wc, double *__restrict__ Sc, double *__restrict__ SWc,
                                       double *__restrict__ SEc, int cpitch, int I, int J)
{
    const int cnx = P.cnx, cny = P.cny;
    auto cin = [&](int a, int b) { return a >= 1 && a <= cnx - 2 && b >= 1 && b <= cny - 2; };
    double out[5] = {0, 0, 0, 0, 0};
    // fully unrolled (the summation order is the loops' order): every array
    // index is a constant, so the stencil and weights stay in registers
    if (cin(I, J)) {
        const int dirs[5][2] = {{0, 0}, {-1, 0}, {0, -1}, {-1, -1}, {1, -1}};
        // every weight and matrix entry the sums can touch, loaded before any
        // of the sums' data-dependent skips, so no load waits on another
        // load's value (all in bounds for an interior coarse vertex: the fine
        // points and their neighbours lie within 2I-2..2I+2, 2J-2..2J+2)
        double pi[3][3], pw[5][3][3], a[3][3][3][3];
        #pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
            #pragma unroll
            for (int dx = -1; dx <= 1; ++dx) pi[dy + 1][dx + 1] = P.col(I, J, dx, dy);
        #pragma unroll
        for (int d = 0; d < 5; ++d)
            #pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
                #pragma unroll
                for (int dx = -1; dx <= 1; ++dx)
                    pw[d][dy + 1][dx + 1] = P.col(I + dirs[d][0], J + dirs[d][1], dx, dy);
        #pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
            #pragma unroll
            for (int dx = -1; dx <= 1; ++dx)
                #pragma unroll
                for (int sy = -1; sy <= 1; ++sy)
                    #pragma unroll
                    for (int sx = -1; sx <= 1; ++sx)
                        a[dy + 1][dx + 1][sy + 1][sx + 1] = Aent(A, 2 * I + dx, 2 * J + dy, sx, sy);
        #pragma unroll
        for (int d = 0; d < 5; ++d) {
            const int ex = dirs[d][0], ey = dirs[d][1];
            const int KI = I + ex, KJ = J + ey;
            if (!cin(KI, KJ)) continue;
            const double (&pj)[3][3] = pw[d];
            double acc = 0.0;
            #pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
                #pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const double wp = pi[dy + 1][dx + 1];
                    const int pi_ = 2 * I + dx, pj_ = 2 * J + dy;
                    if (wp == 0.0 || !A.inner(pi_, pj_)) continue;
                    double inner = 0.0;
                    #pragma unroll
                    for (int sy = -1; sy <= 1; ++sy)
                        #pragma unroll
                        for (int sx = -1; sx <= 1; ++sx) {
                            // q = p + s, offset from 2K
                            const int ox = dx + sx - 2 * ex, oy = dy + sy - 2 * ey;
                            if (ox < -1 || ox > 1 || oy < -1 || oy > 1) continue;
                            if (!A.inner(pi_ + sx, pj_ + sy)) continue;
                            const double wq = pj[oy + 1][ox + 1];
                            if (wq == 0.0) continue;
                            inner += a[dy + 1][dx + 1][sy + 1][sx + 1] * wq;
                        }
                    acc += wp * inner;
                }
            out[d] = d == 0 ? acc : -acc;
        }
    }
    size_t o = (size_t)J * cpitch + I;
    Cc[o] = out[0];
    Wc[o] = out[1];
    Sc[o] = out[2];
    SWc[o] = out[3];
    SEc[o] = out[4];
}

__global__ __launch_bounds__(128) void k_rap(StView A, WView P, double *__restrict__ Cc, double *__restrict__ Wc,
                      double *__restrict__ Sc, double *__restrict__ SWc, double *__restrict__ SEc,
                      int cpitch)
{
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    int J = blockIdx.y;
    if (I >= P.cnx) return;
    rap_at(A, P, Cc, Wc, Sc, SWc, SEc, cpitch, I, J);
}

hipError_t launch_rap(const LevelDev<double> &f, const LevelDev<double> &c, hipStream_t s)
{
    StView A{f.nx, f.ny, f.pitch, f.C, f.W, f.S, f.SW, f.SE, f.npt};
    WView P{f.wt, c.nx, c.ny, c.pitch, c.plane};   // weights onto f live at c's resolution
    dim3 b(128), g((c.nx + 127) / 128, c.ny);
    hipLaunchKernelGGL(k_rap, g, b, 0, s, A, P, c.C, c.W, c.S, c.SW, c.SE, c.pitch);
    return hipGetLastError();
}

// The smallest levels' weights and Galerkin products, level after level, in
// one workgroup: the same per-vertex functions as the two kernels above, with
// a barrier between the steps (each step reads what the step before wrote),
// instead of two short launches per level.
struct TailLevel {
    StView A;
    WView P;
    double *C, *W, *S, *SW, *SE;
    int cpitch;
};
struct TailArgs {
    int n;
    TailLevel lv[SETUP_TAIL_MAX];
};

__global__ __launch_bounds__(256) void k_setup_tail(TailArgs a)
{
#pragma unroll
    for (int k = 0; k < SETUP_TAIL_MAX; ++k) {
        if (k >= a.n) break;
        const TailLevel &t = a.lv[k];
        const int cnx = t.P.cnx, npts = cnx * t.P.cny;
        double *wt = const_cast<double *>(t.P.wt);
        for (int v = threadIdx.x; v < npts; v += blockDim.x)
            interp_weights_at(t.A, cnx, t.P.cny, wt, t.P.cpitch, t.P.cplane, v % cnx, v / cnx);
        __syncthreads();
        for (int v = threadIdx.x; v < npts; v += blockDim.x)
            rap_at(t.A, t.P, t.C, t.W, t.S, t.SW, t.SE, t.cpitch, v % cnx, v / cnx);
        __syncthreads();
    }
}

hipError_t launch_setup_tail(const LevelDev<double> *lv, int l_top, hipStream_t s)
{
    if (l_top < 1 || l_top > SETUP_TAIL_MAX) return hipErrorInvalidValue;
    TailArgs a{};
    a.n = l_top;
    for (int k = 0; k < l_top; ++k) {
        const LevelDev<double> &f = lv[l_top - k], &c = lv[l_top - k - 1];
        if ((long long)c.nx * c.ny > SETUP_TAIL_POINTS) return hipErrorInvalidValue;
        a.lv[k].A = StView{f.nx, f.ny, f.pitch, f.C, f.W, f.S, f.SW, f.SE, f.npt};
        a.lv[k].P = WView{f.wt, c.nx, c.ny, c.pitch, c.plane};
        a.lv[k].C = c.C;
        a.lv[k].W = c.W;
        a.lv[k].S = c.S;
        a.lv[k].SW = c.SW;
        a.lv[k].SE = c.SE;
        a.lv[k].cpitch = c.pitch;
    }
    hipLaunchKernelGGL(k_setup_tail, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace hbmg
