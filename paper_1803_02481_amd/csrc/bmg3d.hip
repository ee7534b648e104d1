// bmg3d.hip -- the 3D path of hipbmg: finite volumes, operator-induced
// interpolation, 27-point Galerkin coarse operators, eight-colour Gauss-Seidel
// V(nu1,nu2)-cycles and the coarsest Cholesky solve (section 2, Algorithm 1;
// section 3: interpolation in 3D, the r/C term, the coarse solve), and the C
// interface declared in include/hipbmg3d.h.
//
// Octant layout.  A level of nx x ny x nz vertices holds every field as eight
// sub-grids, octant o = (i&1) + 2(j&1) + 4(k&1), each mx x my x mz with
// mx = (nx+1)/2 (the odd octants leave their last entry unused), rows pitched
// to px = mx rounded up to 8.  Vertex (i,j,k) sits at
//   o * oct + (k>>1) * plane + (j>>1) * px + (i>>1).
// So one colour of the relaxation is one contiguous sub-grid, its neighbours
// in direction d are the sub-grid of octant o ^ (odd bits of d) shifted by 0
// or -1/+1 rows, and the next coarser level is octant 0 itself.  The kinds of
// fine vertex in the interpolation are octants as well: 0 coarse points,
// 1, 2, 4 on coarse lines, 3, 5, 6 on coarse faces, 7 cell centres; each
// keeps its weights in 2, 4 or 8 octant-sized slots (26 in all).
#include "hipbmg3d.h"
#include "bmg_internal.h"
#include "bmg_model.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
struct Oct {
    int nx, ny, nz;
    int mx, my, mz, px;
    long long plane, oct, field;
};

Oct make_oct(int nx, int ny, int nz)
{
    Oct g;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.mx = (nx + 1) / 2;
    g.my = (ny + 1) / 2;
    g.mz = (nz + 1) / 2;
    g.px = (g.mx + 7) & ~7;
    g.plane = (long long)g.px * g.my;
    g.oct = g.plane * g.mz;
    g.field = 8 * g.oct;
    return g;
}

__host__ __device__ inline int oct_of(int i, int j, int k) { return (i & 1) | ((j & 1) << 1) | ((k & 1) << 2); }

__host__ __device__ inline long long sub_of(const Oct &g, int i, int j, int k)
{
    return (long long)(k >> 1) * g.plane + (long long)(j >> 1) * g.px + (i >> 1);
}

__host__ __device__ inline long long vid(const Oct &g, int i, int j, int k)
{
    return oct_of(i, j, k) * g.oct + sub_of(g, i, j, k);
}

__host__ __device__ inline bool inner(const Oct &g, int i, int j, int k)
{
    return i >= 1 && i <= g.nx - 2 && j >= 1 && j <= g.ny - 2 && k >= 1 && k <= g.nz - 2;
}

// first weight slot of an octant (1, 2, 4: two slots; 3, 5, 6: four; 7: eight)
__host__ __device__ inline int wbase(int o)
{
    return o == 1 ? 0 : o == 2 ? 2 : o == 4 ? 4 : o == 3 ? 6 : o == 5 ? 10 : o == 6 ? 14 : 18;
}

// position of corner m (a subset of the odd bits o) among the corners of o
__host__ __device__ inline int wrank(int o, int m)
{
    int r = 0, s = 0;
    for (int d = 0; d < 3; ++d)
        if ((o >> d) & 1) {
            r |= ((m >> d) & 1) << s;
            ++s;
        }
    return r;
}

constexpr int NWSLOT = 26;

// Logical block of hardware block b in a grid of nb blocks (nb a multiple of
// 8).  Workgroups are dealt to the eight XCDs round-robin (b mod 8), each with
// its own L2; giving every XCD a contiguous range of logical blocks keeps the
// rows and planes that neighbouring blocks re-read in one L2.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb)
{
    return (b & 7u) * (nb >> 3) + (b >> 3);
}

inline unsigned round8(unsigned n) { return (n + 7u) & ~7u; }

// sub-grid coordinates of thread t of an octant
__device__ inline void sub_coords(const Oct &g, long long t, int &a, int &b, int &c)
{
    a = (int)(t % g.px);
    const long long r = t / g.px;
    b = (int)(r % g.my);
    c = (int)(r / g.my);
}

// ---------------------------------------------------------------------------
// stencil access (setup kernels)
// ---------------------------------------------------------------------------
struct Sten {
    const double *p;   // npt 7: fields C, W, S, B; npt 27: C and 13 lower-half connections
    int npt;
    Oct g;
};

// all 27 entries A(p, p+d) of interior vertex (i,j,k), index (dz+1)*9+(dy+1)*3+(dx+1)
__device__ void load27(const Sten &s, int i, int j, int k, double e[27])
{
    const Oct &g = s.g;
    const long long v = vid(g, i, j, k);
    const long long F = g.field;
#pragma unroll
    for (int o = 0; o < 27; ++o) e[o] = 0.0;
    e[13] = s.p[v];
    if (s.npt == 7) {
        e[12] = -s.p[F + v];
        e[14] = -s.p[F + vid(g, i + 1, j, k)];
        e[10] = -s.p[2 * F + v];
        e[16] = -s.p[2 * F + vid(g, i, j + 1, k)];
        e[4] = -s.p[3 * F + v];
        e[22] = -s.p[3 * F + vid(g, i, j, k + 1)];
    } else {
#pragma unroll
        for (int o = 0; o < 13; ++o) {
            const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
            e[o] = -s.p[(1 + o) * F + v];
            e[26 - o] = -s.p[(1 + o) * F + vid(g, i - dx, j - dy, k - dz)];
        }
    }
}

// ---------------------------------------------------------------------------
// layout conversion and finite volumes
// ---------------------------------------------------------------------------
__global__ void k3_to_oct(const double *nat, double *out, Oct g, int interior_only)
{
    const long long n = (long long)g.nx * g.ny * g.nz;
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int i = (int)(t % g.nx), j = (int)((t / g.nx) % g.ny), k = (int)(t / ((long long)g.nx * g.ny));
    const bool keep = !interior_only || inner(g, i, j, k);
    out[vid(g, i, j, k)] = keep ? nat[t] : 0.0;
}

__global__ void k3_from_oct(const double *in, double *nat, Oct g)
{
    const long long n = (long long)g.nx * g.ny * g.nz;
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int i = (int)(t % g.nx), j = (int)((t / g.nx) % g.ny), k = (int)(t / ((long long)g.nx * g.ny));
    nat[t] = inner(g, i, j, k) ? in[vid(g, i, j, k)] : 0.0;
}

__device__ inline double cellv3(const double *D, int nx, int ny, int nz, int ci, int cj, int ck)
{
    if (ci < 0 || cj < 0 || ck < 0 || ci >= nx - 1 || cj >= ny - 1 || ck >= nz - 1) return 0.0;
    return D[((long long)ck * (ny - 1) + cj) * (nx - 1) + ci];
}

// connections of the edges ending at (i,j,k) from the west, south and below:
// the mean of the four cells around the edge (0 where undefined)
__device__ inline double fv_w(const double *D, int nx, int ny, int nz, int i, int j, int k)
{
    if (!(i >= 1 && j >= 1 && j <= ny - 2 && k >= 1 && k <= nz - 2)) return 0.0;
    return 0.25 * (cellv3(D, nx, ny, nz, i - 1, j - 1, k - 1) + cellv3(D, nx, ny, nz, i - 1, j, k - 1) +
                   cellv3(D, nx, ny, nz, i - 1, j - 1, k) + cellv3(D, nx, ny, nz, i - 1, j, k));
}
__device__ inline double fv_s(const double *D, int nx, int ny, int nz, int i, int j, int k)
{
    if (!(j >= 1 && i >= 1 && i <= nx - 2 && k >= 1 && k <= nz - 2)) return 0.0;
    return 0.25 * (cellv3(D, nx, ny, nz, i - 1, j - 1, k - 1) + cellv3(D, nx, ny, nz, i, j - 1, k - 1) +
                   cellv3(D, nx, ny, nz, i - 1, j - 1, k) + cellv3(D, nx, ny, nz, i, j - 1, k));
}
__device__ inline double fv_b(const double *D, int nx, int ny, int nz, int i, int j, int k)
{
    if (!(k >= 1 && i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2)) return 0.0;
    return 0.25 * (cellv3(D, nx, ny, nz, i - 1, j - 1, k - 1) + cellv3(D, nx, ny, nz, i, j - 1, k - 1) +
                   cellv3(D, nx, ny, nz, i - 1, j, k - 1) + cellv3(D, nx, ny, nz, i, j, k - 1));
}

__global__ void k3_fv7(const double *D, int nx, int ny, int nz, double *planes)
{
    const long long n = (long long)nx * ny * nz;
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int i = (int)(t % nx), j = (int)((t / nx) % ny), k = (int)(t / ((long long)nx * ny));
    const double w = fv_w(D, nx, ny, nz, i, j, k);
    const double s = fv_s(D, nx, ny, nz, i, j, k);
    const double b = fv_b(D, nx, ny, nz, i, j, k);
    double c = 0.0;
    if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2 && k >= 1 && k <= nz - 2)
        c = w + fv_w(D, nx, ny, nz, i + 1, j, k) + s + fv_s(D, nx, ny, nz, i, j + 1, k) + b +
            fv_b(D, nx, ny, nz, i, j, k + 1);
    planes[t] = c;
    planes[n + t] = w;
    planes[2 * n + t] = s;
    planes[3 * n + t] = b;
}

// ---------------------------------------------------------------------------
// interpolation weights (section 2; the 3D passes of section 3's cost count)
// ---------------------------------------------------------------------------
struct WArgs {
    Sten s;
    double *w;    // NWSLOT octant-sized slots of the fine level
    Oct c;        // coarse geometry
};

// acc[corner of p] += f * (interpolation row of the interior vertex q)
__device__ inline void add_row(const Oct &g, const double *w, int i, int j, int k, int qi, int qj, int qk, double f,
                               double acc[8])
{
    const int oq = oct_of(qi, qj, qk);
    const int bi = i >> 1, bj = j >> 1, bk = k >> 1;
    if (oq == 0) {
        const int m = ((qi >> 1) - bi) | (((qj >> 1) - bj) << 1) | (((qk >> 1) - bk) << 2);
        acc[m] += f;
        return;
    }
    const long long sq = sub_of(g, qi, qj, qk);
    for (int m = 0; m < 8; ++m) {
        if (m & ~oq) continue;
        const double wq = w[(wbase(oq) + wrank(oq, m)) * g.oct + sq];
        const int ci = (qi >> 1) + (m & 1) - bi, cj = (qj >> 1) + ((m >> 1) & 1) - bj,
                  ck = (qk >> 1) + (m >> 2) - bk;
        acc[ci | (cj << 1) | (ck << 2)] += f * wq;
    }
}

// PASS 1: line vertices (octants 1, 2, 4 by blockIdx.y); 2: face vertices
// (octants 6, 5, 3); 3: cell centres (octant 7).
template <int PASS>
__global__ __launch_bounds__(256) void k3_weights(WArgs a)
{
    const Oct g = a.s.g;
    const int y = blockIdx.y;
    const int o = PASS == 1 ? (1 << y) : PASS == 2 ? (7 ^ (1 << y)) : 7;
    const long long t = blockIdx.x * 256LL + threadIdx.x;
    if (t >= g.oct) return;
    int sa, sb, sc;
    sub_coords(g, t, sa, sb, sc);
    const int i = 2 * sa + (o & 1), j = 2 * sb + ((o >> 1) & 1), k = 2 * sc + (o >> 2);
    if (sa >= g.mx || !inner(g, i, j, k)) return;
    double e[27];
    load27(a.s, i, j, k, e);
    double acc[8];
    for (int m = 0; m < 8; ++m) acc[m] = 0.0;
    if (PASS == 1) {
        // the odd direction t1; the relation along the line after summing the
        // stencil over the two other directions
        const int t1 = y, o1 = t1 == 0 ? 1 : 0, o2 = t1 == 2 ? 1 : 2;
        double den = 0.0, am = 0.0, ap = 0.0;
        for (int u = -1; u <= 1; ++u)
            for (int v = -1; v <= 1; ++v) {
                int d[3];
                d[o1] = u;
                d[o2] = v;
                d[t1] = 0;
                den += e[(d[2] + 1) * 9 + (d[1] + 1) * 3 + (d[0] + 1)];
                d[t1] = -1;
                am += e[(d[2] + 1) * 9 + (d[1] + 1) * 3 + (d[0] + 1)];
                d[t1] = 1;
                ap += e[(d[2] + 1) * 9 + (d[1] + 1) * 3 + (d[0] + 1)];
            }
        acc[0] = -am / den;
        acc[o] = -ap / den;
    } else if (PASS == 2) {
        // the face normal n (the even direction): sum along it, then eliminate
        // the eight in-face neighbours
        const int n = y, o1 = n == 0 ? 1 : 0, o2 = n == 2 ? 1 : 2;
        double at[3][3];
        for (int s = 0; s < 3; ++s)
            for (int r = 0; r < 3; ++r) at[s][r] = 0.0;
        for (int s = -1; s <= 1; ++s)
            for (int r = -1; r <= 1; ++r)
                for (int m = -1; m <= 1; ++m) {
                    int d[3];
                    d[o1] = r;
                    d[o2] = s;
                    d[n] = m;
                    at[s + 1][r + 1] += e[(d[2] + 1) * 9 + (d[1] + 1) * 3 + (d[0] + 1)];
                }
        const double diag = at[1][1];
        for (int s = -1; s <= 1; ++s)
            for (int r = -1; r <= 1; ++r) {
                if (r == 0 && s == 0) continue;
                const double av = at[s + 1][r + 1];
                if (av == 0.0) continue;
                int d[3];
                d[o1] = r;
                d[o2] = s;
                d[n] = 0;
                const int qi = i + d[0], qj = j + d[1], qk = k + d[2];
                if (!inner(g, qi, qj, qk)) continue;
                add_row(g, a.w, i, j, k, qi, qj, qk, -av / diag, acc);
            }
    } else {
        const double diag = e[13];
        for (int q = 0; q < 27; ++q) {
            if (q == 13) continue;
            const double av = e[q];
            if (av == 0.0) continue;
            const int qi = i + q % 3 - 1, qj = j + (q / 3) % 3 - 1, qk = k + q / 9 - 1;
            if (!inner(g, qi, qj, qk)) continue;
            add_row(g, a.w, i, j, k, qi, qj, qk, -av / diag, acc);
        }
    }
    // no weight on boundary coarse vertices
    for (int m = 0; m < 8; ++m) {
        if (m & ~o) continue;
        const int I = (i >> 1) + (m & 1), J = (j >> 1) + ((m >> 1) & 1), K = (k >> 1) + (m >> 2);
        a.w[(wbase(o) + wrank(o, m)) * g.oct + t] = inner(a.c, I, J, K) ? acc[m] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Galerkin coarse operator A_c = P^T A P (section 2), one coarse vertex per
// thread: sum over its 27 fine support vertices p, their 27 couplings q, and
// the corners of q, keeping the lower half and the diagonal.
// ---------------------------------------------------------------------------
struct RArgs {
    Sten s;
    const double *w;
    Oct c;
    double *out;   // 14 coarse fields
};

__device__ inline double weight_on(const Oct &g, const double *w, int pi, int pj, int pk, int m)
{
    const int op = oct_of(pi, pj, pk);
    if (op == 0) return m == 0 ? 1.0 : 0.0;
    return w[(wbase(op) + wrank(op, m)) * g.oct + sub_of(g, pi, pj, pk)];
}

__global__ __launch_bounds__(256) void k3_rap(RArgs a)
{
    const Oct g = a.s.g, c = a.c;
    const long long t = blockIdx.x * 256LL + threadIdx.x;
    if (t >= c.field) return;
    const int oc = (int)(t / c.oct);
    int ca, cb, cc;
    sub_coords(c, t % c.oct, ca, cb, cc);
    const int I = 2 * ca + (oc & 1), J = 2 * cb + ((oc >> 1) & 1), K = 2 * cc + (oc >> 2);
    if (ca >= c.mx || !inner(c, I, J, K)) return;
    double acc[14];
    for (int o = 0; o < 14; ++o) acc[o] = 0.0;
    for (int ez = -1; ez <= 1; ++ez)
        for (int ey = -1; ey <= 1; ++ey)
            for (int ex = -1; ex <= 1; ++ex) {
                const int pi = 2 * I + ex, pj = 2 * J + ey, pk = 2 * K + ez;
                // p's corner that is I: the bit is set where e = -1
                const int mI = (ex == -1 ? 1 : 0) | (ey == -1 ? 2 : 0) | (ez == -1 ? 4 : 0);
                const double wp = weight_on(g, a.w, pi, pj, pk, mI);
                if (wp == 0.0) continue;
                double e[27];
                load27(a.s, pi, pj, pk, e);
                for (int f = 0; f < 27; ++f) {
                    const double av = e[f];
                    if (av == 0.0) continue;
                    const int qi = pi + f % 3 - 1, qj = pj + (f / 3) % 3 - 1, qk = pk + f / 9 - 1;
                    if (!inner(g, qi, qj, qk)) continue;
                    const int oq = oct_of(qi, qj, qk);
                    const double wa = wp * av;
                    for (int m = 0; m < 8; ++m) {
                        if (m & ~oq) continue;
                        const int dI = (qi >> 1) + (m & 1) - I, dJ = (qj >> 1) + ((m >> 1) & 1) - J,
                                  dK = (qk >> 1) + (m >> 2) - K;
                        const int lin = (dK + 1) * 9 + (dJ + 1) * 3 + (dI + 1);
                        if (lin > 13) continue;
                        acc[lin] += wa * weight_on(g, a.w, qi, qj, qk, m);
                    }
                }
            }
    a.out[t] = acc[13];
    for (int o = 0; o < 13; ++o) a.out[(1 + o) * c.field + t] = -acc[o];
}

// level operator in the plain layout: 27 entries per vertex, zero towards the boundary
__global__ void k3_stencil_out(Sten s, double *out)
{
    const Oct &g = s.g;
    const long long n = (long long)g.nx * g.ny * g.nz;
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int i = (int)(t % g.nx), j = (int)((t / g.nx) % g.ny), k = (int)(t / ((long long)g.nx * g.ny));
    double e[27];
    if (inner(g, i, j, k)) {
        load27(s, i, j, k, e);
        for (int o = 0; o < 27; ++o)
            if (o != 13 && !inner(g, i + o % 3 - 1, j + (o / 3) % 3 - 1, k + o / 9 - 1)) e[o] = 0.0;
    } else {
        for (int o = 0; o < 27; ++o) e[o] = 0.0;
    }
    for (int o = 0; o < 27; ++o) out[o * n + t] = e[o];
}

__global__ void k3_interp_out(Oct g, const double *w, double *out)
{
    const long long n = (long long)g.nx * g.ny * g.nz;
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int i = (int)(t % g.nx), j = (int)((t / g.nx) % g.ny), k = (int)(t / ((long long)g.nx * g.ny));
    const bool in = inner(g, i, j, k);
    const int o = oct_of(i, j, k);
    for (int m = 0; m < 8; ++m) {
        double v = 0.0;
        if (in && !(m & ~o)) v = weight_on(g, w, i, j, k, m);
        out[m * n + t] = v;
    }
}

// ---------------------------------------------------------------------------
// solve phase
// ---------------------------------------------------------------------------
struct LArgs {
    Oct g;
    const double *st;  // stencil fields
    const double *b;
    double *x;
    double *r;         // residual out / in
    const double *w;   // weights (fine level)
    Oct c;             // coarse geometry
    const double *xc;
    double *bc;
    double *partials;
    int rescorr;
    double *xcz;       // restriction: the coarse iterate, cleared alongside
    int zc;            // 7-point level whose diagonal is the sum of its connections
};

// index of the neighbour at (DX,DY,DZ) of thread t of octant O
template <int O, int DX, int DY, int DZ>
__device__ __forceinline__ long long nbr(const Oct &g, long long t)
{
    constexpr int ox = (O & 1) + DX, oy = ((O >> 1) & 1) + DY, oz = (O >> 2) + DZ;
    constexpr int on = (ox & 1) | ((oy & 1) << 1) | ((oz & 1) << 2);
    constexpr int sx = ox >> 1, sy = oy >> 1, sz = oz >> 1;
    return on * g.oct + t + sz * g.plane + sy * g.px + sx;
}

template <bool NT>
__device__ __forceinline__ double ldc(const double *p)
{
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

// sum_q A(p,q) x_q over the whole stencil of vertex t of octant O (NT: the
// 7-point coefficients as nontemporal loads; ZC: the 7-point diagonal formed
// as W_p + W_e + S_p + S_n + B_p + B_t in this order instead of loaded, which
// the setup checked is bitwise the stored one; diag receives the diagonal)
template <int NPT, int O, bool NT = false, bool ZC = false>
__device__ __forceinline__ double apply_at(const Oct &g, const double *st, const double *x, long long t,
                                           double *diag = nullptr)
{
    const long long F = g.field;
    const long long v = O * g.oct + t;
    if (NPT == 7) {
        // in a relaxation the coefficients stream through once per sweep
        // (nontemporal); the iterate's octants are read again by the
        // neighbouring colours
        const double *C = st, *W = st + F, *S = st + 2 * F, *B = st + 3 * F;
        const long long xw = nbr<O, -1, 0, 0>(g, t), xe = nbr<O, 1, 0, 0>(g, t);
        const long long ys = nbr<O, 0, -1, 0>(g, t), yn = nbr<O, 0, 1, 0>(g, t);
        const long long zb = nbr<O, 0, 0, -1>(g, t), zt = nbr<O, 0, 0, 1>(g, t);
        const double wv = ldc<NT>(W + v), we = ldc<NT>(W + xe), sv = ldc<NT>(S + v), sn = ldc<NT>(S + yn),
                     bv = ldc<NT>(B + v), bt = ldc<NT>(B + zt);
        const double cv = ZC ? wv + we + sv + sn + bv + bt : ldc<NT>(C + v);
        if (diag) *diag = cv;
        return cv * x[v] - wv * x[xw] - we * x[xe] - sv * x[ys] - sn * x[yn] - bv * x[zb] - bt * x[zt];
    } else {
        double s = ldc<NT>(st + v) * x[v];
#define HB3_PAIR(o, dx, dy, dz)                                                                      \
    {                                                                                                \
        const long long qm = nbr<O, dx, dy, dz>(g, t), qp = nbr<O, -(dx), -(dy), -(dz)>(g, t);      \
        s -= ldc<NT>(st + (1 + o) * F + v) * x[qm];                                                  \
        s -= ldc<NT>(st + (1 + o) * F + qp) * x[qp];                                                 \
    }
        HB3_PAIR(0, -1, -1, -1) HB3_PAIR(1, 0, -1, -1) HB3_PAIR(2, 1, -1, -1)
        HB3_PAIR(3, -1, 0, -1) HB3_PAIR(4, 0, 0, -1) HB3_PAIR(5, 1, 0, -1)
        HB3_PAIR(6, -1, 1, -1) HB3_PAIR(7, 0, 1, -1) HB3_PAIR(8, 1, 1, -1)
        HB3_PAIR(9, -1, -1, 0) HB3_PAIR(10, 0, -1, 0) HB3_PAIR(11, 1, -1, 0)
        HB3_PAIR(12, -1, 0, 0)
#undef HB3_PAIR
        return s;
    }
}

template <int O>
__device__ __forceinline__ bool thread_vertex(const Oct &g, long long t, int &i, int &j, int &k)
{
    int a, b, c;
    sub_coords(g, t, a, b, c);
    i = 2 * a + (O & 1);
    j = 2 * b + ((O >> 1) & 1);
    k = 2 * c + (O >> 2);
    return a < g.mx && inner(g, i, j, k);
}

// x_p += (b_p - (A x)_p) / A_pp at vertex t of octant O
template <int NPT, int O, bool ZC = false>
__device__ __forceinline__ void gs_point(const LArgs &a, long long t)
{
    int i, j, k;
    if (!thread_vertex<O>(a.g, t, i, j, k)) return;
    const long long v = O * a.g.oct + t;
    if (ZC && NPT == 7) {
        double d;
        const double s = apply_at<NPT, O, true, true>(a.g, a.st, a.x, t, &d);
        a.x[v] += (a.b[v] - s) / d;
        return;
    }
    const double s = apply_at<NPT, O, true>(a.g, a.st, a.x, t);
    a.x[v] += (a.b[v] - s) / a.st[v];
}

// one colour of the relaxation on octant O.  On the coarse levels a launch
// holds a wave or less per SIMD; a four-wave occupancy target leaves the
// registers to issue every load of a 27-point row before the first use (at
// the default target they go out in three or four dependent batches)
template <int NPT, int O>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void k3_gs(LArgs a)
{
    const long long t = xcd_block(blockIdx.x, gridDim.x) * 256LL + threadIdx.x;
    if (t >= a.g.oct) return;
    gs_point<NPT, O>(a, t);
}

// 7-point operators: a colour couples only to the three colours that differ
// from it in one index parity, so colours 1, 2, 4 do not couple to each other,
// nor do 3, 5, 6.  Running {0}, {1,2,4}, {3,5,6}, {7} as four launches updates
// every vertex from the same values as the colour order 0..7 (bitwise the
// same sweep), and one thread's three vertices share their neighbours' loads.
template <int G, bool ZC = false>
__global__ __launch_bounds__(256) void k3_gs7g(LArgs a)
{
    const long long t = xcd_block(blockIdx.x, gridDim.x) * 256LL + threadIdx.x;
    if (t >= a.g.oct) return;
    if (G == 0) {
        gs_point<7, 0, ZC>(a, t);
    } else if (G == 1) {
        gs_point<7, 1, ZC>(a, t);
        gs_point<7, 2, ZC>(a, t);
        gs_point<7, 4, ZC>(a, t);
    } else if (G == 2) {
        gs_point<7, 3, ZC>(a, t);
        gs_point<7, 5, ZC>(a, t);
        gs_point<7, 6, ZC>(a, t);
    } else {
        gs_point<7, 7, ZC>(a, t);
    }
}

// residual r = b - A x (STORE) and/or block sums of r^2 (NORM); blockIdx.y = octant
template <int NPT, int O, bool STORE, bool NORM, bool ZC = false>
__device__ __forceinline__ double resid_at(const LArgs &a, long long t)
{
    int i, j, k;
    if (!thread_vertex<O>(a.g, t, i, j, k)) {
        if (STORE) a.r[O * a.g.oct + t] = 0.0;
        return 0.0;
    }
    const long long v = O * a.g.oct + t;
    const double r = a.b[v] - apply_at<NPT, O, false, ZC>(a.g, a.st, a.x, t);
    if (STORE) a.r[v] = r;
    return NORM ? r * r : 0.0;
}

// blocks interleave the octants (octant = block mod 8), so that the eight
// octants of one region run together and share their neighbours in L2
template <int NPT, bool STORE, bool NORM, bool ZC = false>
__global__ __launch_bounds__(256) void k3_resid(LArgs a)
{
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const long long t = (lb >> 3) * 256LL + threadIdx.x;
    double sq = 0.0;
    if (t < a.g.oct) {
        switch (lb & 7) {
        case 0: sq = resid_at<NPT, 0, STORE, NORM, ZC>(a, t); break;
        case 1: sq = resid_at<NPT, 1, STORE, NORM, ZC>(a, t); break;
        case 2: sq = resid_at<NPT, 2, STORE, NORM, ZC>(a, t); break;
        case 3: sq = resid_at<NPT, 3, STORE, NORM, ZC>(a, t); break;
        case 4: sq = resid_at<NPT, 4, STORE, NORM, ZC>(a, t); break;
        case 5: sq = resid_at<NPT, 5, STORE, NORM, ZC>(a, t); break;
        case 6: sq = resid_at<NPT, 6, STORE, NORM, ZC>(a, t); break;
        default: sq = resid_at<NPT, 7, STORE, NORM, ZC>(a, t); break;
        }
    }
    if (NORM) {
        for (int off = 32; off >= 1; off >>= 1) sq += __shfl_xor(sq, off, 64);
        __shared__ double ws[4];
        if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = sq;
        __syncthreads();
        if (threadIdx.x == 0) a.partials[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
    }
}

// ZC check of a 7-point level: clears *flag unless every interior vertex's
// diagonal is bitwise W_p + W_e + S_p + S_n + B_p + B_t (finite volumes of
// pure diffusion build it so); blocks interleave the octants
template <int O>
__device__ __forceinline__ bool zexc7_at(const Oct &g, const double *st, long long t)
{
    int i, j, k;
    if (!thread_vertex<O>(g, t, i, j, k)) return true;
    const long long F = g.field, v = O * g.oct + t;
    const double *C = st, *W = st + F, *S = st + 2 * F, *B = st + 3 * F;
    const long long xe = nbr<O, 1, 0, 0>(g, t), yn = nbr<O, 0, 1, 0>(g, t), zt = nbr<O, 0, 0, 1>(g, t);
    return C[v] == W[v] + W[xe] + S[v] + S[yn] + B[v] + B[zt];
}

__global__ __launch_bounds__(256) void k3_zero_excess7(Oct g, const double *st, int *flag)
{
    const unsigned lb = blockIdx.x;
    const long long t = (lb >> 3) * 256LL + threadIdx.x;
    if (t >= g.oct) return;
    bool ok = true;
    switch (lb & 7) {
    case 0: ok = zexc7_at<0>(g, st, t); break;
    case 1: ok = zexc7_at<1>(g, st, t); break;
    case 2: ok = zexc7_at<2>(g, st, t); break;
    case 3: ok = zexc7_at<3>(g, st, t); break;
    case 4: ok = zexc7_at<4>(g, st, t); break;
    case 5: ok = zexc7_at<5>(g, st, t); break;
    case 6: ok = zexc7_at<6>(g, st, t); break;
    default: ok = zexc7_at<7>(g, st, t); break;
    }
    if (!ok) atomicAnd(flag, 0);
}

__global__ void k3_set_int(int *p, int v) { *p = v; }

// sum of squares of a field's interior entries (the norm of b), block sums
__global__ __launch_bounds__(256) void k3_sumsq(Oct g, const double *f, double *partials)
{
    const long long t = blockIdx.x * 256LL + threadIdx.x;
    double sq = 0.0;
    if (t < g.field) {
        const int o = (int)(t / g.oct);
        int a, b, c;
        sub_coords(g, t % g.oct, a, b, c);
        const int i = 2 * a + (o & 1), j = 2 * b + ((o >> 1) & 1), k = 2 * c + (o >> 2);
        if (a < g.mx && inner(g, i, j, k)) sq = f[t] * f[t];
    }
    for (int off = 32; off >= 1; off >>= 1) sq += __shfl_xor(sq, off, 64);
    __shared__ double ws[4];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// zero a field (a kernel, not a memset node, so that it can sit in a captured graph)
__global__ __launch_bounds__(256) void k3_fill0(double *p, long long n)
{
    for (long long t = blockIdx.x * 256LL + threadIdx.x; t < n; t += (long long)gridDim.x * 256) p[t] = 0.0;
}

// block b: out[b] = sum of partials [b*chunk, min(n, (b+1)*chunk))
__global__ __launch_bounds__(256) void k3_reduce(const double *partials, long long n, long long chunk, double *out)
{
    double s = 0.0;
    const long long lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    for (long long t = lo + threadIdx.x; t < hi; t += 256) s += partials[t];
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    __shared__ double ws[4];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// b_c = P^T r: each coarse vertex gathers its 27 fine support vertices
__global__ __launch_bounds__(256) void k3_restrict(LArgs a)
{
    const Oct g = a.g, c = a.c;
    // blocks interleave the coarse octants: neighbouring coarse vertices,
    // which share fine support vertices, run together
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int oc = lb & 7;
    const long long ts = (lb >> 3) * 256LL + threadIdx.x;
    if (ts >= c.oct) return;
    const long long t = oc * c.oct + ts;
    int ca, cb, cc;
    sub_coords(c, ts, ca, cb, cc);
    const int I = 2 * ca + (oc & 1), J = 2 * cb + ((oc >> 1) & 1), K = 2 * cc + (oc >> 2);
    // the coarse level's iterate starts at zero (every entry, boundary included)
    a.xcz[t] = 0.0;
    if (ca >= c.mx || !inner(c, I, J, K)) {
        a.bc[t] = 0.0;
        return;
    }
    double s = 0.0;
    // unrolled, the fine octant of every support vertex is a constant and the
    // 54 loads can go out together
#pragma unroll
    for (int ez = -1; ez <= 1; ++ez)
#pragma unroll
        for (int ey = -1; ey <= 1; ++ey)
#pragma unroll
            for (int ex = -1; ex <= 1; ++ex) {
                const int pi = 2 * I + ex, pj = 2 * J + ey, pk = 2 * K + ez;
                const int mI = (ex == -1 ? 1 : 0) | (ey == -1 ? 2 : 0) | (ez == -1 ? 4 : 0);
                s += weight_on(g, a.w, pi, pj, pk, mI) * a.r[vid(g, pi, pj, pk)];
            }
    a.bc[t] = s;
}

// x += P x_c (+ r/C at vertices that are not coarse points); blockIdx.y = octant
template <int NPT, int O>
__device__ __forceinline__ void interp_at(const LArgs &a, long long t)
{
    int i, j, k;
    if (!thread_vertex<O>(a.g, t, i, j, k)) return;
    const Oct &g = a.g, &c = a.c;
    const long long v = O * g.oct + t;
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        if (m & ~O) continue;
        const double w = O == 0 ? 1.0 : a.w[(wbase(O) + wrank(O, m)) * g.oct + t];
        s += w * a.xc[vid(c, (i >> 1) + (m & 1), (j >> 1) + ((m >> 1) & 1), (k >> 1) + (m >> 2))];
    }
    double xv = a.x[v] + s;
    if (O != 0 && a.rescorr) xv += a.r[v] / a.st[v];
    a.x[v] = xv;
}

template <int NPT>
__global__ __launch_bounds__(256) void k3_interp(LArgs a)
{
    const long long t = xcd_block(blockIdx.x, gridDim.x) * 256LL + threadIdx.x;
    if (t >= a.g.oct) return;
    switch (blockIdx.y) {
    case 0: interp_at<NPT, 0>(a, t); break;
    case 1: interp_at<NPT, 1>(a, t); break;
    case 2: interp_at<NPT, 2>(a, t); break;
    case 3: interp_at<NPT, 3>(a, t); break;
    case 4: interp_at<NPT, 4>(a, t); break;
    case 5: interp_at<NPT, 5>(a, t); break;
    case 6: interp_at<NPT, 6>(a, t); break;
    default: interp_at<NPT, 7>(a, t); break;
    }
}

// ---------------------------------------------------------------------------
// collapsed levels: levels 0..top in one persistent workgroup (the one-GPU
// form of the paper's coarse-grid redistribution).  Every phase does the
// arithmetic of the grid-wide kernels in the same expression order, so the
// iteration does not depend on the collapse level.
// ---------------------------------------------------------------------------
constexpr int MAXC3 = 8;
constexpr int CWG3 = 512;

struct CLev {
    Oct g;
    int npt;
    const double *st;
    const double *w;
    double *x, *b, *r;
};

struct CArgs {
    CLev lv[MAXC3];
    int top;
    const double *chol;
    const long long *cidx;
    int nc;
    int nu1, nu2, rescorr;
};

// collapsed levels are small (the host caps l* so that every plane offset of a
// collapsed level fits in 32 bits): 32-bit index arithmetic throughout, which
// keeps the runtime-octant stencil within the workgroup's register budget
__device__ __forceinline__ int nbr_rt(const Oct &g, int o, int t, int dx, int dy, int dz)
{
    const int ox = (o & 1) + dx, oy = ((o >> 1) & 1) + dy, oz = (o >> 2) + dz;
    const int on = (ox & 1) | ((oy & 1) << 1) | ((oz & 1) << 2);
    return on * (int)g.oct + t + (oz >> 1) * (int)g.plane + (oy >> 1) * g.px + (ox >> 1);
}

// apply_at with the octant at run time (same expressions, same order)
__device__ __forceinline__ double apply_rt(const CLev &L, int o, int t)
{
    const Oct &g = L.g;
    const int F = (int)g.field;
    const int v = o * (int)g.oct + t;
    const double *st = L.st, *x = L.x;
    if (L.npt == 7) {
        const double *C = st, *W = st + F, *S = st + 2 * F, *B = st + 3 * F;
        const int xw = nbr_rt(g, o, t, -1, 0, 0), xe = nbr_rt(g, o, t, 1, 0, 0);
        const int ys = nbr_rt(g, o, t, 0, -1, 0), yn = nbr_rt(g, o, t, 0, 1, 0);
        const int zb = nbr_rt(g, o, t, 0, 0, -1), zt = nbr_rt(g, o, t, 0, 0, 1);
        const double cv = C[v], wv = W[v], we = W[xe], sv = S[v], sn = S[yn], bv = B[v], bt = B[zt];
        return cv * x[v] - wv * x[xw] - we * x[xe] - sv * x[ys] - sn * x[yn] - bv * x[zb] - bt * x[zt];
    }
    double s = st[v] * x[v];
#pragma unroll
    for (int q = 0; q < 13; ++q) {
        const int dx = q % 3 - 1, dy = (q / 3) % 3 - 1, dz = q / 9 - 1;
        const int qm = nbr_rt(g, o, t, dx, dy, dz), qp = nbr_rt(g, o, t, -dx, -dy, -dz);
        s -= st[(1 + q) * F + v] * x[qm];
        s -= st[(1 + q) * F + qp] * x[qp];
    }
    return s;
}

// collapsed levels are small (fields < 2^31 entries): 32-bit index arithmetic
__device__ __forceinline__ void sub_coords32(const Oct &g, int t, int &a, int &b, int &c)
{
    a = t % g.px;
    const int r = t / g.px;
    b = r % g.my;
    c = r / g.my;
}

__device__ __forceinline__ bool vertex_rt(const Oct &g, int o, int t, int &i, int &j, int &k)
{
    int a, b, c;
    sub_coords32(g, t, a, b, c);
    i = 2 * a + (o & 1);
    j = 2 * b + ((o >> 1) & 1);
    k = 2 * c + (o >> 2);
    return a < g.mx && inner(g, i, j, k);
}

__device__ __forceinline__ void wg_relax(const CLev &L, int sweeps)
{
    for (int it = 0; it < sweeps; ++it)
        for (int o = 0; o < 8; ++o) {
            for (int t = threadIdx.x; t < (int)L.g.oct; t += CWG3) {
                int i, j, k;
                if (!vertex_rt(L.g, o, t, i, j, k)) continue;
                const int v = o * (int)L.g.oct + t;
                const double s = apply_rt(L, o, t);
                L.x[v] += (L.b[v] - s) / L.st[v];
            }
            __syncthreads();
        }
}

__device__ __forceinline__ void wg_residual(const CLev &L)
{
    const int oct = (int)L.g.oct;
    for (int u = threadIdx.x; u < (int)L.g.field; u += CWG3) {
        const int o = u / oct;
        const int t = u - o * oct;
        int i, j, k;
        if (!vertex_rt(L.g, o, t, i, j, k)) {
            L.r[u] = 0.0;
            continue;
        }
        L.r[u] = L.b[u] - apply_rt(L, o, t);
    }
    __syncthreads();
}

__device__ __forceinline__ void wg_restrict(const CLev &F, const CLev &C)
{
    const Oct &g = F.g, &c = C.g;
    const int coct = (int)c.oct;
    for (int u = threadIdx.x; u < (int)c.field; u += CWG3) {
        const int oc = u / coct;
        int ca, cb, cc;
        sub_coords32(c, u - oc * coct, ca, cb, cc);
        const int I = 2 * ca + (oc & 1), J = 2 * cb + ((oc >> 1) & 1), K = 2 * cc + (oc >> 2);
        if (ca >= c.mx || !inner(c, I, J, K)) {
            C.b[u] = 0.0;
            continue;
        }
        double s = 0.0;
        for (int ez = -1; ez <= 1; ++ez)
            for (int ey = -1; ey <= 1; ++ey)
                for (int ex = -1; ex <= 1; ++ex) {
                    const int pi = 2 * I + ex, pj = 2 * J + ey, pk = 2 * K + ez;
                    const int mI = (ex == -1 ? 1 : 0) | (ey == -1 ? 2 : 0) | (ez == -1 ? 4 : 0);
                    s += weight_on(g, F.w, pi, pj, pk, mI) * F.r[vid(g, pi, pj, pk)];
                }
        C.b[u] = s;
    }
    // the coarse iterate starts at zero
    for (long long u = threadIdx.x; u < c.field; u += CWG3) C.x[u] = 0.0;
    __syncthreads();
}

__device__ __forceinline__ void wg_interp(const CLev &F, const CLev &C, int rescorr)
{
    const Oct &g = F.g, &c = C.g;
    const int oct = (int)g.oct;
    for (int u = threadIdx.x; u < (int)g.field; u += CWG3) {
        const int o = u / oct;
        const int t = u - o * oct;
        int i, j, k;
        if (!vertex_rt(g, o, t, i, j, k)) continue;
        double s = 0.0;
        for (int m = 0; m < 8; ++m) {
            if (m & ~o) continue;
            const double w = o == 0 ? 1.0 : F.w[(wbase(o) + wrank(o, m)) * g.oct + t];
            s += w * C.x[vid(c, (i >> 1) + (m & 1), (j >> 1) + ((m >> 1) & 1), (k >> 1) + (m >> 2))];
        }
        double xv = F.x[u] + s;
        if (o != 0 && rescorr) xv += F.r[u] / F.st[u];
        F.x[u] = xv;
    }
    __syncthreads();
}

__device__ void wg_coarse(const CArgs &a, double *y)
{
    const int n = a.nc;
    const double *Lf = a.chol;
    for (int r = threadIdx.x; r < n; r += CWG3) y[r] = a.lv[0].b[a.cidx[r]];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double yk = y[k] / Lf[(long long)k * n + k];
        __syncthreads();
        if (threadIdx.x == 0) y[k] = yk;
        for (int r = k + 1 + threadIdx.x; r < n; r += CWG3) y[r] -= Lf[(long long)r * n + k] * yk;
        __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {
        const double yk = y[k] / Lf[(long long)k * n + k];
        __syncthreads();
        if (threadIdx.x == 0) y[k] = yk;
        for (int r = threadIdx.x; r < k; r += CWG3) y[r] -= Lf[(long long)k * n + r] * yk;
        __syncthreads();
    }
    for (int r = threadIdx.x; r < n; r += CWG3) a.lv[0].x[a.cidx[r]] = y[r];
    __syncthreads();
}

// levels 0..top: down (relax, residual, restrict), the coarse solve, up
// (interpolate, relax).  The caller has set b and x of level top.  On the
// small levels only a wave or two per SIMD has work, so nothing hides memory
// latency: two waves per SIMD leave the registers to issue all 54 loads of a
// 27-point row before the first use (at the default occupancy target the
// compiler keeps two in flight, and a row costs 27 trips to L2).
__global__ __launch_bounds__(CWG3) __attribute__((amdgpu_waves_per_eu(2, 2))) void k3_collapse(CArgs a)
{
    extern __shared__ double y[];
    // levels as values (not references into the argument block), so that
    // their fields stay in scalar registers across the phase loops
    for (int l = a.top; l >= 1; --l) {
        const CLev F = a.lv[l], C = a.lv[l - 1];
        wg_relax(F, a.nu1);
        wg_residual(F);
        wg_restrict(F, C);
    }
    wg_coarse(a, y);
    for (int l = 1; l <= a.top; ++l) {
        const CLev F = a.lv[l], C = a.lv[l - 1];
        wg_interp(F, C, a.rescorr);
        wg_relax(F, a.nu2);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
hipbmg_status fail3(hipbmg_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    hbmg::set_last_error(buf);
    return st;
}

#define HIP3(call)                                                                                  \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return fail3(HIPBMG_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define ST3(call)                                                                                   \
    do {                                                                                            \
        hipbmg_status s_ = (call);                                                                  \
        if (s_ != HIPBMG_OK) return s_;                                                             \
    } while (0)

inline unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

struct Lev3 {
    Oct g;
    int npt = 27;
    int zc = 0;             // 7-point: the diagonal is formed from the connections
    double *st = nullptr;   // npt == 7: 4 fields; 27: 14 fields
    double *w = nullptr;    // NWSLOT octant slots: weights onto the next coarser level
    double *x = nullptr, *b = nullptr, *r = nullptr;
};

constexpr int NPROF3 = 5;

}  // namespace

struct hipbmg3d_hier {
    int L = 0;
    int lstar = 0;                      // levels 0..lstar run in one workgroup
    double model_us[HIPBMG_MAX_LEVELS] = {0};
    Lev3 lv[HIPBMG_MAX_LEVELS];
    hipbmg_params prm;
    int nc = 0;
    double *d_chol = nullptr;
    long long *d_cidx = nullptr;
    double *d_part = nullptr;
    long long npart = 0;
    double *d_sum = nullptr;
    double *h_sum = nullptr;   // pinned
    double *d_nat = nullptr;   // plain-layout staging of the op_* entry points
    std::vector<void *> allocs;
    hipGraph_t graph = nullptr;        // one V-cycle and the residual norm, captured
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;         // the stream the graph is captured on (the caller's may be the null stream)
    int prof = 0;
    std::vector<hipEvent_t> evpool;
    struct ProfMark {
        int k;
        double bytes;
        hipEvent_t e0, e1;
    };
    std::vector<ProfMark> marks;
    double prof_ms[NPROF3] = {0};
    long long prof_n[NPROF3] = {0};
    double prof_b[NPROF3] = {0};   // algorithmic bytes of the launches timed
};

namespace {

hipbmg_status dalloc3(hipbmg3d_hier *h, double **p, long long n)
{
    void *q = nullptr;
    if (hbmg::dev_malloc(&q, (size_t)n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return fail3(HIPBMG_ENOMEM, "device allocation of %lld doubles failed", n);
    }
    h->allocs.push_back(q);
    *p = (double *)q;
    HIP3(hipMemset(q, 0, (size_t)n * sizeof(double)));
    return HIPBMG_OK;
}

void free3(hipbmg3d_hier *h)
{
    hbmg::dev_free_all(h->allocs);
    if (h->h_sum) {
        (void)hipDeviceSynchronize();
        hbmg::pinned_small_free(h->h_sum);
    }
    for (hipEvent_t e : h->evpool) (void)hipEventDestroy(e);
    if (h->exec) (void)hipGraphExecDestroy(h->exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    delete h;
}

// kernel-class timing: an event pair around launches of class k, which
// move `bytes` algorithmic bytes
struct Mark {
    hipbmg3d_hier *h;
    int k;
    hipStream_t s;
    hipEvent_t e1 = nullptr;
    Mark(hipbmg3d_hier *h_, int k_, hipStream_t s_, double bytes = 0.0) : h(h_), k(k_), s(s_)
    {
        if (!h->prof) return;
        const size_t need = 2 * (h->marks.size() + 1);
        while (h->evpool.size() < need) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) {
                (void)hipGetLastError();
                h->prof = 0;
                return;
            }
            h->evpool.push_back(e);
        }
        hipEvent_t e0 = h->evpool[2 * h->marks.size()];
        e1 = h->evpool[2 * h->marks.size() + 1];
        (void)hipEventRecord(e0, s);
        h->marks.push_back({k, bytes, e0, e1});
    }
    ~Mark()
    {
        if (e1) (void)hipEventRecord(e1, s);
    }
};

hipbmg_status prof_collect(hipbmg3d_hier *h)
{
    for (auto &m : h->marks) {
        float ms = 0.f;
        HIP3(hipEventSynchronize(m.e1));
        HIP3(hipEventElapsedTime(&ms, m.e0, m.e1));
        h->prof_ms[m.k] += ms;
        h->prof_n[m.k] += 1;
        h->prof_b[m.k] += m.bytes;
    }
    h->marks.clear();
    return HIPBMG_OK;
}

// algorithmic bytes per vertex of level f's whole grid (FP64): one
// relaxation sweep or residual reads x, b and the stencil's planes (7-point:
// C, W, S, B, or W, S, B with the diagonal formed; 27-point: 14) and writes
// x or r (the norm-only residual writes nothing)
double sweep_bytes_per_vertex(const Lev3 &f)
{
    const double planes = f.npt == 7 ? (f.zc ? 3.0 : 4.0) : 14.0;
    return 8.0 * (3.0 + planes);
}

double grid_vertices(const Lev3 &f) { return (double)f.g.nx * f.g.ny * f.g.nz; }

LArgs largs(const Lev3 &f, const Lev3 *c)
{
    LArgs a{};
    a.g = f.g;
    a.st = f.st;
    a.b = f.b;
    a.x = f.x;
    a.r = f.r;
    a.w = f.w;
    a.zc = f.zc;
    if (c) {
        a.c = c->g;
        a.xc = c->x;
        a.bc = c->b;
    }
    return a;
}

// one colour of a 27-point level (7-point levels run the colour groups)
hipError_t launch_gs_colour27(int o, const LArgs &a, hipStream_t s)
{
    const dim3 grid(round8(nblk(a.g.oct))), block(256);
#define HB3_GS(O) hipLaunchKernelGGL((k3_gs<27, O>), grid, block, 0, s, a)
    switch (o) {
    case 0: HB3_GS(0); break;
    case 1: HB3_GS(1); break;
    case 2: HB3_GS(2); break;
    case 3: HB3_GS(3); break;
    case 4: HB3_GS(4); break;
    case 5: HB3_GS(5); break;
    case 6: HB3_GS(6); break;
    default: HB3_GS(7); break;
    }
#undef HB3_GS
    return hipGetLastError();
}

hipbmg_status relax(hipbmg3d_hier *h, int l, int sweeps, hipStream_t s)
{
    const Lev3 &f = h->lv[l];
    const LArgs a = largs(f, nullptr);
    const dim3 grid(round8(nblk(f.g.oct))), block(256);
    for (int it = 0; it < sweeps; ++it) {
        if (f.npt == 7) {
            for (int gq = 0; gq < 4; ++gq) {
                // colour groups {0}, {1,2,4}, {3,5,6}, {7}: 1/8, 3/8, 3/8, 1/8 of the vertices
                Mark mk(h, l == h->L - 1 ? 0 : 4, s,
                        sweep_bytes_per_vertex(f) * grid_vertices(f) * ((gq == 0 || gq == 3) ? 0.125 : 0.375));
                if (f.zc) {
                    if (gq == 0) hipLaunchKernelGGL((k3_gs7g<0, true>), grid, block, 0, s, a);
                    else if (gq == 1) hipLaunchKernelGGL((k3_gs7g<1, true>), grid, block, 0, s, a);
                    else if (gq == 2) hipLaunchKernelGGL((k3_gs7g<2, true>), grid, block, 0, s, a);
                    else hipLaunchKernelGGL((k3_gs7g<3, true>), grid, block, 0, s, a);
                } else {
                    if (gq == 0) hipLaunchKernelGGL(k3_gs7g<0>, grid, block, 0, s, a);
                    else if (gq == 1) hipLaunchKernelGGL(k3_gs7g<1>, grid, block, 0, s, a);
                    else if (gq == 2) hipLaunchKernelGGL(k3_gs7g<2>, grid, block, 0, s, a);
                    else hipLaunchKernelGGL(k3_gs7g<3>, grid, block, 0, s, a);
                }
                HIP3(hipGetLastError());
            }
            continue;
        }
        for (int o = 0; o < 8; ++o) {
            Mark mk(h, l == h->L - 1 ? 0 : 4, s, sweep_bytes_per_vertex(f) * grid_vertices(f) * 0.125);
            HIP3(launch_gs_colour27(o, a, s));
        }
    }
    return HIPBMG_OK;
}

// d_sum[0] = sum of n partials, in two stages of fixed shape (deterministic)
hipbmg_status reduce_sum(hipbmg3d_hier *h, const double *partials, long long n, hipStream_t s)
{
    const long long nb = std::min<long long>(256, (n + 2047) / 2048);
    const long long chunk = (n + nb - 1) / nb;
    hipLaunchKernelGGL(k3_reduce, dim3((unsigned)nb), dim3(256), 0, s, partials, n, chunk, h->d_sum + 8);
    hipLaunchKernelGGL(k3_reduce, dim3(1), dim3(256), 0, s, (const double *)(h->d_sum + 8), nb, nb, h->d_sum);
    HIP3(hipGetLastError());
    return HIPBMG_OK;
}

// residual of level l: store r (store), or only the squared norm's block
// sums and their sum in d_sum[0] (norm)
hipbmg_status residual(hipbmg3d_hier *h, int l, bool store, bool norm, hipStream_t s)
{
    if (store == norm) return fail3(HIPBMG_EINVAL, "residual: store or norm, not both");
    const Lev3 &f = h->lv[l];
    LArgs a = largs(f, nullptr);
    a.partials = h->d_part;
    const dim3 grid(8 * nblk(f.g.oct)), block(256);   // a multiple of 8, octants interleaved
    Mark mk(h, l == h->L - 1 ? 1 : 4, s, (sweep_bytes_per_vertex(f) - (store ? 0.0 : 8.0)) * grid_vertices(f));
    if (f.npt == 7 && f.zc) {
        if (store) hipLaunchKernelGGL((k3_resid<7, true, false, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k3_resid<7, false, true, true>), grid, block, 0, s, a);
    } else if (f.npt == 7) {
        if (store) hipLaunchKernelGGL((k3_resid<7, true, false>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k3_resid<7, false, true>), grid, block, 0, s, a);
    } else {
        if (store) hipLaunchKernelGGL((k3_resid<27, true, false>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k3_resid<27, false, true>), grid, block, 0, s, a);
    }
    HIP3(hipGetLastError());
    if (norm) ST3(reduce_sum(h, h->d_part, (long long)grid.x, s));
    return HIPBMG_OK;
}

// b_{l-1} = P^T r_l, and x_{l-1} = 0
hipbmg_status restrict_to(hipbmg3d_hier *h, int l, hipStream_t s)
{
    LArgs a = largs(h->lv[l], &h->lv[l - 1]);
    a.xcz = h->lv[l - 1].x;
    // reads r and the 26 weights per coarse cell (3.25 per fine vertex),
    // writes the coarse right-hand side and the zero coarse iterate
    Mark mk(h, l == h->L - 1 ? 2 : 4, s, 8.0 * (1.0 + 3.25 + 0.25) * grid_vertices(h->lv[l]));
    hipLaunchKernelGGL(k3_restrict, dim3(8 * nblk(a.c.oct)), dim3(256), 0, s, a);
    HIP3(hipGetLastError());
    return HIPBMG_OK;
}

hipbmg_status interp_from(hipbmg3d_hier *h, int l, int rescorr, hipStream_t s)
{
    const Lev3 &f = h->lv[l];
    LArgs a = largs(f, &h->lv[l - 1]);
    a.rescorr = rescorr;
    const dim3 grid(round8(nblk(f.g.oct)), 8), block(256);
    // reads and writes x, reads r, C, the weights and the coarse iterate
    Mark mk(h, l == h->L - 1 ? 3 : 4, s, 8.0 * (2.0 + 1.0 + 1.0 + 3.25 + 0.125) * grid_vertices(f));
    if (f.npt == 7) hipLaunchKernelGGL((k3_interp<7>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k3_interp<27>), grid, block, 0, s, a);
    HIP3(hipGetLastError());
    return HIPBMG_OK;
}

// levels 0..top in one workgroup (top = 0: the coarse solve alone)
hipbmg_status collapse(hipbmg3d_hier *h, int top, hipStream_t s)
{
    CArgs a{};
    for (int l = 0; l <= top; ++l) {
        const Lev3 &v = h->lv[l];
        a.lv[l] = CLev{v.g, v.npt, v.st, v.w, v.x, v.b, v.r};
    }
    a.top = top;
    a.chol = h->d_chol;
    a.cidx = h->d_cidx;
    a.nc = h->nc;
    a.nu1 = h->prm.nu1;
    a.nu2 = h->prm.nu2;
    a.rescorr = h->prm.residual_correction;
    Mark mk(h, 4, s);
    hipLaunchKernelGGL(k3_collapse, dim3(1), dim3(CWG3), (size_t)std::max(h->nc, 1) * sizeof(double), s, a);
    HIP3(hipGetLastError());
    return HIPBMG_OK;
}

// Algorithm 1 on level l: x_l and b_l are the level's own fields
hipbmg_status vcycle(hipbmg3d_hier *h, int l, hipStream_t s)
{
    if (l <= h->lstar) return collapse(h, l, s);
    ST3(relax(h, l, h->prm.nu1, s));
    ST3(residual(h, l, true, false, s));
    ST3(restrict_to(h, l, s));
    ST3(vcycle(h, l - 1, s));
    ST3(interp_from(h, l, h->prm.residual_correction, s));
    ST3(relax(h, l, h->prm.nu2, s));
    return HIPBMG_OK;
}

// one cycle and the finest residual norm (into d_sum); replayed from a
// captured graph unless use_graph is 0 or kernel timing is on
hipbmg_status cycle_and_norm(hipbmg3d_hier *h, hipStream_t s)
{
    if (!h->prm.use_graph || h->prof) {
        ST3(vcycle(h, h->L - 1, s));
        return residual(h, h->L - 1, false, true, s);
    }
    if (!h->exec) {
        if (!h->cap) HIP3(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
        hipStream_t c = h->cap;
        HIP3(hipStreamBeginCapture(c, hipStreamCaptureModeThreadLocal));
        hipbmg_status st = vcycle(h, h->L - 1, c);
        if (st == HIPBMG_OK) st = residual(h, h->L - 1, false, true, c);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(c, &g);
        if (st != HIPBMG_OK || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return st != HIPBMG_OK ? st : fail3(HIPBMG_EHIP, "graph capture failed: %s", hipGetErrorString(e2));
        }
        h->graph = g;
        HIP3(hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0));
    }
    HIP3(hipGraphLaunch(h->exec, s));
    return HIPBMG_OK;
}

hipbmg_status read_sum(hipbmg3d_hier *h, hipStream_t s, double *out)
{
    HIP3(hipMemcpyAsync(h->h_sum, h->d_sum, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP3(hipStreamSynchronize(s));
    *out = h->h_sum[0];
    return HIPBMG_OK;
}

hipbmg_status to_oct(const Oct &g, const double *nat, double *out, int interior_only, hipStream_t s)
{
    hipLaunchKernelGGL(k3_to_oct, dim3(nblk((long long)g.nx * g.ny * g.nz)), dim3(256), 0, s, nat, out, g,
                       interior_only);
    HIP3(hipGetLastError());
    return HIPBMG_OK;
}

hipbmg_status from_oct(const Oct &g, const double *in, double *nat, hipStream_t s)
{
    hipLaunchKernelGGL(k3_from_oct, dim3(nblk((long long)g.nx * g.ny * g.nz)), dim3(256), 0, s, in, nat, g);
    HIP3(hipGetLastError());
    return HIPBMG_OK;
}

// host copy of A(p, p+d) for the coarsest assembly
void host_entries(const std::vector<double> &st, int npt, const Oct &g, int i, int j, int k, double e[27])
{
    const long long v = vid(g, i, j, k), F = g.field;
    for (int o = 0; o < 27; ++o) e[o] = 0.0;
    e[13] = st[v];
    if (npt == 7) {
        e[12] = -st[F + v];
        e[14] = -st[F + vid(g, i + 1, j, k)];
        e[10] = -st[2 * F + v];
        e[16] = -st[2 * F + vid(g, i, j + 1, k)];
        e[4] = -st[3 * F + v];
        e[22] = -st[3 * F + vid(g, i, j, k + 1)];
    } else {
        for (int o = 0; o < 13; ++o) {
            const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
            e[o] = -st[(1 + o) * F + v];
            e[26 - o] = -st[(1 + o) * F + vid(g, i - dx, j - dy, k - dz)];
        }
    }
}

constexpr int MAX_COARSE3 = 4096;

hipbmg_status factor_coarsest(hipbmg3d_hier *h, hipStream_t s)
{
    const Lev3 &c = h->lv[0];
    const Oct &g = c.g;
    const int nf = c.npt == 7 ? 4 : 14;
    std::vector<double> st((size_t)nf * g.field);
    HIP3(hipMemcpyAsync(st.data(), c.st, st.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP3(hipStreamSynchronize(s));
    std::vector<long long> cidx;
    std::vector<int> num((size_t)g.nx * g.ny * g.nz, -1);
    for (int k = 1; k <= g.nz - 2; ++k)
        for (int j = 1; j <= g.ny - 2; ++j)
            for (int i = 1; i <= g.nx - 2; ++i) {
                num[((size_t)k * g.ny + j) * g.nx + i] = (int)cidx.size();
                cidx.push_back(vid(g, i, j, k));
            }
    const int n = (int)cidx.size();
    if (n > MAX_COARSE3) return fail3(HIPBMG_EINVAL, "coarsest level has %d unknowns (at most %d)", n, MAX_COARSE3);
    std::vector<double> M((size_t)n * n, 0.0);
    for (int k = 1; k <= g.nz - 2; ++k)
        for (int j = 1; j <= g.ny - 2; ++j)
            for (int i = 1; i <= g.nx - 2; ++i) {
                double e[27];
                host_entries(st, c.npt, g, i, j, k, e);
                const int row = num[((size_t)k * g.ny + j) * g.nx + i];
                for (int o = 0; o < 27; ++o) {
                    const int qi = i + o % 3 - 1, qj = j + (o / 3) % 3 - 1, qk = k + o / 9 - 1;
                    if (!inner(g, qi, qj, qk)) continue;
                    M[(size_t)row * n + num[((size_t)qk * g.ny + qj) * g.nx + qi]] = e[o];
                }
            }
    for (int k = 0; k < n; ++k) {
        double d = M[(size_t)k * n + k];
        for (int m = 0; m < k; ++m) d -= M[(size_t)k * n + m] * M[(size_t)k * n + m];
        if (!(d > 0.0)) return fail3(HIPBMG_ENOTSPD, "coarsest operator not positive definite (pivot %d)", k);
        d = std::sqrt(d);
        M[(size_t)k * n + k] = d;
        for (int r = k + 1; r < n; ++r) {
            double v = M[(size_t)r * n + k];
            for (int m = 0; m < k; ++m) v -= M[(size_t)r * n + m] * M[(size_t)k * n + m];
            M[(size_t)r * n + k] = v / d;
        }
    }
    h->nc = n;
    ST3(dalloc3(h, &h->d_chol, std::max((long long)n * n, 1LL)));
    double *ci = nullptr;
    ST3(dalloc3(h, &ci, std::max(n, 1)));
    h->d_cidx = (long long *)ci;
    if (n > 0) {
        HIP3(hipMemcpyAsync(h->d_chol, M.data(), M.size() * sizeof(double), hipMemcpyHostToDevice, s));
        HIP3(hipMemcpyAsync(h->d_cidx, cidx.data(), cidx.size() * sizeof(long long), hipMemcpyHostToDevice, s));
        HIP3(hipStreamSynchronize(s));
    }
    return HIPBMG_OK;
}

bool odd_ok(int n) { return n >= 3 && (n & 1); }

// mean time (ms) of `reps` repetitions of f on stream s, after one warm-up
template <typename Fn>
hipbmg_status time_ms(hipStream_t s, int reps, Fn f, double *ms)
{
    hipEvent_t e0, e1;
    ST3(f());
    HIP3(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail3(HIPBMG_EHIP, "hipEventCreate failed");
    }
    hipbmg_status st = HIPBMG_OK;
    if (hipEventRecord(e0, s) != hipSuccess) st = fail3(HIPBMG_EHIP, "hipEventRecord failed");
    for (int r = 0; r < reps && st == HIPBMG_OK; ++r) st = f();
    float t = 0.f;
    if (st == HIPBMG_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        st = fail3(HIPBMG_EHIP, "event timing failed");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = t / reps;
    return st;
}

// The model's choice of l*.  For the levels up to 9^3-ish (l <= 3) both of a
// level's terms are measured: its cost inside the workgroup as the growth of
// the collapse launch from top = l-1 to top = l, and its grid-wide cost as one
// eager visit of level l on top of the collapse of levels 0..l-1 minus that
// collapse.  Larger levels take the model's formulas.  The levels hold zeros
// while this runs, which the solve overwrites.
hipbmg_status choose_collapse(hipbmg3d_hier *h, const hbmg::ModelLevel3 *ml, int lcap, hipStream_t s)
{
    const int L = h->L;
    double t_us[HIPBMG_MAX_LEVELS];
    hbmg::model3_choose(ml, L, h->prm.nu1, h->prm.nu2, h->nc, hbmg::model_params(), lcap, t_us);
    const int m = std::min(3, lcap);
    double tc[4] = {0}, tw[4] = {0}, tg[4] = {0};
    for (int top = 0; top <= m; ++top)
        ST3(time_ms(s, 5, [&]() { return collapse(h, top, s); }, &tc[top]));
    for (int l = 1; l <= m; ++l) {
        double t = 0.0;
        h->lstar = l - 1;
        const hipbmg_status st = time_ms(s, 5, [&]() { return vcycle(h, l, s); }, &t);
        h->lstar = 0;
        ST3(st);
        tw[l] = 1e3 * (tc[l] - tc[l - 1]);
        tg[l] = 1e3 * t - 1e3 * tc[l - 1];
    }
    int best = 0;
    for (int ls = 0; ls <= lcap; ++ls) {
        const hbmg::ModelParams &mp = hbmg::model_params();
        double t = 1e3 * tc[0];
        if (ls <= m) {
            for (int l = 1; l < L; ++l) {
                if (l <= m) t += l <= ls ? tw[l] : tg[l];
                else t += hbmg::model3_grid_level_us(ml[l], h->prm.nu1, h->prm.nu2, mp);
            }
        } else {
            // the model's path with its base and its small-level terms replaced by the measured ones
            t += t_us[ls] - hbmg::model_base_us(h->nc, 8, mp);
            for (int l = 1; l <= m; ++l) t += tw[l] - hbmg::model3_wg_level_us(ml[l], h->prm.nu1, h->prm.nu2, mp);
        }
        h->model_us[ls] = t;
        if (t < h->model_us[best]) best = ls;
    }
    h->lstar = best;
    return HIPBMG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C interface
// ---------------------------------------------------------------------------
extern "C" hipbmg_status hipbmg3d_fv7_from_cells(int nx, int ny, int nz, const double *cell, double *planes_out,
                                                 void *stream)
{
    if (!cell || !planes_out) return fail3(HIPBMG_EINVAL, "null argument");
    if (nx < 3 || ny < 3 || nz < 3) return fail3(HIPBMG_EINVAL, "grid too small");
    hipStream_t s = (hipStream_t)stream;
    const long long n = (long long)nx * ny * nz;
    hipLaunchKernelGGL(k3_fv7, dim3(nblk(n)), dim3(256), 0, s, cell, nx, ny, nz, planes_out);
    HIP3(hipGetLastError());
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg3d_setup(int nx, int ny, int nz, int npt, const double *planes,
                                        const hipbmg_params *params, void *stream, hipbmg3d_handle *out)
{
    if (!out || !planes) return fail3(HIPBMG_EINVAL, "null argument");
    *out = nullptr;
    if (!odd_ok(nx) || !odd_ok(ny) || !odd_ok(nz)) return fail3(HIPBMG_EINVAL, "sizes must be odd and >= 3");
    if (npt != 7 && npt != 27) return fail3(HIPBMG_EINVAL, "npt must be 7 or 27");
    hipbmg_params prm;
    hipbmg_default_params(&prm);
    if (params) prm = *params;
    if (prm.nu1 < 0 || prm.nu2 < 0 || prm.nu1 + prm.nu2 < 1 || prm.coarsest_n < 3 || prm.max_cycles < 1 ||
        prm.max_cycles > HIPBMG_MAX_HIST)
        return fail3(HIPBMG_EINVAL, "bad parameters");
    if (prm.precision != HIPBMG_FP64) return fail3(HIPBMG_EINVAL, "the 3D path runs in FP64 only");
    hipStream_t s = (hipStream_t)stream;

    int sx[HIPBMG_MAX_LEVELS], sy[HIPBMG_MAX_LEVELS], sz[HIPBMG_MAX_LEVELS], L = 1;
    sx[0] = nx;
    sy[0] = ny;
    sz[0] = nz;
    while (sx[L - 1] > prm.coarsest_n && sy[L - 1] > prm.coarsest_n && sz[L - 1] > prm.coarsest_n &&
           (sx[L - 1] & 1) && (sy[L - 1] & 1) && (sz[L - 1] & 1) && L < HIPBMG_MAX_LEVELS) {
        sx[L] = (sx[L - 1] + 1) / 2;
        sy[L] = (sy[L - 1] + 1) / 2;
        sz[L] = (sz[L - 1] + 1) / 2;
        ++L;
    }
    {
        const Oct g0 = make_oct(sx[L - 1], sy[L - 1], sz[L - 1]);
        const long long nc = (long long)(g0.nx - 2) * (g0.ny - 2) * (g0.nz - 2);
        if (nc > MAX_COARSE3)
            return fail3(HIPBMG_EINVAL, "coarsest level %dx%dx%d has %lld unknowns (at most %d)", g0.nx, g0.ny,
                         g0.nz, nc, MAX_COARSE3);
    }
    auto t0 = std::chrono::steady_clock::now();
    hipbmg3d_hier *h = new hipbmg3d_hier();
    h->L = L;
    h->prm = prm;
    auto bail = [&](hipbmg_status st) {
        free3(h);
        return st;
    };
    hipbmg_status st;
    for (int l = 0; l < L; ++l) {
        Lev3 &v = h->lv[l];
        v.g = make_oct(sx[L - 1 - l], sy[L - 1 - l], sz[L - 1 - l]);
        v.npt = (l == L - 1) ? npt : 27;
        const int nf = v.npt == 7 ? 4 : 14;
        if ((st = dalloc3(h, &v.st, nf * v.g.field)) != HIPBMG_OK) return bail(st);
        if ((st = dalloc3(h, &v.x, v.g.field)) != HIPBMG_OK) return bail(st);
        if ((st = dalloc3(h, &v.b, v.g.field)) != HIPBMG_OK) return bail(st);
        if ((st = dalloc3(h, &v.r, v.g.field)) != HIPBMG_OK) return bail(st);
        if (l >= 1 && (st = dalloc3(h, &v.w, NWSLOT * v.g.oct)) != HIPBMG_OK) return bail(st);
    }
    const Lev3 &top = h->lv[L - 1];
    const long long nnat = (long long)nx * ny * nz;
    if ((st = dalloc3(h, &h->d_nat, nnat)) != HIPBMG_OK) return bail(st);
    h->npart = 8 * (long long)nblk(top.g.oct) + 8;
    if ((st = dalloc3(h, &h->d_part, h->npart)) != HIPBMG_OK) return bail(st);
    if ((st = dalloc3(h, &h->d_sum, 8 + 256)) != HIPBMG_OK) return bail(st);
    if (hbmg::pinned_small((void **)&h->h_sum, nullptr, 8 * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return bail(fail3(HIPBMG_ENOMEM, "pinned allocation failed"));
    }
    // the finest operator in the octant layout
    const int nf = npt == 7 ? 4 : 14;
    for (int q = 0; q < nf; ++q)
        if ((st = to_oct(top.g, planes + q * nnat, top.st + q * top.g.field, 0, s)) != HIPBMG_OK) return bail(st);
    // a 7-point finest operator whose diagonal is the sum of its six
    // connections (finite volumes of pure diffusion): its relaxation and
    // residual kernels form the diagonal instead of loading it
    // (HIPBMG_NO_ZEXC=1: always load)
    if (npt == 7) {
        int noz = 0;
        if (const char *e = std::getenv("HIPBMG_NO_ZEXC")) noz = std::atoi(e);
        if (!noz) {
            int ok = 0;
            double *dflag = nullptr;   // one double of device memory holds the int flag
            if ((st = dalloc3(h, &dflag, 1)) != HIPBMG_OK) return bail(st);
            int *d_flag = reinterpret_cast<int *>(dflag);
            hipLaunchKernelGGL(k3_set_int, dim3(1), dim3(1), 0, s, d_flag, 1);
            hipLaunchKernelGGL(k3_zero_excess7, dim3(8 * nblk(top.g.oct)), dim3(256), 0, s, top.g,
                               (const double *)top.st, d_flag);
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(&ok, d_flag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return bail(fail3(HIPBMG_EHIP, "zero-excess check failed"));
            h->lv[L - 1].zc = ok;
        }
    }
    // interpolation and Galerkin products, finest to coarsest
    for (int l = L - 1; l >= 1; --l) {
        Lev3 &f = h->lv[l], &c = h->lv[l - 1];
        WArgs wa{Sten{f.st, f.npt, f.g}, f.w, c.g};
        hipLaunchKernelGGL(k3_weights<1>, dim3(nblk(f.g.oct), 3), dim3(256), 0, s, wa);
        hipLaunchKernelGGL(k3_weights<2>, dim3(nblk(f.g.oct), 3), dim3(256), 0, s, wa);
        hipLaunchKernelGGL(k3_weights<3>, dim3(nblk(f.g.oct), 1), dim3(256), 0, s, wa);
        RArgs ra{Sten{f.st, f.npt, f.g}, f.w, c.g, c.st};
        hipLaunchKernelGGL(k3_rap, dim3(nblk(c.g.field)), dim3(256), 0, s, ra);
        if (hipGetLastError() != hipSuccess) return bail(fail3(HIPBMG_EHIP, "setup kernel launch failed"));
    }
    if ((st = factor_coarsest(h, s)) != HIPBMG_OK) return bail(st);
    // the collapse level: forced, or the model's argmin (section 3's model
    // with 3D counts).  Its terms for the small levels are measured here on
    // the hierarchy's own launches; larger levels use the process-wide
    // calibrated machine parameters.
    {
        int lcap = std::min(L - 1, MAXC3 - 1);
        // 32-bit indices in the workgroup: every plane offset of a collapsed level
        while (lcap > 0 && (long long)(h->lv[lcap].npt == 7 ? 4 : 14) * h->lv[lcap].g.field >= (1LL << 31)) --lcap;
        hbmg::ModelLevel3 ml[HIPBMG_MAX_LEVELS];
        for (int l = 0; l < L; ++l)
            ml[l] = hbmg::ModelLevel3{h->lv[l].g.nx, h->lv[l].g.ny, h->lv[l].g.nz, h->lv[l].npt};
        if (prm.collapse_level >= 0) {
            if (prm.collapse_level > lcap)
                return bail(fail3(HIPBMG_EINVAL, "collapse_level %d out of range (at most %d)", prm.collapse_level,
                                  lcap));
            hbmg::model3_choose(ml, L, prm.nu1, prm.nu2, h->nc, hbmg::model_params(), lcap, h->model_us);
            h->lstar = prm.collapse_level;
        } else if ((st = choose_collapse(h, ml, lcap, s)) != HIPBMG_OK) {
            return bail(st);
        }
    }
    if (hipStreamSynchronize(s) != hipSuccess) return bail(fail3(HIPBMG_EHIP, "setup failed on the device"));
    (void)t0;
    *out = h;
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg3d_destroy(hipbmg3d_handle h)
{
    if (h) free3(h);
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg3d_num_levels(hipbmg3d_handle h, int *levels_host)
{
    if (!h || !levels_host) return fail3(HIPBMG_EINVAL, "null argument");
    *levels_host = h->L;
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg3d_level_size(hipbmg3d_handle h, int l, int *nx_host, int *ny_host, int *nz_host)
{
    if (!h || !nx_host || !ny_host || !nz_host) return fail3(HIPBMG_EINVAL, "null argument");
    if (l < 0 || l >= h->L) return fail3(HIPBMG_EINVAL, "level %d out of range", l);
    *nx_host = h->lv[l].g.nx;
    *ny_host = h->lv[l].g.ny;
    *nz_host = h->lv[l].g.nz;
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg3d_get_stencil(hipbmg3d_handle h, int l, double *out, void *stream)
{
    if (!h || !out) return fail3(HIPBMG_EINVAL, "null argument");
    if (l < 0 || l >= h->L) return fail3(HIPBMG_EINVAL, "level %d out of range", l);
    const Lev3 &v = h->lv[l];
    const long long n = (long long)v.g.nx * v.g.ny * v.g.nz;
    hipLaunchKernelGGL(k3_stencil_out, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, Sten{v.st, v.npt, v.g},
                       out);
    HIP3(hipGetLastError());
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg3d_get_interp(hipbmg3d_handle h, int l, double *out, void *stream)
{
    if (!h || !out) return fail3(HIPBMG_EINVAL, "null argument");
    if (l < 1 || l >= h->L) return fail3(HIPBMG_EINVAL, "level %d has no interpolation", l);
    const Lev3 &v = h->lv[l];
    const long long n = (long long)v.g.nx * v.g.ny * v.g.nz;
    hipLaunchKernelGGL(k3_interp_out, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, v.g,
                       (const double *)v.w, out);
    HIP3(hipGetLastError());
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg3d_solve(hipbmg3d_handle h, const double *b, double *u, double tol, void *stream,
                                        hipbmg_info *info)
{
    if (!h || !b || !u) return fail3(HIPBMG_EINVAL, "null argument");
    if (!(tol >= 0.0)) return fail3(HIPBMG_EINVAL, "bad tolerance");
    hipStream_t s = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    Lev3 &f = h->lv[h->L - 1];
    ST3(to_oct(f.g, b, f.b, 1, s));
    ST3(to_oct(f.g, u, f.x, 1, s));
    hipLaunchKernelGGL(k3_sumsq, dim3(nblk(f.g.field)), dim3(256), 0, s, f.g, (const double *)f.b, h->d_part);
    HIP3(hipGetLastError());
    ST3(reduce_sum(h, h->d_part, (long long)nblk(f.g.field), s));
    double bb = 0.0;
    ST3(read_sum(h, s, &bb));
    const double bn = std::sqrt(bb);
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->levels = h->L;
        info->collapse_level = h->lstar;
        for (int l = 0; l < h->L && l < HIPBMG_MAX_LEVELS; ++l) info->model_us[l] = h->model_us[l];
    }
    hipbmg_status rc = HIPBMG_OK;
    int cycles = 0;
    double rel = 0.0;
    if (bn == 0.0) {
        HIP3(hipMemsetAsync(u, 0, (size_t)f.g.nx * f.g.ny * f.g.nz * sizeof(double), s));
        HIP3(hipStreamSynchronize(s));
    } else {
        rc = HIPBMG_ENOCONV;
        while (cycles < h->prm.max_cycles) {
            ST3(cycle_and_norm(h, s));
            double rr = 0.0;
            ST3(read_sum(h, s, &rr));
            rel = std::sqrt(rr) / bn;
            if (info) info->relres_hist[cycles] = rel;
            ++cycles;
            if (!std::isfinite(rel)) {
                rc = fail3(HIPBMG_ENAN, "residual norm is not finite after cycle %d", cycles);
                break;
            }
            if (rel <= tol) {
                rc = HIPBMG_OK;
                break;
            }
        }
        ST3(from_oct(f.g, f.x, u, s));
        HIP3(hipStreamSynchronize(s));
        if (rc == HIPBMG_ENOCONV) fail3(rc, "tolerance not reached in %d cycles", cycles);
    }
    if (h->prof) ST3(prof_collect(h));
    if (info) {
        info->cycles = cycles;
        info->outer_steps = cycles;
        info->relres = rel;
        info->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return rc;
}

extern "C" hipbmg_status hipbmg3d_op_smooth(hipbmg3d_handle h, int l, const double *b, double *x, int sweeps,
                                           void *stream)
{
    if (!h || !b || !x) return fail3(HIPBMG_EINVAL, "null argument");
    if (l < 0 || l >= h->L || sweeps < 0) return fail3(HIPBMG_EINVAL, "bad level or sweeps");
    hipStream_t s = (hipStream_t)stream;
    Lev3 &v = h->lv[l];
    ST3(to_oct(v.g, b, v.b, 1, s));
    ST3(to_oct(v.g, x, v.x, 1, s));
    ST3(relax(h, l, sweeps, s));
    ST3(from_oct(v.g, v.x, x, s));
    HIP3(hipStreamSynchronize(s));
    h->marks.clear();
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg3d_op_residual(hipbmg3d_handle h, int l, const double *b, const double *x,
                                             double *r, void *stream)
{
    if (!h || !b || !x || !r) return fail3(HIPBMG_EINVAL, "null argument");
    if (l < 0 || l >= h->L) return fail3(HIPBMG_EINVAL, "bad level");
    hipStream_t s = (hipStream_t)stream;
    Lev3 &v = h->lv[l];
    ST3(to_oct(v.g, b, v.b, 1, s));
    ST3(to_oct(v.g, x, v.x, 1, s));
    ST3(residual(h, l, true, false, s));
    ST3(from_oct(v.g, v.r, r, s));
    HIP3(hipStreamSynchronize(s));
    h->marks.clear();
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg3d_op_restrict(hipbmg3d_handle h, int l, const double *r, double *bc, void *stream)
{
    if (!h || !r || !bc) return fail3(HIPBMG_EINVAL, "null argument");
    if (l < 1 || l >= h->L) return fail3(HIPBMG_EINVAL, "bad level");
    hipStream_t s = (hipStream_t)stream;
    Lev3 &v = h->lv[l];
    ST3(to_oct(v.g, r, v.r, 1, s));
    ST3(restrict_to(h, l, s));
    ST3(from_oct(h->lv[l - 1].g, h->lv[l - 1].b, bc, s));
    HIP3(hipStreamSynchronize(s));
    h->marks.clear();
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg3d_op_interp_correct(hipbmg3d_handle h, int l, double *x, const double *r,
                                                   const double *xc, int rescorr, void *stream)
{
    if (!h || !x || !r || !xc) return fail3(HIPBMG_EINVAL, "null argument");
    if (l < 1 || l >= h->L) return fail3(HIPBMG_EINVAL, "bad level");
    hipStream_t s = (hipStream_t)stream;
    Lev3 &v = h->lv[l];
    ST3(to_oct(v.g, x, v.x, 1, s));
    ST3(to_oct(v.g, r, v.r, 1, s));
    ST3(to_oct(h->lv[l - 1].g, xc, h->lv[l - 1].x, 1, s));
    ST3(interp_from(h, l, rescorr, s));
    ST3(from_oct(v.g, v.x, x, s));
    HIP3(hipStreamSynchronize(s));
    h->marks.clear();
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg3d_op_coarse_solve(hipbmg3d_handle h, const double *b, double *x, void *stream)
{
    if (!h || !b || !x) return fail3(HIPBMG_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    Lev3 &c = h->lv[0];
    ST3(to_oct(c.g, b, c.b, 1, s));
    hipLaunchKernelGGL(k3_fill0, dim3((unsigned)std::min<long long>(nblk(c.g.field), 2048)), dim3(256), 0, s, c.x,
                       c.g.field);
    HIP3(hipGetLastError());
    ST3(collapse(h, 0, s));
    ST3(from_oct(c.g, c.x, x, s));
    HIP3(hipStreamSynchronize(s));
    h->marks.clear();
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg3d_profile(hipbmg3d_handle h, int enable)
{
    if (!h) return fail3(HIPBMG_EINVAL, "null argument");
    h->prof = enable ? 1 : 0;
    for (int k = 0; k < NPROF3; ++k) {
        h->prof_ms[k] = 0.0;
        h->prof_n[k] = 0;
        h->prof_b[k] = 0.0;
    }
    h->marks.clear();
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg3d_profile_read(hipbmg3d_handle h, int k, double *ms_host, long long *launches_host,
                                               double *bytes_per_launch_host)
{
    if (!h) return fail3(HIPBMG_EINVAL, "null argument");
    if (k < 0 || k >= NPROF3) return fail3(HIPBMG_EINVAL, "kernel class %d out of range", k);
    if (ms_host) *ms_host = h->prof_ms[k];
    if (launches_host) *launches_host = h->prof_n[k];
    if (bytes_per_launch_host) *bytes_per_launch_host = h->prof_n[k] ? h->prof_b[k] / (double)h->prof_n[k] : 0.0;
    return HIPBMG_OK;
}
