// bmg_collapse.hip -- the coarse levels collapsed into one persistent workgroup,
// plus deterministic norm reductions.
//
// The paper (sections 2.2 and 4) stops spreading coarse levels over all
// processors once their halo exchanges cost more than their work, and gathers
// them onto fewer processors chosen by its performance model.  On one GPU the
// corresponding cost is the kernel boundary: a grid-wide launch per
// relaxation / transfer costs microseconds even when a level holds a few
// hundred points.  Levels 0..l* therefore run here, inside ONE workgroup of
// 1024 threads, with a workgroup barrier where the paper's algorithm has a halo
// exchange (after every colour of Gauss-Seidel, after the residual, the
// restriction and the interpolation).  Levels from the coarsest up are staged
// in LDS while they fit; the rest are addressed in global memory (L2
// resident).  The coarsest level is solved with the Cholesky factor computed
// at setup (section 3, coarse-solve cost), in FP64.
#include "bmg_internal.h"

namespace hbmg {

constexpr int CWG = 1024;   // threads of the collapse workgroup

// A collapsed level as the workgroup addresses it: operator planes, iterate x,
// residual scratch r, right-hand side b, and the interpolation weights from
// the next-coarser level.  A level staged in LDS is laid out at compact pitch
// (planes C, W, S, SW, SE, x, r, b, then 8 weight planes at the coarse
// level's size) and its view is built from the workgroup's LDS array where it
// is used, so every access compiles to an LDS instruction; a level in global
// memory uses its own arrays.  Views live in registers.
template <typename T>
struct CV {
    int nx, ny, pitch;
    const T *C, *W, *S, *SW, *SE;
    T *x, *r, *b;
    const T *wt;
    int cpitch, cplane;   // pitch and plane size of the weight planes
};

template <typename T, bool LDS>
__device__ __forceinline__ CV<T> cview(const CollapseArgs<T> &a, int l, int xb)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const LevelDev<T> &g = a.levels[l];
    CV<T> v;
    v.nx = g.nx;
    v.ny = g.ny;
    if (LDS) {
        const int n = g.nx * g.ny;
        T *base = reinterpret_cast<T *>(smem + a.lds_off[l]);
        v.pitch = g.nx;
        v.C = base;
        v.W = base + n;
        v.S = base + 2 * n;
        v.SW = base + 3 * n;
        v.SE = base + 4 * n;
        v.x = base + 5 * n;
        v.r = base + 6 * n;
        v.b = base + 7 * n;
        v.wt = base + 8 * n;
        if (l >= 1) {
            v.cpitch = a.levels[l - 1].nx;
            v.cplane = a.levels[l - 1].nx * a.levels[l - 1].ny;
        } else {
            v.cpitch = v.cplane = 0;
        }
    } else {
        v.pitch = g.pitch;
        v.C = g.C;
        v.W = g.W;
        v.S = g.S;
        v.SW = g.SW;
        v.SE = g.SE;
        v.x = g.x[xb];
        v.r = g.x[1 - xb];
        v.b = g.b;
        v.wt = g.wt;
        v.cpitch = g.cpitch;
        v.cplane = (int)g.cplane;
    }
    return v;
}

// idx / n for 0 <= idx < 2^24 from a float reciprocal, corrected to exact
__device__ __forceinline__ int quot(int idx, int n, float rn)
{
    int q = (int)((float)idx * rn);
    if (q * n > idx) --q;
    else if ((q + 1) * n <= idx) ++q;
    return q;
}

// Residual (b - A x)_p at interior vertex p and the diagonal used by the
// relaxation (9-point form; the SW/SE planes of a 5-point level are zero).
// FP64 levels: standard form with C.  FP32 levels: edge form, the C plane
// holding the excess E = C - sum(connections).
template <typename T> struct EdgeForm { enum { value = 0 }; };
template <> struct EdgeForm<float> { enum { value = 1 }; };

template <typename T>
__device__ __forceinline__ T point_res(const CV<T> &L, const T *x, int p, T &diag)
{
    const int P = L.pitch;
    const T cw = L.W[p], ce = L.W[p + 1], cs = L.S[p], cn = L.S[p + P];
    const T csw = L.SW[p], cne = L.SW[p + P + 1], cse = L.SE[p], cnw = L.SE[p + P - 1];
    const T xp = x[p];
    if (!EdgeForm<T>::value) {
        const T s = L.b[p] + cw * x[p - 1] + ce * x[p + 1] + cs * x[p - P] + cn * x[p + P] +
                    csw * x[p - P - 1] + cne * x[p + P + 1] + cse * x[p - P + 1] + cnw * x[p + P - 1];
        diag = L.C[p];
        return s - L.C[p] * xp;
    } else {
        const T s = L.b[p] + cw * (x[p - 1] - xp) + ce * (x[p + 1] - xp) + cs * (x[p - P] - xp) +
                    cn * (x[p + P] - xp) + csw * (x[p - P - 1] - xp) + cne * (x[p + P + 1] - xp) +
                    cse * (x[p - P + 1] - xp) + cnw * (x[p + P - 1] - xp);
        diag = cw + ce + cs + cn + L.C[p] + csw + cne + cse + cnw;
        return s - L.C[p] * xp;
    }
}

template <typename T>
__device__ __forceinline__ T point_diag(const CV<T> &L, int p)
{
    if (!EdgeForm<T>::value) return L.C[p];
    const int P = L.pitch;
    return L.W[p] + L.W[p + 1] + L.S[p] + L.S[p + P] + L.C[p] + L.SW[p] + L.SW[p + P + 1] + L.SE[p] +
           L.SE[p + P - 1];
}

__device__ __forceinline__ int count_par(int lo, int hi) { return hi >= lo ? (hi - lo) / 2 + 1 : 0; }

// The point loops below are shared by the single collapse workgroup (thread
// tid of nthr = CWG) and the multi-workgroup stage (tid over all its
// workgroups): every point's arithmetic is the same whichever thread does it.

// one colour of Gauss-Seidel: colour k has (i mod 2, j mod 2) = (k & 1, k >> 1)
template <typename T>
__device__ __forceinline__ void gs_colour(const CV<T> &L, int k, int tid, int nthr)
{
    const int i0 = (k & 1) ? 1 : 2, j0 = (k >> 1) ? 1 : 2;
    const int ni = count_par(i0, L.nx - 2), nj = count_par(j0, L.ny - 2);
    const float rni = 1.0f / (float)ni;
    for (int idx = tid; idx < ni * nj; idx += nthr) {
        const int jj = quot(idx, ni, rni);
        const int i = i0 + 2 * (idx - jj * ni), j = j0 + 2 * jj;
        const int p = j * L.pitch + i;
        T d;
        const T r = point_res(L, L.x, p, d);
        L.x[p] += r / d;
    }
}

template <typename T>
__device__ __forceinline__ void zero_interior(const CV<T> &L, int tid, int nthr)
{
    const int ni = L.nx - 2, n = ni * (L.ny - 2);
    const float rni = 1.0f / (float)ni;
    for (int idx = tid; idx < n; idx += nthr) {
        const int jj = quot(idx, ni, rni);
        L.x[(1 + jj) * L.pitch + 1 + idx - jj * ni] = T(0);
    }
}

// r = b - A x on the interior; returns this thread's share of ||r||^2
template <typename T>
__device__ __forceinline__ double residual(const CV<T> &L, int tid, int nthr)
{
    const int ni = L.nx - 2, n = ni * (L.ny - 2);
    const float rni = 1.0f / (float)ni;
    double acc = 0.0;
    for (int idx = tid; idx < n; idx += nthr) {
        const int jj = quot(idx, ni, rni);
        const int p = (1 + jj) * L.pitch + 1 + idx - jj * ni;
        T d;
        const T v = point_res(L, L.x, p, d);
        L.r[p] = v;
        acc += (double)v * v;
    }
    return acc;
}

// b_c = P^T r on the interior coarse vertices (weights in F's weight planes)
template <typename T>
__device__ __forceinline__ void restrict_pt(const CV<T> &F, const CV<T> &Cl, int tid, int nthr)
{
    const int ni = Cl.nx - 2, n = ni * (Cl.ny - 2);
    const float rni = 1.0f / (float)ni;
    const int cp = F.cplane, WP = F.cpitch, P = F.pitch;
    const T *w = F.wt, *r = F.r;
    for (int idx = tid; idx < n; idx += nthr) {
        const int jj = quot(idx, ni, rni);
        const int I = 1 + idx - jj * ni, J = 1 + jj;
        const int f = 2 * J * P + 2 * I;
        const int c = J * WP + I;
        const int cW = c - 1, cS = c - WP, cSW = c - WP - 1;
        T v = r[f] + w[WXL * cp + c] * r[f + 1] + w[WXR * cp + cW] * r[f - 1] +
              w[WYB * cp + c] * r[f + P] + w[WYT * cp + cS] * r[f - P] +
              w[WCSW * cp + c] * r[f + P + 1] + w[WCSE * cp + cW] * r[f + P - 1] +
              w[WCNW * cp + cS] * r[f - P + 1] + w[WCNE * cp + cSW] * r[f - P - 1];
        Cl.b[J * Cl.pitch + I] = v;
    }
}

// x += P x_c (+ r/C at fine-only vertices); x_c is the coarse view's iterate
template <typename T>
__device__ __forceinline__ void interp_correct(const CV<T> &F, const CV<T> &Cl, int rescorr, int tid, int nthr)
{
    const int ni = F.nx - 2, n = ni * (F.ny - 2);
    const float rni = 1.0f / (float)ni;
    const int cp = F.cplane, WP = F.cpitch, CP = Cl.pitch;
    const T *w = F.wt, *xc = Cl.x;
    for (int idx = tid; idx < n; idx += nthr) {
        const int jj = quot(idx, ni, rni);
        const int i = 1 + idx - jj * ni, j = 1 + jj;
        const int p = j * F.pitch + i;
        const int c = (j >> 1) * CP + (i >> 1);
        const int cw = (j >> 1) * WP + (i >> 1);
        T v;
        if (!(i & 1) && !(j & 1)) {
            v = xc[c];
        } else {
            if ((i & 1) && !(j & 1))
                v = w[WXL * cp + cw] * xc[c] + w[WXR * cp + cw] * xc[c + 1];
            else if (!(i & 1) && (j & 1))
                v = w[WYB * cp + cw] * xc[c] + w[WYT * cp + cw] * xc[c + CP];
            else
                v = w[WCSW * cp + cw] * xc[c] + w[WCSE * cp + cw] * xc[c + 1] +
                    w[WCNW * cp + cw] * xc[c + CP] + w[WCNE * cp + cw] * xc[c + CP + 1];
            if (rescorr) v += F.r[p] / point_diag(F, p);
        }
        F.x[p] += v;
    }
}

// deterministic workgroup sum (fixed pairing)
__device__ double block_sum(double v, double *sh)
{
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < CWG / 64; ++k) s += sh[k];
    return s;
}

// Bytes of LDS a level occupies when staged: C, W, S, SW, SE, iterate,
// residual and right-hand side at compact pitch, plus the 8 weight planes
// from the coarser level.
template <typename T>
size_t collapse_lds_bytes(int nx, int ny, int cnx, int cny)
{
    size_t n = (size_t)nx * ny, cn = (size_t)cnx * cny;
    size_t b = (8 * n + 8 * cn) * sizeof(T);
    return (b + 15) / 16 * 16;
}
template size_t collapse_lds_bytes<double>(int, int, int, int);
template size_t collapse_lds_bytes<float>(int, int, int, int);

// Down leg on level l (fine view in LDS if FL, its coarse level if CL):
// relaxations, residual, restriction onto level l-1.
template <typename T, bool FL, bool CL>
__device__ void level_down(const CollapseArgs<T> &a, int l)
{
    const int xb = l == a.top ? a.xb_top : 1;
    const CV<T> F = cview<T, FL>(a, l, xb), Cl = cview<T, CL>(a, l - 1, 1);
    const int tid = threadIdx.x;
    if (l < a.top || a.zero_top) {
        zero_interior(F, tid, CWG);
        __syncthreads();
    }
    for (int s = 0; s < a.nu1; ++s)
        for (int k = 0; k < 4; ++k) {
            gs_colour(F, k, tid, CWG);
            __syncthreads();
        }
    residual(F, tid, CWG);
    __syncthreads();
    restrict_pt(F, Cl, tid, CWG);
    __syncthreads();
}

// Up leg on level l: interpolate and correct from level l-1, relax.
template <typename T, bool FL, bool CL>
__device__ void level_up(const CollapseArgs<T> &a, int l)
{
    const int xb = l == a.top ? a.xb_top : 1;
    const CV<T> F = cview<T, FL>(a, l, xb), Cl = cview<T, CL>(a, l - 1, 1);
    const int tid = threadIdx.x;
    interp_correct(F, Cl, a.rescorr, tid, CWG);
    __syncthreads();
    for (int s = 0; s < a.nu2; ++s)
        for (int k = 0; k < 4; ++k) {
            gs_colour(F, k, tid, CWG);
            __syncthreads();
        }
}

// coarsest level: Cholesky solve in FP64 (column-oriented substitutions)
template <typename T, bool LDS>
__device__ void coarse_solve(const CollapseArgs<T> &a)
{
    const CV<T> L0 = cview<T, LDS>(a, 0, a.top == 0 ? a.xb_top : 1);
    const int nc = a.nc;
    double *y = a.work;
    const int ni = L0.nx - 2, n = ni * (L0.ny - 2);
    for (int idx = threadIdx.x; idx < n; idx += CWG) {
        const int i = 1 + idx % ni, j = 1 + idx / ni;
        const int k = a.cidx[j * L0.nx + i];
        y[k] = (double)L0.b[j * L0.pitch + i];
    }
    __syncthreads();
    for (int k = 0; k < nc; ++k) {            // L y = b
        const double yk = y[k] / a.chol[(size_t)k * nc + k];
        for (int m = k + 1 + threadIdx.x; m < nc; m += CWG) y[m] -= a.chol[(size_t)m * nc + k] * yk;
        __syncthreads();
        if (threadIdx.x == 0) y[k] = yk;
        __syncthreads();
    }
    for (int k = nc - 1; k >= 0; --k) {       // L^T x = y
        const double xk = y[k] / a.chol[(size_t)k * nc + k];
        for (int m = threadIdx.x; m < k; m += CWG) y[m] -= a.chol[(size_t)k * nc + m] * xk;
        __syncthreads();
        if (threadIdx.x == 0) y[k] = xk;
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < n; idx += CWG) {
        const int i = 1 + idx % ni, j = 1 + idx / ni;
        L0.x[j * L0.pitch + i] = (T)y[a.cidx[j * L0.nx + i]];
    }
    __syncthreads();
}

// stage level l into LDS: operator and weights; iterate and residual zero;
// the top level's right-hand side (and iterate) from global memory.  Each
// thread issues all loads of an index (the operator at a vertex, the 8
// weights at a coarse vertex) before storing any, so a level costs one or two
// memory round trips, not one per plane.
template <typename T>
__device__ void stage_in(const CollapseArgs<T> &a, int l)
{
    const LevelDev<T> &g = a.levels[l];
    const CV<T> v = cview<T, true>(a, l, 1);
    const int nx = g.nx, n = g.nx * g.ny, top = a.top;
    const T *xg = g.x[l == top ? a.xb_top : 1];
    int cnx = 1, cn = 0;
    if (l >= 1) {
        cnx = a.levels[l - 1].nx;
        cn = cnx * a.levels[l - 1].ny;
    }
    const float rnx = 1.0f / (float)nx, rcnx = 1.0f / (float)cnx;
    const int m = n > cn ? n : cn;
    T *wt = const_cast<T *>(v.wt);
    for (int idx = threadIdx.x; idx < m; idx += CWG) {
        const bool op = idx < n, wq = idx < cn;
        T c = T(0), w = T(0), s = T(0), sw = T(0), se = T(0), bb = T(0), xx = T(0);
        T wk[8];
        if (op) {
            const int jj = quot(idx, nx, rnx);
            const size_t gp = (size_t)jj * g.pitch + (idx - jj * nx);
            c = g.C[gp];
            w = g.W[gp];
            s = g.S[gp];
            sw = g.SW[gp];
            se = g.SE[gp];
            if (l == top) {
                bb = g.b[gp];
                if (!a.zero_top) xx = xg[gp];
            }
        }
        if (wq) {
            const int jj = quot(idx, cnx, rcnx);
            const size_t cg = (size_t)jj * g.cpitch + (idx - jj * cnx);
            for (int k = 0; k < 8; ++k) wk[k] = g.wt[k * g.cplane + cg];
        }
        if (op) {
            const_cast<T *>(v.C)[idx] = c;
            const_cast<T *>(v.W)[idx] = w;
            const_cast<T *>(v.S)[idx] = s;
            const_cast<T *>(v.SW)[idx] = sw;
            const_cast<T *>(v.SE)[idx] = se;
            v.r[idx] = T(0);
            v.b[idx] = bb;
            v.x[idx] = xx;
        }
        if (wq)
            for (int k = 0; k < 8; ++k) wt[k * cn + idx] = wk[k];
    }
}

template <typename T>
__device__ __forceinline__ void collapse_body(const CollapseArgs<T> &a)
{
    __shared__ double sh[CWG / 64];
    const int top = a.top;
    for (int l = 0; l <= a.lds_top; ++l) stage_in(a, l);
    __syncthreads();
    // down: relax, residual, restrict (levels fill LDS from the coarsest up,
    // so a staged level's coarser neighbour is staged too)
    for (int l = top; l >= 1; --l) {
        if (l <= a.lds_top)
            level_down<T, true, true>(a, l);
        else if (l - 1 <= a.lds_top)
            level_down<T, false, true>(a, l);
        else
            level_down<T, false, false>(a, l);
    }
    if (a.lds_top >= 0)
        coarse_solve<T, true>(a);
    else
        coarse_solve<T, false>(a);
    // up: interpolate and correct, relax
    for (int l = 1; l <= top; ++l) {
        if (l <= a.lds_top)
            level_up<T, true, true>(a, l);
        else if (l - 1 <= a.lds_top)
            level_up<T, false, true>(a, l);
        else
            level_up<T, false, false>(a, l);
    }
    if (top <= a.lds_top) {
        const CV<T> Lt = cview<T, true>(a, top, a.xb_top);
        if (a.want_norm) {
            const double v = block_sum(residual(Lt, (int)threadIdx.x, CWG), sh);
            if (threadIdx.x == 0) a.partials[0] = v;
        }
        // the top level's iterate goes back to global memory
        const LevelDev<T> &g = a.levels[top];
        const int ni = g.nx - 2, n = ni * (g.ny - 2);
        T *xg = g.x[a.xb_top];
        for (int idx = threadIdx.x; idx < n; idx += CWG) {
            const int i = 1 + idx % ni, j = 1 + idx / ni;
            xg[(size_t)j * g.pitch + i] = Lt.x[j * Lt.pitch + i];
        }
    } else if (a.want_norm) {
        const CV<T> Lt = cview<T, false>(a, top, a.xb_top);
        const double v = block_sum(residual(Lt, (int)threadIdx.x, CWG), sh);
        if (threadIdx.x == 0) a.partials[0] = v;
    }
}

template <typename T>
__global__ __launch_bounds__(CWG) void k_collapse(CollapseArgs<T> a)
{
    if (a.active && *a.active == 0) return;
    collapse_body(a);
}

// one workgroup per problem of a batch; converged problems are skipped
template <typename T>
__global__ __launch_bounds__(CWG) void k_collapse_batched(const CollapseArgs<T> *__restrict__ args,
                                                          const int *__restrict__ active)
{
    if (!active[blockIdx.x]) return;
    collapse_body(args[blockIdx.x]);
}

template <typename T>
hipError_t launch_collapse_batched(const CollapseArgs<T> *args, int nprob, int lds_bytes,
                                   const int *active, hipStream_t s)
{
    hipLaunchKernelGGL((k_collapse_batched<T>), dim3(nprob), dim3(CWG), lds_bytes, s, args, active);
    return hipGetLastError();
}
template hipError_t launch_collapse_batched<double>(const CollapseArgs<double> *, int, int, const int *,
                                                    hipStream_t);
template hipError_t launch_collapse_batched<float>(const CollapseArgs<float> *, int, int, const int *,
                                                   hipStream_t);

// ---------------------------------------------------------------------------
// Agglomeration stages on several workgroups of one launch.
// ---------------------------------------------------------------------------

// Longest wait at one grid barrier, in polls (each a device-scope load and a
// short sleep: well over a second); past it the workgroup sets *err and stops
// waiting, and every later barrier of the launch returns at once, so a launch
// whose workgroups were not all resident still ends.
constexpr unsigned kBarrierPollLimit = 1u << 21;

// Barrier among the first K workgroups of the launch.  bar[0] counts
// arrivals, bar[1] is the generation.  The device-scope fences write this
// workgroup's stores back from its XCD's L2 before arriving and invalidate
// stale lines after leaving (the XCDs' L2s are not coherent with each other).
__device__ void grid_bar(unsigned *bar, unsigned K, int *err)
{
    __syncthreads();
    if (threadIdx.x == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        __threadfence();
        const unsigned g = __hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1;
        if (arrived == K) {
            __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(bar + 1, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            for (unsigned polls = 0;
                 __hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g; ++polls) {
                if (polls >= kBarrierPollLimit ||
                    __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __threadfence();
    }
    __syncthreads();
}

// down leg of level l on a stage of K workgroups (thread tid of nthr)
template <typename T>
__device__ void cluster_down(const ClusterArgs<T> &a, int l, int tid, int nthr, unsigned *bar, int K)
{
    const CollapseArgs<T> &c = a.col;
    const CV<T> F = cview<T, false>(c, l, l == a.hi[0] ? a.xb_top : 1), Cl = cview<T, false>(c, l - 1, 1);
    zero_interior(F, tid, nthr);
    grid_bar(bar, K, a.err);
    for (int s = 0; s < c.nu1; ++s)
        for (int k = 0; k < 4; ++k) {
            gs_colour(F, k, tid, nthr);
            grid_bar(bar, K, a.err);
        }
    residual(F, tid, nthr);
    grid_bar(bar, K, a.err);
    restrict_pt(F, Cl, tid, nthr);
    grid_bar(bar, K, a.err);
}

// up leg of level l on a stage of K workgroups
template <typename T>
__device__ void cluster_up(const ClusterArgs<T> &a, int l, int tid, int nthr, unsigned *bar, int K)
{
    const CollapseArgs<T> &c = a.col;
    const CV<T> F = cview<T, false>(c, l, l == a.hi[0] ? a.xb_top : 1), Cl = cview<T, false>(c, l - 1, 1);
    interp_correct(F, Cl, c.rescorr, tid, nthr);
    grid_bar(bar, K, a.err);
    for (int s = 0; s < c.nu2; ++s)
        for (int k = 0; k < 4; ++k) {
            gs_colour(F, k, tid, nthr);
            grid_bar(bar, K, a.err);
        }
}

template <typename T>
__global__ __launch_bounds__(CWG) void k_cluster(ClusterArgs<T> a)
{
    if (a.active && *a.active == 0) return;
    const int wg = blockIdx.x;
    int s = 0;
    // down legs; a workgroup beyond a stage's count leaves the descent there
    for (; s < a.nstage && wg < a.wg[s]; ++s) {
        const int K = a.wg[s];
        for (int l = a.hi[s]; l > a.hi[s + 1]; --l)
            cluster_down(a, l, wg * CWG + (int)threadIdx.x, K * CWG, a.bar + 2 * s, K);
    }
    // workgroup 0, the only one in every stage, collapses the rest
    if (s == a.nstage && wg == 0) collapse_body(a.col);
    // up legs: each stage first waits for the coarser ones
    for (int t = a.nstage - 1; t >= 0; --t) {
        if (wg >= a.wg[t]) continue;
        const int K = a.wg[t];
        grid_bar(a.bar + 2 * t, K, a.err);
        for (int l = a.hi[t + 1] + 1; l <= a.hi[t]; ++l)
            cluster_up(a, l, wg * CWG + (int)threadIdx.x, K * CWG, a.bar + 2 * t, K);
    }
}

template <typename T>
hipError_t launch_cluster(const ClusterArgs<T> &a, hipStream_t s)
{
    hipLaunchKernelGGL((k_cluster<T>), dim3(a.wg[0]), dim3(CWG), a.col.lds_bytes, s, a);
    return hipGetLastError();
}
template hipError_t launch_cluster<double>(const ClusterArgs<double> &, hipStream_t);
template hipError_t launch_cluster<float>(const ClusterArgs<float> &, hipStream_t);

template <typename T>
int cluster_max_resident(int lds_bytes)
{
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(&k_cluster<T>), CWG,
                                                     (size_t)lds_bytes) != hipSuccess)
        return 0;
    return per_cu * cus;
}
template int cluster_max_resident<double>(int);
template int cluster_max_resident<float>(int);

// allow the collapse kernels the large dynamic LDS they stage levels in (called
// at setup, outside any stream capture)
hipError_t collapse_set_attributes()
{
    const void *fns[6] = {reinterpret_cast<const void *>(&k_collapse<double>),
                          reinterpret_cast<const void *>(&k_collapse<float>),
                          reinterpret_cast<const void *>(&k_collapse_batched<double>),
                          reinterpret_cast<const void *>(&k_collapse_batched<float>),
                          reinterpret_cast<const void *>(&k_cluster<double>),
                          reinterpret_cast<const void *>(&k_cluster<float>)};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, COLLAPSE_LDS_BUDGET);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t launch_collapse(const CollapseArgs<T> &a, hipStream_t s)
{
    hipLaunchKernelGGL((k_collapse<T>), dim3(1), dim3(CWG), a.lds_bytes, s, a);
    return hipGetLastError();
}
template hipError_t launch_collapse<double>(const CollapseArgs<double> &, hipStream_t);
template hipError_t launch_collapse<float>(const CollapseArgs<float> &, hipStream_t);

// ---------------------------------------------------------------------------
// Norm helpers: per-block partial sums of squares over interior vertices, then
// one workgroup adds the partials in a fixed order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sumsq(const double *__restrict__ v, int nx, int ny,
                                               int pitch, double *__restrict__ partials)
{
    __shared__ double sh[4];
    const int ni = nx - 2;
    const long long n = (long long)ni * (ny - 2);
    double acc = 0.0;
    for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * 256) {
        const double a = v[(size_t)(1 + idx / ni) * pitch + 1 + idx % ni];
        acc += a * a;
    }
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

hipError_t launch_sumsq(const double *v, int nx, int ny, int pitch, double *partials, int nparts,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_sumsq, dim3(nparts), dim3(256), 0, s, v, nx, ny, pitch, partials);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ partials, int n,
                                                  const double *__restrict__ denom,
                                                  double *__restrict__ out)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) acc += partials[k];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = denom ? sqrt(sh[0]) / denom[0] : sqrt(sh[0]);
}

hipError_t launch_finalize_norm(const double *partials, int n, const double *denom, double *out,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, partials, n, denom, out);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_finalize_check(const double *__restrict__ partials, int n,
                                                        const double *__restrict__ denom, double tol, int k,
                                                        double *__restrict__ hist, int hist_cap, double *last,
                                                        int *flags, double *slot)
{
    __shared__ double sh[4];
    if (flags[0] == 0) return;   // an earlier cycle met the test
    // fixed order: a strided sum per lane, a butterfly within each wave, then
    // the four wave sums in turn
    double acc = 0.0;
    for (int m = threadIdx.x; m < n; m += 256) acc += partials[m];
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double rel = sqrt(((sh[0] + sh[1]) + sh[2]) + sh[3]) / denom[0];
        if (k - 1 < hist_cap) hist[k - 1] = rel;
        last[0] = rel;
        int run = 1;
        if (!isfinite(rel)) {
            run = 0;
            flags[1] = k;
            flags[2] = 2;
        } else if (rel <= tol) {
            run = 0;
            flags[1] = k;
            flags[2] = 1;
        }
        flags[0] = run;
        // host-mapped slot: the host reads it after synchronising on an event
        // recorded behind this kernel, whose system-scope release makes these
        // writes visible
        volatile double *v = slot;
        v[0] = rel;
        v[1] = (double)run;
        v[2] = (double)flags[1];
        v[3] = (double)k;
    }
}

hipError_t launch_finalize_check(const double *partials, int n, const double *denom, double tol, int k,
                                 double *hist, int hist_cap, double *last, int *flags, double *slot,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize_check, dim3(1), dim3(256), 0, s, partials, n, denom, tol, k, hist, hist_cap,
                       last, flags, slot);
    return hipGetLastError();
}

__global__ void k_flags_reset(int *flags)
{
    if (threadIdx.x < 4) flags[threadIdx.x] = threadIdx.x == 0 ? 1 : 0;
}

hipError_t launch_flags_reset(int *flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_flags_reset, dim3(1), dim3(64), 0, s, flags);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Batched norms.  Problem p's norm partials are partials[off[p] .. off[p] +
// cnt[p]); one workgroup per problem adds them in a fixed order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sumsq_batched(const double *const *__restrict__ v,
                                                       const int4 *__restrict__ dims,
                                                       double *__restrict__ partials, int nparts)
{
    __shared__ double sh[4];
    const int p = blockIdx.y;
    const int4 d = dims[p];   // nx, ny, pitch
    const int ni = d.x - 2;
    const long long n = (long long)ni * (d.y - 2);
    const double *x = v[p];
    double acc = 0.0;
    for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < n; idx += (long long)nparts * 256) {
        const double a = x[(size_t)(1 + idx / ni) * d.z + 1 + idx % ni];
        acc += a * a;
    }
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[(size_t)p * nparts + blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

hipError_t launch_sumsq_batched(const double *const *v, const int4 *dims, int nprob, double *partials,
                                int nparts, hipStream_t s)
{
    hipLaunchKernelGGL(k_sumsq_batched, dim3(nparts, nprob), dim3(256), 0, s, v, dims, partials, nparts);
    return hipGetLastError();
}

// out[p] = sqrt(sum of p's partials) / denom[p] (denom may be null); with a
// non-null `active`, an active problem is retired once out[p] <= tol or out[p]
// is not finite
__global__ __launch_bounds__(256) void k_finalize_batched(const double *__restrict__ partials,
                                                          const int *__restrict__ off,
                                                          const int *__restrict__ cnt,
                                                          const double *__restrict__ denom,
                                                          double *__restrict__ out,
                                                          int *__restrict__ active, double tol,
                                                          const double *__restrict__ tol_dev, int tol_stride)
{
    __shared__ double sh[256];
    const int p = blockIdx.x;
    if (active && !active[p]) return;
    double acc = 0.0;
    const double *src = partials + off[p];
    for (int k = threadIdx.x; k < cnt[p]; k += 256) acc += src[k];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double v = denom ? sqrt(sh[0]) / denom[p] : sqrt(sh[0]);
        out[p] = v;
        const double t = tol_dev ? tol_dev[(size_t)tol_stride * p] : tol;
        if (active && (!(v > t) || !isfinite(v))) active[p] = 0;
    }
}

hipError_t launch_finalize_batched(const double *partials, const int *off, const int *cnt,
                                   const double *denom, double *out, int *active, double tol,
                                   const double *tol_dev, int nprob, hipStream_t s, int tol_stride)
{
    hipLaunchKernelGGL(k_finalize_batched, dim3(nprob), dim3(256), 0, s, partials, off, cnt, denom, out,
                       active, tol, tol_dev, tol_stride);
    return hipGetLastError();
}

// number of active problems -> count[0] (one workgroup, fixed order)
__global__ __launch_bounds__(256) void k_count_active(const int *__restrict__ active, int n,
                                                      int *__restrict__ count)
{
    __shared__ int sh[256];
    int c = 0;
    for (int k = threadIdx.x; k < n; k += 256) c += active[k] != 0;
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) count[0] = sh[0];
}

hipError_t launch_count_active(const int *active, int n, int *count, hipStream_t s)
{
    hipLaunchKernelGGL(k_count_active, dim3(1), dim3(256), 0, s, active, n, count);
    return hipGetLastError();
}

}  // namespace hbmg
