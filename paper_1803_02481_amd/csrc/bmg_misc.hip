// bmg_misc.hip -- small element-wise kernels of the solve driver: boundary ring
// clearing, FP32 demotion of a level into edge form, the FP64 outer steps of
// mixed-precision iterative refinement, and a batch's copies of the caller's
// arrays to and from its finest levels.
#include "bmg_misc.h"

#include <algorithm>

namespace hbmg {

template <typename T>
__global__ void k_zero_ring(T *__restrict__ v, int nx, int ny, int pitch)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nx) {
        v[k] = T(0);
        v[(size_t)(ny - 1) * pitch + k] = T(0);
    }
    if (k < ny) {
        v[(size_t)k * pitch] = T(0);
        v[(size_t)k * pitch + nx - 1] = T(0);
    }
}

hipError_t launch_zero_ring(double *v, int nx, int ny, int pitch, hipStream_t s)
{
    const int n = nx > ny ? nx : ny;
    hipLaunchKernelGGL(k_zero_ring<double>, dim3((n + 255) / 256), dim3(256), 0, s, v, nx, ny, pitch);
    return hipGetLastError();
}

hipError_t launch_zero_ring(float *v, int nx, int ny, int pitch, hipStream_t s)
{
    const int n = nx > ny ? nx : ny;
    hipLaunchKernelGGL(k_zero_ring<float>, dim3((n + 255) / 256), dim3(256), 0, s, v, nx, ny, pitch);
    return hipGetLastError();
}

// FP32 edge form of a level: connections rounded to float, and the plane that
// holds C in FP64 holds instead the excess E = C - (sum of the connections),
// rounded to float.  The FP32 kernels form A x as
//   sum_q conn_pq (x_p - x_q) + E_p x_p,
// so the zero row sums of pure-diffusion rows survive the rounding exactly.
__global__ void k_demote_level(LevelDev<double> d, LevelDev<float> f)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    const size_t p = (size_t)j * d.pitch + i, P = d.pitch;
    const size_t pf = (size_t)j * f.pitch + i;
    f.W[pf] = (float)d.W[p];
    f.S[pf] = (float)d.S[p];
    f.SW[pf] = (float)d.SW[p];
    f.SE[pf] = (float)d.SE[p];
    float e = 0.0f;
    if (i >= 1 && i <= d.nx - 2 && j >= 1 && j <= d.ny - 2) {
        double rs = d.W[p] + d.W[p + 1] + d.S[p] + d.S[p + P] + d.SW[p] + d.SW[p + P + 1] + d.SE[p] +
                    d.SE[p + P - 1];
        e = (float)(d.C[p] - rs);
    }
    f.C[pf] = e;
}

__global__ void k_demote_weights(const double *__restrict__ wd, size_t pd, int pitchd,
                                 float *__restrict__ wf, size_t pf, int pitchf, int cnx, int cny)
{
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y;
    if (I >= cnx || J >= cny) return;
    for (int k = 0; k < 8; ++k)
        wf[k * pf + (size_t)J * pitchf + I] = (float)wd[k * pd + (size_t)J * pitchd + I];
}

hipError_t launch_demote_level(const LevelDev<double> &d, const LevelDev<float> &f, int cnx,
                               int cny, hipStream_t s)
{
    hipLaunchKernelGGL(k_demote_level, dim3((d.nx + 255) / 256, d.ny), dim3(256), 0, s, d, f);
    if (d.wt)
        hipLaunchKernelGGL(k_demote_weights, dim3((cnx + 255) / 256, cny), dim3(256), 0, s, d.wt,
                           d.cplane, d.cpitch, f.wt, f.cplane, f.cpitch, cnx, cny);
    return hipGetLastError();
}

// rows per workgroup of the outer residual: fewer partial sums for the
// single-workgroup norm that follows
constexpr int IR_ROWS = 16;

// FP64 outer residual of iterative refinement: r = b - A u (FP64, standard
// form), written demoted to FP32 as the inner right-hand side, with per-block
// partial sums of r^2 in FP64 (each thread adds its IR_ROWS rows in order).
template <int NPT>
__global__ __launch_bounds__(256) void k_ir_residual(LevelDev<double> d, const double *__restrict__ u,
                                                     float *__restrict__ r32, int pitchf,
                                                     double *__restrict__ partials)
{
    __shared__ double sh[4];
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j0 = blockIdx.y * IR_ROWS, j1 = min(j0 + IR_ROWS, d.ny);
    double acc = 0.0;
    if (i < d.nx) {
        for (int j = j0; j < j1; ++j) {
            const size_t p = (size_t)j * d.pitch + i, P = d.pitch;
            float out = 0.0f;
            if (i >= 1 && i <= d.nx - 2 && j >= 1 && j <= d.ny - 2) {
                double s = d.b[p] + d.W[p] * u[p - 1] + d.W[p + 1] * u[p + 1] + d.S[p] * u[p - P] +
                           d.S[p + P] * u[p + P];
                if (NPT == 9)
                    s += d.SW[p] * u[p - P - 1] + d.SW[p + P + 1] * u[p + P + 1] + d.SE[p] * u[p - P + 1] +
                         d.SE[p + P - 1] * u[p + P - 1];
                const double r = s - d.C[p] * u[p];
                acc += r * r;
                out = (float)r;
            }
            r32[(size_t)j * pitchf + i] = out;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        partials[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

hipError_t launch_ir_residual(const LevelDev<double> &d, const double *u, float *r32, int pitchf,
                              double *partials, int *nparts, hipStream_t s)
{
    dim3 g((d.nx + 255) / 256, (d.ny + IR_ROWS - 1) / IR_ROWS);
    *nparts = g.x * g.y;
    if (d.npt == 9)
        hipLaunchKernelGGL(k_ir_residual<9>, g, dim3(256), 0, s, d, u, r32, pitchf, partials);
    else
        hipLaunchKernelGGL(k_ir_residual<5>, g, dim3(256), 0, s, d, u, r32, pitchf, partials);
    return hipGetLastError();
}

// u += (double) e on interior vertices
__global__ void k_ir_update(double *__restrict__ u, int pitch, const float *__restrict__ e,
                            int pitchf, int nx, int ny)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2)
        u[(size_t)j * pitch + i] += (double)e[(size_t)j * pitchf + i];
}

hipError_t launch_ir_update(double *u, int pitch, const float *e, int pitchf, int nx, int ny,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_ir_update, dim3((nx + 255) / 256, ny), dim3(256), 0, s, u, pitch, e,
                       pitchf, nx, ny);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batched forms of the refinement steps: one workgroup per row of a problem
// (rowoff[p]: the first row of problem p, rowoff[nprob] the rows of all),
// found by bisection, looping over the row's 256-column blocks; problems whose
// flag is 0 are skipped
// ---------------------------------------------------------------------------
__device__ __forceinline__ int2 find_row(const int *__restrict__ rowoff, int nprob)
{
    const int r = blockIdx.x;
    int lo = 0, hi = nprob;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rowoff[mid] <= r) lo = mid;
        else hi = mid;
    }
    return make_int2(lo, r - rowoff[lo]);
}

// ZC: every problem's 5-point diagonal is bitwise the ordered sum of its four
// connections (checked at setup), formed instead of loaded.  Each 256-column
// block of a row gives one partial: block bx of row j of problem p is
// partials[boff[p] + j * blocks per row + bx].
template <int NPT, bool ZC>
__global__ __launch_bounds__(256) void k_ir_residual_batched(const LevelDev<double> *__restrict__ d,
                                                             const LevelDev<float> *__restrict__ f,
                                                             const int *__restrict__ active,
                                                             double *__restrict__ partials,
                                                             const int *__restrict__ boff,
                                                             const int *__restrict__ rowoff, int nprob)
{
    __shared__ double sh[2][4];   // alternate blocks: one barrier per block
    const int2 pr = find_row(rowoff, nprob);
    const int p = pr.x, j = pr.y;
    if (!active[p]) return;
    const LevelDev<double> &D = d[p];
    if (D.npt != NPT) return;
    const double *u = D.x[0];
    const int nxb = (D.nx + 255) / 256;
    for (int bx = 0; bx < nxb; ++bx) {
        const int i = bx * 256 + threadIdx.x;
        double acc = 0.0;
        if (i < D.nx) {
            const size_t q = (size_t)j * D.pitch + i, P = D.pitch;
            float out = 0.0f;
            if (i >= 1 && i <= D.nx - 2 && j >= 1 && j <= D.ny - 2) {
                double s = D.b[q] + D.W[q] * u[q - 1] + D.W[q + 1] * u[q + 1] + D.S[q] * u[q - P] +
                           D.S[q + P] * u[q + P];
                if (NPT == 9)
                    s += D.SW[q] * u[q - P - 1] + D.SW[q + P + 1] * u[q + P + 1] + D.SE[q] * u[q - P + 1] +
                         D.SE[q + P - 1] * u[q + P - 1];
                const double cq = ZC && NPT == 5 ? D.W[q] + D.W[q + 1] + D.S[q] + D.S[q + P] : D.C[q];
                const double r = s - cq * u[q];
                acc = r * r;
                out = (float)r;
            }
            f[p].b[(size_t)j * f[p].pitch + i] = out;
        }
        for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
        double *w = sh[bx & 1];
        if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) partials[boff[p] + j * nxb + bx] = ((w[0] + w[1]) + w[2]) + w[3];
    }
}

hipError_t launch_ir_residual_batched(const LevelDev<double> *d, const LevelDev<float> *f,
                                      const int *active, double *partials, const int *boff, const int *rowoff,
                                      int nrows, int npt, int nprob, hipStream_t s, int zc)
{
    dim3 g(nrows);
    if (npt == 9)
        hipLaunchKernelGGL((k_ir_residual_batched<9, false>), g, dim3(256), 0, s, d, f, active, partials, boff,
                           rowoff, nprob);
    else if (zc)
        hipLaunchKernelGGL((k_ir_residual_batched<5, true>), g, dim3(256), 0, s, d, f, active, partials, boff,
                           rowoff, nprob);
    else
        hipLaunchKernelGGL((k_ir_residual_batched<5, false>), g, dim3(256), 0, s, d, f, active, partials, boff,
                           rowoff, nprob);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_ir_update_batched(const LevelDev<double> *__restrict__ d,
                                                           const LevelDev<float> *__restrict__ f,
                                                           const float *const *__restrict__ eptr,
                                                           const int *__restrict__ active,
                                                           const int *__restrict__ rowoff, int nprob)
{
    const int2 pr = find_row(rowoff, nprob);
    const int p = pr.x, j = pr.y;
    if (!active[p]) return;
    const LevelDev<double> &D = d[p];
    if (j < 1 || j > D.ny - 2) return;
    const float *e = (eptr ? eptr[p] : f[p].x[0]) + (size_t)j * f[p].pitch;
    double *x = D.x[0] + (size_t)j * D.pitch;
    for (int i = 1 + threadIdx.x; i <= D.nx - 2; i += 256) x[i] += (double)e[i];
}

hipError_t launch_ir_update_batched(const LevelDev<double> *d, const LevelDev<float> *f, const float *const *eptr,
                                    const int *active, const int *rowoff, int nrows, int nprob, hipStream_t s)
{
    hipLaunchKernelGGL(k_ir_update_batched, dim3(nrows), dim3(256), 0, s, d, f, eptr, active, rowoff, nprob);
    return hipGetLastError();
}

__global__ void k_planes_in(const double *__restrict__ src, int nx, int ny, double *__restrict__ dst, int pitch,
                            size_t plane)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y, k = blockIdx.z;
    if (i < nx) dst[k * plane + (size_t)j * pitch + i] = src[((size_t)k * ny + j) * nx + i];
}

hipError_t launch_planes_in(const double *src, int nx, int ny, int nplanes, double *dst, int pitch, size_t plane,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_planes_in, dim3((nx + 255) / 256, ny, nplanes), dim3(256), 0, s, src, nx, ny, dst, pitch,
                       plane);
    return hipGetLastError();
}

// one wave per row of the batch; the row's problem by bisection of the row
// offsets (the same for all lanes of the wave)
template <bool OUT>
__global__ __launch_bounds__(256) void k_stage_batched(const double *const *__restrict__ user,
                                                       double *const *__restrict__ bdst,
                                                       double *const *__restrict__ xdst,
                                                       const int4 *__restrict__ dims,
                                                       const int *__restrict__ rowoff, int nprob, int rows)
{
    const int lane = threadIdx.x & 63;
    const int waves = gridDim.x * (blockDim.x >> 6);
    const int total = OUT ? rows : 2 * rows;
    for (int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < total; r += waves) {
        const int w = r >= rows;              // in: 0 the right-hand side, 1 the iterate
        const int rr = r - w * rows;
        int lo = 0, hi = nprob;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (rowoff[mid] <= rr) lo = mid;
            else hi = mid;
        }
        const int p = lo;
        const int4 dd = dims[p];
        const int j = rr - rowoff[p];
        if (OUT) {
            const double *src = user[2 * nprob + p];
            double *dst = const_cast<double *>(user[nprob + p]) + (size_t)j * dd.x;
            if (src) {
                src += (size_t)j * dd.z;
#pragma unroll 4
                for (int i = lane; i < dd.x; i += 64) dst[i] = src[i];
            } else {
                for (int i = lane; i < dd.x; i += 64) dst[i] = 0.0;
            }
        } else {
            const double *src = user[w * nprob + p] + (size_t)j * dd.x;
            double *dst = (w ? xdst : bdst)[p] + (size_t)j * dd.z;
            const bool edge = j == 0 || j == dd.y - 1;
#pragma unroll 4
            for (int i = lane; i < dd.x; i += 64)
                dst[i] = edge || i == 0 || i == dd.x - 1 ? 0.0 : src[i];
        }
    }
}

hipError_t launch_stage_batched(const double *const *user, double *const *bdst, double *const *xdst,
                                const int4 *dims, const int *rowoff, int nprob, int rows, int out, hipStream_t s)
{
    const int total = out ? rows : 2 * rows;
    const int blocks = std::max(1, std::min((total + 3) / 4, 4096));
    if (out)
        hipLaunchKernelGGL(k_stage_batched<true>, dim3(blocks), dim3(256), 0, s, user, bdst, xdst, dims, rowoff,
                           nprob, rows);
    else
        hipLaunchKernelGGL(k_stage_batched<false>, dim3(blocks), dim3(256), 0, s, user, bdst, xdst, dims, rowoff,
                           nprob, rows);
    return hipGetLastError();
}

}  // namespace hbmg
