// bmg_resnorm.hip -- the residual norm of the convergence test for any
// operator and iterate: ||b - A u||_2 and ||b||_2 over interior vertices.
//
// One pass over the stencil planes, b and u: each workgroup of 256 threads
// takes 256 columns of a band of RN_ROWS rows, each thread sums its rows'
// squares, the workgroup reduces them in a fixed order into two partial sums,
// and a single workgroup adds the partials in a fixed order.  The result is
// therefore the same bits on every call with the same inputs.
#include "hipbmg.h"
#include "bmg_internal.h"

#include <cmath>
#include <cstdio>
#include <mutex>
#include <vector>

namespace hbmg {

// Scratch of the allocation-free entry point: a fixed array in each device's
// global memory, held until the process ends.  65536 doubles (512 KiB) hold the
// partials of 32767 workgroups, enough for every grid up to 16385 x 16385.
// Every call on a device uses that device's array, so calls that overlap on
// one device race.
constexpr size_t RN_SCRATCH_DOUBLES = 65536;
static __device__ __align__(256) double scratch[RN_SCRATCH_DOUBLES];

constexpr int RN_THREADS = 256;
constexpr int RN_ROWS = 64;

// value of u at (i, j), with the boundary ring read as zero (its entries are
// ignored, as in a solve)
__device__ __forceinline__ double u_in(const double *__restrict__ u, int nx, int ny, int i, int j)
{
    return (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2) ? u[(size_t)j * nx + i] : 0.0;
}

template <int NPT>
__global__ __launch_bounds__(RN_THREADS) void k_resnorm_partials(int nx, int ny, const double *__restrict__ C,
                                                                 const double *__restrict__ W,
                                                                 const double *__restrict__ S,
                                                                 const double *__restrict__ SW,
                                                                 const double *__restrict__ SE,
                                                                 const double *__restrict__ b,
                                                                 const double *__restrict__ u,
                                                                 double *__restrict__ partials)
{
    __shared__ double sh[2][RN_THREADS / 64];
    const int i = blockIdx.x * RN_THREADS + threadIdx.x;
    const int j0 = max(1, (int)blockIdx.y * RN_ROWS), j1 = min((int)(blockIdx.y + 1) * RN_ROWS, ny - 1);
    double rr = 0.0, bb = 0.0;
    if (i >= 1 && i <= nx - 2) {
        for (int j = j0; j < j1; ++j) {
            const size_t p = (size_t)j * nx + i, P = nx;
            const double bp = b[p];
            double s = bp + W[p] * u_in(u, nx, ny, i - 1, j) + W[p + 1] * u_in(u, nx, ny, i + 1, j) +
                       S[p] * u_in(u, nx, ny, i, j - 1) + S[p + P] * u_in(u, nx, ny, i, j + 1);
            if (NPT == 9)
                s += SW[p] * u_in(u, nx, ny, i - 1, j - 1) + SW[p + P + 1] * u_in(u, nx, ny, i + 1, j + 1) +
                     SE[p] * u_in(u, nx, ny, i + 1, j - 1) + SE[p + P - 1] * u_in(u, nx, ny, i - 1, j + 1);
            const double r = s - C[p] * u[p];
            rr += r * r;
            bb += bp * bp;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        rr += __shfl_xor(rr, off, 64);
        bb += __shfl_xor(bb, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = rr;
        sh[1][threadIdx.x >> 6] = bb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const size_t blk = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
        partials[2 * blk] = ((sh[0][0] + sh[0][1]) + sh[0][2]) + sh[0][3];
        partials[2 * blk + 1] = ((sh[1][0] + sh[1][1]) + sh[1][2]) + sh[1][3];
    }
}

// out[0] = sqrt(sum of the residual partials), out[1] = sqrt(sum of the
// right-hand side partials), summed in a fixed order by one workgroup
__global__ __launch_bounds__(RN_THREADS) void k_resnorm_finish(const double *__restrict__ partials, int nblk,
                                                               double *__restrict__ out)
{
    __shared__ double sh[2][RN_THREADS];
    double rr = 0.0, bb = 0.0;
    for (int k = threadIdx.x; k < nblk; k += RN_THREADS) {
        rr += partials[2 * k];
        bb += partials[2 * k + 1];
    }
    sh[0][threadIdx.x] = rr;
    sh[1][threadIdx.x] = bb;
    __syncthreads();
    for (int h = RN_THREADS / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + h];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sqrt(sh[0][0]);
        out[1] = sqrt(sh[1][0]);
    }
}

static dim3 resnorm_grid(int nx, int ny)
{
    return dim3((nx + RN_THREADS - 1) / RN_THREADS, (ny + RN_ROWS - 1) / RN_ROWS);
}

// doubles of scratch one evaluation needs: two partials per workgroup and the
// two results
static size_t resnorm_scratch_doubles(int nx, int ny)
{
    const dim3 g = resnorm_grid(nx, ny);
    return 2 * (size_t)g.x * g.y + 2;
}

// Both kernels on `work` (resnorm_scratch_doubles(nx, ny) doubles of device
// memory), the two norms copied to out_host.
static hipbmg_status resnorm_run(int nx, int ny, int npt, const double *coeffs, const double *b, const double *u,
                                 double *work, double *out_host, hipStream_t s)
{
    const size_t plane = (size_t)nx * ny;
    const double *C = coeffs, *W = coeffs + plane, *S = coeffs + 2 * plane;
    const double *SW = npt == 9 ? coeffs + 3 * plane : nullptr, *SE = npt == 9 ? coeffs + 4 * plane : nullptr;
    const dim3 g = resnorm_grid(nx, ny);
    const int nblk = (int)(g.x * g.y);
    double *out = work + 2 * (size_t)nblk;
    if (npt == 9)
        hipLaunchKernelGGL(k_resnorm_partials<9>, g, dim3(RN_THREADS), 0, s, nx, ny, C, W, S, SW, SE, b, u, work);
    else
        hipLaunchKernelGGL(k_resnorm_partials<5>, g, dim3(RN_THREADS), 0, s, nx, ny, C, W, S, SW, SE, b, u, work);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_resnorm_finish, dim3(1), dim3(RN_THREADS), 0, s, work, nblk, out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(out_host, out, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_last_error(hipGetErrorString(e));
        return HIPBMG_EHIP;
    }
    return HIPBMG_OK;
}

static hipbmg_status resnorm_check(int nx, int ny, int npt, const double *coeffs, const double *b, const double *u,
                                   const double *out_host)
{
    if (!coeffs || !b || !u || !out_host) {
        set_last_error("null argument");
        return HIPBMG_EINVAL;
    }
    if (nx < 3 || ny < 3 || (npt != 5 && npt != 9)) {
        set_last_error("need nx, ny >= 3 and npt 5 or 9");
        return HIPBMG_EINVAL;
    }
    return HIPBMG_OK;
}

}  // namespace hbmg

using namespace hbmg;

extern "C" hipbmg_status hipbmg_residual_norm(int nx, int ny, int npt, const double *coeffs, const double *b,
                                              const double *u, double *out_host, void *stream)
{
    hipbmg_status st = resnorm_check(nx, ny, npt, coeffs, b, u, out_host);
    if (st != HIPBMG_OK) return st;
    std::vector<void *> owned;
    void *work = nullptr;
    if (dev_malloc(&work, resnorm_scratch_doubles(nx, ny) * sizeof(double)) != hipSuccess || !work) {
        set_last_error("scratch allocation failed");
        return HIPBMG_ENOMEM;
    }
    owned.push_back(work);
    st = resnorm_run(nx, ny, npt, coeffs, b, u, (double *)work, out_host, (hipStream_t)stream);
    dev_free_all(owned);
    return st;
}

// Device address of this device's scratch array.  In host code `scratch` is
// only a stand-in for the device symbol: its address is asked from the runtime
// once per device, with that device current, and kept.
static hipbmg_status scratch_of_device(double **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *ptr[kMaxDevices] = {};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_last_error("no usable current device");
        return HIPBMG_EHIP;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_last_error(e != hipSuccess ? hipGetErrorString(e) : "scratch symbol has no address");
            return HIPBMG_EHIP;
        }
        ptr[dev] = (double *)p;
    }
    *out = ptr[dev];
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_residual_norm_noalloc(int nx, int ny, int npt, const double *coeffs,
                                                      const double *b, const double *u, double *out_host,
                                                      void *stream)
{
    hipbmg_status st = resnorm_check(nx, ny, npt, coeffs, b, u, out_host);
    if (st != HIPBMG_OK) return st;
    const size_t need = resnorm_scratch_doubles(nx, ny);
    if (need > RN_SCRATCH_DOUBLES) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "a %d x %d grid needs %zu doubles of scratch; the allocation-free limit is %zu",
                      nx, ny, need, RN_SCRATCH_DOUBLES);
        set_last_error(msg);
        return HIPBMG_EINVAL;
    }
    double *sp = nullptr;
    st = scratch_of_device(&sp);
    if (st != HIPBMG_OK) return st;
    // every partial and both results are written before they are read: nothing
    // left by an earlier call needs clearing
    return resnorm_run(nx, ny, npt, coeffs, b, u, sp, out_host, (hipStream_t)stream);
}
