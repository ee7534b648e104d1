// bmg_calib.hip -- measurement of the machine parameters of the collapse-level
// performance model.  The paper determines gamma by timing a local stencil
// matrix-vector product and alpha, beta with standard network benchmarks
// (section 3, postal model and its parameter table); on one GPU the
// corresponding quantities are measured here:
//   alpha_launch  gap between two dependent kernels on one stream
//   hbm / cache   streaming bandwidth with the relaxation's access mix (five
//                 arrays read, one written), out of HBM and out of cache
// and, by timing the solver's own kernels on a synthetic hierarchy
// (calibrate_on_kernels), the step latencies of the streaming kernels and the
// barrier-phase and bandwidth terms of collapsed levels.  Micro-kernels for a
// bare barrier and one workgroup's L2 bandwidth are timed as well, for
// comparison with the fitted values.
#include "hipbmg.h"
#include "bmg_internal.h"
#include "bmg_model.h"

#include <algorithm>
#include <vector>

namespace hbmg {

__global__ void k_empty(int) {}

// read five arrays, write one: the access mix of a relaxation sweep
__global__ __launch_bounds__(256) void k_stream_mix(const double2 *__restrict__ a,
                                                    const double2 *__restrict__ b,
                                                    const double2 *__restrict__ c,
                                                    const double2 *__restrict__ d,
                                                    const double2 *__restrict__ e,
                                                    double2 *__restrict__ o, long long n2, int reps)
{
    for (int rep = 0; rep < reps; ++rep)
        for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n2; i += (long long)gridDim.x * 256) {
            double2 va = a[i], vb = b[i], vc = c[i], vd = d[i], ve = e[i];
            double2 r;
            r.x = va.x + vb.x * vc.x + vd.x * ve.x;
            r.y = va.y + vb.y * vc.y + vd.y * ve.y;
            o[i] = r;
        }
}

// one workgroup: `iters` rounds of a dependent access + barrier
template <bool LDS>
__global__ __launch_bounds__(1024) void k_barrier(double *__restrict__ g, int iters, double *out)
{
    __shared__ double sh[1024];
    double *buf = LDS ? sh : g;
    const int t = threadIdx.x;
    buf[t] = (double)t;
    __syncthreads();
    double acc = 0.0;
    for (int k = 0; k < iters; ++k) {
        const double v = buf[(t + 1 + k) & 1023];
        __syncthreads();
        buf[t] = v + 1.0;
        acc += v;
        __syncthreads();
    }
    if (t == 0) out[0] = acc;
}

// one workgroup streaming an L2-resident buffer (read + write)
__global__ __launch_bounds__(1024) void k_wg_stream(double2 *__restrict__ g, long long n2, int reps)
{
    for (int r = 0; r < reps; ++r)
        for (long long i = threadIdx.x; i < n2; i += 1024) {
            double2 v = g[i];
            v.x += 1.0;
            v.y -= 1.0;
            g[i] = v;
        }
}

// best of `reps` timed repetitions after one warm-up; ok turns false if any
// HIP call fails (the launches included)
template <typename F>
static float time_ms(hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps, bool &ok, F &&launch)
{
    launch();   // warm-up
    float best = 1e30f;
    for (int r = 0; r < reps && ok; ++r) {
        float ms = 0.f;
        ok = ok && hipEventRecord(e0, s) == hipSuccess;
        launch();
        ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(e1, s) == hipSuccess &&
             hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        best = std::min(best, ms);
    }
    return best;
}

}  // namespace hbmg

using namespace hbmg;

extern "C" hipbmg_status hipbmg_calibrate(void *stream, double *out_host)
{
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return HIPBMG_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return HIPBMG_EHIP;
    }
    ModelParams p = model_params();
    hipbmg_status st = HIPBMG_OK;
    bool ok = true;   // every timing's HIP calls succeeded
    const long long nbig = 1LL << 24;      // doubles per array: 134 MB, far beyond the caches
    const long long nsmall = 1LL << 20;    // 8 MB per array: cache resident
    double *buf = nullptr, *small = nullptr;
    const size_t bytes = 6 * nbig * sizeof(double);
    if (hipMalloc(&buf, bytes) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return HIPBMG_ENOMEM;
    }
    if (hipMalloc(&small, 4 * 1024 * 1024) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(buf);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return HIPBMG_ENOMEM;
    }
    ok = hipMemsetAsync(buf, 0, bytes, s) == hipSuccess && hipMemsetAsync(small, 0, 4 * 1024 * 1024, s) == hipSuccess;
    {
        // dependent launch gap
        const int n = 200;
        float ms = time_ms(s, e0, e1, 3, ok, [&] {
            for (int k = 0; k < n; ++k) hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, s, k);
        });
        p.alpha_launch_us = 1e3 * ms / n;

        // streaming bandwidth, relaxation access mix
        auto mix = [&](long long n2, int grid, int reps) {
            const double2 *a = reinterpret_cast<const double2 *>(buf);
            const long long nd2 = nbig / 2;
            hipLaunchKernelGGL(k_stream_mix, dim3(grid), dim3(256), 0, s, a, a + nd2, a + 2 * nd2,
                               a + 3 * nd2, a + 4 * nd2, reinterpret_cast<double2 *>(buf) + 5 * nd2, n2, reps);
        };
        ms = time_ms(s, e0, e1, 5, ok, [&] { mix(nbig / 2, 8192, 1); });
        const double hbm_gbps = 6.0 * nbig * 8.0 / (ms * 1e-3) / 1e9;
        // cache-resident: six 8 MB arrays (48 MB, inside the last-level
        // cache), twenty passes in one launch so the launch gap does not count
        ms = time_ms(s, e0, e1, 5, ok, [&] { mix(nsmall / 2, 2048, 20); });
        const double cache_gbps = 20.0 * 6.0 * nsmall * 8.0 / (ms * 1e-3) / 1e9;
        p.beta_hbm_us_per_B = 1.0 / (hbm_gbps * 1e3);
        p.beta_cache_us_per_B = 1.0 / (cache_gbps * 1e3);

        // one row-pair step of a plain streaming sweep: one wave, 64 steps
        double sweep_step_us = 0.0;
        {
            const int nx = 121, ny = 2 * 64 + 1, pitch = 128;
            const size_t plane = (size_t)ny * pitch;
            double *lv = nullptr;
            if (hipMalloc(&lv, 9 * plane * sizeof(double)) == hipSuccess) {
                ok = ok && hipMemsetAsync(lv, 0, 9 * plane * sizeof(double), s) == hipSuccess;
                StreamArgs<double> a{};
                a.nx = nx;
                a.ny = ny;
                a.pitch = pitch;
                a.C = lv;
                a.W = lv + plane;
                a.S = lv + 2 * plane;
                a.SW = lv + 3 * plane;
                a.SE = lv + 4 * plane;
                a.b = lv + 7 * plane;
                a.x_in = lv + 5 * plane;
                a.x_out = lv + 6 * plane;
                a.rb = 64;
                int g;
                stream_geometry(nx, ny, 5, SV_SWEEP, a.rb, &a.nstrips, &a.nblocks, &a.ntiles, &g);
                ms = time_ms(s, e0, e1, 5, ok, [&] { (void)launch_stream<double>(5, SV_SWEEP, a, g, s); });
                sweep_step_us = std::max(0.05, (1e3 * ms - p.alpha_launch_us) / (a.rb + 1));
                ok = ok && hipStreamSynchronize(s) == hipSuccess;
                (void)hipFree(lv);
            } else {
                (void)hipGetLastError();
            }
        }

        // barriers in one workgroup
        const int iters = 2000;
        double *out = small + 1024 * 64;
        ms = time_ms(s, e0, e1, 3, ok, [&] {
            hipLaunchKernelGGL((k_barrier<false>), dim3(1), dim3(1024), 0, s, small, iters, out);
        });
        const double bar_glb_us = 1e3 * ms / (2.0 * iters);
        ms = time_ms(s, e0, e1, 3, ok, [&] {
            hipLaunchKernelGGL((k_barrier<true>), dim3(1), dim3(1024), 0, s, small, iters, out);
        });
        const double bar_lds_us = 1e3 * ms / (2.0 * iters);

        // one workgroup on L2-resident data
        const long long n2 = (1LL << 18) / 2;   // 2 MB
        ms = time_ms(s, e0, e1, 3, ok, [&] {
            hipLaunchKernelGGL(k_wg_stream, dim3(1), dim3(1024), 0, s, reinterpret_cast<double2 *>(small), n2, 4);
        });
        const double wg_gbps = 4.0 * 2.0 * n2 * 16.0 / (ms * 1e-3) / 1e9;
        if (!ok || hipStreamSynchronize(s) != hipSuccess) st = HIPBMG_EHIP;
        (void)hipFree(buf);
        (void)hipFree(small);
        buf = small = nullptr;
        // the step latencies and collapsed-level terms from the solver's own kernels
        if (st == HIPBMG_OK) st = calibrate_on_kernels(stream, p);
        if (st == HIPBMG_OK) {
            p.calibrated = 1;
            model_params() = p;
        }
        if (out_host) {
            for (int k = 0; k < 64; ++k) out_host[k] = 0.0;
            out_host[0] = p.alpha_launch_us;
            out_host[1] = hbm_gbps;
            out_host[2] = cache_gbps;
            for (int q = 0; q < 2; ++q) {
                out_host[3 + 2 * q] = p.step_dn_us[q];
                out_host[4 + 2 * q] = p.step_up_us[q];
                out_host[7 + q] = p.t_base_us[q];
                out_host[9 + 2 * q] = p.alpha_bar_us[q][0];
                out_host[10 + 2 * q] = p.alpha_bar_us[q][1];
                out_host[13 + 2 * q] = p.beta_wg_us_per_B[q][0] > 0 ? 1e-3 / p.beta_wg_us_per_B[q][0] : 0.0;
                out_host[14 + 2 * q] = p.beta_wg_us_per_B[q][1] > 0 ? 1e-3 / p.beta_wg_us_per_B[q][1] : 0.0;
            }
            out_host[17] = bar_lds_us;
            out_host[18] = bar_glb_us;
            out_host[19] = wg_gbps;
            out_host[20] = sweep_step_us;
            for (int q = 0; q < 2; ++q) {
                out_host[21 + 2 * q] = p.t0_dn_us[q];
                out_host[22 + 2 * q] = p.t0_up_us[q];
            }
            for (int q = 0; q < 2; ++q)
                for (int k = 0; k < MODEL_STAGE_SIZES; ++k) {
                    out_host[25 + 16 * q + k] = p.alpha_stage_us[q][k];
                    out_host[33 + 16 * q + k] =
                        p.beta_stage_us_per_B[q][k] > 0 ? 1e-3 / p.beta_stage_us_per_B[q][k] : 0.0;
                }
        }
    }
    if (buf) (void)hipFree(buf);
    if (small) (void)hipFree(small);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}
