// bmg_misc.h -- declarations of the element-wise solve-driver kernels.
#pragma once
#include "bmg_internal.h"

namespace hbmg {

hipError_t launch_zero_ring(double *v, int nx, int ny, int pitch, hipStream_t s);
hipError_t launch_zero_ring(float *v, int nx, int ny, int pitch, hipStream_t s);
// FP64 level -> FP32 edge-form level (and its interpolation weights)
hipError_t launch_demote_level(const LevelDev<double> &d, const LevelDev<float> &f, int cnx,
                               int cny, hipStream_t s);
// r32 = (float)(b - A u) with FP64 partial sums of squares; *nparts partials written
hipError_t launch_ir_residual(const LevelDev<double> &d, const double *u, float *r32, int pitchf,
                              double *partials, int *nparts, hipStream_t s);
// u += (double) e
hipError_t launch_ir_update(double *u, int pitch, const float *e, int pitchf, int nx, int ny,
                            hipStream_t s);

// batched forms: one workgroup per row of a problem (rowoff[p]: the first row
// of problem p, rowoff[nprob] = nrows); inactive problems skipped.  The FP64
// iterate is x[0] of the finest level, the FP32 correction x[0] of the FP32
// finest level.  The residual writes one partial per 256-column block of a
// row: block bx of row j of problem p at partials[boff[p] + j * ((nx + 255) /
// 256) + bx].  zc: every problem's 5-point diagonal is bitwise the ordered sum
// of its four connections (checked at setup), so the residual forms it
// instead of loading it
hipError_t launch_ir_residual_batched(const LevelDev<double> *d, const LevelDev<float> *f,
                                      const int *active, double *partials, const int *boff, const int *rowoff,
                                      int nrows, int npt, int nprob, hipStream_t s, int zc = 0);
// u += e for every active problem; e from eptr[p] (device array of device
// pointers with the FP32 level's pitch), or the FP32 finest x[0] if eptr is null
hipError_t launch_ir_update_batched(const LevelDev<double> *d, const LevelDev<float> *f, const float *const *eptr,
                                    const int *active, const int *rowoff, int nrows, int nprob, hipStream_t s);
// planes [nplanes][ny][nx] (contiguous) into a level's padded planes
// (dst + k * plane, rows of `pitch`); the padding is left as it is
hipError_t launch_planes_in(const double *src, int nx, int ny, int nplanes, double *dst, int pitch, size_t plane,
                            hipStream_t s);
// the caller's arrays of a batch to and from the finest levels' padded planes,
// one wave per row over all problems (rowoff[p]: the first row of problem p in
// the batch, rowoff[nprob] the rows of all; dims[p] = (nx, ny, pitch)).
// In (out == 0): user[p] -> bdst[p] and user[nprob + p] -> xdst[p], with 0 on
// the boundary ring.  Out (out == 1): user[2 nprob + p] (padded; null gives
// zeros) -> user[nprob + p], every vertex as it is.
hipError_t launch_stage_batched(const double *const *user, double *const *bdst, double *const *xdst,
                                const int4 *dims, const int *rowoff, int nprob, int rows, int out, hipStream_t s);

}  // namespace hbmg
