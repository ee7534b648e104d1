// bmg_stream.hip -- streaming four-colour Gauss-Seidel relaxation for gfx950.
//
// One relaxation (section 2: pointwise Gauss-Seidel with four colours,
// colour k = (i mod 2) + 2 (j mod 2), colours 0,1,2,3 in turn) done in ONE pass
// over HBM instead of four:
//
//   * A wave (64 lanes) owns a strip of column pairs; lane t holds the even
//     column 2t and the odd column 2t+1.  Neighbour columns come from the
//     adjacent lanes by cross-lane shuffles, so no LDS and no barriers.
//   * The wave walks up the strip two rows per step.  Step j (j even) updates
//     colours 0 and 1 on row j, then colours 2 and 3 on row j-1.  Every value
//     a colour reads is then exactly the value the colour-by-colour sweep would
//     read: colour 0/1 on row j see rows j+-1 before colours 2/3 touch them,
//     and colours 2/3 on row j-1 see rows j-2 and j after colours 0/1.  After
//     step j rows j-1 and j are final.
//   * Strips overlap by a few halo lanes that recompute their neighbour's
//     columns (no lane reads a value another wave writes), and each block of
//     rows is preceded by one or two prologue steps that rebuild the state of
//     the rows below it.  The kernel therefore reads x_in and writes x_out.
//
// Fused variants (one HBM pass each):
//   - residual r = b - A x on the final rows (rows j-2, j-1 at step j), q = r/C
//     stored at fine-only vertices, and the restriction b_c = P^T r of coarse
//     row (j-2)/2 (Algorithm 1, restrict residual; section 3, interpolation
//     with the r/C term);
//   - interpolate-and-correct x += P x_c (+ q) applied to each row as it is
//     loaded, before the relaxation (Algorithm 1, interpolate and correct);
//   - residual norm partial sums for the convergence test.
//
// The tile index is remapped so that the 8 XCDs (WG i runs on XCD i mod 8)
// each get a contiguous band of strips and share halo rows in their own L2.
#include "bmg_internal.h"

#include <map>
#include <mutex>
#include <type_traits>
#include "bmg_weights.h"

namespace hbmg {

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

template <typename T>
__device__ __forceinline__ void ld2(const T *__restrict__ p, T &a, T &b)
{
    typename Vec2<T>::type v = *reinterpret_cast<const typename Vec2<T>::type *>(p);
    a = v.x;
    b = v.y;
}

template <typename T>
__device__ __forceinline__ void st2(T *__restrict__ p, T a, T b)
{
    typename Vec2<T>::type v;
    v.x = a;
    v.y = b;
    *reinterpret_cast<typename Vec2<T>::type *>(p) = v;
}

// value of lane-1 / lane+1 by the GFX9 whole-wave DPP shifts (wave_shr:1,
// wave_shl:1): a VALU move with no LDS round trip.  Lane 0 / lane 63 receive
// 0; those are halo lanes whose results are never stored.
__device__ __forceinline__ int dpp_from_lower(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int dpp_from_upper(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true); }
template <typename T> __device__ __forceinline__ T fromL(T v);
template <typename T> __device__ __forceinline__ T fromR(T v);
template <> __device__ __forceinline__ float fromL(float v) { return __int_as_float(dpp_from_lower(__float_as_int(v))); }
template <> __device__ __forceinline__ float fromR(float v) { return __int_as_float(dpp_from_upper(__float_as_int(v))); }
template <> __device__ __forceinline__ double fromL(double v)
{
    return __hiloint2double(dpp_from_lower(__double2hiint(v)), dpp_from_lower(__double2loint(v)));
}
template <> __device__ __forceinline__ double fromR(double v)
{
    return __hiloint2double(dpp_from_upper(__double2hiint(v)), dpp_from_upper(__double2loint(v)));
}

__device__ __forceinline__ int xcd_tile_fn()
{
    const int per = gridDim.x >> 3;
    return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// One row of the lane's column pair.  The c*/w*/q* fields hold the raw inputs
// of the interpolate-and-correct step until the row is finished.
template <typename T>
struct Row {
    T x0, x1, b0, b1, C0, C1, W0, W1, S0, S1, SW0, SW1, SE0, SE1;
    T ca, cu, w0, w1, w2, w3, w4, w5, q0, q1;
};

// Residual b - (A x) at the even column of row `cu` (rows `bl` below and `ab`
// above), and the diagonal used by the relaxation.  All lanes must call: the
// functions shuffle.  FP64 levels hold C in the C plane (standard form); FP32
// levels hold the excess E = C - sum(connections) there and use the edge form
//   (A x)_p = sum_q conn_pq (x_p - x_q) + E_p x_p,   diag = sum_q conn_pq + E_p,
// which keeps zero row sums exact after rounding to FP32.
template <typename T> struct IsEdge { enum { value = 0 }; };
template <> struct IsEdge<float> { enum { value = 1 }; };

template <typename T, int NPT>
__device__ __forceinline__ T res_even(const Row<T> &bl, const Row<T> &cu, const Row<T> &ab, T &diag)
{
    const T xw = fromL(cu.x1);
    T xsw = T(0), xnw = T(0), cnw = T(0);
    if (NPT == 9) {
        xsw = fromL(bl.x1);
        xnw = fromL(ab.x1);
        cnw = fromL(ab.SE1);
    }
    const T x = cu.x0;
    if (!IsEdge<T>::value) {
        T s = cu.b0 + cu.W0 * xw + cu.W1 * cu.x1 + cu.S0 * bl.x0 + ab.S0 * ab.x0;
        if (NPT == 9) s += cu.SW0 * xsw + ab.SW1 * ab.x1 + cu.SE0 * bl.x1 + cnw * xnw;
        diag = cu.C0;
        return s - cu.C0 * x;
    } else {
        T s = cu.b0 + cu.W0 * (xw - x) + cu.W1 * (cu.x1 - x) + cu.S0 * (bl.x0 - x) + ab.S0 * (ab.x0 - x);
        T d = cu.W0 + cu.W1 + cu.S0 + ab.S0 + cu.C0;
        if (NPT == 9) {
            s += cu.SW0 * (xsw - x) + ab.SW1 * (ab.x1 - x) + cu.SE0 * (bl.x1 - x) + cnw * (xnw - x);
            d += cu.SW0 + ab.SW1 + cu.SE0 + cnw;
        }
        diag = d;
        return s - cu.C0 * x;
    }
}

template <typename T, int NPT>
__device__ __forceinline__ T res_odd(const Row<T> &bl, const Row<T> &cu, const Row<T> &ab, T &diag)
{
    const T xe = fromR(cu.x0), we = fromR(cu.W0);
    T xne = T(0), xse = T(0), cne = T(0);
    if (NPT == 9) {
        xne = fromR(ab.x0);
        xse = fromR(bl.x0);
        cne = fromR(ab.SW0);
    }
    const T x = cu.x1;
    if (!IsEdge<T>::value) {
        T s = cu.b1 + cu.W1 * cu.x0 + we * xe + cu.S1 * bl.x1 + ab.S1 * ab.x1;
        if (NPT == 9) s += cu.SW1 * bl.x0 + cne * xne + cu.SE1 * xse + ab.SE0 * ab.x0;
        diag = cu.C1;
        return s - cu.C1 * x;
    } else {
        T s = cu.b1 + cu.W1 * (cu.x0 - x) + we * (xe - x) + cu.S1 * (bl.x1 - x) + ab.S1 * (ab.x1 - x);
        T d = cu.W1 + we + cu.S1 + ab.S1 + cu.C1;
        if (NPT == 9) {
            s += cu.SW1 * (bl.x0 - x) + cne * (xne - x) + cu.SE1 * (xse - x) + ab.SE0 * (ab.x0 - x);
            d += cu.SW1 + cne + cu.SE1 + ab.SE0;
        }
        diag = d;
        return s - cu.C1 * x;
    }
}

// ZC9: on a 9-point level whose rows at least two vertices from the boundary
// have zero row sums, the setup stored there exactly the sum of the eight
// connections, W_p + W_e + S_p + S_n + SW_p + SW_ne + SE_p + SE_nw in this
// order, as the diagonal (FP64), and an FP32 edge-form copy has a zero excess
// there.  The kernels then load C only at the rows and columns next to the
// boundary and form the FP64 diagonal of the deep vertices from the row and
// the row above it (ab: its S, SW, SE), bitwise the stored value.
__device__ __forceinline__ bool deep9(int j, int e, int o, int nx, int ny)
{
    return j >= 2 && j <= ny - 3 && e >= 2 && o <= nx - 3;
}

template <typename T>
__device__ __forceinline__ void complete_C9(Row<T> &r, const Row<T> &ab, bool deep)
{
    const T we = fromR(r.W0), cne = fromR(ab.SW0), cnw = fromL(ab.SE1);
    if (deep && !IsEdge<T>::value) {
        r.C0 = r.W0 + r.W1 + r.S0 + ab.S0 + r.SW0 + ab.SW1 + r.SE0 + cnw;
        r.C1 = r.W1 + we + r.S1 + ab.S1 + r.SW1 + cne + r.SE1 + ab.SE0;
    }
}

// The next row pair's loads are issued before the current step is computed,
// so their latency overlaps the step's arithmetic.  It costs registers (FP64
// two-sweep kernels drop to one wave per SIMD); measured on gfx950 it is
// neutral for FP64 and faster for the FP32 levels of mixed precision.
constexpr bool kPrefetch = true;

template <int V> struct VariantFlags;
template <> struct VariantFlags<SV_SWEEP>       { enum { ZX = 0, INTERP = 0, RES = 0, RQ = 0, NORM = 0 }; };
template <> struct VariantFlags<SV_SWEEP_ZX>    { enum { ZX = 1, INTERP = 0, RES = 0, RQ = 0, NORM = 0 }; };
template <> struct VariantFlags<SV_SWEEP_RQ>    { enum { ZX = 0, INTERP = 0, RES = 1, RQ = 1, NORM = 0 }; };
template <> struct VariantFlags<SV_SWEEP_RQ_ZX> { enum { ZX = 1, INTERP = 0, RES = 1, RQ = 1, NORM = 0 }; };
template <> struct VariantFlags<SV_INTERP>      { enum { ZX = 0, INTERP = 1, RES = 0, RQ = 0, NORM = 0 }; };
template <> struct VariantFlags<SV_INTERP_NORM> { enum { ZX = 0, INTERP = 1, RES = 1, RQ = 0, NORM = 1 }; };
template <> struct VariantFlags<SV_SWEEP_NORM>  { enum { ZX = 0, INTERP = 0, RES = 1, RQ = 0, NORM = 1 }; };

__host__ __device__ constexpr int halo_left(int npt, int res) { return 1 + (npt == 9) + res; }
__host__ __device__ constexpr int halo_right(int npt, int interp) { return 1 + (npt == 9) + interp; }

// Per-lane constants of a strip.
struct LaneCtx {
    int t, e, o, pitch, ny;
    bool own, ie, io, cv;
};

// Window of one relaxation stage walking up the strip: rows j-3..j+1 around
// step j, the residual of row j-3 and the restriction weights of the coarse
// row below.
template <typename T>
struct Stage {
    Row<T> rm3, rm2, rm1, r0, rp1;
    T rr3e, rr3o, ytp, cnwp, cnep;
    double acc;
};

template <typename T>
__device__ __forceinline__ void stage_rotate(Stage<T> &S)
{
    S.rm3 = S.rm1;
    S.rm2 = S.r0;
    S.rm1 = S.rp1;
}

// One step j of a relaxation stage whose rows j and j+1 are in S.r0, S.rp1
// (mode 0: colours 0, 1 only; 1: full step, nothing stored; 2: full step,
// stores if WRITE).  With RES the residual of the final rows j-2 and j-1 is
// formed, with RQ stored as q = r/C and restricted onto coarse row (j-2)/2,
// with NORM its squares are accumulated.
template <typename T, int NPT, bool WRITE, bool RES, bool RQ, bool NORM, bool WROW = false, bool STOREX = true,
          bool STOREQ = true>
__device__ __forceinline__ void stage_step(Stage<T> &S, int j, int mode, const LaneCtx &L,
                                           const StreamArgs<T> &a)
{
    const bool rj = j >= 1 && j <= L.ny - 2;
    const bool rjm = j - 1 >= 1 && j - 1 <= L.ny - 2;
    // colours 0 and 1 on row j
    {
        T d;
        T r = res_even<T, NPT>(S.rm1, S.r0, S.rp1, d);
        if (rj && L.ie) S.r0.x0 += r / d;
        r = res_odd<T, NPT>(S.rm1, S.r0, S.rp1, d);
        if (rj && L.io) S.r0.x1 += r / d;
    }
    if (mode != 0) {
        // colours 2 and 3 on row j-1
        T d;
        T r = res_even<T, NPT>(S.rm2, S.rm1, S.r0, d);
        if (rjm && L.ie) S.rm1.x0 += r / d;
        r = res_odd<T, NPT>(S.rm2, S.rm1, S.r0, d);
        if (rjm && L.io) S.rm1.x1 += r / d;

        if (WRITE && STOREX && mode == 2 && L.own) {
            if (rjm) st2(a.x_out + (size_t)(j - 1) * L.pitch + L.e, S.rm1.x0, S.rm1.x1);
            if (rj) st2(a.x_out + (size_t)j * L.pitch + L.e, S.r0.x0, S.r0.x1);
        }
        if (RES) {
            // residuals of the final rows j-2 (even) and j-1 (odd)
            const bool rA = j - 2 >= 1 && j - 2 <= L.ny - 2;
            T dae, dao, dbe, dbo;
            T ae = res_even<T, NPT>(S.rm3, S.rm2, S.rm1, dae);
            T ao = res_odd<T, NPT>(S.rm3, S.rm2, S.rm1, dao);
            T be = res_even<T, NPT>(S.rm2, S.rm1, S.r0, dbe);
            T bo = res_odd<T, NPT>(S.rm2, S.rm1, S.r0, dbo);
            if (!(rA && L.ie)) ae = T(0);
            if (!(rA && L.io)) ao = T(0);
            if (!(rjm && L.ie)) be = T(0);
            if (!(rjm && L.io)) bo = T(0);
            if (NORM && WRITE && mode == 2 && L.own)
                S.acc += (double)ae * ae + (double)ao * ao + (double)be * be + (double)bo * bo;
            if (RQ) {
                if (WRITE && STOREQ && mode == 2 && L.own) {
                    if (rA && L.io) a.q_out[(size_t)(j - 2) * L.pitch + L.o] = ao / dao;
                    if (rjm) st2(a.q_out + (size_t)(j - 1) * L.pitch + L.e,
                                 L.ie ? be / dbe : T(0), L.io ? bo / dbo : T(0));
                }
                // restriction onto coarse row jc = (j-2)/2, coarse column L.t
                const int jc = (j - 2) >> 1;
                const bool jcin = j - 2 >= 2 && jc <= a.cny - 2;
                T xl = T(0), xr = T(0), yb = T(0), yt = T(0), csw = T(0), cse = T(0),
                  cnw = T(0), cne = T(0);
                if (WROW) {
                    // the weights came in with rows j-2 (x-line pair) and j-1
                    // (the other six) when an earlier stage interpolated them
                    xl = S.rm2.w0;
                    xr = S.rm2.w1;
                    yb = S.rm1.w0;
                    yt = S.rm1.w1;
                    csw = S.rm1.w2;
                    cse = S.rm1.w3;
                    cnw = S.rm1.w4;
                    cne = S.rm1.w5;
                } else if (L.cv && j - 2 >= 0 && jc <= a.cny - 1) {
                    const size_t co = (size_t)jc * a.cpitch + L.t;
                    const long long cp = a.cplane;
                    xl = a.wt[WXL * cp + co];
                    xr = a.wt[WXR * cp + co];
                    yb = a.wt[WYB * cp + co];
                    yt = a.wt[WYT * cp + co];
                    csw = a.wt[WCSW * cp + co];
                    cse = a.wt[WCSE * cp + co];
                    cnw = a.wt[WCNW * cp + co];
                    cne = a.wt[WCNE * cp + co];
                }
                T lxr = fromL(xr), lcse = fromL(cse), lcnep = fromL(S.cnep);
                T lao = fromL(ao), lbo = fromL(bo), lr3o = fromL(S.rr3o);
                T bcv = ae + xl * ao + lxr * lao + yb * be + S.ytp * S.rr3e + csw * bo + lcse * lbo +
                        S.cnwp * S.rr3o + lcnep * lr3o;
                if (WRITE && mode == 2 && L.own && jcin && L.t >= 1 && L.t <= a.cnx - 2)
                    a.bc[(size_t)jc * a.cpitch + L.t] = bcv;
                S.ytp = yt;
                S.cnwp = cnw;
                S.cnep = cne;
            }
            S.rr3e = be;
            S.rr3o = bo;
        }
    }
}

template <typename T, int NPT, int V>
__device__ __forceinline__ void stream_tile(const StreamArgs<T> &a, const int tile)
{
    using F = VariantFlags<V>;
    constexpr int HL = halo_left(NPT, F::RES);
    constexpr int HR = halo_right(NPT, F::INTERP);
    constexpr int OWN = 64 - HL - HR;

    const int strip = tile % a.nstrips;
    const int blk = tile / a.nstrips;
    const int lane = threadIdx.x & 63;   // lane in the wave; a workgroup may hold several strips
    const int t = strip * OWN + lane - HL;   // column pair index
    const int e = 2 * t, o = 2 * t + 1;
    const int nx = a.nx, ny = a.ny, pitch = a.pitch;
    const bool colv = t >= 0 && e < nx;      // pair in the allocation (o may be padding)
    const bool own = lane >= HL && lane < 64 - HR && colv;
    const bool ie = e >= 1 && e <= nx - 2;
    const bool io = o >= 1 && o <= nx - 2;
    const bool cv = F::INTERP || F::RQ ? (t >= 0 && t < a.cnx) : false;   // coarse column t

    // issue the loads of row j (no use of the loaded values: they stay in
    // flight while the previous rows are being computed)
    auto load_raw = [&](Row<T> &r, int j) {
        const bool rv = colv && j >= 0 && j < ny;
        r = Row<T>{};
        if (rv) {
            const size_t off = (size_t)j * pitch + e;
            if (!F::ZX) ld2(a.x_in + off, r.x0, r.x1);
            ld2(a.b + off, r.b0, r.b1);
            ld2(a.C + off, r.C0, r.C1);
            ld2(a.W + off, r.W0, r.W1);
            ld2(a.S + off, r.S0, r.S1);
            if (NPT == 9) {
                ld2(a.SW + off, r.SW0, r.SW1);
                ld2(a.SE + off, r.SE0, r.SE1);
            }
        }
        if (F::INTERP) {
            const bool rin = j >= 1 && j <= ny - 2;
            if (cv && rin) {
                const int jc = j >> 1;
                const size_t co = (size_t)jc * a.cpitch + t;
                const T *wt = a.wt;
                const long long cp = a.cplane;
                r.ca = a.xc[co];
                if (j & 1) {
                    r.cu = a.xc[co + a.cpitch];
                    r.w0 = wt[WYB * cp + co];
                    r.w1 = wt[WYT * cp + co];
                    r.w2 = wt[WCSW * cp + co];
                    r.w3 = wt[WCSE * cp + co];
                    r.w4 = wt[WCNW * cp + co];
                    r.w5 = wt[WCNE * cp + co];
                } else {
                    r.w0 = wt[WXL * cp + co];
                    r.w1 = wt[WXR * cp + co];
                }
                if (a.rescorr) ld2(a.q_in + (size_t)j * pitch + e, r.q0, r.q1);
            }
        }
    };
    // x += P x_c (+ r/C at fine-only vertices) on a loaded row; coarse column t
    auto finish_row = [&](Row<T> &r, int j) {
        if (F::INTERP) {
            const bool rin = j >= 1 && j <= ny - 2;
            if ((j & 1) == 0) {
                const T xb = fromR(r.ca);
                if (rin && ie) r.x0 += r.ca;
                if (rin && io) r.x1 += r.w0 * r.ca + r.w1 * xb + r.q1;
            } else {
                const T xb = fromR(r.ca), xd = fromR(r.cu);
                if (rin && ie) r.x0 += r.w0 * r.ca + r.w1 * r.cu + r.q0;
                if (rin && io) r.x1 += r.w2 * r.ca + r.w3 * xb + r.w4 * r.cu + r.w5 * xd + r.q1;
            }
        }
    };

    const int nsteps = (ny - 1) / 2;            // steps j = 2, 4, ..., ny-1
    const int s0 = blk * a.rb;
    const int s1 = min(s0 + a.rb, nsteps);
    const int jfirst = 2 + 2 * s0;
    constexpr int PRO = F::RES ? 2 : 1;         // prologue steps

    const LaneCtx L{t, e, o, pitch, ny, own, ie, io, cv};
    Stage<T> S{};
    Row<T> n0, n1;
    Row<T> &rm1 = S.rm1, &r0 = S.r0, &rp1 = S.rp1;

    // state below the first prologue step: only row j-1 is read by a partial
    // step (colours 0 and 1); rows j-2, j-3 are rotated in before any use
    const int jstart = jfirst - 2 * PRO;
    load_raw(rm1, jstart - 1);
    finish_row(rm1, jstart - 1);
    if (kPrefetch) {
        load_raw(n0, jstart);
        load_raw(n1, jstart + 1);
    }

    const int last = s1 - 1 - s0;
    for (int step = -PRO; step <= last; ++step) {
        const int j = jfirst + 2 * step;
        const int mode = step < 0 ? (step == -PRO ? 0 : 1) : 2;   // 0 partial, 1 full, 2 write
        if (kPrefetch) {
            r0 = n0;
            rp1 = n1;
            if (step < last) {      // prefetch the next row pair
                load_raw(n0, j + 2);
                load_raw(n1, j + 3);
            }
        } else {
            load_raw(r0, j);
            load_raw(rp1, j + 1);
        }
        finish_row(r0, j);
        finish_row(rp1, j + 1);
        stage_step<T, NPT, true, F::RES, F::RQ, F::NORM>(S, j, mode, L, a);
        stage_rotate(S);
    }
    if (F::NORM) {
        // wave reduction in a fixed order -> one partial per tile
        double acc = S.acc;
        for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) a.partials[tile] = acc;
    }
}

// Two relaxations, then residual, r/C and restriction, in ONE pass (temporal
// blocking of the two pre-relaxations of Algorithm 1).  Stage A (first
// relaxation) runs one row-pair step ahead of stage B (second relaxation);
// stage B takes A's final rows as its "old" rows, so it is exactly the
// second colour-by-colour sweep.  A's results are correct on fewer lanes than
// a loaded row, so the halo is the sum of both stages' halos, and each block
// of rows starts with three A steps and two B steps of prologue.
template <typename T, int NPT, bool ZX, bool STOREQ = true, bool ZC9 = false>
__device__ __forceinline__ void stream2_tile(const StreamArgs<T> &a, const int tile)
{
    constexpr int HA = 1 + (NPT == 9);          // lanes of A's garbage margin per side
    constexpr int HL = HA + halo_left(NPT, 1);
    constexpr int HR = HA + halo_right(NPT, 0);
    constexpr int OWN = 64 - HL - HR;

    const int strip = tile % a.nstrips;
    const int blk = tile / a.nstrips;
    const int lane = threadIdx.x & 63;   // lane in the wave; a workgroup may hold several strips
    const int t = strip * OWN + lane - HL;
    const int e = 2 * t, o = 2 * t + 1;
    const int nx = a.nx, ny = a.ny, pitch = a.pitch;
    const bool colv = t >= 0 && e < nx;
    const bool own = lane >= HL && lane < 64 - HR && colv;
    const bool ie = e >= 1 && e <= nx - 2;
    const bool io = o >= 1 && o <= nx - 2;
    const bool cv = t >= 0 && t < a.cnx;
    const LaneCtx L{t, e, o, pitch, ny, own, ie, io, cv};

    auto load_row = [&](Row<T> &r, int j) {
        r = Row<T>{};
        if (colv && j >= 0 && j < ny) {
            const size_t off = (size_t)j * pitch + e;
            if (!ZX) ld2(a.x_in + off, r.x0, r.x1);
            ld2(a.b + off, r.b0, r.b1);
            if (!ZC9 || !deep9(j, e, o, nx, ny)) ld2(a.C + off, r.C0, r.C1);
            ld2(a.W + off, r.W0, r.W1);
            ld2(a.S + off, r.S0, r.S1);
            if (NPT == 9) {
                ld2(a.SW + off, r.SW0, r.SW1);
                ld2(a.SE + off, r.SE0, r.SE1);
            }
        }
    };

    const int nsteps = (ny - 1) / 2;
    const int s0 = blk * a.rb;
    const int s1 = min(s0 + a.rb, nsteps);
    const int jfirst = 2 + 2 * s0, jlast = 2 + 2 * (s1 - 1);

    Stage<T> A{}, B{};
    load_row(A.rm1, jfirst - 7);
    Row<T> N0, N1;                 // rows ja and ja+1, loaded one step ahead
    load_row(N0, jfirst - 6);
    load_row(N1, jfirst - 5);
    // one step; AM, BM: the stages' modes (BM < 0: B not yet active), MORE:
    // the next step's rows are loaded.  The prologue steps and the last one
    // are separate copies, so the steady loop has no conditional stage.
    auto step = [&](const int ja, auto am, auto bm, auto mo) {
        constexpr int AM = decltype(am)::value, BM = decltype(bm)::value;
        constexpr bool MORE = decltype(mo)::value;
        A.r0 = N0;
        A.rp1 = N1;
        if (MORE) {
            load_row(N0, ja + 2);
            load_row(N1, ja + 3);
        }
        if (ZC9) {
            // diagonals of rows ja-1 and ja, whose rows above are loaded
            complete_C9(A.rm1, A.r0, deep9(ja - 1, e, o, nx, ny));
            complete_C9(A.r0, A.rp1, deep9(ja, e, o, nx, ny));
        }
        stage_step<T, NPT, false, false, false, false>(A, ja, AM, L, a);
        const int jb = ja - 2;
        if constexpr (BM >= 0) {
            if (BM == 0) B.rm1 = A.rm3;   // A-final row jb-1 (first B step, jb = jfirst - 4)
            B.r0 = A.rm2;                  // A-final rows jb, jb+1 as B's old rows
            B.rp1 = A.rm1;
            stage_step<T, NPT, true, true, true, false, false, true, STOREQ>(B, jb, BM, L, a);
            stage_rotate(B);
        }
        stage_rotate(A);
    };
    using M0 = std::integral_constant<int, 0>;
    using M1 = std::integral_constant<int, 1>;
    using M2 = std::integral_constant<int, 2>;
    using Off = std::integral_constant<int, -1>;
    // A starts at jfirst - 6 (mode 0, then 1); B at jb = jfirst - 4 (mode 0),
    // jfirst - 2 (mode 1), then mode 2; the last step is ja = jlast + 2 >= jfirst + 2
    step(jfirst - 6, M0{}, Off{}, std::true_type{});
    step(jfirst - 4, M1{}, Off{}, std::true_type{});
    step(jfirst - 2, M1{}, M0{}, std::true_type{});
    step(jfirst, M1{}, M1{}, std::true_type{});
    int ja = jfirst + 2;
    for (; ja < jlast + 2; ja += 2) step(ja, M1{}, M2{}, std::true_type{});
    step(ja, M1{}, M2{}, std::false_type{});
}

// The finest level's post-relaxation of cycle k and both pre-relaxations of
// cycle k+1 in ONE pass (5-point operators).  Stage P interpolates and
// corrects each loaded row (x_in + P x_c + r/C, the r/C of the loaded
// iterate computed here from the raw rows around it -- the same residual the
// previous pass's stage B formed before storing that iterate), relaxes it and
// accumulates its residual norm (the convergence test of cycle k); the
// iterate after cycle k itself is not stored (the solve rebuilds the stopping
// cycle's with this kernel's P stage alone, PONLY).  Stage A relaxes P's
// final rows; stage B relaxes A's final rows, stores them in x_out2 and forms
// the residual and the restriction b_c of cycle k+1.  Each stage lags the
// previous one by one row-pair step; rows are loaded one row ahead of stage
// P, because the r/C of an odd row needs the raw row above it.  Per column,
// the lanes whose results are exact shrink by one for P's r/C and by one per
// stage, so 5 halo lanes are needed on each side; a row block starts with
// four P, three A and two B prologue steps.
// PONLY && PNORM: stage P alone with its norm and the iterate stored, for a
// cycle known to be the last (two prologue steps, as the norm's residual
// reads the row below a block's first final row).
// ZC: the C plane is not loaded.  FP64 levels form C_p = ((W_p + W_e) + S_p) + S_n
// from the connections of the row and the row above (the setup checked that
// this is bitwise the stored C at every interior vertex); FP32 edge-form
// levels have a zero excess.  The results are bitwise those of loading C.
// WF (FP64): the interpolation weights are not loaded either.  P forms them
// from the connections of the rows it loads, with the expressions the setup
// used to store them (bmg_weights.h), so they are bitwise the stored ones: an
// x-line vertex from its own row and the S of the row above, a y-line vertex
// and a cell centre from their row, the row above and the x-line weights of
// the rows below and above.  The S plane of each row is therefore loaded one
// step ahead of the rest of the row.
template <typename T, bool PONLY, bool PNORM = false, bool ZC = false, bool WF = false>
__device__ __forceinline__ void stream3_tile(const StreamArgs<T> &a, const int tile)
{
    constexpr int NPT = 5;
    constexpr int HL = 5, HR = 5, OWN = 64 - HL - HR;
    const int strip = tile % a.nstrips;
    const int blk = tile / a.nstrips;
    const int lane = threadIdx.x & 63;   // lane in the wave; a workgroup may hold several strips
    const int t = strip * OWN + lane - HL;
    const int e = 2 * t, o = 2 * t + 1;
    const int nx = a.nx, ny = a.ny, pitch = a.pitch;
    const bool colv = t >= 0 && e < nx;
    const bool own = lane >= HL && lane < 64 - HR && colv;
    const bool ie = e >= 1 && e <= nx - 2;
    const bool io = o >= 1 && o <= nx - 2;
    const bool cv = t >= 0 && t < a.cnx;
    const LaneCtx L{t, e, o, pitch, ny, own, ie, io, cv};

    // issue the loads of row j (no use of the loaded values: they stay in
    // flight while the previous rows are being computed); with_s = false
    // leaves the S plane out (WF: loaded a step earlier)
    auto load_raw = [&](Row<T> &r, int j, bool with_s = true) {
        const bool rv = colv && j >= 0 && j < ny;
        r = Row<T>{};
        if (rv) {
            const size_t off = (size_t)j * pitch + e;
            ld2(a.x_in + off, r.x0, r.x1);
            ld2(a.b + off, r.b0, r.b1);
            if (!ZC) ld2(a.C + off, r.C0, r.C1);
            ld2(a.W + off, r.W0, r.W1);
            if (with_s) ld2(a.S + off, r.S0, r.S1);
        }
        const bool rin = j >= 1 && j <= ny - 2;
        if (cv && rin) {
            const int jc = j >> 1;
            const size_t co = (size_t)jc * a.cpitch + t;
            const T *wt = a.wt;
            const long long cp = a.cplane;
            r.ca = a.xc[co];
            if (j & 1) {
                r.cu = a.xc[co + a.cpitch];
                if (WF) return;
                r.w0 = wt[WYB * cp + co];
                r.w1 = wt[WYT * cp + co];
                r.w2 = wt[WCSW * cp + co];
                r.w3 = wt[WCSE * cp + co];
                r.w4 = wt[WCNW * cp + co];
                r.w5 = wt[WCNE * cp + co];
            } else if (!WF) {
                r.w0 = wt[WXL * cp + co];
                r.w1 = wt[WXR * cp + co];
            }
        }
    };
    // the S plane of row j alone (WF)
    auto load_s = [&](T &s0v, T &s1v, int j) {
        s0v = s1v = T(0);
        if (colv && j >= 0 && j < ny) ld2(a.S + (size_t)j * pitch + e, s0v, s1v);
    };
    // ZC: the diagonal of row r once the S of the row above it (sn0, sn1) is
    // loaded; every lane calls (the east connection of the odd column is the
    // next lane's W)
    auto complete_Cs = [&](Row<T> &r, T sn0, T sn1) {
        if (ZC && !IsEdge<T>::value) {
            const T we = fromR(r.W0);
            r.C0 = r.W0 + r.W1 + r.S0 + sn0;
            r.C1 = r.W1 + we + r.S1 + sn1;
        }
    };
    auto complete_C = [&](Row<T> &r, const Row<T> &ab) { complete_Cs(r, ab.S0, ab.S1); };
    // WF: weights of the x-line vertex (o, j) of even row r, sn1 the S at
    // (o, j+1).  w0, w1 are the stored form (zero on boundary coarse vertices
    // and for a vertex that is not interior); w2, w3 keep the weights before
    // the coarse-boundary zeroing, which the cell centres above and below use.
    // Every lane calls.
    auto inner_v = [&](int i, int j) { return i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2; };
    auto cin = [&](int I, int J) { return I >= 1 && I <= a.cnx - 2 && J >= 1 && J <= a.cny - 2; };
    auto xline_row = [&](Row<T> &r, int j, T sn1) {
        if constexpr (WF) {
            const T we = fromR(r.W0);
            double ww_, we_;
            xline_weights(r.C1, sn1, r.S1, r.W1, 0.0, 0.0, we, 0.0, 0.0, ww_, we_);
            const bool in = inner_v(o, j);
            const int J = j >> 1;
            r.w2 = in ? ww_ : 0.0;
            r.w3 = in ? we_ : 0.0;
            r.w0 = in && cin(t, J) ? ww_ : 0.0;
            r.w1 = in && cin(t + 1, J) ? we_ : 0.0;
        }
    };
    // WF: weights of the y-line vertex (e, j) and the cell centre (o, j) of
    // odd row r; bl and ab are the even rows below and above (their x-line
    // weights formed), ab also gives the north connections.  Every lane calls.
    auto odd_row_weights = [&](Row<T> &r, int j, const Row<T> &bl, const Row<T> &ab) {
        if constexpr (WF) {
            double ys, yn;
            yline_weights(r.C0, r.W1, r.W0, r.S0, 0.0, 0.0, ab.S0, 0.0, 0.0, ys, yn);
            const bool iny = inner_v(e, j);
            ys = iny ? ys : 0.0;
            yn = iny ? yn : 0.0;
            // the y-line vertex east of the centre is the next lane's
            const T eb = fromR(T(ys)), etp = fromR(T(yn));
            const T ce = fromR(r.W0);
            const T d = r.C1, cs = r.S1, cn = ab.S1, cw = r.W1;
            const double wcsw = centre_weight(0.0, cs, bl.w2, cw, ys, d);
            const double wcse = centre_weight(0.0, cs, bl.w3, ce, eb, d);
            const double wcnw = centre_weight(0.0, cn, ab.w2, cw, yn, d);
            const double wcne = centre_weight(0.0, cn, ab.w3, ce, etp, d);
            const bool inc = inner_v(o, j);
            const int J = j >> 1;
            r.w0 = iny && cin(t, J) ? ys : 0.0;
            r.w1 = iny && cin(t, J + 1) ? yn : 0.0;
            r.w2 = inc && cin(t, J) ? wcsw : 0.0;
            r.w3 = inc && cin(t + 1, J) ? wcse : 0.0;
            r.w4 = inc && cin(t, J + 1) ? wcnw : 0.0;
            r.w5 = inc && cin(t + 1, J + 1) ? wcne : 0.0;
        }
    };
    // x += P x_c (+ r/C at fine-only vertices) on a loaded row; coarse column t
    auto finish_row = [&](Row<T> &r, int j, T q0, T q1) {
        const bool rin = j >= 1 && j <= ny - 2;
        if ((j & 1) == 0) {
            const T xb = fromR(r.ca);
            if (rin && ie) r.x0 += r.ca;
            if (rin && io) r.x1 += r.w0 * r.ca + r.w1 * xb + q1;
        } else {
            const T xb = fromR(r.ca), xd = fromR(r.cu);
            if (rin && ie) r.x0 += r.w0 * r.ca + r.w1 * r.cu + q0;
            if (rin && io) r.x1 += r.w2 * r.ca + r.w3 * xb + r.w4 * r.cu + r.w5 * xd + q1;
        }
    };
    // r/C of the raw iterate: odd column of an even row cu, and both columns
    // of an odd row cu (bl, ab: the raw rows below and above)
    const bool rc = a.rescorr != 0;
    auto rc_odd = [&](const Row<T> &bl, const Row<T> &cu, const Row<T> &ab) {
        T d;
        const T r = res_odd<T, NPT>(bl, cu, ab, d);
        return rc ? r / d : T(0);
    };
    auto rc_even = [&](const Row<T> &bl, const Row<T> &cu, const Row<T> &ab) {
        T d;
        const T r = res_even<T, NPT>(bl, cu, ab, d);
        return rc ? r / d : T(0);
    };

    const int nsteps = (ny - 1) / 2;
    const int s0 = blk * a.rb;
    const int s1 = min(s0 + a.rb, nsteps);
    const int jfirst = 2 + 2 * s0, jlast = 2 + 2 * (s1 - 1);
    // P alone (the rebuild) needs one prologue step, two with its norm; with A and B, four
    const int jp0 = PONLY ? (PNORM ? jfirst - 4 : jfirst - 2) : jfirst - 8, jpend = PONLY ? jlast : jlast + 4;

    StreamArgs<T> aB = a;          // stage B stores the next cycle's iterate
    aB.x_out = a.x_out2;
    Stage<T> P{}, A{}, B{};
    Row<T> Rm1, Rn;                // raw rows jp-1 and jp
    Row<T> N1, N2;                 // raw rows jp+1 and jp+2, loaded one step ahead
    T sa0 = T(0), sa1 = T(0);      // WF: S of row jp+3, loaded one step ahead of its row
    {
        Row<T> Ra;
        load_raw(Ra, jp0 - 2);
        load_raw(Rm1, jp0 - 1);
        load_raw(Rn, jp0);
        load_raw(N1, jp0 + 1);
        load_raw(N2, jp0 + 2);
        if (WF) load_s(sa0, sa1, jp0 + 3);
        complete_C(Ra, Rm1);
        complete_C(Rm1, Rn);
        if (WF) {
            complete_C(Rn, N1);
            xline_row(Ra, jp0 - 2, Rm1.S1);
            xline_row(Rn, jp0, N1.S1);
            odd_row_weights(Rm1, jp0 - 1, Ra, Rn);
        }
        P.rm1 = Rm1;
        finish_row(P.rm1, jp0 - 1, rc_even(Ra, Rm1, Rn), rc_odd(Ra, Rm1, Rn));
    }
    // one step; HASA, HASB: stages A and B active (false only in the first
    // four steps), MORE: the next step's rows are loaded (false in the last).
    // The first and last steps are separate copies of the step, so the steady
    // loop runs every stage unconditionally and its windows rotate without the
    // copies a conditional stage would need.
    auto step = [&](const int jp, auto ha, auto hb, auto mo) {
        constexpr bool HASA = decltype(ha)::value, HASB = decltype(hb)::value, MORE = decltype(mo)::value;
        Row<T> R1 = N1;
        Row<T> R2 = N2;
        const T s3a = sa0, s3b = sa1;  // WF: S of row jp+3
        if (MORE) {
            // the next step's rows: in flight while this step computes
            load_raw(N1, jp + 3, !WF);
            load_raw(N2, jp + 4);
            if (WF) {
                N1.S0 = s3a;
                N1.S1 = s3b;
                load_s(sa0, sa1, jp + 5);
            }
        }
        if (WF) {
            // diagonals of rows jp+1 and jp+2 (row jp's is formed), then the
            // weights of the x-line vertices of row jp+2 and of the y-line
            // vertices and cell centres of row jp+1
            complete_C(R1, R2);
            complete_Cs(R2, s3a, s3b);
            xline_row(R2, jp + 2, s3b);
            odd_row_weights(R1, jp + 1, Rn, R2);
        } else {
            // diagonals of rows jp and jp+1, whose rows above are now loaded
            complete_C(Rn, R1);
            complete_C(R1, R2);
        }
        const T q1_even_row = rc_odd(Rm1, Rn, R1);
        const T q0_odd_row = rc_even(Rn, R1, R2), q1_odd_row = rc_odd(Rn, R1, R2);
        P.r0 = Rn;
        P.rp1 = R1;
        finish_row(P.r0, jp, T(0), q1_even_row);
        finish_row(P.rp1, jp + 1, q0_odd_row, q1_odd_row);
        Rm1 = R1;
        Rn = R2;
        const int modeP = jp == jp0 ? 0 : (jp >= jfirst && jp <= jlast ? 2 : 1);
        if (PONLY) {
            stage_step<T, NPT, true, PNORM, false, PNORM>(P, jp, modeP, L, a);
            stage_rotate(P);
            return;
        }
        // the iterate after cycle k is not stored: only the stopping cycle's
        // is needed, and it is rebuilt from this pass's inputs afterwards
        stage_step<T, NPT, true, true, false, true, false, false>(P, jp, modeP, L, a);
        const int ja = jp - 2;
        if constexpr (HASA) {
            if (ja == jfirst - 6) A.rm1 = P.rm3;   // P-final row ja-1
            A.r0 = P.rm2;
            A.rp1 = P.rm1;
            stage_step<T, NPT, false, false, false, false>(A, ja, ja == jfirst - 6 ? 0 : 1, L, a);
            const int jb = ja - 2;
            if constexpr (HASB) {
                if (jb == jfirst - 4) B.rm1 = A.rm3;
                B.r0 = A.rm2;
                B.rp1 = A.rm1;
                const int modeB = jb < jfirst - 2 ? 0 : (jb == jfirst - 2 ? 1 : 2);
                // weights from the rows P loaded; r/C not stored (the next
                // pass's P forms it from the stored iterate)
                stage_step<T, NPT, true, true, true, false, true, true, false>(B, jb, modeB, L, aB);
                stage_rotate(B);
            }
            stage_rotate(A);
        }
        stage_rotate(P);
        };
    using Y = std::true_type;
    using N = std::false_type;
    if (PONLY) {
        int jp = jp0;
        for (; jp < jpend; jp += 2) step(jp, N{}, N{}, Y{});
        step(jp, N{}, N{}, N{});
    } else {
        // A joins at jp0 + 4, B at jp0 + 8 = jfirst, and jpend >= jfirst + 4
        step(jp0, N{}, N{}, Y{});
        step(jp0 + 2, N{}, N{}, Y{});
        step(jp0 + 4, Y{}, N{}, Y{});
        step(jp0 + 6, Y{}, N{}, Y{});
        int jp = jp0 + 8;
        for (; jp < jpend; jp += 2) step(jp, Y{}, Y{}, Y{});
        step(jp, Y{}, Y{}, N{});
    }
    if (!PONLY || PNORM) {
        double acc = P.acc;
        for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) a.partials[tile] = acc;
    }
}

template <typename T, bool PONLY, bool PNORM = false, bool ZC = false, bool WF = false>
__global__ __launch_bounds__(64) void k_stream3(StreamArgs<T> a)
{
    if (a.active && *a.active == 0) return;
    const int tile = xcd_tile_fn();
    if (tile >= a.ntiles) return;
    stream3_tile<T, PONLY, PNORM, ZC, WF && !IsEdge<T>::value>(a, tile);
}

// Zero-excess check of a 5-point level (see launch_zero_excess_check): one
// thread per vertex; any interior mismatch clears *flag (set to 1 beforehand)
template <typename T>
__global__ void k_zero_excess(LevelDev<T> A, int *flag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i < 1 || i > A.nx - 2 || j < 1 || j > A.ny - 2) return;
    const size_t p = (size_t)j * A.pitch + i, P = A.pitch;
    bool ok;
    if (IsEdge<T>::value)
        ok = A.C[p] == T(0);
    else
        ok = A.C[p] == A.W[p] + A.W[p + 1] + A.S[p] + A.S[p + P];
    if (!ok) atomicAnd(flag, 0);
}

__global__ void k_set_int(int *p, int v) { *p = v; }

// ZC9 setup of an FP64 9-point level.  set = 0: clear *flag if a vertex at
// least two vertices from the boundary has a diagonal further than 1e-12 of
// itself from the ordered sum of its connections (not a zero-row-sum row);
// set = 1: store that sum as the diagonal there.
__global__ void k_rowsum_diag(LevelDev<double> A, int *flag, int set)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i < 2 || i > A.nx - 3 || j < 2 || j > A.ny - 3) return;
    const size_t p = (size_t)j * A.pitch + i, P = A.pitch;
    const double rs = A.W[p] + A.W[p + 1] + A.S[p] + A.S[p + P] + A.SW[p] + A.SW[p + P + 1] + A.SE[p] +
                      A.SE[p + P - 1];
    if (set) {
        if (*flag) A.C[p] = rs;
    } else if (!(fabs(A.C[p] - rs) <= 1e-12 * fabs(A.C[p]))) atomicAnd(flag, 0);
}

// ZC9 check of an FP32 edge-form 9-point level: clear *flag unless every
// vertex at least two vertices from the boundary has a zero excess
__global__ void k_zero_excess9(LevelDev<float> A, int *flag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i < 2 || i > A.nx - 3 || j < 2 || j > A.ny - 3) return;
    if (A.C[(size_t)j * A.pitch + i] != 0.0f) atomicAnd(flag, 0);
}

hipError_t launch_rowsum_diag(const LevelDev<double> &A, int *flag, int set, hipStream_t s)
{
    if (!set) hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, flag, A.npt == 9 ? 1 : 0);
    if (A.npt == 9)
        hipLaunchKernelGGL(k_rowsum_diag, dim3((A.nx + 255) / 256, A.ny), dim3(256), 0, s, A, flag, set);
    return hipGetLastError();
}

hipError_t launch_zero_excess9(const LevelDev<float> &A, int *flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, flag, A.npt == 9 ? 1 : 0);
    if (A.npt == 9)
        hipLaunchKernelGGL(k_zero_excess9, dim3((A.nx + 255) / 256, A.ny), dim3(256), 0, s, A, flag);
    return hipGetLastError();
}

template <typename T>
static hipError_t zero_excess_check(const LevelDev<T> &A, int *flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, flag, A.npt == 5 ? 1 : 0);
    if (A.npt == 5)
        hipLaunchKernelGGL(k_zero_excess<T>, dim3((A.nx + 255) / 256, A.ny), dim3(256), 0, s, A, flag);
    return hipGetLastError();
}

hipError_t launch_zero_excess_check(const LevelDev<double> &A, int *flag, hipStream_t s)
{
    return zero_excess_check(A, flag, s);
}

hipError_t launch_zero_excess_check(const LevelDev<float> &A, int *flag, hipStream_t s)
{
    return zero_excess_check(A, flag, s);
}

// XCD-aware tile order: WG i runs on XCD i mod 8, so consecutive tiles (the
// neighbouring strips of a row band) are given to the same XCD
__device__ __forceinline__ int xcd_tile()
{
    const int per = gridDim.x >> 3;
    return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

template <typename T, int NPT, int V>
__global__ __launch_bounds__(64) void k_stream(StreamArgs<T> a)
{
    if (a.active && *a.active == 0) return;
    const int tile = xcd_tile();
    if (tile >= a.ntiles) return;
    stream_tile<T, NPT, V>(a, tile);
}

template <typename T, int NPT, bool ZX, bool STOREQ = true, bool ZC9 = false>
__global__ __launch_bounds__(64) void k_stream2(StreamArgs<T> a)
{
    if (a.active && *a.active == 0) return;
    const int tile = xcd_tile();
    if (tile >= a.ntiles) return;
    stream2_tile<T, NPT, ZX, STOREQ, ZC9>(a, tile);
}

// The up leg's first pass with the r/C term formed from the loaded rows
// instead of read from a stored plane (section 3, interpolation with r/C):
// the iterate this pass loads is the pre-relaxed one whose residual the down
// leg restricted, so b - A x of the raw rows is that residual, computed by
// the same expressions as the down leg's (bitwise the stored values).  Then
// x += P x_c + r/C and one relaxation.  Rows are loaded two rows ahead of the
// relaxation, because the r/C of an odd row needs the raw row above it.  The
// r/C costs one lane of exact columns on each side.
template <typename T, int NPT, bool ZC9 = false>
__device__ __forceinline__ void interp_rc_tile(const StreamArgs<T> &a, const int tile)
{
    constexpr int HL = 1 + halo_left(NPT, 0), HR = 1 + halo_right(NPT, 0), OWN = 64 - HL - HR;
    const int strip = tile % a.nstrips;
    const int blk = tile / a.nstrips;
    const int lane = threadIdx.x & 63;   // lane in the wave; a workgroup may hold several strips
    const int t = strip * OWN + lane - HL;
    const int e = 2 * t, o = 2 * t + 1;
    const int nx = a.nx, ny = a.ny, pitch = a.pitch;
    const bool colv = t >= 0 && e < nx;
    const bool own = lane >= HL && lane < 64 - HR && colv;
    const bool ie = e >= 1 && e <= nx - 2;
    const bool io = o >= 1 && o <= nx - 2;
    const bool cv = t >= 0 && t < a.cnx;
    const LaneCtx L{t, e, o, pitch, ny, own, ie, io, cv};

    auto load_raw = [&](Row<T> &r, int j) {
        const bool rv = colv && j >= 0 && j < ny;
        r = Row<T>{};
        if (rv) {
            const size_t off = (size_t)j * pitch + e;
            ld2(a.x_in + off, r.x0, r.x1);
            ld2(a.b + off, r.b0, r.b1);
            if (!ZC9 || !deep9(j, e, o, nx, ny)) ld2(a.C + off, r.C0, r.C1);
            ld2(a.W + off, r.W0, r.W1);
            ld2(a.S + off, r.S0, r.S1);
            if (NPT == 9) {
                ld2(a.SW + off, r.SW0, r.SW1);
                ld2(a.SE + off, r.SE0, r.SE1);
            }
        }
        const bool rin = j >= 1 && j <= ny - 2;
        if (cv && rin) {
            const int jc = j >> 1;
            const size_t co = (size_t)jc * a.cpitch + t;
            const T *wt = a.wt;
            const long long cp = a.cplane;
            r.ca = a.xc[co];
            if (j & 1) {
                r.cu = a.xc[co + a.cpitch];
                r.w0 = wt[WYB * cp + co];
                r.w1 = wt[WYT * cp + co];
                r.w2 = wt[WCSW * cp + co];
                r.w3 = wt[WCSE * cp + co];
                r.w4 = wt[WCNW * cp + co];
                r.w5 = wt[WCNE * cp + co];
            } else {
                r.w0 = wt[WXL * cp + co];
                r.w1 = wt[WXR * cp + co];
            }
        }
    };
    auto finish_row = [&](Row<T> &r, int j, T q0, T q1) {
        const bool rin = j >= 1 && j <= ny - 2;
        if ((j & 1) == 0) {
            const T xb = fromR(r.ca);
            if (rin && ie) r.x0 += r.ca;
            if (rin && io) r.x1 += r.w0 * r.ca + r.w1 * xb + q1;
        } else {
            const T xb = fromR(r.ca), xd = fromR(r.cu);
            if (rin && ie) r.x0 += r.w0 * r.ca + r.w1 * r.cu + q0;
            if (rin && io) r.x1 += r.w2 * r.ca + r.w3 * xb + r.w4 * r.cu + r.w5 * xd + q1;
        }
    };
    const bool rc = a.rescorr != 0;
    auto rc_odd = [&](const Row<T> &bl, const Row<T> &cu, const Row<T> &ab) {
        T d;
        const T r = res_odd<T, NPT>(bl, cu, ab, d);
        return rc ? r / d : T(0);
    };
    auto rc_even = [&](const Row<T> &bl, const Row<T> &cu, const Row<T> &ab) {
        T d;
        const T r = res_even<T, NPT>(bl, cu, ab, d);
        return rc ? r / d : T(0);
    };

    const int nsteps = (ny - 1) / 2;
    const int s0 = blk * a.rb;
    const int s1 = min(s0 + a.rb, nsteps);
    const int jfirst = 2 + 2 * s0, jlast = 2 + 2 * (s1 - 1);
    const int jp0 = jfirst - 2;   // one prologue step
    Stage<T> P{};
    Row<T> Rm1, Rn, N1, N2;       // raw rows jp-1, jp; jp+1, jp+2 loaded a step ahead
    {
        Row<T> Ra;
        load_raw(Ra, jp0 - 2);
        load_raw(Rm1, jp0 - 1);
        load_raw(Rn, jp0);
        load_raw(N1, jp0 + 1);
        load_raw(N2, jp0 + 2);
        if (ZC9) {
            complete_C9(Ra, Rm1, deep9(jp0 - 2, e, o, nx, ny));
            complete_C9(Rm1, Rn, deep9(jp0 - 1, e, o, nx, ny));
        }
        P.rm1 = Rm1;
        finish_row(P.rm1, jp0 - 1, rc_even(Ra, Rm1, Rn), rc_odd(Ra, Rm1, Rn));
    }
    // one step (MODE: the stage's mode, MORE: the next rows are loaded); the
    // prologue step and the last one are separate copies of it
    auto step = [&](const int jp, auto md, auto mo) {
        constexpr int MODE = decltype(md)::value;
        constexpr bool MORE = decltype(mo)::value;
        Row<T> R1 = N1, R2 = N2;
        if (MORE) {
            load_raw(N1, jp + 3);
            load_raw(N2, jp + 4);
        }
        if (ZC9) {
            // diagonals of rows jp and jp+1, whose rows above are loaded
            complete_C9(Rn, R1, deep9(jp, e, o, nx, ny));
            complete_C9(R1, R2, deep9(jp + 1, e, o, nx, ny));
        }
        const T q1_even_row = rc_odd(Rm1, Rn, R1);
        const T q0_odd_row = rc_even(Rn, R1, R2), q1_odd_row = rc_odd(Rn, R1, R2);
        P.r0 = Rn;
        P.rp1 = R1;
        finish_row(P.r0, jp, T(0), q1_even_row);
        finish_row(P.rp1, jp + 1, q0_odd_row, q1_odd_row);
        Rm1 = R1;
        Rn = R2;
        stage_step<T, NPT, true, false, false, false>(P, jp, MODE, L, a);
        stage_rotate(P);
    };
    // jp0 = jfirst - 2 < jlast
    step(jp0, std::integral_constant<int, 0>{}, std::true_type{});
    int jp = jfirst;
    for (; jp < jlast; jp += 2) step(jp, std::integral_constant<int, 2>{}, std::true_type{});
    step(jp, std::integral_constant<int, 2>{}, std::false_type{});
}

template <typename T, int NPT, bool ZC9 = false>
__global__ __launch_bounds__(64) void k_interp_rc(StreamArgs<T> a)
{
    if (a.active && *a.active == 0) return;
    const int tile = xcd_tile();
    if (tile >= a.ntiles) return;
    interp_rc_tile<T, NPT, ZC9>(a, tile);
}

// Batched form: one launch covers the same stage of many problems.  map[w] =
// (problem, tile) of wave w; a workgroup holds W waves, so W consecutive
// entries (neighbouring strips of one row block) share a CU.  Problems whose
// flag in `active` is 0 are skipped (converged).
template <typename T, int NPT, int V, int W>
__global__ __launch_bounds__(64 * W) void k_stream_batched(const StreamArgs<T> *__restrict__ args,
                                                           const int2 *__restrict__ map, int nmap,
                                                           const int *__restrict__ active)
{
    const int w = (int)blockIdx.x * W + (int)(threadIdx.x >> 6);
    if (w >= nmap) return;
    const int2 m = map[w];
    if (!active[m.x]) return;
    const StreamArgs<T> a = args[m.x];
    if (V == SV_SWEEP2_RQ)
        stream2_tile<T, NPT, false>(a, m.y);
    else if (V == SV_SWEEP2_RQ_ZX)
        stream2_tile<T, NPT, true>(a, m.y);
    else
        stream_tile<T, NPT, (V >= SV_SWEEP2_RQ ? SV_SWEEP : V)>(a, m.y);
}

int stream_owned_pairs(int npt, int variant)
{
    if (variant == SV_FUSED3 || variant == SV_FUSED3_P || variant == SV_FUSED3_PN) return 54;
    if (variant == SV_INTERP_RC) return 64 - (1 + halo_left(npt, 0)) - (1 + halo_right(npt, 0));
    if (variant == SV_SWEEP2_RQ || variant == SV_SWEEP2_RQ_ZX || variant == SV_SWEEP2_R || variant == SV_SWEEP2_R_ZX)
        return 64 - (1 + (npt == 9)) - halo_left(npt, 1) - (1 + (npt == 9)) - halo_right(npt, 0);
    int res = (variant == SV_SWEEP_RQ || variant == SV_SWEEP_RQ_ZX || variant == SV_INTERP_NORM ||
               variant == SV_SWEEP_NORM);
    int interp = (variant == SV_INTERP || variant == SV_INTERP_NORM);
    return 64 - halo_left(npt, res) - halo_right(npt, interp);
}

void stream_geometry(int nx, int ny, int npt, int variant, int rb, int *nstrips, int *nblocks,
                     int *ntiles, int *grid)
{
    int own = stream_owned_pairs(npt, variant);
    int pairs = (nx + 1) / 2;
    int nsteps = (ny - 1) / 2;
    *nstrips = (pairs + own - 1) / own;
    *nblocks = (nsteps + rb - 1) / rb;
    *ntiles = *nstrips * *nblocks;
    *grid = (*ntiles + 7) / 8 * 8;
}

// the pipelined finest kernel: variant x zero-excess x formed weights
template <typename T, bool PONLY, bool PNORM>
static void launch_f3(const StreamArgs<T> &a, dim3 g, dim3 b, hipStream_t s)
{
    const int k = (a.zexc ? 1 : 0) + (a.wform ? 2 : 0);
    switch (k) {
    case 0: hipLaunchKernelGGL((k_stream3<T, PONLY, PNORM, false, false>), g, b, 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_stream3<T, PONLY, PNORM, true, false>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_stream3<T, PONLY, PNORM, false, true>), g, b, 0, s, a); break;
    default: hipLaunchKernelGGL((k_stream3<T, PONLY, PNORM, true, true>), g, b, 0, s, a); break;
    }
}

template <typename T>
static hipError_t launch_fused3(int variant, const StreamArgs<T> &a, dim3 g, dim3 b, hipStream_t s)
{
    if (variant == SV_FUSED3) launch_f3<T, false, false>(a, g, b, s);
    else if (variant == SV_FUSED3_P) launch_f3<T, true, false>(a, g, b, s);
    else launch_f3<T, true, true>(a, g, b, s);
    return hipGetLastError();
}

template <typename T, int NPT>
static hipError_t launch_v(int variant, const StreamArgs<T> &a, int grid, hipStream_t s)
{
    dim3 g(grid), b(64);
    switch (variant) {
    case SV_SWEEP: hipLaunchKernelGGL((k_stream<T, NPT, SV_SWEEP>), g, b, 0, s, a); break;
    case SV_SWEEP_ZX: hipLaunchKernelGGL((k_stream<T, NPT, SV_SWEEP_ZX>), g, b, 0, s, a); break;
    case SV_SWEEP_RQ: hipLaunchKernelGGL((k_stream<T, NPT, SV_SWEEP_RQ>), g, b, 0, s, a); break;
    case SV_SWEEP_RQ_ZX: hipLaunchKernelGGL((k_stream<T, NPT, SV_SWEEP_RQ_ZX>), g, b, 0, s, a); break;
    case SV_INTERP: hipLaunchKernelGGL((k_stream<T, NPT, SV_INTERP>), g, b, 0, s, a); break;
    case SV_INTERP_NORM: hipLaunchKernelGGL((k_stream<T, NPT, SV_INTERP_NORM>), g, b, 0, s, a); break;
    case SV_SWEEP_NORM: hipLaunchKernelGGL((k_stream<T, NPT, SV_SWEEP_NORM>), g, b, 0, s, a); break;
    case SV_SWEEP2_RQ: hipLaunchKernelGGL((k_stream2<T, NPT, false>), g, b, 0, s, a); break;
    case SV_SWEEP2_RQ_ZX: hipLaunchKernelGGL((k_stream2<T, NPT, true>), g, b, 0, s, a); break;
    case SV_SWEEP2_R: hipLaunchKernelGGL((k_stream2<T, NPT, false, false>), g, b, 0, s, a); break;
    case SV_SWEEP2_R_ZX:
        // a.zexc on a 9-point level: the deep vertices' diagonal is formed (ZC9)
        if (NPT == 9 && a.zexc) hipLaunchKernelGGL((k_stream2<T, NPT, true, false, NPT == 9>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_stream2<T, NPT, true, false>), g, b, 0, s, a);
        break;
    case SV_INTERP_RC:
        if (NPT == 9 && a.zexc) hipLaunchKernelGGL((k_interp_rc<T, NPT, NPT == 9>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_interp_rc<T, NPT>), g, b, 0, s, a);
        break;
    case SV_FUSED3:
    case SV_FUSED3_P:
    case SV_FUSED3_PN:
        if (NPT != 5) return hipErrorInvalidValue;
        return launch_fused3<T>(variant, a, g, b, s);
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// device function of one single-problem streaming variant (nullptr if none)
template <typename T, int NPT>
static const void *kernel_of(int variant)
{
    switch (variant) {
    case SV_SWEEP: return reinterpret_cast<const void *>(&k_stream<T, NPT, SV_SWEEP>);
    case SV_SWEEP_ZX: return reinterpret_cast<const void *>(&k_stream<T, NPT, SV_SWEEP_ZX>);
    case SV_SWEEP_RQ: return reinterpret_cast<const void *>(&k_stream<T, NPT, SV_SWEEP_RQ>);
    case SV_SWEEP_RQ_ZX: return reinterpret_cast<const void *>(&k_stream<T, NPT, SV_SWEEP_RQ_ZX>);
    case SV_INTERP: return reinterpret_cast<const void *>(&k_stream<T, NPT, SV_INTERP>);
    case SV_INTERP_NORM: return reinterpret_cast<const void *>(&k_stream<T, NPT, SV_INTERP_NORM>);
    case SV_SWEEP_NORM: return reinterpret_cast<const void *>(&k_stream<T, NPT, SV_SWEEP_NORM>);
    case SV_SWEEP2_RQ: return reinterpret_cast<const void *>(&k_stream2<T, NPT, false>);
    case SV_SWEEP2_RQ_ZX: return reinterpret_cast<const void *>(&k_stream2<T, NPT, true>);
    case SV_SWEEP2_R: return reinterpret_cast<const void *>(&k_stream2<T, NPT, false, false>);
    case SV_SWEEP2_R_ZX: return reinterpret_cast<const void *>(&k_stream2<T, NPT, true, false>);
    case SV_INTERP_RC: return reinterpret_cast<const void *>(&k_interp_rc<T, NPT>);
    case SV_FUSED3: return NPT == 5 ? reinterpret_cast<const void *>(&k_stream3<T, false>) : nullptr;
    case SV_FUSED3_P: return NPT == 5 ? reinterpret_cast<const void *>(&k_stream3<T, true>) : nullptr;
    case SV_FUSED3_PN: return NPT == 5 ? reinterpret_cast<const void *>(&k_stream3<T, true, true>) : nullptr;
    default: return nullptr;
    }
}

int stream_resident(int npt, int variant, int fp32)
{
    const void *k = nullptr;
    if (fp32)
        k = npt == 9 ? kernel_of<float, 9>(variant) : kernel_of<float, 5>(variant);
    else
        k = npt == 9 ? kernel_of<double, 9>(variant) : kernel_of<double, 5>(variant);
    int dev = 0, ncu = 0, per = 0;
    if (!k || hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    // the answer depends only on the kernel and the device: kept after the
    // first query (a handle's setup asks for many levels and variants)
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, int> cache;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find({dev, k});
        if (it != cache.end()) return it->second;
    }
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, 64, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    std::lock_guard<std::mutex> g(mu);
    cache[{dev, k}] = ncu * per;
    return ncu * per;
}

int stream_steps_per_tile(int variant, int rb)
{
    switch (variant) {
    case SV_FUSED3: return rb + 6;
    case SV_FUSED3_P: return rb + 1;
    case SV_FUSED3_PN: return rb + 2;
    case SV_SWEEP2_RQ:
    case SV_SWEEP2_RQ_ZX:
    case SV_SWEEP2_R:
    case SV_SWEEP2_R_ZX: return rb + 4;
    case SV_SWEEP_RQ:
    case SV_SWEEP_RQ_ZX:
    case SV_INTERP_NORM:
    case SV_SWEEP_NORM: return rb + 2;
    default: return rb + 1;
    }
}

template <typename T>
hipError_t launch_stream(int npt, int variant, const StreamArgs<T> &a, int grid, hipStream_t s)
{
    if (npt == 5) return launch_v<T, 5>(variant, a, grid, s);
    if (npt == 9) return launch_v<T, 9>(variant, a, grid, s);
    return hipErrorInvalidValue;
}

template <typename T, int NPT, int W>
static hipError_t launch_vb(int variant, const StreamArgs<T> *args, const int2 *map, int nmap,
                            const int *active, hipStream_t s)
{
    dim3 g((nmap + W - 1) / W), b(64 * W);
    switch (variant) {
#define HB_CASE(V)                                                                                    \
    case V: hipLaunchKernelGGL((k_stream_batched<T, NPT, V, W>), g, b, 0, s, args, map, nmap, active); break;
    HB_CASE(SV_SWEEP)
    HB_CASE(SV_SWEEP_ZX)
    HB_CASE(SV_SWEEP_RQ)
    HB_CASE(SV_SWEEP_RQ_ZX)
    HB_CASE(SV_INTERP)
    HB_CASE(SV_INTERP_NORM)
    HB_CASE(SV_SWEEP_NORM)
    HB_CASE(SV_SWEEP2_RQ)
    HB_CASE(SV_SWEEP2_RQ_ZX)
#undef HB_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_stream_batched(int npt, int variant, const StreamArgs<T> *args, const int2 *map,
                                 int nmap, const int *active, int wpg, hipStream_t s)
{
    if (nmap <= 0) return hipSuccess;
#define HB_W(W)                                                                          \
    if (wpg == W) {                                                                      \
        if (npt == 5) return launch_vb<T, 5, W>(variant, args, map, nmap, active, s);    \
        if (npt == 9) return launch_vb<T, 9, W>(variant, args, map, nmap, active, s);    \
        return hipErrorInvalidValue;                                                     \
    }
    HB_W(1)
    HB_W(2)
    HB_W(4)
#undef HB_W
    return hipErrorInvalidValue;
}
template hipError_t launch_stream_batched<double>(int, int, const StreamArgs<double> *, const int2 *,
                                                  int, const int *, int, hipStream_t);
template hipError_t launch_stream_batched<float>(int, int, const StreamArgs<float> *, const int2 *, int,
                                                 const int *, int, hipStream_t);

template hipError_t launch_stream<double>(int, int, const StreamArgs<double> &, int, hipStream_t);
template hipError_t launch_stream<float>(int, int, const StreamArgs<float> &, int, hipStream_t);

// The pipelined finest pass over many problems: map[w] = (problem, tile) of
// wave w as in k_stream_batched.  active may be null (the rebuild of every
// stopped problem's iterate after the cycles).
template <typename T, bool PONLY, bool ZC, int W>
__global__ __launch_bounds__(64 * W) void k_stream3_batched(const StreamArgs<T> *__restrict__ args,
                                                            const int2 *__restrict__ map, int nmap,
                                                            const int *__restrict__ active)
{
    const int w = (int)blockIdx.x * W + (int)(threadIdx.x >> 6);
    if (w >= nmap) return;
    const int2 m = map[w];
    if (active && !active[m.x]) return;
    const StreamArgs<T> a = args[m.x];
    stream3_tile<T, PONLY, false, ZC, false>(a, m.y);
}

template <typename T, bool PONLY, bool ZC>
static hipError_t launch_s3b(const StreamArgs<T> *args, const int2 *map, int nmap, const int *active, int wpg,
                             hipStream_t s)
{
    switch (wpg) {
    case 1: hipLaunchKernelGGL((k_stream3_batched<T, PONLY, ZC, 1>), dim3(nmap), dim3(64), 0, s, args, map, nmap, active); break;
    case 2: hipLaunchKernelGGL((k_stream3_batched<T, PONLY, ZC, 2>), dim3((nmap + 1) / 2), dim3(128), 0, s, args, map, nmap, active); break;
    case 4: hipLaunchKernelGGL((k_stream3_batched<T, PONLY, ZC, 4>), dim3((nmap + 3) / 4), dim3(256), 0, s, args, map, nmap, active); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_stream3_batched(int variant, int zc, const StreamArgs<T> *args, const int2 *map, int nmap,
                                  const int *active, int wpg, hipStream_t s)
{
    if (nmap <= 0) return hipSuccess;
    if (variant == SV_FUSED3)
        return zc ? launch_s3b<T, false, true>(args, map, nmap, active, wpg, s)
                  : launch_s3b<T, false, false>(args, map, nmap, active, wpg, s);
    if (variant == SV_FUSED3_P)
        return zc ? launch_s3b<T, true, true>(args, map, nmap, active, wpg, s)
                  : launch_s3b<T, true, false>(args, map, nmap, active, wpg, s);
    return hipErrorInvalidValue;
}
template hipError_t launch_stream3_batched<double>(int, int, const StreamArgs<double> *, const int2 *, int,
                                                   const int *, int, hipStream_t);
template hipError_t launch_stream3_batched<float>(int, int, const StreamArgs<float> *, const int2 *, int,
                                                  const int *, int, hipStream_t);

// ---------------------------------------------------------------------------
// Tile kernels for the small coarse levels (9-point, V(2,1)).  On levels too
// small to fill the device a streaming wave's time is its chain of row-pair
// steps (one memory round trip and four dependent colour updates each, plus
// the prologue steps).  Here a workgroup of NW waves loads a whole tile at
// once: the strip's 64 lanes of column pairs by NW * 4 rows, four consecutive
// rows per wave.  A relaxation is then two phases, because on a 9-point
// stencil the even rows (colours 0 and 1) depend only on the odd rows and the
// odd rows (colours 2 and 3) only on the even rows: every wave relaxes its
// even rows, the waves swap the rows at their edges through LDS and meet at
// a barrier, then the odd rows.  Each point is updated by the same
// expressions (res_even / res_odd, interpolation, restriction) from the same
// values as in the colour-by-colour sweep, so the results are bitwise those
// of the streaming kernels.  Rows at the tile's edges see missing
// neighbours and are recomputed by the neighbouring tiles: a down tile owning
// row-pair steps [s0, s1) loads rows 2 s0 - 6 .. 2 s1 + 3, an up tile rows
// 2 s0 - 2 .. 2 s1 + 1; columns have the streaming kernels' halo lanes.
// ---------------------------------------------------------------------------
constexpr int TILE_RPW = 4;   // rows per wave

int tile_steps(int nw, int down) { return down ? (nw * TILE_RPW - 10) / 2 : (nw * TILE_RPW - 4) / 2; }

int tile_owned_pairs(int npt, int down)
{
    return down ? stream_owned_pairs(npt, SV_SWEEP2_RQ_ZX) : stream_owned_pairs(npt, SV_INTERP);
}

void tile_geometry(int nx, int ny, int npt, int nw, int down, int *nstrips, int *nblocks, int *ntiles)
{
    const int own = tile_owned_pairs(npt, down), r = tile_steps(nw, down);
    *nstrips = ((nx + 1) / 2 + own - 1) / own;
    *nblocks = ((ny - 1) / 2 + r - 1) / r;
    *ntiles = *nstrips * *nblocks;
}

template <typename T>
__device__ __forceinline__ void tile_relax_row(const Row<T> &bl, Row<T> &cu, const Row<T> &ab, int j,
                                               const LaneCtx &L)
{
    const bool rj = j >= 1 && j <= L.ny - 2;
    T d;
    T r = res_even<T, 9>(bl, cu, ab, d);
    if (rj && L.ie) cu.x0 += r / d;
    r = res_odd<T, 9>(bl, cu, ab, d);
    if (rj && L.io) cu.x1 += r / d;
}

template <typename T>
__device__ __forceinline__ void tile_load_row(Row<T> &r, int j, bool with_x, const LaneCtx &L, bool colv,
                                              const StreamArgs<T> &a)
{
    r = Row<T>{};
    if (colv && j >= 0 && j < L.ny) {
        const size_t off = (size_t)j * L.pitch + L.e;
        if (with_x) ld2(a.x_in + off, r.x0, r.x1);
        ld2(a.b + off, r.b0, r.b1);
        ld2(a.C + off, r.C0, r.C1);
        ld2(a.W + off, r.W0, r.W1);
        ld2(a.S + off, r.S0, r.S1);
        ld2(a.SW + off, r.SW0, r.SW1);
        ld2(a.SE + off, r.SE0, r.SE1);
    }
}

// the connections of row j that the row below reads (S, SW, SE)
template <typename T>
__device__ __forceinline__ void tile_load_above(Row<T> &r, int j, const LaneCtx &L, bool colv,
                                                const StreamArgs<T> &a)
{
    r = Row<T>{};
    if (colv && j >= 0 && j < L.ny) {
        const size_t off = (size_t)j * L.pitch + L.e;
        ld2(a.S + off, r.S0, r.S1);
        ld2(a.SW + off, r.SW0, r.SW1);
        ld2(a.SE + off, r.SE0, r.SE1);
    }
}

// Two relaxations from x = 0, residual, r/C and restriction onto the coarse
// right-hand side (the down leg of a coarse level; stream2_tile's work).
template <typename T, int NW>
__global__ __launch_bounds__(64 * NW) void k_tile_down(StreamArgs<T> a)
{
    constexpr int NPT = 9;
    constexpr int HA = 1 + (NPT == 9);
    constexpr int HL = HA + halo_left(NPT, 1);
    constexpr int HR = HA + halo_right(NPT, 0);
    constexpr int OWN = 64 - HL - HR;
    constexpr int R = (NW * TILE_RPW - 10) / 2;
    __shared__ T xs[2][NW][64][2];   // x of each wave's first [0] and last [1] row
    __shared__ T rs[NW][64][2];      // residual of each wave's last row
    if (a.active && *a.active == 0) return;
    const int tile = blockIdx.x;
    if (tile >= a.ntiles) return;
    const int strip = tile % a.nstrips, blk = tile / a.nstrips;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int t = strip * OWN + lane - HL;
    const int e = 2 * t, o = 2 * t + 1;
    const int nx = a.nx, ny = a.ny, pitch = a.pitch;
    const bool colv = t >= 0 && e < nx;
    const bool own = lane >= HL && lane < 64 - HR && colv;
    const bool ie = e >= 1 && e <= nx - 2;
    const bool io = o >= 1 && o <= nx - 2;
    const bool cv = t >= 0 && t < a.cnx;
    const LaneCtx L{t, e, o, pitch, ny, own, ie, io, cv};
    const int nsteps = (ny - 1) / 2;
    const int s0 = blk * R, s1 = min(s0 + R, nsteps);
    const int jw0 = 2 * s0 - 6 + TILE_RPW * w;

    Row<T> rw[TILE_RPW], up;
#pragma unroll
    for (int k = 0; k < TILE_RPW; ++k) tile_load_row(rw[k], jw0 + k, false, L, colv, a);
    tile_load_above(up, jw0 + TILE_RPW, L, colv, a);
    if (w == NW - 1) up = Row<T>{};   // the row above the tile is not loaded
    // the restriction weights of coarse rows jw0/2 - 1 .. jw0/2 + 1, loaded
    // with the rows so that their latency overlaps the relaxations
    T wxl[2], wxr[2], wyb[2], wcsw[2], wcse[2], wyt[2], wcnw[2], wcne[2];
    {
        const long long cp = a.cplane;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int jc = (jw0 >> 1) + h;
            wxl[h] = wxr[h] = wyb[h] = wcsw[h] = wcse[h] = wyt[h] = wcnw[h] = wcne[h] = T(0);
            if (cv && jc >= 0 && jc <= a.cny - 1) {
                const size_t co = (size_t)jc * a.cpitch + t;
                wxl[h] = a.wt[WXL * cp + co];
                wxr[h] = a.wt[WXR * cp + co];
                wyb[h] = a.wt[WYB * cp + co];
                wcsw[h] = a.wt[WCSW * cp + co];
                wcse[h] = a.wt[WCSE * cp + co];
            }
            if (cv && jc - 1 >= 0 && jc - 1 <= a.cny - 1) {
                const size_t co = (size_t)(jc - 1) * a.cpitch + t;
                wyt[h] = a.wt[WYT * cp + co];
                wcnw[h] = a.wt[WCNW * cp + co];
                wcne[h] = a.wt[WCNE * cp + co];
            }
        }
    }
    auto below = [&](bool zero) {
        Row<T> r{};
        if (w > 0 && !zero) {
            r.x0 = xs[1][w - 1][lane][0];
            r.x1 = xs[1][w - 1][lane][1];
        }
        return r;
    };
    auto above = [&]() {
        Row<T> r = up;
        if (w < NW - 1) {
            r.x0 = xs[0][w + 1][lane][0];
            r.x1 = xs[0][w + 1][lane][1];
        }
        return r;
    };
#pragma unroll
    for (int sweep = 0; sweep < 2; ++sweep) {
        {   // even rows: colours 0 and 1 (the first sweep starts from x = 0)
            const Row<T> b0 = below(sweep == 0);
            tile_relax_row(b0, rw[0], rw[1], jw0, L);
            tile_relax_row(rw[1], rw[2], rw[3], jw0 + 2, L);
            xs[0][w][lane][0] = rw[0].x0;
            xs[0][w][lane][1] = rw[0].x1;
        }
        __syncthreads();
        {   // odd rows: colours 2 and 3
            tile_relax_row(rw[0], rw[1], rw[2], jw0 + 1, L);
            const Row<T> a3 = above();
            tile_relax_row(rw[2], rw[3], a3, jw0 + 3, L);
            xs[1][w][lane][0] = rw[3].x0;
            xs[1][w][lane][1] = rw[3].x1;
        }
        __syncthreads();
    }
    // residuals of the final rows, zero outside the interior
    T res_e[TILE_RPW], res_o[TILE_RPW], dg_e[TILE_RPW], dg_o[TILE_RPW];
    {
        const Row<T> b0 = below(false), a3 = above();
#pragma unroll
        for (int k = 0; k < TILE_RPW; ++k) {
            const Row<T> &bl = k == 0 ? b0 : rw[k - 1];
            const Row<T> &ab = k == TILE_RPW - 1 ? a3 : rw[k + 1];
            res_e[k] = res_even<T, NPT>(bl, rw[k], ab, dg_e[k]);
            res_o[k] = res_odd<T, NPT>(bl, rw[k], ab, dg_o[k]);
            const int j = jw0 + k;
            const bool rr = j >= 1 && j <= ny - 2;
            if (!(rr && ie)) res_e[k] = T(0);
            if (!(rr && io)) res_o[k] = T(0);
        }
    }
    rs[w][lane][0] = res_e[TILE_RPW - 1];
    rs[w][lane][1] = res_o[TILE_RPW - 1];
    // the iterate and r/C of the rows this tile owns
    if (own) {
#pragma unroll
        for (int k = 0; k < TILE_RPW; ++k) {
            const int j = jw0 + k;
            if (j >= 2 * s0 + 1 && j <= 2 * s1 && j >= 1 && j <= ny - 2)
                st2(a.x_out + (size_t)j * pitch + e, rw[k].x0, rw[k].x1);
            if (j >= 2 * s0 && j <= 2 * s1 - 1 && j >= 1 && j <= ny - 2) {
                if ((k & 1) == 0) {
                    if (io) a.q_out[(size_t)j * pitch + o] = res_o[k] / dg_o[k];
                } else {
                    st2(a.q_out + (size_t)j * pitch + e, ie ? res_e[k] / dg_e[k] : T(0),
                        io ? res_o[k] / dg_o[k] : T(0));
                }
            }
        }
    }
    __syncthreads();
    // restriction onto coarse rows jw0/2 and jw0/2 + 1: fine rows 2jc-1, 2jc, 2jc+1
    T r3e = w > 0 ? rs[w - 1][lane][0] : T(0), r3o = w > 0 ? rs[w - 1][lane][1] : T(0);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int jc = (jw0 >> 1) + h;
        const int k = 2 * h;                       // row 2jc is rw[k], 2jc+1 is rw[k+1]
        const T xl = wxl[h], xr = wxr[h], yb = wyb[h], csw = wcsw[h], cse = wcse[h];
        const T ytp = wyt[h], cnwp = wcnw[h], cnep = wcne[h];
        const T ae = res_e[k], ao = res_o[k], be = res_e[k + 1], bo = res_o[k + 1];
        T lxr = fromL(xr), lcse = fromL(cse), lcnep = fromL(cnep);
        T lao = fromL(ao), lbo = fromL(bo), lr3o = fromL(r3o);
        T bcv = ae + xl * ao + lxr * lao + yb * be + ytp * r3e + csw * bo + lcse * lbo + cnwp * r3o +
                lcnep * lr3o;
        if (own && jc >= s0 && jc < s1 && jc >= 1 && jc <= a.cny - 2 && t >= 1 && t <= a.cnx - 2)
            a.bc[(size_t)jc * a.cpitch + t] = bcv;
        r3e = be;
        r3o = bo;
    }
}

// Interpolate and correct (x += P x_c + r/C), then one relaxation (the up
// leg of a coarse level with one post-relaxation; stream_tile's SV_INTERP).
template <typename T, int NW>
__global__ __launch_bounds__(64 * NW) void k_tile_up(StreamArgs<T> a)
{
    constexpr int NPT = 9;
    constexpr int HL = halo_left(NPT, 0);
    constexpr int HR = halo_right(NPT, 1);
    constexpr int OWN = 64 - HL - HR;
    constexpr int R = (NW * TILE_RPW - 4) / 2;
    __shared__ T xs[2][NW][64][2];
    if (a.active && *a.active == 0) return;
    const int tile = blockIdx.x;
    if (tile >= a.ntiles) return;
    const int strip = tile % a.nstrips, blk = tile / a.nstrips;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int t = strip * OWN + lane - HL;
    const int e = 2 * t, o = 2 * t + 1;
    const int nx = a.nx, ny = a.ny, pitch = a.pitch;
    const bool colv = t >= 0 && e < nx;
    const bool own = lane >= HL && lane < 64 - HR && colv;
    const bool ie = e >= 1 && e <= nx - 2;
    const bool io = o >= 1 && o <= nx - 2;
    const bool cv = t >= 0 && t < a.cnx;
    const LaneCtx L{t, e, o, pitch, ny, own, ie, io, cv};
    const int nsteps = (ny - 1) / 2;
    const int s0 = blk * R, s1 = min(s0 + R, nsteps);
    const int jw0 = 2 * s0 - 2 + TILE_RPW * w;

    Row<T> rw[TILE_RPW], up;
#pragma unroll
    for (int k = 0; k < TILE_RPW; ++k) {
        Row<T> &r = rw[k];
        const int j = jw0 + k;
        tile_load_row(r, j, true, L, colv, a);
        // the interpolation's inputs, as the streaming up leg loads them
        const bool rin = j >= 1 && j <= ny - 2;
        if (cv && rin) {
            const int jc = j >> 1;
            const size_t co = (size_t)jc * a.cpitch + t;
            const T *wt = a.wt;
            const long long cp = a.cplane;
            r.ca = a.xc[co];
            if (j & 1) {
                r.cu = a.xc[co + a.cpitch];
                r.w0 = wt[WYB * cp + co];
                r.w1 = wt[WYT * cp + co];
                r.w2 = wt[WCSW * cp + co];
                r.w3 = wt[WCSE * cp + co];
                r.w4 = wt[WCNW * cp + co];
                r.w5 = wt[WCNE * cp + co];
            } else {
                r.w0 = wt[WXL * cp + co];
                r.w1 = wt[WXR * cp + co];
            }
            if (a.rescorr) ld2(a.q_in + (size_t)j * pitch + e, r.q0, r.q1);
        }
    }
    tile_load_above(up, jw0 + TILE_RPW, L, colv, a);
    if (w == NW - 1) up = Row<T>{};
    // x += P x_c (+ r/C at fine-only vertices)
#pragma unroll
    for (int k = 0; k < TILE_RPW; ++k) {
        Row<T> &r = rw[k];
        const int j = jw0 + k;
        const bool rin = j >= 1 && j <= ny - 2;
        if ((j & 1) == 0) {
            const T xb = fromR(r.ca);
            if (rin && ie) r.x0 += r.ca;
            if (rin && io) r.x1 += r.w0 * r.ca + r.w1 * xb + r.q1;
        } else {
            const T xb = fromR(r.ca), xd = fromR(r.cu);
            if (rin && ie) r.x0 += r.w0 * r.ca + r.w1 * r.cu + r.q0;
            if (rin && io) r.x1 += r.w2 * r.ca + r.w3 * xb + r.w4 * r.cu + r.w5 * xd + r.q1;
        }
    }
    xs[0][w][lane][0] = rw[0].x0;
    xs[0][w][lane][1] = rw[0].x1;
    xs[1][w][lane][0] = rw[TILE_RPW - 1].x0;
    xs[1][w][lane][1] = rw[TILE_RPW - 1].x1;
    __syncthreads();
    {   // even rows
        Row<T> b0{};
        if (w > 0) {
            b0.x0 = xs[1][w - 1][lane][0];
            b0.x1 = xs[1][w - 1][lane][1];
        }
        tile_relax_row(b0, rw[0], rw[1], jw0, L);
        tile_relax_row(rw[1], rw[2], rw[3], jw0 + 2, L);
        // first rows are read again only in the odd phase
        xs[0][w][lane][0] = rw[0].x0;
        xs[0][w][lane][1] = rw[0].x1;
    }
    __syncthreads();
    {   // odd rows
        tile_relax_row(rw[0], rw[1], rw[2], jw0 + 1, L);
        Row<T> a3 = up;
        if (w < NW - 1) {
            a3.x0 = xs[0][w + 1][lane][0];
            a3.x1 = xs[0][w + 1][lane][1];
        }
        tile_relax_row(rw[2], rw[3], a3, jw0 + 3, L);
    }
    if (own) {
#pragma unroll
        for (int k = 0; k < TILE_RPW; ++k) {
            const int j = jw0 + k;
            if (j >= 2 * s0 + 1 && j <= 2 * s1 && j >= 1 && j <= ny - 2)
                st2(a.x_out + (size_t)j * pitch + e, rw[k].x0, rw[k].x1);
        }
    }
}

template <typename T>
hipError_t launch_tile(int down, int nw, const StreamArgs<T> &a, hipStream_t s)
{
    if (a.ntiles <= 0) return hipSuccess;
    if (nw == 8) {
        if (down) hipLaunchKernelGGL((k_tile_down<T, 8>), dim3(a.ntiles), dim3(512), 0, s, a);
        else hipLaunchKernelGGL((k_tile_up<T, 8>), dim3(a.ntiles), dim3(512), 0, s, a);
    } else if (nw == 4) {
        if (down) hipLaunchKernelGGL((k_tile_down<T, 4>), dim3(a.ntiles), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_tile_up<T, 4>), dim3(a.ntiles), dim3(256), 0, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template hipError_t launch_tile<double>(int, int, const StreamArgs<double> &, hipStream_t);
template hipError_t launch_tile<float>(int, int, const StreamArgs<float> &, hipStream_t);

}  // namespace hbmg
