// bmg_host.hip -- host runtime of hipbmg: hierarchy construction, the V-cycle
// launch plan, the collapse-level performance model, the FP64 and mixed
// precision solve drivers, and the C interface declared in include/hipbmg.h.
#include "hipbmg.h"
#include "bmg_internal.h"
#include "bmg_misc.h"
#include "bmg_model.h"

#include <atomic>
#include <thread>
#include <algorithm>
#include <map>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

using namespace hbmg;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static hipbmg_status fail(hipbmg_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(call)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(HIPBMG_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));        \
    } while (0)

#define STCHK(call)                                                                         \
    do {                                                                                    \
        hipbmg_status s_ = (call);                                                          \
        if (s_ != HIPBMG_OK) return s_;                                                     \
    } while (0)

extern "C" const char *hipbmg_last_error(void) { return g_err.c_str(); }

// the message of the calling thread's last failure, for the other entry-point files
void hbmg::set_last_error(const char *msg) { g_err = msg; }

// ---------------------------------------------------------------------------
// handle memory: the caller's allocator, or hipMalloc
// ---------------------------------------------------------------------------
namespace {
struct BlockOwner {
    hipbmg_free_fn fn;
    void *ctx;
};
std::mutex g_alloc_mu;
hipbmg_alloc_fn g_alloc_fn = nullptr;
hipbmg_free_fn g_free_fn = nullptr;
void *g_alloc_ctx = nullptr;
std::unordered_map<void *, BlockOwner> g_blocks;   // blocks made by a registered allocator
}  // namespace

hipError_t hbmg::dev_malloc(void **p, size_t bytes)
{
    hipbmg_alloc_fn fa;
    hipbmg_free_fn ff;
    void *ctx;
    {
        std::lock_guard<std::mutex> g(g_alloc_mu);
        fa = g_alloc_fn;
        ff = g_free_fn;
        ctx = g_alloc_ctx;
    }
    if (!fa) return hipMalloc(p, bytes);
    void *q = fa(bytes, ctx);
    if (!q) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    if (reinterpret_cast<uintptr_t>(q) % 256 != 0) {   // the kernels assume 256-byte aligned planes
        ff(q, ctx);
        *p = nullptr;
        return hipErrorInvalidValue;
    }
    {
        std::lock_guard<std::mutex> g(g_alloc_mu);
        g_blocks[q] = BlockOwner{ff, ctx};
    }
    *p = q;
    return hipSuccess;
}

void hbmg::dev_free_all(std::vector<void *> &v)
{
    std::vector<BlockOwner> own(v.size(), BlockOwner{nullptr, nullptr});
    bool any = false;
    {
        std::lock_guard<std::mutex> g(g_alloc_mu);
        for (size_t k = 0; k < v.size(); ++k) {
            auto it = g_blocks.find(v[k]);
            if (it != g_blocks.end()) {
                own[k] = it->second;
                g_blocks.erase(it);
                any = true;
            }
        }
    }
    if (any) (void)hipDeviceSynchronize();
    for (size_t k = 0; k < v.size(); ++k) {
        if (!v[k]) continue;
        if (own[k].fn) own[k].fn(v[k], own[k].ctx);
        else (void)hipFree(v[k]);
    }
    v.clear();
}

// Small pinned host buffers (a handle's scalars, flags and host-mapped test
// slots) are 512-byte slots of slabs of mapped, coherent pinned memory that
// stay allocated until the process ends: hipHostMalloc and above all
// hipHostFree cost tens to hundreds of microseconds a call, which dominated
// building and destroying the many small handles of a batch.
namespace {
constexpr size_t PIN_SLOT = 512, PIN_SLAB = 256 * PIN_SLOT;
std::mutex g_pin_mu;
std::vector<std::pair<char *, char *>> g_pin_slabs;   // host and device address of each slab
std::vector<char *> g_pin_free;                       // free slots (host addresses)
}  // namespace

hipError_t hbmg::pinned_small(void **host, void **dev, size_t bytes)
{
    if (bytes > PIN_SLOT) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> g(g_pin_mu);
    if (g_pin_free.empty()) {
        void *h = nullptr, *d = nullptr;
        hipError_t e = hipHostMalloc(&h, PIN_SLAB, hipHostMallocMapped | hipHostMallocCoherent);
        if (e != hipSuccess) return e;
        e = hipHostGetDevicePointer(&d, h, 0);
        if (e != hipSuccess) {
            (void)hipHostFree(h);
            return e;
        }
        g_pin_slabs.push_back({static_cast<char *>(h), static_cast<char *>(d)});
        for (size_t k = PIN_SLAB / PIN_SLOT; k-- > 0;) g_pin_free.push_back(static_cast<char *>(h) + k * PIN_SLOT);
    }
    char *p = g_pin_free.back();
    g_pin_free.pop_back();
    std::memset(p, 0, PIN_SLOT);
    *host = p;
    if (dev) {
        *dev = nullptr;
        for (const auto &sl : g_pin_slabs)
            if (p >= sl.first && p < sl.first + PIN_SLAB) *dev = sl.second + (p - sl.first);
    }
    return hipSuccess;
}

void hbmg::pinned_small_free(void *host)
{
    if (!host) return;
    std::lock_guard<std::mutex> g(g_pin_mu);
    g_pin_free.push_back(static_cast<char *>(host));
}

// Larger pinned host buffers (a batch's host tables) are blocks of a power of
// two bytes (at least 4 KiB), kept on per-size free lists for the process.
namespace {
std::map<size_t, std::vector<void *>> g_pin_blocks;   // guarded by g_pin_mu
}  // namespace

hipError_t hbmg::pinned_block(void **host, size_t bytes, size_t *cap)
{
    size_t c = 4096;
    while (c < bytes) c <<= 1;
    *host = nullptr;
    {
        std::lock_guard<std::mutex> g(g_pin_mu);
        std::vector<void *> &v = g_pin_blocks[c];
        if (!v.empty()) {
            *host = v.back();
            v.pop_back();
        }
    }
    if (!*host) {
        const hipError_t e = hipHostMalloc(host, c);
        if (e != hipSuccess) {
            *host = nullptr;
            return e;
        }
    }
    std::memset(*host, 0, c);
    *cap = c;
    return hipSuccess;
}

void hbmg::pinned_block_free(void *host, size_t cap)
{
    if (!host) return;
    std::lock_guard<std::mutex> g(g_pin_mu);
    g_pin_blocks[cap].push_back(host);
}

extern "C" hipbmg_status hipbmg_set_allocator(hipbmg_alloc_fn alloc_fn, hipbmg_free_fn free_fn, void *ctx)
{
    if ((alloc_fn == nullptr) != (free_fn == nullptr)) {
        hbmg::set_last_error("hipbmg_set_allocator: give both functions, or neither");
        return HIPBMG_EINVAL;
    }
    std::lock_guard<std::mutex> g(g_alloc_mu);
    g_alloc_fn = alloc_fn;
    g_free_fn = free_fn;
    g_alloc_ctx = alloc_fn ? ctx : nullptr;
    return HIPBMG_OK;
}

extern "C" void hipbmg_default_params(hipbmg_params *p)
{
    if (!p) return;
    p->nu1 = 2;
    p->nu2 = 1;
    p->coarsest_n = 3;
    p->collapse_level = -1;
    p->residual_correction = 1;
    p->max_cycles = 500;
    p->precision = HIPBMG_FP64;
    p->inner_max_cycles = 32;
    p->inner_tol = 1e-4;
    p->use_graph = 1;
    p->cluster_wg = -1;
    p->cluster_top = -1;
}

// ---------------------------------------------------------------------------
// hierarchy
// ---------------------------------------------------------------------------
constexpr int RING = 8;          // host-mapped convergence-test slots
constexpr int PROF_RING = 256;   // profiling event pairs in flight

struct hipbmg_hier {
    int L = 0, nx = 0, ny = 0, npt = 5;
    hipbmg_params prm{};
    std::vector<LevelDev<double>> lv;
    std::vector<LevelDev<float>> lv32;
    LevelDev<double> *d_lv = nullptr;
    LevelDev<float> *d_lv32 = nullptr;
    std::vector<void *> allocs;
    char *arena = nullptr;        // the unused part of the handle's current zeroed chunk
    size_t arena_left = 0;
    size_t arena_next = size_t(1) << 20;   // size of the next chunk (doubling to 16 MiB)
    double *d_chol = nullptr;
    int *d_cidx = nullptr;
    double *d_work = nullptr;
    int nc = 0;
    double *d_partials = nullptr;
    size_t n_partials = 0;
    double *d_scal = nullptr;   // [0] ||b||, [1] relres, [2] ||r|| (mixed outer), [3] inner relres
    double *h_scal = nullptr;   // pinned mirror
    int lstar = 0;
    // agglomeration stages between the grid-wide kernels and the collapse
    int cl_nstage = 0;
    int cl_wg[CLUSTER_MAX_STAGES] = {}, cl_hi[CLUSTER_MAX_STAGES] = {};
    unsigned *d_bar = nullptr;   // grid barriers of the stages
    int *d_err = nullptr;        // a stage barrier gave up waiting
    double search_us = 0.0;
    int search_expanded = 0;
    double path_us = 0.0;        // model time of one cycle of the configuration in use
    double model_us[HIPBMG_MAX_LEVELS] = {};
    double setup_ms = 0.0;
    std::vector<int> rb;        // row-block steps per level, pre-relaxation (down) kernels
    std::vector<int> rb_up;     // row-block steps per level, interpolation (up) kernels
    std::vector<char> rc_level; // level forms r/C in its up leg (no q plane)
    // the level's two kernels form the diagonal of its deep vertices (FP64 [0],
    // FP32 [1]; only levels with rc_level)
    std::vector<char> zc9[2];
    int zc9_form = 1;           // HIPBMG_ZC9_LOAD=1: keep the stored diagonal but load it (tests)
    int inner_adapt = 1;        // HIPBMG_INNER_ADAPT=0: every inner solve to inner_tol
    // waves per tile of the level's tile kernels, 0 for the streaming kernels:
    // the down leg, and the up leg of the FP64 [0] and FP32 [1] levels
    std::vector<char> tile_dn, tile_up[2];
    int no_lds = 0;             // HIPBMG_NO_LDS=1: keep collapsed levels in global memory
    int no_fuse2 = 0;           // HIPBMG_NO_FUSE2=1: run the two pre-relaxations as two passes
    int fused3 = 0;             // finest post-relaxation fused with the next cycle's pre-relaxations
    int rb3 = 0;                // row-block steps of the pipelined finest kernel
    int zexc[2] = {0, 0};       // the pipelined pass forms the finest diagonal ([0] FP64, [1] FP32)
    int wform = 0;              // the FP64 pipelined pass forms the interpolation weights
    double *x3_64 = nullptr;    // third iterate buffer of the pipelined finest level
    float *x3_32 = nullptr;
    // device-side stopping: run flag, residual history, and a ring of
    // host-mapped slots through which the host sees each cycle's test
    int *d_flags = nullptr;               // [0] run, [1] stopping cycle, [2] reason
    int *h_flags = nullptr;               // pinned mirror of d_flags
    double *d_hist = nullptr;             // relres after each cycle of the current solve
    double *ring_host = nullptr, *ring_dev = nullptr;   // RING x {relres, run, stop, k}
    hipEvent_t ring_ev[RING] = {};
    int ahead = 2;                        // cycles enqueued beyond the last test seen
    // live timing of the finest-level streaming kernels (HIP events on the
    // solve stream), kept in a ring and collected in order once complete
    int prof_on = 0;
    long long prof_head = 0, prof_tail = 0;
    int prof_cycle = 0;                   // cycle being enqueued
    int prof_var[PROF_RING];
    int prof_prec[PROF_RING];
    int prof_cyc[PROF_RING];
    int prof_slot[PROF_RING];             // 3 * level + leg (0 down, 1 up, 2 collapse)
    bool prof_fine[PROF_RING];            // a finest-level streaming kernel
    hipEvent_t ev0[PROF_RING] = {}, ev1[PROF_RING] = {};
    double prof_ms[2][SV_COUNT] = {};
    long long prof_cnt[2][SV_COUNT] = {};
    double lvl_ms[2][3 * HIPBMG_MAX_LEVELS] = {};
    long long lvl_cnt[2][3 * HIPBMG_MAX_LEVELS] = {};
    // the model's inputs at setup (per-level terms are reported from them)
    ModelLevel ml[HIPBMG_MAX_LEVELS] = {};
    ModelParams mp{};
    ~hipbmg_hier()
    {
        for (int k = 0; k < PROF_RING; ++k) {
            if (ev0[k]) (void)hipEventDestroy(ev0[k]);
            if (ev1[k]) (void)hipEventDestroy(ev1[k]);
        }
        for (int k = 0; k < RING; ++k)
            if (ring_ev[k]) (void)hipEventDestroy(ring_ev[k]);
        dev_free_all(allocs);
        // the pinned slots go back to the pool for the next handle: nothing
        // of this handle may still write them
        if (h_scal || h_flags || ring_host) (void)hipDeviceSynchronize();
        pinned_small_free(h_scal);
        pinned_small_free(h_flags);
        pinned_small_free(ring_host);
    }
};

template <typename T> struct PrecIdx { enum { v = 0 }; };
template <> struct PrecIdx<float> { enum { v = 1 }; };

// Record the start of a profiled launch of level `level`, leg 0 (down), 1
// (up) or 2 (collapse, variant -1); returns its ring slot or -1.  Mode 1
// records finest-level streaming kernels only, mode 2 everything.
static int prof_begin(hipbmg_hier *h, int variant, int prec, int level, int leg, bool fine, hipStream_t s)
{
    if (!h->prof_on || (h->prof_on == 1 && !fine) || h->prof_tail - h->prof_head >= PROF_RING) return -1;
    const int k = (int)(h->prof_tail++ % PROF_RING);
    h->prof_var[k] = variant;
    h->prof_prec[k] = prec;
    h->prof_cyc[k] = h->prof_cycle;
    h->prof_slot[k] = 3 * level + leg;
    h->prof_fine[k] = fine;
    (void)hipEventRecord(h->ev0[k], s);
    return k;
}

static void prof_end(hipbmg_hier *h, int k, hipStream_t s)
{
    if (k >= 0) (void)hipEventRecord(h->ev1[k], s);
}

// Collect recorded pairs in order: all of them if `wait`, else those already
// complete.  With `final`, pairs of cycles after `last_cycle` (cycles the
// device skipped once the convergence test was met) are dropped; without it,
// collection stops at the first pair of a cycle after `last_cycle`, whose
// fate is not known yet.
static void prof_collect(hipbmg_hier *h, bool wait, int last_cycle = 1 << 30, bool final = true)
{
    while (h->prof_head < h->prof_tail) {
        const int k = (int)(h->prof_head % PROF_RING);
        if (!final && h->prof_cyc[k] > last_cycle) break;
        if (!wait && hipEventQuery(h->ev1[k]) != hipSuccess) {
            (void)hipGetLastError();
            break;
        }
        float ms = 0.f;
        if (h->prof_cyc[k] <= last_cycle && hipEventElapsedTime(&ms, h->ev0[k], h->ev1[k]) == hipSuccess) {
            const int q = h->prof_prec[k];
            if (h->prof_fine[k] && h->prof_var[k] >= 0) {
                h->prof_ms[q][h->prof_var[k]] += ms;
                h->prof_cnt[q][h->prof_var[k]] += 1;
            }
            h->lvl_ms[q][h->prof_slot[k]] += ms;
            h->lvl_cnt[q][h->prof_slot[k]] += 1;
        }
        (void)hipGetLastError();
        ++h->prof_head;
    }
}

static int pitch_for(int nx) { return (nx + 63) / 64 * 64; }   // >= nx+1 for odd nx

// A handle's device arrays, zeroed, 256-byte aligned and 256 bytes longer than
// asked.  The setup reserves one zeroed block for every array it knows it will
// cut (the levels, the pipelined pass's third iterate and some room for the
// small ones) and cuts them from it in order, so a hierarchy makes one
// allocator call and one fill for them, not one of each per array (each costs
// microseconds of host time, serialised in the runtime when many hierarchies
// are built at once, and the binding's allocator is a Python callback).  An
// array that no longer fits is cut from a chunk zeroed once when taken (1 MiB,
// doubling to 16 MiB) if it is at most 8 MiB, and gets a block of its own if
// larger.
constexpr size_t ARENA_CHUNK = size_t(16) << 20;

static size_t dalloc_bytes(size_t n, size_t elem) { return (n * elem + 256 + 255) / 256 * 256; }

static hipbmg_status arena_reserve(hipbmg_hier *h, size_t bytes, hipStream_t s)
{
    void *q = nullptr;
    if (dev_malloc(&q, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(HIPBMG_ENOMEM, "device allocation of %zu bytes failed", bytes);
    }
    h->allocs.push_back(q);
    HIPCHK(hipMemsetAsync(q, 0, bytes, s));
    h->arena = static_cast<char *>(q);
    h->arena_left = bytes;
    return HIPBMG_OK;
}

template <typename T>
static hipbmg_status dalloc(hipbmg_hier *h, T **p, size_t n, hipStream_t s)
{
    const size_t bytes = dalloc_bytes(n, sizeof(T));
    void *q = nullptr;
    if (bytes > h->arena_left && bytes > ARENA_CHUNK / 2) {
        if (dev_malloc(&q, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(HIPBMG_ENOMEM, "device allocation of %zu bytes failed", n * sizeof(T));
        }
        h->allocs.push_back(q);
        HIPCHK(hipMemsetAsync(q, 0, bytes, s));
        *p = static_cast<T *>(q);
        return HIPBMG_OK;
    }
    if (bytes > h->arena_left) {
        const size_t chunk = std::max(h->arena_next, bytes);
        if (dev_malloc(&q, chunk) != hipSuccess) {
            (void)hipGetLastError();
            return fail(HIPBMG_ENOMEM, "device allocation of %zu bytes failed", chunk);
        }
        h->allocs.push_back(q);
        HIPCHK(hipMemsetAsync(q, 0, chunk, s));
        h->arena = static_cast<char *>(q);
        h->arena_left = chunk;
        h->arena_next = std::min(2 * h->arena_next, ARENA_CHUNK);
    }
    *p = reinterpret_cast<T *>(h->arena);
    h->arena += bytes;
    h->arena_left -= bytes;
    return HIPBMG_OK;
}

// bytes alloc_levels cuts for levels of these sizes
template <typename T>
static size_t levels_bytes(const std::vector<int> &sx, const std::vector<int> &sy)
{
    size_t t = 0;
    for (size_t l = 0; l < sx.size(); ++l) {
        t += dalloc_bytes((size_t)sy[l] * pitch_for(sx[l]) * 9, sizeof(T));
        if (l >= 1) t += dalloc_bytes((size_t)sy[l - 1] * pitch_for(sx[l - 1]) * 8, sizeof(T));
    }
    return t;
}

// grid barriers of the agglomeration stages and their give-up flag (zero)
static hipbmg_status alloc_stage_barriers(hipbmg_hier *h, hipStream_t s)
{
    if (h->d_bar) return HIPBMG_OK;
    hipbmg_status st = dalloc(h, &h->d_bar, 2 * CLUSTER_MAX_STAGES, s);
    if (st == HIPBMG_OK) st = dalloc(h, &h->d_err, 1, s);
    return st;
}


template <typename T>
static hipbmg_status alloc_levels(hipbmg_hier *h, std::vector<LevelDev<T>> &lv,
                                  const std::vector<int> &sx, const std::vector<int> &sy,
                                  hipStream_t s)
{
    const int L = (int)sx.size();
    lv.assign(L, LevelDev<T>{});
    for (int l = 0; l < L; ++l) {
        LevelDev<T> &d = lv[l];
        d.nx = sx[l];
        d.ny = sy[l];
        d.pitch = pitch_for(d.nx);
        d.npt = (l == L - 1) ? h->npt : 9;
        d.plane = (size_t)d.ny * d.pitch;
        T *blk = nullptr;
        STCHK(dalloc(h, &blk, d.plane * 9, s));
        d.C = blk;
        d.W = blk + d.plane;
        d.S = blk + 2 * d.plane;
        d.SW = blk + 3 * d.plane;
        d.SE = blk + 4 * d.plane;
        d.x[0] = blk + 5 * d.plane;
        d.x[1] = blk + 6 * d.plane;
        d.b = blk + 7 * d.plane;
        d.q = blk + 8 * d.plane;
        d.wt = nullptr;
        if (l >= 1) {
            d.cpitch = pitch_for(sx[l - 1]);
            d.cplane = (size_t)sy[l - 1] * d.cpitch;
            STCHK(dalloc(h, &d.wt, d.cplane * 8, s));
        }
    }
    return HIPBMG_OK;
}

// dense Cholesky of the coarsest operator (interior unknowns), on the host
static hipbmg_status factor_coarsest(hipbmg_hier *h, hipStream_t s)
{
    const LevelDev<double> &c = h->lv[0];
    const int nx = c.nx, ny = c.ny;
    std::vector<double> pl(5 * c.plane);
    HIPCHK(hipMemcpyAsync(pl.data(), c.C, 5 * c.plane * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    auto at = [&](int k, int i, int j) { return pl[k * c.plane + (size_t)j * c.pitch + i]; };
    std::vector<int> cidx((size_t)nx * ny, -1);
    int n = 0;
    for (int j = 1; j <= ny - 2; ++j)
        for (int i = 1; i <= nx - 2; ++i) cidx[(size_t)j * nx + i] = n++;
    std::vector<double> M((size_t)n * n, 0.0);
    auto put = [&](int i, int j, int di, int dj, double v) {
        int a = cidx[(size_t)j * nx + i];
        int ii = i + di, jj = j + dj;
        if (ii < 1 || ii > nx - 2 || jj < 1 || jj > ny - 2) return;
        M[(size_t)a * n + cidx[(size_t)jj * nx + ii]] = v;
    };
    for (int j = 1; j <= ny - 2; ++j)
        for (int i = 1; i <= nx - 2; ++i) {
            put(i, j, 0, 0, at(0, i, j));
            put(i, j, -1, 0, -at(1, i, j));
            put(i, j, 1, 0, -at(1, i + 1, j));
            put(i, j, 0, -1, -at(2, i, j));
            put(i, j, 0, 1, -at(2, i, j + 1));
            put(i, j, -1, -1, -at(3, i, j));
            put(i, j, 1, 1, -at(3, i + 1, j + 1));
            put(i, j, 1, -1, -at(4, i, j));
            put(i, j, -1, 1, -at(4, i - 1, j + 1));
        }
    for (int k = 0; k < n; ++k) {
        double d = M[(size_t)k * n + k];
        for (int m = 0; m < k; ++m) d -= M[(size_t)k * n + m] * M[(size_t)k * n + m];
        if (!(d > 0.0)) return fail(HIPBMG_ENOTSPD, "coarsest operator not positive definite (pivot %d)", k);
        d = std::sqrt(d);
        M[(size_t)k * n + k] = d;
        for (int r = k + 1; r < n; ++r) {
            double v = M[(size_t)r * n + k];
            for (int m = 0; m < k; ++m) v -= M[(size_t)r * n + m] * M[(size_t)k * n + m];
            M[(size_t)r * n + k] = v / d;
        }
        for (int r = 0; r < k; ++r) M[(size_t)r * n + k] = 0.0;
    }
    h->nc = n;
    STCHK(dalloc(h, &h->d_chol, (size_t)n * n, s));
    STCHK(dalloc(h, &h->d_cidx, (size_t)nx * ny, s));
    STCHK(dalloc(h, &h->d_work, (size_t)n + 1, s));
    HIPCHK(hipMemcpyAsync(h->d_chol, M.data(), M.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->d_cidx, cidx.data(), cidx.size() * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return HIPBMG_OK;
}

// row-block length of the streaming kernels: long blocks amortise the
// prologue, short blocks give small levels enough waves
static int pick_rb(int nx, int ny, int npt)
{
    int nst, nbl, nt, g;
    for (int rb : {64, 32, 16, 8, 4}) {
        stream_geometry(nx, ny, npt, SV_SWEEP_RQ, rb, &nst, &nbl, &nt, &g);
        if (nt >= 1024) return rb;
    }
    return 4;
}

// Row-block length by residency rounds: a launch of `nt` one-wave workgroups
// on a device that holds `resident` of them at once takes ceil(nt/resident)
// rounds of (steps per tile) row-pair steps each.  The length that minimises
// that product wins; ties go to the longer block (fewer re-read prologue rows).
// the kernel that dominates a level's down leg (its last pre-relaxation, fused
// with residual and restriction) and its up leg (the interpolating relaxation)
static int variant_down(const hipbmg_params &prm, bool fine, bool rc = false)
{
    if (rc) return SV_SWEEP2_R_ZX;
    return prm.nu1 >= 2 ? (fine ? SV_SWEEP2_RQ : SV_SWEEP2_RQ_ZX) : (fine ? SV_SWEEP_RQ : SV_SWEEP_RQ_ZX);
}
static int variant_up(bool fine, bool rc = false) { return fine ? SV_INTERP_NORM : (rc ? SV_INTERP_RC : SV_INTERP); }

// Small coarse levels run the tile kernels instead of the streaming ones:
// 9-point levels of a V(2,1) cycle with the two pre-relaxations fused, up to
// a vertex count per leg and precision where they measured faster on gfx950
// (4097^2 blocks): every down leg up to 513^2 (HIPBMG_TILE_MAX), the up legs
// of FP32 levels up to 257^2 (HIPBMG_TILE_UP_MAX); FP64 up legs stay
// streaming (HIPBMG_TILE_UP_MAX64, default 0).  8-wave tiles where a level
// still gets 64 of them, 4-wave tiles otherwise (HIPBMG_TILE_NW forces one).
static long long tile_limit(const char *env, long long dflt)
{
    if (const char *e = std::getenv(env)) return std::atoll(e);
    return dflt;
}

static int tile_waves(const hipbmg_hier *h, int nx, int ny, int npt, bool fine, bool rc, long long lim)
{
    if (fine || rc || npt != 9 || h->prm.nu1 != 2 || h->prm.nu2 != 1 || h->no_fuse2 || (long long)nx * ny > lim)
        return 0;
    if (const char *e = std::getenv("HIPBMG_TILE_NW")) {
        const int v = std::atoi(e);
        if (v == 4 || v == 8) return v;
    }
    int nst, nbl, nt;
    tile_geometry(nx, ny, npt, 8, 1, &nst, &nbl, &nt);
    return nt >= 64 ? 8 : 4;
}

// Levels whose up leg forms r/C from the rows it loads instead of reading the
// q plane the down leg would store (16 bytes per vertex less): coarse levels
// of at least HIPBMG_RC_MIN vertices (default 2^20, where the two legs are
// bandwidth-bound rather than latency-bound), with the two pre-relaxations
// fused into one pass.
static bool rc_on_the_fly(const hipbmg_hier *h, int nx, int ny, bool fine)
{
    long long lim = 1LL << 20;
    if (const char *e = std::getenv("HIPBMG_RC_MIN")) lim = std::atoll(e);
    return !fine && h->prm.nu1 == 2 && !h->no_fuse2 && (long long)nx * ny >= lim;
}

// The model's view of level l: launch geometry of its down and up kernels and
// whether it is staged in LDS when collapsed (levels fill the LDS budget from
// the coarsest up, as the collapse launch stages them).
static void model_levels(const hipbmg_hier *h, int fp32, ModelLevel *ml)
{
    const int L = h->L;
    size_t used = 0;
    bool fits = !h->no_lds;
    // cache residency: a level's down leg follows the previous cycle's finest
    // pass, so its data is in HBM unless the whole hierarchy fits in the
    // last-level cache; its up leg follows the coarser levels only, so its
    // data is cached if it and every coarser level fit
    const double word = fp32 ? 4.0 : 8.0, cache = h->mp.cache_bytes > 0 ? h->mp.cache_bytes : model_params().cache_bytes;
    std::vector<double> below(L + 1, 0.0);   // footprint of levels 0..l-1
    for (int l = 0; l < L; ++l) {
        const LevelDev<double> &A = h->lv[l];
        const double planes_l = (A.npt == 5 ? 3.0 : 5.0) + 4.0 + (l ? 2.0 : 0.0);
        below[l + 1] = below[l] + (double)A.nx * A.ny * word * planes_l;
    }
    const bool all_fit = below[L] < cache;
    for (int l = 0; l < L; ++l) {
        const LevelDev<double> &A = h->lv[l];
        const bool fine = l == L - 1;
        const int nsteps = (A.ny - 1) / 2;
        ml[l].nx = A.nx;
        ml[l].ny = A.ny;
        ml[l].npt = A.npt;
        // steps per wave, residency rounds, and loaded bytes per algorithmic
        // byte (64 loaded lanes per owned strip; steps walked per owned step)
        auto describe = [&](int variant, int rb, ModelKernel &k) {
            int nst, nbl, nt, g;
            stream_geometry(A.nx, A.ny, A.npt, variant, rb, &nst, &nbl, &nt, &g);
            const int res = stream_resident(A.npt, variant, fp32);
            const int rbe = std::max(1, std::min(rb, nsteps));
            k.steps = stream_steps_per_tile(variant, rbe);
            k.rounds = res > 0 ? (nt + res - 1) / res : 1;
            k.reread = 64.0 / stream_owned_pairs(A.npt, variant) * (double)k.steps / rbe;
        };
        ml[l].dn_cold = all_fit ? 0 : 1;
        ml[l].up_cold = below[l + 1] < cache ? 0 : 1;
        const bool rc = h->rc_level[l] != 0;
        ml[l].rc = rc ? 1 : 0;
        describe(variant_down(h->prm, fine, rc), h->rb[l], ml[l].dn);
        describe(variant_up(fine, rc), h->rb_up[l], ml[l].up);
        ml[l].pipelined = fine && h->fused3 ? 1 : 0;
        if (ml[l].pipelined) describe(SV_FUSED3, h->rb3, ml[l].pipe);
        else ml[l].pipe = ModelKernel{0, 0, 1.0};
        ml[l].zexc = ml[l].pipelined && h->zexc[fp32 ? 1 : 0] ? 1 : 0;
        ml[l].zc9 = rc && h->zc9_form && h->zc9[fp32 ? 1 : 0][l] ? 1 : 0;
        const int cnx = l ? h->lv[l - 1].nx : 0, cny = l ? h->lv[l - 1].ny : 0;
        const size_t bytes = fp32 ? collapse_lds_bytes<float>(A.nx, A.ny, cnx, cny)
                                  : collapse_lds_bytes<double>(A.nx, A.ny, cnx, cny);
        fits = fits && used + bytes <= (size_t)COLLAPSE_LDS_BUDGET;
        if (fits) used += bytes;
        ml[l].in_lds = fits ? 1 : 0;
    }
}

// shortest row block the residency choice may take (HIPBMG_RB_MIN overrides):
// on levels too small to fill the device a wave's time is its sequential
// steps, so one-step blocks (each with its own prologue) are the fastest
static int rb_floor()
{
    if (const char *e = std::getenv("HIPBMG_RB_MIN")) {
        const int k = std::atoi(e);
        if (k >= 1 && k <= 64) return k;
    }
    return 1;
}

static int pick_rb_rounds(int nx, int ny, int npt, int variant, int resident, int rbmax)
{
    const int nsteps = (ny - 1) / 2, lo = rb_floor();
    const int hi = std::max(lo, std::min(rbmax, nsteps));
    int best = hi;
    long long bestc = -1;
    for (int rb = hi; rb >= lo; --rb) {
        int nst, nbl, nt, g;
        stream_geometry(nx, ny, npt, variant, rb, &nst, &nbl, &nt, &g);
        const long long rounds = (nt + resident - 1) / resident;
        const long long c = rounds * stream_steps_per_tile(variant, rb);
        if (bestc < 0 || c < bestc) {
            bestc = c;
            best = rb;
        }
    }
    return best;
}

static double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

extern "C" hipbmg_status hipbmg_setup(int nx, int ny, int npt, const double *coeffs,
                                      const hipbmg_params *params, void *stream,
                                      hipbmg_handle *out)
{
    const double t0 = now_ms();
    if (!out) return fail(HIPBMG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!coeffs) return fail(HIPBMG_EINVAL, "coeffs is NULL");
    if (nx < 3 || ny < 3 || !(nx & 1) || !(ny & 1))
        return fail(HIPBMG_EINVAL, "grid %d x %d: sizes must be odd and >= 3", nx, ny);
    if (npt != 5 && npt != 9) return fail(HIPBMG_EINVAL, "npt must be 5 or 9 (got %d)", npt);
    hipbmg_params prm;
    hipbmg_default_params(&prm);
    if (params) prm = *params;
    if (prm.nu1 < 1 || prm.nu2 < 1 || prm.nu1 > 16 || prm.nu2 > 16)
        return fail(HIPBMG_EINVAL, "nu1 and nu2 must be in [1, 16]");
    if (prm.coarsest_n < 3) return fail(HIPBMG_EINVAL, "coarsest_n must be >= 3");
    if (prm.max_cycles < 1) return fail(HIPBMG_EINVAL, "max_cycles must be >= 1");
    if (prm.precision != HIPBMG_FP64 && prm.precision != HIPBMG_MIXED)
        return fail(HIPBMG_EINVAL, "unknown precision %d", prm.precision);
    if (prm.precision == HIPBMG_MIXED && (prm.inner_max_cycles < 1 || !(prm.inner_tol > 0.0)))
        return fail(HIPBMG_EINVAL, "mixed precision needs inner_max_cycles >= 1 and inner_tol > 0");
    if ((long long)nx * ny > (1LL << 31)) return fail(HIPBMG_EINVAL, "grid too large");
    hipStream_t s = (hipStream_t)stream;

    std::vector<int> sx{nx}, sy{ny};
    // every other vertex is kept; a side with an even number of vertices ends
    // in a boundary vertex at an odd index and cannot be coarsened again
    while (sx.back() > prm.coarsest_n && sy.back() > prm.coarsest_n && (sx.back() & 1) &&
           (sy.back() & 1) && (int)sx.size() < HIPBMG_MAX_LEVELS) {
        sx.push_back((sx.back() + 1) / 2);
        sy.push_back((sy.back() + 1) / 2);
    }
    std::reverse(sx.begin(), sx.end());
    std::reverse(sy.begin(), sy.end());
    const int L = (int)sx.size();
    if (prm.collapse_level >= L)
        return fail(HIPBMG_EINVAL, "collapse_level %d >= number of levels %d", prm.collapse_level, L);
    if ((long long)(sx[0] - 2) * (sy[0] - 2) > 4096)
        return fail(HIPBMG_EINVAL, "coarsest level %d x %d too large for the dense solve", sx[0], sy[0]);

    if (collapse_set_attributes() != hipSuccess)
        return fail(HIPBMG_EHIP, "cannot enable %d bytes of LDS for the collapse kernel", COLLAPSE_LDS_BUDGET);
    hipbmg_hier *h = new hipbmg_hier();
    if (const char *e = std::getenv("HIPBMG_NO_LDS")) h->no_lds = std::atoi(e);
    if (const char *e = std::getenv("HIPBMG_NO_FUSE2")) h->no_fuse2 = std::atoi(e);
    h->L = L;
    h->nx = nx;
    h->ny = ny;
    h->npt = npt;
    h->prm = prm;
    auto bail = [&](hipbmg_status st) {
        delete h;
        return st;
    };
    {
        const bool mixed = prm.precision == HIPBMG_MIXED;
        const size_t fplane = (size_t)ny * pitch_for(nx);
        size_t need = levels_bytes<double>(sx, sy) + (mixed ? levels_bytes<float>(sx, sy) : 0) + (size_t(1) << 20);
        if (npt == 5 && prm.nu1 == 2 && prm.nu2 == 1 && L >= 2)
            need += dalloc_bytes(fplane, sizeof(double)) + (mixed ? dalloc_bytes(fplane, sizeof(float)) : 0);
        const hipbmg_status rs = arena_reserve(h, need, s);
        if (rs != HIPBMG_OK) return bail(rs);
    }
    hipbmg_status st = alloc_levels(h, h->lv, sx, sy, s);
    if (st != HIPBMG_OK) return bail(st);
    // finest operator, as given
    LevelDev<double> &F = h->lv[L - 1];
    const int nplanes = npt == 5 ? 3 : 5;
    if (launch_planes_in(coeffs, nx, ny, nplanes, F.C, F.pitch, F.plane, s) != hipSuccess)
        return bail(fail(HIPBMG_EHIP, "copy of the stencil planes failed"));
    // coarse operators: interpolation weights and Galerkin products.  On the
    // large coarse levels whose up leg forms r/C from its rows, a vertex at
    // least two vertices from the boundary has a zero row sum in exact
    // arithmetic (the Galerkin operator of a pure-diffusion operator); where
    // the computed diagonal agrees with the ordered sum of the connections to
    // 1e-12 at every such vertex, that sum is stored as the diagonal before
    // the level's own weights and Galerkin product are formed, so every later
    // step sees one operator, and the level's streaming kernels form it
    // instead of loading it (HIPBMG_NO_ZC9=1: keep the computed diagonal)
    h->zc9[0].assign(L, 0);
    h->zc9[1].assign(L, 0);
    int no_zc9 = 0;
    if (const char *e = std::getenv("HIPBMG_NO_ZC9")) no_zc9 = std::atoi(e);
    if (const char *e = std::getenv("HIPBMG_ZC9_LOAD")) h->zc9_form = std::atoi(e) ? 0 : 1;
    if (const char *e = std::getenv("HIPBMG_INNER_ADAPT")) h->inner_adapt = std::atoi(e);
    int *d_zflag = nullptr, *d_zf9 = nullptr;
    st = dalloc(h, &d_zflag, 1, s);
    if (st == HIPBMG_OK) st = dalloc(h, &d_zf9, L, s);
    if (st != HIPBMG_OK) return bail(st);
    std::vector<char> zc9_ran(L, 0);
    // the smallest levels (coarse grids of at most SETUP_TAIL_POINTS vertices,
    // none of them forming its diagonal) in one launch (HIPBMG_SETUP_TAIL=0:
    // two launches per level throughout)
    auto zc9_here = [&](const LevelDev<double> &c) {
        return !no_zc9 && c.npt == 9 && rc_on_the_fly(h, c.nx, c.ny, false);
    };
    int l_tail = 0;
    {
        int tail_on = 1;
        if (const char *e = std::getenv("HIPBMG_SETUP_TAIL")) tail_on = std::atoi(e);
        while (tail_on && l_tail + 1 <= L - 1 && l_tail + 1 <= SETUP_TAIL_MAX &&
               (long long)h->lv[l_tail].nx * h->lv[l_tail].ny <= SETUP_TAIL_POINTS && !zc9_here(h->lv[l_tail]))
            ++l_tail;
        if (l_tail < 2) l_tail = 0;   // one level: no launch to save
    }
    for (int l = L - 1; l >= 1; --l) {
        const LevelDev<double> &f = h->lv[l], &c = h->lv[l - 1];
        if (l <= l_tail) {
            if (launch_setup_tail(h->lv.data(), l_tail, s) != hipSuccess)
                return bail(fail(HIPBMG_EHIP, "setup kernel launch failed: %s",
                                 hipGetErrorString(hipGetLastError())));
            break;
        }
        if (launch_interp_weights(f, c.nx, c.ny, f.wt, f.cpitch, f.cplane, s) != hipSuccess ||
            launch_rap(f, c, s) != hipSuccess)
            return bail(fail(HIPBMG_EHIP, "setup kernel launch failed: %s",
                             hipGetErrorString(hipGetLastError())));
        if (zc9_here(c)) {
            // the check, then the store where it passed, both on the device;
            // the outcomes are read back together after the loop
            if (launch_rowsum_diag(c, d_zf9 + (l - 1), 0, s) != hipSuccess ||
                launch_rowsum_diag(c, d_zf9 + (l - 1), 1, s) != hipSuccess)
                return bail(fail(HIPBMG_EHIP, "row-sum diagonal setup failed"));
            zc9_ran[l - 1] = 1;
        }
    }
    if (std::find(zc9_ran.begin(), zc9_ran.end(), 1) != zc9_ran.end()) {
        std::vector<int> ok(L, 0);
        if (hipMemcpyAsync(ok.data(), d_zf9, L * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return bail(fail(HIPBMG_EHIP, "row-sum diagonal setup failed"));
        for (int m = 0; m < L; ++m)
            if (zc9_ran[m]) h->zc9[0][m] = (char)(ok[m] != 0);
    }
    st = dalloc(h, &h->d_lv, L, s);
    if (st != HIPBMG_OK) return bail(st);
    if (hipMemcpyAsync(h->d_lv, h->lv.data(), L * sizeof(LevelDev<double>), hipMemcpyHostToDevice, s) !=
        hipSuccess)
        return bail(fail(HIPBMG_EHIP, "hipMemcpyAsync failed"));
    st = factor_coarsest(h, s);
    if (st != HIPBMG_OK) return bail(st);

    // FP32 edge-form copy of every level for mixed precision
    if (prm.precision == HIPBMG_MIXED) {
        st = alloc_levels(h, h->lv32, sx, sy, s);
        if (st != HIPBMG_OK) return bail(st);
        for (int l = 0; l < L; ++l) {
            int cnx = l ? sx[l - 1] : 0, cny = l ? sy[l - 1] : 0;
            if (launch_demote_level(h->lv[l], h->lv32[l], cnx, cny, s) != hipSuccess)
                return bail(fail(HIPBMG_EHIP, "demote launch failed"));
            if (h->zc9[0][l]) {
                // the FP32 copy's excess at the deep vertices: zero if the
                // stored diagonal is the demotion's own sum of the connections
                int ok = 0;
                if (launch_zero_excess9(h->lv32[l], d_zflag, s) != hipSuccess ||
                    hipMemcpyAsync(&ok, d_zflag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess)
                    return bail(fail(HIPBMG_EHIP, "zero-excess check failed"));
                h->zc9[1][l] = (char)ok;
            }
        }
        st = dalloc(h, &h->d_lv32, L, s);
        if (st != HIPBMG_OK) return bail(st);
        if (hipMemcpyAsync(h->d_lv32, h->lv32.data(), L * sizeof(LevelDev<float>),
                           hipMemcpyHostToDevice, s) != hipSuccess)
            return bail(fail(HIPBMG_EHIP, "hipMemcpyAsync failed"));
    }

    // streaming geometry and reduction scratch
    // Each leg's row block from the residency rounds of the kernel that
    // dominates it (the last pre-relaxation going down, the interpolation
    // coming up), in the precision the cycles run in.  HIPBMG_RB_MODE=fixed
    // takes the longest of 64, 32, ... 4 that still gives 1024 tiles.
    h->rb.resize(L);
    h->rb_up.resize(L);
    h->rc_level.assign(L, 0);
    h->tile_dn.assign(L, 0);
    h->tile_up[0].assign(L, 0);
    h->tile_up[1].assign(L, 0);
    size_t np = 4096;
    {
        bool fixed = false;
        if (const char *e = std::getenv("HIPBMG_RB_MODE")) fixed = std::string(e) == "fixed";
        const int fp32 = prm.precision == HIPBMG_MIXED;
        for (int l = 0; l < L; ++l) {
            const int lnpt = h->lv[l].npt;
            const bool fine = l == L - 1;
            h->rc_level[l] = rc_on_the_fly(h, sx[l], sy[l], fine) ? 1 : 0;
            const bool rcl = h->rc_level[l] != 0;
            h->tile_dn[l] = (char)tile_waves(h, sx[l], sy[l], lnpt, fine, rcl, tile_limit("HIPBMG_TILE_MAX", 513LL * 513));
            h->tile_up[0][l] = (char)tile_waves(h, sx[l], sy[l], lnpt, fine, rcl, tile_limit("HIPBMG_TILE_UP_MAX64", 0));
            h->tile_up[1][l] = (char)tile_waves(h, sx[l], sy[l], lnpt, fine, rcl, tile_limit("HIPBMG_TILE_UP_MAX", 257LL * 257));
            const int vdn = variant_down(prm, fine, h->rc_level[l]), vup = variant_up(fine, h->rc_level[l]);
            const int rdn = fixed ? 0 : stream_resident(lnpt, vdn, fp32);
            const int rup = fixed ? 0 : stream_resident(lnpt, vup, fp32);
            h->rb[l] = rdn > 0 ? pick_rb_rounds(sx[l], sy[l], lnpt, vdn, rdn, 256) : pick_rb(sx[l], sy[l], lnpt);
            h->rb_up[l] = rup > 0 ? pick_rb_rounds(sx[l], sy[l], lnpt, vup, rup, 256) : pick_rb(sx[l], sy[l], lnpt);
            if (const char *e = std::getenv("HIPBMG_RB")) {   // one fixed length everywhere (tuning)
                const int v = std::atoi(e);
                if (v >= 1 && v <= 4096) h->rb[l] = h->rb_up[l] = v;
            }
            if (fine)
                if (const char *e = std::getenv("HIPBMG_RB_FINEST")) {   // tuning override
                    const int v = std::atoi(e);
                    if (v >= 1 && v <= 4096) h->rb[l] = h->rb_up[l] = v;
                }
            if (const char *e = std::getenv("HIPBMG_RB_AT")) {   // tuning override "nx:down:up"
                int anx = 0, adn = 0, aup = 0;
                if (std::sscanf(e, "%d:%d:%d", &anx, &adn, &aup) == 3 && anx == sx[l]) {
                    if (adn >= 1 && adn <= 4096) h->rb[l] = adn;
                    if (aup >= 1 && aup <= 4096) h->rb_up[l] = aup;
                }
            }
            int nst, nbl, nt, g;
            stream_geometry(sx[l], sy[l], lnpt, SV_INTERP_NORM, h->rb_up[l], &nst, &nbl, &nt, &g);
            np = std::max(np, (size_t)nt);
            stream_geometry(sx[l], sy[l], lnpt, SV_SWEEP_NORM, h->rb_up[l], &nst, &nbl, &nt, &g);
            np = std::max(np, (size_t)nt);
        }
    }
    if (npt == 5) {
        // pipelined finest kernel: its row block from the residency rounds of
        // the precision the cycles run in (HIPBMG_RB_FUSED3 overrides)
        const int resident = stream_resident(5, SV_FUSED3, prm.precision == HIPBMG_MIXED);
        h->rb3 = resident > 0 ? pick_rb_rounds(nx, ny, 5, SV_FUSED3, resident, 256) : h->rb[L - 1];
        if (const char *e = std::getenv("HIPBMG_RB_FUSED3")) {
            const int v = std::atoi(e);
            if (v >= 1 && v <= 4096) h->rb3 = v;
        }
        int nst, nbl, nt, g;
        stream_geometry(sx[L - 1], sy[L - 1], npt, SV_FUSED3, h->rb3, &nst, &nbl, &nt, &g);
        np = std::max(np, (size_t)nt);
    }
    np = std::max(np, (size_t)((nx + 255) / 256) * ny);   // refinement residual partials
    h->n_partials = np;
    st = dalloc(h, &h->d_partials, np, s);
    if (st != HIPBMG_OK) return bail(st);
    st = dalloc(h, &h->d_scal, 8, s);
    if (st != HIPBMG_OK) return bail(st);
    if (pinned_small((void **)&h->h_scal, nullptr, 8 * sizeof(double)) != hipSuccess ||
        pinned_small((void **)&h->h_flags, nullptr, 4 * sizeof(int)) != hipSuccess)
        return bail(fail(HIPBMG_ENOMEM, "pinned host allocation failed"));
    // device-side stopping: run flag, residual history, host-mapped test slots
    st = dalloc(h, &h->d_flags, 4, s);
    if (st == HIPBMG_OK) st = dalloc(h, &h->d_hist, HIPBMG_MAX_HIST, s);
    if (st != HIPBMG_OK) return bail(st);
    if (pinned_small((void **)&h->ring_host, (void **)&h->ring_dev, RING * 4 * sizeof(double)) != hipSuccess ||
        !h->ring_dev)
        return bail(fail(HIPBMG_ENOMEM, "host-mapped allocation failed"));
    for (int k = 0; k < RING * 4; ++k) h->ring_host[k] = 0.0;
    if (const char *e = std::getenv("HIPBMG_AHEAD")) {   // cycles enqueued ahead of the last test seen
        const int v = std::atoi(e);
        if (v >= 0 && v < RING) h->ahead = v;
    }

    // finest level pipelined across cycles (5-point finest, V(2,1), finest
    // level not collapsed); HIPBMG_NO_FUSE3=1 disables it
    {
        int nof3 = 0;
        if (const char *e = std::getenv("HIPBMG_NO_FUSE3")) nof3 = std::atoi(e);
        h->fused3 = (!nof3 && !h->no_fuse2 && npt == 5 && prm.nu1 == 2 && prm.nu2 == 1 && L >= 2) ? 1 : 0;
        if (h->fused3) {
            const LevelDev<double> &F = h->lv[L - 1];
            st = dalloc(h, &h->x3_64, F.plane, s);
            if (st == HIPBMG_OK && prm.precision == HIPBMG_MIXED) st = dalloc(h, &h->x3_32, F.plane, s);
            if (st != HIPBMG_OK) return bail(st);
            // a finest operator whose diagonal is exactly the sum of its
            // connections (pure diffusion, as finite volumes build it) need
            // not be loaded by the pipelined pass (HIPBMG_NO_ZEXC=1: always load)
            int noz = 0;
            if (const char *e = std::getenv("HIPBMG_NO_ZEXC")) noz = std::atoi(e);
            if (!noz) {
                int *d_ok = nullptr;
                st = dalloc(h, &d_ok, 2, s);
                if (st != HIPBMG_OK) return bail(st);
                int ok[2] = {0, 0};
                if (launch_zero_excess_check(F, d_ok, s) != hipSuccess ||
                    (prm.precision == HIPBMG_MIXED && launch_zero_excess_check(h->lv32[L - 1], d_ok + 1, s) != hipSuccess) ||
                    hipMemcpyAsync(ok, d_ok, (prm.precision == HIPBMG_MIXED ? 2 : 1) * sizeof(int),
                                   hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess)
                    return bail(fail(HIPBMG_EHIP, "zero-excess check failed"));
                h->zexc[0] = ok[0];
                h->zexc[1] = ok[1];
            }
            // HIPBMG_WFORM=1: the FP64 pass forms the finest level's
            // interpolation weights from the rows it loads instead of reading
            // the stored ones (bitwise the same; 16 B per vertex fewer, but on
            // gfx950 the pass is no faster: its eight extra divisions per lane
            // and step land on a wave that already stalls on dependent
            // arithmetic at one wave per SIMD)
            int wf = 0;
            if (const char *e = std::getenv("HIPBMG_WFORM")) wf = std::atoi(e);
            h->wform = wf ? 1 : 0;
        }
    }
    // collapse level from the performance model (sections 3 and 4)
    ModelLevel *ml = h->ml;
    model_levels(h, prm.precision == HIPBMG_MIXED, ml);
    h->mp = model_params();
    int best = model_choose(ml, L, prm.nu1, prm.nu2, h->nc, prm.precision == HIPBMG_MIXED ? 4 : 8, h->mp,
                            h->model_us);
    // the collapse workgroup indexes a level's planes with 32-bit integers
    int lcap = -1;
    for (int l = 0; l < L; ++l) {
        if (h->lv[l].plane > (size_t)(1 << 30) || 8 * h->lv[l].cplane > (size_t)(1 << 30)) break;
        lcap = l;
    }
    if (prm.collapse_level > lcap)
        return bail(fail(HIPBMG_EINVAL, "collapse_level %d: level too large for one workgroup", prm.collapse_level));
    if (best > lcap) {
        best = 0;
        for (int l = 1; l <= lcap; ++l)
            if (h->model_us[l] < h->model_us[best]) best = l;
    }
    h->lstar = prm.collapse_level >= 0 ? prm.collapse_level : best;
    // agglomeration stages: the redistribution search of section 4 over
    // (level, workgroups), or one forced stage (cluster_wg = 0: neither)
    if (prm.cluster_wg != 0) {
        const int word = prm.precision == HIPBMG_MIXED ? 4 : 8;
        const int res = prm.precision == HIPBMG_MIXED ? cluster_max_resident<float>(COLLAPSE_LDS_BUDGET)
                                                      : cluster_max_resident<double>(COLLAPSE_LDS_BUDGET);
        const int max_wg = std::min(256, res);
        const ModelPath path = model_search(ml, L, prm.nu1, prm.nu2, h->nc, word, h->mp, max_wg, lcap);
        h->search_us = path.t_us;
        h->search_expanded = path.expanded;
        if (prm.cluster_wg >= 2) {
            const int K = prm.cluster_wg, top = prm.cluster_top;
            if (K > 256 || (K & (K - 1)) != 0)
                return bail(fail(HIPBMG_EINVAL, "cluster_wg %d: must be a power of two from 2 to 256", K));
            if (K > max_wg)
                return bail(fail(HIPBMG_EINVAL, "cluster_wg %d: only %d workgroups fit on the device", K, max_wg));
            if (prm.collapse_level < 0 || top <= prm.collapse_level || top > L - 2 || top > lcap)
                return bail(fail(HIPBMG_EINVAL, "cluster_top %d: needs collapse_level < cluster_top <= %d", top,
                                 std::min(L - 2, lcap)));
            h->cl_nstage = 1;
            h->cl_wg[0] = K;
            h->cl_hi[0] = top;
        } else if (prm.cluster_wg == -1 && prm.collapse_level < 0 && std::isfinite(path.t_us)) {
            h->lstar = path.lstar;
            h->cl_nstage = std::min(path.nstage, CLUSTER_MAX_STAGES);
            for (int k = 0; k < h->cl_nstage; ++k) {
                h->cl_wg[k] = path.wg[k];
                h->cl_hi[k] = path.hi[k];
            }
        } else if (prm.cluster_wg != 0 && prm.cluster_wg != -1) {
            return bail(fail(HIPBMG_EINVAL, "cluster_wg %d: must be -1, 0 or a power of two from 2 to 256",
                             prm.cluster_wg));
        }
        // HIPBMG_STAGES="K1:top1,K2:top2,..." forces several stages above a
        // forced collapse level (decreasing workgroups and levels)
        if (const char *e = std::getenv("HIPBMG_STAGES")) {
            if (prm.collapse_level < 0 || prm.cluster_wg != -1)
                return bail(fail(HIPBMG_EINVAL, "HIPBMG_STAGES needs collapse_level >= 0 and cluster_wg = -1"));
            int n = 0, wg[CLUSTER_MAX_STAGES], hi[CLUSTER_MAX_STAGES];
            const char *c = e;
            while (*c && n < CLUSTER_MAX_STAGES) {
                int K = 0, top = 0, used = 0;
                if (std::sscanf(c, "%d:%d%n", &K, &top, &used) != 2) break;
                const bool ok = K >= 2 && K <= max_wg && (K & (K - 1)) == 0 && top <= std::min(L - 2, lcap) &&
                                top > prm.collapse_level && (n == 0 || (K < wg[n - 1] && top < hi[n - 1]));
                if (!ok) return bail(fail(HIPBMG_EINVAL, "HIPBMG_STAGES: bad stage %d:%d", K, top));
                wg[n] = K;
                hi[n] = top;
                ++n;
                c += used;
                if (*c == ',') ++c;
            }
            h->cl_nstage = n;
            for (int k = 0; k < n; ++k) {
                h->cl_wg[k] = wg[k];
                h->cl_hi[k] = hi[k];
            }
        }
        h->path_us = model_path_us(ml, L, prm.nu1, prm.nu2, h->nc, word, h->mp, h->lstar, h->cl_nstage, h->cl_wg,
                                   h->cl_hi);
        if (h->cl_nstage > 0) {
            st = alloc_stage_barriers(h, s);
            if (st != HIPBMG_OK) return bail(st);
        }
    } else {
        h->path_us = h->model_us[h->lstar];
    }
    if (h->lstar >= L - 1) h->fused3 = 0;   // the finest level itself is collapsed
    if (hipStreamSynchronize(s) != hipSuccess) return bail(fail(HIPBMG_EHIP, "setup failed: %s",
                                                             hipGetErrorString(hipGetLastError())));
    h->setup_ms = now_ms() - t0;
    *out = h;
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_destroy(hipbmg_handle h)
{
    if (h) {
        (void)hipDeviceSynchronize();
        delete h;
    }
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_level_size(hipbmg_handle h, int l, int *nx, int *ny)
{
    if (!h) return fail(HIPBMG_EINVAL, "null handle");
    if (l < 0 || l >= h->L) return fail(HIPBMG_EINVAL, "level %d out of range [0,%d)", l, h->L);
    if (nx) *nx = h->lv[l].nx;
    if (ny) *ny = h->lv[l].ny;
    return HIPBMG_OK;
}

// ---------------------------------------------------------------------------
// V-cycle launch plan (Algorithm 1 with levels 0..l* collapsed)
// ---------------------------------------------------------------------------
template <typename T>
static StreamArgs<T> base_args(const LevelDev<T> &A, int rb)
{
    StreamArgs<T> a{};
    a.nx = A.nx;
    a.ny = A.ny;
    a.pitch = A.pitch;
    a.C = A.C;
    a.W = A.W;
    a.S = A.S;
    a.SW = A.SW;
    a.SE = A.SE;
    a.b = A.b;
    a.rb = rb;
    return a;
}

template <typename T>
static hipError_t run_stream(const LevelDev<T> &A, int variant, StreamArgs<T> a, hipStream_t s,
                             int *ntiles_out = nullptr)
{
    int g;
    stream_geometry(A.nx, A.ny, A.npt, variant, a.rb, &a.nstrips, &a.nblocks, &a.ntiles, &g);
    if (ntiles_out) *ntiles_out = a.ntiles;
    return launch_stream<T>(A.npt, variant, a, g, s);
}

// Launch arguments of the collapsed levels 0..top: levels from the coarsest up
// are staged in LDS while they fit (lds_in_budget gives the same test).
template <typename T>
static CollapseArgs<T> collapse_args(const hipbmg_hier *h, const std::vector<LevelDev<T>> &lv,
                                     const LevelDev<T> *d_lv, int top, int xb_top, int zero_top, int want_norm)
{
    CollapseArgs<T> c{};
    c.levels = d_lv;
    c.top = top;
    c.xb_top = xb_top;
    c.zero_top = zero_top;
    c.nu1 = h->prm.nu1;
    c.nu2 = h->prm.nu2;
    c.rescorr = h->prm.residual_correction;
    c.chol = h->d_chol;
    c.cidx = h->d_cidx;
    c.nc = h->nc;
    c.work = h->d_work;
    c.partials = h->d_partials;
    c.want_norm = want_norm;
    c.lds_top = -1;
    size_t off = 0;
    for (int l = 0; l <= top; ++l) {
        const size_t bytes = collapse_lds_bytes<T>(lv[l].nx, lv[l].ny, l ? lv[l - 1].nx : 0, l ? lv[l - 1].ny : 0);
        if (off + bytes > (size_t)COLLAPSE_LDS_BUDGET || h->no_lds) break;
        c.lds_off[l] = (int)off;
        off += bytes;
        c.lds_top = l;
    }
    c.lds_bytes = (int)off;
    return c;
}

// Agglomeration stages above collapse level lstar: stage k on wg[k]
// workgroups from level hi[k] down; workgroup 0 collapses levels 0..lstar
// (from zero, no norm); the highest stage level's iterate ends in x[1].
template <typename T>
static ClusterArgs<T> cluster_args(const hipbmg_hier *h, const std::vector<LevelDev<T>> &lv,
                                   const LevelDev<T> *d_lv, int lstar, int nstage, const int *wg, const int *hi,
                                   const int *active)
{
    ClusterArgs<T> a{};
    a.col = collapse_args<T>(h, lv, d_lv, lstar, 1, 1, 0);
    a.nstage = nstage;
    for (int k = 0; k < nstage; ++k) {
        a.wg[k] = wg[k];
        a.hi[k] = hi[k];
    }
    a.hi[nstage] = lstar;
    a.xb_top = 1;
    a.bar = h->d_bar;
    a.err = h->d_err;
    a.active = active;
    return a;
}

// Enqueue one V-cycle on the hierarchy `lv` whose finest iterate is in
// x[cur] (or is zero if zero_start).  The finest post-relaxation leaves its
// residual norm partials in d_partials (*nparts of them).  Returns the buffer
// index holding the new finest iterate.
template <typename T>
static hipError_t enqueue_vcycle(hipbmg_hier *h, const std::vector<LevelDev<T>> &lv,
                                 const LevelDev<T> *d_lv, int cur, bool zero_start, int *new_cur,
                                 int *nparts, hipStream_t s, bool skip_finest = false,
                                 const int *active = nullptr)
{
    // skip_finest: run levels L-2..0 only (the finest level's kernels are
    // issued by the caller); *new_cur then receives the buffer of level L-2's
    // correction
    const int L = skip_finest ? h->L - 1 : h->L, ls = h->lstar;
    const int nu1 = h->prm.nu1, nu2 = h->prm.nu2, rc = h->prm.residual_correction;
    // highest level below the grid-wide kernels: the first stage's, or l*
    const int gtop = h->cl_nstage > 0 ? h->cl_hi[0] : ls;
    int xb_after[HIPBMG_MAX_LEVELS], xres[HIPBMG_MAX_LEVELS];
    hipError_t e = hipSuccess;
    for (int l = L - 1; l > gtop; --l) {
        const LevelDev<T> &A = lv[l], &Cl = lv[l - 1];
        const bool fine = l == h->L - 1;
        int xb = fine ? cur : 0;
        const bool zero = !fine || zero_start;
        // the last two pre-relaxations run as one fused pass unless disabled
        const int nk = (nu1 >= 2 && !h->no_fuse2) ? nu1 - 1 : nu1;
        for (int k = 1; k <= nk; ++k) {
            const bool last = k == nk, zx = zero && k == 1;
            const bool two = last && nk < nu1;
            const bool rcl = h->rc_level[l] && two;
            const int v = last ? (two ? (zx ? (rcl ? SV_SWEEP2_R_ZX : SV_SWEEP2_RQ_ZX)
                                            : (rcl ? SV_SWEEP2_R : SV_SWEEP2_RQ))
                                      : (zx ? SV_SWEEP_RQ_ZX : SV_SWEEP_RQ))
                               : (zx ? SV_SWEEP_ZX : SV_SWEEP);
            StreamArgs<T> a = base_args(A, h->rb[l]);
            a.x_in = A.x[xb];
            a.x_out = A.x[1 - xb];
            if (v == SV_SWEEP2_R_ZX) a.zexc = h->zc9_form && h->zc9[PrecIdx<T>::v][l];
            if (last) {
                a.q_out = A.q;
                a.bc = Cl.b;
                a.wt = A.wt;
                a.cnx = Cl.nx;
                a.cny = Cl.ny;
                a.cpitch = Cl.pitch;
                a.cplane = (long long)Cl.plane;
            }
            const int pk = prof_begin(h, v, PrecIdx<T>::v, l, 0, fine, s);
            a.active = active;
            if (v == SV_SWEEP2_RQ_ZX && h->tile_dn[l]) {
                const int nw = h->tile_dn[l];
                int nbl;
                a.rb = tile_steps(nw, 1);
                tile_geometry(A.nx, A.ny, A.npt, nw, 1, &a.nstrips, &nbl, &a.ntiles);
                a.nblocks = nbl;
                if ((e = launch_tile<T>(1, nw, a, s)) != hipSuccess) return e;
            } else if ((e = run_stream(A, v, a, s)) != hipSuccess) {
                return e;
            }
            prof_end(h, pk, s);
            xb = 1 - xb;
        }
        xb_after[l] = xb;
    }
    if (h->cl_nstage > 0) {
        // levels 0..gtop in one launch: the stages, then the collapse
        const ClusterArgs<T> c = cluster_args<T>(h, lv, d_lv, ls, h->cl_nstage, h->cl_wg, h->cl_hi, active);
        const int pk = prof_begin(h, -1, PrecIdx<T>::v, gtop, 2, false, s);
        if ((e = launch_cluster<T>(c, s)) != hipSuccess) return e;
        prof_end(h, pk, s);
        xres[gtop] = c.xb_top;
    } else {
        // levels 0..l* in one workgroup
        const bool fine = ls == h->L - 1;
        CollapseArgs<T> c = collapse_args<T>(h, lv, d_lv, ls, fine ? cur : 1, fine ? (zero_start ? 1 : 0) : 1,
                                             fine ? 1 : 0);
        c.active = active;
        const int pk = prof_begin(h, -1, PrecIdx<T>::v, ls, 2, false, s);
        if ((e = launch_collapse<T>(c, s)) != hipSuccess) return e;
        prof_end(h, pk, s);
        xres[ls] = c.xb_top;
        if (fine) {
            *new_cur = cur;
            *nparts = 1;
            return hipSuccess;
        }
    }
    for (int l = gtop + 1; l < L; ++l) {
        const LevelDev<T> &A = lv[l], &Cl = lv[l - 1];
        const bool fine = l == h->L - 1;
        int xb = xb_after[l];
        for (int k = 1; k <= nu2; ++k) {
            const bool first = k == 1, last = k == nu2;
            // a level whose down leg stored no q forms r/C in its first up pass
            int v = first ? (fine && last ? SV_INTERP_NORM : (h->rc_level[l] ? SV_INTERP_RC : SV_INTERP))
                          : (fine && last ? SV_SWEEP_NORM : SV_SWEEP);
            StreamArgs<T> a = base_args(A, h->rb_up[l]);
            a.x_in = A.x[xb];
            a.x_out = A.x[1 - xb];
            if (v == SV_INTERP_RC) a.zexc = h->zc9_form && h->zc9[PrecIdx<T>::v][l];
            if (first) {
                a.xc = Cl.x[xres[l - 1]];
                a.wt = A.wt;
                a.q_in = A.q;
                a.rescorr = rc;
                a.cnx = Cl.nx;
                a.cny = Cl.ny;
                a.cpitch = Cl.pitch;
                a.cplane = (long long)Cl.plane;
            }
            a.partials = h->d_partials;
            int nt = 0;
            const int pk = prof_begin(h, v, PrecIdx<T>::v, l, 1, fine, s);
            a.active = active;
            if (v == SV_INTERP && h->tile_up[PrecIdx<T>::v][l]) {
                const int nw = h->tile_up[PrecIdx<T>::v][l];
                int nbl;
                a.rb = tile_steps(nw, 0);
                tile_geometry(A.nx, A.ny, A.npt, nw, 0, &a.nstrips, &nbl, &a.ntiles);
                a.nblocks = nbl;
                if ((e = launch_tile<T>(0, nw, a, s)) != hipSuccess) return e;
            } else if ((e = run_stream(A, v, a, s, &nt)) != hipSuccess) {
                return e;
            }
            prof_end(h, pk, s);
            if (fine && last) *nparts = nt;
            xb = 1 - xb;
        }
        xres[l] = xb;
    }
    *new_cur = xres[L - 1];
    return hipSuccess;
}

template <typename T> static T *&x3_of(hipbmg_hier *h);
template <> double *&x3_of<double>(hipbmg_hier *h) { return h->x3_64; }
template <> float *&x3_of<float>(hipbmg_hier *h) { return h->x3_32; }

// Run up to max_cycles V-cycles on the hierarchy lv (FP64 levels, or the FP32
// levels of a mixed solve) from its finest iterate x[0] (or from zero), with
// the convergence test ||r|| / denom[0] <= tol after every cycle taken on the
// device.  The host enqueues up to `ahead` cycles beyond the last test it has
// seen; once a test is met the device clears the run flag and every launch of
// later cycles returns at once, so the iterate stays the one of the stopping
// cycle.  With the finest level pipelined, cycle k's post-relaxation, norm and
// cycle k+1's pre-relaxations and restriction are one pass over three
// iterate buffers.  On return *result is the finest buffer holding the
// iterate after the last cycle run, *cycles_done their number, and the
// residual history of the run is in d_hist.
template <typename T>
static hipbmg_status run_cycles(hipbmg_hier *h, const std::vector<LevelDev<T>> &lv, const LevelDev<T> *d_lv,
                                bool zero_start, int max_cycles, double tol, const double *d_denom,
                                hipStream_t s, const T **result, int *cycles_done)
{
    const int L = h->L;
    const LevelDev<T> &F = lv[L - 1];
    const int *act = h->d_flags;
    const bool pipe = h->fused3 != 0;
    T *xb[3] = {F.x[0], F.x[1], pipe ? x3_of<T>(h) : nullptr};
    // the convergence-test events, made on the handle's first solve (the
    // hierarchies of a batch never need them)
    for (int k = 0; k < RING; ++k)
        if (!h->ring_ev[k] && hipEventCreateWithFlags(&h->ring_ev[k], hipEventDisableTiming) != hipSuccess) {
            h->ring_ev[k] = nullptr;
            return fail(HIPBMG_EHIP, "event creation failed");
        }

    std::vector<const T *> res_after((size_t)max_cycles + 1, F.x[0]);
    // pipelined: the inputs of each cycle's finest pass (iterate buffer,
    // coarse correction), to rebuild the stopping cycle's iterate
    std::vector<int> in_i((size_t)max_cycles + 1, 0);
    std::vector<const T *> in_xc((size_t)max_cycles + 1, nullptr);
    HIPCHK(launch_flags_reset(h->d_flags, s));
    if (pipe) {
        // pre-relaxations of cycle 1 and the restriction of its residual
        const LevelDev<T> &Cl = lv[L - 2];
        StreamArgs<T> a = base_args(F, h->rb[L - 1]);
        a.x_in = xb[0];
        a.x_out = xb[1];
        a.q_out = F.q;
        a.bc = Cl.b;
        a.wt = F.wt;
        a.cnx = Cl.nx;
        a.cny = Cl.ny;
        a.cpitch = Cl.pitch;
        a.cplane = (long long)Cl.plane;
        HIPCHK(run_stream(F, zero_start ? SV_SWEEP2_RQ_ZX : SV_SWEEP2_RQ, a, s));
    }
    int k = 0, seen = 0, i = 1, cur = 0;
    bool stopped = false;
    // a cycle known to be the last (the cap) runs stage P alone, storing its
    // iterate and forming its norm, instead of also relaxing for a next cycle
    // that never comes and then rebuilding (HIPBMG_NO_LAST_PASS=1 keeps the
    // rebuild)
    int stored_last = 0;
    bool last_pass = true;
    if (const char *e = std::getenv("HIPBMG_NO_LAST_PASS")) last_pass = std::atoi(e) == 0;
    while (k < max_cycles && !stopped) {
        ++k;
        h->prof_cycle = k;
        int np = 0;
        if (pipe) {
            const LevelDev<T> &Cl = lv[L - 2];
            int cc = 0, dummy = 0;
            hipError_t e = enqueue_vcycle<T>(h, lv, d_lv, 0, false, &cc, &dummy, s, true, act);
            if (e != hipSuccess) return fail(HIPBMG_EHIP, "V-cycle launch failed: %s", hipGetErrorString(e));
            StreamArgs<T> a = base_args(F, h->rb3);
            a.zexc = h->zexc[PrecIdx<T>::v];
            a.wform = PrecIdx<T>::v == 0 ? h->wform : 0;
            a.x_in = xb[i];
            a.x_out = xb[(i + 1) % 3];
            a.x_out2 = xb[(i + 2) % 3];
            a.xc = Cl.x[cc];
            a.wt = F.wt;
            a.rescorr = h->prm.residual_correction;
            a.bc = Cl.b;
            a.cnx = Cl.nx;
            a.cny = Cl.ny;
            a.cpitch = Cl.pitch;
            a.cplane = (long long)Cl.plane;
            a.partials = h->d_partials;
            a.active = act;
            const int vf = last_pass && k == max_cycles ? SV_FUSED3_PN : SV_FUSED3;
            if (vf == SV_FUSED3_PN) stored_last = k;
            const int pk = prof_begin(h, vf, PrecIdx<T>::v, L - 1, 1, true, s);
            HIPCHK(run_stream(F, vf, a, s, &np));
            prof_end(h, pk, s);
            res_after[k] = xb[(i + 1) % 3];
            in_i[k] = i;
            in_xc[k] = Cl.x[cc];
            i = (i + 2) % 3;
        } else {
            int nc = 0;
            hipError_t e = enqueue_vcycle<T>(h, lv, d_lv, cur, zero_start && k == 1, &nc, &np, s, false, act);
            if (e != hipSuccess) return fail(HIPBMG_EHIP, "V-cycle launch failed: %s", hipGetErrorString(e));
            cur = nc;
            res_after[k] = F.x[cur];
        }
        HIPCHK(launch_finalize_check(h->d_partials, np, d_denom, tol, k, h->d_hist, HIPBMG_MAX_HIST, h->d_scal + 1,
                                     h->d_flags, h->ring_dev + 4 * (k % RING), s));
        HIPCHK(hipEventRecord(h->ring_ev[k % RING], s));
        // the tests of earlier cycles, `ahead` cycles behind the newest
        while (seen < k - h->ahead && !stopped) {
            ++seen;
            HIPCHK(hipEventSynchronize(h->ring_ev[seen % RING]));
            prof_collect(h, false, seen, false);
            const volatile double *slot = h->ring_host + 4 * (seen % RING);
            if (slot[1] == 0.0) stopped = true;
        }
    }
    // the flags come back with the same synchronisation that ends the cycles
    HIPCHK(hipMemcpyAsync(h->h_flags, h->d_flags, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const int kdone = h->h_flags[0] ? k : h->h_flags[1];
    prof_collect(h, true, kdone);
    if (pipe && kdone > 0 && kdone != stored_last) {
        // the pipelined pass does not store the iterate after its cycle; the
        // stopping cycle's is rebuilt by the pass's own interpolation and
        // relaxation stage from that pass's inputs, which later (skipped)
        // cycles left untouched
        const LevelDev<T> &Cl = lv[L - 2];
        const int ik = in_i[kdone];
        StreamArgs<T> a = base_args(F, h->rb3);
        a.zexc = h->zexc[PrecIdx<T>::v];
        a.wform = PrecIdx<T>::v == 0 ? h->wform : 0;
        a.x_in = xb[ik];
        a.x_out = xb[(ik + 1) % 3];
        a.xc = in_xc[kdone];
        a.wt = F.wt;
        a.rescorr = h->prm.residual_correction;
        a.cnx = Cl.nx;
        a.cny = Cl.ny;
        a.cpitch = Cl.pitch;
        a.cplane = (long long)Cl.plane;
        HIPCHK(run_stream(F, SV_FUSED3_P, a, s));
    }
    *cycles_done = kdone;
    *result = res_after[kdone];
    return HIPBMG_OK;
}

static hipbmg_status read_scalars(hipbmg_hier *h, int first, int n, hipStream_t s)
{
    HIPCHK(hipMemcpyAsync(h->h_scal + first, h->d_scal + first, n * sizeof(double),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return HIPBMG_OK;
}

static void fill_info_common(hipbmg_hier *h, hipbmg_info *info)
{
    if (!info) return;
    info->levels = h->L;
    info->collapse_level = h->lstar;
    for (int l = 0; l < HIPBMG_MAX_LEVELS; ++l) {
        info->model_us[l] = l < h->L ? h->model_us[l] : 0.0;
        info->rb_down[l] = l < h->L ? h->rb[l] : 0;
        info->rb_up[l] = l < h->L ? h->rb_up[l] : 0;
    }
    info->rb_pipelined = h->fused3 ? h->rb3 : 0;
    info->setup_ms = h->setup_ms;
    info->cluster_stages = h->cl_nstage;
    for (int k = 0; k < 4; ++k) {
        info->cluster_wg[k] = k < h->cl_nstage ? h->cl_wg[k] : 0;
        info->cluster_hi[k] = k < h->cl_nstage ? h->cl_hi[k] : 0;
    }
    info->search_us = h->search_us;
    info->search_expanded = h->search_expanded;
    info->path_us = h->path_us;
}

// A stage barrier that gave up waiting (its workgroups were not all resident)
// leaves a flag: report it, and reset the barriers for the next solve.
static hipbmg_status check_stage_barriers(hipbmg_hier *h, hipStream_t s)
{
    if (h->cl_nstage == 0) return HIPBMG_OK;
    int err = 0;
    HIPCHK(hipMemcpyAsync(&err, h->d_err, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (!err) return HIPBMG_OK;
    HIPCHK(hipMemsetAsync(h->d_err, 0, sizeof(int), s));
    HIPCHK(hipMemsetAsync(h->d_bar, 0, 2 * CLUSTER_MAX_STAGES * sizeof(unsigned), s));
    HIPCHK(hipStreamSynchronize(s));
    return fail(HIPBMG_EHIP, "an agglomeration-stage barrier gave up waiting (workgroups not all resident)");
}

static hipbmg_status solve_fp64(hipbmg_hier *h, double tol, hipStream_t s, hipbmg_info *info,
                                const double **res_out)
{
    int cycles = 0;
    STCHK(run_cycles<double>(h, h->lv, h->d_lv, false, h->prm.max_cycles, tol, h->d_scal, s, res_out, &cycles));
    std::vector<double> hist(std::min(cycles, HIPBMG_MAX_HIST));
    if (!hist.empty())
        HIPCHK(hipMemcpy(hist.data(), h->d_hist, hist.size() * sizeof(double), hipMemcpyDeviceToHost));
    STCHK(read_scalars(h, 1, 1, s));
    const double rel = cycles > 0 ? h->h_scal[1] : 1.0;
    if (info) {
        info->cycles = cycles;
        info->outer_steps = cycles;
        info->relres = rel;
        for (size_t m = 0; m < hist.size(); ++m) info->relres_hist[m] = hist[m];
    }
    if (h->h_flags[0] == 0 && h->h_flags[2] == 2)
        return fail(HIPBMG_ENAN, "residual norm is not finite after cycle %d", cycles);
    if (h->h_flags[0] != 0)
        return fail(HIPBMG_ENOCONV, "relres %.3e > tol %.3e after %d cycles", rel, tol, cycles);
    return HIPBMG_OK;
}

// FP64 iterative refinement: the outer residual r = b - A u in FP64 (demoted
// into the FP32 right-hand side), inner FP32 V-cycles on A e = r from e = 0 to
// a relative residual of inner_tol, u += e.
static hipbmg_status solve_mixed(hipbmg_hier *h, double tol, hipStream_t s, hipbmg_info *info)
{
    const int L = h->L;
    const LevelDev<double> &F = h->lv[L - 1];
    const LevelDev<float> &F32 = h->lv32[L - 1];
    int cycles = 0, steps = 0;
    double rel = 1.0;
    hipbmg_status st = HIPBMG_ENOCONV;
    const double bnorm = h->h_scal[0];
    for (;;) {
        int np = 0;
        HIPCHK(launch_ir_residual(F, F.x[0], F32.b, F32.pitch, h->d_partials, &np, s));
        HIPCHK(launch_finalize_norm(h->d_partials, np, nullptr, h->d_scal + 2, s));
        STCHK(read_scalars(h, 2, 1, s));
        const double rnorm = h->h_scal[2];
        rel = rnorm / bnorm;
        if (info && steps < HIPBMG_MAX_HIST) info->relres_hist[steps] = rel;
        if (!std::isfinite(rel)) {
            st = HIPBMG_ENAN;
            break;
        }
        if (rel <= tol) {
            st = HIPBMG_OK;
            break;
        }
        if (cycles >= h->prm.max_cycles) break;
        ++steps;
        // inner FP32 solve of A e = r from e = 0, relative to ||r|| (on the
        // device), to inner_tol or to what the outer tolerance still needs
        // (half of tol / relres), whichever is looser
        const int cap = std::min(h->prm.inner_max_cycles, h->prm.max_cycles - cycles);
        const float *e32 = nullptr;
        int done = 0;
        double itol = h->prm.inner_tol;
        if (h->inner_adapt) itol = std::max(itol, 0.5 * tol / rel);
        STCHK(run_cycles<float>(h, h->lv32, h->d_lv32, true, cap, itol, h->d_scal + 2, s, &e32, &done));
        cycles += done;
        HIPCHK(launch_ir_update(F.x[0], F.pitch, e32, F32.pitch, F.nx, F.ny, s));
    }
    if (info) {
        info->cycles = cycles;
        info->outer_steps = steps;
        info->relres = rel;
    }
    if (st == HIPBMG_ENAN) return fail(HIPBMG_ENAN, "residual norm is not finite");
    if (st == HIPBMG_ENOCONV)
        return fail(HIPBMG_ENOCONV, "relres %.3e > tol %.3e after %d FP32 cycles", rel, tol, cycles);
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_solve(hipbmg_handle h, const double *b, double *u, double tol,
                                      void *stream, hipbmg_info *info)
{
    const double t0 = now_ms();
    if (!h) return fail(HIPBMG_EINVAL, "null handle");
    if (!b || !u) return fail(HIPBMG_EINVAL, "b and u must be device pointers");
    if (!(tol > 0.0)) return fail(HIPBMG_EINVAL, "tol must be > 0");
    hipStream_t s = (hipStream_t)stream;
    const int L = h->L, nx = h->nx, ny = h->ny;
    const LevelDev<double> &F = h->lv[L - 1];
    if (info) {
        memset(info, 0, sizeof *info);
        fill_info_common(h, info);
    }
    HIPCHK(hipMemcpy2DAsync(F.b, F.pitch * sizeof(double), b, nx * sizeof(double), nx * sizeof(double),
                            ny, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpy2DAsync(F.x[0], F.pitch * sizeof(double), u, nx * sizeof(double),
                            nx * sizeof(double), ny, hipMemcpyDeviceToDevice, s));
    HIPCHK(launch_zero_ring(F.x[0], nx, ny, F.pitch, s));
    HIPCHK(launch_zero_ring(F.b, nx, ny, F.pitch, s));
    const int nparts = 1024;
    HIPCHK(launch_sumsq(F.b, nx, ny, F.pitch, h->d_partials, nparts, s));
    HIPCHK(launch_finalize_norm(h->d_partials, nparts, nullptr, h->d_scal, s));
    STCHK(read_scalars(h, 0, 1, s));
    const double bnorm = h->h_scal[0];
    if (!std::isfinite(bnorm)) return fail(HIPBMG_ENAN, "||b|| is not finite");
    if (bnorm == 0.0) {
        HIPCHK(hipMemsetAsync(u, 0, (size_t)nx * ny * sizeof(double), s));
        HIPCHK(hipStreamSynchronize(s));
        if (info) info->solve_ms = now_ms() - t0;
        return HIPBMG_OK;
    }
    const double *res = F.x[0];
    hipbmg_status st = h->prm.precision == HIPBMG_MIXED ? solve_mixed(h, tol, s, info)
                                                         : solve_fp64(h, tol, s, info, &res);
    if (st != HIPBMG_OK && st != HIPBMG_ENOCONV && st != HIPBMG_ENAN) return st;
    STCHK(check_stage_barriers(h, s));
    std::string msg = g_err;
    HIPCHK(hipMemcpy2DAsync(u, nx * sizeof(double), res, F.pitch * sizeof(double),
                            nx * sizeof(double), ny, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    if (info) info->solve_ms = now_ms() - t0;
    g_err = msg;
    return st;
}

// ---------------------------------------------------------------------------
// inspection and single operations
// ---------------------------------------------------------------------------
extern "C" hipbmg_status hipbmg_get_stencil(hipbmg_handle h, int l, double *out, void *stream)
{
    if (!h || !out) return fail(HIPBMG_EINVAL, "null argument");
    if (l < 0 || l >= h->L) return fail(HIPBMG_EINVAL, "level out of range");
    hipStream_t s = (hipStream_t)stream;
    const LevelDev<double> &A = h->lv[l];
    for (int k = 0; k < 5; ++k)
        HIPCHK(hipMemcpy2DAsync(out + (size_t)k * A.nx * A.ny, A.nx * sizeof(double), A.C + k * A.plane,
                                A.pitch * sizeof(double), A.nx * sizeof(double), A.ny,
                                hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_get_interp(hipbmg_handle h, int l, double *out, void *stream)
{
    if (!h || !out) return fail(HIPBMG_EINVAL, "null argument");
    if (l < 1 || l >= h->L) return fail(HIPBMG_EINVAL, "level must be in [1, L)");
    hipStream_t s = (hipStream_t)stream;
    const LevelDev<double> &A = h->lv[l], &C = h->lv[l - 1];
    for (int k = 0; k < 8; ++k)
        HIPCHK(hipMemcpy2DAsync(out + (size_t)k * C.nx * C.ny, C.nx * sizeof(double), A.wt + k * A.cplane,
                                A.cpitch * sizeof(double), C.nx * sizeof(double), C.ny,
                                hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return HIPBMG_OK;
}

template <typename T>
static hipbmg_status to_pitched(T *dst, int pitch, const T *src, int nx, int ny, hipStream_t s)
{
    HIPCHK(hipMemcpy2DAsync(dst, pitch * sizeof(T), src, nx * sizeof(T), nx * sizeof(T), ny,
                            hipMemcpyDeviceToDevice, s));
    HIPCHK(launch_zero_ring(dst, nx, ny, pitch, s));
    return HIPBMG_OK;
}

template <typename T>
static hipbmg_status from_pitched(T *dst, const T *src, int pitch, int nx, int ny, hipStream_t s)
{
    HIPCHK(hipMemcpy2DAsync(dst, nx * sizeof(T), src, pitch * sizeof(T), nx * sizeof(T), ny,
                            hipMemcpyDeviceToDevice, s));
    return HIPBMG_OK;
}

// The levels a single operation of precision T runs on: the FP64 hierarchy,
// or the FP32 edge-form copy that a mixed-precision handle holds.
static hipbmg_status op_levels(hipbmg_hier *h, const std::vector<LevelDev<double>> **lv)
{
    *lv = &h->lv;
    return HIPBMG_OK;
}

static hipbmg_status op_levels(hipbmg_hier *h, const std::vector<LevelDev<float>> **lv)
{
    if (h->lv32.empty()) return fail(HIPBMG_EINVAL, "FP32 operations need a mixed-precision handle");
    *lv = &h->lv32;
    return HIPBMG_OK;
}

template <typename T>
static hipbmg_status op_smooth(hipbmg_hier *h, int l, const T *b, T *x, int sweeps, hipStream_t s)
{
    if (!h || !b || !x) return fail(HIPBMG_EINVAL, "null argument");
    if (l < 0 || l >= h->L || sweeps < 0) return fail(HIPBMG_EINVAL, "bad level or sweeps");
    const std::vector<LevelDev<T>> *lv = nullptr;
    STCHK(op_levels(h, &lv));
    const LevelDev<T> &A = (*lv)[l];
    STCHK(to_pitched(A.b, A.pitch, b, A.nx, A.ny, s));
    STCHK(to_pitched(A.x[0], A.pitch, x, A.nx, A.ny, s));
    int xb = 0;
    for (int k = 0; k < sweeps; ++k) {
        StreamArgs<T> a = base_args(A, h->rb[l]);
        a.x_in = A.x[xb];
        a.x_out = A.x[1 - xb];
        HIPCHK(run_stream(A, SV_SWEEP, a, s));
        xb = 1 - xb;
    }
    STCHK(from_pitched(x, A.x[xb], A.pitch, A.nx, A.ny, s));
    HIPCHK(hipStreamSynchronize(s));
    return HIPBMG_OK;
}

template <typename T>
static hipbmg_status op_smooth_restrict(hipbmg_hier *h, int l, const T *b, T *x, int sweeps, T *q, T *bc,
                                        hipStream_t s)
{
    if (!h || !b || !x || !q || !bc) return fail(HIPBMG_EINVAL, "null argument");
    if (l < 1 || l >= h->L) return fail(HIPBMG_EINVAL, "level must be in [1, L)");
    if (sweeps != 1 && sweeps != 2) return fail(HIPBMG_EINVAL, "sweeps must be 1 or 2");
    const std::vector<LevelDev<T>> *lv = nullptr;
    STCHK(op_levels(h, &lv));
    const LevelDev<T> &A = (*lv)[l], &C = (*lv)[l - 1];
    STCHK(to_pitched(A.b, A.pitch, b, A.nx, A.ny, s));
    STCHK(to_pitched(A.x[0], A.pitch, x, A.nx, A.ny, s));
    HIPCHK(hipMemsetAsync(A.q, 0, A.plane * sizeof(T), s));
    HIPCHK(hipMemsetAsync(C.b, 0, C.plane * sizeof(T), s));
    StreamArgs<T> a = base_args(A, h->rb[l]);
    a.x_in = A.x[0];
    a.x_out = A.x[1];
    a.q_out = A.q;
    a.bc = C.b;
    a.wt = A.wt;
    a.cnx = C.nx;
    a.cny = C.ny;
    a.cpitch = C.pitch;
    a.cplane = (long long)C.plane;
    HIPCHK(run_stream(A, sweeps == 2 ? SV_SWEEP2_RQ : SV_SWEEP_RQ, a, s));
    STCHK(from_pitched(x, A.x[1], A.pitch, A.nx, A.ny, s));
    STCHK(from_pitched(q, A.q, A.pitch, A.nx, A.ny, s));
    STCHK(from_pitched(bc, C.b, C.pitch, C.nx, C.ny, s));
    HIPCHK(hipStreamSynchronize(s));
    return HIPBMG_OK;
}

template <typename T>
static hipbmg_status op_interp_smooth(hipbmg_hier *h, int l, const T *b, T *x, const T *q, const T *xc,
                                      int rescorr, double *sumsq_host, hipStream_t s)
{
    if (!h || !b || !x || !q || !xc) return fail(HIPBMG_EINVAL, "null argument");
    if (l < 1 || l >= h->L) return fail(HIPBMG_EINVAL, "level must be in [1, L)");
    const std::vector<LevelDev<T>> *lv = nullptr;
    STCHK(op_levels(h, &lv));
    const LevelDev<T> &A = (*lv)[l], &C = (*lv)[l - 1];
    STCHK(to_pitched(A.b, A.pitch, b, A.nx, A.ny, s));
    STCHK(to_pitched(A.x[0], A.pitch, x, A.nx, A.ny, s));
    STCHK(to_pitched(A.q, A.pitch, q, A.nx, A.ny, s));
    STCHK(to_pitched(C.x[1], C.pitch, xc, C.nx, C.ny, s));
    StreamArgs<T> a = base_args(A, h->rb_up[l]);
    a.x_in = A.x[0];
    a.x_out = A.x[1];
    a.xc = C.x[1];
    a.wt = A.wt;
    a.q_in = A.q;
    a.rescorr = rescorr;
    a.cnx = C.nx;
    a.cny = C.ny;
    a.cpitch = C.pitch;
    a.cplane = (long long)C.plane;
    a.partials = h->d_partials;
    int nt = 0;
    HIPCHK(run_stream(A, sumsq_host ? SV_INTERP_NORM : SV_INTERP, a, s, &nt));
    if (sumsq_host) {
        HIPCHK(launch_finalize_norm(h->d_partials, nt, nullptr, h->d_scal + 5, s));
        STCHK(read_scalars(h, 5, 1, s));
        *sumsq_host = h->h_scal[5] * h->h_scal[5];
    }
    STCHK(from_pitched(x, A.x[1], A.pitch, A.nx, A.ny, s));
    HIPCHK(hipStreamSynchronize(s));
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_op_smooth(hipbmg_handle h, int l, const double *b, double *x,
                                          int sweeps, void *stream)
{
    return op_smooth<double>(h, l, b, x, sweeps, (hipStream_t)stream);
}

extern "C" hipbmg_status hipbmg_op_smooth_restrict(hipbmg_handle h, int l, const double *b, double *x,
                                                   int sweeps, double *q, double *bc, void *stream)
{
    return op_smooth_restrict<double>(h, l, b, x, sweeps, q, bc, (hipStream_t)stream);
}

extern "C" hipbmg_status hipbmg_op_interp_smooth(hipbmg_handle h, int l, const double *b, double *x,
                                                 const double *q, const double *xc, int rescorr,
                                                 double *sumsq_host, void *stream)
{
    return op_interp_smooth<double>(h, l, b, x, q, xc, rescorr, sumsq_host, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// FP32 edge-form levels of a mixed-precision handle
// ---------------------------------------------------------------------------
extern "C" hipbmg_status hipbmg_get_level32(hipbmg_handle h, int l, float *stencil_out, float *interp_out,
                                            void *stream)
{
    if (!h || !stencil_out) return fail(HIPBMG_EINVAL, "null argument");
    if (l < 0 || l >= h->L) return fail(HIPBMG_EINVAL, "level out of range");
    if (interp_out && l < 1) return fail(HIPBMG_EINVAL, "level 0 has no interpolation weights");
    const std::vector<LevelDev<float>> *lv = nullptr;
    STCHK(op_levels(h, &lv));
    hipStream_t s = (hipStream_t)stream;
    const LevelDev<float> &A = (*lv)[l];
    for (int k = 0; k < 5; ++k)
        HIPCHK(hipMemcpy2DAsync(stencil_out + (size_t)k * A.nx * A.ny, A.nx * sizeof(float), A.C + k * A.plane,
                                A.pitch * sizeof(float), A.nx * sizeof(float), A.ny, hipMemcpyDeviceToDevice, s));
    if (interp_out) {
        const LevelDev<float> &C = (*lv)[l - 1];
        for (int k = 0; k < 8; ++k)
            HIPCHK(hipMemcpy2DAsync(interp_out + (size_t)k * C.nx * C.ny, C.nx * sizeof(float),
                                    A.wt + k * A.cplane, A.cpitch * sizeof(float), C.nx * sizeof(float), C.ny,
                                    hipMemcpyDeviceToDevice, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_op32_smooth(hipbmg_handle h, int l, const float *b, float *x, int sweeps,
                                            void *stream)
{
    return op_smooth<float>(h, l, b, x, sweeps, (hipStream_t)stream);
}

extern "C" hipbmg_status hipbmg_op32_smooth_restrict(hipbmg_handle h, int l, const float *b, float *x,
                                                     int sweeps, float *q, float *bc, void *stream)
{
    return op_smooth_restrict<float>(h, l, b, x, sweeps, q, bc, (hipStream_t)stream);
}

extern "C" hipbmg_status hipbmg_op32_interp_smooth(hipbmg_handle h, int l, const float *b, float *x,
                                                   const float *q, const float *xc, int rescorr,
                                                   double *sumsq_host, void *stream)
{
    return op_interp_smooth<float>(h, l, b, x, q, xc, rescorr, sumsq_host, (hipStream_t)stream);
}

extern "C" hipbmg_status hipbmg_op32_inner(hipbmg_handle h, const float *r, float *e, int cycles, double rnorm,
                                           double inner_tol, double *hist_host, int *cycles_host, void *stream)
{
    if (!h || !r || !e) return fail(HIPBMG_EINVAL, "null argument");
    if (cycles < 1 || cycles > HIPBMG_MAX_HIST) return fail(HIPBMG_EINVAL, "cycles must be in [1, %d]", HIPBMG_MAX_HIST);
    if (!(rnorm > 0.0) || !std::isfinite(rnorm)) return fail(HIPBMG_EINVAL, "rnorm must be finite and > 0");
    if (!(inner_tol >= 0.0)) return fail(HIPBMG_EINVAL, "inner_tol must be >= 0");
    const std::vector<LevelDev<float>> *lv = nullptr;
    STCHK(op_levels(h, &lv));
    hipStream_t s = (hipStream_t)stream;
    const LevelDev<float> &F = (*lv)[h->L - 1];
    STCHK(to_pitched(F.b, F.pitch, r, F.nx, F.ny, s));
    h->h_scal[2] = rnorm;
    HIPCHK(hipMemcpyAsync(h->d_scal + 2, h->h_scal + 2, sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    const float *res = nullptr;
    int done = 0;
    STCHK(run_cycles<float>(h, h->lv32, h->d_lv32, true, cycles, inner_tol, h->d_scal + 2, s, &res, &done));
    if (hist_host && done > 0)
        HIPCHK(hipMemcpyAsync(hist_host, h->d_hist, done * sizeof(double), hipMemcpyDeviceToHost, s));
    STCHK(from_pitched(e, res, F.pitch, F.nx, F.ny, s));
    HIPCHK(hipStreamSynchronize(s));
    if (cycles_host) *cycles_host = done;
    return HIPBMG_OK;
}

// ---------------------------------------------------------------------------
// finite-volume operator and adjoint gradient
// ---------------------------------------------------------------------------
extern "C" hipbmg_status hipbmg_fv5_from_cells(int nx, int ny, const double *cell, int is_log,
                                               double *coeffs_out, void *stream)
{
    if (!cell || !coeffs_out) return fail(HIPBMG_EINVAL, "null argument");
    if (nx < 3 || ny < 3) return fail(HIPBMG_EINVAL, "grid too small");
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)nx * ny;
    HIPCHK(launch_fv5(nx, ny, cell, is_log, coeffs_out, coeffs_out + n, coeffs_out + 2 * n, nx, s));
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_fv5_from_cells_batched(int nprob, int nx, int ny, const double *cell, int is_log,
                                                       double *coeffs_out, void *stream)
{
    if (!cell || !coeffs_out) return fail(HIPBMG_EINVAL, "null argument");
    if (nprob < 1 || nprob > 65535) return fail(HIPBMG_EINVAL, "nprob must be in 1..65535");
    if (nx < 3 || ny < 3) return fail(HIPBMG_EINVAL, "grid too small");
    const size_t n = (size_t)nx * ny;
    HIPCHK(launch_fv5(nx, ny, cell, is_log, coeffs_out, coeffs_out + n, coeffs_out + 2 * n, nx, (hipStream_t)stream,
                      nprob, 3 * n));
    return HIPBMG_OK;
}

// ---------------------------------------------------------------------------
// the paper's distributed model (host only)
// ---------------------------------------------------------------------------
extern "C" hipbmg_status hipbmg_paper_model(int D, int L, const int *N_host, const int *P_host, int ns, int ncolors,
                                            int nu1, int nu2, int redundant, double alpha, double beta, double gamma,
                                            double *terms_host, double *total_host)
{
    if (!N_host || !P_host || !total_host) return fail(HIPBMG_EINVAL, "null argument");
    if ((D != 2 && D != 3) || L < 1 || L > HIPBMG_MAX_LEVELS || ns < 1 || ncolors < 1 || nu1 < 0 || nu2 < 0)
        return fail(HIPBMG_EINVAL, "bad model arguments");
    for (int i = 0; i < L * D; ++i)
        if (N_host[i] < 1 || P_host[i] < 1) return fail(HIPBMG_EINVAL, "sizes and processor counts must be >= 1");
    const PaperMachine m{alpha, beta, gamma};
    double total = 0.0;
    for (int l = 0; l < L; ++l) {
        const int *N = N_host + l * D, *P = P_host + l * D;
        int n[3], nc[3];
        for (int d = 0; d < D; ++d) n[d] = (N[d] + P[d] - 1) / P[d];
        double t[6] = {0, 0, 0, 0, 0, 0};
        if (l == 0) {
            // agglomeration of the coarsest grid onto one processor, then the
            // Cholesky substitutions (the factor is computed at setup)
            int one[3] = {1, 1, 1};
            double nn = 1.0;
            for (int d = 0; d < D; ++d) nn *= N[d];
            t[5] = paper_agglomerate(D, N, P, one, redundant, m) + nn * nn * m.gamma;
        } else {
            const int *Nc = N_host + (l - 1) * D, *Pc = P_host + (l - 1) * D;
            for (int d = 0; d < D; ++d) nc[d] = (Nc[d] + Pc[d] - 1) / Pc[d];
            t[0] = paper_smooth(D, n, ns, ncolors, nu1, nu2, m);
            t[1] = paper_residual(D, n, ns, m);
            t[2] = paper_restrict(D, n, ns, m);
            t[3] = paper_interp(D, n, nc, m);
            // the coarse right-hand side is gathered when level l-1 runs on fewer processors
            t[4] = paper_agglomerate(D, Nc, P, Pc, redundant, m);
        }
        for (int k = 0; k < 6; ++k) total += t[k];
        if (terms_host)
            for (int k = 0; k < 6; ++k) terms_host[l * 6 + k] = t[k];
    }
    *total_host = total;
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_paper_enumerate(int D, const int *N_host, const int *P_host, int max,
                                                int *grids_host, int *count_host)
{
    if (!N_host || !P_host || !grids_host || !count_host) return fail(HIPBMG_EINVAL, "null argument");
    if (D < 1 || D > 3 || max < 0) return fail(HIPBMG_EINVAL, "bad arguments");
    for (int d = 0; d < D; ++d)
        if (N_host[d] < 1 || P_host[d] < 1) return fail(HIPBMG_EINVAL, "sizes and processor counts must be >= 1");
    *count_host = paper_enumerate(D, N_host, P_host, max, grids_host);
    return HIPBMG_OK;
}

static hipbmg_status paper_setup_check(const hipbmg_paper_setup *st, const int *N, const int *P, PaperSetup *out)
{
    if (!st || !N || !P) return fail(HIPBMG_EINVAL, "null argument");
    if ((st->D != 2 && st->D != 3) || st->limit < 1 || st->coarsest < 1 || st->ns < 1 || st->ncolors < 1 ||
        st->nu1 < 0 || st->nu2 < 0)
        return fail(HIPBMG_EINVAL, "bad model setup");
    for (int d = 0; d < st->D; ++d)
        if (N[d] < 1 || P[d] < 1) return fail(HIPBMG_EINVAL, "sizes and processor counts must be >= 1");
    *out = PaperSetup{st->D,  st->limit, st->coarsest,  st->ns, st->ncolors,
                      st->nu1, st->nu2,  st->redundant, PaperMachine{st->alpha, st->beta, st->gamma}};
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_paper_search(const hipbmg_paper_setup *setup, const int *N_host, const int *P_host,
                                             int max_path, int *path_host, int *len_host, double *t_host)
{
    PaperSetup ps;
    const hipbmg_status st = paper_setup_check(setup, N_host, P_host, &ps);
    if (st != HIPBMG_OK) return st;
    if (!path_host || !len_host || !t_host || max_path < 1) return fail(HIPBMG_EINVAL, "null argument");
    std::vector<std::vector<int>> path;
    *t_host = paper_search(ps, N_host, P_host, &path);
    if ((int)path.size() > max_path) return fail(HIPBMG_EINVAL, "path longer than max_path");
    for (size_t k = 0; k < path.size(); ++k)
        for (int d = 0; d < ps.D; ++d) path_host[k * ps.D + d] = path[k][d];
    *len_host = (int)path.size();
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_paper_astar(const hipbmg_paper_setup *setup, const int *N_host, const int *P_host,
                                            int max_path, int *path_host, int *len_host, double *t_host,
                                            int *expanded_host)
{
    PaperSetup ps;
    const hipbmg_status st = paper_setup_check(setup, N_host, P_host, &ps);
    if (st != HIPBMG_OK) return st;
    if (!path_host || !len_host || !t_host || !expanded_host || max_path < 1)
        return fail(HIPBMG_EINVAL, "null argument");
    std::vector<std::vector<int>> path;
    *t_host = paper_astar(ps, N_host, P_host, &path, expanded_host);
    if ((int)path.size() > max_path) return fail(HIPBMG_EINVAL, "path longer than max_path");
    for (size_t k = 0; k < path.size(); ++k)
        for (int d = 0; d < ps.D; ++d) path_host[k * ps.D + d] = path[k][d];
    *len_host = (int)path.size();
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_paper_path_cost(const hipbmg_paper_setup *setup, const int *N_host,
                                                const int *P_host, const int *path_host, int len, double *t_host)
{
    PaperSetup ps;
    const hipbmg_status st = paper_setup_check(setup, N_host, P_host, &ps);
    if (st != HIPBMG_OK) return st;
    if ((!path_host && len > 0) || len < 0 || !t_host) return fail(HIPBMG_EINVAL, "null argument");
    std::vector<std::vector<int>> seq(len);
    for (int k = 0; k < len; ++k) seq[k].assign(path_host + k * ps.D, path_host + (k + 1) * ps.D);
    *t_host = paper_path_cost(ps, N_host, P_host, seq);
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_fv5_aniso(int nx, int ny, const double *dx_cell, const double *dy_cell, double hx,
                                          double hy, double *coeffs_out, void *stream)
{
    if (!dx_cell || !dy_cell || !coeffs_out) return fail(HIPBMG_EINVAL, "null argument");
    if (nx < 3 || ny < 3) return fail(HIPBMG_EINVAL, "grid too small");
    if (!(hx > 0.0) || !(hy > 0.0) || !std::isfinite(hx) || !std::isfinite(hy))
        return fail(HIPBMG_EINVAL, "spacings must be positive and finite");
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)nx * ny;
    HIPCHK(launch_fv5_aniso(nx, ny, dx_cell, dy_cell, hx, hy, coeffs_out, coeffs_out + n, coeffs_out + 2 * n, nx,
                            s));
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_grad_logD(int nx, int ny, const double *theta, const double *u,
                                          const double *lam, double *grad_out, void *stream)
{
    if (!theta || !u || !lam || !grad_out) return fail(HIPBMG_EINVAL, "null argument");
    if (nx < 3 || ny < 3) return fail(HIPBMG_EINVAL, "grid too small");
    HIPCHK(launch_grad_logD(nx, ny, theta, u, lam, grad_out, (hipStream_t)stream));
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_grad_logD_batched(int nprob, int nx, int ny, const double *theta, const double *u,
                                                  const double *lam, double *grad_out, void *stream)
{
    if (!theta || !u || !lam || !grad_out) return fail(HIPBMG_EINVAL, "null argument");
    if (nprob < 1 || nprob > 65535) return fail(HIPBMG_EINVAL, "nprob must be in 1..65535");
    if (nx < 3 || ny < 3) return fail(HIPBMG_EINVAL, "grid too small");
    HIPCHK(launch_grad_logD(nx, ny, theta, u, lam, grad_out, (hipStream_t)stream, nprob));
    return HIPBMG_OK;
}

// ---------------------------------------------------------------------------
// live kernel timing
// ---------------------------------------------------------------------------
extern "C" hipbmg_status hipbmg_profile(hipbmg_handle h, int enable)
{
    if (!h) return fail(HIPBMG_EINVAL, "null handle");
    if (enable && !h->ev0[0])
        for (int k = 0; k < PROF_RING; ++k) {
            HIPCHK(hipEventCreate(&h->ev0[k]));
            HIPCHK(hipEventCreate(&h->ev1[k]));
        }
    if (enable < 0 || enable > 2) return fail(HIPBMG_EINVAL, "enable must be 0, 1 or 2");
    prof_collect(h, true);   // pairs still pending belong to the previous setting
    h->prof_on = enable;
    if (enable) {
        memset(h->prof_ms, 0, sizeof h->prof_ms);
        memset(h->prof_cnt, 0, sizeof h->prof_cnt);
        memset(h->lvl_ms, 0, sizeof h->lvl_ms);
        memset(h->lvl_cnt, 0, sizeof h->lvl_cnt);
    }
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_profile_read(hipbmg_handle h, int precision, int variant,
                                             double *total_ms_host, long long *launches_host,
                                             double *bytes_per_launch_host)
{
    if (!h) return fail(HIPBMG_EINVAL, "null handle");
    if (precision < 0 || precision > 1 || variant < 0 || variant >= SV_COUNT)
        return fail(HIPBMG_EINVAL, "bad precision or kernel index");
    if (total_ms_host) *total_ms_host = h->prof_ms[precision][variant];
    if (launches_host) *launches_host = h->prof_cnt[precision][variant];
    if (bytes_per_launch_host) {
        // algorithmic bytes of one launch on the finest level (every vertex of
        // the grid, boundary ring included): the relaxation reads x, b and the
        // stencil planes and writes x; the fused variants add their extra fields
        const LevelDev<double> &F = h->lv[h->L - 1];
        const double n = (double)F.nx * F.ny, w = precision ? 4.0 : 8.0;
        const double s = F.npt == 5 ? 3.0 : 5.0;
        double per = (s + 3.0) * w;
        if (variant == SV_SWEEP_ZX || variant == SV_SWEEP_RQ_ZX) per -= w;
        if (variant == SV_SWEEP2_RQ_ZX) per -= w;
        if (variant == SV_SWEEP_RQ || variant == SV_SWEEP_RQ_ZX || variant == SV_SWEEP2_RQ ||
            variant == SV_SWEEP2_RQ_ZX)
            per += w + 2.0 * w + 0.25 * w;
        if (variant == SV_INTERP || variant == SV_INTERP_NORM) per += 0.25 * w + 2.0 * w + w;
        // interpolation inputs and the weights once, coarse rhs (the
        // relaxation's x write is the next cycle's iterate; the post-relaxed
        // iterate and r/C are not stored, r/C is formed from the loaded rows)
        if (variant == SV_FUSED3) per += 0.25 * w + 2.0 * w + 0.25 * w;
        if (variant == SV_FUSED3_P || variant == SV_FUSED3_PN || variant == SV_INTERP_RC) per += 0.25 * w + 2.0 * w;
        if (variant == SV_SWEEP2_R_ZX) per -= w;
        if (variant == SV_SWEEP2_R || variant == SV_SWEEP2_R_ZX) per += 2.0 * w + 0.25 * w;
        // a pipelined pass over a zero-excess operator forms C instead of loading it
        const bool f3 = variant == SV_FUSED3 || variant == SV_FUSED3_P || variant == SV_FUSED3_PN;
        if (f3 && h->zexc[precision]) per -= w;
        // and forms the weights (FP64): the 8 weight planes at quarter size are not read
        if (f3 && precision == 0 && h->wform) per -= 2.0 * w;
        *bytes_per_launch_host = per * n;
    }
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_profile_levels(hipbmg_handle h, int precision, double *ms_host, long long *n_host)
{
    if (!h || !ms_host) return fail(HIPBMG_EINVAL, "null argument");
    if (precision < 0 || precision > 1) return fail(HIPBMG_EINVAL, "bad precision");
    for (int k = 0; k < 3 * HIPBMG_MAX_LEVELS; ++k) {
        ms_host[k] = h->lvl_ms[precision][k];
        if (n_host) n_host[k] = h->lvl_cnt[precision][k];
    }
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_model_levels(hipbmg_handle h, double *grid_us_host, double *wg_us_host,
                                             double *base_us_host)
{
    if (!h || !grid_us_host || !wg_us_host || !base_us_host) return fail(HIPBMG_EINVAL, "null argument");
    const int word = h->prm.precision == HIPBMG_MIXED ? 4 : 8;
    for (int l = 0; l < HIPBMG_MAX_LEVELS; ++l) {
        grid_us_host[l] = l < h->L ? model_grid_level_us(h->ml[l], l == h->L - 1, h->prm.nu1, h->prm.nu2, word, h->mp)
                                   : 0.0;
        wg_us_host[l] = (l >= 1 && l < h->L) ? model_wg_level_us(h->ml[l], h->prm.nu1, h->prm.nu2, word, h->mp) : 0.0;
    }
    base_us_host[0] = model_base_us(h->nc, word, h->mp);
    return HIPBMG_OK;
}

// ---------------------------------------------------------------------------
// Calibration of the model on the kernels themselves.  A synthetic hierarchy
// (D = 1 on 257 x 257 vertices, FP64 and FP32 levels) is built; the collapse
// launch is timed with every level as its top, and the down and up kernels of
// every level are timed back to back.  The collapsed-level terms (alpha_bar,
// beta_wg, separately for levels staged in LDS and levels left in global
// memory) are fitted to the per-level increments of the collapse time, the
// step latencies to the grid kernels on levels too small to be
// bandwidth-bound.  This is the single-GPU form of measuring the model's
// parameters with benchmarks of the operations the solver performs.
// ---------------------------------------------------------------------------
// least squares y = a + b x over the samples, with a, b >= 0 (a, b unchanged
// if there is no sample)
static void fit_nonneg(const std::vector<double> &x, const std::vector<double> &y, double *a, double *b)
{
    const size_t n = x.size();
    if (n == 0) return;
    double mx = 0.0, my = 0.0;
    for (size_t i = 0; i < n; ++i) {
        mx += x[i];
        my += y[i];
    }
    mx /= (double)n;
    my /= (double)n;
    double sxy = 0.0, sxx = 0.0;
    for (size_t i = 0; i < n; ++i) {
        sxy += (x[i] - mx) * (y[i] - my);
        sxx += (x[i] - mx) * (x[i] - mx);
    }
    double bb = (n > 1 && sxx > 0.0) ? sxy / sxx : 0.0, aa = my - bb * mx;
    if (bb < 0.0) {
        bb = 0.0;
        aa = my;
    }
    if (aa < 0.0) {   // through the origin
        double s0 = 0.0, s1 = 0.0;
        for (size_t i = 0; i < n; ++i) {
            s0 += x[i] * y[i];
            s1 += x[i] * x[i];
        }
        aa = 0.0;
        bb = s1 > 0.0 ? std::max(0.0, s0 / s1) : 0.0;
    }
    *a = aa;
    *b = bb;
}

static double median(std::vector<double> v)
{
    std::sort(v.begin(), v.end());
    const size_t n = v.size();
    return n % 2 ? v[n / 2] : 0.5 * (v[n / 2 - 1] + v[n / 2]);
}

// One launch timed as it runs inside a solve: after a large write has pushed
// everything else out of the caches, bracketed by events on the stream (the
// launch gap after the previous kernel is included).  Minimum over reps.
struct ColdTimer {
    hipStream_t s;
    hipEvent_t e0, e1;
    void *flush;
    size_t flush_bytes;
    template <typename F>
    double us(int reps, F &&launch)
    {
        double best = 1e30;
        for (int r = 0; r < reps; ++r) {
            (void)hipMemsetAsync(flush, r & 0xff, flush_bytes, s);
            (void)hipEventRecord(e0, s);
            launch();
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            best = std::min(best, 1e3 * (double)ms);
        }
        return best;
    }
};

template <typename T>
static hipError_t calibrate_precision(hipbmg_hier *h, const std::vector<LevelDev<T>> &lv, const LevelDev<T> *d_lv,
                                      ColdTimer &ct, ModelParams &p)
{
    hipStream_t s = ct.s;
    const int L = h->L, nu1 = h->prm.nu1, nu2 = h->prm.nu2, word = (int)sizeof(T);
    const int q = word == 4 ? 1 : 0;
    ModelLevel ml[HIPBMG_MAX_LEVELS];
    model_levels(h, q, ml);
    // collapse launch with each level as its top
    std::vector<double> tc(L);
    for (int top = 0; top < L; ++top) {
        const CollapseArgs<T> c = collapse_args<T>(h, lv, d_lv, top, 1, 1, 0);
        tc[top] = ct.us(3, [&] { (void)launch_collapse<T>(c, s); });
    }
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    p.t_base_us[q] = std::max(0.0, tc[0] - p.alpha_launch_us);
    std::vector<double> xs[2], ys[2];
    for (int l = 1; l < L; ++l) {
        const int g = ml[l].in_lds ? 0 : 1;
        xs[g].push_back(model_wg_bytes(lv[l].nx, lv[l].ny, nu1, nu2, word));
        ys[g].push_back(tc[l] - tc[l - 1]);
    }
    const double P = model_wg_phases(nu1, nu2);
    for (int g = 0; g < 2; ++g) {
        double a = P * p.alpha_bar_us[q][g], b = p.beta_wg_us_per_B[q][g];
        fit_nonneg(xs[g], ys[g], &a, &b);
        p.alpha_bar_us[q][g] = a / P;
        p.beta_wg_us_per_B[q][g] = b;
    }
    // agglomeration stages: one launch of K workgroups running levels
    // 2..top, with levels 0..1 collapsed on workgroup 0, for every top (top = 1:
    // the stage runs no level); the increments are the levels' costs on K
    // workgroups, fitted to phases x alpha_stage + bytes x beta_stage
    {
        if (alloc_stage_barriers(h, s) != HIPBMG_OK) return hipErrorOutOfMemory;
        const int max_wg = std::min(256, cluster_max_resident<T>(COLLAPSE_LDS_BUDGET));
        for (int k = 0; k < MODEL_STAGE_SIZES && L >= 4; ++k) {
            const int K = 2 << k;
            if (K > max_wg) break;
            std::vector<double> bx, by;
            double prev = 0.0;
            for (int top = 1; top <= L - 2; ++top) {
                const int wg[1] = {K}, hi[1] = {top};
                const ClusterArgs<T> a = cluster_args<T>(h, lv, d_lv, 1, 1, wg, hi, nullptr);
                const double t = ct.us(3, [&] { (void)launch_cluster<T>(a, s); });
                if (top >= 2) {
                    bx.push_back(model_wg_bytes(lv[top].nx, lv[top].ny, nu1, nu2, word));
                    by.push_back(t - prev);
                }
                prev = t;
            }
            double a = P * p.alpha_stage_us[q][k], b = p.beta_stage_us_per_B[q][k];
            fit_nonneg(bx, by, &a, &b);
            p.alpha_stage_us[q][k] = a / P;
            p.beta_stage_us_per_B[q][k] = b;
        }
        int err = 0;
        if (hipMemcpy(&err, h->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess || err)
            return hipErrorLaunchFailure;
        p.stages_calibrated = 1;
    }
    // grid kernels of every level below the finest (zero-start pre-relaxation
    // fused with residual and restriction; interpolating relaxation), each at
    // two row-block lengths: on a level whose waves all fit in one residency
    // round and whose bytes take a small part of the time, the difference
    // gives the step latency and the rest the kernel's fixed cost
    std::vector<double> sdn, sup, fdn, fup;
    const int vdn = nu1 >= 2 ? SV_SWEEP2_RQ_ZX : SV_SWEEP_RQ_ZX;
    for (int l = 1; l < L; ++l) {
        const LevelDev<T> &A = lv[l], &Cl = lv[l - 1];
        const int nsteps = (A.ny - 1) / 2;
        if (nsteps < 4) continue;
        const double nbytes = (double)A.nx * A.ny * word * 12.0;
        for (int leg = 0; leg < 2; ++leg) {
            const int v = leg == 0 ? vdn : SV_INTERP;
            StreamArgs<T> a = base_args(A, 1);
            if (leg == 0) {
                a.x_in = A.x[0];
                a.x_out = A.x[1];
                a.q_out = A.q;
                a.bc = Cl.b;
            } else {
                a.x_in = A.x[1];
                a.x_out = A.x[0];
                a.xc = Cl.x[1];
                a.q_in = A.q;
                a.rescorr = h->prm.residual_correction;
            }
            a.wt = A.wt;
            a.cnx = Cl.nx;
            a.cny = Cl.ny;
            a.cpitch = Cl.pitch;
            a.cplane = (long long)Cl.plane;
            const int rbs[2] = {1, 4};
            double tt[2];
            bool ok = true;
            for (int m = 0; m < 2; ++m) {
                a.rb = rbs[m];
                tt[m] = ct.us(3, [&] { (void)run_stream(A, v, a, s); });
                int nst, nbl, nt, gg;
                stream_geometry(A.nx, A.ny, A.npt, v, rbs[m], &nst, &nbl, &nt, &gg);
                const int res = stream_resident(A.npt, v, q);
                ok = ok && res > 0 && nt <= res && nbytes * p.beta_cache_us_per_B < 0.3 * tt[m];
            }
            if (!ok) continue;
            const int s0 = stream_steps_per_tile(v, 1), s1 = stream_steps_per_tile(v, 4);
            const double step = std::max(0.05, (tt[1] - tt[0]) / (s1 - s0));
            (leg == 0 ? sdn : sup).push_back(step);
            (leg == 0 ? fdn : fup).push_back(std::max(0.0, tt[0] - s0 * step));
        }
    }
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    if (!sdn.empty()) {
        p.step_dn_us[q] = median(sdn);
        p.t0_dn_us[q] = median(fdn);
    }
    if (!sup.empty()) {
        p.step_up_us[q] = median(sup);
        p.t0_up_us[q] = median(fup);
    }
    return hipStreamSynchronize(s);
}

hipbmg_status hbmg::calibrate_on_kernels(void *stream, ModelParams &p)
{
    hipStream_t s = (hipStream_t)stream;
    const int n = 257;
    const size_t ncell = (size_t)(n - 1) * (n - 1);
    std::vector<double> ones(ncell, 1.0);
    double *cells = nullptr, *planes = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipbmg_handle h = nullptr;
    hipbmg_status st = HIPBMG_OK;
    auto cleanup = [&] {
        if (h) hipbmg_destroy(h);
        if (cells) (void)hipFree(cells);
        if (planes) (void)hipFree(planes);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (hipMalloc(&cells, ncell * sizeof(double)) != hipSuccess ||
        hipMalloc(&planes, 3 * (size_t)n * n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return fail(HIPBMG_ENOMEM, "calibration: device allocation failed");
    }
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
        hipMemcpyAsync(cells, ones.data(), ncell * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess) {
        cleanup();
        return fail(HIPBMG_EHIP, "calibration: event or copy failed");
    }
    if ((st = hipbmg_fv5_from_cells(n, n, cells, 0, planes, s)) != HIPBMG_OK) {
        cleanup();
        return st;
    }
    hipbmg_params prm;
    hipbmg_default_params(&prm);
    prm.precision = HIPBMG_MIXED;
    prm.collapse_level = 0;
    prm.cluster_wg = 0;
    if ((st = hipbmg_setup(n, n, 5, planes, &prm, stream, &h)) != HIPBMG_OK) {
        cleanup();
        return st;
    }
    void *flush = nullptr;
    const size_t flush_bytes = (size_t)512 << 20;   // beyond L2 and the 256 MB last-level cache
    if (hipMalloc(&flush, flush_bytes) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return fail(HIPBMG_ENOMEM, "calibration: device allocation failed");
    }
    ColdTimer ct{s, e0, e1, flush, flush_bytes};
    hipError_t e = calibrate_precision<double>(h, h->lv, h->d_lv, ct, p);
    if (e == hipSuccess) e = calibrate_precision<float>(h, h->lv32, h->d_lv32, ct, p);
    if (e != hipSuccess) st = fail(HIPBMG_EHIP, "calibration launches failed: %s", hipGetErrorString(e));
    (void)hipStreamSynchronize(s);
    (void)hipFree(flush);
    cleanup();
    return st;
}

// ---------------------------------------------------------------------------
// Batched solves: many independent problems of different sizes.  Every
// problem keeps its own hierarchy (and its own collapse level from the model);
// one launch runs the same stage of the V-cycle for all problems (depth d from
// the finest level, the kernel's position within the level), mapping each
// workgroup to a (problem, tile) pair; the collapsed levels run one workgroup
// per problem.  Converged problems are retired on the device and skipped by
// every later launch.  A cycle is captured once as a hipGraph and replayed.
// ---------------------------------------------------------------------------
struct BLaunch {
    int kind;            // 0 streaming stage, 1 collapse, 2 pipelined finest pass
    int npt, variant;
    int wpg;             // streaming stage: strips (waves) per workgroup
    int zc;              // pipelined pass: every problem forms its diagonal
    void *d_args;        // StreamArgs<T>[nprob] or CollapseArgs<T>[nprob]
    int2 *d_map;
    int nmap;
    int lds_bytes;
};

struct BPlan {
    std::vector<BLaunch> launches;
    int end_cur = 0;
    bool built = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void *> allocs;   // device tables of the launches
};

static void drop_plan(BPlan &p)
{
    if (p.exec) (void)hipGraphExecDestroy(p.exec);
    if (p.graph) (void)hipGraphDestroy(p.graph);
    dev_free_all(p.allocs);
    p = BPlan{};
}

struct hipbmg_batch {
    int n = 0;
    hipbmg_params prm{};
    std::vector<hipbmg_hier *> hs;
    std::vector<void *> allocs;
    int *d_active = nullptr, *d_active2 = nullptr, *d_count = nullptr;
    double *d_relres = nullptr, *d_bnorm = nullptr, *d_rnorm = nullptr, *d_irel = nullptr;
    double *d_partials = nullptr, *d_bpart = nullptr;
    int *d_poff = nullptr, *d_pcnt = nullptr, *d_boff = nullptr, *d_bcnt = nullptr;
    int *d_roff = nullptr, *d_rcnt = nullptr;
    double **d_bptr = nullptr, **d_xptr = nullptr;
    int4 *d_dims = nullptr;
    // the caller's arrays of a solve ([0, n) b, [n, 2n) u, [2n, 3n) each
    // problem's result plane) and the first row of each problem in the batch
    const double **d_user = nullptr, **h_user = nullptr;
    int *d_rowoff = nullptr;
    int rows = 0;
    LevelDev<double> *d_fine64 = nullptr;
    LevelDev<float> *d_fine32 = nullptr;
    double *d_rpart = nullptr;   // refinement residual partials (segments d_roff / d_rcnt)
    int n_partials = 0;
    std::vector<int> h_pcnt;
    double *h_relres = nullptr;
    int *h_active = nullptr, *h_count = nullptr;
    double *d_tol = nullptr, *h_tol = nullptr;   // [0] the solve's tolerance, [1] the inner FP32 tolerance
    double *d_itol = nullptr, *h_itol = nullptr; // each problem's inner FP32 tolerance of the current step
    int max_nx = 0, max_ny = 0, fine_npt = 5;
    BPlan plan64[2], plan32[2][2];
    int rb_cap = 0;                           // row blocks of the batched launches (0: per-level rule)
    int wpg = 1;                              // strips (one wave each) per workgroup of the batched launches
    // pipelined finest level: every problem's finest post-relaxation and the
    // next cycle's pre-relaxations run as one pass (as for a single problem)
    bool pipe = false;
    int zc[2] = {0, 0};                       // every problem's pass forms its diagonal (FP64, FP32)
    BPlan pipe64[4], pipe32[4];               // [0..2] a cycle with iterate rotation i, [3] the first cycle
    std::vector<int> cc64, cc32;              // coarse buffer holding each problem's coarse correction
    StreamArgs<double> *d_rb64 = nullptr, *h_rb64 = nullptr;   // rebuild of the stopping cycles' iterates
    StreamArgs<float> *d_rb32 = nullptr, *h_rb32 = nullptr;
    int *d_rbact = nullptr, *h_rbact = nullptr;
    float **d_eptr = nullptr, **h_eptr = nullptr;              // each problem's FP32 correction
    int *h_act2 = nullptr;
    void *h_block = nullptr;                  // pinned block holding every h_ table above
    size_t h_block_cap = 0;
    char *tab_next = nullptr;                 // unused part of the current table chunk
    size_t tab_left = 0;
    std::vector<void *> seg_allocs;           // norm segment tables (rebuilt with the plans)
    hipStream_t ws = nullptr;                 // own stream: graphs cannot be captured on the null stream
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    ~hipbmg_batch()
    {
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (ws) (void)hipStreamDestroy(ws);
        for (auto &p : plan64) drop_plan(p);
        for (auto &q : plan32)
            for (auto &p : q) drop_plan(p);
        for (auto &p : pipe64) drop_plan(p);
        for (auto &p : pipe32) drop_plan(p);
        dev_free_all(seg_allocs);
        dev_free_all(allocs);
        for (hipbmg_hier *h : hs) delete h;   // each waits for the device first
        hbmg::pinned_block_free(h_block, h_block_cap);
    }
};

template <typename T>
static hipbmg_status balloc_to(std::vector<void *> &owner, T **p, size_t n, hipStream_t s)
{
    void *q = nullptr;
    if (dev_malloc(&q, n * sizeof(T) + 64) != hipSuccess) {
        (void)hipGetLastError();
        return fail(HIPBMG_ENOMEM, "device allocation of %zu bytes failed", n * sizeof(T));
    }
    owner.push_back(q);
    HIPCHK(hipMemsetAsync(q, 0, n * sizeof(T) + 64, s));
    *p = static_cast<T *>(q);
    return HIPBMG_OK;
}

// the batch's own tables: up to 256 KiB cut from zeroed 1 MiB chunks, larger
// ones a block each (zeroed, 64 bytes longer than asked)
template <typename T>
static hipbmg_status balloc(hipbmg_batch *B, T **p, size_t n, hipStream_t s)
{
    const size_t bytes = (n * sizeof(T) + 64 + 255) / 256 * 256;
    if (bytes > (size_t(256) << 10)) return balloc_to(B->allocs, p, n, s);
    if (bytes > B->tab_left) {
        char *c = nullptr;
        STCHK(balloc_to(B->allocs, &c, (size_t(1) << 20) - 64, s));
        B->tab_next = c;
        B->tab_left = size_t(1) << 20;
    }
    *p = reinterpret_cast<T *>(B->tab_next);
    B->tab_next += bytes;
    B->tab_left -= bytes;
    return HIPBMG_OK;
}

template <typename T>
static const std::vector<LevelDev<T>> &levels_of(hipbmg_hier *h);
template <>
const std::vector<LevelDev<double>> &levels_of<double>(hipbmg_hier *h) { return h->lv; }
template <>
const std::vector<LevelDev<float>> &levels_of<float>(hipbmg_hier *h) { return h->lv32; }
template <typename T>
static const LevelDev<T> *dlevels_of(hipbmg_hier *h);
template <>
const LevelDev<double> *dlevels_of<double>(hipbmg_hier *h) { return h->d_lv; }
template <>
const LevelDev<float> *dlevels_of<float>(hipbmg_hier *h) { return h->d_lv32; }

// Row blocks of the batched launches: the tiles of all problems share the
// device, so the single-problem residency rounds do not apply; the longest
// of 64, 32, ... 4 that gives a level 1024 tiles of its own keeps the
// prologue overhead low.
template <typename T>
static int batch_rb(const hipbmg_batch *B, const LevelDev<T> &A)
{
    if (const char *e = std::getenv("HIPBMG_RB")) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= 4096) return v;
    }
    if (B->rb_cap > 0) return std::max(1, std::min(B->rb_cap, (A.ny - 1) / 2));
    return pick_rb(A.nx, A.ny, A.npt);
}

// Record the launches of one V-cycle of every problem (same order as
// enqueue_vcycle) and group them into batched stages.  pipe_i >= 0: the
// finest level pipelined, its pass reading iterate buffer pipe_i of
// {x[0], x[1], x3} and writing the next two; pipe_first adds the finest
// pre-relaxations of the first cycle (from x[0], or from zero) before it.
template <typename T>
static hipbmg_status build_plan(hipbmg_batch *B, int cur, bool zero_start, BPlan &plan, hipStream_t s,
                                int pipe_i = -1, bool pipe_first = false)
{
    const int n = B->n;
    const int nu1 = B->prm.nu1, nu2 = B->prm.nu2, rc = B->prm.residual_correction;
    struct Rec {
        int p, npt, variant;
        StreamArgs<T> a;
    };
    // key: phase (0 down, 2 up), depth, k
    std::vector<std::vector<std::vector<Rec>>> down, up;
    std::vector<CollapseArgs<T>> cargs(n);
    int lds_max = 0, end_cur = -1;
    int off = 0;
    std::vector<int> poff(n), pcnt(n);
    for (int p = 0; p < n; ++p) {
        hipbmg_hier *h = B->hs[p];
        const std::vector<LevelDev<T>> &lv = levels_of<T>(h);
        const int L = h->L, ls = h->lstar;
        int xb_after[HIPBMG_MAX_LEVELS], xres[HIPBMG_MAX_LEVELS];
        for (int l = L - 1; l > ls; --l) {
            const int d = L - 1 - l;
            const LevelDev<T> &A = lv[l], &Cl = lv[l - 1];
            const bool fine = l == L - 1;
            if (fine && pipe_i >= 0 && !pipe_first) {
                xb_after[l] = 0;   // the previous cycle's pass did these pre-relaxations
                continue;
            }
            int xb = fine ? cur : 0;
            const bool zero = !fine || zero_start;
            const int nk = (nu1 >= 2 && !h->no_fuse2) ? nu1 - 1 : nu1;
            for (int k = 1; k <= nk; ++k) {
                const bool last = k == nk, zx = zero && k == 1, two = last && nk < nu1;
                const int v = last ? (two ? (zx ? SV_SWEEP2_RQ_ZX : SV_SWEEP2_RQ) : (zx ? SV_SWEEP_RQ_ZX : SV_SWEEP_RQ))
                                   : (zx ? SV_SWEEP_ZX : SV_SWEEP);
                StreamArgs<T> a = base_args(A, batch_rb(B, A));
                a.x_in = A.x[xb];
                a.x_out = A.x[1 - xb];
                if (last) {
                    a.q_out = A.q;
                    a.bc = Cl.b;
                    a.wt = A.wt;
                    a.cnx = Cl.nx;
                    a.cny = Cl.ny;
                    a.cpitch = Cl.pitch;
                    a.cplane = (long long)Cl.plane;
                }
                int g;
                stream_geometry(A.nx, A.ny, A.npt, v, a.rb, &a.nstrips, &a.nblocks, &a.ntiles, &g);
                if ((int)down.size() <= d) down.resize(d + 1);
                if ((int)down[d].size() < k) down[d].resize(k);
                down[d][k - 1].push_back({p, A.npt, v, a});
                xb = 1 - xb;
            }
            xb_after[l] = xb;
        }
        const bool cfine = ls == L - 1;
        CollapseArgs<T> c = collapse_args<T>(h, lv, dlevels_of<T>(h), ls, cfine ? cur : 1,
                                             cfine ? (zero_start ? 1 : 0) : 1, cfine ? 1 : 0);
        lds_max = std::max(lds_max, c.lds_bytes);
        xres[ls] = c.xb_top;
        int pc = 1;
        for (int l = ls + 1; l < L; ++l) {
            const int d = L - 1 - l;
            const LevelDev<T> &A = lv[l], &Cl = lv[l - 1];
            const bool fine = l == L - 1;
            if (fine && pipe_i >= 0) {
                // this cycle's interpolation, relaxation and norm, and the
                // next cycle's pre-relaxations and restriction, in one pass
                T *x3[3] = {A.x[0], A.x[1], x3_of<T>(h)};
                StreamArgs<T> a = base_args(A, batch_rb(B, A));
                a.x_in = x3[pipe_i];
                a.x_out = x3[(pipe_i + 1) % 3];
                a.x_out2 = x3[(pipe_i + 2) % 3];
                a.xc = Cl.x[xres[l - 1]];
                a.wt = A.wt;
                a.rescorr = rc;
                a.bc = Cl.b;
                a.cnx = Cl.nx;
                a.cny = Cl.ny;
                a.cpitch = Cl.pitch;
                a.cplane = (long long)Cl.plane;
                a.zexc = B->zc[PrecIdx<T>::v];
                int g;
                stream_geometry(A.nx, A.ny, A.npt, SV_FUSED3, a.rb, &a.nstrips, &a.nblocks, &a.ntiles, &g);
                pc = a.ntiles;
                if ((int)up.size() <= d) up.resize(d + 1);
                if (up[d].empty()) up[d].resize(1);
                up[d][0].push_back({p, A.npt, SV_FUSED3, a});
                (PrecIdx<T>::v ? B->cc32 : B->cc64)[p] = xres[l - 1];
                xres[l] = (pipe_i + 2) % 3;
                continue;
            }
            int xb = xb_after[l];
            for (int k = 1; k <= nu2; ++k) {
                const bool first = k == 1, last = k == nu2;
                const int v = first ? (fine && last ? SV_INTERP_NORM : SV_INTERP) : (fine && last ? SV_SWEEP_NORM : SV_SWEEP);
                StreamArgs<T> a = base_args(A, batch_rb(B, A));
                a.x_in = A.x[xb];
                a.x_out = A.x[1 - xb];
                if (first) {
                    a.xc = Cl.x[xres[l - 1]];
                    a.wt = A.wt;
                    a.q_in = A.q;
                    a.rescorr = rc;
                    a.cnx = Cl.nx;
                    a.cny = Cl.ny;
                    a.cpitch = Cl.pitch;
                    a.cplane = (long long)Cl.plane;
                }
                int g;
                stream_geometry(A.nx, A.ny, A.npt, v, a.rb, &a.nstrips, &a.nblocks, &a.ntiles, &g);
                if (fine && last) pc = a.ntiles;
                if ((int)up.size() <= d) up.resize(d + 1);
                if ((int)up[d].size() < k) up[d].resize(k);
                up[d][k - 1].push_back({p, A.npt, v, a});
                xb = 1 - xb;
            }
            xres[l] = xb;
        }
        const int ec = xres[L - 1];
        if (end_cur >= 0 && ec != end_cur) return fail(HIPBMG_EINVAL, "batched plan: buffer parity differs between problems");
        end_cur = ec;
        poff[p] = off;
        pcnt[p] = pc;
        off += pc;
        cargs[p] = c;
    }
    // partial-sum segments of the finest norm: the same geometry (hence the
    // same segments) for every plan of the batch, so one buffer serves all
    if (!B->d_partials) {
        STCHK(balloc_to(B->seg_allocs, &B->d_partials, (size_t)off + 1, s));
        STCHK(balloc_to(B->seg_allocs, &B->d_poff, n, s));
        STCHK(balloc_to(B->seg_allocs, &B->d_pcnt, n, s));
        HIPCHK(hipMemcpyAsync(B->d_poff, poff.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(B->d_pcnt, pcnt.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
        B->n_partials = off;
        B->h_pcnt = pcnt;
    } else if (off != B->n_partials || pcnt != B->h_pcnt) {
        return fail(HIPBMG_EINVAL, "batched plan: norm segments differ between plans");
    }
    double *parts = B->d_partials;
    for (auto &dd : up)
        for (auto &kk : dd)
            for (Rec &r : kk) r.a.partials = parts + poff[r.p];
    for (int p = 0; p < n; ++p) cargs[p].partials = parts + poff[p];
    // materialise the stages: every launch's tables are packed into one host
    // buffer, uploaded to one device block of the plan (one allocation and one
    // copy per plan, not two of each per launch)
    const size_t first_launch = plan.launches.size();
    std::vector<char> tab;
    std::vector<std::pair<size_t, size_t>> offs;   // per launch: args, map (SIZE_MAX: none)
    auto put = [&](const void *src, size_t bytes) {
        const size_t o = (tab.size() + 255) / 256 * 256;
        tab.resize(o + bytes);
        std::memcpy(tab.data() + o, src, bytes);
        return o;
    };
    auto add_stage = [&](std::vector<Rec> &recs) -> hipbmg_status {
        if (recs.empty()) return HIPBMG_OK;
        std::vector<StreamArgs<T>> args(n);
        std::vector<int2> map;
        for (Rec &r : recs) {
            if (r.variant != recs[0].variant || r.npt != recs[0].npt)
                return fail(HIPBMG_EINVAL, "batched plan: mixed kernels in one stage");
            args[r.p] = r.a;
            for (int tl = 0; tl < r.a.ntiles; ++tl) map.push_back(make_int2(r.p, tl));
        }
        BLaunch bl{};
        bl.kind = recs[0].variant == SV_FUSED3 ? 2 : 0;
        bl.npt = recs[0].npt;
        bl.variant = recs[0].variant;
        bl.wpg = B->wpg;
        bl.zc = B->zc[PrecIdx<T>::v];
        const size_t oa = put(args.data(), n * sizeof(StreamArgs<T>));
        const size_t om = put(map.data(), map.size() * sizeof(int2));
        offs.push_back({oa, om});
        bl.nmap = (int)map.size();
        plan.launches.push_back(bl);
        return HIPBMG_OK;
    };
    for (size_t d = 0; d < down.size(); ++d)
        for (auto &kk : down[d]) STCHK(add_stage(kk));
    {
        BLaunch bl{};
        bl.kind = 1;
        offs.push_back({put(cargs.data(), n * sizeof(CollapseArgs<T>)), SIZE_MAX});
        bl.lds_bytes = lds_max;
        plan.launches.push_back(bl);
    }
    for (int d = (int)up.size() - 1; d >= 0; --d)
        for (auto &kk : up[d]) STCHK(add_stage(kk));
    char *dt = nullptr;
    STCHK(balloc_to(plan.allocs, &dt, tab.size(), s));
    HIPCHK(hipMemcpyAsync(dt, tab.data(), tab.size(), hipMemcpyHostToDevice, s));
    for (size_t k = 0; k < offs.size(); ++k) {
        BLaunch &bl = plan.launches[first_launch + k];
        bl.d_args = dt + offs[k].first;
        bl.d_map = offs[k].second == SIZE_MAX ? nullptr : reinterpret_cast<int2 *>(dt + offs[k].second);
    }
    HIPCHK(hipStreamSynchronize(s));
    plan.end_cur = end_cur;
    plan.built = true;
    return HIPBMG_OK;
}

template <typename T>
static hipError_t run_plan_launches(hipbmg_batch *B, BPlan &plan, const int *active, hipStream_t s)
{
    hipError_t e = hipSuccess;
    for (BLaunch &bl : plan.launches) {
        if (bl.kind == 0)
            e = launch_stream_batched<T>(bl.npt, bl.variant, static_cast<const StreamArgs<T> *>(bl.d_args),
                                         bl.d_map, bl.nmap, active, bl.wpg, s);
        else if (bl.kind == 2)
            e = launch_stream3_batched<T>(bl.variant, bl.zc, static_cast<const StreamArgs<T> *>(bl.d_args),
                                          bl.d_map, bl.nmap, active, bl.wpg, s);
        else
            e = launch_collapse_batched<T>(static_cast<const CollapseArgs<T> *>(bl.d_args), B->n,
                                           bl.lds_bytes, active, s);
        if (e != hipSuccess) return e;
    }
    return e;
}

// one V-cycle of all active problems plus their residual norms and
// retirement; replayed from a captured graph when use_graph is set
template <typename T>
static hipbmg_status batch_cycle(hipbmg_batch *B, BPlan &plan, int *active, const double *denom, double *out,
                                 const double *tol_dev, hipStream_t s, int tol_stride = 0)
{
    // the tolerance is read from device memory when the test runs: a replayed
    // graph then applies the tolerance of the current solve, not the one of
    // the solve that captured it
    auto enqueue = [&]() -> hipError_t {
        hipError_t e = run_plan_launches<T>(B, plan, active, s);
        if (e != hipSuccess) return e;
        e = launch_finalize_batched(B->d_partials, B->d_poff, B->d_pcnt, denom, out, active, 0.0, tol_dev, B->n,
                                    s, tol_stride);
        if (e != hipSuccess) return e;
        return launch_count_active(active, B->n, B->d_count, s);
    };
    if (!B->prm.use_graph) {
        HIPCHK(enqueue());
        return HIPBMG_OK;
    }
    // one graph per (plan, active buffer, denominator, output) combination:
    // the plans are only ever used with one combination each
    if (!plan.exec) {
        HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue();
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(s, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(HIPBMG_EHIP, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
        }
        plan.graph = g;
        HIPCHK(hipGraphInstantiate(&plan.exec, g, nullptr, nullptr, 0));
    }
    HIPCHK(hipGraphLaunch(plan.exec, s));
    return HIPBMG_OK;
}

static hipbmg_status batch_read(hipbmg_batch *B, const double *d_vals, const int *d_act, hipStream_t s)
{
    HIPCHK(hipMemcpyAsync(B->h_relres, d_vals, B->n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(B->h_active, d_act, B->n * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(B->h_count, B->d_count, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return HIPBMG_OK;
}

// (Re)build every plan of the batch for its current row blocks: FP64 cycles
// from buffer 0 (and from 1 if a cycle changes the parity); FP32 inner cycles
// from zero, then from where the previous cycle ended.
static hipbmg_status build_plans(hipbmg_batch *B, hipStream_t s)
{
    HIPCHK(hipStreamSynchronize(s));
    for (auto &p : B->plan64) drop_plan(p);
    for (auto &q : B->plan32)
        for (auto &p : q) drop_plan(p);
    for (auto &p : B->pipe64) drop_plan(p);
    for (auto &p : B->pipe32) drop_plan(p);
    dev_free_all(B->seg_allocs);
    B->d_partials = nullptr;
    B->d_poff = B->d_pcnt = nullptr;
    B->n_partials = 0;
    B->h_pcnt.clear();
    if (B->pipe) {
        // the first cycle (pre-relaxations from x[0] or zero, then the pass
        // on buffer 1) and the three buffer rotations of the later cycles
        hipbmg_status st = HIPBMG_OK;
        if (B->prm.precision == HIPBMG_MIXED) {
            st = build_plan<float>(B, 0, true, B->pipe32[3], s, 1, true);
            for (int i = 0; i < 3 && st == HIPBMG_OK; ++i) st = build_plan<float>(B, 0, false, B->pipe32[i], s, i);
        } else {
            st = build_plan<double>(B, 0, false, B->pipe64[3], s, 1, true);
            for (int i = 0; i < 3 && st == HIPBMG_OK; ++i) st = build_plan<double>(B, 0, false, B->pipe64[i], s, i);
        }
        return st;
    }
    hipbmg_status st = build_plan<double>(B, 0, false, B->plan64[0], s);
    if (st == HIPBMG_OK && B->plan64[0].end_cur != 0) st = build_plan<double>(B, 1, false, B->plan64[1], s);
    if (st == HIPBMG_OK && B->prm.precision == HIPBMG_MIXED) {
        st = build_plan<float>(B, 0, true, B->plan32[1][0], s);
        const int c1 = B->plan32[1][0].end_cur;
        if (st == HIPBMG_OK) st = build_plan<float>(B, c1, false, B->plan32[0][c1], s);
        const int c2 = B->plan32[0][c1].end_cur;
        if (st == HIPBMG_OK && c2 != c1) st = build_plan<float>(B, c2, false, B->plan32[0][c2], s);
    }
    return st;
}

template <typename T>
static double time_plan_us(hipbmg_batch *B, BPlan &plan, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    (void)run_plan_launches<T>(B, plan, B->d_active, s);   // warm-up
    double best = 1e30;
    for (int r = 0; r < 3; ++r) {
        (void)hipEventRecord(e0, s);
        (void)run_plan_launches<T>(B, plan, B->d_active, s);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        best = std::min(best, 1e3 * (double)ms);
    }
    return best;
}

// Autotuner of the batched tile shape.  A workgroup's tile is W neighbouring
// strips of column pairs (one wave each, 54-62 owned pairs per strip by the
// kernel's halo) times a block of rb row-pair steps; in a batched launch the
// tiles of every problem share the device, so the best shape is not the
// single-problem one.  Each candidate (W in {1, 2, 4}) x (cap on rb in
// {1, ..., 64}, or the single-problem rule) is built into plans and one
// steady-state V-cycle of the batch is timed (every problem active, on the
// zero data of a fresh hierarchy); the fastest is kept.  The choice is
// remembered per batch signature (sizes, stencil, precision, cycle) for the
// life of the process.  HIPBMG_BATCH_TUNE=0 keeps one strip per workgroup
// and the single-problem rule; HIPBMG_BATCH_WPG=1, 2 or 4 fixes W.
static hipbmg_status tune_batch(hipbmg_batch *B, hipStream_t s)
{
    // shared by every thread that sets up batches: guarded; the key holds
    // every parameter that shapes the plans
    static std::mutex cache_mu;
    static std::map<std::string, std::pair<int, int>> cache;
    std::vector<std::pair<int, int>> sz;
    for (hipbmg_hier *h : B->hs) sz.push_back({h->nx, h->ny});
    std::sort(sz.begin(), sz.end());
    std::string key = std::to_string(B->fine_npt) + "/" + std::to_string(B->prm.precision) + "/" +
                      std::to_string(B->prm.nu1) + "," + std::to_string(B->prm.nu2) + "/c" +
                      std::to_string(B->prm.coarsest_n) + "/l" + std::to_string(B->prm.collapse_level) + "/r" +
                      std::to_string(B->prm.residual_correction) + ":";
    for (auto &q : sz) key += std::to_string(q.first) + "x" + std::to_string(q.second) + ";";
    bool tune = true;
    if (const char *e = std::getenv("HIPBMG_BATCH_TUNE")) tune = std::atoi(e) != 0;
    int wfix = 0;
    if (const char *e = std::getenv("HIPBMG_BATCH_WPG")) {
        const int v = std::atoi(e);
        if (v == 1 || v == 2 || v == 4) wfix = v;
    }
    key += "w" + std::to_string(wfix) + "p" + std::to_string(B->pipe ? 1 : 0);
    if (!tune) {
        B->rb_cap = 0;
        B->wpg = wfix ? wfix : 1;
        return build_plans(B, s);
    }
    {
        std::lock_guard<std::mutex> lk(cache_mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            B->rb_cap = it->second.first;
            B->wpg = it->second.second;
        } else {
            B->rb_cap = -1;
        }
    }
    if (B->rb_cap >= 0) return build_plans(B, s);
    std::vector<int> ones(B->n, 1);
    HIPCHK(hipMemcpyAsync(B->d_active, ones.data(), B->n * sizeof(int), hipMemcpyHostToDevice, s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(HIPBMG_EHIP, "event creation failed");
    }
    const bool mixed = B->prm.precision == HIPBMG_MIXED;
    int best = 0, best_w = 1;
    double tbest = 1e30;
    hipbmg_status st = HIPBMG_OK;
    for (int w : {1, 2, 4}) {
        if (wfix && w != wfix) continue;
        B->wpg = w;
        for (int cap : {0, 1, 2, 4, 8, 16, 32, 64}) {
            B->rb_cap = cap;
            if ((st = build_plans(B, s)) != HIPBMG_OK) break;
            double us;
            if (B->pipe) {
                us = mixed ? time_plan_us<float>(B, B->pipe32[0], s, e0, e1)
                           : time_plan_us<double>(B, B->pipe64[0], s, e0, e1);
            } else if (mixed) {
                const int c1 = B->plan32[1][0].end_cur;
                us = time_plan_us<float>(B, B->plan32[0][c1], s, e0, e1);
            } else {
                us = time_plan_us<double>(B, B->plan64[0], s, e0, e1);
            }
            if (std::getenv("HIPBMG_VERBOSE"))
                std::fprintf(stderr, "hipbmg: batch of %d, %d strips per workgroup, row-block cap %d: %.1f us per cycle\n",
                             B->n, w, cap, us);
            if (us < tbest) {
                tbest = us;
                best = cap;
                best_w = w;
            }
        }
        if (st != HIPBMG_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != HIPBMG_OK) return st;
    HIPCHK(hipMemsetAsync(B->d_active, 0, B->n * sizeof(int), s));
    {
        std::lock_guard<std::mutex> lk(cache_mu);
        cache[key] = {best, best_w};
    }
    B->rb_cap = best;
    B->wpg = best_w;
    return build_plans(B, s);
}

extern "C" hipbmg_status hipbmg_setup_batched(int nprob, const int *nx, const int *ny, int npt,
                                              const double *const *coeffs, const hipbmg_params *params,
                                              void *stream, hipbmg_batch_handle *out)
{
    if (!out) return fail(HIPBMG_EINVAL, "out is NULL");
    *out = nullptr;
    if (nprob < 1 || !nx || !ny || !coeffs) return fail(HIPBMG_EINVAL, "bad batch arguments");
    hipStream_t s = (hipStream_t)stream;
    hipbmg_params prm;
    hipbmg_default_params(&prm);
    if (params) prm = *params;
    prm.cluster_wg = 0;   // a batch collapses each problem at its own l*, no stages
    hipbmg_batch *B = new hipbmg_batch();
    B->n = nprob;
    B->prm = prm;
    auto bail = [&](hipbmg_status st) {
        std::string m = g_err;
        delete B;
        g_err = m;
        return st;
    };
    // The problems' hierarchies are independent: the first is built on the
    // caller's stream, the others on several host threads with a stream each
    // (HIPBMG_SETUP_THREADS, default 8; 1 builds them in turn), so that one
    // problem's kernels run while another's host steps and read-backs go on.
    {
        B->hs.assign(nprob, nullptr);
        std::vector<hipbmg_status> sts(nprob, HIPBMG_OK);
        std::vector<std::string> msgs(nprob);
        auto build = [&](int p, hipStream_t sp) {
            sts[p] = hipbmg_setup(nx[p], ny[p], npt, coeffs[p], &prm, sp, &B->hs[p]);
            if (sts[p] != HIPBMG_OK) msgs[p] = g_err;   // the worker's own last error
        };
        build(0, s);
        int nth = 8;
        if (const char *e = std::getenv("HIPBMG_SETUP_THREADS")) nth = std::max(1, std::atoi(e));
        nth = std::min(nth, nprob - 1);
        if (sts[0] == HIPBMG_OK && nth >= 1) {
            int dev = 0;
            if (hipGetDevice(&dev) != hipSuccess) return bail(fail(HIPBMG_EHIP, "hipGetDevice failed"));
            std::atomic<int> next{1};
            std::vector<std::thread> pool;
            for (int t = 0; t < nth; ++t)
                pool.emplace_back([&, t] {
                    (void)t;
                    hipStream_t sp = nullptr;
                    if (hipSetDevice(dev) != hipSuccess ||
                        hipStreamCreateWithFlags(&sp, hipStreamNonBlocking) != hipSuccess) {
                        (void)hipGetLastError();
                        sp = nullptr;
                    }
                    for (int p; (p = next.fetch_add(1)) < nprob;) {
                        if (!sp) {
                            sts[p] = HIPBMG_EHIP;
                            msgs[p] = "cannot create a setup stream";
                            continue;
                        }
                        build(p, sp);
                    }
                    if (sp) {
                        (void)hipStreamSynchronize(sp);
                        (void)hipStreamDestroy(sp);
                    }
                });
            for (std::thread &th : pool) th.join();
        } else if (sts[0] == HIPBMG_OK) {
            for (int p = 1; p < nprob; ++p) build(p, s);
        }
        for (int p = 0; p < nprob; ++p)
            if (sts[p] != HIPBMG_OK) {
                (void)fail(sts[p], "problem %d: %s", p, msgs[p].c_str());
                return bail(sts[p]);
            }
        for (int p = 0; p < nprob; ++p) {
            B->max_nx = std::max(B->max_nx, nx[p]);
            B->max_ny = std::max(B->max_ny, ny[p]);
        }
    }
    B->fine_npt = npt;
    hipbmg_status st = HIPBMG_OK;
    auto chk = [&](hipbmg_status x) {
        if (st == HIPBMG_OK) st = x;
    };
    chk(balloc(B, &B->d_active, nprob, s));
    chk(balloc(B, &B->d_active2, nprob, s));
    chk(balloc(B, &B->d_count, 1, s));
    chk(balloc(B, &B->d_tol, 2, s));
    chk(balloc(B, &B->d_itol, nprob, s));
    chk(balloc(B, &B->d_relres, nprob, s));
    chk(balloc(B, &B->d_bnorm, nprob, s));
    chk(balloc(B, &B->d_rnorm, nprob, s));
    chk(balloc(B, &B->d_irel, nprob, s));
    chk(balloc(B, &B->d_bpart, (size_t)nprob * 64, s));
    chk(balloc(B, &B->d_boff, nprob, s));
    chk(balloc(B, &B->d_bcnt, nprob, s));
    chk(balloc(B, &B->d_roff, (size_t)nprob + 1, s));
    chk(balloc(B, &B->d_rcnt, nprob, s));
    chk(balloc(B, &B->d_bptr, nprob, s));
    chk(balloc(B, &B->d_xptr, nprob, s));
    chk(balloc(B, &B->d_dims, nprob, s));
    chk(balloc(B, &B->d_user, 3 * (size_t)nprob, s));
    chk(balloc(B, &B->d_rowoff, (size_t)nprob + 1, s));
    chk(balloc(B, &B->d_fine64, nprob, s));
    if (prm.precision == HIPBMG_MIXED) chk(balloc(B, &B->d_fine32, nprob, s));
    if (st != HIPBMG_OK) return bail(st);
    std::vector<int> boff(nprob), bcnt(nprob, 64), roff(nprob + 1), rcnt(nprob);
    std::vector<double *> bptr(nprob), xptr(nprob);
    std::vector<int4> dims(nprob);
    std::vector<int> rowoff(nprob + 1, 0);
    std::vector<LevelDev<double>> f64(nprob);
    std::vector<LevelDev<float>> f32(nprob);
    size_t roffs = 0;
    for (int p = 0; p < nprob; ++p) {
        const LevelDev<double> &F = B->hs[p]->lv[B->hs[p]->L - 1];
        boff[p] = 64 * p;
        bptr[p] = F.b;
        xptr[p] = F.x[0];
        dims[p] = make_int4(F.nx, F.ny, F.pitch, 0);
        rowoff[p + 1] = rowoff[p] + F.ny;
        f64[p] = F;
        if (prm.precision == HIPBMG_MIXED) f32[p] = B->hs[p]->lv32[B->hs[p]->L - 1];
        roff[p] = (int)roffs;
        rcnt[p] = ((F.nx + 255) / 256) * F.ny;
        roffs += rcnt[p];
    }
    roff[nprob] = (int)roffs;
    if (balloc(B, &B->d_rpart, roffs + 1, s) != HIPBMG_OK) return bail(HIPBMG_ENOMEM);
    auto up = [&](void *dst, const void *src, size_t bytes) {
        if (st == HIPBMG_OK && hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) != hipSuccess)
            st = fail(HIPBMG_EHIP, "batch table upload failed");
    };
    up(B->d_boff, boff.data(), nprob * sizeof(int));
    up(B->d_bcnt, bcnt.data(), nprob * sizeof(int));
    up(B->d_roff, roff.data(), (nprob + 1) * sizeof(int));
    up(B->d_rcnt, rcnt.data(), nprob * sizeof(int));
    up(B->d_bptr, bptr.data(), nprob * sizeof(double *));
    up(B->d_xptr, xptr.data(), nprob * sizeof(double *));
    up(B->d_dims, dims.data(), nprob * sizeof(int4));
    up(B->d_rowoff, rowoff.data(), (nprob + 1) * sizeof(int));
    B->rows = rowoff[nprob];
    up(B->d_fine64, f64.data(), nprob * sizeof(LevelDev<double>));
    if (prm.precision == HIPBMG_MIXED) up(B->d_fine32, f32.data(), nprob * sizeof(LevelDev<float>));
    if (st != HIPBMG_OK) return bail(st);
    // the batch's pinned host tables, cut from one pooled block
    {
        size_t need = 0;
        auto room = [&](size_t bytes) {
            const size_t o = need;
            need += (bytes + 63) & ~size_t(63);
            return o;
        };
        const size_t n = (size_t)nprob;
        const size_t o_relres = room(n * sizeof(double)), o_active = room(n * sizeof(int)),
                     o_count = room(sizeof(int)), o_tol = room(2 * sizeof(double)),
                     o_itol = room(n * sizeof(double)), o_user = room(3 * n * sizeof(double *)),
                     o_rb64 = room(n * sizeof(StreamArgs<double>)), o_rb32 = room(n * sizeof(StreamArgs<float>)),
                     o_rbact = room(n * sizeof(int)), o_eptr = room(n * sizeof(float *)),
                     o_act2 = room(n * sizeof(int));
        if (hbmg::pinned_block(&B->h_block, need, &B->h_block_cap) != hipSuccess)
            return bail(fail(HIPBMG_ENOMEM, "hipHostMalloc failed"));
        char *base = static_cast<char *>(B->h_block);
        B->h_relres = reinterpret_cast<double *>(base + o_relres);
        B->h_active = reinterpret_cast<int *>(base + o_active);
        B->h_count = reinterpret_cast<int *>(base + o_count);
        B->h_tol = reinterpret_cast<double *>(base + o_tol);
        B->h_itol = reinterpret_cast<double *>(base + o_itol);
        B->h_user = reinterpret_cast<const double **>(base + o_user);
        B->h_rb64 = reinterpret_cast<StreamArgs<double> *>(base + o_rb64);
        B->h_rb32 = reinterpret_cast<StreamArgs<float> *>(base + o_rb32);
        B->h_rbact = reinterpret_cast<int *>(base + o_rbact);
        B->h_eptr = reinterpret_cast<float **>(base + o_eptr);
        B->h_act2 = reinterpret_cast<int *>(base + o_act2);
    }
    // the finest level pipelined across cycles when every problem's is (as
    // hipbmg_setup decided it: 5-point, V(2,1), not collapsed); its pass forms
    // the diagonal when every problem's operator allows it.
    // HIPBMG_BATCH_PIPE=0 keeps one pass per leg.
    {
        bool pipe = true;
        if (const char *e = std::getenv("HIPBMG_BATCH_PIPE")) pipe = std::atoi(e) != 0;
        B->zc[0] = B->zc[1] = 1;
        for (hipbmg_hier *h : B->hs) {
            pipe = pipe && h->fused3 && h->lstar < h->L - 1;
            B->zc[0] = B->zc[0] && h->zexc[0];
            B->zc[1] = B->zc[1] && h->zexc[1];
        }
        B->pipe = pipe;
        B->cc64.assign(nprob, 0);
        B->cc32.assign(nprob, 0);
        if (pipe) {
            if (prm.precision == HIPBMG_MIXED) {
                chk(balloc(B, &B->d_rb32, nprob, s));
                chk(balloc(B, &B->d_eptr, nprob, s));
            } else {
                chk(balloc(B, &B->d_rb64, nprob, s));
            }
            chk(balloc(B, &B->d_rbact, nprob, s));
            if (st != HIPBMG_OK) return bail(st);
        }
    }
    st = tune_batch(B, s);
    if (st != HIPBMG_OK) return bail(st);
    if (hipStreamSynchronize(s) != hipSuccess) return bail(fail(HIPBMG_EHIP, "batch setup failed"));
    if (hipStreamCreateWithFlags(&B->ws, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming) != hipSuccess)
        return bail(fail(HIPBMG_EHIP, "stream creation failed"));
    *out = B;
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_batch_tile_shape(hipbmg_batch_handle B, int problem, int level,
                                                 int *strips_per_group, int *rb_cap, int *rb)
{
    if (!B) return fail(HIPBMG_EINVAL, "handle is NULL");
    if (problem < 0 || problem >= B->n) return fail(HIPBMG_EINVAL, "problem %d out of range [0, %d)", problem, B->n);
    const hipbmg_hier *h = B->hs[problem];
    if (level < 0 || level >= h->L) return fail(HIPBMG_EINVAL, "level %d out of range [0, %d)", level, h->L);
    if (strips_per_group) *strips_per_group = B->wpg;
    if (rb_cap) *rb_cap = B->rb_cap;
    if (rb) *rb = level > h->lstar ? batch_rb<double>(B, h->lv[level]) : 0;
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_destroy_batched(hipbmg_batch_handle B)
{
    if (B) {
        (void)hipDeviceSynchronize();
        delete B;
    }
    return HIPBMG_OK;
}

// ||b|| per problem; the finest level's b and x[0] are loaded beforehand
static hipbmg_status batch_bnorm(hipbmg_batch *B, hipStream_t s)
{
    HIPCHK(launch_sumsq_batched(B->d_bptr, B->d_dims, B->n, B->d_bpart, 64, s));
    HIPCHK(launch_finalize_batched(B->d_bpart, B->d_boff, B->d_bcnt, nullptr, B->d_bnorm, nullptr, 0.0, nullptr,
                                   B->n, s));
    return HIPBMG_OK;
}

// The pipelined pass does not store the iterate after its own cycle.  After
// the cycles, every problem's iterate after its stopping cycle kstop[p] (0:
// none) is rebuilt by the pass's interpolation and relaxation stage alone from
// that cycle's inputs, which the later launches (skipped once the problem
// retired) left untouched; cycle k ran the pass on buffer (1 + 2 (k - 1)) mod 3
// of {x[0], x[1], x3}.  out[p] receives the buffer holding the iterate.
template <typename T>
static hipbmg_status batch_rebuild(hipbmg_batch *B, const BPlan &plan, const std::vector<int> &kstop,
                                   StreamArgs<T> *h_args, StreamArgs<T> *d_args, std::vector<T *> &out,
                                   hipStream_t s)
{
    const BLaunch &fl = plan.launches.back();   // the pass's stage: every problem's tiles
    if (fl.kind != 2) return fail(HIPBMG_EINVAL, "batched plan: no pipelined pass to rebuild from");
    const int rc = B->prm.residual_correction;
    bool any = false;
    for (int p = 0; p < B->n; ++p) {
        hipbmg_hier *h = B->hs[p];
        const std::vector<LevelDev<T>> &lv = levels_of<T>(h);
        const LevelDev<T> &F = lv[h->L - 1], &Cl = lv[h->L - 2];
        T *x3[3] = {F.x[0], F.x[1], x3_of<T>(h)};
        h_args[p] = StreamArgs<T>{};
        B->h_rbact[p] = kstop[p] > 0;
        out[p] = x3[0];
        if (kstop[p] <= 0) continue;
        any = true;
        const int i = (1 + 2 * (kstop[p] - 1)) % 3;
        StreamArgs<T> a = base_args(F, batch_rb(B, F));
        a.x_in = x3[i];
        a.x_out = x3[(i + 1) % 3];
        a.xc = Cl.x[(PrecIdx<T>::v ? B->cc32 : B->cc64)[p]];
        a.wt = F.wt;
        a.rescorr = rc;
        a.cnx = Cl.nx;
        a.cny = Cl.ny;
        a.cpitch = Cl.pitch;
        a.cplane = (long long)Cl.plane;
        int g;
        stream_geometry(F.nx, F.ny, F.npt, SV_FUSED3, a.rb, &a.nstrips, &a.nblocks, &a.ntiles, &g);
        h_args[p] = a;
        out[p] = x3[(i + 1) % 3];
    }
    if (!any) return HIPBMG_OK;
    HIPCHK(hipMemcpyAsync(d_args, h_args, B->n * sizeof(StreamArgs<T>), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(B->d_rbact, B->h_rbact, B->n * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(launch_stream3_batched<T>(SV_FUSED3_P, fl.zc, d_args, fl.d_map, fl.nmap, B->d_rbact, fl.wpg, s));
    return HIPBMG_OK;
}

extern "C" hipbmg_status hipbmg_solve_batched(hipbmg_batch_handle B, const double *const *b, double *const *u,
                                              double tol, void *stream, hipbmg_info *infos)
{
    const double t0 = now_ms();
    if (!B) return fail(HIPBMG_EINVAL, "null handle");
    if (!b || !u) return fail(HIPBMG_EINVAL, "b and u must be arrays of device pointers");
    if (!(tol > 0.0)) return fail(HIPBMG_EINVAL, "tol must be > 0");
    // the batch works on its own stream, ordered after the caller's stream's
    // earlier work and before its later work
    hipStream_t s_user = (hipStream_t)stream;
    hipStream_t s = B->ws;
    HIPCHK(hipEventRecord(B->ev_in, s_user));
    HIPCHK(hipStreamWaitEvent(s, B->ev_in, 0));
    const int n = B->n;
    for (int p = 0; p < n; ++p)
        if (!b[p] || !u[p]) return fail(HIPBMG_EINVAL, "problem %d: null pointer", p);
    // every problem's b and u into its finest level in one launch, the
    // boundary ring cleared
    for (int p = 0; p < n; ++p) {
        B->h_user[p] = b[p];
        B->h_user[n + p] = u[p];
    }
    HIPCHK(hipMemcpyAsync(B->d_user, B->h_user, 2 * n * sizeof(double *), hipMemcpyHostToDevice, s));
    HIPCHK(launch_stage_batched(B->d_user, B->d_bptr, B->d_xptr, B->d_dims, B->d_rowoff, n, B->rows, 0, s));
    for (int p = 0; p < n; ++p) {
        hipbmg_hier *h = B->hs[p];
        const LevelDev<double> &F = h->lv[h->L - 1];
        if (infos) {
            memset(&infos[p], 0, sizeof(hipbmg_info));
            fill_info_common(h, &infos[p]);
            for (int l = 0; l < h->L; ++l) infos[p].rb_down[l] = infos[p].rb_up[l] = batch_rb(B, h->lv[l]);
            infos[p].rb_pipelined = B->pipe ? batch_rb(B, F) : 0;
        }
    }
    STCHK(batch_bnorm(B, s));
    HIPCHK(hipMemcpyAsync(B->h_relres, B->d_bnorm, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<double> bnorm(B->h_relres, B->h_relres + n);
    std::vector<int> act(n), cycles(n, 0), steps(n, 0), done_cur(n, 0);
    std::vector<double> rel(n, 0.0);
    int nbad = 0;
    for (int p = 0; p < n; ++p) {
        act[p] = bnorm[p] > 0.0 && std::isfinite(bnorm[p]);
        if (!std::isfinite(bnorm[p])) ++nbad;
    }
    HIPCHK(hipMemcpyAsync(B->d_active, act.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
    // the tolerances the (possibly graph-replayed) convergence tests read
    B->h_tol[0] = tol;
    B->h_tol[1] = B->prm.inner_tol;
    HIPCHK(hipMemcpyAsync(B->d_tol, B->h_tol, 2 * sizeof(double), hipMemcpyHostToDevice, s));
    hipbmg_status result = HIPBMG_OK;
    int cur = 0;
    std::vector<double *> res64(n, nullptr);
    if (B->prm.precision != HIPBMG_MIXED && B->pipe) {
        std::vector<int> kstop(n, 0);
        int i = 1;
        for (int c = 0; c < B->prm.max_cycles; ++c) {
            BPlan &plan = c == 0 ? B->pipe64[3] : B->pipe64[i];
            STCHK(batch_cycle<double>(B, plan, B->d_active, B->d_bnorm, B->d_relres, B->d_tol, s));
            STCHK(batch_read(B, B->d_relres, B->d_active, s));
            for (int p = 0; p < n; ++p)
                if (act[p]) {
                    rel[p] = B->h_relres[p];
                    if (infos && cycles[p] < HIPBMG_MAX_HIST) infos[p].relres_hist[cycles[p]] = rel[p];
                    kstop[p] = ++cycles[p];
                    if (!B->h_active[p]) act[p] = 0;
                }
            i = plan.end_cur;
            if (B->h_count[0] == 0) break;
        }
        STCHK(batch_rebuild<double>(B, B->pipe64[0], kstop, B->h_rb64, B->d_rb64, res64, s));
        for (int p = 0; p < n; ++p) steps[p] = cycles[p];
    } else if (B->prm.precision != HIPBMG_MIXED) {
        for (int c = 0; c < B->prm.max_cycles; ++c) {
            BPlan &plan = B->plan64[cur];
            STCHK(batch_cycle<double>(B, plan, B->d_active, B->d_bnorm, B->d_relres, B->d_tol, s));
            STCHK(batch_read(B, B->d_relres, B->d_active, s));
            for (int p = 0; p < n; ++p)
                if (act[p]) {
                    rel[p] = B->h_relres[p];
                    if (infos && cycles[p] < HIPBMG_MAX_HIST) infos[p].relres_hist[cycles[p]] = rel[p];
                    ++cycles[p];
                    if (!B->h_active[p]) {
                        act[p] = 0;
                        done_cur[p] = plan.end_cur;
                    }
                }
            cur = plan.end_cur;
            if (B->h_count[0] == 0) break;
        }
        for (int p = 0; p < n; ++p)
            if (act[p]) done_cur[p] = cur;
        for (int p = 0; p < n; ++p) steps[p] = cycles[p];
    } else {
        // FP64 iterative refinement around batched FP32 V-cycles
        int total = 0;
        while (true) {
            HIPCHK(launch_ir_residual_batched(B->d_fine64, B->d_fine32, B->d_active, B->d_rpart, B->d_roff,
                                              B->d_rowoff, B->rows, B->fine_npt, n, s, B->zc[0]));
            HIPCHK(launch_finalize_batched(B->d_rpart, B->d_roff, B->d_rcnt, nullptr, B->d_rnorm, B->d_active,
                                           -1.0, nullptr, n, s));
            HIPCHK(launch_finalize_batched(B->d_rpart, B->d_roff, B->d_rcnt, B->d_bnorm, B->d_relres, B->d_active,
                                           tol, nullptr, n, s));
            HIPCHK(launch_count_active(B->d_active, n, B->d_count, s));
            STCHK(batch_read(B, B->d_relres, B->d_active, s));
            for (int p = 0; p < n; ++p)
                if (act[p]) {
                    rel[p] = B->h_relres[p];
                    if (infos && steps[p] < HIPBMG_MAX_HIST) infos[p].relres_hist[steps[p]] = rel[p];
                    if (!B->h_active[p]) act[p] = 0;
                    else ++steps[p];
                }
            if (B->h_count[0] == 0 || total >= B->prm.max_cycles) break;
            // inner FP32 solves of A e = r for the active problems, each to
            // inner_tol or to what its outer tolerance still needs (half of
            // tol / relres), whichever is looser
            const bool adapt = B->hs[0]->inner_adapt != 0;
            for (int p = 0; p < n; ++p)
                B->h_itol[p] = adapt && act[p] && rel[p] > 0.0 ? std::max(B->prm.inner_tol, 0.5 * tol / rel[p])
                                                               : B->prm.inner_tol;
            HIPCHK(hipMemcpyAsync(B->d_itol, B->h_itol, n * sizeof(double), hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(B->d_active2, B->d_active, n * sizeof(int), hipMemcpyDeviceToDevice, s));
            if (B->pipe) {
                // pipelined finest level: each problem's inner solve stops at
                // its own cycle, whose iterate is rebuilt after the cycles
                std::vector<int> in2(act), kin(n, 0);
                int i = 1;
                for (int k = 0; k < B->prm.inner_max_cycles && total < B->prm.max_cycles; ++k) {
                    BPlan &plan = k == 0 ? B->pipe32[3] : B->pipe32[i];
                    STCHK(batch_cycle<float>(B, plan, B->d_active2, B->d_rnorm, B->d_irel, B->d_itol, s, 1));
                    i = plan.end_cur;
                    ++total;
                    HIPCHK(hipMemcpyAsync(B->h_count, B->d_count, sizeof(int), hipMemcpyDeviceToHost, s));
                    HIPCHK(hipMemcpyAsync(B->h_act2, B->d_active2, n * sizeof(int), hipMemcpyDeviceToHost, s));
                    HIPCHK(hipStreamSynchronize(s));
                    for (int p = 0; p < n; ++p) {
                        if (act[p]) ++cycles[p];
                        if (in2[p]) {
                            ++kin[p];
                            if (!B->h_act2[p]) in2[p] = 0;
                        }
                    }
                    if (B->h_count[0] == 0) break;
                }
                std::vector<float *> e32(n, nullptr);
                STCHK(batch_rebuild<float>(B, B->pipe32[0], kin, B->h_rb32, B->d_rb32, e32, s));
                for (int p = 0; p < n; ++p) B->h_eptr[p] = e32[p];
                HIPCHK(hipMemcpyAsync(B->d_eptr, B->h_eptr, n * sizeof(float *), hipMemcpyHostToDevice, s));
                HIPCHK(launch_ir_update_batched(B->d_fine64, B->d_fine32, B->d_eptr, B->d_active, B->d_rowoff,
                                                B->rows, n, s));
                continue;
            }
            int icur = 0;
            for (int k = 0; k < B->prm.inner_max_cycles && total < B->prm.max_cycles; ++k) {
                BPlan &plan = k == 0 ? B->plan32[1][0] : B->plan32[0][icur];
                STCHK(batch_cycle<float>(B, plan, B->d_active2, B->d_rnorm, B->d_irel, B->d_itol, s, 1));
                icur = plan.end_cur;
                ++total;
                HIPCHK(hipMemcpyAsync(B->h_count, B->d_count, sizeof(int), hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                for (int p = 0; p < n; ++p)
                    if (act[p]) ++cycles[p];
                if (B->h_count[0] == 0) break;
            }
            if (icur != 0) return fail(HIPBMG_EINVAL, "batched refinement expects the correction in buffer 0");
            HIPCHK(launch_ir_update_batched(B->d_fine64, B->d_fine32, nullptr, B->d_active, B->d_rowoff,
                                            B->rows, n, s));
        }
        for (int p = 0; p < n; ++p) done_cur[p] = 0;
    }
    // every problem's result (zero where b is) to its u in one launch
    for (int p = 0; p < n; ++p) {
        hipbmg_hier *h = B->hs[p];
        const LevelDev<double> &F = h->lv[h->L - 1];
        B->h_user[2 * n + p] = bnorm[p] == 0.0 ? nullptr : res64[p] ? res64[p] : F.x[done_cur[p]];
    }
    HIPCHK(hipMemcpyAsync(B->d_user + 2 * n, B->h_user + 2 * n, n * sizeof(double *), hipMemcpyHostToDevice, s));
    HIPCHK(launch_stage_batched(B->d_user, B->d_bptr, B->d_xptr, B->d_dims, B->d_rowoff, n, B->rows, 1, s));
    for (int p = 0; p < n; ++p) {
        const bool ok = bnorm[p] == 0.0 || rel[p] <= tol;
        if (!std::isfinite(rel[p]) || !std::isfinite(bnorm[p])) result = HIPBMG_ENAN;
        else if (!ok && result == HIPBMG_OK) result = HIPBMG_ENOCONV;
        if (infos) {
            infos[p].cycles = cycles[p];
            infos[p].outer_steps = steps[p];
            infos[p].relres = rel[p];
        }
    }
    HIPCHK(hipEventRecord(B->ev_out, s));
    HIPCHK(hipStreamWaitEvent(s_user, B->ev_out, 0));
    HIPCHK(hipStreamSynchronize(s));
    const double ms = now_ms() - t0;
    if (infos)
        for (int p = 0; p < n; ++p) infos[p].solve_ms = ms;
    if (result == HIPBMG_ENAN) return fail(HIPBMG_ENAN, "a residual norm is not finite");
    if (result == HIPBMG_ENOCONV) return fail(HIPBMG_ENOCONV, "some problems did not reach tol");
    (void)nbad;
    return HIPBMG_OK;
}
