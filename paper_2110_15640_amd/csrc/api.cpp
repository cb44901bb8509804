// Host runtime of libmcrt.so: context, resident grids and opacity tables,
// input validation, solve planning and the paper's post-processing of the
// tallies into observables (Sect. 5).  Implements include/mcrt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <thread>
#include <type_traits>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mcrt.h"
#include "mcrt_internal.hpp"

namespace mcrt {
// Checks of borrowed per-cell arrays on the device (kernels.hip): bit 0 T,
// 1 P, 2 rho, 3 winds, 4 cloud opacities, 5 cloud g set in *bad where a cell
// fails.
void launch_check_cells(const float* T, const float* P, const double* rho, const float* u, const float* v,
                        const float* w, const float* cs, const float* ca, const float* cg, size_t n, int* bad,
                        hipStream_t stream);
}  // namespace mcrt

using namespace mcrt;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

constexpr double kPi = 3.14159265358979323846;

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct GridRes {
    GridDev dev{};
    int ncell = 0;
    std::vector<DevBuf> bufs;
    size_t bytes = 0;
    double r0 = 0.0, r_toa = 0.0;
    int refs = 0;
};

struct OpacRes {
    int kind = 0, nspec = 0, ng = 0, nT = 0, nP = 0;
    double lam_min = 0.0, dlnlam = 0.0;
    std::vector<double> lam_um, g_weights, k_ray;
    double* lnk = nullptr;     // CK: [nspec][ng][nT][nP]; HIRES: [nT][nP][nlam]
    float* lnk_f32 = nullptr;  // HIRES: the same table rounded to FP32 (read by the mixed form)
    double* T_grid = nullptr;  // [nT]
    double* lnP_grid = nullptr;
    double* k_ray_dev = nullptr;
    double* gw_dev = nullptr;  // g-ordinate weights
    std::vector<DevBuf> bufs;
    size_t bytes = 0;
    int refs = 0;
};

// An execution slot: a stream, its timing events and its scratch arena.
// Blocking solves use the context's main slot; each serving worker owns one.
struct Slot {
    hipStream_t stream = nullptr;
    hipStream_t stream2 = nullptr;  // second stream of a blocking transmission solve
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;  // ordering between the two streams
    std::vector<hipEvent_t> prof_ev;  // pairs around timed launches
    std::map<std::string, DevBuf> scratch;  // grow-only, by role
    bool stream_ordered = false;  // serving slots allocate with hipMallocAsync
    // Fixed arena (the allocation-free solve): scratch is carved from it in
    // order, from offset 0 at every call, instead of allocated.
    char* arena = nullptr;
    size_t arena_cap = 0, arena_off = 0;
};

struct Request;

// A recorded solve (params.graph): the instantiated graph and the pinned host
// copies of the per-batch solve tables that its copy nodes read.
struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* pinned = nullptr;
    int32_t gid = 0, oid = 0;
    std::vector<int32_t> gids, oids;  // every grid and table of a recorded batch
    uint64_t used = 0;
    ~GraphEntry()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (pinned) (void)hipHostFree(pinned);
    }
};
constexpr size_t kMaxGraphs = 16;

}  // namespace

namespace {

// Scratch of the allocation-free solve (mcrt_solve_noalloc): one fixed array
// per GPU the library runs on, held until the process ends and shared by
// every context on that GPU.  Host code never passes the array's name to the
// device: its address on each GPU comes from hipGetSymbolAddress (taken once
// per device when a context is created) and only that address is used.
constexpr size_t kNoallocBytes = MCRT_NOALLOC_SCRATCH_BYTES;
constexpr int kNoallocDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];
std::mutex g_noalloc_mu;                     // guards g_noalloc_ptr
void* g_noalloc_ptr[kNoallocDevices] = {};   // device address of `scratch` per GPU
std::mutex g_noalloc_run[kNoallocDevices];   // one allocation-free solve per GPU at a time

}  // namespace

struct mcrt_ctx {
    int device = 0;
    int n_cu = 256;
    uint64_t budget = 0;
    uint64_t in_use = 0;
    mutable std::mutex mem_mu;  // in_use, reserved, served
    std::mutex mu;      // grids, opacs, refs
    std::mutex main_mu; // blocking solves on the main slot
    Slot main;
    Slot na;            // allocation-free solves: the device's fixed scratch array
    std::map<int32_t, std::unique_ptr<GridRes>> grids;
    std::map<int32_t, std::unique_ptr<OpacRes>> opacs;
    int32_t next_grid = 1, next_opac = 1;
    bool poisoned = false;
    // recorded blocking solves (params.graph), keyed by their arguments
    std::mutex graph_mu;
    std::map<std::string, std::unique_ptr<GraphEntry>> graphs;
    uint64_t graph_clock = 0;
    // serving
    std::mutex q_mu;
    std::condition_variable q_cv;
    std::deque<Request*> queue;
    std::map<uint64_t, std::unique_ptr<Request>> requests;
    std::vector<std::thread> workers;
    std::vector<std::unique_ptr<Slot>> wslots;
    uint64_t reserved = 0;  // bytes admitted to running requests (their estimates)
    uint64_t served = 0;    // bytes of in_use the running requests allocated
    uint64_t next_ticket = 1;
    int n_workers = 3;
    bool stopping = false;
    std::atomic<int> n_running{0};   // served requests on the device now
    hipMemPool_t pool = nullptr;     // the workers' stream-ordered scratch (private to the context)
};

namespace {

int hip_check(mcrt_ctx* ctx, hipError_t e, const char* what)
{
    if (e == hipSuccess) return MCRT_OK;
    if (ctx) ctx->poisoned = true;
    return fail(MCRT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Device memory held or promised, in bytes (caller holds mem_mu): what is
// allocated, plus what admitted requests may still allocate (an admitted
// request's allocations are charged to its reservation, not twice).
uint64_t held_locked(const mcrt_ctx* ctx)
{
    return ctx->in_use + (ctx->reserved > ctx->served ? ctx->reserved - ctx->served : 0);
}

#define HIPTRY(expr)                                          \
    do {                                                      \
        int _rc = hip_check(ctx, (expr), #expr);              \
        if (_rc != MCRT_OK) return _rc;                       \
    } while (0)

// Device allocation charged to the context's budget.  A stream-ordered
// allocation (serving slots) was admitted against the budget beforehand.
int dev_alloc(mcrt_ctx* ctx, size_t bytes, DevBuf& out, hipStream_t ordered = nullptr)
{
    if (bytes == 0) bytes = 8;
    bool trim = false;
    {
        std::lock_guard<std::mutex> lk(ctx->mem_mu);
        if (!ordered && held_locked(ctx) + bytes > ctx->budget)
            return fail(MCRT_EBUDGET, "allocation of %zu bytes exceeds the HBM budget (%llu in use, %llu reserved, "
                        "budget %llu)", bytes, (unsigned long long)ctx->in_use, (unsigned long long)ctx->reserved,
                        (unsigned long long)ctx->budget);
        ctx->in_use += bytes;
        if (ordered) ctx->served += bytes;
        // memory the workers' pool keeps after frees is not in in_use: hand it
        // back to the device before a blocking allocation would go past the budget
        if (!ordered && ctx->pool) {
            uint64_t reserved = 0, used = 0;
            if (hipMemPoolGetAttribute(ctx->pool, hipMemPoolAttrReservedMemCurrent, &reserved) == hipSuccess &&
                hipMemPoolGetAttribute(ctx->pool, hipMemPoolAttrUsedMemCurrent, &used) == hipSuccess)
                trim = ctx->in_use + (reserved > used ? reserved - used : 0) > ctx->budget;
        }
    }
    if (trim) (void)hipMemPoolTrimTo(ctx->pool, 0);
    void* p = nullptr;
    hipError_t e = ordered ? (ctx->pool ? hipMallocFromPoolAsync(&p, bytes, ctx->pool, ordered)
                                        : hipMallocAsync(&p, bytes, ordered))
                           : hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        std::lock_guard<std::mutex> lk(ctx->mem_mu);
        ctx->in_use -= bytes;
        if (ordered) ctx->served -= bytes;
        return fail(MCRT_ENOMEM, "device allocation of %zu bytes: %s", bytes, hipGetErrorString(e));
    }
    out.p = p;
    out.bytes = bytes;
    return MCRT_OK;
}

void dev_free(mcrt_ctx* ctx, DevBuf& b, hipStream_t ordered = nullptr)
{
    if (b.p) {
        if (ordered) (void)hipFreeAsync(b.p, ordered);
        else (void)hipFree(b.p);
        std::lock_guard<std::mutex> lk(ctx->mem_mu);
        ctx->in_use -= b.bytes;
        if (ordered) ctx->served -= b.bytes;
    }
    b.p = nullptr;
    b.bytes = 0;
}

// Scratch buffer of at least `bytes` under `name` in slot `sl` (grow-only).
int slot_scratch(mcrt_ctx* ctx, Slot& sl, hipStream_t st, const char* name, size_t bytes, void** out)
{
    if (sl.arena) {
        const size_t at = (sl.arena_off + 255) & ~(size_t)255;
        if (at > sl.arena_cap || bytes > sl.arena_cap - at)
            return fail(MCRT_EINVAL, "scratch '%s' (%zu bytes) does not fit in the fixed scratch of %zu bytes", name,
                        bytes, sl.arena_cap);
        *out = sl.arena + at;
        sl.arena_off = at + bytes;
        return MCRT_OK;
    }
    DevBuf& b = sl.scratch[name];
    if (b.bytes < bytes) {
        if (b.p) {
            if (!sl.stream_ordered) {  // the old buffer may still be read by queued work
                HIPTRY(hipStreamSynchronize(st));
                HIPTRY(hipStreamSynchronize(sl.stream));
            }
            dev_free(ctx, b, sl.stream_ordered ? st : nullptr);
        }
        int rc = dev_alloc(ctx, bytes, b, sl.stream_ordered ? st : nullptr);
        if (rc) return rc;
    }
    *out = b.p;
    return MCRT_OK;
}

void release_scratch(mcrt_ctx* ctx, Slot& sl)
{
    for (auto& kv : sl.scratch) dev_free(ctx, kv.second, sl.stream_ordered ? sl.stream : nullptr);
    sl.scratch.clear();
}

// A stream on a hardware queue of its own: made with a CU mask that covers
// every CU, which the runtime serves with a new queue instead of a share of
// its few default ones.  Kernels of two streams that share a queue run one
// after the other, so streams meant to overlap (the serving workers, the
// two halves of a transmission solve) are made this way.  Where the runtime
// refuses CU-masked streams, an ordinary stream does the same work (the
// results do not depend on it; only the overlap may be lost).
int own_queue_stream(hipStream_t* st, int n_cu)
{
    std::vector<uint32_t> mask((size_t)(std::max(n_cu, 1) + 31) / 32, 0xffffffffu);
    if (n_cu % 32) mask.back() = (1u << (n_cu % 32)) - 1u;
    if (hipExtStreamCreateWithCUMask(st, (uint32_t)mask.size(), mask.data()) == hipSuccess) return MCRT_OK;
    (void)hipGetLastError();
    hipError_t e = hipStreamCreateWithFlags(st, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(MCRT_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    return MCRT_OK;
}

int slot_init(Slot& sl, bool own_queue = false, int n_cu = 0)
{
    hipError_t e;
    if (own_queue) {
        if (int rc = own_queue_stream(&sl.stream, n_cu)) return rc;
    } else if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess) {
        return fail(MCRT_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    if ((e = hipEventCreate(&sl.ev0)) != hipSuccess || (e = hipEventCreate(&sl.ev1)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&sl.fork, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&sl.join, hipEventDisableTiming)) != hipSuccess)
        return fail(MCRT_EDEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    return MCRT_OK;
}

void slot_destroy(mcrt_ctx* ctx, Slot& sl)
{
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    release_scratch(ctx, sl);
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    for (auto e : sl.prof_ev) (void)hipEventDestroy(e);
    sl.prof_ev.clear();
    if (sl.ev0) (void)hipEventDestroy(sl.ev0);
    if (sl.ev1) (void)hipEventDestroy(sl.ev1);
    if (sl.fork) (void)hipEventDestroy(sl.fork);
    if (sl.join) (void)hipEventDestroy(sl.join);
    if (sl.stream2) {
        (void)hipStreamSynchronize(sl.stream2);
        (void)hipStreamDestroy(sl.stream2);
    }
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    sl.stream = sl.stream2 = nullptr;
    sl.ev0 = sl.ev1 = sl.fork = sl.join = nullptr;
}

template <typename T>
int upload(mcrt_ctx* ctx, std::vector<DevBuf>& bufs, size_t& total, const T* host, size_t n, T** dev,
           hipStream_t st)
{
    DevBuf b;
    int rc = dev_alloc(ctx, n * sizeof(T), b);
    if (rc) return rc;
    bufs.push_back(b);
    total += b.bytes;
    HIPTRY(hipMemcpyAsync(b.p, host, n * sizeof(T), hipMemcpyHostToDevice, st));
    *dev = (T*)b.p;
    return MCRT_OK;
}

bool finite_all(const double* a, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

bool finite_all(const float* a, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

bool increasing(const double* a, size_t n)
{
    for (size_t i = 1; i < n; ++i)
        if (!(a[i] > a[i - 1])) return false;
    return true;
}

int validate_grid(const mcrt_grid_desc* d)
{
    if (!d) return fail(MCRT_EINVAL, "grid descriptor is NULL");
    if (d->geometry != MCRT_SPHERICAL && d->geometry != MCRT_PLANE_PARALLEL)
        return fail(MCRT_EINVAL, "unknown geometry %d", d->geometry);
    if (d->nlay < 1 || d->nlon < 1 || d->nlat < 1) return fail(MCRT_EINVAL, "grid dimensions must be >= 1");
    if ((long long)d->nlon * d->nlat * d->nlay > (1LL << 31) - 1) return fail(MCRT_EINVAL, "grid too large");
    if (d->nlon > 2048 || d->nlat > 1024 || d->nlay > 2048)
        return fail(MCRT_EINVAL, "grid dimensions are limited to 2048 x 1024 x 2048 (lon x lat x layers)");
    if (!d->r_edges || !d->T || !d->P || !d->rho) return fail(MCRT_EINVAL, "r_edges, T, P and rho are required");
    if (!finite_all(d->r_edges, d->nlay + 1) || !increasing(d->r_edges, d->nlay + 1))
        return fail(MCRT_EINVAL, "r_edges must be finite and strictly increasing");
    if (d->geometry == MCRT_PLANE_PARALLEL) {
        if (d->nlon != 1 || d->nlat != 1) return fail(MCRT_EINVAL, "a slab has nlon = nlat = 1");
    } else {
        if (!(d->r_edges[0] > 0.0)) return fail(MCRT_EINVAL, "r_edges[0] (R0) must be > 0");
        if (!d->lat_edges || !d->lon_edges) return fail(MCRT_EINVAL, "lat_edges and lon_edges are required");
        if (!finite_all(d->lat_edges, d->nlat + 1) || !increasing(d->lat_edges, d->nlat + 1) ||
            std::fabs(d->lat_edges[0] + kPi / 2) > 1e-12 || std::fabs(d->lat_edges[d->nlat] - kPi / 2) > 1e-12)
            return fail(MCRT_EINVAL, "lat_edges must increase from -pi/2 to pi/2");
        if (!finite_all(d->lon_edges, d->nlon + 1) || !increasing(d->lon_edges, d->nlon + 1) ||
            std::fabs(d->lon_edges[0] + kPi) > 1e-12 || std::fabs(d->lon_edges[d->nlon] - kPi) > 1e-12)
            return fail(MCRT_EINVAL, "lon_edges must increase from -pi to pi");
    }
    if (d->flags & ~MCRT_BORROW_DEVICE) return fail(MCRT_EINVAL, "unknown grid flags");
    if (d->cld_ksca || d->cld_kabs || d->cld_g)
        if (!(d->cld_ksca && d->cld_kabs && d->cld_g))
            return fail(MCRT_EINVAL, "cloud needs cld_ksca, cld_kabs and cld_g together");
    if (!std::isfinite(d->omega_rot)) return fail(MCRT_EINVAL, "omega_rot must be finite");
    if (d->flags & MCRT_BORROW_DEVICE) return MCRT_OK;  // per-cell values are checked on the device
    size_t n = (size_t)d->nlon * d->nlat * d->nlay;
    for (size_t c = 0; c < n; ++c) {
        if (!(std::isfinite(d->T[c]) && d->T[c] > 0.0f)) return fail(MCRT_EINVAL, "T[%zu] must be finite and > 0", c);
        if (!(std::isfinite(d->P[c]) && d->P[c] > 0.0f)) return fail(MCRT_EINVAL, "P[%zu] must be finite and > 0", c);
        if (!(std::isfinite(d->rho[c]) && d->rho[c] >= 0.0)) return fail(MCRT_EINVAL, "rho[%zu] must be finite and >= 0", c);
    }
    const float* wind[3] = {d->u, d->v, d->w};
    for (int q = 0; q < 3; ++q)
        if (wind[q] && !finite_all(wind[q], n)) return fail(MCRT_EINVAL, "winds must be finite");
    if (d->cld_ksca) {
        for (size_t c = 0; c < n; ++c) {
            if (!(std::isfinite(d->cld_ksca[c]) && d->cld_ksca[c] >= 0.0f && std::isfinite(d->cld_kabs[c]) &&
                  d->cld_kabs[c] >= 0.0f))
                return fail(MCRT_EINVAL, "cloud opacities must be finite and >= 0");
            if (!(std::fabs(d->cld_g[c]) < 1.0f)) return fail(MCRT_EINVAL, "cloud g must satisfy |g| < 1");
        }
    }
    return MCRT_OK;
}

// Borrowed per-cell arrays: device memory of the context's device, whose
// values pass the same checks as a host grid's (run on the device).
int check_borrowed(mcrt_ctx* ctx, const mcrt_grid_desc* d, size_t n, hipStream_t st)
{
    const void* ptrs[9] = {d->T, d->P, d->rho, d->u, d->v, d->w, d->cld_ksca, d->cld_kabs, d->cld_g};
    for (const void* p : ptrs) {
        if (!p) continue;
        hipPointerAttribute_t at{};
        if (hipPointerGetAttributes(&at, p) != hipSuccess || at.type != hipMemoryTypeDevice ||
            at.device != ctx->device) {
            (void)hipGetLastError();
            return fail(MCRT_EINVAL, "borrowed grid arrays must be device memory of device %d", ctx->device);
        }
    }
    // on the caller's stream: the check reads the arrays after the caller's
    // earlier work on that stream (e.g. the kernels that wrote them)
    int* bad = nullptr;
    HIPTRY(hipMalloc(&bad, sizeof(int)));
    int h = 0;
    hipError_t e = hipMemcpyAsync(bad, &h, sizeof(int), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        launch_check_cells(d->T, d->P, d->rho, d->u, d->v, d->w, d->cld_ksca, d->cld_kabs, d->cld_g, n, bad, st);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(bad);
    HIPTRY(e);
    if (h & 1) return fail(MCRT_EINVAL, "T must be finite and > 0");
    if (h & 2) return fail(MCRT_EINVAL, "P must be finite and > 0");
    if (h & 4) return fail(MCRT_EINVAL, "rho must be finite and >= 0");
    if (h & 8) return fail(MCRT_EINVAL, "winds must be finite");
    if (h & 16) return fail(MCRT_EINVAL, "cloud opacities must be finite and >= 0");
    if (h & 32) return fail(MCRT_EINVAL, "cloud g must satisfy |g| < 1");
    return MCRT_OK;
}

int validate_opacity(const mcrt_opacity_desc* d)
{
    if (!d) return fail(MCRT_EINVAL, "opacity descriptor is NULL");
    if (d->kind != MCRT_OPAC_CK && d->kind != MCRT_OPAC_HIRES) return fail(MCRT_EINVAL, "unknown opacity kind");
    if (d->nspec < 1 || d->ng < 1 || d->nT < 1 || d->nP < 1) return fail(MCRT_EINVAL, "table dimensions must be >= 1");
    if (d->kind == MCRT_OPAC_HIRES && d->ng != 1) return fail(MCRT_EINVAL, "a high-resolution table has ng = 1");
    if (!d->T_grid || !d->P_grid || !d->kappa || !d->k_ray) return fail(MCRT_EINVAL, "missing table arrays");
    if (!finite_all(d->T_grid, d->nT) || !increasing(d->T_grid, d->nT) || !(d->T_grid[0] > 0.0))
        return fail(MCRT_EINVAL, "T_grid must be positive and strictly increasing");
    if (!finite_all(d->P_grid, d->nP) || !increasing(d->P_grid, d->nP) || !(d->P_grid[0] > 0.0))
        return fail(MCRT_EINVAL, "P_grid must be positive and strictly increasing");
    size_t n = (size_t)d->nspec * d->ng * d->nT * d->nP;
    for (size_t i = 0; i < n; ++i)
        if (!(std::isfinite(d->kappa[i]) && d->kappa[i] >= 0.0f))
            return fail(MCRT_EINVAL, "kappa[%zu] must be finite and >= 0", i);
    for (int s = 0; s < d->nspec; ++s)
        if (!(std::isfinite(d->k_ray[s]) && d->k_ray[s] >= 0.0)) return fail(MCRT_EINVAL, "k_ray must be >= 0");
    if (d->kind == MCRT_OPAC_CK) {
        if (!d->lam_um || !d->g_weights) return fail(MCRT_EINVAL, "a ck table needs lam_um and g_weights");
        double ws = 0.0;
        for (int g = 0; g < d->ng; ++g) {
            if (!(d->g_weights[g] >= 0.0)) return fail(MCRT_EINVAL, "g_weights must be >= 0");
            ws += d->g_weights[g];
        }
        if (std::fabs(ws - 1.0) > 1e-9) return fail(MCRT_EINVAL, "g_weights must sum to 1 (got %.12g)", ws);
        // a k-distribution is sorted: kappa non-decreasing in g at every (band, T, P)
        const size_t tp = (size_t)d->nT * d->nP;
        for (int s = 0; s < d->nspec; ++s)
            for (int g = 0; g + 1 < d->ng; ++g) {
                const float* a = d->kappa + ((size_t)s * d->ng + g) * tp;
                for (size_t q = 0; q < tp; ++q)
                    if (!(a[q] <= a[q + tp]))
                        return fail(MCRT_EINVAL, "ck kappa must be non-decreasing in g (band %d, g %d)", s, g);
            }
        for (int s = 0; s < d->nspec; ++s)
            if (!(d->lam_um[s] > 0.0 && std::isfinite(d->lam_um[s]))) return fail(MCRT_EINVAL, "lam_um must be > 0");
    } else {
        if (!(d->lam_min_um > 0.0) || !(d->dlnlam > 0.0) || !std::isfinite(d->lam_min_um) || !std::isfinite(d->dlnlam))
            return fail(MCRT_EINVAL, "lam_min_um and dlnlam must be > 0");
    }
    return MCRT_OK;
}

GridRes* find_grid(mcrt_ctx* ctx, int32_t id)
{
    auto it = ctx->grids.find(id);
    return it == ctx->grids.end() ? nullptr : it->second.get();
}

OpacRes* find_opac(mcrt_ctx* ctx, int32_t id)
{
    auto it = ctx->opacs.find(id);
    return it == ctx->opacs.end() ? nullptr : it->second.get();
}

struct SolvePlan {
    std::vector<int> specs;
    int ng = 1;
    int n_out = 0;
    int n_obs = 0;
    std::vector<double> obs;  // 3 * n_obs
    hipStream_t stream = nullptr;
};

int plan_common(hipStream_t def_stream, GridRes* g, OpacRes* op, const mcrt_solve_params* p, int mode, SolvePlan& pl)
{
    if (!p) return fail(MCRT_EINVAL, "params is NULL");
    if (p->precision != MCRT_FP64 && p->precision != MCRT_MIXED) return fail(MCRT_EINVAL, "unknown precision");
    if (p->n_spec < 0) return fail(MCRT_EINVAL, "n_spec < 0");
    int nspec_tab = op->nspec;
    if (p->spec_idx) {
        for (int s = 0; s < p->n_spec; ++s) {
            if (p->spec_idx[s] < 0 || p->spec_idx[s] >= nspec_tab)
                return fail(MCRT_EINVAL, "spec_idx[%d] = %d out of range", s, p->spec_idx[s]);
            pl.specs.push_back(p->spec_idx[s]);
        }
    } else {
        for (int s = 0; s < nspec_tab; ++s) pl.specs.push_back(s);
    }
    if (pl.specs.empty()) return fail(MCRT_EINVAL, "no spectral points selected");
    pl.ng = op->kind == MCRT_OPAC_CK ? op->ng : 1;
    pl.stream = p->stream ? (hipStream_t)p->stream : def_stream;
    if (mode == MCRT_MODE_TRANSMISSION) {
        if (g->dev.geom != 0) return fail(MCRT_EINVAL, "transmission needs a spherical grid");
        if (!(p->r_star > 0.0) || !std::isfinite(p->r_star)) return fail(MCRT_EINVAL, "r_star must be > 0");
        if (p->ld_law < 0 || p->ld_law > 6) return fail(MCRT_EINVAL, "ld_law must be 0 to 6");
        if (!std::isfinite(p->ld_c1) || !std::isfinite(p->ld_c2) || !std::isfinite(p->transit_y) ||
            !std::isfinite(p->transit_z))
            return fail(MCRT_EINVAL, "limb-darkening coefficients and the transit position must be finite");
        if (p->ms_transmission != 0 && p->ms_transmission != 1) return fail(MCRT_EINVAL, "ms_transmission must be 0 or 1");
        pl.n_out = 1;
        if (!p->ms_transmission) {
            if (p->n_b < 1 || p->n_alpha < 1 || (long long)p->n_b * p->n_alpha > (1LL << 30))
                return fail(MCRT_EINVAL, "n_b and n_alpha must be >= 1 with n_b * n_alpha <= 2^30");
            return MCRT_OK;
        }
        if (!(p->a_orbit > p->r_star) || !std::isfinite(p->a_orbit))
            return fail(MCRT_EINVAL, "transmission with multiple scattering needs a_orbit > r_star");
    }
    if (p->n_packets < 1 || p->n_packets > (1ULL << 40)) return fail(MCRT_EINVAL, "n_packets must be in [1, 2^40]");
    if (p->n_obs < 0 || p->n_obs > kMaxObs) return fail(MCRT_EINVAL, "n_obs must be in [0, %d]", kMaxObs);
    if (!(p->rr_survive > 0.0 && p->rr_survive <= 1.0)) return fail(MCRT_EINVAL, "rr_survive must be in (0, 1]");
    if (!(p->rr_threshold >= 0.0) || !std::isfinite(p->rr_threshold)) return fail(MCRT_EINVAL, "rr_threshold >= 0");
    if (!(p->emis_bias >= 0.0 && p->emis_bias <= 1.0)) return fail(MCRT_EINVAL, "emis_bias must be in [0, 1]");
    if (!(p->tau_peel_max > 0.0)) return fail(MCRT_EINVAL, "tau_peel_max must be > 0");
    if (!(p->tau_vert_max >= 0.0)) return fail(MCRT_EINVAL, "tau_vert_max must be >= 0");
    if (p->max_events < 1) return fail(MCRT_EINVAL, "max_events must be >= 1");
    if (p->absorption != MCRT_SURVIVAL && p->absorption != MCRT_CONTINUOUS) return fail(MCRT_EINVAL, "bad absorption");
    if (p->cloud_phase < 0 || p->cloud_phase > 2)
        return fail(MCRT_EINVAL, "cloud_phase must be 0 (HG), 1 (TTHG) or 2 (Draine)");
    if (!(p->draine_alpha >= 0.0 && p->draine_alpha <= 1.0)) return fail(MCRT_EINVAL, "draine_alpha must be in [0, 1]");
    if (p->forced < 0 || p->forced > 3 || (p->forced_first != 0 && p->forced_first != 1))
        return fail(MCRT_EINVAL, "forced must be 0 to 3 and forced_first 0 or 1");
    if (p->forced && (p->absorption != MCRT_SURVIVAL || p->surface_albedo > 0.0))
        return fail(MCRT_EINVAL, "forced interactions need survival biasing and an absorbing lower boundary");
    if (!(p->surface_albedo >= 0.0 && p->surface_albedo <= 1.0))
        return fail(MCRT_EINVAL, "surface_albedo must be in [0, 1]");
    if (!(p->mu0 <= 1.0)) return fail(MCRT_EINVAL, "mu0 must be <= 1");
    if (mode == MCRT_MODE_EMISSION && g->dev.geom != 0) return fail(MCRT_EINVAL, "emission needs a spherical grid");
    if (mode == MCRT_MODE_TRANSMISSION) {  // one observer, along -x
        pl.n_obs = 1;
        pl.obs = {-1.0, 0.0, 0.0};
        return MCRT_OK;
    }
    if (p->n_obs == 0) {
        if (!(mode == MCRT_MODE_ALBEDO && g->dev.geom == 1))
            return fail(MCRT_EINVAL, "n_obs = 0 is only allowed for slab albedo (backscatter)");
        pl.n_obs = 0;
        pl.n_out = 1;
        return MCRT_OK;
    }
    if (!p->obs_dir && !p->obs_phase) return fail(MCRT_EINVAL, "observers need obs_phase or obs_dir");
    pl.n_obs = p->n_obs;
    pl.n_out = p->n_obs;
    for (int o = 0; o < p->n_obs; ++o) {
        double v[3];
        if (p->obs_dir) {
            v[0] = p->obs_dir[3 * o];
            v[1] = p->obs_dir[3 * o + 1];
            v[2] = p->obs_dir[3 * o + 2];
            double n = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            if (!(std::fabs(n - 1.0) < 1e-9)) return fail(MCRT_EINVAL, "obs_dir[%d] is not a unit vector", o);
        } else {
            double ph = p->obs_phase[o];
            if (!std::isfinite(ph)) return fail(MCRT_EINVAL, "obs_phase must be finite");
            double a = mode == MCRT_MODE_ALBEDO ? ph : kPi * (1.0 - 2.0 * ph);
            v[0] = std::cos(a);
            v[1] = std::sin(a);
            v[2] = 0.0;
        }
        pl.obs.insert(pl.obs.end(), v, v + 3);
    }
    return MCRT_OK;
}

void fill_results(const SolvePlan& pl, const std::vector<double>& perg_val, const std::vector<double>& perg_se,
                  const std::vector<double>& g_w, const std::vector<double>& sums, int row_w,
                  const std::vector<double>& counters, const std::vector<double>& ltot, mcrt_result* r)
{
    int ns = (int)pl.specs.size(), ng = pl.ng, no = pl.n_out;
    for (int s = 0; s < ns; ++s)
        for (int o = 0; o < no; ++o) {
            double v = 0.0, e2 = 0.0;
            for (int g = 0; g < ng; ++g) {
                double w = g_w[g];
                size_t i = ((size_t)s * ng + g) * no + o;
                v += w * perg_val[i];
                e2 += w * w * perg_se[i] * perg_se[i];
            }
            if (r->value) r->value[(size_t)s * no + o] = v;
            if (r->stderr_) r->stderr_[(size_t)s * no + o] = std::sqrt(e2);
        }
    if (r->per_g) std::copy(perg_val.begin(), perg_val.end(), r->per_g);
    if (r->sums) {
        for (size_t sg = 0; sg < (size_t)ns * ng; ++sg)
            for (int o = 0; o < no; ++o) {
                r->sums[(sg * no + o) * 2] = sums[sg * row_w + 2 * o];
                r->sums[(sg * no + o) * 2 + 1] = sums[sg * row_w + 2 * o + 1];
            }
    }
    if (r->counters) std::copy(counters.begin(), counters.end(), r->counters);
    if (r->l_tot) std::copy(ltot.begin(), ltot.end(), r->l_tot);
}

// Timed-launch bracket: events 2i and 2i+1 around the i-th launch.
int prof_events(mcrt_ctx* ctx, Slot& sl, size_t n_launch)
{
    while (sl.prof_ev.size() < 2 * n_launch) {
        hipEvent_t e;
        HIPTRY(hipEventCreate(&e));
        sl.prof_ev.push_back(e);
    }
    return MCRT_OK;
}

int prof_collect(mcrt_ctx* ctx, Slot& sl, size_t n_launch, mcrt_result* r)
{
    double tot = 0.0;
    for (size_t i = 0; i < n_launch; ++i) {
        float ms = 0.0f;
        HIPTRY(hipEventElapsedTime(&ms, sl.prof_ev[2 * i], sl.prof_ev[2 * i + 1]));
        tot += ms;
    }
    r->kernel_ms = tot;
    r->kernel_launches = (int64_t)n_launch;
    return MCRT_OK;
}

int finish_timing(mcrt_ctx* ctx, Slot& sl, hipStream_t st, mcrt_result* r)
{
    HIPTRY(hipEventRecord(sl.ev1, st));
    HIPTRY(hipEventSynchronize(sl.ev1));
    float ms = 0.0f;
    HIPTRY(hipEventElapsedTime(&ms, sl.ev0, sl.ev1));
    if (r) r->elapsed_ms = ms;
    return MCRT_OK;
}

// Looks up a grid and an opacity table and holds a reference on both for
// the duration of a solve (mcrt_*_free return EBUSY meanwhile).
struct Lease {
    mcrt_ctx* ctx = nullptr;
    GridRes* g = nullptr;
    OpacRes* op = nullptr;
    ~Lease()
    {
        if (!ctx) return;
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (g) g->refs--;
        if (op) op->refs--;
    }
};

// Forget recorded solves of a grid (gid != 0), a table (oid != 0), or all.
void drop_graphs(mcrt_ctx* ctx, int32_t gid, int32_t oid)
{
    std::lock_guard<std::mutex> gk(ctx->graph_mu);
    for (auto it = ctx->graphs.begin(); it != ctx->graphs.end();) {
        const GraphEntry& e = *it->second;
        const bool hit = (gid == 0 && oid == 0) || (gid != 0 && e.gid == gid) || (oid != 0 && e.oid == oid) ||
                         (gid != 0 && std::find(e.gids.begin(), e.gids.end(), gid) != e.gids.end()) ||
                         (oid != 0 && std::find(e.oids.begin(), e.oids.end(), oid) != e.oids.end());
        it = hit ? ctx->graphs.erase(it) : std::next(it);
    }
}

// Blocking solves keep their scratch in the main slot for the next one.
// When it stands in the way of an upload or a served request, and no blocking
// solve is running, it is released (with the recorded solves, which bake its
// addresses in).  Returns whether anything was released.  Never called with
// main_mu held.
bool reclaim_main(mcrt_ctx* ctx)
{
    std::unique_lock<std::mutex> lk(ctx->main_mu, std::try_to_lock);
    if (!lk.owns_lock() || ctx->main.scratch.empty()) return false;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->main.stream);
    drop_graphs(ctx, 0, 0);
    release_scratch(ctx, ctx->main);
    return true;
}

int lease(mcrt_ctx* ctx, int32_t gid, int32_t oid, Lease& L)
{
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->poisoned) return fail(MCRT_EDEVICE, "context is unusable after an earlier device error");
    auto gi = ctx->grids.find(gid);
    if (gi == ctx->grids.end()) return fail(MCRT_ENOTFOUND, "grid %d not found", gid);
    auto oi = ctx->opacs.find(oid);
    if (oi == ctx->opacs.end()) return fail(MCRT_ENOTFOUND, "opacity %d not found", oid);
    L.ctx = ctx;
    L.g = gi->second.get();
    L.op = oi->second.get();
    L.g->refs++;
    L.op->refs++;
    return MCRT_OK;
}

// Solves per persistent launch for a serving request: a fixed share of the
// budget, so that the admission estimate and the allocation agree, and at
// most kServeLaunchPackets packets (about 30 ms of the whole device), so that
// a long request reaches the device as a sequence of launches whose share of
// the device is chosen anew: a launch sized to a third of the device while
// three requests ran keeps only that third after the other two finish, until
// it ends.
constexpr uint64_t kServeLaunchPackets = 1ull << 23;
int serving_batch(mcrt_ctx* ctx, int max_batch, int nsolve, uint64_t per_solve, uint64_t packets_per_solve)
{
    uint64_t cap = std::min<uint64_t>(ctx->budget / 8, 24ULL << 30);
    int batch = max_batch > 0 ? max_batch : nsolve;
    int fit = (int)std::max<uint64_t>(1, cap / std::max<uint64_t>(per_solve, 1));
    int short_launch = (int)std::max<uint64_t>(1, kServeLaunchPackets / std::max<uint64_t>(packets_per_solve, 1));
    return std::max(1, std::min(std::min(std::min(batch, fit), short_launch), nsolve));
}

// Persistent blocks of a served launch: the device's blocks shared among the
// requests running now, so that the launches of concurrent requests are
// resident together instead of queueing behind one whole-device grid.
int serving_blocks(mcrt_ctx* ctx, int bpc)
{
    const int k = std::max(1, ctx->n_running.load());
    return std::max(ctx->n_cu, ctx->n_cu * bpc / k);
}

// Sky-plane axes of observer o for images: vertical e_v = z projected on the
// plane normal to o (x when o is along z), horizontal e_h = e_v x o.
void sky_axes(const double* o, double* out)
{
    double ref[3] = {0.0, 0.0, 1.0};
    double v[3];
    for (int pass = 0; pass < 2; ++pass) {
        const double d = ref[0] * o[0] + ref[1] * o[1] + ref[2] * o[2];
        for (int q = 0; q < 3; ++q) v[q] = ref[q] - d * o[q];
        if (std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) >= 1e-12) break;
        ref[0] = 1.0; ref[1] = 0.0; ref[2] = 0.0;
    }
    const double n = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int q = 0; q < 3; ++q) v[q] /= n;
    out[0] = v[1] * o[2] - v[2] * o[1];
    out[1] = v[2] * o[0] - v[0] * o[2];
    out[2] = v[0] * o[1] - v[1] * o[0];
    out[3] = v[0]; out[4] = v[1]; out[5] = v[2];
}

// Albedo and emission.  The (spec, g) solves are grouped into batches; per
// batch every solve gets its own optics (and emission CDF) slot, then one
// persistent transport launch runs all their packets and a fixed-order
// reduction turns the packet rows into one tally row per solve.
int solve_packets(mcrt_ctx* ctx, Slot& sl, hipStream_t def_stream, int32_t gid, int32_t oid,
                  const mcrt_solve_params* p, mcrt_result* res, int mode)
{
    if (!res) return fail(MCRT_EINVAL, "result is NULL");
    Lease ls;
    int rc = lease(ctx, gid, oid, ls);
    if (rc) return rc;
    GridRes* g = ls.g;
    OpacRes* op = ls.op;
    SolvePlan pl;
    rc = plan_common(def_stream, g, op, p, mode, pl);
    if (rc) return rc;
    if (op->kind == MCRT_OPAC_HIRES && mode == MCRT_MODE_ALBEDO)
        return fail(MCRT_EINVAL, "albedo solves take a correlated-k table");
    if (op->kind == MCRT_OPAC_HIRES && pl.n_out != 1)
        return fail(MCRT_EINVAL, "high-resolution emission is Doppler-shifted per observer: pass one observer per call");
    if (p->max_batch < 0 || p->tune_ev_threshold < 0 || p->tune_ev_threshold > 64 || p->tune_blocks_per_cu < 0 ||
        p->tune_blocks_per_cu > 16 || p->tune_wave_batch < 0)
        return fail(MCRT_EINVAL, "bad batching / tuning parameters");
    if ((p->contrib || p->image_npix) && sl.stream_ordered)
        return fail(MCRT_EINVAL, "contribution functions and images are computed by blocking solves only");
    if (p->contrib && !res->cf) return fail(MCRT_EINVAL, "contrib needs result.cf");
    if (p->image_npix < 0 || p->image_npix > 4096) return fail(MCRT_EINVAL, "image_npix must be in [0, 4096]");
    if (p->image_npix && (!res->image || g->dev.geom != 0))
        return fail(MCRT_EINVAL, "images need result.image and a spherical grid");
    if (mode == MCRT_MODE_TRANSMISSION && (p->contrib || p->image_npix || p->g_sampling))
        return fail(MCRT_EINVAL, "contribution functions, images and g-ordinate sampling are defined for "
                                 "albedo and emission");
    const bool gs = p->g_sampling != 0;
    if (p->g_sampling < 0 || p->g_sampling > 3) return fail(MCRT_EINVAL, "g_sampling must be 0 to 3");
    if (gs && op->kind != MCRT_OPAC_CK) return fail(MCRT_EINVAL, "g-ordinate sampling needs a correlated-k table");
    if (gs && (p->contrib || p->image_npix))
        return fail(MCRT_EINVAL, "g-ordinate sampling does not combine with contribution functions or images");
    HIPTRY(hipSetDevice(ctx->device));
    hipStream_t st = pl.stream;
    const bool mixed = p->precision == MCRT_MIXED;
    const int ncell = g->ncell;
    const int ns = (int)pl.specs.size(), ng = pl.ng, nsolve = ns * ng;
    const int no = pl.n_out;
    const int pw = 2 * no + kNCounters;  // tally columns
    const int row_w = pw + 2;           // + (L_tot, N_emit)
    const int prow = no + kNCounters;   // packet row
    const uint64_t N = p->n_packets;

    // per-solve device footprint and the batch size the budget allows
    const size_t opt_b = (size_t)ncell * 5 * (sizeof(double) + (mixed ? sizeof(float) : 0));
    const size_t src_b = mode == MCRT_MODE_EMISSION ? (size_t)ncell * 2 * sizeof(double) : 0;
    const size_t row_b = (size_t)N * prow * sizeof(double);
    // with g-ordinate sampling a band's packets (one range) serve its ng solves
    const size_t per_solve = opt_b + src_b + (gs ? row_b / ng : row_b);
    const int chunks = reduce_rows_chunks(N);
    const size_t cf_n = p->contrib ? (size_t)ns * no * 2 * ncell : 0;  // [spec][observer][2][cell]
    const int npix = p->image_npix;
    const size_t img_n = (size_t)ns * no * npix * npix;  // [spec][observer][row][column]
    int batch;
    if (sl.arena) {
        // the largest batch whose scratch, carved below in this order, fits the arena
        auto carved = [&](int b) {
            size_t t = 0;
            auto add = [&t](size_t x) { t = ((t + 255) & ~(size_t)255) + x; };
            add(sizeof(double) * 5 * (size_t)ncell * b);
            if (mixed) add(sizeof(float) * 5 * (size_t)ncell * b);
            add(row_b * (size_t)(gs ? b / ng : b));
            add(sizeof(double) * (size_t)nsolve * row_w);
            add(sizeof(double) * (size_t)b * chunks * pw);
            add(sizeof(SolveDev) * (size_t)b);
            add(sizeof(PrepSlot) * (size_t)b);
            add(sizeof(unsigned long long) * kXcds);
            if (mode == MCRT_MODE_EMISSION) {
                add(src_b * b);
                add(sizeof(double) * prep_scratch_doubles(ncell, b));
            }
            if (op->kind == MCRT_OPAC_HIRES) add(sizeof(double) * (size_t)ncell);
            if (cf_n) add(sizeof(double) * cf_n);
            if (img_n) add(sizeof(double) * img_n);
            return t;
        };
        const int step = gs ? ng : 1;  // whole bands per launch with g-ordinate sampling
        int lo = step, hi = std::max(step, std::min(p->max_batch > 0 ? p->max_batch : nsolve, nsolve) / step * step);
        hi = std::min(hi, kMaxSolvesPerLaunch / step * step);
        if (carved(lo) > sl.arena_cap)
            return fail(MCRT_EINVAL, "one launch of this solve needs %zu bytes of scratch, more than the fixed %zu",
                        carved(lo), sl.arena_cap);
        while (lo < hi) {
            const int mid = (lo / step + (hi / step - lo / step + 1) / 2) * step;
            if (carved(mid) <= sl.arena_cap) lo = mid;
            else hi = mid - step;
        }
        batch = lo;
    } else if (sl.stream_ordered) {
        batch = serving_batch(ctx, p->max_batch, nsolve, per_solve, gs ? N / ng + 1 : N);  // as admitted
    } else {
        batch = p->max_batch > 0 ? p->max_batch : nsolve;
        uint64_t room;
        {
            // the slot's own scratch is regrown in place (each buffer freed
            // before its larger successor is allocated), so it counts as room:
            // repeated calls then plan the same launches as the first
            uint64_t own = 0;
            for (const auto& kv : sl.scratch) own += kv.second.bytes;
            std::lock_guard<std::mutex> mk(ctx->mem_mu);
            const uint64_t held = held_locked(ctx);
            room = ctx->budget - std::min(ctx->budget, held - std::min(held, own));
        }
        uint64_t cap = room / 2;  // half of what the budget leaves: fewer launches, fewer drain tails
        int fit = (int)std::max<uint64_t>(1, cap / std::max<size_t>(per_solve, 1));
        batch = std::max(1, std::min(std::min(batch, fit), nsolve));
    }
    batch = std::min(batch, kMaxSolvesPerLaunch);
    if (gs) batch = std::max(ng, batch / ng * ng);  // whole bands per launch
    void *v_opt, *v_optf = nullptr, *v_src = nullptr, *v_rows, *v_sums, *v_part, *v_ps = nullptr,
                 *v_shift = nullptr, *v_solves, *v_slots, *v_ctr;
    if ((rc = slot_scratch(ctx, sl, st, "optics", sizeof(double) * 5 * (size_t)ncell * batch, &v_opt))) return rc;
    if (mixed && (rc = slot_scratch(ctx, sl, st, "optics_f32", sizeof(float) * 5 * (size_t)ncell * batch, &v_optf)))
        return rc;
    if ((rc = slot_scratch(ctx, sl, st, "rows", row_b * (gs ? batch / ng : batch), &v_rows))) return rc;
    if ((rc = slot_scratch(ctx, sl, st, "sums", sizeof(double) * (size_t)nsolve * row_w, &v_sums))) return rc;
    if ((rc = slot_scratch(ctx, sl, st, "row_part", sizeof(double) * (size_t)batch * chunks * pw, &v_part))) return rc;
    if ((rc = slot_scratch(ctx, sl, st, "solves", sizeof(SolveDev) * (size_t)batch, &v_solves))) return rc;
    if ((rc = slot_scratch(ctx, sl, st, "prep_slots", sizeof(PrepSlot) * (size_t)batch, &v_slots))) return rc;
    if ((rc = slot_scratch(ctx, sl, st, "dispenser", sizeof(unsigned long long) * kXcds, &v_ctr))) return rc;
    if (mode == MCRT_MODE_EMISSION) {
        if ((rc = slot_scratch(ctx, sl, st, "sources", src_b * batch, &v_src))) return rc;
        if ((rc = slot_scratch(ctx, sl, st, "prep_scratch", sizeof(double) * prep_scratch_doubles(ncell, batch), &v_ps)))
            return rc;
    }
    if (op->kind == MCRT_OPAC_HIRES)
        if ((rc = slot_scratch(ctx, sl, st, "shift", sizeof(double) * (size_t)ncell, &v_shift))) return rc;
    void* v_cf = nullptr;  // contribution functions
    if (p->contrib && (rc = slot_scratch(ctx, sl, st, "contrib", sizeof(double) * cf_n, &v_cf))) return rc;
    void* v_img = nullptr;  // images
    if (npix && (rc = slot_scratch(ctx, sl, st, "image", sizeof(double) * img_n, &v_img))) return rc;
    double* sums = (double*)v_sums;

    BatchArgs A{};
    A.counter = (unsigned long long*)v_ctr;
    A.rows = (double*)v_rows;
    A.row_w = prow;
    A.seed = p->seed;
    A.scattering = p->scattering ? 1 : 0;
    A.absorption = p->absorption;
    A.n_obs = pl.n_obs;
    A.n_out = no;
    A.max_events = p->max_events;
    A.rr_threshold = p->rr_threshold;
    A.rr_survive = p->rr_survive;
    A.tau_peel_max = p->tau_peel_max;
    A.mu0 = p->mu0;
    A.r_toa = g->r_toa;
    for (int q = 0; q < 3 * pl.n_obs; ++q) A.obs[0][q] = A.obs[1][q] = pl.obs[q];
    A.batch = p->tune_wave_batch > 0 ? p->tune_wave_batch : 64;
    A.ev_threshold = p->tune_ev_threshold > 0 ? p->tune_ev_threshold : 16;
    A.cloud_phase = p->cloud_phase;
    A.draine_alpha = p->draine_alpha;
    A.forced = p->forced;
    A.forced_first = p->forced_first;
    A.surface_albedo = p->surface_albedo;
    A.trans_ms = mode == MCRT_MODE_TRANSMISSION ? 1 : 0;
    if (A.trans_ms) {
        const double q = p->r_star / p->a_orbit;
        A.peel_w = kPi * (q * q);
        A.ld = LimbDark{p->ld_law, p->ld_c1, p->ld_c2, p->transit_y, p->transit_z, p->r_star};
    } else {
        A.peel_w = 1.0;
    }
    const int bpc = p->tune_blocks_per_cu > 0 ? p->tune_blocks_per_cu : 4;
    const int pblocks = ctx->n_cu * bpc;
    if (npix) {
        A.npix = npix;
        A.img_half = g->r_toa;
        for (int o = 0; o < pl.n_obs; ++o) sky_axes(&pl.obs[3 * o], &A.img_axes[6 * o]);
    }

    const bool use_graph = p->graph != 0 && !sl.stream_ordered;
    const bool prof = p->profile != 0 && !use_graph;
    const int nbatches = (nsolve + batch - 1) / batch;
    if (prof && (rc = prof_events(ctx, sl, (size_t)nbatches))) return rc;
    res->kernel_ms = 0.0;
    res->kernel_launches = 0;

    // Replayable form: the whole device chain below is recorded once per set
    // of arguments (ids, parameters, launch shape, stream and the scratch
    // addresses it bakes in) and replayed afterwards.
    GraphEntry* ge = nullptr;
    bool capture = false;
    std::string gkey;
    if (use_graph) {
        auto add = [&gkey](const void* v, size_t n) { gkey.append((const char*)v, n); };
        const int32_t ids[3] = {mode, gid, oid};
        add(ids, sizeof ids);
        const double dpar[15] = {p->rr_threshold, p->rr_survive, p->emis_bias, p->tau_vert_max, p->tau_peel_max,
                                 p->mu0, (double)p->max_events, p->surface_albedo, p->r_star, p->a_orbit,
                                 p->ld_c1, p->ld_c2, p->transit_y, p->transit_z, p->draine_alpha};
        add(dpar, sizeof dpar);
        const int64_t ipar[16] = {(int64_t)p->seed, (int64_t)N, p->precision, p->decorrelate, p->scattering,
                                  p->absorption, batch, A.ev_threshold, bpc, A.batch, npix, p->g_sampling,
                                  p->cloud_phase, p->ld_law, p->forced, p->forced_first};
        add(ipar, sizeof ipar);
        add(pl.obs.data(), sizeof(double) * pl.obs.size());
        add(pl.specs.data(), sizeof(int) * pl.specs.size());
        const void* ptrs[16] = {p->packet_dump, st, v_opt, v_optf, v_src, v_rows, v_sums, v_part,
                                v_solves, v_slots, v_ctr, v_ps, v_shift, v_cf, v_img,
                                (const void*)(uintptr_t)pl.n_obs};
        add(ptrs, sizeof ptrs);
        std::lock_guard<std::mutex> gk(ctx->graph_mu);
        auto it = ctx->graphs.find(gkey);
        if (it != ctx->graphs.end()) {
            ge = it->second.get();
        } else {
            if (ctx->graphs.size() >= kMaxGraphs) {  // drop the least recently used
                auto lru = ctx->graphs.begin();
                for (auto q = ctx->graphs.begin(); q != ctx->graphs.end(); ++q)
                    if (q->second->used < lru->second->used) lru = q;
                ctx->graphs.erase(lru);
            }
            std::unique_ptr<GraphEntry> e(new GraphEntry());
            e->gid = gid;
            e->oid = oid;
            HIPTRY(hipHostMalloc(&e->pinned, (sizeof(SolveDev) + sizeof(PrepSlot)) * (size_t)nbatches * batch));
            ge = e.get();
            ctx->graphs[gkey] = std::move(e);
            capture = true;
        }
        ge->used = ++ctx->graph_clock;
    }
    SolveDev* pin_solves = ge ? (SolveDev*)ge->pinned : nullptr;
    PrepSlot* pin_slots = ge ? (PrepSlot*)(pin_solves + (size_t)nbatches * batch) : nullptr;
    std::vector<std::vector<SolveDev>> host_solves(use_graph ? 0 : nbatches);
    std::vector<std::vector<PrepSlot>> host_slots(use_graph ? 0 : nbatches);

    // The device chain: tally clear, Doppler shifts, then per batch the solve
    // tables, preparation, births, transport and reduction.
    auto enqueue = [&]() -> int {
        launch_fill_f64(sums, (size_t)nsolve * row_w, 0.0, st);
        if (v_cf) launch_fill_f64((double*)v_cf, cf_n, 0.0, st);
        if (v_img) launch_fill_f64((double*)v_img, img_n, 0.0, st);
        if (op->kind == MCRT_OPAC_HIRES)
            launch_doppler_shift(g->dev, pl.obs[0], pl.obs[1], pl.obs[2], op->dlnlam, (double*)v_shift, st);
        for (int bt = 0; bt < nbatches; ++bt) {
            const int s0 = bt * batch, s1 = std::min(nsolve, s0 + batch), nb = s1 - s0;
            SolveDev* hsv;
            PrepSlot* hps;
            if (use_graph) {
                hsv = pin_solves + (size_t)bt * batch;
                hps = pin_slots + (size_t)bt * batch;
            } else {
                host_solves[bt].resize(nb);
                host_slots[bt].resize(nb);
                hsv = host_solves[bt].data();
                hps = host_slots[bt].data();
            }
            for (int sg = s0; sg < s1; ++sg) {
                const int slot = sg - s0;
                const int b = pl.specs[sg / ng], gi = sg % ng;
                PrepSlot& P = hps[slot];
                P = PrepSlot{};
                P.lnk = op->kind == MCRT_OPAC_CK ? op->lnk + ((size_t)b * op->ng + gi) * op->nT * op->nP : nullptr;
                P.k_ray = op->k_ray[b];
                P.n = b;
                const double lam = op->kind == MCRT_OPAC_CK ? op->lam_um[b] : op->lam_min * std::exp(b * op->dlnlam);
                P.lam_cm = lam * 1e-4;
                P.opt = (double*)v_opt + (size_t)slot * 5 * ncell;
                P.optf = mixed ? (float*)v_optf + (size_t)slot * 5 * ncell : nullptr;
                P.cdf = mode == MCRT_MODE_EMISSION ? (double*)v_src + (size_t)slot * 2 * ncell : nullptr;
                P.wbirth = P.cdf ? P.cdf + ncell : nullptr;
                P.stats = sums + (size_t)sg * row_w + pw;
                SolveDev& S = hsv[slot];
                S = SolveDev{};
                if (gs) {  // the band's packets belong to its g = 0 solve; the others are empty ranges after it
                    const unsigned long long band0 = (unsigned long long)(slot / ng) * N;
                    S.begin = gi == 0 ? band0 : band0 + N;
                    S.n = gi == 0 ? N : 0;
                    S.pbase = band0;
                    S.tag = p->decorrelate ? (uint32_t)(1 + b * ng) : 0u;
                    S.gs_n = gi == 0 ? ng : 0;
                    S.gs_scheme = p->g_sampling;
                    S.gs_w = op->gw_dev;
                } else {
                    S.begin = (unsigned long long)slot * N;
                    S.n = N;
                    S.pbase = S.begin;
                    S.tag = p->decorrelate ? (uint32_t)(1 + b * ng + gi) : 0u;
                }
                S.ltot = mode == MCRT_MODE_EMISSION ? P.stats : nullptr;
                S.mode = mode == MCRT_MODE_EMISSION ? 1 : (mode == MCRT_MODE_TRANSMISSION ? 2 : 0);
                S.grid = 0;
                S.cdf = P.cdf;
                S.wbirth = P.wbirth;
                if (v_cf || v_img) {  // scaled as the band value: w_g pi / N, or w_g L_tot / (N R_TOA^2)
                    const double wg = op->kind == MCRT_OPAC_CK ? op->g_weights[gi] : 1.0;
                    S.cf = v_cf ? (double*)v_cf + (size_t)(sg / ng) * no * 2 * ncell : nullptr;
                    S.img = v_img ? (double*)v_img + (size_t)(sg / ng) * no * npix * npix : nullptr;
                    S.cf_w = mode == MCRT_MODE_ALBEDO ? wg * kPi / (double)N
                                                      : wg / ((double)N * g->r_toa * g->r_toa);
                    S.cf_ltot = mode == MCRT_MODE_EMISSION ? P.stats : nullptr;
                }
                if (mixed) {
                    const float* f = P.optf;
                    S.a_ext = f; S.a_abs = f + ncell; S.omega = f + 2 * (size_t)ncell; S.p_gas = f + 3 * (size_t)ncell;
                    S.g_cld = f + 4 * (size_t)ncell;
                } else {
                    const double* d = P.opt;
                    S.a_ext = d; S.a_abs = d + ncell; S.omega = d + 2 * (size_t)ncell; S.p_gas = d + 3 * (size_t)ncell;
                    S.g_cld = d + 4 * (size_t)ncell;
                }
            }
            HIPTRY(hipMemcpyAsync(v_slots, hps, sizeof(PrepSlot) * nb, hipMemcpyHostToDevice, st));
            HIPTRY(hipMemcpyAsync(v_solves, hsv, sizeof(SolveDev) * nb, hipMemcpyHostToDevice, st));
            launch_prep_optics(g->dev, ncell, (const PrepSlot*)v_slots, nb, op->kind == MCRT_OPAC_HIRES ? 1 : 0, op->nT,
                               op->nP, op->T_grid, op->lnP_grid, op->lnk, op->nspec, (const double*)v_shift,
                               p->cloud_phase == 2 ? 1 : 0, p->draine_alpha, st);
            if (mode == MCRT_MODE_EMISSION)
                launch_prep_sources(g->dev, ncell, (const PrepSlot*)v_slots, nb, p->tau_vert_max, p->emis_bias,
                                    (double*)v_ps, st);
            A.solves = (const SolveDev*)v_solves;
            A.n_solves = nb;
            A.total = (unsigned long long)(gs ? nb / ng : nb) * N;
            launch_init_dispensers(A.counter, A.total, st);
            launch_births(g->dev, A, false, st);
            if (prof) HIPTRY(hipEventRecord(sl.prof_ev[2 * bt], st));
            launch_transport_persistent(g->dev, A, mixed, false, sl.stream_ordered ? serving_blocks(ctx, bpc) : pblocks,
                                        bpc, st);
            if (prof) HIPTRY(hipEventRecord(sl.prof_ev[2 * bt + 1], st));
            double* dump = p->packet_dump ? p->packet_dump + (size_t)(gs ? s0 / ng : s0) * N * no : nullptr;
            launch_reduce_rows(A, nullptr, nb, (double*)v_part, chunks, sums + (size_t)s0 * row_w, row_w, dump, st);
            // the next batch reuses the slots: in eager form its pageable host tables are
            // copied only after this batch ran
            if (!use_graph && bt + 1 < nbatches) HIPTRY(hipStreamSynchronize(st));
        }
        return MCRT_OK;
    };
    if (use_graph) {
        if (capture) {
            HIPTRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            int crc = enqueue();
            hipGraph_t gr = nullptr;
            hipError_t ee = hipStreamEndCapture(st, &gr);
            if (crc == MCRT_OK && ee == hipSuccess)
                ee = hipGraphInstantiate(&ge->exec, gr, nullptr, nullptr, 0);
            ge->graph = gr;
            if (crc != MCRT_OK || ee != hipSuccess) {
                std::lock_guard<std::mutex> gk(ctx->graph_mu);
                ctx->graphs.erase(gkey);
                if (crc != MCRT_OK) return crc;
                HIPTRY(ee);
            }
        }
        HIPTRY(hipEventRecord(sl.ev0, st));
        HIPTRY(hipGraphLaunch(ge->exec, st));
    } else {
        HIPTRY(hipEventRecord(sl.ev0, st));
        if ((rc = enqueue())) return rc;
    }
    HIPTRY(hipGetLastError());
    std::vector<double> hs((size_t)nsolve * row_w);
    HIPTRY(hipMemcpyAsync(hs.data(), sums, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, st));
    if ((rc = finish_timing(ctx, sl, st, res))) return rc;
    if (prof && (rc = prof_collect(ctx, sl, (size_t)nbatches, res))) return rc;
    if (use_graph) res->kernel_ms = res->elapsed_ms;  // the whole replay

    // Post-processing (Sect. 5.2 A_g = pi E; Sect. 5.3 F_p = L_tot/(N R_TOA^2) sum F)
    std::vector<double> val((size_t)nsolve * no), se((size_t)nsolve * no), cnt((size_t)nsolve * kNCounters),
        ltot(nsolve);
    const double Nd = (double)N;
    for (int sg = 0; sg < nsolve; ++sg) {
        const double* row = hs.data() + (size_t)sg * row_w;
        if (mode == MCRT_MODE_TRANSMISSION) {
            // (R_p/R*)^2 = (R0^2 + 2 (R_TOA - R0) <W0 - F>) / R*^2  (Sect. 5.1)
            const double dr = g->r_toa - g->r0, rs2 = p->r_star * p->r_star;
            const double m = row[0] / Nd;
            const double var = std::max(row[1] / Nd - m * m, 0.0) / Nd;
            val[sg] = (g->r0 * g->r0 + 2.0 * dr * m) / rs2;
            se[sg] = 2.0 * dr * std::sqrt(var) / rs2;
            for (int t = 0; t < kNCounters; ++t) cnt[(size_t)sg * kNCounters + t] = row[2 * no + t];
            continue;
        }
        double scale;
        if (mode == MCRT_MODE_ALBEDO) {
            scale = kPi;
        } else {
            ltot[sg] = row[pw];
            scale = row[pw] / (g->r_toa * g->r_toa);
        }
        for (int o = 0; o < no; ++o) {
            double m = row[2 * o] / Nd;
            double var = std::max(row[2 * o + 1] / Nd - m * m, 0.0) / Nd;
            val[(size_t)sg * no + o] = scale * m;
            se[(size_t)sg * no + o] = scale * std::sqrt(var);
        }
        for (int t = 0; t < kNCounters; ++t) cnt[(size_t)sg * kNCounters + t] = row[2 * no + t];
    }
    std::vector<double> gw = op->kind == MCRT_OPAC_CK ? op->g_weights : std::vector<double>{1.0};
    if (gs) {  // band values from the band's packets (in its g = 0 row): pi sum F / N,
               // or sum_g(w_g L_g) sum F / (N R_TOA^2); reported in the g = 0 slot
        for (int sb = 0; sb < ns; ++sb) {
            const double* row = hs.data() + (size_t)sb * ng * row_w;
            double scale = kPi;
            if (mode == MCRT_MODE_EMISSION) {
                double lb = 0.0;
                for (int gi = 0; gi < ng; ++gi) lb += op->g_weights[gi] * ltot[(size_t)sb * ng + gi];
                scale = lb / (g->r_toa * g->r_toa);
            }
            for (int gi = 0; gi < ng; ++gi)
                for (int o = 0; o < no; ++o) {
                    const size_t at = ((size_t)sb * ng + gi) * no + o;
                    if (gi > 0) {
                        val[at] = se[at] = 0.0;
                        continue;
                    }
                    const double m = row[2 * o] / Nd;
                    const double var = std::max(row[2 * o + 1] / Nd - m * m, 0.0) / Nd;
                    val[at] = scale * m;
                    se[at] = scale * std::sqrt(var);
                }
        }
        gw.assign(ng, 0.0);
        gw[0] = 1.0;
    }
    fill_results(pl, val, se, gw, hs, row_w, cnt, ltot, res);
    if (v_cf) {  // contribution functions, normalised per (band, observer)
        HIPTRY(hipMemcpy(res->cf, v_cf, sizeof(double) * cf_n, hipMemcpyDeviceToHost));
        for (size_t b = 0; b < (size_t)ns * no; ++b) {
            double* blk = res->cf + b * 2 * ncell;
            double tot = 0.0;
            for (size_t c = 0; c < 2 * (size_t)ncell; ++c) tot += blk[c];
            for (size_t c = 0; c < 2 * (size_t)ncell; ++c) blk[c] = tot > 0.0 ? blk[c] / tot : 0.0;
        }
    }
    if (v_img) HIPTRY(hipMemcpy(res->image, v_img, sizeof(double) * img_n, hipMemcpyDeviceToHost));
    return MCRT_OK;
}

// Transmission: chord geometry once, then per block of up to 64 spectral
// rows: alpha gather -> chord optical depths -> fixed-order tally.
int solve_chords(mcrt_ctx* ctx, Slot& sl, hipStream_t def_stream, int32_t gid, int32_t oid,
                 const mcrt_solve_params* p, mcrt_result* res)
{
    if (!res) return fail(MCRT_EINVAL, "result is NULL");
    Lease ls;
    int rc = lease(ctx, gid, oid, ls);
    if (rc) return rc;
    GridRes* g = ls.g;
    OpacRes* op = ls.op;
    SolvePlan pl;
    rc = plan_common(def_stream, g, op, p, MCRT_MODE_TRANSMISSION, pl);
    if (rc) return rc;
    if (p->contrib || p->image_npix || p->g_sampling)
        return fail(MCRT_EINVAL, "contribution functions, images and g-ordinate sampling are defined for "
                                 "albedo and emission");
    HIPTRY(hipSetDevice(ctx->device));
    hipStream_t st = pl.stream;
    const int ncell = g->ncell;
    const int nch = p->n_b * p->n_alpha;
    const int ns = (int)pl.specs.size(), ng = pl.ng;
    const int nrow = ns * ng;
    const int kSlot = 64;
    const int nslot_max = std::min(kSlot, nrow);
    void *v_cnt, *v_off, *v_b, *v_ok, *v_alpha, *v_part, *v_sums, *v_shift = nullptr, *v_nl = nullptr;
    if ((rc = slot_scratch(ctx, sl, st, "chord_cnt", sizeof(int) * (size_t)nch, &v_cnt))) return rc;
    if ((rc = slot_scratch(ctx, sl, st, "chord_off", sizeof(long long) * ((size_t)nch + 1), &v_off))) return rc;
    if ((rc = slot_scratch(ctx, sl, st, "chord_b", sizeof(double) * (size_t)nch, &v_b))) return rc;
    if ((rc = slot_scratch(ctx, sl, st, "chord_ok", sizeof(int) * (size_t)nch, &v_ok))) return rc;
    // Blocking solves with more than one block of rows alternate the blocks
    // between two streams with their own extinction and partial-sum buffers,
    // so that one block's extinction rows are formed while the previous
    // block's chords are summed; served requests use their one stream.
    const int nbuf = (!sl.stream_ordered && nrow > kSlot) ? 2 : 1;
    if (nbuf == 2 && !sl.stream2)  // made on first use, so that slots that never need it hold no queue
        if ((rc = own_queue_stream(&sl.stream2, ctx->n_cu))) return rc;
    const size_t alpha_n = (size_t)ncell * nslot_max;
    int tblocks = chord_tau_blocks(nch);
    const size_t part_n = (size_t)tblocks * 2 * nslot_max;
    if ((rc = slot_scratch(ctx, sl, st, "alpha_blk", sizeof(double) * alpha_n * nbuf, &v_alpha))) return rc;
    if ((rc = slot_scratch(ctx, sl, st, "chord_part", sizeof(double) * part_n * nbuf, &v_part))) return rc;
    if ((rc = slot_scratch(ctx, sl, st, "chord_sums", sizeof(double) * (size_t)nrow * 2, &v_sums))) return rc;
    void* v_tp = nullptr;
    if (op->kind == MCRT_OPAC_HIRES) {
        if ((rc = slot_scratch(ctx, sl, st, "shift", sizeof(double) * (size_t)ncell, &v_shift))) return rc;
        if ((rc = slot_scratch(ctx, sl, st, "nlist", sizeof(int) * (size_t)ns, &v_nl))) return rc;
        if ((rc = slot_scratch(ctx, sl, st, "cell_tp", sizeof(CellTP) * (size_t)ncell, &v_tp))) return rc;
    }
    const uint32_t tag = 0;  // chords are common to all spectral points
    const bool prof = p->profile != 0;
    const int nblk_rows = (nrow + kSlot - 1) / kSlot;
    if (prof && (rc = prof_events(ctx, sl, (size_t)nblk_rows))) return rc;
    res->kernel_ms = 0.0;
    res->kernel_launches = 0;
    HIPTRY(hipEventRecord(sl.ev0, st));
    launch_chord_count(g->dev, p->n_b, p->n_alpha, p->seed, tag, (int*)v_cnt, st);
    launch_exclusive_scan_int((int*)v_cnt, (long long*)v_off, nch, nullptr, st);
    long long nseg = 0;
    HIPTRY(hipMemcpyAsync(&nseg, (long long*)v_off + nch, sizeof(long long), hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    res->n_segments = nseg;
    void *v_sc, *v_sl;
    if ((rc = slot_scratch(ctx, sl, st, "seg_cell", sizeof(uint32_t) * (size_t)std::max(nseg, 1LL), &v_sc))) return rc;
    if ((rc = slot_scratch(ctx, sl, st, "seg_len", sizeof(double) * (size_t)std::max(nseg, 1LL), &v_sl))) return rc;
    const LimbDark ld{p->ld_law, p->ld_c1, p->ld_c2, p->transit_y, p->transit_z, p->r_star};
    const bool mixed = p->precision == MCRT_MIXED;
    if (mixed)
        launch_chord_fill(g->dev, p->n_b, p->n_alpha, p->seed, tag, (long long*)v_off, (uint32_t*)v_sc, (float*)v_sl,
                          (double*)v_b, (int*)v_ok, ld, st);
    else
        launch_chord_fill(g->dev, p->n_b, p->n_alpha, p->seed, tag, (long long*)v_off, (uint32_t*)v_sc, (double*)v_sl,
                          (double*)v_b, (int*)v_ok, ld, st);
    if (op->kind == MCRT_OPAC_HIRES) {
        launch_doppler_shift(g->dev, -1.0, 0.0, 0.0, op->dlnlam, (double*)v_shift, st);
        launch_cell_tp(g->dev, ncell, op->nT, op->nP, op->T_grid, op->lnP_grid, (CellTP*)v_tp, st);
        HIPTRY(hipMemcpyAsync(v_nl, pl.specs.data(), sizeof(int) * ns, hipMemcpyHostToDevice, st));
    }
    // Per block of up to 64 spectral rows: extinction of every cell (FP64, or
    // FP32 in the mixed form: half the bytes the chords gather), then the
    // chords' optical depths, accumulated in FP64 either way.
    auto rows_block = [&](auto* alpha, int r0, int nslot, hipStream_t st, double* part) {
        using R = std::remove_pointer_t<decltype(alpha)>;
        if (op->kind == MCRT_OPAC_CK) {
            for (int q = 0; q < nslot; ++q) {
                int rr = r0 + q, b = pl.specs[rr / ng], gi = rr % ng;
                const double* tab = op->lnk + ((size_t)b * op->ng + gi) * op->nT * op->nP;
                OpticsDev<R> od{alpha + q, nullptr, nullptr, nullptr, nullptr};
                launch_ck_optics(g->dev, ncell, tab, op->nT, op->nP, op->T_grid, op->lnP_grid, op->k_ray[b], od, nslot,
                                 st);
            }
        } else {
            const R* tab;
            if constexpr (sizeof(R) == sizeof(float)) tab = op->lnk_f32;
            else tab = op->lnk;
            launch_hires_alpha_block(g->dev, ncell, tab, op->nspec, op->nP, (const CellTP*)v_tp, op->k_ray_dev,
                                     (double*)v_shift, (int*)v_nl + r0, nslot, nslot, alpha, st);
        }
        if (prof) (void)hipEventRecord(sl.prof_ev[2 * (r0 / kSlot)], st);
        launch_chord_tau(p->n_b, p->n_alpha, (long long*)v_off, (uint32_t*)v_sc, (const R*)v_sl, (double*)v_b, (int*)v_ok,
                         (const R*)alpha, nslot, part, tblocks, st);
        if (prof) (void)hipEventRecord(sl.prof_ev[2 * (r0 / kSlot) + 1], st);
        launch_reduce_partials(part, tblocks, 2 * nslot, (double*)v_sums + 2 * (size_t)r0, st);
    };
    hipStream_t st2 = nbuf == 2 ? sl.stream2 : st;
    if (nbuf == 2) {  // the second stream starts after the common work above
        HIPTRY(hipEventRecord(sl.fork, st));
        HIPTRY(hipStreamWaitEvent(st2, sl.fork, 0));
    }
    for (int r0 = 0; r0 < nrow; r0 += kSlot) {
        const int nslot = std::min(kSlot, nrow - r0), b = (r0 / kSlot) % nbuf;
        hipStream_t sb = b ? st2 : st;
        double* part = (double*)v_part + part_n * b;
        if (mixed) rows_block((float*)v_alpha + alpha_n * b, r0, nslot, sb, part);
        else rows_block((double*)v_alpha + alpha_n * b, r0, nslot, sb, part);
    }
    if (nbuf == 2) {  // the first stream waits for the second's last block
        HIPTRY(hipEventRecord(sl.join, st2));
        HIPTRY(hipStreamWaitEvent(st, sl.join, 0));
    }
    HIPTRY(hipGetLastError());
    std::vector<double> hs((size_t)nrow * 2);
    HIPTRY(hipMemcpyAsync(hs.data(), v_sums, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, st));
    if ((rc = finish_timing(ctx, sl, st, res))) return rc;
    if (prof && (rc = prof_collect(ctx, sl, (size_t)nblk_rows, res))) return rc;

    // (R_p/R*)^2 = (R0^2 + 2 <I>)/R*^2, <I> = (R_TOA - R0)/N sum (1 - e^-tau) b  (Sect. 5.1)
    const double dr = g->r_toa - g->r0, Nd = (double)nch, rs2 = p->r_star * p->r_star;
    std::vector<double> val(nrow), se(nrow), cnt((size_t)nrow * kNCounters, 0.0), ltot(nrow, 0.0);
    for (int r = 0; r < nrow; ++r) {
        double s1 = hs[2 * r], s2 = hs[2 * r + 1];
        double I = dr * s1 / Nd;
        double m = s1 / Nd;
        double var = std::max(s2 / Nd - m * m, 0.0) / Nd;
        val[r] = (g->r0 * g->r0 + 2.0 * I) / rs2;
        se[r] = 2.0 * dr * std::sqrt(var) / rs2;
    }
    std::vector<double> gw = op->kind == MCRT_OPAC_CK ? op->g_weights : std::vector<double>{1.0};
    // sums rows are [row][2] already (n_out = 1)
    std::vector<double> sumrows(hs);
    fill_results(pl, val, se, gw, sumrows, 2, cnt, ltot, res);
    return MCRT_OK;
}

// ------------------------------------------------------------------ batch
// Many albedo / emission requests on grids of uneven size: every item's
// (spectral point, g) solves are flattened into one list and packed, as far
// as the budget allows, into multi-grid persistent launches; preparation runs
// per item, the transport per launch, the tally reduction per solve.
int solve_batch(mcrt_ctx* ctx, Slot& sl, hipStream_t def_stream, int n_items, const mcrt_batch_item* items,
                const mcrt_solve_params* common, mcrt_result* results)
{
    if (n_items < 1 || !items || !common || !results) return fail(MCRT_EINVAL, "batch needs items, params, results");
    if (common->contrib || common->image_npix || common->g_sampling)
        return fail(MCRT_EINVAL, "contribution functions, images and g-ordinate sampling are single-solve options");
    struct Item {
        Lease ls;
        SolvePlan pl;
        mcrt_solve_params p;
        int mode;
        int gslot;  // index into the batch grid table
        int first;  // first flattened solve
    };
    std::vector<std::unique_ptr<Item>> it(n_items);
    std::vector<GridRes*> grids;
    int rc;
    int no = -1;
    for (int q = 0; q < n_items; ++q) {
        it[q].reset(new Item());
        Item& I = *it[q];
        const mcrt_batch_item& b = items[q];
        if (b.mode != MCRT_MODE_ALBEDO && b.mode != MCRT_MODE_EMISSION)
            return fail(MCRT_EINVAL, "batch item %d: mode must be albedo or emission", q);
        if ((rc = lease(ctx, b.grid_id, b.opac_id, I.ls))) return rc;
        if (I.ls.g->dev.geom != 0) return fail(MCRT_EINVAL, "batch item %d: batched solves take spherical grids", q);
        if (I.ls.op->kind != MCRT_OPAC_CK) return fail(MCRT_EINVAL, "batch item %d: batched solves take ck tables", q);
        I.p = *common;
        I.p.spec_idx = b.spec_idx;
        I.p.n_spec = b.n_spec;
        I.p.n_packets = b.n_packets;
        I.p.packet_dump = nullptr;
        I.mode = b.mode;
        if ((rc = plan_common(def_stream, I.ls.g, I.ls.op, &I.p, I.mode, I.pl))) return rc;
        if (no >= 0 && I.pl.n_out != no) return fail(MCRT_EINVAL, "batch items must have the same number of observers");
        no = I.pl.n_out;
        auto f = std::find(grids.begin(), grids.end(), I.ls.g);
        I.gslot = (int)(f - grids.begin());
        if (f == grids.end()) grids.push_back(I.ls.g);
    }
    if (common->max_batch < 0 || common->tune_ev_threshold < 0 || common->tune_ev_threshold > 64 ||
        common->tune_blocks_per_cu < 0 || common->tune_blocks_per_cu > 16 || common->tune_wave_batch < 0)
        return fail(MCRT_EINVAL, "bad batching / tuning parameters");
    hipStream_t st = common->stream ? (hipStream_t)common->stream : def_stream;
    const bool mixed = common->precision == MCRT_MIXED;
    const int pw = 2 * no + kNCounters, row_w = pw + 2, prow = no + kNCounters;
    // flattened solves
    struct Flat {
        int item, spec, g;
        uint64_t bytes;
    };
    std::vector<Flat> fl;
    for (int q = 0; q < n_items; ++q) {
        Item& I = *it[q];
        I.first = (int)fl.size();
        const uint64_t nc = (uint64_t)I.ls.g->ncell;
        const uint64_t by = nc * 5 * (8 + (mixed ? 4 : 0)) + (I.mode == MCRT_MODE_EMISSION ? nc * 16 : 0) +
                            (uint64_t)I.p.n_packets * prow * 8 + 4 * 256;  // + alignment
        for (size_t s = 0; s < I.pl.specs.size(); ++s)
            for (int g = 0; g < I.pl.ng; ++g) fl.push_back(Flat{q, (int)s, g, by});
    }
    const int nsolve = (int)fl.size();
    uint64_t room;
    {
        std::lock_guard<std::mutex> mk(ctx->mem_mu);
        room = ctx->budget - std::min(ctx->budget, held_locked(ctx));
    }
    const uint64_t cap = std::min<uint64_t>(room / 2, 24ULL << 30);
    // launches: consecutive solves while the footprint fits (and <= max_batch)
    std::vector<std::pair<int, int>> launches;
    for (int s0 = 0; s0 < nsolve;) {
        uint64_t acc = 0;
        int s1 = s0;
        while (s1 < nsolve && (s1 == s0 || acc + fl[s1].bytes <= cap) && s1 - s0 < kMaxSolvesPerLaunch &&
               (common->max_batch <= 0 || s1 - s0 < common->max_batch)) {
            acc += fl[s1].bytes;
            ++s1;
        }
        launches.push_back({s0, s1});
        s0 = s1;
    }
    uint64_t max_bytes = 0, max_n = 1, max_slots = 1, max_prep = 16;
    int max_ncell = 1;
    for (auto& L : launches) {
        uint64_t acc = 0, mx = 1;
        for (int s = L.first; s < L.second; ++s) {
            acc += fl[s].bytes;
            mx = std::max<uint64_t>(mx, it[fl[s].item]->p.n_packets);
        }
        max_bytes = std::max(max_bytes, acc);
        max_n = std::max(max_n, mx);
        max_slots = std::max<uint64_t>(max_slots, (uint64_t)(L.second - L.first));
    }
    for (GridRes* g : grids) max_ncell = std::max(max_ncell, g->ncell);
    for (auto& L : launches) max_prep = std::max<uint64_t>(max_prep, prep_scratch_doubles(max_ncell, L.second - L.first));
    const int chunks = reduce_rows_chunks(max_n);
    void *v_arena, *v_sums, *v_part, *v_solves, *v_slots, *v_ctr, *v_grids, *v_ps;
    if ((rc = slot_scratch(ctx, sl, st, "batch_arena", max_bytes, &v_arena))) return rc;
    if ((rc = slot_scratch(ctx, sl, st, "sums", sizeof(double) * (size_t)nsolve * row_w, &v_sums))) return rc;
    if ((rc = slot_scratch(ctx, sl, st, "row_part", sizeof(double) * max_slots * chunks * pw, &v_part))) return rc;
    if ((rc = slot_scratch(ctx, sl, st, "solves", sizeof(SolveDev) * max_slots, &v_solves))) return rc;
    if ((rc = slot_scratch(ctx, sl, st, "prep_slots", sizeof(PrepSlot) * max_slots, &v_slots))) return rc;
    if ((rc = slot_scratch(ctx, sl, st, "dispenser", sizeof(unsigned long long) * kXcds, &v_ctr))) return rc;
    if ((rc = slot_scratch(ctx, sl, st, "grid_table", sizeof(GridDev) * grids.size(), &v_grids))) return rc;
    if ((rc = slot_scratch(ctx, sl, st, "prep_scratch", sizeof(double) * max_prep, &v_ps))) return rc;
    double* sums = (double*)v_sums;
    std::vector<GridDev> hgrids;
    for (GridRes* g : grids) hgrids.push_back(g->dev);

    BatchArgs A{};
    A.counter = (unsigned long long*)v_ctr;
    A.row_w = prow;
    A.grids = (const GridDev*)v_grids;
    A.seed = common->seed;
    A.scattering = common->scattering ? 1 : 0;
    A.absorption = common->absorption;
    A.n_obs = no;
    A.n_out = no;
    A.max_events = common->max_events;
    A.rr_threshold = common->rr_threshold;
    A.rr_survive = common->rr_survive;
    A.tau_peel_max = common->tau_peel_max;
    A.mu0 = common->mu0;
    A.r_toa = 0.0;  // per grid in multi-grid launches
    for (int q = 0; q < n_items; ++q) {
        const int m = it[q]->mode == MCRT_MODE_EMISSION ? 1 : 0;
        for (int k = 0; k < 3 * no; ++k) A.obs[m][k] = it[q]->pl.obs[k];
    }
    A.batch = common->tune_wave_batch > 0 ? common->tune_wave_batch : 64;
    A.ev_threshold = common->tune_ev_threshold > 0 ? common->tune_ev_threshold : 16;
    A.cloud_phase = common->cloud_phase;
    A.draine_alpha = common->draine_alpha;
    A.forced = common->forced;
    A.forced_first = common->forced_first;
    A.surface_albedo = common->surface_albedo;
    A.peel_w = 1.0;
    const int bpc = common->tune_blocks_per_cu > 0 ? common->tune_blocks_per_cu : 4;
    const int pblocks = ctx->n_cu * bpc;
    // Replayable form (params.graph): the chain below is recorded once per set
    // of arguments (items, parameters, launch partition, stream and scratch
    // addresses) with its host tables in pinned memory, and replayed after.
    const bool use_graph = common->graph != 0 && !sl.stream_ordered;
    const bool prof = common->profile != 0 && !use_graph;
    if (prof && (rc = prof_events(ctx, sl, launches.size()))) return rc;
    GraphEntry* ge = nullptr;
    bool capture = false;
    std::string gkey;
    size_t n_tab = 0;  // solve slots over all launches
    for (auto& L : launches) n_tab += (size_t)(L.second - L.first);
    if (use_graph) {
        auto add = [&gkey](const void* v, size_t n) { gkey.append((const char*)v, n); };
        add("batch", 5);
        for (int q = 0; q < n_items; ++q) {
            const Item& I = *it[q];
            const int64_t ip[5] = {I.mode, items[q].grid_id, items[q].opac_id, (int64_t)I.p.n_packets,
                                   (int64_t)I.pl.specs.size()};
            add(ip, sizeof ip);
            add(I.pl.specs.data(), sizeof(int) * I.pl.specs.size());
            add(I.pl.obs.data(), sizeof(double) * I.pl.obs.size());
        }
        const double dpar[10] = {common->rr_threshold, common->rr_survive, common->emis_bias, common->tau_vert_max,
                                 common->tau_peel_max, common->mu0, (double)common->max_events,
                                 common->surface_albedo, common->draine_alpha, 0.0};
        add(dpar, sizeof dpar);
        const int64_t ipar[13] = {(int64_t)common->seed, common->precision, common->decorrelate, common->scattering,
                                  common->absorption, A.ev_threshold, bpc, A.batch, common->cloud_phase,
                                  common->forced, common->forced_first, (int64_t)launches.size(), n_items};
        add(ipar, sizeof ipar);
        add(launches.data(), sizeof(launches[0]) * launches.size());
        const void* ptrs[10] = {st, v_arena, v_sums, v_part, v_solves, v_slots, v_ctr, v_grids, v_ps, nullptr};
        add(ptrs, sizeof ptrs);
        std::lock_guard<std::mutex> gk(ctx->graph_mu);
        auto gi = ctx->graphs.find(gkey);
        if (gi != ctx->graphs.end()) {
            ge = gi->second.get();
        } else {
            if (ctx->graphs.size() >= kMaxGraphs) {  // drop the least recently used
                auto lru = ctx->graphs.begin();
                for (auto q = ctx->graphs.begin(); q != ctx->graphs.end(); ++q)
                    if (q->second->used < lru->second->used) lru = q;
                ctx->graphs.erase(lru);
            }
            std::unique_ptr<GraphEntry> e(new GraphEntry());
            for (int q = 0; q < n_items; ++q) {
                e->gids.push_back(items[q].grid_id);
                e->oids.push_back(items[q].opac_id);
            }
            HIPTRY(hipHostMalloc(&e->pinned, sizeof(GridDev) * grids.size() + (sizeof(SolveDev) + sizeof(PrepSlot)) * n_tab));
            ge = e.get();
            ctx->graphs[gkey] = std::move(e);
            capture = true;
        }
        ge->used = ++ctx->graph_clock;
    }
    // host tables: pinned (graph) or pageable (eager; kept until the end)
    std::vector<GridDev> e_grids;
    std::vector<SolveDev> e_solves;
    std::vector<PrepSlot> e_slots;
    GridDev* t_grids;
    SolveDev* t_solves;
    PrepSlot* t_slots;
    if (use_graph) {
        t_grids = (GridDev*)ge->pinned;
        t_solves = (SolveDev*)(t_grids + grids.size());
        t_slots = (PrepSlot*)(t_solves + n_tab);
    } else {
        e_grids.resize(grids.size());
        e_solves.resize(n_tab);
        e_slots.resize(n_tab);
        t_grids = e_grids.data();
        t_solves = e_solves.data();
        t_slots = e_slots.data();
    }
    for (size_t q = 0; q < grids.size(); ++q) t_grids[q] = hgrids[q];

    auto enqueue = [&]() -> int {
        HIPTRY(hipMemcpyAsync(v_grids, t_grids, sizeof(GridDev) * grids.size(), hipMemcpyHostToDevice, st));
        launch_fill_f64(sums, (size_t)nsolve * row_w, 0.0, st);
        size_t tab0 = 0;
        for (size_t li = 0; li < launches.size(); ++li) {
            const int s0 = launches[li].first, s1 = launches[li].second, nb = s1 - s0;
            SolveDev* hsv = t_solves + tab0;
            PrepSlot* hps = t_slots + tab0;
            tab0 += (size_t)nb;
            char* arena = (char*)v_arena;
            uint64_t begin = 0;
            for (int sg = s0; sg < s1; ++sg) {
                const Flat& F = fl[sg];
                Item& I = *it[F.item];
                const int ncell = I.ls.g->ncell;
                const int b = I.pl.specs[F.spec];
                OpacRes* op = I.ls.op;
                PrepSlot& P = hps[sg - s0];
                P = PrepSlot{};
                P.lnk = op->lnk + ((size_t)b * op->ng + F.g) * op->nT * op->nP;
                P.k_ray = op->k_ray[b];
                P.n = b;
                P.lam_cm = op->lam_um[b] * 1e-4;
                auto take = [&](size_t bytes) {
                    char* r = arena;
                    arena += (bytes + 255) & ~(size_t)255;
                    return r;
                };
                P.opt = (double*)take(sizeof(double) * 5 * (size_t)ncell);
                P.optf = mixed ? (float*)take(sizeof(float) * 5 * (size_t)ncell) : nullptr;
                P.cdf = P.wbirth = nullptr;
                if (I.mode == MCRT_MODE_EMISSION) {
                    P.cdf = (double*)take(sizeof(double) * 2 * (size_t)ncell);
                    P.wbirth = P.cdf + ncell;
                }
                P.stats = sums + (size_t)sg * row_w + pw;
                SolveDev& S = hsv[sg - s0];
                S = SolveDev{};
                S.begin = begin;
                S.pbase = begin;
                S.n = I.p.n_packets;
                begin += S.n;
                S.tag = common->decorrelate ? (uint32_t)(1 + b * I.pl.ng + F.g) : 0u;
                S.mode = I.mode == MCRT_MODE_EMISSION ? 1 : 0;
                S.grid = I.gslot;
                S.cdf = P.cdf;
                S.wbirth = P.wbirth;
                if (mixed) {
                    const float* f = P.optf;
                    S.a_ext = f; S.a_abs = f + ncell; S.omega = f + 2 * (size_t)ncell; S.p_gas = f + 3 * (size_t)ncell;
                    S.g_cld = f + 4 * (size_t)ncell;
                } else {
                    const double* d = P.opt;
                    S.a_ext = d; S.a_abs = d + ncell; S.omega = d + 2 * (size_t)ncell; S.p_gas = d + 3 * (size_t)ncell;
                    S.g_cld = d + 4 * (size_t)ncell;
                }
            }
            double* rows = (double*)arena;  // rows after the optics of the launch
            HIPTRY(hipMemcpyAsync(v_slots, hps, sizeof(PrepSlot) * nb, hipMemcpyHostToDevice, st));
            HIPTRY(hipMemcpyAsync(v_solves, hsv, sizeof(SolveDev) * nb, hipMemcpyHostToDevice, st));
            // preparation per run of consecutive solves of one item (one grid, one table)
            for (int a = s0; a < s1;) {
                int e = a;
                while (e < s1 && fl[e].item == fl[a].item) ++e;
                Item& I = *it[fl[a].item];
                OpacRes* op = I.ls.op;
                const PrepSlot* ps = (const PrepSlot*)v_slots + (a - s0);
                launch_prep_optics(I.ls.g->dev, I.ls.g->ncell, ps, e - a, 0, op->nT, op->nP, op->T_grid, op->lnP_grid,
                                   op->lnk, op->nspec, nullptr, common->cloud_phase == 2 ? 1 : 0,
                                   common->draine_alpha, st);
                if (I.mode == MCRT_MODE_EMISSION)
                    launch_prep_sources(I.ls.g->dev, I.ls.g->ncell, ps, e - a, I.p.tau_vert_max, I.p.emis_bias,
                                        (double*)v_ps, st);
                a = e;
            }
            A.rows = rows;
            A.solves = (const SolveDev*)v_solves;
            A.n_solves = nb;
            A.total = begin;
            launch_init_dispensers(A.counter, A.total, st);
            launch_births(hgrids[0], A, true, st);
            if (prof) HIPTRY(hipEventRecord(sl.prof_ev[2 * li], st));
            launch_transport_persistent(hgrids[0], A, mixed, true, pblocks, bpc, st);
            if (prof) HIPTRY(hipEventRecord(sl.prof_ev[2 * li + 1], st));
            int chunks_l = 1;
            for (int sg = s0; sg < s1; ++sg)
                chunks_l = std::max(chunks_l, reduce_rows_chunks(it[fl[sg].item]->p.n_packets));
            launch_reduce_rows(A, nullptr, nb, (double*)v_part, chunks_l, sums + (size_t)s0 * row_w, row_w, nullptr,
                               st);
            // in eager form the next launch's pageable tables are copied only after
            // this launch ran; stream order alone protects the reused device buffers
            if (!use_graph && li + 1 < launches.size()) HIPTRY(hipStreamSynchronize(st));
        }
        return MCRT_OK;
    };
    if (use_graph) {
        if (capture) {
            HIPTRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            int crc = enqueue();
            hipGraph_t gr = nullptr;
            hipError_t ee = hipStreamEndCapture(st, &gr);
            if (crc == MCRT_OK && ee == hipSuccess) ee = hipGraphInstantiate(&ge->exec, gr, nullptr, nullptr, 0);
            ge->graph = gr;
            if (crc != MCRT_OK || ee != hipSuccess) {
                std::lock_guard<std::mutex> gk(ctx->graph_mu);
                ctx->graphs.erase(gkey);
                if (crc != MCRT_OK) return crc;
                HIPTRY(ee);
            }
        }
        HIPTRY(hipEventRecord(sl.ev0, st));
        HIPTRY(hipGraphLaunch(ge->exec, st));
    } else {
        HIPTRY(hipEventRecord(sl.ev0, st));
        if ((rc = enqueue())) return rc;
    }
    HIPTRY(hipGetLastError());
    std::vector<double> hs((size_t)nsolve * row_w);
    HIPTRY(hipMemcpyAsync(hs.data(), sums, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, st));
    mcrt_result tr{};
    if ((rc = finish_timing(ctx, sl, st, &tr))) return rc;
    if (prof && (rc = prof_collect(ctx, sl, launches.size(), &tr))) return rc;
    if (use_graph) tr.kernel_ms = tr.elapsed_ms;  // the whole replay
    // per item post-processing, as for the single-request solves
    for (int q = 0; q < n_items; ++q) {
        Item& I = *it[q];
        const int ns = (int)I.pl.specs.size(), ng = I.pl.ng, nsq = ns * ng;
        const double Nd = (double)I.p.n_packets;
        std::vector<double> val((size_t)nsq * no), se((size_t)nsq * no), cnt((size_t)nsq * kNCounters), ltot(nsq),
            rows((size_t)nsq * row_w);
        for (int k = 0; k < nsq; ++k) {
            const double* row = hs.data() + (size_t)(I.first + k) * row_w;
            std::copy(row, row + row_w, rows.begin() + (size_t)k * row_w);
            double scale = kPi;
            if (I.mode == MCRT_MODE_EMISSION) {
                ltot[k] = row[pw];
                scale = row[pw] / (I.ls.g->r_toa * I.ls.g->r_toa);
            }
            for (int o = 0; o < no; ++o) {
                double m = row[2 * o] / Nd;
                double var = std::max(row[2 * o + 1] / Nd - m * m, 0.0) / Nd;
                val[(size_t)k * no + o] = scale * m;
                se[(size_t)k * no + o] = scale * std::sqrt(var);
            }
            for (int t = 0; t < kNCounters; ++t) cnt[(size_t)k * kNCounters + t] = row[2 * no + t];
        }
        fill_results(I.pl, val, se, I.ls.op->g_weights, rows, row_w, cnt, ltot, &results[q]);
        results[q].elapsed_ms = tr.elapsed_ms;
        results[q].kernel_ms = tr.kernel_ms;
        results[q].kernel_launches = tr.kernel_launches;
    }
    return MCRT_OK;
}

// ------------------------------------------------------------------ serving
enum { R_QUEUED = 0, R_RUNNING = 1, R_DONE = 2, R_FAILED = 3, R_CANCELLED = 4 };
using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    int mode = 0;
    int32_t gid = 0, oid = 0;
    mcrt_solve_params p{};
    std::vector<int32_t> spec;
    std::vector<double> phase, dir;
    int status = R_QUEUED;
    int rc = MCRT_OK;
    std::string err;
    int ns = 0, ng = 1, no = 1;
    uint64_t est = 0;
    std::vector<double> value, se, per_g, sums, counters, l_tot;
    double elapsed_ms = 0.0, kernel_ms = 0.0;
    int64_t launches = 0;
    int64_t n_segments = 0;
    Clock::time_point t_sub, t_start, t_done;
};

int run_solve(mcrt_ctx* ctx, Slot& sl, hipStream_t st, int mode, int32_t gid, int32_t oid,
              const mcrt_solve_params* p, mcrt_result* res)
{
    if (mode == MCRT_MODE_TRANSMISSION && !p->ms_transmission) return solve_chords(ctx, sl, st, gid, oid, p, res);
    if (mode == MCRT_MODE_ALBEDO || mode == MCRT_MODE_EMISSION || mode == MCRT_MODE_TRANSMISSION)
        return solve_packets(ctx, sl, st, gid, oid, p, res, mode);
    return fail(MCRT_EINVAL, "unknown mode %d", mode);
}

int blocking_solve(mcrt_ctx* ctx, int mode, int32_t gid, int32_t oid, const mcrt_solve_params* p, mcrt_result* res)
{
    std::lock_guard<std::mutex> lk(ctx->main_mu);
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(MCRT_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    return run_solve(ctx, ctx->main, ctx->main.stream, mode, gid, oid, p, res);
}

// Device bytes a request allocates (its scratch), for admission.
uint64_t estimate_bytes(mcrt_ctx* ctx, const Request& r, GridRes* g, OpacRes* op)
{
    const uint64_t ncell = (uint64_t)g->ncell;
    const uint64_t nsolve = (uint64_t)r.ns * r.ng;
    if (r.mode == MCRT_MODE_TRANSMISSION && !r.p.ms_transmission) {
        const uint64_t nch = (uint64_t)r.p.n_b * r.p.n_alpha;
        const uint64_t nrow = nsolve, nslot = std::min<uint64_t>(64, nrow);
        const uint64_t tblocks = (uint64_t)chord_tau_blocks((int)nch);
        const uint64_t segs = nch * (2ULL * g->dev.nlay + 2ULL * g->dev.nlat + g->dev.nlon + 8ULL);
        return nch * (4 + 8 + 8 + 4) + 8 + ncell * nslot * 8 + tblocks * 2 * nslot * 8 + nrow * 16 + ncell * 8 +
               ncell * sizeof(CellTP) + nrow * 4 + segs * 12 + (1ULL << 20);
    }
    const bool mixed = r.p.precision == MCRT_MIXED;
    const uint64_t N = r.p.n_packets;
    const uint64_t no = (uint64_t)r.no;
    const uint64_t pw = 2 * no + kNCounters, row_w = pw + 2, prow = no + kNCounters;
    const uint64_t opt_b = ncell * 5 * (8 + (mixed ? 4 : 0));
    const uint64_t src_b = r.mode == MCRT_MODE_EMISSION ? ncell * 16 : 0;
    const uint64_t row_b = N * prow * 8;
    const uint64_t gsn = r.p.g_sampling ? N / (uint64_t)r.ng + 1 : N;
    uint64_t batch = (uint64_t)serving_batch(ctx, r.p.max_batch, (int)nsolve, opt_b + src_b + row_b, gsn);
    if (r.p.g_sampling) batch = std::max<uint64_t>(r.ng, batch / r.ng * r.ng);  // whole bands, as the solve rounds
    const uint64_t chunks = (uint64_t)reduce_rows_chunks(N);
    uint64_t b = opt_b * batch + row_b * batch + nsolve * row_w * 8 + batch * chunks * pw * 8 +
                 batch * (sizeof(SolveDev) + sizeof(PrepSlot)) + 64;
    if (r.mode == MCRT_MODE_EMISSION) b += src_b * batch + prep_scratch_doubles((int)ncell, (int)batch) * 8;
    if (op->kind == MCRT_OPAC_HIRES) b += ncell * 8;
    return b + (1ULL << 20);
}

void worker_main(mcrt_ctx* ctx, Slot* sl)
{
    (void)hipSetDevice(ctx->device);
    std::unique_lock<std::mutex> lk(ctx->q_mu);
    for (;;) {
        // With no admitted request left, memory held now (grids, tables, the
        // blocking solves' scratch) only shrinks if the caller frees it, so
        // the head of the queue is taken then and fails if it does not fit,
        // rather than blocking every request behind it.
        ctx->q_cv.wait(lk, [&] {
            if (ctx->stopping) return true;
            if (ctx->queue.empty()) return false;
            std::lock_guard<std::mutex> mk(ctx->mem_mu);
            return ctx->reserved == 0 || held_locked(ctx) + ctx->queue.front()->est <= ctx->budget;
        });
        if (ctx->stopping) return;
        Request* r = ctx->queue.front();
        ctx->queue.pop_front();
        bool fits;
        uint64_t held;
        for (int attempt = 0;; ++attempt) {
            {
                std::lock_guard<std::mutex> mk(ctx->mem_mu);
                held = held_locked(ctx);
                fits = held + r->est <= ctx->budget;
                if (fits) ctx->reserved += r->est;
            }
            if (fits || attempt > 0) break;
            lk.unlock();  // the blocking solves' kept scratch gives way, if no blocking solve runs
            const bool freed = reclaim_main(ctx);
            lk.lock();
            if (!freed) break;
        }
        if (!fits) {
            char msg[160];
            std::snprintf(msg, sizeof msg, "request needs %llu bytes of scratch; %llu of the budget of %llu are held",
                          (unsigned long long)r->est, (unsigned long long)held, (unsigned long long)ctx->budget);
            r->rc = MCRT_EBUDGET;
            r->err = msg;
            r->t_start = r->t_done = Clock::now();
            r->status = R_FAILED;
            ctx->q_cv.notify_all();
            continue;
        }
        r->status = R_RUNNING;
        r->t_start = Clock::now();
        ctx->n_running++;
        lk.unlock();
        mcrt_result res{};
        res.value = r->value.data();
        res.stderr_ = r->se.data();
        res.per_g = r->per_g.data();
        res.sums = r->sums.data();
        res.counters = r->counters.data();
        res.l_tot = r->l_tot.data();
        int rc = run_solve(ctx, *sl, sl->stream, r->mode, r->gid, r->oid, &r->p, &res);
        std::string err = rc ? std::string(mcrt_last_error()) : std::string();
        ctx->n_running--;
        release_scratch(ctx, *sl);
        (void)hipStreamSynchronize(sl->stream);
        lk.lock();
        {
            std::lock_guard<std::mutex> mk(ctx->mem_mu);
            ctx->reserved -= r->est;
        }
        r->rc = rc;
        r->err = err;
        r->elapsed_ms = res.elapsed_ms;
        r->kernel_ms = res.kernel_ms;
        r->launches = res.kernel_launches;
        r->n_segments = res.n_segments;
        r->t_done = Clock::now();
        r->status = rc ? R_FAILED : R_DONE;
        ctx->q_cv.notify_all();
    }
}

void stop_workers(mcrt_ctx* ctx)
{
    {
        std::lock_guard<std::mutex> lk(ctx->q_mu);
        ctx->stopping = true;
        for (Request* r : ctx->queue) {
            r->status = R_CANCELLED;
            r->rc = MCRT_ECANCELLED;
        }
        ctx->queue.clear();
        ctx->q_cv.notify_all();
    }
    const bool had_workers = !ctx->workers.empty();
    for (auto& t : ctx->workers) t.join();
    ctx->workers.clear();
    for (auto& sl : ctx->wslots) slot_destroy(ctx, *sl);
    ctx->wslots.clear();
    // hand the memory the workers' pool kept back to the device
    if (had_workers && ctx->pool) {
        (void)hipMemPoolTrimTo(ctx->pool, 0);
        (void)hipMemPoolDestroy(ctx->pool);
        ctx->pool = nullptr;
    }
    (void)hipGetLastError();
}

int submit(mcrt_ctx* ctx, int mode, int32_t gid, int32_t oid, const mcrt_solve_params* p, uint64_t* ticket)
{
    if (mode != MCRT_MODE_ALBEDO && mode != MCRT_MODE_EMISSION && mode != MCRT_MODE_TRANSMISSION)
        return fail(MCRT_EINVAL, "unknown mode %d", mode);
    if (p->contrib || p->image_npix)
        return fail(MCRT_EINVAL, "contribution functions and images are computed by blocking solves only");
    std::unique_ptr<Request> r(new Request());
    r->mode = mode;
    r->gid = gid;
    r->oid = oid;
    r->p = *p;
    r->p.stream = nullptr;
    r->p.packet_dump = nullptr;
    Lease ls;
    int rc = lease(ctx, gid, oid, ls);
    if (rc) return rc;
    SolvePlan pl;
    if ((rc = plan_common(nullptr, ls.g, ls.op, p, mode, pl))) return rc;
    if (p->spec_idx) {
        r->spec.assign(p->spec_idx, p->spec_idx + p->n_spec);
        r->p.spec_idx = r->spec.data();
    }
    if (p->obs_phase && p->n_obs > 0) {
        r->phase.assign(p->obs_phase, p->obs_phase + p->n_obs);
        r->p.obs_phase = r->phase.data();
    }
    if (p->obs_dir && p->n_obs > 0) {
        r->dir.assign(p->obs_dir, p->obs_dir + 3 * p->n_obs);
        r->p.obs_dir = r->dir.data();
    }
    r->ns = (int)pl.specs.size();
    r->ng = pl.ng;
    r->no = pl.n_out;
    const size_t nv = (size_t)r->ns * r->no, ng = (size_t)r->ns * r->ng;
    r->value.assign(nv, 0.0);
    r->se.assign(nv, 0.0);
    r->per_g.assign(ng * r->no, 0.0);
    r->sums.assign(ng * r->no * 2, 0.0);
    r->counters.assign(ng * kNCounters, 0.0);
    r->l_tot.assign(ng, 0.0);
    r->est = estimate_bytes(ctx, *r, ls.g, ls.op);
    bool crowded;
    {
        std::lock_guard<std::mutex> mk(ctx->mem_mu);
        crowded = held_locked(ctx) + r->est > ctx->budget;
    }
    if (crowded) reclaim_main(ctx);  // the blocking solves' kept scratch gives way to served requests
    {
        std::lock_guard<std::mutex> mk(ctx->mem_mu);
        const uint64_t resident = ctx->in_use - ctx->served;  // not freed when running requests end
        if (r->est + resident > ctx->budget)
            return fail(MCRT_EBUDGET, "request needs %llu bytes of scratch; the budget leaves %llu",
                        (unsigned long long)r->est, (unsigned long long)(ctx->budget - std::min(ctx->budget, resident)));
    }
    std::lock_guard<std::mutex> lk(ctx->q_mu);
    if (ctx->stopping) return fail(MCRT_EINVAL, "context is shutting down");
    if (ctx->workers.empty()) {
        // The workers' stream-ordered scratch comes from a memory pool of this
        // context.  It keeps up to the budget's worth of freed memory, so that
        // a request reuses what earlier ones freed instead of having it
        // returned to the device and mapped again at every synchronisation;
        // blocking allocations trim it when in_use plus what it keeps would
        // pass the budget.
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = ctx->device;
        hipMemPool_t pool = nullptr;
        if (hipMemPoolCreate(&pool, &props) != hipSuccess || !pool) {
            (void)hipGetLastError();
            return fail(MCRT_EDEVICE, "hipMemPoolCreate failed");
        }
        uint64_t keep = ctx->budget;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        {
            std::lock_guard<std::mutex> mk(ctx->mem_mu);
            ctx->pool = pool;
        }
        for (int w = 0; w < ctx->n_workers; ++w) {
            std::unique_ptr<Slot> sl(new Slot());
            if ((rc = slot_init(*sl, true, ctx->n_cu))) return rc;
            sl->stream_ordered = true;
            ctx->wslots.push_back(std::move(sl));
        }
        for (int w = 0; w < ctx->n_workers; ++w) ctx->workers.emplace_back(worker_main, ctx, ctx->wslots[w].get());
    }
    r->ticket = ctx->next_ticket++;
    r->t_sub = Clock::now();
    *ticket = r->ticket;
    ctx->queue.push_back(r.get());
    ctx->requests[r->ticket] = std::move(r);
    ctx->q_cv.notify_all();
    return MCRT_OK;
}

int wait_request(mcrt_ctx* ctx, uint64_t ticket, mcrt_result* out)
{
    std::unique_lock<std::mutex> lk(ctx->q_mu);
    auto it = ctx->requests.find(ticket);
    if (it == ctx->requests.end()) return fail(MCRT_ENOTFOUND, "ticket %llu not found", (unsigned long long)ticket);
    Request* r = it->second.get();
    ctx->q_cv.wait(lk, [&] { return r->status >= R_DONE; });
    int rc = r->rc;
    if (rc == MCRT_OK && out) {
        if (out->value) std::copy(r->value.begin(), r->value.end(), out->value);
        if (out->stderr_) std::copy(r->se.begin(), r->se.end(), out->stderr_);
        if (out->per_g) std::copy(r->per_g.begin(), r->per_g.end(), out->per_g);
        if (out->sums) std::copy(r->sums.begin(), r->sums.end(), out->sums);
        if (out->counters) std::copy(r->counters.begin(), r->counters.end(), out->counters);
        if (out->l_tot) std::copy(r->l_tot.begin(), r->l_tot.end(), out->l_tot);
        out->elapsed_ms = r->elapsed_ms;
        out->kernel_ms = r->kernel_ms;
        out->kernel_launches = r->launches;
        out->n_segments = r->n_segments;
        out->queued_ms = std::chrono::duration<double, std::milli>(r->t_start - r->t_sub).count();
        out->latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_sub).count();
    }
    std::string err = r->err;
    ctx->requests.erase(it);
    if (rc) g_err = err;
    return rc;
}

int grid_upload(mcrt_ctx* ctx, const mcrt_grid_desc* d, hipStream_t st, int32_t* grid_id)
{
    int rc = validate_grid(d);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->poisoned) return fail(MCRT_EDEVICE, "context is unusable after an earlier device error");
    HIPTRY(hipSetDevice(ctx->device));
    const bool slab = d->geometry == MCRT_PLANE_PARALLEL;
    const int nlon = d->nlon, nlat = d->nlat, nlay = d->nlay;
    const size_t n = (size_t)nlon * nlat * nlay;
    const bool borrow = (d->flags & MCRT_BORROW_DEVICE) != 0;
    if (borrow && (rc = check_borrowed(ctx, d, n, st))) return rc;
    // host-side edge tables
    std::vector<double> lat(nlat + 1), lon(nlon + 1);
    if (slab) {
        lat = {-kPi / 2, kPi / 2};
        lon = {-kPi, kPi};
    } else {
        std::copy(d->lat_edges, d->lat_edges + nlat + 1, lat.begin());
        std::copy(d->lon_edges, d->lon_edges + nlon + 1, lon.begin());
    }
    std::vector<double> lc2(nlat + 1), ls2(nlat + 1), lsn(nlat + 1), los(nlon), loc(nlon), volr(nlay);
    for (int e = 0; e <= nlat; ++e) {
        double c = std::cos(lat[e]), s = std::sin(lat[e]);
        lc2[e] = c * c;
        ls2[e] = s * s;
        lsn[e] = s;
    }
    for (int e = 0; e < nlon; ++e) {
        los[e] = std::sin(lon[e]);
        loc[e] = std::cos(lon[e]);
    }
    for (int k = 0; k < nlay; ++k)
        volr[k] = (std::pow(d->r_edges[k + 1], 3.0) - std::pow(d->r_edges[k], 3.0)) / 3.0;

    std::unique_ptr<GridRes> G(new GridRes());
    GridDev& gd = G->dev;
    gd.geom = slab ? 1 : 0;
    gd.nlon = nlon;
    gd.nlat = nlat;
    gd.nlay = nlay;
    gd.max_cross = 4 * (nlay + nlat + nlon) + 16;
    gd.omega_rot = d->omega_rot;
    auto cleanup = [&](int code) {
        (void)hipStreamSynchronize(st);
        for (auto& b : G->bufs) dev_free(ctx, b);
        return code;
    };
    double* dp;
    float* fp;
#define UP(field, host, cnt, ptr)                                            \
    do {                                                                     \
        int _r = upload(ctx, G->bufs, G->bytes, host, cnt, &ptr, st);            \
        if (_r) return cleanup(_r);                                          \
        gd.field = ptr;                                                      \
    } while (0)
    UP(r, d->r_edges, (size_t)nlay + 1, dp);
    UP(lat, lat.data(), lat.size(), dp);
    UP(lat_c2, lc2.data(), lc2.size(), dp);
    UP(lat_s2, ls2.data(), ls2.size(), dp);
    UP(lat_sin, lsn.data(), lsn.size(), dp);
    UP(lon, lon.data(), lon.size(), dp);
    UP(lon_s, los.data(), los.size(), dp);
    UP(lon_c, loc.data(), loc.size(), dp);
    UP(vol_r, volr.data(), volr.size(), dp);
    std::vector<double> faces;
    faces.reserve((size_t)nlay + 1 + 3 * ((size_t)nlat + 1) + 2 * (size_t)nlon);
    faces.insert(faces.end(), d->r_edges, d->r_edges + nlay + 1);
    gd.lat_base = (int)faces.size();
    for (int e = 0; e <= nlat; ++e) faces.insert(faces.end(), {lat[e], ls2[e], lc2[e]});
    gd.lon_base = (int)faces.size();
    for (int e = 0; e < nlon; ++e) faces.insert(faces.end(), {los[e], loc[e]});
    UP(faces, faces.data(), faces.size(), dp);
    if (borrow) {  // read in place; the caller owns them
        gd.T = d->T;
        gd.P = d->P;
        gd.rho = d->rho;
        gd.u = d->u;
        gd.v = d->v;
        gd.w = d->w;
        gd.cld_ksca = d->cld_ksca;
        gd.cld_kabs = d->cld_kabs;
        gd.cld_g = d->cld_g;
    } else {
        UP(T, d->T, n, fp);
        UP(P, d->P, n, fp);
        UP(rho, d->rho, n, dp);
        if (d->u) UP(u, d->u, n, fp);
        if (d->v) UP(v, d->v, n, fp);
        if (d->w) UP(w, d->w, n, fp);
        if (d->cld_ksca) {
            UP(cld_ksca, d->cld_ksca, n, fp);
            UP(cld_kabs, d->cld_kabs, n, fp);
            UP(cld_g, d->cld_g, n, fp);
        }
    }
#undef UP
    // the host arrays (and the edge tables above) are read before return
    if (hipError_t e = hipStreamSynchronize(st)) return cleanup(hip_check(ctx, e, "hipStreamSynchronize"));
    G->ncell = (int)n;
    G->r0 = d->r_edges[0];
    G->r_toa = d->r_edges[nlay];
    int32_t id = ctx->next_grid++;
    ctx->grids[id] = std::move(G);
    *grid_id = id;
    return MCRT_OK;
}


int opacity_upload(mcrt_ctx* ctx, const mcrt_opacity_desc* d, hipStream_t st, int32_t* opac_id)
{
    int rc = validate_opacity(d);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->poisoned) return fail(MCRT_EDEVICE, "context is unusable after an earlier device error");
    HIPTRY(hipSetDevice(ctx->device));
    std::unique_ptr<OpacRes> O(new OpacRes());
    O->kind = d->kind;
    O->nspec = d->nspec;
    O->ng = d->ng;
    O->nT = d->nT;
    O->nP = d->nP;
    O->lam_min = d->lam_min_um;
    O->dlnlam = d->dlnlam;
    O->k_ray.assign(d->k_ray, d->k_ray + d->nspec);
    if (d->kind == MCRT_OPAC_CK) {
        O->lam_um.assign(d->lam_um, d->lam_um + d->nspec);
        O->g_weights.assign(d->g_weights, d->g_weights + d->ng);
    } else {
        O->g_weights = {1.0};
    }
    const size_t nTP = (size_t)d->nT * d->nP;
    const size_t ntab = (size_t)d->nspec * d->ng * nTP;
    std::vector<double> lnk(ntab);
    if (d->kind == MCRT_OPAC_CK) {
        for (size_t i = 0; i < ntab; ++i) lnk[i] = d->kappa[i] > 0.0f ? std::log((double)d->kappa[i]) : -INFINITY;
    } else {
        // [lam][T][P] -> [T][P][lam]: consecutive wavelengths are contiguous
        const size_t nl = (size_t)d->nspec;
        for (size_t l = 0; l < nl; ++l)
            for (size_t tp = 0; tp < nTP; ++tp) {
                float kv = d->kappa[l * nTP + tp];
                lnk[tp * nl + l] = kv > 0.0f ? std::log((double)kv) : -INFINITY;
            }
    }
    std::vector<double> lnP(d->nP);
    for (int q = 0; q < d->nP; ++q) lnP[q] = std::log(d->P_grid[q]);
    auto cleanup = [&](int code) {
        (void)hipStreamSynchronize(st);
        for (auto& b : O->bufs) dev_free(ctx, b);
        return code;
    };
    if ((rc = upload(ctx, O->bufs, O->bytes, lnk.data(), lnk.size(), &O->lnk, st))) return cleanup(rc);
    std::vector<float> lnk32;
    if (d->kind == MCRT_OPAC_HIRES) {
        // the mixed form rounds every table value to FP32 before use; ln of
        // an FP32 kappa is finite (|ln| < 104) or -inf, so the copy keeps the
        // zero-kappa corners
        lnk32.resize(ntab);
        for (size_t i = 0; i < ntab; ++i) lnk32[i] = (float)lnk[i];
        if ((rc = upload(ctx, O->bufs, O->bytes, lnk32.data(), lnk32.size(), &O->lnk_f32, st))) return cleanup(rc);
    }
    if ((rc = upload(ctx, O->bufs, O->bytes, d->T_grid, (size_t)d->nT, &O->T_grid, st))) return cleanup(rc);
    if ((rc = upload(ctx, O->bufs, O->bytes, lnP.data(), lnP.size(), &O->lnP_grid, st))) return cleanup(rc);
    if ((rc = upload(ctx, O->bufs, O->bytes, d->k_ray, (size_t)d->nspec, &O->k_ray_dev, st))) return cleanup(rc);
    if ((rc = upload(ctx, O->bufs, O->bytes, O->g_weights.data(), O->g_weights.size(), &O->gw_dev, st)))
        return cleanup(rc);
    // the staged host tables are read before return
    if (hipError_t e = hipStreamSynchronize(st)) return cleanup(hip_check(ctx, e, "hipStreamSynchronize"));
    int32_t id = ctx->next_opac++;
    ctx->opacs[id] = std::move(O);
    *opac_id = id;
    return MCRT_OK;
}

}  // namespace

extern "C" {

const char* mcrt_last_error(void) { return g_err.c_str(); }

int mcrt_create(int device, uint64_t hbm_budget_bytes, mcrt_ctx** out)
{
    if (!out) return fail(MCRT_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) return fail(MCRT_EDEVICE, "no HIP device available");
    if (device < 0 || device >= ndev) return fail(MCRT_EINVAL, "device %d out of range (have %d)", device, ndev);
    std::unique_ptr<mcrt_ctx> ctx(new mcrt_ctx());
    ctx->device = device;
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(MCRT_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    size_t fr = 0, tot = 0;
    e = hipMemGetInfo(&fr, &tot);
    if (e != hipSuccess) return fail(MCRT_EDEVICE, "hipMemGetInfo: %s", hipGetErrorString(e));
    ctx->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)fr);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->n_cu = prop.multiProcessorCount;
    int rc = slot_init(ctx->main);
    if (rc) return rc;
    if ((rc = slot_init(ctx->na))) return rc;
    if (device < kNoallocDevices) {
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        if (!g_noalloc_ptr[device]) {
            void* ptr = nullptr;
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return fail(MCRT_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            g_noalloc_ptr[device] = ptr;
        }
        ctx->na.arena = (char*)g_noalloc_ptr[device];
        ctx->na.arena_cap = kNoallocBytes;
    }
    *out = ctx.release();
    return MCRT_OK;
}

void mcrt_destroy(mcrt_ctx* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    stop_workers(ctx);
    drop_graphs(ctx, 0, 0);
    slot_destroy(ctx, ctx->main);
    slot_destroy(ctx, ctx->na);
    for (auto& kv : ctx->grids)
        for (auto& b : kv.second->bufs) dev_free(ctx, b);
    for (auto& kv : ctx->opacs)
        for (auto& b : kv.second->bufs) dev_free(ctx, b);
    delete ctx;
}

uint64_t mcrt_memory_in_use(const mcrt_ctx* ctx)
{
    if (!ctx) return 0;
    std::lock_guard<std::mutex> lk(ctx->mem_mu);
    return ctx->in_use;
}

int mcrt_serve_config(mcrt_ctx* ctx, int32_t n_workers)
{
    if (!ctx) return fail(MCRT_EINVAL, "ctx is NULL");
    if (n_workers < 1 || n_workers > 16) return fail(MCRT_EINVAL, "n_workers must be in [1, 16]");
    std::lock_guard<std::mutex> lk(ctx->q_mu);
    if (!ctx->workers.empty()) return fail(MCRT_EBUSY, "workers already started");
    ctx->n_workers = n_workers;
    return MCRT_OK;
}

int mcrt_submit(mcrt_ctx* ctx, int32_t mode, int32_t grid_id, int32_t opac_id, const mcrt_solve_params* params,
                uint64_t* ticket)
{
    if (!ctx || !params || !ticket) return fail(MCRT_EINVAL, "ctx, params and ticket are required");
    return submit(ctx, mode, grid_id, opac_id, params, ticket);
}

int mcrt_poll(mcrt_ctx* ctx, uint64_t ticket, int32_t* done)
{
    if (!ctx || !done) return fail(MCRT_EINVAL, "ctx and done are required");
    std::lock_guard<std::mutex> lk(ctx->q_mu);
    auto it = ctx->requests.find(ticket);
    if (it == ctx->requests.end()) return fail(MCRT_ENOTFOUND, "ticket %llu not found", (unsigned long long)ticket);
    *done = it->second->status >= R_DONE ? 1 : 0;
    return MCRT_OK;
}

int mcrt_wait(mcrt_ctx* ctx, uint64_t ticket, mcrt_result* result)
{
    if (!ctx) return fail(MCRT_EINVAL, "ctx is NULL");
    return wait_request(ctx, ticket, result);
}

int mcrt_cancel(mcrt_ctx* ctx, uint64_t ticket)
{
    if (!ctx) return fail(MCRT_EINVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->q_mu);
    auto it = ctx->requests.find(ticket);
    if (it == ctx->requests.end()) return fail(MCRT_ENOTFOUND, "ticket %llu not found", (unsigned long long)ticket);
    Request* r = it->second.get();
    if (r->status == R_QUEUED) {
        for (auto q = ctx->queue.begin(); q != ctx->queue.end(); ++q)
            if (*q == r) {
                ctx->queue.erase(q);
                break;
            }
        r->status = R_CANCELLED;
        r->rc = MCRT_ECANCELLED;
        r->err = "request was cancelled";
        ctx->q_cv.notify_all();
        return MCRT_OK;
    }
    if (r->status == R_RUNNING) return fail(MCRT_EBUSY, "request %llu is already running", (unsigned long long)ticket);
    return MCRT_OK;  // already finished: nothing to cancel
}

void mcrt_default_params(mcrt_solve_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->seed = 211015640ULL;
    p->n_packets = 100000;
    p->precision = MCRT_FP64;
    p->scattering = 1;
    p->absorption = MCRT_SURVIVAL;
    p->rr_threshold = 1e-3;
    p->rr_survive = 0.1;
    p->emis_bias = 0.5;
    p->tau_vert_max = 30.0;
    p->tau_peel_max = 50.0;
    p->max_events = 1000000;
    p->mu0 = 0.0;
    p->n_b = 256;
    p->n_alpha = 360;
    p->r_star = 6.957e10;
    p->draine_alpha = 0.5;
}

int mcrt_grid_upload(mcrt_ctx* ctx, const mcrt_grid_desc* d, void* stream, int32_t* grid_id)
{
    if (!ctx || !grid_id) return fail(MCRT_EINVAL, "ctx and grid_id are required");
    int rc = grid_upload(ctx, d, (hipStream_t)stream, grid_id);
    if (rc == MCRT_EBUDGET && reclaim_main(ctx)) rc = grid_upload(ctx, d, (hipStream_t)stream, grid_id);
    return rc;
}

int mcrt_grid_free(mcrt_ctx* ctx, int32_t grid_id)
{
    if (!ctx) return fail(MCRT_EINVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->grids.find(grid_id);
    if (it == ctx->grids.end()) return fail(MCRT_ENOTFOUND, "grid %d not found", grid_id);
    if (it->second->refs > 0) return fail(MCRT_EBUSY, "grid %d is in use by a running solve", grid_id);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->main.stream);
    drop_graphs(ctx, grid_id, 0);
    for (auto& b : it->second->bufs) dev_free(ctx, b);
    ctx->grids.erase(it);
    return MCRT_OK;
}

int mcrt_opacity_upload(mcrt_ctx* ctx, const mcrt_opacity_desc* d, void* stream, int32_t* opac_id)
{
    if (!ctx || !opac_id) return fail(MCRT_EINVAL, "ctx and opac_id are required");
    int rc = opacity_upload(ctx, d, (hipStream_t)stream, opac_id);
    if (rc == MCRT_EBUDGET && reclaim_main(ctx)) rc = opacity_upload(ctx, d, (hipStream_t)stream, opac_id);
    return rc;
}

int mcrt_opacity_free(mcrt_ctx* ctx, int32_t opac_id)
{
    if (!ctx) return fail(MCRT_EINVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->opacs.find(opac_id);
    if (it == ctx->opacs.end()) return fail(MCRT_ENOTFOUND, "opacity %d not found", opac_id);
    if (it->second->refs > 0) return fail(MCRT_EBUSY, "opacity %d is in use by a running solve", opac_id);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->main.stream);
    drop_graphs(ctx, 0, opac_id);
    for (auto& b : it->second->bufs) dev_free(ctx, b);
    ctx->opacs.erase(it);
    return MCRT_OK;
}

int mcrt_autotune(mcrt_ctx* ctx, int32_t mode, int32_t grid_id, int32_t opac_id, mcrt_solve_params* params,
                  double* best_packets_per_s)
{
    if (!ctx || !params) return fail(MCRT_EINVAL, "ctx and params are required");
    if (mode != MCRT_MODE_ALBEDO && mode != MCRT_MODE_EMISSION)
        return fail(MCRT_EINVAL, "autotuning applies to the packet transport (albedo, emission)");
    // trial: up to 4 spectral points spread over the request with the
    // request's packet count (at most 1e6) each, all in one batch, so that
    // the end-of-launch tail weighs about as much as in the real launches
    std::vector<int32_t> all;
    int ng = 1;  // solves per spectral point (the g-ordinates, unless sampled per packet)
    {
        Lease ls;
        int rc = lease(ctx, grid_id, opac_id, ls);
        if (rc) return rc;
        if (params->spec_idx && params->n_spec > 0) all.assign(params->spec_idx, params->spec_idx + params->n_spec);
        else
            for (int q = 0; q < ls.op->nspec; ++q) all.push_back(q);
        if (ls.op->kind == MCRT_OPAC_CK && !params->g_sampling) ng = ls.op->ng;
    }
    std::vector<int32_t> spec;
    const int nt = std::min<int>(4, (int)all.size());
    for (int q = 0; q < nt; ++q) spec.push_back(all[(size_t)q * all.size() / nt]);
    mcrt_solve_params t = *params;
    t.spec_idx = spec.data();
    t.n_spec = (int32_t)spec.size();
    t.n_packets = std::min<uint64_t>(params->n_packets, 1000000);
    t.max_batch = 0;
    t.packet_dump = nullptr;
    t.profile = 0;
    t.graph = 0;
    t.contrib = 0;
    t.image_npix = 0;
    const int evs[4] = {20, 24, 28, 32}, bpcs[2] = {3, 4}, wbs[2] = {32, 128};
    double best = -1.0;
    int be = evs[0], bb = bpcs[0], bw = wbs[0];
    std::vector<double> v(64 * 8), e(64 * 8);
    mcrt_result r{};
    r.value = v.data();
    r.stderr_ = e.data();
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) {
                t.tune_ev_threshold = evs[a];
                t.tune_blocks_per_cu = bpcs[b];
                t.tune_wave_batch = wbs[c];
                if (v.size() < (size_t)t.n_spec * std::max(1, t.n_obs)) {
                    v.resize((size_t)t.n_spec * std::max(1, t.n_obs));
                    e.resize(v.size());
                    r.value = v.data();
                    r.stderr_ = e.data();
                }
                int rc = blocking_solve(ctx, mode, grid_id, opac_id, &t, &r);
                if (rc) return rc;
                double rate = (double)t.n_packets * t.n_spec * ng / std::max(r.elapsed_ms, 1e-3) * 1e3;
                if (rate > best) {
                    best = rate;
                    be = evs[a];
                    bb = bpcs[b];
                    bw = wbs[c];
                }
            }
    params->tune_ev_threshold = be;
    params->tune_blocks_per_cu = bb;
    params->tune_wave_batch = bw;
    if (best_packets_per_s) *best_packets_per_s = best;
    return MCRT_OK;
}

int mcrt_solve_batch(mcrt_ctx* ctx, int32_t n_items, const mcrt_batch_item* items, const mcrt_solve_params* params,
                     mcrt_result* results)
{
    if (!ctx) return fail(MCRT_EINVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->main_mu);
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(MCRT_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    return solve_batch(ctx, ctx->main, ctx->main.stream, n_items, items, params, results);
}

int mcrt_solve_albedo(mcrt_ctx* ctx, int32_t grid_id, int32_t opac_id, const mcrt_solve_params* params,
                      mcrt_result* result)
{
    if (!ctx) return fail(MCRT_EINVAL, "ctx is NULL");
    return blocking_solve(ctx, MCRT_MODE_ALBEDO, grid_id, opac_id, params, result);
}

int mcrt_solve_emission(mcrt_ctx* ctx, int32_t grid_id, int32_t opac_id, const mcrt_solve_params* params,
                        mcrt_result* result)
{
    if (!ctx) return fail(MCRT_EINVAL, "ctx is NULL");
    return blocking_solve(ctx, MCRT_MODE_EMISSION, grid_id, opac_id, params, result);
}

int mcrt_solve_transmission(mcrt_ctx* ctx, int32_t grid_id, int32_t opac_id, const mcrt_solve_params* params,
                            mcrt_result* result)
{
    if (!ctx) return fail(MCRT_EINVAL, "ctx is NULL");
    return blocking_solve(ctx, MCRT_MODE_TRANSMISSION, grid_id, opac_id, params, result);
}

int mcrt_solve_noalloc(mcrt_ctx* ctx, int32_t mode, int32_t grid_id, int32_t opac_id,
                       const mcrt_solve_params* params, mcrt_result* result)
{
    if (!ctx) return fail(MCRT_EINVAL, "ctx is NULL");
    if (mode != MCRT_MODE_ALBEDO && mode != MCRT_MODE_EMISSION)
        return fail(MCRT_EINVAL, "the allocation-free solve takes MCRT_MODE_ALBEDO or MCRT_MODE_EMISSION");
    if (!params) return fail(MCRT_EINVAL, "params is NULL");
    if (params->graph) return fail(MCRT_EINVAL, "graph (recorded solves keep pinned host tables) is not available "
                                                "to the allocation-free solve");
    if (!ctx->na.arena) return fail(MCRT_EINVAL, "device %d has no fixed scratch", ctx->device);
    std::lock_guard<std::mutex> lk(g_noalloc_run[ctx->device]);
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(MCRT_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    ctx->na.arena_off = 0;
    return solve_packets(ctx, ctx->na, ctx->na.stream, grid_id, opac_id, params, result, mode);
}

}  // extern "C"
