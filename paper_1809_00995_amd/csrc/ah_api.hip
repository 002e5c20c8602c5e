// ah_api.hip -- host side of the C ABI declared in include/ah.h: parameter
// validation, the context's device scratch, the launch sequence of each entry
// point, graph capture of step sequences, and the autotuner.  All GPU work of
// a context is ordered on its stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ah.h"
#include "ah_device.hpp"
#include "k_common.hpp"
#include "k_measure.hpp"
#include "k_step_plain.hpp"
#include "k_step_tiled_launch.hpp"
#include "k_step_tiled2_api.hpp"

using namespace ah;

struct ah_ctx {
    int nreal = 0;
    int prec = AH_FP64;
    int layout = AH_LAYOUT_15;
    int zh = 0;                       // z_halo of every realization
    hipStream_t stream = nullptr;
    std::vector<ah_params> p;
    std::vector<int64_t> step;        // host mirror of each realization's step index
    std::vector<int32_t> copy;        // host mirror of the copy holding its state
    RealDesc *d_desc = nullptr;
    int64_t *d_step = nullptr;
    int32_t *d_copy = nullptr;
    Coef *d_coef = nullptr;           // [2][nreal]: steps n and n+1 of a pass
    Slot *d_slots = nullptr;          // measurement slots
    ah_obs *d_obs = nullptr;
    int64_t slot_cap = 0;             // slots allocated, in states (x nreal)
    unsigned long long *d_gauss = nullptr;  // [nreal][2]
    // launch configuration
    int kernel = AH_KERNEL_AUTO;
    int tile_y = 0;                   // 0: default
    std::vector<int> cz;              // per-realization z-chunk, 0: default
    int tile_y2 = 0;                  // the same for the two-step kernel
    std::vector<int> cz2;
    int batched = 0;                  // 1: one persistent launch per step
    int graph_steps = 0;              // > 0: replay runs of unmeasured steps from a graph
    // batched work lists (rebuilt when the configuration changes): single-step
    // tiles and two-step tiles
    BatchItem *d_items = nullptr;
    int n_items = 0, items_ty = 0, grid_step = 0, grid_meas = 0;
    bool items_valid = false;
    BatchItem *d_items2 = nullptr;
    int n_items2 = 0, items2_ty = 0, grid2 = 0;
    bool items2_off32 = false, items2_valid = false;
    BatchItem *d_items_m = nullptr;   // the read-only measuring pass
    int n_items_m = 0, grid_m = 0;
    bool items_m_valid = false, items_m_off32 = false;
    // graph replay
    hipStream_t gstream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool gexec_valid = false;
    std::string err;
};

namespace {

thread_local std::string g_init_err;

int fail(ah_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c)
        c->err = buf;
    else
        g_init_err = buf;
    return code;
}

#define HIP_TRY(ctx, call)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), AH_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));     \
    } while (0)

#define TRY(x)                 \
    do {                       \
        int rc_ = (x);         \
        if (rc_ != AH_OK)      \
            return rc_;        \
    } while (0)

int grid_for(int64_t n, int threads, int cap) {
    int64_t b = (n + threads - 1) / threads;
    return (int)(b < cap ? (b < 1 ? 1 : b) : cap);
}

// Stored sites per plane: nx*ny*nz, plus the halo planes of a slab.
int64_t sites_of(const ah_params &q) { return (int64_t)q.nx * q.ny * (q.nz + 2 * q.z_halo); }

// Device description of realization q stored at `planes`.
RealDesc make_desc(const ah_params &q, void *planes) {
    RealDesc d;
    d.base = (char *)planes;
    d.nx = q.nx;
    d.ny = q.ny;
    d.nz = q.nz;
    d.elem = q.precision == AH_FP64 ? 8 : 4;
    d.layout = q.layout;
    d.zh = q.z_halo;
    d.N = sites_of(q);
    d.dx = q.dx;
    d.dt = q.dt;
    d.tau0 = q.tau0;
    d.tau_ref = q.tau_ref;
    d.era_p = q.era_p;
    d.s = q.s;
    d.lambda0 = q.lambda0;
    d.e0 = q.e0;
    d.sigma = q.sigma;
    d.step0 = q.step0;
    d.n_end = q.n_end;
    d.s_late = q.s_late;
    d.tau_s = q.tau_s;
    return d;
}

double scale_factor_host(const ah_params &p, double tau) {
    double t = tau > 0.0 ? tau : 0.0;
    return std::pow(t / p.tau_ref, p.era_p);
}

int validate(const ah_params &q, int r, const ah_buffers &b, int prec, int layout) {
    auto bad = [&](int code, const char *what) {
        return fail(nullptr, code, "realization %d: %s", r, what);
    };
    if (q.nx < 4 || q.ny < 4 || q.nz < 4)
        return bad(AH_E_INVALID, "extents must be >= 4");
    if (q.z_halo < 0 || q.z_halo > 2 || q.reserved != 0)
        return bad(AH_E_INVALID, "z_halo must be 0, 1 or 2 and reserved 0");
    if (sites_of(q) >= (int64_t)1 << 31)
        return bad(AH_E_INVALID, "nx*ny*(nz + 2 z_halo) must be < 2^31");
    if (q.z_halo > 0 && q.nx % 64 != 0)
        return bad(AH_E_INVALID, "a slab (z_halo > 0) needs the tiled kernels: nx % 64 == 0");
    if (q.z_halo > 0 && q.init != AH_INIT_NONE && q.init != AH_INIT_VACUUM)
        return bad(AH_E_INVALID, "a slab (z_halo > 0) takes AH_INIT_NONE or AH_INIT_VACUUM");
    if (q.precision != prec)
        return bad(AH_E_INVALID, "all realizations must share one precision");
    if (q.precision != AH_FP64 && q.precision != AH_FP32)
        return bad(AH_E_INVALID, "precision must be AH_FP64 or AH_FP32");
    if (!(q.dx > 0.0) || !(q.dt > 0.0) || !std::isfinite(q.dx) || !std::isfinite(q.dt))
        return bad(AH_E_INVALID, "dx and dt must be positive and finite");
    if (!(q.dt / q.dx < 1.0 / std::sqrt(3.0)))
        return bad(AH_E_DOMAIN, "CFL condition dt/dx < 1/sqrt(3) violated");
    if (!(q.s >= -4.0 && q.s <= 1.0))
        return bad(AH_E_DOMAIN, "s must lie in [-4, 1]");
    if (!std::isfinite(q.tau_s) || (q.tau_s > 0.0 && !(q.s_late >= -4.0 && q.s_late <= 1.0)))
        return bad(AH_E_DOMAIN, "s_late must lie in [-4, 1] and tau_s be finite");
    const bool growth = q.s < 0.0 || (q.tau_s > 0.0 && q.s_late < 0.0);
    if (growth && !(scale_factor_host(q, q.tau0 + (double)q.step0 * q.dt) > 0.0))
        return bad(AH_E_DOMAIN, "s < 0 needs a(tau_step0) > 0");
    if (!(q.era_p >= 0.0) || !std::isfinite(q.era_p))
        return bad(AH_E_DOMAIN, "era_p must be >= 0");
    if (!(q.tau_ref > 0.0) || !std::isfinite(q.tau_ref) || !std::isfinite(q.tau0))
        return bad(AH_E_DOMAIN, "tau_ref must be > 0 and tau0 finite");
    if (!(q.lambda0 >= 0.0) || !(q.e0 > 0.0) || !(q.sigma > 0.0))
        return bad(AH_E_DOMAIN, "need lambda0 >= 0, e0 > 0, sigma > 0");
    if (q.init < AH_INIT_RANDOM_PHASE || q.init > AH_INIT_NONE)
        return bad(AH_E_INVALID, "bad init kind");
    if (q.layout != AH_LAYOUT_15 && q.layout != AH_LAYOUT_20)
        return bad(AH_E_INVALID, "layout must be AH_LAYOUT_15 or AH_LAYOUT_20");
    if (q.layout != layout)
        return bad(AH_E_INVALID, "all realizations must share one layout");
    if (q.n_end < 0 || (q.n_end > 0 && q.n_end < q.step0))
        return bad(AH_E_INVALID, "n_end must be 0 or >= step0");
    double tau_half = q.tau0 + ((double)q.step0 + 0.5) * q.dt;
    if (!(scale_factor_host(q, tau_half) > 0.0))
        return bad(AH_E_DOMAIN, "a(tau_{step0+1/2}) must be > 0");
    if (!b.planes)
        return bad(AH_E_INVALID, "NULL planes pointer");
    if (((uintptr_t)b.planes & 255u) != 0)
        return bad(AH_E_INVALID, "planes must be 256-byte aligned");
    return AH_OK;
}

bool frozen(const ah_ctx *c, int r) {
    return c->p[r].n_end > 0 && c->step[r] >= c->p[r].n_end;
}

void invalidate_plans(ah_ctx *c) {
    c->items_valid = false;
    c->items2_valid = false;
    c->items_m_valid = false;
    if (c->gexec)
        (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->gexec_valid = false;
}

// Measurement slots for at least `states` measured states of every realization.
// The context starts with kMinSlotStates (ah_init), so calls that measure up to
// that many states never allocate; beyond it the capacity at least doubles.
constexpr int64_t kMinSlotStates = 64;

int ensure_slots(ah_ctx *c, int64_t states) {
    if (states <= c->slot_cap)
        return AH_OK;
    states = std::max(states, std::max(2 * c->slot_cap, kMinSlotStates));
    if (c->d_slots)
        (void)hipFree(c->d_slots);
    if (c->d_obs)
        (void)hipFree(c->d_obs);
    c->d_slots = nullptr;
    c->d_obs = nullptr;
    c->slot_cap = 0;
    size_t n = (size_t)states * c->nreal;
    HIP_TRY(c, hipMalloc(&c->d_slots, n * sizeof(Slot)));
    HIP_TRY(c, hipMalloc(&c->d_obs, n * sizeof(ah_obs)));
    c->slot_cap = states;
    return AH_OK;
}

int launch_zero(ah_ctx *c, void *p, size_t bytes) {
    int64_t words = (int64_t)(bytes / 8);
    hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(words, 256, 1024)), dim3(256), 0, c->stream,
                       (unsigned long long *)p, words);
    HIP_TRY(c, hipGetLastError());
    return AH_OK;
}

// steps = 0: coefficients of the current state; 1 or 2: of the next pass
// (one or two steps), advancing the device counters.
int launch_bookkeep(ah_ctx *c, int steps) {
    hipLaunchKernelGGL(k_bookkeep, dim3((c->nreal + 63) / 64), dim3(64), 0, c->stream, c->d_desc,
                       c->d_step, c->d_copy, c->d_coef, c->nreal, steps);
    HIP_TRY(c, hipGetLastError());
    return AH_OK;
}

bool tiled_ok(const ah_ctx *c) {
    for (const auto &q : c->p)
        if (q.nx % 64 != 0)
            return false;
    return true;
}

bool use_tiled(const ah_ctx *c, int r) {
    return c->kernel == AH_KERNEL_TILED || c->kernel == AH_KERNEL_TILED2 ||
           (c->kernel == AH_KERNEL_AUTO && c->p[r].nx % 64 == 0);
}

// Unmeasured steps go in pairs through the two-step kernel: explicitly, or by
// default in the 20-plane layout.
bool use_tiled2(const ah_ctx *c) {
    if (c->layout != AH_LAYOUT_20 || !tiled_ok(c))
        return false;
    return c->kernel == AH_KERNEL_TILED2 || c->kernel == AH_KERNEL_AUTO;
}

// The batched kernel needs tiled shapes and one common step index (so every
// realization measures at the same steps).  It advances one step per launch.
bool batch_ok(const ah_ctx *c) {
    if (!c->batched || c->kernel == AH_KERNEL_PLAIN || !tiled_ok(c))
        return false;
    for (const auto &q : c->p)
        if (q.step0 != c->p[0].step0)
            return false;
    return true;
}

// Tile height of the batched kernel: it must serve the measuring mode too.
int batch_ty(const ah_ctx *c) {
    const bool fp64 = c->prec == AH_FP64;
    int ty = c->tile_y > 0 ? c->tile_y : (fp64 ? 4 : 8);
    return std::min(ty, tiled_ty_max(fp64, MODE_STEP_MEASURE));
}

int launch_tiled(ah_ctx *c, int r, int mode, Slot *slot) {
    const ah_params &q = c->p[r];
    int rc = launch_step_tiled(c->prec == AH_FP64, mode, c->d_desc, c->d_coef, r, q.nx, q.ny, q.nz,
                               c->tile_y, c->cz[r], slot, c->stream);
    if (rc)
        return fail(c, AH_E_HIP, "tiled kernel launch (mode %d) failed: %s", mode,
                    hipGetErrorString((hipError_t)rc));
    return AH_OK;
}

int launch_measure_plain(ah_ctx *c, int r, Slot *slot, int8_t *wind) {
    const int64_t N = sites_of(c->p[r]);
    dim3 grid(grid_for(N, kMeasureThreads, 4096));
    if (c->prec == AH_FP64)
        hipLaunchKernelGGL(k_measure_plain<double>, grid, dim3(kMeasureThreads), 0, c->stream,
                           c->d_desc, c->d_coef, r, slot, wind);
    else
        hipLaunchKernelGGL(k_measure_plain<float>, grid, dim3(kMeasureThreads), 0, c->stream,
                           c->d_desc, c->d_coef, r, slot, wind);
    HIP_TRY(c, hipGetLastError());
    return AH_OK;
}

// Advance realization r by one step (the coefficients are already on the
// device); with slot != NULL also measure the state it reads into slot.
int launch_step(ah_ctx *c, int r, Slot *slot) {
    if (use_tiled(c, r))
        return launch_tiled(c, r, slot ? MODE_STEP_MEASURE : MODE_STEP, slot);
    if (slot)
        TRY(launch_measure_plain(c, r, slot, nullptr));
    const int64_t N = sites_of(c->p[r]);
    dim3 grid((unsigned)((N + 255) / 256));
    if (c->prec == AH_FP64)
        hipLaunchKernelGGL(k_step_plain<double>, grid, dim3(256), 0, c->stream, c->d_desc, c->d_coef, r);
    else
        hipLaunchKernelGGL(k_step_plain<float>, grid, dim3(256), 0, c->stream, c->d_desc, c->d_coef, r);
    HIP_TRY(c, hipGetLastError());
    return AH_OK;
}

// Measure the current state of realization r into slot (standalone pass).
int launch_measure(ah_ctx *c, int r, Slot *slot, int8_t *wind) {
    if (!use_tiled(c, r))
        return launch_measure_plain(c, r, slot, wind);
    const ah_params &q = c->p[r];
    int rc = launch_measure_tiled(c->prec == AH_FP64, c->d_desc, c->d_coef, r, q.nx, q.ny, q.nz,
                                  sites_of(q), c->tile_y, c->cz[r], slot, wind, c->stream);
    if (rc)
        return fail(c, AH_E_HIP, "measuring kernel launch failed: %s",
                    hipGetErrorString((hipError_t)rc));
    return AH_OK;
}

int launch_finalize(ah_ctx *c, int64_t nslots) {
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)((nslots + 63) / 64)), dim3(64), 0, c->stream,
                       c->d_desc, c->d_slots, c->d_obs, (int)nslots, c->nreal);
    HIP_TRY(c, hipGetLastError());
    return AH_OK;
}

// Work list of the batched kernel: the tiles of every realization, largest
// realizations first, each realization's tiles in x-fastest order so that
// neighbours are consecutive items.
int build_items(ah_ctx *c) {
    if (c->items_valid)
        return AH_OK;
    const bool fp64 = c->prec == AH_FP64;
    const int ty = batch_ty(c);
    std::vector<int> order(c->nreal);
    for (int r = 0; r < c->nreal; ++r)
        order[r] = r;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return sites_of(c->p[a]) > sites_of(c->p[b]); });
    std::vector<BatchItem> items;
    for (int r : order) {
        const ah_params &q = c->p[r];
        int t = ty, z = c->cz[r];
        // with pairs through the two-step kernel, the single-step passes of
        // the batch (measured and odd steps) walk the chunks tuned for it
        if (z <= 0 && use_tiled2(c))
            z = c->cz2[r];
        tiled_defaults(fp64, q.nx, q.ny, q.nz, t, z);
        const int tiles = (q.nx / 64) * ((q.ny + ty - 1) / ty) * ((q.nz + z - 1) / z);
        for (int k = 0; k < tiles; ++k)
            items.push_back(BatchItem{ r, k, z, 0 });
    }
    if (c->d_items)
        (void)hipFree(c->d_items);
    c->d_items = nullptr;
    HIP_TRY(c, hipMalloc(&c->d_items, items.size() * sizeof(BatchItem)));
    HIP_TRY(c, hipMemcpyAsync(c->d_items, items.data(), items.size() * sizeof(BatchItem),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int rc = batch_dispatch(fp64, MODE_STEP, ty, nullptr, nullptr, nullptr, 0, nullptr, 0, nullptr,
                            &c->grid_step);
    if (rc == 0)
        rc = batch_dispatch(fp64, MODE_STEP_MEASURE, ty, nullptr, nullptr, nullptr, 0, nullptr, 0,
                            nullptr, &c->grid_meas);
    if (rc)
        return fail(c, AH_E_HIP, "occupancy query failed: %s", hipGetErrorString((hipError_t)rc));
    c->n_items = (int)items.size();
    c->items_ty = ty;
    c->items_valid = true;
    return AH_OK;
}

// Work list of the batched two-step kernel (same order, two-step tile shape).
int build_items2(ah_ctx *c) {
    if (c->items2_valid)
        return AH_OK;
    const bool fp64 = c->prec == AH_FP64;
    int ty = c->tile_y2;
    if (ty <= 0) {
        std::vector<int> nys(c->nreal);
        std::vector<long> ws(c->nreal);
        for (int r = 0; r < c->nreal; ++r) {
            nys[r] = c->p[r].ny;
            ws[r] = (long)c->p[r].nx * c->p[r].nz;
        }
        ty = tiled2_default_ty(fp64, nys.data(), ws.data(), c->nreal);
    }
    std::vector<int> order(c->nreal);
    for (int r = 0; r < c->nreal; ++r)
        order[r] = r;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return sites_of(c->p[a]) > sites_of(c->p[b]); });
    std::vector<BatchItem> items;
    for (int r : order) {
        const ah_params &q = c->p[r];
        int t = ty, z = c->cz2[r];
        tiled2_defaults(fp64, q.nx, q.ny, q.nz, t, z, false);
        const int tiles = (q.nx / 64) * ((q.ny + ty - 1) / ty) * ((q.nz + z - 1) / z);
        for (int k = 0; k < tiles; ++k)
            items.push_back(BatchItem{ r, k, z, 0 });
    }
    if (c->d_items2)
        (void)hipFree(c->d_items2);
    c->d_items2 = nullptr;
    HIP_TRY(c, hipMalloc(&c->d_items2, items.size() * sizeof(BatchItem)));
    HIP_TRY(c, hipMemcpyAsync(c->d_items2, items.data(), items.size() * sizeof(BatchItem),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    bool off32 = true;
    for (const auto &q : c->p)
        off32 = off32 && fits_off32(sites_of(q), fp64 ? 8 : 4);
    int rc = batch2_dispatch(fp64, ty, off32, nullptr, nullptr, nullptr, 0, c->nreal, 0, nullptr,
                             &c->grid2);
    if (rc)
        return fail(c, AH_E_HIP, "occupancy query failed: %s", hipGetErrorString((hipError_t)rc));
    c->n_items2 = (int)items.size();
    c->items2_ty = ty;
    c->items2_off32 = off32;
    c->items2_valid = true;
    return AH_OK;
}

// Work list of the batched read-only measuring pass: the two-step kernel's
// z-chunks (the pairs that follow walk them), 4-row tiles, the same order.
int build_items_m(ah_ctx *c) {
    if (c->items_m_valid)
        return AH_OK;
    const bool fp64 = c->prec == AH_FP64;
    const int ty = kMeasureBatchTY;
    std::vector<int> order(c->nreal);
    for (int r = 0; r < c->nreal; ++r)
        order[r] = r;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return sites_of(c->p[a]) > sites_of(c->p[b]); });
    std::vector<BatchItem> items;
    for (int r : order) {
        const ah_params &q = c->p[r];
        int t = ty, z = c->cz2[r] > 0 ? c->cz2[r] : c->cz[r];
        tiled_defaults(fp64, q.nx, q.ny, q.nz, t, z);
        const int tiles = (q.nx / 64) * ((q.ny + ty - 1) / ty) * ((q.nz + z - 1) / z);
        for (int k = 0; k < tiles; ++k)
            items.push_back(BatchItem{ r, k, z, 0 });
    }
    if (c->d_items_m)
        (void)hipFree(c->d_items_m);
    c->d_items_m = nullptr;
    HIP_TRY(c, hipMalloc(&c->d_items_m, items.size() * sizeof(BatchItem)));
    HIP_TRY(c, hipMemcpyAsync(c->d_items_m, items.data(), items.size() * sizeof(BatchItem),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    bool off32 = true;
    for (const auto &q : c->p)
        off32 = off32 && fits_off32(sites_of(q), fp64 ? 8 : 4);
    int rc = measure_batch_dispatch(fp64, off32, nullptr, nullptr, nullptr, 0, nullptr, 0, nullptr,
                                    &c->grid_m);
    if (rc)
        return fail(c, AH_E_HIP, "occupancy query failed: %s", hipGetErrorString((hipError_t)rc));
    c->n_items_m = (int)items.size();
    c->items_m_off32 = off32;
    c->items_m_valid = true;
    return AH_OK;
}

// One pass over memory of every realization: bookkeeping for `steps` (1 or
// 2) steps, then the kernels: the batched kernel of that many steps, or one
// launch per realization.  slots_row[r] receives the measurement of
// realization r when want_meas[r] (slots_row == NULL: no measurement;
// two-step passes never measure).  With skip_frozen the host leaves out
// realizations that reached n_end (the device skips them anyway, which keeps
// captured graphs valid).
int launch_pass(ah_ctx *c, int steps, Slot *slots_row, const char *want_meas, bool skip_frozen) {
    TRY(launch_bookkeep(c, steps));
    if (steps == 2 && batch_ok(c)) {
        TRY(build_items2(c));
        int rc = batch2_dispatch(c->prec == AH_FP64, c->items2_ty, c->items2_off32, c->d_desc,
                                 c->d_coef, c->d_items2, c->n_items2, c->nreal, c->grid2,
                                 c->stream, nullptr);
        if (rc)
            return fail(c, AH_E_HIP, "batched two-step kernel launch failed: %s",
                        hipGetErrorString((hipError_t)rc));
        return AH_OK;
    }
    if (steps == 2) {
        for (int r = 0; r < c->nreal; ++r) {
            if (skip_frozen && frozen(c, r))
                continue;
            const ah_params &q = c->p[r];
            int rc = launch_step_tiled2(c->prec == AH_FP64, c->d_desc, c->d_coef, r, c->nreal, q.nx,
                                        q.ny, q.nz, q.z_halo, c->tile_y2, c->cz2[r], c->stream);
            if (rc)
                return fail(c, AH_E_HIP, "two-step kernel launch failed: %s",
                            hipGetErrorString((hipError_t)rc));
        }
        return AH_OK;
    }
    if (batch_ok(c)) {
        TRY(build_items(c));
        const int mode = slots_row ? MODE_STEP_MEASURE : MODE_STEP;
        int rc = batch_dispatch(c->prec == AH_FP64, mode, c->items_ty, c->d_desc, c->d_coef,
                                c->d_items, c->n_items, slots_row,
                                slots_row ? c->grid_meas : c->grid_step, c->stream, nullptr);
        if (rc)
            return fail(c, AH_E_HIP, "batched kernel launch failed: %s",
                        hipGetErrorString((hipError_t)rc));
        return AH_OK;
    }
    for (int r = 0; r < c->nreal; ++r) {
        if (skip_frozen && frozen(c, r))
            continue;
        Slot *slot = slots_row && want_meas[r] ? slots_row + r : nullptr;
        TRY(launch_step(c, r, slot));
    }
    return AH_OK;
}

// Host mirror of k_bookkeep for one pass of `steps` steps.
void mirror_pass(ah_ctx *c, int steps) {
    for (int r = 0; r < c->nreal; ++r) {
        if (frozen(c, r))
            continue;
        c->step[r] += 1;
        c->copy[r] ^= 1;
        if (steps == 2 && !frozen(c, r))
            c->step[r] += 1;
    }
}

// Passes that advance g steps: pairs through the two-step kernel where it is
// in use, then a single step for an odd one.
std::vector<int> pass_plan(const ah_ctx *c, int64_t g) {
    std::vector<int> v;
    const bool two = use_tiled2(c);
    for (int64_t k = 0; k < g;) {
        const int s = two && g - k >= 2 ? 2 : 1;
        v.push_back(s);
        k += s;
    }
    return v;
}

// Capture graph_steps unmeasured steps once (on the context's own stream)
// and replay it reps times, ordered after the caller's stream work and
// before anything the caller enqueues later.
int run_graph(ah_ctx *c, int64_t reps) {
    if (!c->gstream) {
        HIP_TRY(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
        HIP_TRY(c, hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
        HIP_TRY(c, hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
    }
    if (batch_ok(c)) {
        TRY(build_items(c));     // outside the capture: they copy and synchronise
        if (use_tiled2(c))
            TRY(build_items2(c));
    }
    const std::vector<int> plan = pass_plan(c, c->graph_steps);
    if (!c->gexec_valid) {
        hipStream_t user = c->stream;
        HIP_TRY(c, hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
        c->stream = c->gstream;
        int rc = AH_OK;
        for (size_t k = 0; k < plan.size() && rc == AH_OK; ++k)
            rc = launch_pass(c, plan[k], nullptr, nullptr, false);
        c->stream = user;
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(c->gstream, &graph);
        if (rc != AH_OK) {
            if (graph)
                (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess)
            return fail(c, AH_E_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess)
            return fail(c, AH_E_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
        c->gexec_valid = true;
    }
    HIP_TRY(c, hipEventRecord(c->ev_in, c->stream));
    HIP_TRY(c, hipStreamWaitEvent(c->gstream, c->ev_in, 0));
    for (int64_t k = 0; k < reps; ++k)
        HIP_TRY(c, hipGraphLaunch(c->gexec, c->gstream));
    HIP_TRY(c, hipEventRecord(c->ev_out, c->gstream));
    HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_out, 0));
    for (int64_t k = 0; k < reps; ++k)
        for (int s : plan)
            mirror_pass(c, s);
    return AH_OK;
}

void release(ah_ctx *c) {
    if (!c)
        return;
    if (c->gexec)
        (void)hipGraphExecDestroy(c->gexec);
    if (c->ev_in)
        (void)hipEventDestroy(c->ev_in);
    if (c->ev_out)
        (void)hipEventDestroy(c->ev_out);
    if (c->gstream)
        (void)hipStreamDestroy(c->gstream);
    void *ptrs[] = { c->d_desc, c->d_step, c->d_copy, c->d_coef, c->d_slots, c->d_obs, c->d_gauss,
                     c->d_items, c->d_items2, c->d_items_m };
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
    delete c;
}

// ---- measurement without a context: the static scratch ----------------
//
// ah_measure_noalloc keeps its descriptors, coefficients and sums in one
// file-scope device array instead of memory it allocates.  Each GPU the
// library runs on holds its own copy of the array (until the process ends);
// host code reaches it only through the address hipGetSymbolAddress returns
// for the device that is current, never through the array's name.

constexpr size_t align256(size_t n) { return (n + 255) / 256 * 256; }
constexpr size_t kNoallocDescOff = 0;
constexpr size_t kNoallocCoefOff = align256(AH_NOALLOC_MAX_REAL * sizeof(RealDesc));
constexpr size_t kNoallocSlotOff = kNoallocCoefOff + align256(AH_NOALLOC_MAX_REAL * sizeof(Coef));
constexpr size_t kNoallocBytes = kNoallocSlotOff + align256(AH_NOALLOC_MAX_REAL * sizeof(Slot));
static_assert(sizeof(Slot) % 8 == 0, "slots are cleared in 64-bit words");

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

} // namespace

static __device__ __align__(256) unsigned long long scratch[kNoallocBytes / 8];

namespace {

// Device address of `scratch` on the current device, looked up once per device.
int noalloc_scratch(char **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(nullptr, AH_E_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(nullptr, AH_E_INVALID, "device %d beyond the %d the library tracks", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(nullptr, AH_E_HIP, "hipGetSymbolAddress(scratch) failed: %s",
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = (char *)g_scratch_ptr[dev];
    return AH_OK;
}

// Slot r of the static scratch: its descriptor, the coefficients of S_{step0}
// (first copy) and zeroed sums.
__global__ void k_noalloc_setup(RealDesc d, int r, RealDesc *descs, Coef *coefs, Slot *slots) {
    unsigned long long *w = reinterpret_cast<unsigned long long *>(slots + r);
    for (int i = threadIdx.x; i < (int)(sizeof(Slot) / 8); i += blockDim.x)
        w[i] = 0ull;
    if (threadIdx.x == 0) {
        descs[r] = d;
        coefs[r] = coef_at(d, d.step0, 0);
    }
}

} // namespace

extern "C" {

const char *ah_error_string(int code) {
    switch (code) {
    case AH_OK: return "ok";
    case AH_E_INVALID: return "invalid argument";
    case AH_E_NOMEM: return "out of memory";
    case AH_E_HIP: return "HIP runtime error";
    case AH_E_DOMAIN: return "parameters outside the method's domain";
    case AH_E_STATE: return "invalid state for this call";
    case AH_E_NONFINITE: return "non-finite field values";
    default: return "unknown status";
    }
}

const char *ah_last_error(const ah_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_init_err.c_str();
}

int ah_init(ah_ctx **out, int32_t n_real, const ah_params *p, const ah_buffers *buf,
            void *hip_stream) {
    g_init_err.clear();
    if (!out)
        return fail(nullptr, AH_E_INVALID, "ctx output pointer is NULL");
    *out = nullptr;
    if (n_real < 1 || !p || !buf)
        return fail(nullptr, AH_E_INVALID, "need n_real >= 1 and non-NULL params and buffers");
    for (int r = 0; r < n_real; ++r) {
        TRY(validate(p[r], r, buf[r], p[0].precision, p[0].layout));
        if (p[r].z_halo != p[0].z_halo)
            return fail(nullptr, AH_E_INVALID, "all realizations must share one z_halo");
    }

    ah_ctx *c = new (std::nothrow) ah_ctx;
    if (!c)
        return fail(nullptr, AH_E_NOMEM, "host allocation failed");
    c->nreal = n_real;
    c->prec = p[0].precision;
    c->layout = p[0].layout;
    c->zh = p[0].z_halo;
    c->stream = (hipStream_t)hip_stream;
    c->p.assign(p, p + n_real);
    c->step.resize(n_real);
    c->copy.assign(n_real, 0);
    c->cz.assign(n_real, 0);
    c->cz2.assign(n_real, 0);

    std::vector<RealDesc> desc(n_real);
    for (int r = 0; r < n_real; ++r) {
        desc[r] = make_desc(p[r], buf[r].planes);
        c->step[r] = p[r].step0;
    }

    auto hip_fail = [&](hipError_t e, const char *what) {
        g_init_err = std::string(what) + " failed: " + hipGetErrorString(e);
        release(c);
        return AH_E_HIP;
    };
    hipError_t e;
    {
        // set-up of ah_measure_noalloc's static scratch on this device
        char *unused = nullptr;
        const int rc = noalloc_scratch(&unused);
        if (rc != AH_OK) {
            release(c);
            return rc;
        }
    }
    if ((e = hipMalloc(&c->d_desc, n_real * sizeof(RealDesc))) != hipSuccess)
        return hip_fail(e, "hipMalloc(desc)");
    if ((e = hipMalloc(&c->d_step, n_real * sizeof(int64_t))) != hipSuccess)
        return hip_fail(e, "hipMalloc(step)");
    if ((e = hipMalloc(&c->d_copy, n_real * sizeof(int32_t))) != hipSuccess)
        return hip_fail(e, "hipMalloc(copy)");
    if ((e = hipMalloc(&c->d_coef, 2 * n_real * sizeof(Coef))) != hipSuccess)
        return hip_fail(e, "hipMalloc(coef)");
    if ((e = hipMalloc(&c->d_gauss, n_real * 2 * sizeof(unsigned long long))) != hipSuccess)
        return hip_fail(e, "hipMalloc(gauss)");
    if ((e = hipMemcpyAsync(c->d_desc, desc.data(), n_real * sizeof(RealDesc),
                            hipMemcpyHostToDevice, c->stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(desc)");
    if ((e = hipMemcpyAsync(c->d_step, c->step.data(), n_real * sizeof(int64_t),
                            hipMemcpyHostToDevice, c->stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(step)");
    if ((e = hipMemcpyAsync(c->d_copy, c->copy.data(), n_real * sizeof(int32_t),
                            hipMemcpyHostToDevice, c->stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(copy)");
    for (int r = 0; r < n_real; ++r) {
        if (p[r].init == AH_INIT_NONE)
            continue;
        dim3 grid(grid_for(desc[r].N, 256, 8192));
        if (c->prec == AH_FP64)
            hipLaunchKernelGGL(k_init<double>, grid, dim3(256), 0, c->stream, c->d_desc, r,
                               (int)p[r].init, (uint64_t)p[r].seed);
        else
            hipLaunchKernelGGL(k_init<float>, grid, dim3(256), 0, c->stream, c->d_desc, r,
                               (int)p[r].init, (uint64_t)p[r].seed);
        if ((e = hipGetLastError()) != hipSuccess)
            return hip_fail(e, "k_init launch");
    }
    if ((e = hipMalloc(&c->d_slots, kMinSlotStates * n_real * sizeof(Slot))) != hipSuccess)
        return hip_fail(e, "hipMalloc(slots)");
    if ((e = hipMalloc(&c->d_obs, kMinSlotStates * n_real * sizeof(ah_obs))) != hipSuccess)
        return hip_fail(e, "hipMalloc(obs)");
    c->slot_cap = kMinSlotStates;
    // the host vectors above are stack memory: make sure the copies are done
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess)
        return hip_fail(e, "hipStreamSynchronize");
    *out = c;
    return AH_OK;
}

int ah_step(ah_ctx *c, int64_t nsteps, int32_t measure_every, ah_obs *out, int64_t out_cap,
            int64_t *n_out) {
    if (!c)
        return fail(nullptr, AH_E_INVALID, "NULL context");
    c->err.clear();
    if (nsteps < 0 || measure_every < 0)
        return fail(c, AH_E_INVALID, "nsteps and measure_every must be >= 0");
    if (measure_every > 0 && (!out || !n_out))
        return fail(c, AH_E_INVALID, "measuring needs out and n_out");
    if (c->kernel == AH_KERNEL_TILED && !tiled_ok(c))
        return fail(c, AH_E_INVALID, "tiled kernel needs nx %% 64 == 0");

    // plan: which call-steps measure, per realization (host mirror of the counters)
    std::vector<int64_t> n = c->step;
    std::vector<std::vector<char>> meas;   // [slot][r]
    std::vector<int64_t> meas_at;          // call-step index of each slot
    if (measure_every > 0) {
        for (int64_t i = 0; i < nsteps; ++i) {
            std::vector<char> row(c->nreal, 0);
            bool any = false;
            for (int r = 0; r < c->nreal; ++r) {
                const ah_params &q = c->p[r];
                bool active = q.n_end <= 0 || n[r] < q.n_end;
                if (active && n[r] % measure_every == 0) {
                    row[r] = 1;
                    any = true;
                }
                if (active)
                    ++n[r];
            }
            if (any) {
                meas.push_back(row);
                meas_at.push_back(i);
            }
        }
        if ((int64_t)meas.size() > out_cap)
            return fail(c, AH_E_INVALID, "out_cap %lld too small: %zu measurements",
                        (long long)out_cap, meas.size());
        TRY(ensure_slots(c, (int64_t)meas.size()));
        if (!meas.empty())
            TRY(launch_zero(c, c->d_slots, meas.size() * c->nreal * sizeof(Slot)));
    }

    // a slab with one halo plane a side cannot take pairs
    const bool two = use_tiled2(c) && c->zh != 1;
    if (c->zh > 0) {
        // slabs: the caller refreshes the halo between passes, so one per call
        int64_t passes = 0, j = 0;
        size_t nm = 0;
        while (j < nsteps) {
            const bool measured = nm < meas.size() && meas_at[nm] == j;
            const int64_t stop = nm < meas.size() ? meas_at[nm] : nsteps;
            const int64_t adv = measured ? 1 : (two && stop - j >= 2 ? 2 : 1);
            nm += measured ? 1 : 0;
            j += adv;
            ++passes;
        }
        if (passes > 1)
            return fail(c, AH_E_INVALID,
                        "a slab context advances one pass per call (%lld steps need %lld)",
                        (long long)nsteps, (long long)passes);
    }

    // FP32 with pairs: a measured state whose next stop is an even number of
    // steps away is measured by a read-only pass (one persistent launch in the
    // batched form) and then stepped in pairs (at 512^3: 2.0 + 2.7 ms against
    // 3.7 + 2.1 ms for the fused measuring step and the odd single step that
    // would follow); FP64 pairs cost more than that saves, and slabs keep the
    // fused step.
    const bool ro_measure = two && c->prec == AH_FP32 && c->zh == 0;
    size_t next = 0;
    int64_t i = 0;
    while (i < nsteps) {
        if (next < meas.size() && meas_at[next] == i) {
            const int64_t stop = next + 1 < meas.size() ? meas_at[next + 1] : nsteps;
            if (ro_measure && (stop - i) % 2 == 0) {
                TRY(launch_bookkeep(c, 0));
                if (batch_ok(c)) {
                    // frozen realizations (past their n_end) are skipped on the device
                    TRY(build_items_m(c));
                    int rc = measure_batch_dispatch(false, c->items_m_off32, c->d_desc, c->d_coef, c->d_items_m,
                                                    c->n_items_m, c->d_slots + next * c->nreal,
                                                    c->grid_m, c->stream, nullptr);
                    if (rc)
                        return fail(c, AH_E_HIP, "batched measuring kernel launch failed: %s",
                                    hipGetErrorString((hipError_t)rc));
                } else {
                    for (int r = 0; r < c->nreal; ++r)
                        if (meas[next][r])
                            TRY(launch_measure(c, r, c->d_slots + next * c->nreal + r, nullptr));
                }
                ++next;
                continue;   // the steps from i go in pairs
            }
            // measured states take a single-step pass with the fused measurement
            TRY(launch_pass(c, 1, c->d_slots + next * c->nreal, meas[next].data(), true));
            mirror_pass(c, 1);
            ++next;
            ++i;
            continue;
        }
        const int64_t stop = next < meas.size() ? meas_at[next] : nsteps;
        if (c->graph_steps > 0 && stop - i >= c->graph_steps) {
            const int64_t reps = (stop - i) / c->graph_steps;
            TRY(run_graph(c, reps));
            i += reps * c->graph_steps;
            continue;
        }
        const int s = two && stop - i >= 2 ? 2 : 1;
        TRY(launch_pass(c, s, nullptr, nullptr, true));
        mirror_pass(c, s);
        i += s;
    }

    if (measure_every > 0) {
        *n_out = (int64_t)meas.size();
        if (meas.empty())
            return AH_OK;
        const int64_t nslots = (int64_t)meas.size() * c->nreal;
        TRY(launch_finalize(c, nslots));
        HIP_TRY(c, hipMemcpyAsync(out, c->d_obs, nslots * sizeof(ah_obs), hipMemcpyDeviceToHost,
                                  c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (int64_t k = 0; k < nslots; ++k)
            if (out[k].nonfinite > 0)
                return fail(c, AH_E_NONFINITE, "measurement at step %lld saw %lld non-finite sites",
                            (long long)out[k].step, (long long)out[k].nonfinite);
    } else if (n_out) {
        *n_out = 0;
    }
    return AH_OK;
}

int ah_measure(ah_ctx *c, ah_obs *out, int8_t *wind_dev) {
    if (!c)
        return fail(nullptr, AH_E_INVALID, "NULL context");
    c->err.clear();
    if (!out)
        return fail(c, AH_E_INVALID, "NULL out");
    TRY(ensure_slots(c, 1));
    TRY(launch_zero(c, c->d_slots, c->nreal * sizeof(Slot)));
    TRY(launch_bookkeep(c, 0));
    int64_t off = 0;
    for (int r = 0; r < c->nreal; ++r) {
        TRY(launch_measure(c, r, c->d_slots + r, wind_dev ? wind_dev + off : nullptr));
        off += 3 * sites_of(c->p[r]);
    }
    TRY(launch_finalize(c, c->nreal));
    HIP_TRY(c, hipMemcpyAsync(out, c->d_obs, c->nreal * sizeof(ah_obs), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int r = 0; r < c->nreal; ++r)
        if (out[r].nonfinite > 0)
            return fail(c, AH_E_NONFINITE, "realization %d: %lld non-finite sites", r,
                        (long long)out[r].nonfinite);
    return AH_OK;
}

int ah_measure_noalloc(int32_t n_real, const ah_params *p, const ah_buffers *buf,
                       ah_obs *out_dev, int8_t *wind_dev, void *hip_stream) {
    g_init_err.clear();
    if (n_real < 1 || n_real > AH_NOALLOC_MAX_REAL)
        return fail(nullptr, AH_E_INVALID,
                    "n_real %d outside [1, %d]: the static scratch holds %d states per call",
                    (int)n_real, AH_NOALLOC_MAX_REAL, AH_NOALLOC_MAX_REAL);
    if (!p || !buf || !out_dev)
        return fail(nullptr, AH_E_INVALID, "need non-NULL params, buffers and out_dev");
    for (int r = 0; r < n_real; ++r)
        TRY(validate(p[r], r, buf[r], p[0].precision, p[0].layout));
    char *base = nullptr;
    TRY(noalloc_scratch(&base));
    RealDesc *descs = (RealDesc *)(base + kNoallocDescOff);
    Coef *coefs = (Coef *)(base + kNoallocCoefOff);
    Slot *slots = (Slot *)(base + kNoallocSlotOff);
    hipStream_t st = (hipStream_t)hip_stream;
    const bool fp64 = p[0].precision == AH_FP64;
    hipError_t e;
    for (int r = 0; r < n_real; ++r) {
        hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(64), 0, st, make_desc(p[r], buf[r].planes),
                           r, descs, coefs, slots);
        if ((e = hipGetLastError()) != hipSuccess)
            return fail(nullptr, AH_E_HIP, "k_noalloc_setup launch failed: %s", hipGetErrorString(e));
    }
    // the kernels ah_measure takes by default: tiled where nx % 64 == 0
    int64_t off = 0;
    for (int r = 0; r < n_real; ++r) {
        const ah_params &q = p[r];
        int8_t *w = wind_dev ? wind_dev + off : nullptr;
        if (q.nx % 64 == 0) {
            int rc = launch_measure_tiled(fp64, descs, coefs, r, q.nx, q.ny, q.nz, sites_of(q), 0, 0,
                                          slots + r, w, st);
            if (rc)
                return fail(nullptr, AH_E_HIP, "tiled measuring kernel launch failed: %s",
                            hipGetErrorString((hipError_t)rc));
        } else {
            dim3 grid(grid_for(sites_of(q), kMeasureThreads, 4096));
            if (fp64)
                hipLaunchKernelGGL(k_measure_plain<double>, grid, dim3(kMeasureThreads), 0, st, descs,
                                   coefs, r, slots + r, w);
            else
                hipLaunchKernelGGL(k_measure_plain<float>, grid, dim3(kMeasureThreads), 0, st, descs,
                                   coefs, r, slots + r, w);
            if ((e = hipGetLastError()) != hipSuccess)
                return fail(nullptr, AH_E_HIP, "measuring kernel launch failed: %s",
                            hipGetErrorString(e));
        }
        off += 3 * sites_of(q);
    }
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)((n_real + 63) / 64)), dim3(64), 0, st, descs,
                       slots, out_dev, (int)n_real, (int)n_real);
    if ((e = hipGetLastError()) != hipSuccess)
        return fail(nullptr, AH_E_HIP, "k_finalize launch failed: %s", hipGetErrorString(e));
    return AH_OK;
}

int ah_gauss_residual(ah_ctx *c, double *max_abs, double *rms) {
    if (!c)
        return fail(nullptr, AH_E_INVALID, "NULL context");
    c->err.clear();
    if (!max_abs || !rms)
        return fail(c, AH_E_INVALID, "NULL output");
    if (c->zh > 0)
        return fail(c, AH_E_INVALID, "the Gauss residual is not available for slabs");
    TRY(launch_zero(c, c->d_gauss, c->nreal * 2 * sizeof(unsigned long long)));
    TRY(launch_bookkeep(c, 0));
    for (int r = 0; r < c->nreal; ++r) {
        dim3 grid(grid_for(sites_of(c->p[r]), kMeasureThreads, 4096));
        if (c->prec == AH_FP64)
            hipLaunchKernelGGL(k_gauss<double>, grid, dim3(kMeasureThreads), 0, c->stream,
                               c->d_desc, c->d_coef, r, c->d_gauss + 2 * r);
        else
            hipLaunchKernelGGL(k_gauss<float>, grid, dim3(kMeasureThreads), 0, c->stream,
                               c->d_desc, c->d_coef, r, c->d_gauss + 2 * r);
        HIP_TRY(c, hipGetLastError());
    }
    std::vector<unsigned long long> h(2 * c->nreal);
    HIP_TRY(c, hipMemcpyAsync(h.data(), c->d_gauss, h.size() * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int r = 0; r < c->nreal; ++r) {
        double m, s;
        std::memcpy(&m, &h[2 * r], sizeof m);
        std::memcpy(&s, &h[2 * r + 1], sizeof s);
        max_abs[r] = m;
        rms[r] = std::sqrt(s / (double)sites_of(c->p[r]));
    }
    return AH_OK;
}

int ah_current_planes(const ah_ctx *c, int32_t r, int32_t plane_of_field[10]) {
    if (!c || !plane_of_field || r < 0 || r >= c->nreal)
        return AH_E_INVALID;
    for (int f = 0; f < 10; ++f)
        plane_of_field[f] = field_plane(f, c->copy[r], c->layout);
    return AH_OK;
}

int ah_current_step(const ah_ctx *c, int32_t r, int64_t *n) {
    if (!c || !n || r < 0 || r >= c->nreal)
        return AH_E_INVALID;
    *n = c->step[r];
    return AH_OK;
}

int ah_set_kernel(ah_ctx *c, int32_t kernel, int32_t tile_y, int32_t chunk_z) {
    if (!c)
        return fail(nullptr, AH_E_INVALID, "NULL context");
    c->err.clear();
    if (kernel < AH_KERNEL_AUTO || kernel > AH_KERNEL_TILED2)
        return fail(c, AH_E_INVALID, "unknown kernel %d", kernel);
    const bool fp64 = c->prec == AH_FP64;
    if (chunk_z < 0)
        return fail(c, AH_E_INVALID, "chunk_z must be >= 0");
    if (kernel == AH_KERNEL_TILED2) {
        if (tile_y != 0 && !tiled2_ty_valid(fp64, tile_y))
            return fail(c, AH_E_INVALID,
                        "two-step kernel: tile_y must be 0, 4, 8 or 9 (FP32), 0, 4 or 5 (FP64)");
        if (c->layout != AH_LAYOUT_20)
            return fail(c, AH_E_INVALID, "two-step kernel needs AH_LAYOUT_20");
    } else if (tile_y != 0 && !tiled_ty_valid(fp64, tile_y)) {
        return fail(c, AH_E_INVALID, "tile_y must be 0, 2, 4, 8 (or 16 for FP32)");
    }
    if ((kernel == AH_KERNEL_TILED || kernel == AH_KERNEL_TILED2) && !tiled_ok(c))
        return fail(c, AH_E_INVALID, "tiled kernel needs nx %% 64 == 0");
    if (kernel == AH_KERNEL_PLAIN && c->zh > 0)
        return fail(c, AH_E_INVALID, "slabs (z_halo > 0) need the tiled kernels");
    c->kernel = kernel;
    const bool two = kernel == AH_KERNEL_TILED2;
    c->tile_y = two ? 0 : tile_y;
    c->cz.assign(c->nreal, two ? 0 : chunk_z);
    c->tile_y2 = two ? tile_y : 0;
    c->cz2.assign(c->nreal, two ? chunk_z : 0);
    invalidate_plans(c);
    return AH_OK;
}

int ah_set_launch(ah_ctx *c, int32_t batched, int32_t graph_steps) {
    if (!c)
        return fail(nullptr, AH_E_INVALID, "NULL context");
    c->err.clear();
    if ((batched != 0 && batched != 1) || graph_steps < 0 || graph_steps > 4096)
        return fail(c, AH_E_INVALID, "batched must be 0 or 1 and graph_steps in 0..4096");
    if (c->zh > 0 && (batched != 0 || graph_steps != 0))
        return fail(c, AH_E_INVALID, "slabs (z_halo > 0) run unbatched without graphs");
    c->batched = batched;
    c->graph_steps = graph_steps;
    invalidate_plans(c);
    return AH_OK;
}

int ah_autotune(ah_ctx *c, int32_t *tile_y, int32_t *chunk_z) {
    if (!c)
        return fail(nullptr, AH_E_INVALID, "NULL context");
    c->err.clear();
    if (c->kernel == AH_KERNEL_PLAIN || !tiled_ok(c))
        return fail(c, AH_E_STATE, "autotuning needs the tiled kernel (nx %% 64 == 0)");
    if (c->zh > 0)
        return fail(c, AH_E_STATE, "autotuning is not available for slabs");
    const bool fp64 = c->prec == AH_FP64;
    // the kernel that runs the unmeasured steps, and in which launch form
    const bool two = use_tiled2(c);
    const bool for_batch = batch_ok(c);
    const int ty_cap = c->batched ? tiled_ty_max(fp64, MODE_STEP_MEASURE) : tiled_ty_max(fp64, MODE_STEP);
    std::vector<int> tys;
    for (int t : { 4, 5, 8, 9, 16 })
        if (two ? tiled2_ty_valid(fp64, t) : (tiled_ty_valid(fp64, t) && t <= ty_cap))
            tys.push_back(t);

    // distinct shapes; each is timed on a scratch lattice of its own, so the
    // caller's fields are not touched
    struct Shape {
        int nx, ny, nz, count;
        std::vector<double> ms;   // per candidate tile height: est. ms per step
        std::vector<int> cz;      // per candidate tile height: best z-chunk
    };
    std::vector<Shape> shapes;
    std::vector<int> shape_of(c->nreal);
    for (int r = 0; r < c->nreal; ++r) {
        const ah_params &q = c->p[r];
        int k = 0;
        while (k < (int)shapes.size() &&
               !(shapes[k].nx == q.nx && shapes[k].ny == q.ny && shapes[k].nz == q.nz))
            ++k;
        if (k == (int)shapes.size())
            shapes.push_back(Shape{ q.nx, q.ny, q.nz, 0, {}, {} });
        shapes[k].count++;
        shape_of[r] = k;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    RealDesc *d_desc = nullptr;
    Coef *d_coef = nullptr;
    int64_t *d_step = nullptr;
    int32_t *d_copy = nullptr;
    char *scratch = nullptr;
    int rc = AH_OK;
    auto hip_ok = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && rc == AH_OK)
            rc = fail(c, AH_E_HIP, "autotune: %s failed: %s", what, hipGetErrorString(e));
        return rc == AH_OK;
    };
    if (hip_ok(hipEventCreate(&e0), "hipEventCreate") && hip_ok(hipEventCreate(&e1), "hipEventCreate") &&
        hip_ok(hipMalloc(&d_desc, sizeof(RealDesc)), "hipMalloc") &&
        hip_ok(hipMalloc(&d_coef, 2 * sizeof(Coef)), "hipMalloc") &&
        hip_ok(hipMalloc(&d_step, sizeof(int64_t)), "hipMalloc") &&
        hip_ok(hipMalloc(&d_copy, sizeof(int32_t)), "hipMalloc")) {
        for (Shape &sh : shapes) {
            // The cost per plane is what is tuned.  With one launch per
            // realization the shape itself is timed (at most 128 planes), as
            // it will run.  The batched form keeps the chip busy with many
            // realizations at once, so there the same tile shape is timed on
            // a lattice tall enough that every candidate chunk gives at least
            // four blocks per compute unit: the planes a chunk walks beyond
            // its own are then weighed at full occupancy (timed on the shape
            // alone, a 128^3 realization of an ensemble took 16-plane chunks).
            const int ty_big = tys.back();
            const long txy = (long)(sh.nx / 64) * ((sh.ny + ty_big - 1) / ty_big);
            const int nz_own = std::min(sh.nz, 128);
            int nzs = for_batch ? (int)std::min<long>(16384, 128 * ((1024 + txy - 1) / txy)) : nz_own;
            if (nzs < nz_own)
                nzs = nz_own;
            const int layout = two ? AH_LAYOUT_20 : AH_LAYOUT_15;
            auto scratch_bytes = [&](int planes_z) {
                return (size_t)sh.nx * sh.ny * planes_z * plane_count(layout) * (fp64 ? 8 : 4);
            };
            hipError_t me = hipMalloc(&scratch, scratch_bytes(nzs));
            if (me != hipSuccess && nzs > nz_own) {
                // no room for the tall lattice: time the shape itself
                (void)hipGetLastError();
                scratch = nullptr;
                nzs = nz_own;
                me = hipMalloc(&scratch, scratch_bytes(nzs));
            }
            if (!hip_ok(me, "hipMalloc(scratch)"))
                break;
            const int64_t N = (int64_t)sh.nx * sh.ny * nzs;
            const ah_params &q0 = c->p[0];
            RealDesc d{};
            d.base = scratch;
            d.nx = sh.nx;
            d.ny = sh.ny;
            d.nz = nzs;
            d.elem = fp64 ? 8 : 4;
            d.layout = layout;
            d.N = N;
            d.dx = q0.dx;
            d.dt = q0.dt;
            d.tau0 = 1.0;
            d.tau_ref = 2.0;
            d.era_p = 1.0;
            d.s = 1.0;
            d.lambda0 = q0.lambda0;
            d.e0 = q0.e0;
            d.sigma = q0.sigma;
            const int64_t s0 = 0;
            const int32_t cp0 = 0;
            hip_ok(hipMemcpyAsync(d_desc, &d, sizeof d, hipMemcpyHostToDevice, c->stream), "copy");
            hip_ok(hipMemcpyAsync(d_step, &s0, sizeof s0, hipMemcpyHostToDevice, c->stream), "copy");
            hip_ok(hipMemcpyAsync(d_copy, &cp0, sizeof cp0, hipMemcpyHostToDevice, c->stream), "copy");
            dim3 ig(grid_for(N, 256, 8192));
            if (fp64)
                hipLaunchKernelGGL(k_init<double>, ig, dim3(256), 0, c->stream, d_desc, 0,
                                   (int)AH_INIT_RANDOM_PHASE, (uint64_t)12345);
            else
                hipLaunchKernelGGL(k_init<float>, ig, dim3(256), 0, c->stream, d_desc, 0,
                                   (int)AH_INIT_RANDOM_PHASE, (uint64_t)12345);
            // coefficients of steps 0 and 1, read from copy 0 by every timed launch
            hipLaunchKernelGGL(k_bookkeep, dim3(1), dim3(64), 0, c->stream, d_desc, d_step, d_copy,
                               d_coef, 1, two ? 2 : 0);
            hip_ok(hipGetLastError(), "launch");
            for (int t : tys) {
                double best = 1e300;
                int best_cz = 8;
                for (int z : { 8, 16, 32, 64, 128 }) {
                    if (z > nzs || z > sh.nz || rc != AH_OK)
                        continue;
                    for (int k = 0; k < 4 && rc == AH_OK; ++k) {
                        if (k == 1)
                            hip_ok(hipEventRecord(e0, c->stream), "hipEventRecord");
                        hip_ok((hipError_t)(two ? launch_step_tiled2(fp64, d_desc, d_coef, 0, 1,
                                                                     sh.nx, sh.ny, nzs, 0, t, z,
                                                                     c->stream)
                                                 : launch_step_tiled(fp64, MODE_STEP, d_desc, d_coef,
                                                                     0, sh.nx, sh.ny, nzs, t, z,
                                                                     nullptr, c->stream)),
                               "tiled launch");
                    }
                    float ms = 0.f;
                    hip_ok(hipEventRecord(e1, c->stream), "hipEventRecord");
                    hip_ok(hipEventSynchronize(e1), "hipEventSynchronize");
                    hip_ok(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
                    // per plane and step
                    const double per_plane = ms / 3.0 / nzs / (two ? 2.0 : 1.0);
                    if (per_plane < best) {
                        best = per_plane;
                        best_cz = z;
                    }
                }
                sh.ms.push_back(best * sh.nz);
                sh.cz.push_back(best_cz);
            }
            (void)hipStreamSynchronize(c->stream);
            (void)hipFree(scratch);
            scratch = nullptr;
            if (rc != AH_OK)
                break;
        }
    }
    (void)hipStreamSynchronize(c->stream);
    if (scratch)
        (void)hipFree(scratch);
    if (d_desc)
        (void)hipFree(d_desc);
    if (d_coef)
        (void)hipFree(d_coef);
    if (d_step)
        (void)hipFree(d_step);
    if (d_copy)
        (void)hipFree(d_copy);
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (rc != AH_OK)
        return rc;

    // one tile height for the context: least total estimated time per step
    int bi = 0;
    double bt = 1e300;
    for (size_t i = 0; i < tys.size(); ++i) {
        double tot = 0.0;
        for (const Shape &sh : shapes)
            tot += sh.ms[i] * sh.count;
        if (tot < bt) {
            bt = tot;
            bi = (int)i;
        }
    }
    int &ty_set = two ? c->tile_y2 : c->tile_y;
    std::vector<int> &cz_set = two ? c->cz2 : c->cz;
    ty_set = tys[bi];
    for (int r = 0; r < c->nreal; ++r)
        cz_set[r] = shapes[shape_of[r]].cz[bi];
    invalidate_plans(c);
    if (tile_y)
        *tile_y = ty_set;
    if (chunk_z)
        for (int r = 0; r < c->nreal; ++r)
            chunk_z[r] = cz_set[r];
    return AH_OK;
}

int ah_free(ah_ctx *c) {
    if (!c)
        return AH_OK;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (c->gstream && e == hipSuccess)
        e = hipStreamSynchronize(c->gstream);
    release(c);
    return e == hipSuccess ? AH_OK : AH_E_HIP;
}

} // extern "C"
