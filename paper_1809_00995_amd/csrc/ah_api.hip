// ah_api.hip -- host side of the C ABI declared in include/ah.h: parameter
// validation, the context's device scratch, and the launch sequence of each
// entry point.  All GPU work of a context goes on its stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ah.h"
#include "ah_device.hpp"
#include "k_common.hpp"
#include "k_measure.hpp"
#include "k_step_plain.hpp"
#include "k_step_tiled.hpp"

using namespace ah;

struct ah_ctx {
    int nreal = 0;
    int prec = AH_FP64;
    hipStream_t stream = nullptr;
    std::vector<ah_params> p;
    std::vector<int64_t> step;        // host mirror of each realization's step index
    RealDesc *d_desc = nullptr;
    int64_t *d_step = nullptr;
    Coef *d_coef = nullptr;
    Slot *d_slots = nullptr;          // measurement slots
    ah_obs *d_obs = nullptr;
    int64_t slot_cap = 0;             // slots allocated, in states (x nreal)
    unsigned long long *d_gauss = nullptr;  // [nreal][2]
    int kernel = AH_KERNEL_AUTO;
    int tile_y = 0, chunk_z = 0;
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

double scale_factor_host(const ah_params &p, double tau) {
    double t = tau > 0.0 ? tau : 0.0;
    return std::pow(t / p.tau_ref, p.era_p);
}

int validate(const ah_params &q, int r, const ah_buffers &b, int prec) {
    auto bad = [&](int code, const char *what) {
        return fail(nullptr, code, "realization %d: %s", r, what);
    };
    if (q.nx < 4 || q.ny < 4 || q.nz < 4)
        return bad(AH_E_INVALID, "extents must be >= 4");
    if ((int64_t)q.nx * q.ny * q.nz >= (int64_t)1 << 31)
        return bad(AH_E_INVALID, "nx*ny*nz must be < 2^31");
    if (q.precision != prec)
        return bad(AH_E_INVALID, "all realizations must share one precision");
    if (q.precision != AH_FP64 && q.precision != AH_FP32)
        return bad(AH_E_INVALID, "precision must be AH_FP64 or AH_FP32");
    if (!(q.dx > 0.0) || !(q.dt > 0.0) || !std::isfinite(q.dx) || !std::isfinite(q.dt))
        return bad(AH_E_INVALID, "dx and dt must be positive and finite");
    if (!(q.dt / q.dx < 1.0 / std::sqrt(3.0)))
        return bad(AH_E_DOMAIN, "CFL condition dt/dx < 1/sqrt(3) violated");
    if (!(q.s >= 0.0 && q.s <= 1.0))
        return bad(AH_E_DOMAIN, "s must lie in [0, 1]");
    if (!(q.era_p >= 0.0) || !std::isfinite(q.era_p))
        return bad(AH_E_DOMAIN, "era_p must be >= 0");
    if (!(q.tau_ref > 0.0) || !std::isfinite(q.tau_ref) || !std::isfinite(q.tau0))
        return bad(AH_E_DOMAIN, "tau_ref must be > 0 and tau0 finite");
    if (!(q.lambda0 >= 0.0) || !(q.e0 > 0.0) || !(q.sigma > 0.0))
        return bad(AH_E_DOMAIN, "need lambda0 >= 0, e0 > 0, sigma > 0");
    if (q.init < AH_INIT_RANDOM_PHASE || q.init > AH_INIT_NONE || q.reserved != 0)
        return bad(AH_E_INVALID, "bad init kind or reserved field");
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

int ensure_slots(ah_ctx *c, int64_t states) {
    if (states <= c->slot_cap)
        return AH_OK;
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

int launch_bookkeep(ah_ctx *c, int advance) {
    hipLaunchKernelGGL(k_bookkeep, dim3((c->nreal + 63) / 64), dim3(64), 0, c->stream, c->d_desc,
                       c->d_step, c->d_coef, c->nreal, advance);
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
    return c->kernel == AH_KERNEL_TILED || (c->kernel == AH_KERNEL_AUTO && c->p[r].nx % 64 == 0);
}

int launch_tiled(ah_ctx *c, int r, int mode, Slot *slot, int8_t *wind) {
    const ah_params &q = c->p[r];
    int rc = launch_step_tiled(c->prec == AH_FP64, mode, c->d_desc, c->d_coef, r, q.nx, q.ny, q.nz,
                               c->tile_y, c->chunk_z, slot, wind, c->stream);
    if (rc)
        return fail(c, AH_E_HIP, "tiled kernel launch (mode %d) failed: %s", mode,
                    hipGetErrorString((hipError_t)rc));
    return AH_OK;
}

int launch_measure_plain(ah_ctx *c, int r, Slot *slot, int8_t *wind) {
    const ah_params &q = c->p[r];
    const int64_t N = (int64_t)q.nx * q.ny * q.nz;
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
        return launch_tiled(c, r, slot ? MODE_STEP_MEASURE : MODE_STEP, slot, nullptr);
    if (slot)
        TRY(launch_measure_plain(c, r, slot, nullptr));
    const ah_params &q = c->p[r];
    const int64_t N = (int64_t)q.nx * q.ny * q.nz;
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
    if (use_tiled(c, r))
        return launch_tiled(c, r, MODE_MEASURE, slot, wind);
    return launch_measure_plain(c, r, slot, wind);
}

int launch_finalize(ah_ctx *c, int64_t nslots) {
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)((nslots + 63) / 64)), dim3(64), 0, c->stream,
                       c->d_desc, c->d_slots, c->d_obs, (int)nslots, c->nreal);
    HIP_TRY(c, hipGetLastError());
    return AH_OK;
}

void release(ah_ctx *c) {
    if (!c)
        return;
    void *ptrs[] = { c->d_desc, c->d_step, c->d_coef, c->d_slots, c->d_obs, c->d_gauss };
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
    delete c;
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
    for (int r = 0; r < n_real; ++r)
        TRY(validate(p[r], r, buf[r], p[0].precision));

    ah_ctx *c = new (std::nothrow) ah_ctx;
    if (!c)
        return fail(nullptr, AH_E_NOMEM, "host allocation failed");
    c->nreal = n_real;
    c->prec = p[0].precision;
    c->stream = (hipStream_t)hip_stream;
    c->p.assign(p, p + n_real);
    c->step.resize(n_real);

    std::vector<RealDesc> desc(n_real);
    for (int r = 0; r < n_real; ++r) {
        const ah_params &q = p[r];
        RealDesc &d = desc[r];
        d.base = (char *)buf[r].planes;
        d.nx = q.nx;
        d.ny = q.ny;
        d.nz = q.nz;
        d.elem = c->prec == AH_FP64 ? 8 : 4;
        d.N = (int64_t)q.nx * q.ny * q.nz;
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
        c->step[r] = q.step0;
    }

    auto hip_fail = [&](hipError_t e, const char *what) {
        g_init_err = std::string(what) + " failed: " + hipGetErrorString(e);
        release(c);
        return AH_E_HIP;
    };
    hipError_t e;
    if ((e = hipMalloc(&c->d_desc, n_real * sizeof(RealDesc))) != hipSuccess)
        return hip_fail(e, "hipMalloc(desc)");
    if ((e = hipMalloc(&c->d_step, n_real * sizeof(int64_t))) != hipSuccess)
        return hip_fail(e, "hipMalloc(step)");
    if ((e = hipMalloc(&c->d_coef, n_real * sizeof(Coef))) != hipSuccess)
        return hip_fail(e, "hipMalloc(coef)");
    if ((e = hipMalloc(&c->d_gauss, n_real * 2 * sizeof(unsigned long long))) != hipSuccess)
        return hip_fail(e, "hipMalloc(gauss)");
    if ((e = hipMemcpyAsync(c->d_desc, desc.data(), n_real * sizeof(RealDesc),
                            hipMemcpyHostToDevice, c->stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(desc)");
    if ((e = hipMemcpyAsync(c->d_step, c->step.data(), n_real * sizeof(int64_t),
                            hipMemcpyHostToDevice, c->stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(step)");
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

    size_t next = 0;
    for (int64_t i = 0; i < nsteps; ++i) {
        const bool measuring = next < meas.size() && meas_at[next] == i;
        TRY(launch_bookkeep(c, 1));
        for (int r = 0; r < c->nreal; ++r) {
            const ah_params &q = c->p[r];
            if (q.n_end > 0 && c->step[r] >= q.n_end)
                continue;
            Slot *slot = measuring && meas[next][r] ? c->d_slots + next * c->nreal + r : nullptr;
            TRY(launch_step(c, r, slot));
            ++c->step[r];
        }
        if (measuring)
            ++next;
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
        const ah_params &q = c->p[r];
        TRY(launch_measure(c, r, c->d_slots + r, wind_dev ? wind_dev + off : nullptr));
        off += 3 * (int64_t)q.nx * q.ny * q.nz;
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

int ah_gauss_residual(ah_ctx *c, double *max_abs, double *rms) {
    if (!c)
        return fail(nullptr, AH_E_INVALID, "NULL context");
    c->err.clear();
    if (!max_abs || !rms)
        return fail(c, AH_E_INVALID, "NULL output");
    TRY(launch_zero(c, c->d_gauss, c->nreal * 2 * sizeof(unsigned long long)));
    TRY(launch_bookkeep(c, 0));
    for (int r = 0; r < c->nreal; ++r) {
        const ah_params &q = c->p[r];
        const int64_t N = (int64_t)q.nx * q.ny * q.nz;
        dim3 grid(grid_for(N, kMeasureThreads, 4096));
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
        const ah_params &q = c->p[r];
        max_abs[r] = m;
        rms[r] = std::sqrt(s / ((double)q.nx * q.ny * q.nz));
    }
    return AH_OK;
}

int ah_current_planes(const ah_ctx *c, int32_t r, int32_t plane_of_field[10]) {
    if (!c || !plane_of_field || r < 0 || r >= c->nreal)
        return AH_E_INVALID;
    const int par = (int)((c->step[r] - c->p[r].step0) & 1);
    for (int f = 0; f < 10; ++f)
        plane_of_field[f] = field_plane(f, par);
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
    if (kernel < AH_KERNEL_AUTO || kernel > AH_KERNEL_TILED)
        return fail(c, AH_E_INVALID, "unknown kernel %d", kernel);
    if (chunk_z < 0 || (tile_y != 0 && !tiled_ty_valid(c->prec == AH_FP64, tile_y)))
        return fail(c, AH_E_INVALID, "tile_y must be 0, 2, 4, 8 (or 16 for FP32); chunk_z >= 0");
    if (kernel == AH_KERNEL_TILED && !tiled_ok(c))
        return fail(c, AH_E_INVALID, "tiled kernel needs nx %% 64 == 0");
    c->kernel = kernel;
    c->tile_y = tile_y;
    c->chunk_z = chunk_z;
    return AH_OK;
}

int ah_free(ah_ctx *c) {
    if (!c)
        return AH_OK;
    hipError_t e = hipStreamSynchronize(c->stream);
    release(c);
    return e == hipSuccess ? AH_OK : AH_E_HIP;
}

} // extern "C"
