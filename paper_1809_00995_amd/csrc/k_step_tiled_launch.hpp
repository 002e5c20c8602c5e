// k_step_tiled_launch.hpp -- host launchers of the tiled single-step kernels
// (k_step_tiled.hpp), single realizations and the batched form.  Kept apart
// from the kernels: a launcher's body instantiates every kernel it can launch
// in the translation unit that includes it, so only the C ABI's unit does.
#pragma once

#include "k_measure_tiled.hpp"
#include "k_step_tiled.hpp"
#include "k_step_tiled2_api.hpp"

namespace ah {

// Tile height and z-chunk used when the caller leaves them at 0.
inline void tiled_defaults(bool fp64, int nx, int ny, int nz, int &ty, int &cz) {
    if (ty <= 0)
        ty = fp64 ? 4 : 8;
    if (cz <= 0) {
        const long tiles_xy = (long)(nx / 64) * ((ny + ty - 1) / ty);
        long chunks = (4096 + tiles_xy - 1) / tiles_xy;       // aim at ~4096 blocks
        const long max_chunks = (nz + 7) / 8;                  // but at least ~8 planes each
        if (chunks > max_chunks)
            chunks = max_chunks;
        if (chunks < 1)
            chunks = 1;
        cz = (int)((nz + chunks - 1) / chunks);
    }
}

template <typename T, int TY, int MODE>
hipError_t launch_tiled_ty(const RealDesc *desc, const Coef *coef, int r, int nx, int ny, int nz,
                           int cz, Slot *slot, hipStream_t stream) {
    const long blocks = (long)(nx / 64) * ((ny + TY - 1) / TY) * ((nz + cz - 1) / cz);
    hipLaunchKernelGGL((k_step_tiled<T, TY, MODE>), dim3((unsigned)blocks), dim3(64 * TY), 0,
                       stream, desc, coef, r, cz, slot, 0);
    return hipGetLastError();
}

template <typename T, int MODE>
hipError_t launch_tiled_mode(int ty, const RealDesc *desc, const Coef *coef, int r, int nx, int ny,
                             int nz, int cz, Slot *slot, hipStream_t stream) {
    // The measuring modes hold ~220 VGPRs: keep them at tiles that do not
    // spill (FP32 <= 8 rows, FP64 <= 4).  The update is the same arithmetic
    // for every tile height, so this only changes the order of the sums.
    constexpr bool MEAS = MODE != MODE_STEP;
    constexpr int TYMAX = MEAS ? (sizeof(T) == 4 ? 8 : 4) : (sizeof(T) == 4 ? 16 : 8);
    if (ty > TYMAX)
        ty = TYMAX;
    switch (ty) {
    case 2: return launch_tiled_ty<T, 2, MODE>(desc, coef, r, nx, ny, nz, cz, slot, stream);
    case 4: return launch_tiled_ty<T, 4, MODE>(desc, coef, r, nx, ny, nz, cz, slot, stream);
    default:
        if constexpr (TYMAX >= 16)
            if (ty == 16)
                return launch_tiled_ty<T, 16, MODE>(desc, coef, r, nx, ny, nz, cz, slot, stream);
        if constexpr (TYMAX >= 8)
            return launch_tiled_ty<T, 8, MODE>(desc, coef, r, nx, ny, nz, cz, slot, stream);
        return hipErrorInvalidValue;
    }
}

// Valid tile heights: FP32 2, 4, 8, 16; FP64 2, 4, 8.
inline bool tiled_ty_valid(bool fp64, int ty) {
    return ty == 2 || ty == 4 || ty == 8 || (!fp64 && ty == 16);
}

// Launch one tiled kernel (MODE_STEP or MODE_STEP_MEASURE) for realization r.
inline int launch_step_tiled(bool fp64, int mode, const RealDesc *desc, const Coef *coef, int r,
                             int nx, int ny, int nz, int tile_y, int chunk_z, Slot *slot,
                             hipStream_t stream) {
    int ty = tile_y, cz = chunk_z;
    // the measuring mode holds ~160-230 VGPRs: 4-row tiles (two or three blocks
    // per CU) are its default
    if (ty <= 0 && mode != MODE_STEP)
        ty = 4;
    tiled_defaults(fp64, nx, ny, nz, ty, cz);
    if (nx % 64 != 0 || !tiled_ty_valid(fp64, ty) || cz < 1)
        return (int)hipErrorInvalidValue;
    hipError_t e;
    if (fp64)
        e = mode == MODE_STEP ? launch_tiled_mode<double, MODE_STEP>(ty, desc, coef, r, nx, ny, nz, cz, slot, stream)
                              : launch_tiled_mode<double, MODE_STEP_MEASURE>(ty, desc, coef, r, nx, ny, nz, cz, slot, stream);
    else
        e = mode == MODE_STEP ? launch_tiled_mode<float, MODE_STEP>(ty, desc, coef, r, nx, ny, nz, cz, slot, stream)
                              : launch_tiled_mode<float, MODE_STEP_MEASURE>(ty, desc, coef, r, nx, ny, nz, cz, slot, stream);
    return (int)e;
}

template <typename T, int TY>
hipError_t launch_measure_ty(const RealDesc *desc, const Coef *coef, int r, int nx, int ny, int nz,
                             int cz, bool off32, Slot *slot, int8_t *wind, hipStream_t stream) {
    const long blocks = (long)(nx / 64) * ((ny + TY - 1) / TY) * ((nz + cz - 1) / cz);
    if (off32)
        hipLaunchKernelGGL((k_measure_tiled<T, TY, true>), dim3((unsigned)blocks), dim3(64 * TY), 0,
                           stream, desc, coef, r, cz, slot, wind);
    else
        hipLaunchKernelGGL((k_measure_tiled<T, TY, false>), dim3((unsigned)blocks), dim3(64 * TY), 0,
                           stream, desc, coef, r, cz, slot, wind);
    return hipGetLastError();
}

// Launch the read-only measuring pass for realization r: tile heights 2, 4
// (the default) or 8; other values take the default.  stored_sites: the
// elements of one field plane (nx ny (nz + 2 z_halo)), which decides the
// address form.
inline int launch_measure_tiled(bool fp64, const RealDesc *desc, const Coef *coef, int r, int nx,
                                int ny, int nz, long stored_sites, int tile_y, int chunk_z,
                                Slot *slot, int8_t *wind, hipStream_t stream) {
    int ty = (tile_y == 2 || tile_y == 4 || tile_y == 8) ? tile_y : 4, cz = chunk_z;
    tiled_defaults(fp64, nx, ny, nz, ty, cz);
    if (nx % 64 != 0 || cz < 1)
        return (int)hipErrorInvalidValue;
    const bool off32 = fits_off32(stored_sites, fp64 ? 8 : 4);
    hipError_t e;
#define AH_MEAS(T)                                                                                  \
    (ty == 2 ? launch_measure_ty<T, 2>(desc, coef, r, nx, ny, nz, cz, off32, slot, wind, stream)    \
     : ty == 8 ? launch_measure_ty<T, 8>(desc, coef, r, nx, ny, nz, cz, off32, slot, wind, stream)  \
               : launch_measure_ty<T, 4>(desc, coef, r, nx, ny, nz, cz, off32, slot, wind, stream))
    e = fp64 ? AH_MEAS(double) : AH_MEAS(float);
#undef AH_MEAS
    return (int)e;
}

// Tile height of the batched read-only measuring pass.
constexpr int kMeasureBatchTY = 4;

template <typename T, bool OFF32>
hipError_t measure_batch_t(const RealDesc *desc, const Coef *coef, const BatchItem *items,
                           int n_items, Slot *slots, int grid, hipStream_t stream, int *grid_out) {
    constexpr int TY = kMeasureBatchTY;
    if (grid_out) {
        int per_cu = 0, dev = 0, cus = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_measure_batch<T, TY, OFF32>,
                                                             64 * TY, 0);
        *grid_out = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
        return e;
    }
    if (grid > n_items)
        grid = n_items;
    if (grid < 1)
        return hipSuccess;
    hipLaunchKernelGGL((k_measure_batch<T, TY, OFF32>), dim3((unsigned)grid), dim3(64 * TY), 0,
                       stream, desc, coef, items, n_items, slots);
    return hipGetLastError();
}

// The batched read-only measuring pass: with grid_out != NULL only the
// resident-block count (occupancy x compute units) is returned; otherwise the
// kernel is launched on `grid` blocks over the n_items items.  off32: every
// realization's planes are below 4 GiB.
inline int measure_batch_dispatch(bool fp64, bool off32, const RealDesc *desc, const Coef *coef,
                                  const BatchItem *items, int n_items, Slot *slots, int grid,
                                  hipStream_t stream, int *grid_out) {
    hipError_t e;
    if (fp64)
        e = off32 ? measure_batch_t<double, true>(desc, coef, items, n_items, slots, grid, stream, grid_out)
                  : measure_batch_t<double, false>(desc, coef, items, n_items, slots, grid, stream, grid_out);
    else
        e = off32 ? measure_batch_t<float, true>(desc, coef, items, n_items, slots, grid, stream, grid_out)
                  : measure_batch_t<float, false>(desc, coef, items, n_items, slots, grid, stream, grid_out);
    return (int)e;
}

// Largest tile height of a mode (the measuring modes hold ~220 VGPRs).
inline int tiled_ty_max(bool fp64, int mode) {
    return mode != MODE_STEP ? (fp64 ? 4 : 8) : (fp64 ? 8 : 16);
}

template <typename T, int TY, int MODE>
hipError_t batch_grid_ty(int *grid) {
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step_batch<T, TY, MODE>, 64 * TY, 0);
    *grid = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
    return e;
}

template <typename T, int TY, int MODE>
hipError_t launch_batch_ty(const RealDesc *desc, const Coef *coef, const BatchItem *items,
                           int n_items, Slot *slots, int grid, hipStream_t stream) {
    if (grid > n_items)
        grid = n_items;
    if (grid < 1)
        return hipSuccess;
    hipLaunchKernelGGL((k_step_batch<T, TY, MODE>), dim3((unsigned)grid), dim3(64 * TY), 0, stream,
                       desc, coef, items, n_items, slots);
    return hipGetLastError();
}

// Dispatch over (precision, tile height, mode) of the batched kernel.  With
// grid_out != NULL only the resident-block count of that kernel is returned
// (occupancy x compute units); otherwise the kernel is launched on `grid`
// blocks.  Tile heights: FP32 2, 4, 8 (16 for MODE_STEP); FP64 2, 4 (8 for
// MODE_STEP).
inline int batch_dispatch(bool fp64, int mode, int ty, const RealDesc *desc, const Coef *coef,
                          const BatchItem *items, int n_items, Slot *slots, int grid,
                          hipStream_t stream, int *grid_out) {
    if (ty > tiled_ty_max(fp64, mode) || !tiled_ty_valid(fp64, ty))
        return (int)hipErrorInvalidValue;
#define AH_BATCH(T, TY_, M)                                                                        \
    (grid_out ? batch_grid_ty<T, TY_, M>(grid_out)                                                 \
              : launch_batch_ty<T, TY_, M>(desc, coef, items, n_items, slots, grid, stream))
    hipError_t e = hipErrorInvalidValue;
    if (fp64) {
        if (mode == MODE_STEP)
            e = ty == 2 ? AH_BATCH(double, 2, MODE_STEP) : ty == 4 ? AH_BATCH(double, 4, MODE_STEP)
                                                                   : AH_BATCH(double, 8, MODE_STEP);
        else
            e = ty == 2 ? AH_BATCH(double, 2, MODE_STEP_MEASURE) : AH_BATCH(double, 4, MODE_STEP_MEASURE);
    } else {
        if (mode == MODE_STEP)
            e = ty == 2 ? AH_BATCH(float, 2, MODE_STEP) : ty == 4 ? AH_BATCH(float, 4, MODE_STEP)
              : ty == 8 ? AH_BATCH(float, 8, MODE_STEP) : AH_BATCH(float, 16, MODE_STEP);
        else
            e = ty == 2 ? AH_BATCH(float, 2, MODE_STEP_MEASURE)
              : ty == 4 ? AH_BATCH(float, 4, MODE_STEP_MEASURE) : AH_BATCH(float, 8, MODE_STEP_MEASURE);
    }
#undef AH_BATCH
    return (int)e;
}

} // namespace ah
