// k_step_tiled2_api.hpp -- host interface of the two-steps-per-pass kernels
// (k_step_tiled2.hpp): tile-height choice and the launchers.  The kernels are
// compiled in translation units of their own, one per element type
// (k_step_tiled2_f32.hip, k_step_tiled2_f64.hip), so that each can take the
// code-generation options measured best for it; this header carries no device
// code.
#pragma once

#include <hip/hip_runtime.h>

#include "ah_device.hpp"

namespace ah {

// Tile heights of the two-step kernel.  LDS per block: FP32 112 KB at TY = 8,
// 122 KB at TY = 9; FP64 143 KB at TY = 4, 163 KB at TY = 5 (a workgroup may
// hold up to 160 KiB on gfx950).  TY = 9 (FP32) and TY = 5 (FP64) give 12 and
// 8 wavefronts, an equal number on each of a CU's four SIMDs.
inline bool tiled2_ty_valid(bool fp64, int ty) {
    return fp64 ? (ty == 4 || ty == 5) : (ty == 4 || ty == 8 || ty == 9);
}

// Default tile height for lattices with the given y extents (weights: sites
// per unit of y): the balanced height (9 FP32, 5 FP64) unless its ragged last
// rows of tiles idle more than 2 % of the sites beyond the smaller height's.
inline int tiled2_default_ty(bool fp64, const int *ny, const long *weight, int n) {
    const int big = fp64 ? 5 : 9, small = big - 1;
    double pad_big = 0, pad_small = 0, total = 0;
    for (int i = 0; i < n; ++i) {
        pad_big += (double)weight[i] * ((ny[i] + big - 1) / big * big - ny[i]);
        pad_small += (double)weight[i] * ((ny[i] + small - 1) / small * small - ny[i]);
        total += (double)weight[i] * ny[i];
    }
    return pad_big <= pad_small + 0.02 * total ? big : small;
}

// Resident blocks of the two-step kernel on the whole chip: one per compute
// unit (its LDS holds one block), on the 256 compute units of an MI355X.
constexpr long kTiled2Slots = 256;

// Default tile height and z-chunk of the two-step kernel (values > 0 are kept).
// Chunks hold at most 192 planes (at 1024^3 FP32, 2 chunks of 512 planes take
// 23.1 ms per pair, 4 of 256 23.8 ms, 5-7 of 205-147 planes 21.4-21.5 ms) and
// at least 32 where nz allows.  For one launch over one realization, a block
// walks its chunk at a pace set by its own compute unit, so the launch lasts
// about (rounds of kTiled2Slots blocks) x (planes per chunk + 2) x (a block's
// time per plane); the longest chunks within 1 % of the least such cost are
// taken (measured per pair: FP64 512^3 171 -> 128 planes 6.49 -> 6.32 ms, FP64
// 384^3 77 -> 64 planes 3.00 -> 2.79 ms, FP64 256^3 32 -> 43 planes 0.91 ->
// 0.85 ms), and the lower tile height where that cost is more than 2 % below
// the default height's (FP32, 9 -> 8 rows: 1024 x 1024 x 128 2.86 -> 2.74 ms,
// 384^3 1.30 -> 1.22 ms, 256^3 0.364 -> 0.350 ms, 768^3 9.63 -> 9.34 ms; 512^3
// and 1024^3 keep 9 rows and 103 and 171 planes).  Work lists of the batched
// launch (one_launch = false) share the chip between realizations and aim at
// ~2048 blocks per realization instead.
// Chunk count of the one-launch cost model for tile height ty: the longest
// chunks within 1 % of the least cost; *cost_out gets that cost, in plane
// times of a block of the default height.
inline long tiled2_chunks(bool fp64, int nx, int ny, int nz, int ty, double *cost_out) {
    const long tiles_xy = (long)(nx / 64) * ((ny + ty - 1) / ty);
    long lo = (nz + 191) / 192, hi = (nz + 31) / 32;
    if (lo < 1)
        lo = 1;
    if (hi < lo)
        hi = lo;
    // a block's time per plane relative to one of the default height: its rows,
    // and the 1.6 % (FP32, 8 against 9 rows) or 8.5 % (FP64, 4 against 5) more
    // time per site that the relatively larger ring of the lower tile costs
    const int big = fp64 ? 5 : 9;
    const double per_block = ty == big ? 1.0 : (double)ty / big * (fp64 ? 1.085 : 1.016);
    auto cost = [&](long k) {
        const long len = (nz + k - 1) / k, used = (nz + len - 1) / len;
        return (double)((tiles_xy * used + kTiled2Slots - 1) / kTiled2Slots) * (len + 2) *
               per_block;
    };
    double least = cost(lo);
    for (long k = lo + 1; k <= hi; ++k)
        least = cost(k) < least ? cost(k) : least;
    long chunks = lo;
    while (cost(chunks) > 1.01 * least)   // ends at the least-cost count at the latest
        ++chunks;
    if (cost_out)
        *cost_out = cost(chunks);
    return chunks;
}

inline void tiled2_defaults(bool fp64, int nx, int ny, int nz, int &ty, int &cz,
                            bool one_launch = true) {
    const bool ty_default = ty <= 0;
    if (ty_default) {
        const long w = (long)nx * nz;
        ty = tiled2_default_ty(fp64, &ny, &w, 1);
    }
    if (cz > 0)
        return;
    long chunks;
    if (one_launch) {
        double c_ty = 0;
        chunks = tiled2_chunks(fp64, nx, ny, nz, ty, &c_ty);
        if (ty_default) {
            // the other height when its rounds of blocks fit the chip more than 2 %
            // better (a 1024 x 1024 x 128 slab: 2048 tiles of 8 rows are 8 full
            // rounds, 1824 of 9 rows 7.1)
            const int other = ty == (fp64 ? 5 : 9) ? ty - 1 : ty + 1;
            double c_o = 0;
            const long k_o = tiled2_chunks(fp64, nx, ny, nz, other, &c_o);
            if (c_o < 0.98 * c_ty) {
                ty = other;
                chunks = k_o;
            }
        }
    } else {
        const long tiles_xy = (long)(nx / 64) * ((ny + ty - 1) / ty);
        long lo = (nz + 191) / 192, hi = (nz + 31) / 32;
        if (lo < 1)
            lo = 1;
        if (hi < lo)
            hi = lo;
        chunks = (2048 + tiles_xy - 1) / tiles_xy;
        chunks = chunks < lo ? lo : (chunks > hi ? hi : chunks);
    }
    cz = (int)((nz + chunks - 1) / chunks);
}

// Whether every plane of an nx*ny*nz lattice of elem-byte values is below
// 4 GiB (32-bit byte offsets).
inline bool fits_off32(long n_sites, int elem) {
    return (unsigned long long)n_sites * (unsigned long long)elem <= (1ull << 32);
}

// Defined in k_step_tiled2.hpp, instantiated for float and double in their own
// translation units.
template <typename T>
int launch_step_tiled2_t(const RealDesc *desc, const Coef *coef, int r, int nreal, int nx, int ny,
                         int nz, int zh, int ty, int cz, hipStream_t stream);
template <typename T>
int batch2_dispatch_t(int ty, bool off32, const RealDesc *desc, const Coef *coef,
                      const BatchItem *items, int n_items, int nreal, int grid, hipStream_t stream,
                      int *grid_out);
extern template int launch_step_tiled2_t<float>(const RealDesc *, const Coef *, int, int, int, int,
                                                int, int, int, int, hipStream_t);
extern template int launch_step_tiled2_t<double>(const RealDesc *, const Coef *, int, int, int,
                                                 int, int, int, int, int, hipStream_t);
extern template int batch2_dispatch_t<float>(int, bool, const RealDesc *, const Coef *,
                                             const BatchItem *, int, int, int, hipStream_t, int *);
extern template int batch2_dispatch_t<double>(int, bool, const RealDesc *, const Coef *,
                                              const BatchItem *, int, int, int, hipStream_t, int *);

// Launch the two-step kernel for realization r (nx % 64 == 0, 20-plane layout;
// nz planes advanced, zh halo planes a side for a slab); tile_y, chunk_z 0
// pick the defaults.
inline int launch_step_tiled2(bool fp64, const RealDesc *desc, const Coef *coef, int r, int nreal,
                              int nx, int ny, int nz, int zh, int tile_y, int chunk_z,
                              hipStream_t stream) {
    int ty = tile_y, cz = chunk_z;
    tiled2_defaults(fp64, nx, ny, nz, ty, cz);
    if (nx % 64 != 0 || !tiled2_ty_valid(fp64, ty) || cz < 1)
        return (int)hipErrorInvalidValue;
    return fp64 ? launch_step_tiled2_t<double>(desc, coef, r, nreal, nx, ny, nz, zh, ty, cz, stream)
                : launch_step_tiled2_t<float>(desc, coef, r, nreal, nx, ny, nz, zh, ty, cz, stream);
}

// The batched two-step kernel: with grid_out != NULL only its resident-block
// count (occupancy x compute units) is returned; otherwise it is launched on
// `grid` blocks.  off32: every realization's planes are below 4 GiB.
inline int batch2_dispatch(bool fp64, int ty, bool off32, const RealDesc *desc, const Coef *coef,
                           const BatchItem *items, int n_items, int nreal, int grid,
                           hipStream_t stream, int *grid_out) {
    if (!tiled2_ty_valid(fp64, ty))
        return (int)hipErrorInvalidValue;
    return fp64 ? batch2_dispatch_t<double>(ty, off32, desc, coef, items, n_items, nreal, grid,
                                            stream, grid_out)
                : batch2_dispatch_t<float>(ty, off32, desc, coef, items, n_items, nreal, grid,
                                           stream, grid_out);
}

} // namespace ah
