// k_step_tiled.hpp -- z-streaming tiled step kernel (not yet available).
#pragma once

#include "ah_device.hpp"

namespace ah {

inline int launch_step_tiled(bool fp64, const RealDesc *desc, const Coef *coef, int r, int nx,
                             int ny, int nz, int tile_y, int chunk_z, hipStream_t stream) {
    (void)fp64; (void)desc; (void)coef; (void)r; (void)nx; (void)ny; (void)nz;
    (void)tile_y; (void)chunk_z; (void)stream;
    return (int)hipErrorNotSupported;
}

} // namespace ah
