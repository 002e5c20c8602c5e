// k_step_tiled2_f32.hip -- the float two-steps-per-pass kernels (one and
// many realizations), compiled on their own so that their code generation can
// differ from the rest of the library's.
#include "k_step_tiled2.hpp"

namespace ah {

template int launch_step_tiled2_t<float>(const RealDesc *, const Coef *, int, int, int, int, int, int,
                                      int, int, hipStream_t);
template int batch2_dispatch_t<float>(int, bool, const RealDesc *, const Coef *, const BatchItem *,
                                   int, int, int, hipStream_t, int *);

} // namespace ah
