// k_step_batch2_f64.hip -- the double two-steps-per-pass kernel of many
// realizations (the batched form), apart from the one-realization kernel: it
// holds more registers (the item loop), and the scheduler that helps that one
// makes this one spill more.
#include "k_step_tiled2.hpp"

namespace ah {

template int batch2_dispatch_t<double>(int, bool, const RealDesc *, const Coef *, const BatchItem *,
                                   int, int, int, hipStream_t, int *);

} // namespace ah
