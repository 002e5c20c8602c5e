// k_step_tiled2_f64.hip -- the double two-steps-per-pass kernel of one
// realization, compiled on its own so that its code generation can differ from
// the rest of the library's.
#include "k_step_tiled2.hpp"

namespace ah {

template int launch_step_tiled2_t<double>(const RealDesc *, const Coef *, int, int, int, int, int, int,
                                      int, int, hipStream_t);

} // namespace ah
