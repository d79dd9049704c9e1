// k_dslash instantiations: FP64, 12-real + U(1) angle links.
#include "dslash_kernel.h"

namespace lqcd {

template int dslash_launch_fmt<double, 8>(const DslashCall&, const DslashCfg&, hipStream_t);

}  // namespace lqcd
