// k_dslash instantiations: FP32, 12-real + U(1) angle links.
#include "dslash_kernel.h"

namespace lqcd {

template int dslash_launch_fmt<float, 8>(const DslashCall&, const DslashCfg&, hipStream_t);

}  // namespace lqcd
