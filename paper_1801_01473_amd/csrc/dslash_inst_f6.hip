// k_dslash instantiations: FP32, 12-real links.
#include "dslash_kernel.h"

namespace lqcd {

template int dslash_launch_fmt<float, 6>(const DslashCall&, const DslashCfg&, hipStream_t);

}  // namespace lqcd
