// k_dslash instantiations: FP32, 18-real links.
#include "dslash_kernel.h"

namespace lqcd {

template int dslash_launch_fmt<float, 9>(const DslashCall&, const DslashCfg&, hipStream_t);

}  // namespace lqcd
