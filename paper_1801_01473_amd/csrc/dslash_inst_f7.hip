// k_dslash instantiations: FP32, 12-real + determinant links.
#include "dslash_kernel.h"

namespace lqcd {

template int dslash_launch_fmt<float, 7>(const DslashCall&, const DslashCfg&, hipStream_t);

}  // namespace lqcd
