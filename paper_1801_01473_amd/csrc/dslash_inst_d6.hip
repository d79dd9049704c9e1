// k_dslash instantiations: FP64, 12-real links.
#include "dslash_kernel.h"

namespace lqcd {

template int dslash_launch_fmt<double, 6>(const DslashCall&, const DslashCfg&, hipStream_t);

}  // namespace lqcd
