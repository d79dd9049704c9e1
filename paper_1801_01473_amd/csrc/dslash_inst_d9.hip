// k_dslash instantiations: FP64, 18-real links.
#include "dslash_kernel.h"

namespace lqcd {

template int dslash_launch_fmt<double, 9>(const DslashCall&, const DslashCfg&, hipStream_t);

// The FP64 residual mode (b - A x with FP64 18-real links; FP32 or FP64 store).
int dslash_launch_res(const DslashCall& c, const DslashCfg& cfg, hipStream_t st) {
  if (c.r_prec == LQCD_F32) return launch_b<double, 9, DM_RES, float>(c, cfg, st);
  return launch_b<double, 9, DM_RES, double>(c, cfg, st);
}

}  // namespace lqcd
