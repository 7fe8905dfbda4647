// Register weights kernel variants with L = 9 row blocks (the kernel is
// in weights_reg_kernel.hpp).
#include "weights_reg_kernel.hpp"

namespace orbf {

bool launch_weights_reg_9(orbf_ctx* ctx, const WeightsParams& P,
                          int64_t grid, int pl, size_t dyn) {
  if (P.K <= 72) {
    launch_reg_variant<9>(ctx, P, grid, pl, dyn);
    return true;
  }
  return false;
}

}  // namespace orbf
