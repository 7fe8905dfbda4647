// Register weights kernel variants with L = 7, 8 row blocks (the kernel is
// in weights_reg_kernel.hpp).
#include "weights_reg_kernel.hpp"

namespace orbf {

bool launch_weights_reg_7_8(orbf_ctx* ctx, const WeightsParams& P,
                            int64_t grid, int pl, size_t dyn) {
  if (P.K <= 56) {
    launch_reg_variant<7>(ctx, P, grid, pl, dyn);
    return true;
  }
  if (P.K <= 64) {
    launch_reg_variant<8>(ctx, P, grid, pl, dyn);
    return true;
  }
  return false;
}

}  // namespace orbf
