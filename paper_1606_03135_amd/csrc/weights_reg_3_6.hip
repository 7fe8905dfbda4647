// Register weights kernel variants with L = 3, 4, 5, 6 row blocks (the kernel is
// in weights_reg_kernel.hpp).
#include "weights_reg_kernel.hpp"

namespace orbf {

bool launch_weights_reg_3_6(orbf_ctx* ctx, const WeightsParams& P,
                            int64_t grid, int pl, size_t dyn) {
  if (P.K <= 24) {
    launch_reg_variant<3>(ctx, P, grid, pl, dyn);
    return true;
  }
  if (P.K <= 32) {
    launch_reg_variant<4>(ctx, P, grid, pl, dyn);
    return true;
  }
  if (P.K <= 40) {
    launch_reg_variant<5>(ctx, P, grid, pl, dyn);
    return true;
  }
  if (P.K <= 48) {
    launch_reg_variant<6>(ctx, P, grid, pl, dyn);
    return true;
  }
  return false;
}

}  // namespace orbf
