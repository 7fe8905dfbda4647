// Launcher of the register weights kernel (Sec. 4.1, eqs. rbffd_linsys,
// orbffd_eq, orbffd_rhs); the kernel and its design notes are in
// weights_reg_kernel.hpp, its variants in weights_reg_3_6.hip,
// weights_reg_7_8.hip and weights_reg_9.hip.
#include "orbf_internal.hpp"
#include "weights_common.hpp"

namespace orbf {

bool launch_weights_reg_3_6(orbf_ctx* ctx, const WeightsParams& P,
                            int64_t grid, int pl, size_t dyn);
bool launch_weights_reg_7_8(orbf_ctx* ctx, const WeightsParams& P,
                            int64_t grid, int pl, size_t dyn);
bool launch_weights_reg_9(orbf_ctx* ctx, const WeightsParams& P,
                          int64_t grid, int pl, size_t dyn);

// Launch the register kernel if a variant covers K; `pl` = 1, 2 or 3 blocks
// of eight right-hand sides per pass.  Returns false if no variant covers K.
bool launch_weights_reg(orbf_ctx* ctx, const WeightsParams& P, int64_t grid,
                        int pl) {
  if (P.M > 35) return false;
  // acceptance mode always takes 16 right-hand sides per pass
  if (P.accept) pl = 2;
  if (pl < 1 || pl > 3) pl = 2;
  const size_t dyn =
      ((size_t)8 * pl * P.M + (size_t)3 * P.n * (P.l + 1)) * sizeof(double);
  return launch_weights_reg_3_6(ctx, P, grid, pl, dyn) ||
         launch_weights_reg_7_8(ctx, P, grid, pl, dyn) ||
         launch_weights_reg_9(ctx, P, grid, pl, dyn);
}

}  // namespace orbf
