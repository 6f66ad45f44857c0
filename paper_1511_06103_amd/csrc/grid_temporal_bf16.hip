// Multi-step grid kernels with BF16 message operands.
#include "grid_temporal.h"

namespace mf {
namespace temporal {

hipError_t launch_bf16(const StepArgs& a, int conn, int compat, int K, int ks, hipStream_t s) {
  return ForPrec<P_BF16>::launch(a, conn, compat, K, ks, s);
}

}  // namespace temporal
}  // namespace mf
