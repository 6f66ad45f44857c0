// Multi-step grid kernels with F16 message operands.
#include "grid_temporal.h"

namespace mf {
namespace temporal {

hipError_t launch_f16(const StepArgs& a, int conn, int compat, int K, int ks, hipStream_t s) {
  return ForPrec<P_F16>::launch(a, conn, compat, K, ks, s);
}

}  // namespace temporal
}  // namespace mf
