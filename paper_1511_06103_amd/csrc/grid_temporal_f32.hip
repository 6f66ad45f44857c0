// Multi-step grid kernels with F32 message operands.
#include "grid_temporal.h"

namespace mf {
namespace temporal {

hipError_t launch_f32(const StepArgs& a, int conn, int compat, int K, int ks, hipStream_t s) {
  return ForPrec<P_F32>::launch(a, conn, compat, K, ks, s);
}

}  // namespace temporal
}  // namespace mf
