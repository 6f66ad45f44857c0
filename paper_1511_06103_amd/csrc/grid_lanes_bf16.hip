// Label-parallel grid step kernels with BF16 message operands.
#include "grid_lanes.h"

namespace mf {
namespace lanes {

hipError_t launch_bf16(const StepArgs& a, int conn, int compat, hipStream_t s) {
  return ForPrec<P_BF16>::launch(a, conn, compat, s);
}

hipError_t launch_many_bf16(const ManyArgs& m, int L, int conn, int compat, hipStream_t s) {
  return ForPrec<P_BF16>::launch_many(m, L, conn, compat, s);
}

}  // namespace lanes
}  // namespace mf
