// Label-parallel grid step kernels with F16 message operands.
#include "grid_lanes.h"

namespace mf {
namespace lanes {

hipError_t launch_f16(const StepArgs& a, int conn, int compat, hipStream_t s) {
  return ForPrec<P_F16>::launch(a, conn, compat, s);
}

hipError_t launch_many_f16(const ManyArgs& m, int L, int conn, int compat, hipStream_t s) {
  return ForPrec<P_F16>::launch_many(m, L, conn, compat, s);
}

}  // namespace lanes
}  // namespace mf
