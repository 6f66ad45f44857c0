// Dispatch of the label-parallel grid step kernels; the kernels are in
// grid_lanes.h and are instantiated per message precision in
// grid_lanes_{f32,bf16,f16}.hip so the three compile in parallel.
#include "grid_lanes.h"

namespace mf {

int grid_lanes_tiles(int B, int H, int W, int L) { return lanes::tiles(B, H, W, L); }

hipError_t launch_grid_step_lanes(const StepArgs& a, int conn, int compat, int prec, hipStream_t s) {
  if (a.L > kSmallLabels) return launch_grid_step_large(a, conn, compat, prec, s);
  switch (prec) {
    case MF_P_F32: return lanes::launch_f32(a, conn, compat, s);
    case MF_P_BF16MSG: return lanes::launch_bf16(a, conn, compat, s);
    default: return lanes::launch_f16(a, conn, compat, s);
  }
}

hipError_t launch_grid_step_lanes_many(const ManyArgs& m, int L, int conn, int compat, int prec, hipStream_t s) {
  switch (prec) {
    case MF_P_F32: return lanes::launch_many_f32(m, L, conn, compat, s);
    case MF_P_BF16MSG: return lanes::launch_many_bf16(m, L, conn, compat, s);
    default: return lanes::launch_many_f16(m, L, conn, compat, s);
  }
}

}  // namespace mf
