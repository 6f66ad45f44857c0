// Grid step kernels of the non-fixed step rules (mf_rule): the single-step
// tile body of grid_lanes.h (one lane per node, 64 x 4 tiles, FP32
// messages) with the rule's update in place of the fixed-step one.
#include "grid_lanes.h"

namespace mf {
namespace {

// Tiles dealt to workgroups XCD by XCD, as in the fixed-step kernel.
template <int LG, int LC, int CONN, int COMPAT, int RULE>
__global__ __launch_bounds__(64 * 4) void rule_step_kernel(StepArgs a, RuleArgs r) {
  __shared__ lanes::Smem<LG, 1, 64, 4, P_F32> sm;
  const int tiles_x = (a.W + 63) / 64, per_item = tiles_x * ((a.H + 3) / 4);
  const int t = lanes::xcd_tile(blockIdx.x, per_item * a.B);
  const int b = t / per_item, q = t - b * per_item;
  const int ty = q / tiles_x, tx = q - ty * tiles_x;
  lanes::tile_step<LG, 1, LC, CONN, COMPAT, P_F32, 64, 4, RULE>(a, 1.0f - a.alpha, b, tx * 64, ty * 4, sm, &r);
}

template <int LG, int LC, int RULE>
hipError_t go(const StepArgs& a, const RuleArgs& r, int conn, int compat, hipStream_t s) {
  const dim3 grid(((a.W + 63) / 64) * ((a.H + 3) / 4) * a.B), block(64 * 4);
  if (conn == 4) {
    if (compat == MF_COMPAT_POTTS)
      hipLaunchKernelGGL((rule_step_kernel<LG, LC, 4, MF_COMPAT_POTTS, RULE>), grid, block, 0, s, a, r);
    else
      hipLaunchKernelGGL((rule_step_kernel<LG, LC, 4, MF_COMPAT_GENERAL, RULE>), grid, block, 0, s, a, r);
  } else {
    if (compat == MF_COMPAT_POTTS)
      hipLaunchKernelGGL((rule_step_kernel<LG, LC, 8, MF_COMPAT_POTTS, RULE>), grid, block, 0, s, a, r);
    else
      hipLaunchKernelGGL((rule_step_kernel<LG, LC, 8, MF_COMPAT_GENERAL, RULE>), grid, block, 0, s, a, r);
  }
  return hipGetLastError();
}

// Label slots as for the fixed-step single-step kernel.
template <int RULE>
hipError_t by_labels(const StepArgs& a, const RuleArgs& r, int conn, int compat, hipStream_t s) {
  switch (lanes::slots_for(a.L)) {
    case 2: return a.L == 2 ? go<2, 2, RULE>(a, r, conn, compat, s) : go<2, 0, RULE>(a, r, conn, compat, s);
    case 21: return go<21, 21, RULE>(a, r, conn, compat, s);
    case 4: return go<4, 0, RULE>(a, r, conn, compat, s);
    case 8: return go<8, 0, RULE>(a, r, conn, compat, s);
    case 16: return go<16, 0, RULE>(a, r, conn, compat, s);
    default: return go<32, 0, RULE>(a, r, conn, compat, s);
  }
}

}  // namespace

hipError_t launch_grid_rule_step(const StepArgs& a, const RuleArgs& r, int conn, int compat, int rule,
                                 hipStream_t s) {
  switch (rule) {
    case MF_RULE_ADAPTIVE:
      if (a.L != 2) return hipErrorInvalidValue;
      return go<2, 2, MF_RULE_ADAPTIVE>(a, r, conn, compat, s);
    case MF_RULE_ADHOC: return by_labels<MF_RULE_ADHOC>(a, r, conn, compat, s);
    case MF_RULE_MOMENTUM: return by_labels<MF_RULE_MOMENTUM>(a, r, conn, compat, s);
    case MF_RULE_ADAM: return by_labels<MF_RULE_ADAM>(a, r, conn, compat, s);
    case MF_RULE_SWEEP: return by_labels<MF_RULE_SWEEP>(a, r, conn, compat, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mf
