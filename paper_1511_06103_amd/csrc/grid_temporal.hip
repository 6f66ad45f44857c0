// Dispatch of the multi-step (temporal blocking) grid kernels; the kernel
// itself is in grid_temporal.h, instantiated per message precision in
// grid_temporal_{f32,bf16,f16}.hip so the three compile in parallel.
#include "grid_temporal.h"

namespace mf {

int grid_max_steps_per_launch(int L, int prec) {
  const size_t per = (size_t)(prec == MF_P_F32 ? 12 : 8);
  const size_t kMax = 160 * 1024;
  const int lp = L == 2 ? 2 : L == 21 ? 21 : L <= 4 ? 4 : L <= 8 ? 8 : L <= 16 ? 16 : 32;
  if ((size_t)lp * 24 * 24 * per <= kMax) return 4;
  if ((size_t)lp * 22 * 22 * per <= kMax) return 3;
  return 2;
}

hipError_t launch_grid_multi_step(const StepArgs& a, int conn, int compat, int prec, int K, int ks,
                                  hipStream_t s) {
  switch (prec) {
    case MF_P_F32: return temporal::launch_f32(a, conn, compat, K, ks, s);
    case MF_P_BF16MSG: return temporal::launch_bf16(a, conn, compat, K, ks, s);
    default: return temporal::launch_f16(a, conn, compat, K, ks, s);
  }
}

}  // namespace mf
