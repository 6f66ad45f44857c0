// Dispatch of the multi-step (temporal blocking) grid kernels; the kernel
// itself is in grid_temporal.h, instantiated per message precision in
// grid_temporal_{f32,bf16,f16}.hip so the three compile in parallel.
#include "grid_temporal.h"

namespace mf {

int grid_max_steps_per_launch(int L, int compat, int prec) {
  switch (prec) {
    case MF_P_F32: return temporal::ForPrec<P_F32>::kmax(L, compat);
    case MF_P_BF16MSG: return temporal::ForPrec<P_BF16>::kmax(L, compat);
    default: return temporal::ForPrec<P_F16>::kmax(L, compat);
  }
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
