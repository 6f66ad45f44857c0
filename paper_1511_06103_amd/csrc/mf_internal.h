// Internal declarations shared by the host library and the kernel files.
// Not part of the public ABI (see include/mf.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "mf.h"

namespace mf {

// Grid step tile: TX x TY nodes per 256-thread workgroup, one node per
// thread, with a one-node halo staged in LDS.
constexpr int kTileX = 64;
constexpr int kTileY = 4;
constexpr int kThreads = kTileX * kTileY;

struct StepArgs {
  const float* unary;      // [B][L][N]
  const float* state_in;   // [B][L][N]
  float* state_out;        // [B][L][N]
  const float* theta;      // [L][L] (general) or nullptr
  int B, L, N, H, W;
  float alpha;
  float potts_w;
};

struct FreeEnergyArgs {
  const float* unary;
  const float* state;
  const float* theta;
  int B, L, N, H, W;
  float potts_w;
  double* partials;        // [B][n_blocks]
  int n_blocks;            // workgroups per batch item
};

// Workspace layout (offsets in bytes from the 256-aligned workspace start).
struct WorkspaceLayout {
  size_t flags = 0;        // int32[64]: [0] non-finite input seen
  size_t partials = 0;     // double[B][n_blocks]
  size_t f_out = 0;        // double[B]
  size_t total = 0;
  int n_blocks = 0;
};

// Launchers (return hipSuccess or the launch error).
hipError_t launch_init(const float* unary, float* state, int B, int L, int N, int mode,
                       int* flags, hipStream_t s);
hipError_t launch_grid_step(const StepArgs& a, int conn, int compat, int precision, hipStream_t s);
// ks <= K sub-steps in one launch of the K-halo kernel; K <= grid_max_steps_per_launch.
hipError_t launch_grid_multi_step(const StepArgs& a, int conn, int compat, int precision, int K, int ks,
                                  hipStream_t s);
int grid_max_steps_per_launch(int L, int precision);
hipError_t launch_grid_free_energy(const FreeEnergyArgs& a, int conn, int compat, double* f_out,
                                   hipStream_t s);
hipError_t launch_clear_flags(int* flags, int n, hipStream_t s);
hipError_t launch_exp(const float* state, float* q, size_t count, hipStream_t s);
hipError_t launch_dense_kernel(const float* f, int n, int dim, uint16_t* K, hipStream_t s);

int grid_blocks_per_item(int H, int W);

}  // namespace mf
