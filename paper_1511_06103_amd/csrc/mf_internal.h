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

// Continuous batching: up to kMaxSlots problems advanced by one launch.
constexpr int kMaxSlots = 48;
// Label counts of the per-thread kernels (the batched, fused and rule grid
// kernels, CSR, dense, adjoint, Lipschitz, the small free energy); grids with
// more labels (up to MF_MAX_LABELS) take one step per launch with Theta S on
// the matrix cores (grid_large.hip).
constexpr int kSmallLabels = 32;
struct ManyArgs {
  StepArgs slot[kMaxSlots];
  float one_minus_alpha[kMaxSlots];
  int tile_begin[kMaxSlots + 1];
  int count;
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

struct CsrStepArgs {
  const float* unary;      // [B][L][N]
  const float* state_in;   // [B][L][N]
  float* state_out;        // [B][L][N]
  const void* q_in;        // [B][N][LQ] node-major q of state_in: FP32, or BF16 / FP16
                           // in the message-precision modes
  void* q_out;             // [B][N][LQ] node-major q of state_out
  const int* row_ptr;      // [N + 1]
  const int* col;          // [nnz]
  const float* w;          // [nnz] or nullptr
  long long nnz;
  const float* theta;
  int B, L, N;
  float alpha;
  float potts_w;
  int lanes;               // mf_desc.csr_lanes: 1 = one lane per node; otherwise the default
};

struct CsrFreeEnergyArgs {
  const float* unary;
  const float* state;
  const float* theta;
  const int* row_ptr;
  const int* col;
  const float* w;
  long long nnz;
  int B, L, N;
  float potts_w;
  double* partials;
  int n_blocks;
};

struct DenseStepArgs {
  const uint16_t* K;       // [N][N] bf16 bits, row-major (the caller's)
  uint16_t* Kt;            // the same K zero-padded to Np x Np in MFMA operand order:
                           // [Np/64][Np/32][4][64 lanes][8]
  const float* unary;      // [B][L][N]
  const float* state_in;   // [B][L][N]
  float* state_out;
  const uint16_t* q_in;    // [B][Np/32][NS][2][64 lanes][8] bf16 planes of q(state_in)
  uint16_t* q_out;         // planes of q(state_out)
  float* s_part;           // [B][KS][Np][32] partial S
  const float* t_in;       // [B][NEB][32] column sums of q(state_in) per 16-node block
  float* t_out;
  const float* theta;      // [L][L] (general)
  const float* cooc;       // [L][L] or nullptr
  int B, L, N, Np, KS, NRB, NEB, jchunk;
  float alpha, potts_w, inv_n;
};

// Step rules other than the fixed proximal step (grid_rules.hip).
struct RuleArgs {
  float* mom;              // [B][L][N] momentum average (MOMENTUM, ADAM)
  float* sq;               // [B][L][N] second moment (ADAM)
  float gamma1, gamma2, eps, v0;
  float d;                 // 1 / alpha - 1
  int init;                // 1: write the rule state of q^0 (mom = m, sq = v0) only
  int colour;              // SWEEP: the colour class this launch updates
};

// Power method for the tangent-space Lipschitz constant (lipschitz_kernels.hip).
struct LipArgs {
  const float* v;          // [L][N] current iterate, before its scale
  float* w;                // [L][N] output
  double* sc;              // [2 + kSmallLabels]: scale of v, shift, column sums T of scaled v
  double* res;             // [4]: rho, lambda, run-1 stopped, run-2 stopped
  double* part;            // [blocks][np] FP64 partial sums
  int np;                  // 3, or 3 + kSmallLabels on a dense graph (column sums)
  int graph, compat, L, N, H, W;
  float potts_w;
  const float* theta;      // [L][L] (general)
  const int32_t* row_ptr;  // CSR
  const int32_t* col;
  const float* csr_w;
  long long nnz;
  const uint16_t* K;       // dense [N][N] bf16 bits
  const float* cooc;       // dense co-occurrence [L][L] or nullptr
};

struct DenseGeometry {
  int Np = 0, NRB = 0, NEB = 0, KS = 0, jchunk = 0;   // NEB: 16-node blocks of the per-node kernels
};

struct DenseFreeEnergyArgs {
  const uint16_t* K;
  const float* unary;
  const float* state;
  const float* theta;
  const float* cooc;
  double* qd;              // [B][N][L] scratch
  int B, L, N;
  float potts_w;
  double* partials;
  int n_blocks;
};

struct AdjointArgs {
  const float* g_in;       // [B][L][N] dLoss / d ell^{t+1}
  float* g_out;            // [B][L][N] dLoss / d ell^t
  const float* ell_t;      // [B][L][N]
  const float* ell_t1;     // [B][L][N]
  float* u_bar;            // [B][L][N] accumulated
  float* s_bar;            // [B][L][N] scratch: Theta^T m_bar
  const float* theta;
  double* theta_tile;      // [parts][L][L] per-tile FP64 sums over the steps so far
  double* theta_stage;     // [stages][L][L] FP64 sums of 32 tile sums each
  double* theta_acc;       // [L][L] the gradient, written once at the end
  int B, L, N, H, W;
  float alpha, potts_w;
};

// Workspace layout (offsets in bytes from the 256-aligned workspace start).
struct WorkspaceLayout {
  size_t flags = 0;        // int32[64]: [0] bit 0 non-finite input, bit 1 malformed CSR
  size_t partials = 0;     // double[B][n_blocks]
  size_t f_out = 0;        // double[B]
  size_t csr_q = 0;        // [2][B][N][LQ] q, FP32 or 16-bit per message mode (CSR only)
  size_t dq = 0;           // uint16[2][B][NS * 32 * Np] q planes (dense only)
  size_t dk = 0;           // uint16[Np * Np] K in MFMA operand order
  size_t ds = 0;           // float[B][KS][Np][32] partial S
  size_t dt = 0;           // float[2][B][NRB][32] column sums
  size_t dqd = 0;          // double[B][N][L] free-energy scratch
  size_t rule_state = 0;   // float[1 or 2][B][L][N] momentum / ADAM state
  size_t xch = 0;          // uint64[tiles][2][L][64] halo exchange of the persistent grid kernel
  size_t xch_bytes = 0;
  DenseGeometry dg;
  int dense_ns = 0;
  size_t total = 0;
  int n_blocks = 0;
};

// Launchers (return hipSuccess or the launch error).
hipError_t launch_init(const float* unary, float* state, int B, int L, int N, int mode,
                       int* flags, hipStream_t s);
// ks <= K sub-steps in one launch of the K-halo kernel; K <= grid_max_steps_per_launch.
// Small grids (N <= 1024 nodes, L <= kWholeMaxLabels): one workgroup per
// problem holds the whole grid in LDS and runs ks steps in one launch.
constexpr int kWholeMaxLabels = 8;
constexpr int kWholeMaxSteps = 256;   // steps per launch the library picks for them
bool grid_whole_fits(int L, int N);
// init >= 0: the launch starts with the initialisation of that mf_init_mode
// (flags[0] set on a non-finite input, as the initialisation kernel does);
// q_out != nullptr: it ends by writing q = exp(log q) of the last step.
hipError_t launch_grid_whole(const StepArgs& a, int conn, int compat, int precision, int ks, int init, int* flags,
                             float* q_out, hipStream_t s);
hipError_t launch_grid_multi_step(const StepArgs& a, int conn, int compat, int precision, int K, int ks,
                                  hipStream_t s);
int grid_max_steps_per_launch(int L, int compat, int precision);
hipError_t launch_grid_free_energy(const FreeEnergyArgs& a, int conn, int compat, double* f_out,
                                   hipStream_t s);
hipError_t launch_clear_flags(int* flags, int n, hipStream_t s);
hipError_t launch_copy_flags(const int* flags, int32_t* out, hipStream_t s);   // out[0] = flags[0]
hipError_t launch_lip_center(const LipArgs& a, const float* v0, hipStream_t s);
hipError_t launch_lip_hvp(const LipArgs& a, hipStream_t s);
hipError_t launch_lip_reduce(const LipArgs& a, int n_blocks, int mode, hipStream_t s);
int lip_blocks(int graph, int N, int H, int W);
// One step of a non-fixed rule on a grid (FP32 messages, one step per launch).
hipError_t launch_grid_rule_step(const StepArgs& a, const RuleArgs& r, int conn, int compat, int rule,
                                 hipStream_t s);
hipError_t launch_exp(const float* state, float* q, size_t count, hipStream_t s);
hipError_t launch_dense_kernel(const float* f, int n, int dim, uint16_t* K, hipStream_t s);
int dense_planes(int precision);
DenseGeometry dense_geometry(int N, int B);
hipError_t launch_dense_prepare(const DenseStepArgs& a, int NS, hipStream_t s);
hipError_t launch_dense_tile_k(const DenseStepArgs& a, hipStream_t s);
hipError_t launch_dense_step(const DenseStepArgs& a, int NS, int compat, hipStream_t s);
hipError_t launch_dense_free_energy(const DenseFreeEnergyArgs& a, int compat, hipStream_t s);

hipError_t launch_reduce_partials(const double* partials, int n_blocks, int B, double* out, hipStream_t s);

int csr_label_stride(int L);
hipError_t launch_csr_check(const int* row_ptr, const int* col, int N, long long nnz, int* flags,
                            hipStream_t s);
// Bytes per element of the node-major q copy: 4 (FP32) or 2 (BF16 / FP16 messages).
int csr_q_bytes(int precision);
hipError_t launch_csr_q_from_state(const float* state, void* qn, int B, int L, int N, int precision,
                                   hipStream_t s);
hipError_t launch_csr_step(const CsrStepArgs& a, int compat, int precision, hipStream_t s);
hipError_t launch_csr_free_energy(const CsrFreeEnergyArgs& a, int compat, hipStream_t s);

size_t adjoint_theta_parts(int B, int H, int W);
size_t adjoint_theta_stages(int B, int H, int W);
hipError_t launch_adjoint_step(const AdjointArgs& a, int conn, int compat, hipStream_t s);
// theta_acc = sum over tiles of theta_tile, in a fixed order (after the last step).
hipError_t launch_adjoint_theta_reduce(const AdjointArgs& a, hipStream_t s);
hipError_t launch_adjoint_init(const float* g0, const float* ell0, float* u_bar, int B, int L, int N,
                               hipStream_t s);
hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t s);
hipError_t launch_fill_f64(double* p, size_t n, hipStream_t s);
hipError_t launch_copy_f32(const float* src, float* dst, size_t n, hipStream_t s);
hipError_t launch_f64_to_f32(const double* src, float* dst, size_t n, hipStream_t s);

int grid_lanes_tiles(int B, int H, int W, int L);
// One step per launch; grids with more than kSmallLabels labels go to the
// matrix-core kernel of grid_large.hip.
hipError_t launch_grid_step_lanes(const StepArgs& a, int conn, int compat, int prec, hipStream_t s);
hipError_t launch_grid_step_large(const StepArgs& a, int conn, int compat, int prec, hipStream_t s);
hipError_t launch_grid_step_lanes_many(const ManyArgs& m, int L, int conn, int compat, int prec, hipStream_t s);

int grid_blocks_per_item(int H, int W);

// Every step of a launch in one resident workgroup per 16 x 16 tile, the
// halo exchanged through tagged words (grid_persist.hip): general Theta,
// 8 < L <= kSmallLabels, at most kPersistMaxTiles tiles and no more than the
// device keeps resident (grid_persist_capacity, from the occupancy query).  Steps per launch at most kPersistMaxSteps.  Bit 2 of flags: a
// halo wait gave up.
constexpr int kPersistMaxTiles = 256;
constexpr int kPersistMaxSteps = MF_PERSIST_STEPS_PER_LAUNCH;
bool grid_persist_eligible(int L, int compat);
size_t grid_persist_exchange_bytes(int B, int H, int W, int L);
int grid_persist_capacity(int L, int conn, int precision);
// init >= 0: the launch starts with the initialisation of that mf_init_mode
// (flags bit 0 on a non-finite input); q_out != nullptr: it ends by writing
// q = exp(log q) of the last step.
hipError_t launch_grid_persist(const StepArgs& a, int conn, int precision, uint64_t* xch, unsigned tag0, int ks,
                               int* flags, int init, float* q_out, hipStream_t s);

}  // namespace mf
