// Initialisation, q write-out, the FP64 free energy of grid problems and the
// deterministic FP64 reduction shared by every graph kind.  The step kernels
// are in grid_lanes.h (one step per launch) and grid_temporal.h (several).
//
// Layout: label-major [B][L][N], N = H * W, n = y * W + x.
#include <hip/hip_runtime.h>

#include "mf_internal.h"

namespace mf {
namespace {

// log q^0 per node (Eq. 6 reading): -u - lse(-u) (mode 0), uniform (mode 1),
// or the caller's state, checked (mode 2).  Sets flags[0] on a non-finite
// input.  A node's label slots are split over LPN consecutive lanes, LG
// each (the label count rounded up to LG * LPN), so that a grid of N nodes
// runs LPN * N threads; the node's max and sum reduce over its lanes with an
// xor butterfly, whose two operands at each level are the same in both
// lanes of a pair, so every lane holds the same lse.
template <int LG, int LPN>
__global__ __launch_bounds__(256) void init_kernel(const float* __restrict__ unary, float* __restrict__ state,
                                                   int L, int N, int mode, int* __restrict__ flags) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int n = t / LPN, l0 = (t % LPN) * LG;
  const int b = blockIdx.y;
  if (n >= N) return;   // the LPN lanes of a node leave together (LPN divides 64)
  const size_t base = (size_t)b * L * N + n;
  bool bad = false;
  if (mode == 0) {
    float v[LG];
    float mx = -INFINITY;
#pragma unroll
    for (int j = 0; j < LG; ++j) {
      const int l = l0 + j;
      v[j] = l < L ? -unary[base + (size_t)l * N] : -INFINITY;
      if (l < L) bad |= !isfinite(v[j]);
      mx = fmaxf(mx, v[j]);
    }
#pragma unroll
    for (int off = LPN / 2; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, LPN));
    float se = 0.f;
#pragma unroll
    for (int j = 0; j < LG; ++j) se += l0 + j < L ? expf(v[j] - mx) : 0.f;
#pragma unroll
    for (int off = LPN / 2; off > 0; off >>= 1) se += __shfl_xor(se, off, LPN);
    const float lse = mx + logf(se);
#pragma unroll
    for (int j = 0; j < LG; ++j)
      if (l0 + j < L) state[base + (size_t)(l0 + j) * N] = v[j] - lse;
  } else if (mode == 1) {
    const float u0 = -logf((float)L);
#pragma unroll
    for (int j = 0; j < LG; ++j) {
      const int l = l0 + j;
      if (l < L) {
        bad |= !isfinite(unary[base + (size_t)l * N]);
        state[base + (size_t)l * N] = u0;
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < LG; ++j) {
      const int l = l0 + j;
      if (l < L) {
        bad |= !isfinite(unary[base + (size_t)l * N]);
        bad |= !isfinite(state[base + (size_t)l * N]);
      }
    }
  }
  if (bad) atomicOr(flags, 1);
}

__global__ __launch_bounds__(64) void clear_kernel(int* __restrict__ p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

__global__ __launch_bounds__(64) void copy_flag_kernel(const int* __restrict__ flags, int32_t* __restrict__ out) {
  if (threadIdx.x == 0) out[0] = flags[0];
}

__global__ __launch_bounds__(256) void exp_kernel(const float* __restrict__ s, float* __restrict__ q,
                                                  size_t count) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) q[i] = expf(s[i]);
}

// Four elements per thread (both pointers 16-byte aligned, count % 4 == 0).
__global__ __launch_bounds__(256) void exp4_kernel(const float4* __restrict__ s, float4* __restrict__ q,
                                                   size_t count4) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count4) {
    const float4 v = s[i];
    q[i] = make_float4(expf(v.x), expf(v.y), expf(v.z), expf(v.w));
  }
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic 256-thread block sum in FP64; the result is valid in thread 0.
__device__ inline double block_sum(double v) {
  __shared__ double red[4];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = (red[0] + red[1]) + (red[2] + red[3]);
  return t;
}

// Per-node free-energy contribution in FP64 (Eq. 7):
//   sum_l q_l (u_l + log q_l) + 1/2 sum_l q_l (Theta S)_l
// The 1/2 counts each edge once, since it appears in the message of both ends.
template <int CONN, int COMPAT>
__global__ __launch_bounds__(256) void grid_fe_kernel(FreeEnergyArgs a) {
  const int L = a.L, N = a.N, H = a.H, W = a.W;
  const int b = blockIdx.y;
  const int n = blockIdx.x * 256 + threadIdx.x;
  double f = 0.0;
  if (n < N) {
    const int y = n / W, x = n - (n / W) * W;
    const size_t base = (size_t)b * L * N;
    const float* st = a.state + base;
    double S[kSmallLabels];
#pragma unroll
    for (int l = 0; l < kSmallLabels; ++l) S[l] = 0.0;
    for (int dy = -1; dy <= 1; ++dy) {
      for (int dx = -1; dx <= 1; ++dx) {
        if (dx == 0 && dy == 0) continue;
        if (CONN == 4 && dx != 0 && dy != 0) continue;
        const int yy = y + dy, xx = x + dx;
        if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
        const int j = yy * W + xx;
#pragma unroll
        for (int l = 0; l < kSmallLabels; ++l)
          if (l < L) S[l] += exp((double)st[(size_t)l * N + j]);
      }
    }
    double tot = 0.0;
#pragma unroll
    for (int l = 0; l < kSmallLabels; ++l) tot += S[l];
#pragma unroll
    for (int l = 0; l < kSmallLabels; ++l) {
      if (l >= L) continue;
      const double lq = (double)st[(size_t)l * N + n];
      const double q = exp(lq);
      double pm;
      if (COMPAT == MF_COMPAT_POTTS) {
        pm = (double)a.potts_w * (tot - S[l]);
      } else {
        pm = 0.0;
#pragma unroll
        for (int k = 0; k < kSmallLabels; ++k)
          if (k < L) pm += (double)a.theta[l * L + k] * S[k];
      }
      f += q * ((double)a.unary[base + (size_t)l * N + n] + lq + 0.5 * pm);
    }
  }
  const double t = block_sum(f);
  if (threadIdx.x == 0) a.partials[(size_t)b * a.n_blocks + blockIdx.x] = t;
}

// The same per-node terms for grids with more labels than grid_fe_kernel
// holds in registers.  The pairwise half-term is taken in the transposed
// order, 1/2 sum_l q_l (Theta S)_l = 1/2 sum_k S_k (Theta^T q)_k, over chunks
// of kSmallLabels labels of S, each chunk of Theta^T q formed from every q_l.
template <int CONN, int COMPAT>
__global__ __launch_bounds__(256) void grid_fe_large_kernel(FreeEnergyArgs a) {
  constexpr int KC = kSmallLabels;
  const int L = a.L, N = a.N, H = a.H, W = a.W;
  const int b = blockIdx.y;
  const int n = blockIdx.x * 256 + threadIdx.x;
  double f = 0.0;
  if (n < N) {
    const int y = n / W, x = n - (n / W) * W;
    const size_t base = (size_t)b * L * N;
    const float* st = a.state + base;
    int nbr[8];
    int nn = 0;
    for (int dy = -1; dy <= 1; ++dy) {
      for (int dx = -1; dx <= 1; ++dx) {
        if (dx == 0 && dy == 0) continue;
        if (CONN == 4 && dx != 0 && dy != 0) continue;
        const int yy = y + dy, xx = x + dx;
        if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
        nbr[nn++] = yy * W + xx;
      }
    }
    double qtot = 0.0;
    for (int l = 0; l < L; ++l) {
      const double lq = (double)st[(size_t)l * N + n];
      const double q = exp(lq);
      qtot += q;
      f += q * ((double)a.unary[base + (size_t)l * N + n] + lq);
    }
    double pair = 0.0;
    for (int k0 = 0; k0 < L; k0 += KC) {
      double S[KC];
#pragma unroll
      for (int k = 0; k < KC; ++k) S[k] = 0.0;
      for (int t = 0; t < nn; ++t) {
#pragma unroll
        for (int k = 0; k < KC; ++k)
          if (k0 + k < L) S[k] += exp((double)st[(size_t)(k0 + k) * N + nbr[t]]);
      }
      if (COMPAT == MF_COMPAT_POTTS) {
        // Theta = w (1 1^T - I): sum_k S_k (w qtot - w q_k)
#pragma unroll
        for (int k = 0; k < KC; ++k) {
          if (k0 + k < L) {
            const double qk = exp((double)st[(size_t)(k0 + k) * N + n]);
            pair += S[k] * (double)a.potts_w * (qtot - qk);
          }
        }
      } else {
        double r[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) r[k] = 0.0;
        for (int l = 0; l < L; ++l) {
          const double q = exp((double)st[(size_t)l * N + n]);
          const float* th = a.theta + (size_t)l * L + k0;
#pragma unroll
          for (int k = 0; k < KC; ++k)
            if (k0 + k < L) r[k] += (double)th[k] * q;
        }
#pragma unroll
        for (int k = 0; k < KC; ++k) pair += S[k] * r[k];
      }
    }
    f += 0.5 * pair;
  }
  const double t = block_sum(f);
  if (threadIdx.x == 0) a.partials[(size_t)b * a.n_blocks + blockIdx.x] = t;
}

// Sum the per-block partials of one batch item in a fixed order.
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double* __restrict__ partials,
                                                              int n_blocks, double* __restrict__ out) {
  const int b = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n_blocks; i += 256) s += partials[(size_t)b * n_blocks + i];
  const double t = block_sum(s);
  if (threadIdx.x == 0) out[b] = t;
}

}  // namespace

int grid_blocks_per_item(int H, int W) { return (H * W + 255) / 256; }

template <int LG, int LPN>
void init_lg(const float* unary, float* state, int B, int L, int N, int mode, int* flags, hipStream_t s) {
  const dim3 grid((unsigned)(((size_t)N * LPN + 255) / 256), B), block(256);
  hipLaunchKernelGGL((init_kernel<LG, LPN>), grid, block, 0, s, unary, state, L, N, mode, flags);
}

hipError_t launch_init(const float* unary, float* state, int B, int L, int N, int mode, int* flags,
                       hipStream_t s) {
  if (L <= 2) init_lg<2, 1>(unary, state, B, L, N, mode, flags, s);
  else if (L <= 4) init_lg<4, 1>(unary, state, B, L, N, mode, flags, s);
  else if (L <= 8) init_lg<4, 2>(unary, state, B, L, N, mode, flags, s);
  else if (L <= 16) init_lg<4, 4>(unary, state, B, L, N, mode, flags, s);
  else if (L <= 24) init_lg<6, 4>(unary, state, B, L, N, mode, flags, s);
  else if (L <= 32) init_lg<8, 4>(unary, state, B, L, N, mode, flags, s);
  else if (L <= 64) init_lg<8, 8>(unary, state, B, L, N, mode, flags, s);
  else init_lg<16, 8>(unary, state, B, L, N, mode, flags, s);
  return hipGetLastError();
}

hipError_t launch_clear_flags(int* flags, int n, hipStream_t s) {
  hipLaunchKernelGGL(clear_kernel, dim3(1), dim3(64), 0, s, flags, n);
  return hipGetLastError();
}

hipError_t launch_copy_flags(const int* flags, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(copy_flag_kernel, dim3(1), dim3(64), 0, s, flags, out);
  return hipGetLastError();
}

hipError_t launch_exp(const float* state, float* q, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (count % 4 == 0 && ((uintptr_t)state & 15u) == 0 && ((uintptr_t)q & 15u) == 0) {
    const size_t c4 = count / 4;
    hipLaunchKernelGGL(exp4_kernel, dim3((unsigned)((c4 + 255) / 256)), dim3(256), 0, s, (const float4*)state,
                       (float4*)q, c4);
  } else {
    hipLaunchKernelGGL(exp_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, state, q, count);
  }
  return hipGetLastError();
}

hipError_t launch_grid_free_energy(const FreeEnergyArgs& a, int conn, int compat, double* f_out,
                                   hipStream_t s) {
  dim3 grid(a.n_blocks, a.B);
  if (a.L > kSmallLabels) {
    if (conn == 4) {
      if (compat == MF_COMPAT_POTTS) hipLaunchKernelGGL((grid_fe_large_kernel<4, MF_COMPAT_POTTS>), grid, dim3(256), 0, s, a);
      else hipLaunchKernelGGL((grid_fe_large_kernel<4, MF_COMPAT_GENERAL>), grid, dim3(256), 0, s, a);
    } else {
      if (compat == MF_COMPAT_POTTS) hipLaunchKernelGGL((grid_fe_large_kernel<8, MF_COMPAT_POTTS>), grid, dim3(256), 0, s, a);
      else hipLaunchKernelGGL((grid_fe_large_kernel<8, MF_COMPAT_GENERAL>), grid, dim3(256), 0, s, a);
    }
  } else if (conn == 4) {
    if (compat == MF_COMPAT_POTTS) hipLaunchKernelGGL((grid_fe_kernel<4, MF_COMPAT_POTTS>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((grid_fe_kernel<4, MF_COMPAT_GENERAL>), grid, dim3(256), 0, s, a);
  } else {
    if (compat == MF_COMPAT_POTTS) hipLaunchKernelGGL((grid_fe_kernel<8, MF_COMPAT_POTTS>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((grid_fe_kernel<8, MF_COMPAT_GENERAL>), grid, dim3(256), 0, s, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_partials(a.partials, a.n_blocks, a.B, f_out, s);
}

hipError_t launch_reduce_partials(const double* partials, int n_blocks, int B, double* out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(B), dim3(256), 0, s, partials, n_blocks, out);
  return hipGetLastError();
}

}  // namespace mf
