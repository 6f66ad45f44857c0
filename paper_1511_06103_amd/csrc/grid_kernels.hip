// Grid kernels: initialisation, the parallel proximal step on 4/8-connected
// grids, and the FP64 free energy.
//
// Step (Eq. 15 with the fixed step of Eq. 16):
//   q_j   = exp(log q_j)                       staged in LDS with a 1-node halo
//   S_i   = sum of q_j over the grid neighbours of i (free boundary, unit weight)
//   m_i   = u_i + Theta S_i                    (Potts: w (sum(S_i) 1 - S_i))
//   z_i   = (1 - alpha) log q_i - alpha m_i
//   log q_i <- z_i - logsumexp(z_i)
//
// Layout: label-major [B][L][N], N = H * W, n = y * W + x.  One thread owns
// one node and keeps its L labels in registers; a 64 x 4 tile maps each
// 64-wide wavefront onto one row segment, so every global access of a
// label plane is one contiguous 256-byte run per wavefront.
#include <hip/hip_runtime.h>

#include "mf_internal.h"

namespace mf {
namespace {

constexpr int HX = kTileX + 2;
constexpr int HY = kTileY + 2;
constexpr int HN = HX * HY;

enum { P_F32 = 0, P_BF16 = 1, P_F16 = 2 };

// Message operand storage in LDS for each precision mode.
template <int PREC> struct MsgT;
template <> struct MsgT<P_F32> {
  using T = float;
  __device__ static T enc(float x) { return x; }
  __device__ static float dec(T x) { return x; }
};
template <> struct MsgT<P_BF16> {
  using T = unsigned short;
  // Round to nearest even on the low 16 bits; q is finite and non-negative.
  __device__ static T enc(float x) {
    unsigned int u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (T)(u >> 16);
  }
  __device__ static float dec(T x) { return __uint_as_float(((unsigned int)x) << 16); }
};
template <> struct MsgT<P_F16> {
  using T = _Float16;
  __device__ static T enc(float x) { return (T)x; }
  __device__ static float dec(T x) { return (float)x; }
};

// Halo ring of a kTileX x kTileY tile: the two full rows above and below
// (HX nodes each) and the left/right column of every interior row.
constexpr int kHalo = 2 * HX + 2 * kTileY;

__device__ inline int halo_lds_pos(int h) {
  if (h < HX) return h;                                   // top row
  if (h < 2 * HX) return (HY - 1) * HX + (h - HX);        // bottom row
  const int k = h - 2 * HX;                               // sides, rows 1..kTileY
  return (1 + (k >> 1)) * HX + ((k & 1) ? HX - 1 : 0);
}

// One step for a 64 x 4 tile.  Every global load is issued before the
// first use (own log q and u of the node, plus this thread's share of the
// halo), so one memory latency covers the whole tile even at one wavefront
// per SIMD.
// The tile body is shared by the single-problem kernel and the many-problem
// (continuous batching) kernel, so a problem gets bitwise the same iterates
// whichever kernel advances it.
template <int LP, bool EXACT, int CONN, int COMPAT, int PREC>
__device__ inline void grid_step_tile(const StepArgs& a, float one_minus_alpha, int b, int x0, int y0,
                                      typename MsgT<PREC>::T* __restrict__ qs) {
  using M = MsgT<PREC>;
  constexpr int HREG = (LP * kHalo + kThreads - 1) / kThreads;
  const int L = EXACT ? LP : a.L;
  const int N = a.N, H = a.H, W = a.W;
  const size_t base = (size_t)b * L * N;
  const float* __restrict__ lin = a.state_in + base;
  const int tid = threadIdx.x;
  const int tx = tid % kTileX, ty = tid / kTileX;
  const int x = x0 + tx, y = y0 + ty;
  const bool inside = x < W && y < H;
  const int n = inside ? y * W + x : 0;
  const float* __restrict__ ug = a.unary + base + n;

  float ell[LP], uu[LP], hv[HREG];
#pragma unroll
  for (int l = 0; l < LP; ++l) {
    ell[l] = 0.f;
    uu[l] = 0.f;
    if (l < L && inside) {
      ell[l] = lin[(size_t)l * N + n];
      uu[l] = ug[(size_t)l * N];
    }
  }
#pragma unroll
  for (int r = 0; r < HREG; ++r) {
    const int f = tid + r * kThreads;
    hv[r] = -INFINITY;
    if (f < L * kHalo) {
      const int l = f / kHalo;
      const int pos = halo_lds_pos(f - l * kHalo);
      const int hy = pos / HX, hx = pos - (pos / HX) * HX;
      const int gy = y0 + hy - 1, gx = x0 + hx - 1;
      if (gy >= 0 && gy < H && gx >= 0 && gx < W) hv[r] = lin[(size_t)l * N + gy * W + gx];
    }
  }

  const int p = (ty + 1) * HX + (tx + 1);
#pragma unroll
  for (int l = 0; l < LP; ++l)
    if (l < L) qs[l * HN + p] = M::enc(inside ? __expf(ell[l]) : 0.f);
#pragma unroll
  for (int r = 0; r < HREG; ++r) {
    const int f = tid + r * kThreads;
    if (f < L * kHalo) {
      const int l = f / kHalo;
      qs[l * HN + halo_lds_pos(f - l * kHalo)] = M::enc(__expf(hv[r]));   // exp(-inf) = 0 off-grid
    }
  }
  __syncthreads();
  if (!inside) return;

  float S[LP];
#pragma unroll
  for (int l = 0; l < LP; ++l) {
    S[l] = 0.f;
    if (l < L) {
      const typename M::T* q = qs + l * HN + p;
      float s = M::dec(q[-HX]) + M::dec(q[-1]) + M::dec(q[1]) + M::dec(q[HX]);
      if (CONN == 8) s += (M::dec(q[-HX - 1]) + M::dec(q[-HX + 1])) + (M::dec(q[HX - 1]) + M::dec(q[HX + 1]));
      S[l] = s;
    }
  }

  float z[LP];
  if (COMPAT == MF_COMPAT_POTTS) {
    float tot = 0.f;
#pragma unroll
    for (int l = 0; l < LP; ++l) tot += S[l];
#pragma unroll
    for (int l = 0; l < LP; ++l) {
      const float m = uu[l] + a.potts_w * (tot - S[l]);
      z[l] = one_minus_alpha * ell[l] - a.alpha * m;
    }
  } else {
    const float* __restrict__ th = a.theta;
#pragma unroll
    for (int l = 0; l < LP; ++l) {
      float acc = 0.f;
      if (l < L) {
#pragma unroll
        for (int k = 0; k < LP; ++k)
          if (k < L) acc = fmaf(th[l * L + k], S[k], acc);
      }
      const float m = uu[l] + acc;
      z[l] = one_minus_alpha * ell[l] - a.alpha * m;
    }
  }

  float mx = -INFINITY;
#pragma unroll
  for (int l = 0; l < LP; ++l)
    if (l < L) mx = fmaxf(mx, z[l]);
  float se = 0.f;
#pragma unroll
  for (int l = 0; l < LP; ++l)
    if (l < L) se += __expf(z[l] - mx);
  const float lse = mx + __logf(se);
  float* __restrict__ out = a.state_out + base + n;
#pragma unroll
  for (int l = 0; l < LP; ++l)
    if (l < L) out[(size_t)l * N] = z[l] - lse;
}

template <int LP, bool EXACT, int CONN, int COMPAT, int PREC>
__global__ __launch_bounds__(kThreads) void grid_step_kernel(StepArgs a, float one_minus_alpha) {
  __shared__ typename MsgT<PREC>::T qs[LP * HN];
  grid_step_tile<LP, EXACT, CONN, COMPAT, PREC>(a, one_minus_alpha, blockIdx.z, blockIdx.x * kTileX,
                                                blockIdx.y * kTileY, qs);
}

// Many independent problems in one launch: slot k owns workgroups
// [tile_begin[k], tile_begin[k + 1]); each workgroup runs one tile of its
// problem.  Every slot shares L, connectivity, compatibility kind and
// message precision; sizes, alpha and the arrays are per slot.
template <int LP, bool EXACT, int CONN, int COMPAT, int PREC>
__global__ __launch_bounds__(kThreads) void grid_step_many_kernel(ManyArgs m) {
  __shared__ typename MsgT<PREC>::T qs[LP * HN];
  const int blk = blockIdx.x;
  int k = 0;
  while (k + 1 < m.count && blk >= m.tile_begin[k + 1]) ++k;
  const int t = blk - m.tile_begin[k];
  const int tiles_x = (m.slot[k].W + kTileX - 1) / kTileX;
  const int tiles_per_item = tiles_x * ((m.slot[k].H + kTileY - 1) / kTileY);
  const int b = t / tiles_per_item;
  const int r = t - b * tiles_per_item;
  const int ty = r / tiles_x, tx = r - (r / tiles_x) * tiles_x;
  grid_step_tile<LP, EXACT, CONN, COMPAT, PREC>(m.slot[k], m.one_minus_alpha[k], b, tx * kTileX, ty * kTileY, qs);
}

// Initial log q per node: -u - lse(-u) (mode 0) or -log L (mode 1); mode 2
// only checks the caller's state.  Sets flags[0] on a non-finite input.
__global__ __launch_bounds__(256) void init_kernel(const float* __restrict__ unary,
                                                   float* __restrict__ state, int L, int N,
                                                   int mode, int* __restrict__ flags) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (n >= N) return;
  const size_t base = (size_t)b * L * N + n;
  bool bad = false;
  float mx = -INFINITY;
  for (int l = 0; l < L; ++l) {
    const float v = unary[base + (size_t)l * N];
    bad |= !isfinite(v);
    mx = fmaxf(mx, -v);
  }
  if (mode == 0) {
    float se = 0.f;
    for (int l = 0; l < L; ++l) se += expf(-unary[base + (size_t)l * N] - mx);
    const float lse = mx + logf(se);
    for (int l = 0; l < L; ++l) state[base + (size_t)l * N] = -unary[base + (size_t)l * N] - lse;
  } else if (mode == 1) {
    const float v = -logf((float)L);
    for (int l = 0; l < L; ++l) state[base + (size_t)l * N] = v;
  } else {
    for (int l = 0; l < L; ++l) bad |= !isfinite(state[base + (size_t)l * N]);
  }
  if (bad) atomicOr(flags, 1);
}

__global__ __launch_bounds__(64) void clear_kernel(int* __restrict__ p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void exp_kernel(const float* __restrict__ s, float* __restrict__ q,
                                                  size_t count) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) q[i] = expf(s[i]);
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
    double S[MF_MAX_LABELS];
    for (int l = 0; l < L; ++l) S[l] = 0.0;
    for (int dy = -1; dy <= 1; ++dy) {
      for (int dx = -1; dx <= 1; ++dx) {
        if (dx == 0 && dy == 0) continue;
        if (CONN == 4 && dx != 0 && dy != 0) continue;
        const int yy = y + dy, xx = x + dx;
        if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
        const int j = yy * W + xx;
        for (int l = 0; l < L; ++l) S[l] += exp((double)st[(size_t)l * N + j]);
      }
    }
    double tot = 0.0;
    for (int l = 0; l < L; ++l) tot += S[l];
    for (int l = 0; l < L; ++l) {
      const double lq = (double)st[(size_t)l * N + n];
      const double q = exp(lq);
      double pm;
      if (COMPAT == MF_COMPAT_POTTS) {
        pm = (double)a.potts_w * (tot - S[l]);
      } else {
        pm = 0.0;
        for (int k = 0; k < L; ++k) pm += (double)a.theta[l * L + k] * S[k];
      }
      f += q * ((double)a.unary[base + (size_t)l * N + n] + lq + 0.5 * pm);
    }
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

template <int LP, bool EXACT, int CONN, int COMPAT, int PREC>
hipError_t step_launch(const StepArgs& a, hipStream_t s) {
  dim3 grid((a.W + kTileX - 1) / kTileX, (a.H + kTileY - 1) / kTileY, a.B);
  const float om = (float)(1.0 - (double)a.alpha);
  hipLaunchKernelGGL((grid_step_kernel<LP, EXACT, CONN, COMPAT, PREC>), grid, dim3(kThreads), 0, s, a, om);
  return hipGetLastError();
}

template <int LP, bool EXACT, int CONN, int COMPAT>
hipError_t step_prec(const StepArgs& a, int prec, hipStream_t s) {
  switch (prec) {
    case MF_P_F32: return step_launch<LP, EXACT, CONN, COMPAT, P_F32>(a, s);
    case MF_P_BF16MSG: return step_launch<LP, EXACT, CONN, COMPAT, P_BF16>(a, s);
    default: return step_launch<LP, EXACT, CONN, COMPAT, P_F16>(a, s);
  }
}

template <int LP, bool EXACT>
hipError_t step_lp(const StepArgs& a, int conn, int compat, int prec, hipStream_t s) {
  if (conn == 4) {
    return compat == MF_COMPAT_POTTS ? step_prec<LP, EXACT, 4, MF_COMPAT_POTTS>(a, prec, s)
                                     : step_prec<LP, EXACT, 4, MF_COMPAT_GENERAL>(a, prec, s);
  }
  return compat == MF_COMPAT_POTTS ? step_prec<LP, EXACT, 8, MF_COMPAT_POTTS>(a, prec, s)
                                   : step_prec<LP, EXACT, 8, MF_COMPAT_GENERAL>(a, prec, s);
}

template <int LP, bool EXACT, int CONN, int COMPAT, int PREC>
hipError_t many_launch(const ManyArgs& m, int total_tiles, hipStream_t s) {
  hipLaunchKernelGGL((grid_step_many_kernel<LP, EXACT, CONN, COMPAT, PREC>), dim3(total_tiles), dim3(kThreads), 0,
                     s, m);
  return hipGetLastError();
}

template <int LP, bool EXACT, int CONN, int COMPAT>
hipError_t many_prec(const ManyArgs& m, int total, int prec, hipStream_t s) {
  switch (prec) {
    case MF_P_F32: return many_launch<LP, EXACT, CONN, COMPAT, P_F32>(m, total, s);
    case MF_P_BF16MSG: return many_launch<LP, EXACT, CONN, COMPAT, P_BF16>(m, total, s);
    default: return many_launch<LP, EXACT, CONN, COMPAT, P_F16>(m, total, s);
  }
}

template <int LP, bool EXACT>
hipError_t many_lp(const ManyArgs& m, int total, int conn, int compat, int prec, hipStream_t s) {
  if (conn == 4) {
    return compat == MF_COMPAT_POTTS ? many_prec<LP, EXACT, 4, MF_COMPAT_POTTS>(m, total, prec, s)
                                     : many_prec<LP, EXACT, 4, MF_COMPAT_GENERAL>(m, total, prec, s);
  }
  return compat == MF_COMPAT_POTTS ? many_prec<LP, EXACT, 8, MF_COMPAT_POTTS>(m, total, prec, s)
                                   : many_prec<LP, EXACT, 8, MF_COMPAT_GENERAL>(m, total, prec, s);
}

}  // namespace

int grid_tiles(int B, int H, int W) {
  return B * ((W + kTileX - 1) / kTileX) * ((H + kTileY - 1) / kTileY);
}

hipError_t launch_grid_step_many(const ManyArgs& m, int L, int conn, int compat, int prec, hipStream_t s) {
  const int total = m.tile_begin[m.count];
  if (total <= 0) return hipSuccess;
  if (L == 2) return many_lp<2, true>(m, total, conn, compat, prec, s);
  if (L == 21) return many_lp<21, true>(m, total, conn, compat, prec, s);
  if (L <= 4) return many_lp<4, false>(m, total, conn, compat, prec, s);
  if (L <= 8) return many_lp<8, false>(m, total, conn, compat, prec, s);
  if (L <= 16) return many_lp<16, false>(m, total, conn, compat, prec, s);
  return many_lp<32, false>(m, total, conn, compat, prec, s);
}

int grid_blocks_per_item(int H, int W) { return (H * W + 255) / 256; }

hipError_t launch_init(const float* unary, float* state, int B, int L, int N, int mode, int* flags,
                       hipStream_t s) {
  dim3 grid((N + 255) / 256, B);
  hipLaunchKernelGGL(init_kernel, grid, dim3(256), 0, s, unary, state, L, N, mode, flags);
  return hipGetLastError();
}

hipError_t launch_clear_flags(int* flags, int n, hipStream_t s) {
  hipLaunchKernelGGL(clear_kernel, dim3(1), dim3(64), 0, s, flags, n);
  return hipGetLastError();
}

hipError_t launch_exp(const float* state, float* q, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(exp_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, state, q, count);
  return hipGetLastError();
}

hipError_t launch_grid_step(const StepArgs& a, int conn, int compat, int prec, hipStream_t s) {
  const int L = a.L;
  if (L == 2) return step_lp<2, true>(a, conn, compat, prec, s);
  if (L == 21) return step_lp<21, true>(a, conn, compat, prec, s);
  if (L <= 4) return step_lp<4, false>(a, conn, compat, prec, s);
  if (L <= 8) return step_lp<8, false>(a, conn, compat, prec, s);
  if (L <= 16) return step_lp<16, false>(a, conn, compat, prec, s);
  return step_lp<32, false>(a, conn, compat, prec, s);
}

hipError_t launch_grid_free_energy(const FreeEnergyArgs& a, int conn, int compat, double* f_out,
                                   hipStream_t s) {
  dim3 grid(a.n_blocks, a.B);
  if (conn == 4) {
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
