// Fully connected CRF: explicit N x N Gaussian kernel K (BF16), the
// parallel proximal step with S = K Q on MFMA, and the FP64 free energy.
//
// Model (dense CRF with co-occurrence, Sec. 4.2 semantic segmentation):
//   S_i  = sum_j K_ij q_j                          (K symmetric, K_ii = 0)
//   m_i  = u_i + Theta S_i  [+ C (T - q_i) / N],  T = sum_j q_j
//   log q_i <- normalise((1 - alpha) log q_i - alpha m_i)      (Eq. 15, 16)
//
// S = K Q is a real dense contraction and runs on v_mfma_f32_16x16x32_bf16.
// The operand Q is q split into NS bfloat16 planes, q = q_0 + q_1 (+ q_2),
// each plane holding the rounding residual of the previous one: three planes
// carry 24 significant bits (the FP32 mode), two planes 16 bits, one plane
// is plain BF16 messages.  K is given in BF16, so every product is exact
// and only the FP32 accumulation rounds.  The step is bound by streaming K
// (2 bytes per multiply-add pair of each row), not by the MFMA rate, so the
// extra planes cost little.
//
// Work split: a workgroup owns a 64-row block and one of KS slices of the
// j range; each of its four wavefronts accumulates a 16 x 32 (rows x
// labels, L padded to 32) tile in registers.  Slices write FP32 partial
// sums; the last workgroup of a row block to finish (counted with a
// device-scope atomic, after a release fence) adds the KS partials in a
// fixed order and runs the per-node step, so the result is deterministic.
// That workgroup also writes the next Q planes and the block's column sums
// of q, which the co-occurrence term of the next step reduces in a fixed
// order.
#include <hip/hip_runtime.h>

#include "mf_internal.h"

namespace mf {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kRB = 64;      // rows per workgroup
constexpr int kLP = 32;      // padded label count of the MFMA tiles

__device__ inline unsigned short f2bf_rne(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

__device__ inline float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// K_ij = exp(-|f_i - f_j|^2 / 2) in FP32, K_ii = 0, rounded to BF16 (nearest even).
__global__ __launch_bounds__(256) void dense_kernel_build(const float* __restrict__ f, int n, int dim,
                                                          unsigned short* __restrict__ K) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= n) return;
  float d2 = 0.f;
  for (int k = 0; k < dim; ++k) {
    const float d = f[(size_t)i * dim + k] - f[(size_t)j * dim + k];
    d2 = fmaf(d, d, d2);
  }
  K[(size_t)i * n + j] = (i == j) ? (unsigned short)0 : f2bf_rne(expf(-0.5f * d2));
}

// Split q (FP32) of one node into NS BF16 planes and store them label-major.
template <int NS>
__device__ inline void store_planes(unsigned short* __restrict__ planes, int Np, int l, int i, float q) {
  float r = q;
#pragma unroll
  for (int p = 0; p < NS; ++p) {
    const unsigned short h = f2bf_rne(r);
    planes[((size_t)p * kLP + l) * Np + i] = h;
    r -= bf2f(h);
  }
}

// q^0 planes and per-block column sums from the initial state.  One
// wavefront per 64-node block; lane = node.
template <int NS>
__global__ __launch_bounds__(64) void dense_prepare_kernel(DenseStepArgs a) {
  const int rb = blockIdx.x, b = blockIdx.y;
  const int lane = threadIdx.x;
  const int i = rb * kRB + lane;
  const int L = a.L, N = a.N, Np = a.Np;
  unsigned short* planes = a.q_out + (size_t)b * NS * kLP * Np;
  for (int l = 0; l < kLP; ++l) {
    float q = 0.f;
    if (i < N && l < L) q = __expf(a.state_in[((size_t)b * L + l) * N + i]);
    store_planes<NS>(planes, Np, l, i, q);
    const float t = wave_sum_f(q);
    if (lane == 0) a.t_out[((size_t)b * a.NRB + rb) * kLP + l] = t;
  }
  if (lane == 0) a.counters[b * a.NRB + rb] = 0;
}

template <int NS, int COMPAT, bool COOC>
__global__ __launch_bounds__(256) void dense_step_kernel(DenseStepArgs a, float one_minus_alpha) {
  const int b = blockIdx.y;
  const int rb = blockIdx.x / a.KS, ks = blockIdx.x - (blockIdx.x / a.KS) * a.KS;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int L = a.L, N = a.N, Np = a.Np;
  const unsigned short* __restrict__ K = a.K;
  const unsigned short* __restrict__ Q = a.q_in + (size_t)b * NS * kLP * Np;

  // --- S partial = K[rows, j-slice] Q[j-slice, :] on MFMA -------------------
  const int r0 = rb * kRB + wave * 16;
  const int row = r0 + (lane & 15);
  const int kq = 8 * (lane >> 4);
  const int jb = ks * a.jchunk;
  const int je = min(jb + a.jchunk, Np);
  f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
  const bool vec_ok = (N & 7) == 0;
  for (int j0 = jb; j0 < je; j0 += 32) {
    const int kk = j0 + kq;
    bf16x8 av;
    if (vec_ok && row < N && kk + 8 <= N) {
      av = *reinterpret_cast<const bf16x8*>(K + (size_t)row * N + kk);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const unsigned short v = (row < N && kk + e < N) ? K[(size_t)row * N + kk + e] : (unsigned short)0;
        av[e] = __builtin_bit_cast(__bf16, v);
      }
    }
#pragma unroll
    for (int p = 0; p < NS; ++p) {
      const unsigned short* qp = Q + ((size_t)p * kLP + (lane & 15)) * Np + kk;
      const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(qp);
      const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(qp + (size_t)16 * Np);
      acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b0, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b1, acc1, 0, 0, 0);
    }
  }
  // lane holds rows r0 + 4*(lane/16) + i, labels lane%16 and 16 + lane%16
  float* sp = a.s_part + ((size_t)b * a.KS + ks) * Np * kLP;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = r0 + 4 * (lane >> 4) + i;
    sp[(size_t)r * kLP + (lane & 15)] = acc0[i];
    sp[(size_t)r * kLP + 16 + (lane & 15)] = acc1[i];
  }

  // --- the last slice of this row block runs the per-node step ---------------
  __shared__ int is_last;
  __shared__ float Ts[kLP];
  __threadfence();
  __syncthreads();
  if (tid == 0) is_last = (atomicAdd(&a.counters[b * a.NRB + rb], 1) == a.KS - 1);
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  if (COOC) {
    if (tid < kLP) {
      float t = 0.f;
      for (int k = 0; k < a.NRB; ++k) t += a.t_in[((size_t)b * a.NRB + k) * kLP + tid];
      Ts[tid] = t;
    }
    __syncthreads();
  }
  if (tid == 0) a.counters[b * a.NRB + rb] = 0;
  if (wave != 0) return;

  const int i = rb * kRB + lane;
  const bool inside = i < N;
  float S[kLP], ell[kLP], z[kLP], e[kLP];
#pragma unroll
  for (int l = 0; l < kLP; ++l) S[l] = 0.f;
  for (int k = 0; k < a.KS; ++k) {
    const float4* src = reinterpret_cast<const float4*>(a.s_part + (((size_t)b * a.KS + k) * Np + i) * kLP);
#pragma unroll
    for (int v = 0; v < kLP / 4; ++v) {
      const float4 x = src[v];
      S[4 * v] += x.x;
      S[4 * v + 1] += x.y;
      S[4 * v + 2] += x.z;
      S[4 * v + 3] += x.w;
    }
  }
  const size_t base = (size_t)b * L * N + (inside ? i : 0);
  float qo[kLP];
#pragma unroll
  for (int l = 0; l < kLP; ++l) {
    ell[l] = (inside && l < L) ? a.state_in[base + (size_t)l * N] : 0.f;
    qo[l] = (inside && l < L) ? __expf(ell[l]) : 0.f;
  }

  float tot = 0.f;
  if (COMPAT == MF_COMPAT_POTTS) {
#pragma unroll
    for (int l = 0; l < kLP; ++l) tot += (l < L) ? S[l] : 0.f;
  }
  float mx = -INFINITY;
#pragma unroll
  for (int l = 0; l < kLP; ++l) {
    z[l] = -INFINITY;
    if (l < L) {
      float m = inside ? a.unary[base + (size_t)l * N] : 0.f;
      if (COMPAT == MF_COMPAT_POTTS) {
        m += a.potts_w * (tot - S[l]);
      } else {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < kLP; ++k)
          if (k < L) acc = fmaf(a.theta[l * L + k], S[k], acc);
        m += acc;
      }
      if (COOC) {
        float c = 0.f;
#pragma unroll
        for (int k = 0; k < kLP; ++k)
          if (k < L) c = fmaf(a.cooc[l * L + k], Ts[k] - qo[k], c);
        m += c * a.inv_n;
      }
      z[l] = one_minus_alpha * ell[l] - a.alpha * m;
      mx = fmaxf(mx, z[l]);
    }
  }
  float se = 0.f;
#pragma unroll
  for (int l = 0; l < kLP; ++l) {
    e[l] = (l < L) ? __expf(z[l] - mx) : 0.f;
    se += e[l];
  }
  const float lse = mx + __logf(se);
  const float inv = 1.0f / se;
  unsigned short* planes = a.q_out + (size_t)b * NS * kLP * Np;
#pragma unroll
  for (int l = 0; l < kLP; ++l) {
    const float q = inside ? e[l] * inv : 0.f;
    if (inside && l < L) a.state_out[base + (size_t)l * N] = z[l] - lse;
    store_planes<NS>(planes, Np, l, i, q);
    const float t = wave_sum_f(q);
    if (lane == 0) a.t_out[((size_t)b * a.NRB + rb) * kLP + l] = t;
  }
}

// FP64 free energy.  qd[b][j][l] = exp(log q) in FP64 (node-major).
__global__ __launch_bounds__(256) void dense_fe_prep_kernel(const float* __restrict__ state, double* __restrict__ qd,
                                                            int L, int N) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int b = blockIdx.y;
  if (j >= N) return;
  for (int l = 0; l < L; ++l)
    qd[((size_t)b * N + j) * L + l] = exp((double)state[((size_t)b * L + l) * N + j]);
}

__device__ inline double wave_sum_dd(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// f_i = sum_l q_il (u_il + log q_il) + 1/2 q_i . (Theta S_i) + 1/(2N) q_i . C (T - q_i)
template <int COMPAT, bool COOC>
__global__ __launch_bounds__(256) void dense_fe_kernel(DenseFreeEnergyArgs a) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int b = blockIdx.y;
  const int L = a.L, N = a.N;
  const double* qd = a.qd + (size_t)b * N * L;
  double f = 0.0;
  if (i < N) {
    double S[kLP], T[kLP];
#pragma unroll
    for (int l = 0; l < kLP; ++l) S[l] = T[l] = 0.0;
    for (int j = 0; j < N; ++j) {
      const double k = (double)bf2f(a.K[(size_t)j * N + i]);   // K symmetric: column read, coalesced
      const double* qj = qd + (size_t)j * L;
#pragma unroll
      for (int l = 0; l < kLP; ++l) {
        if (l < L) {
          const double q = qj[l];
          S[l] += k * q;
          T[l] += q;
        }
      }
    }
    double tot = 0.0;
#pragma unroll
    for (int l = 0; l < kLP; ++l) tot += S[l];
    const size_t base = (size_t)b * L * N + i;
    const double* qi = qd + (size_t)i * L;
#pragma unroll
    for (int l = 0; l < kLP; ++l) {
      if (l < L) {
        const double lq = (double)a.state[base + (size_t)l * N];
        const double q = qi[l];
        double pm = 0.0;
        if (COMPAT == MF_COMPAT_POTTS) {
          pm = (double)a.potts_w * (tot - S[l]);
        } else {
#pragma unroll
          for (int k = 0; k < kLP; ++k)
            if (k < L) pm += (double)a.theta[l * L + k] * S[k];
        }
        if (COOC) {
          double c = 0.0;
#pragma unroll
          for (int k = 0; k < kLP; ++k)
            if (k < L) c += (double)a.cooc[l * L + k] * (T[k] - qi[k]);
          pm += c / (double)N;
        }
        f += q * ((double)a.unary[base + (size_t)l * N] + lq + 0.5 * pm);
      }
    }
  }
  __shared__ double red[4];
  f = wave_sum_dd(f);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = f;
  __syncthreads();
  if (threadIdx.x == 0) a.partials[(size_t)b * a.n_blocks + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

template <int NS>
hipError_t step_ns(const DenseStepArgs& a, int compat, hipStream_t s) {
  dim3 grid(a.NRB * a.KS, a.B);
  const float om = (float)(1.0 - (double)a.alpha);
  const bool cooc = a.cooc != nullptr;
  if (compat == MF_COMPAT_POTTS) {
    if (cooc) hipLaunchKernelGGL((dense_step_kernel<NS, MF_COMPAT_POTTS, true>), grid, dim3(256), 0, s, a, om);
    else hipLaunchKernelGGL((dense_step_kernel<NS, MF_COMPAT_POTTS, false>), grid, dim3(256), 0, s, a, om);
  } else {
    if (cooc) hipLaunchKernelGGL((dense_step_kernel<NS, MF_COMPAT_GENERAL, true>), grid, dim3(256), 0, s, a, om);
    else hipLaunchKernelGGL((dense_step_kernel<NS, MF_COMPAT_GENERAL, false>), grid, dim3(256), 0, s, a, om);
  }
  return hipGetLastError();
}

}  // namespace

int dense_planes(int precision) { return precision == MF_P_F32 ? 3 : precision == MF_P_F16MSG ? 2 : 1; }

DenseGeometry dense_geometry(int N, int B) {
  DenseGeometry g;
  g.Np = (N + kRB - 1) / kRB * kRB;
  g.NRB = g.Np / kRB;
  // slices of the j range: enough workgroups to cover the compute units,
  // each slice at least 256 columns wide
  int ks = (512 + g.NRB * B - 1) / (g.NRB * B);
  const int max_ks = g.Np / 256 > 0 ? g.Np / 256 : 1;
  ks = ks < 1 ? 1 : (ks > max_ks ? max_ks : ks);
  const int chunks = g.Np / 32;
  g.jchunk = (chunks + ks - 1) / ks * 32;
  g.KS = (g.Np + g.jchunk - 1) / g.jchunk;
  return g;
}

hipError_t launch_dense_kernel(const float* f, int n, int dim, uint16_t* K, hipStream_t s) {
  dim3 grid((n + 255) / 256, n);
  hipLaunchKernelGGL(dense_kernel_build, grid, dim3(256), 0, s, f, n, dim, K);
  return hipGetLastError();
}

hipError_t launch_dense_prepare(const DenseStepArgs& a, int NS, hipStream_t s) {
  dim3 grid(a.NRB, a.B);
  switch (NS) {
    case 3: hipLaunchKernelGGL(dense_prepare_kernel<3>, grid, dim3(64), 0, s, a); break;
    case 2: hipLaunchKernelGGL(dense_prepare_kernel<2>, grid, dim3(64), 0, s, a); break;
    default: hipLaunchKernelGGL(dense_prepare_kernel<1>, grid, dim3(64), 0, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_dense_step(const DenseStepArgs& a, int NS, int compat, hipStream_t s) {
  switch (NS) {
    case 3: return step_ns<3>(a, compat, s);
    case 2: return step_ns<2>(a, compat, s);
    default: return step_ns<1>(a, compat, s);
  }
}

hipError_t launch_dense_free_energy(const DenseFreeEnergyArgs& a, int compat, hipStream_t s) {
  dim3 grid((a.N + 255) / 256, a.B);
  hipLaunchKernelGGL(dense_fe_prep_kernel, grid, dim3(256), 0, s, a.state, a.qd, a.L, a.N);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const bool cooc = a.cooc != nullptr;
  if (compat == MF_COMPAT_POTTS) {
    if (cooc) hipLaunchKernelGGL((dense_fe_kernel<MF_COMPAT_POTTS, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((dense_fe_kernel<MF_COMPAT_POTTS, false>), grid, dim3(256), 0, s, a);
  } else {
    if (cooc) hipLaunchKernelGGL((dense_fe_kernel<MF_COMPAT_GENERAL, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((dense_fe_kernel<MF_COMPAT_GENERAL, false>), grid, dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace mf
