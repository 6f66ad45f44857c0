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
// Layout in HBM: both MFMA operands are stored in the order the matrix
// cores take them, so every operand load of a wavefront reads 1 KiB of
// contiguous memory (a row-major K would make each load touch 16 rows 8 KiB
// apart: 16 address translations and half-used cache lines per load).  K is
// copied once per solve (mf_init, mf_solve) into the workspace as
// [Np/64][Np/32][4][64][8]: 64-row block, 32-column chunk, 16-row tile,
// lane, element, where lane x of tile t holds row 16 t + x % 16, columns
// 8 (x / 16) .. + 7 of the chunk, zero past N.  The q planes are written by
// the step itself as [Np/32][NS][2][64][8]: column chunk, plane, label half,
// lane, element, where lane x holds label 16 h + x % 16 at nodes
// 8 (x / 16) .. + 7 of the chunk.
//
// Work split: a workgroup owns a 64-row block and one of KS slices of the
// j range; its eight wavefronts split the slice's 32-column chunks and each
// accumulates the whole 64 x 32 (rows x labels, L padded to 32) tile in
// registers.  Slices write FP32 partial sums.  A second kernel, one
// workgroup per 64-row block, adds the KS partials in a fixed order and
// runs the per-node step, so the result is deterministic; it also writes
// the next Q planes and the block's column sums of q, which the
// co-occurrence term of the next step reduces in a fixed order.  The
// hand-off between the two is the kernel boundary: the eight XCDs of the
// MI355X have separate L2 caches, and a device-scope fence per workgroup
// (to hand the partials to a last-arriving workgroup inside one kernel)
// writes back the issuing XCD's L2 every time.
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

// Sum over the 64 lanes in the VALU, one fixed order: rotations by 8, 4, 2
// and 1 within each row of 16 lanes (DPP), then rows 0 + 1 and 2 + 3
// (v_permlane16_swap) and the two half-waves (v_permlane32_swap).  Lane 0
// holds the sum.
template <int N>
__device__ inline float row_ror(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x120 + N, 0xF, 0xF, false));
}
__device__ inline float wave_sum_dpp(float v) {
  v += row_ror<8>(v);
  v += row_ror<4>(v);
  v += row_ror<2>(v);
  v += row_ror<1>(v);
  const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = __uint_as_float(p[0]) + __uint_as_float(p[1]);
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
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

// Split q (FP32) of label l at node i into NS BF16 planes, stored in the
// B-operand order of the step kernel.
template <int NS>
__device__ inline void store_planes(unsigned short* __restrict__ planes, int l, int i, float q) {
  const int k = i & 31;
  const size_t at = ((size_t)(i >> 5) * NS * 2 + (l >> 4)) * 512 + ((l & 15) + 16 * (k >> 3)) * 8 + (k & 7);
  float r = q;
#pragma unroll
  for (int p = 0; p < NS; ++p) {
    const unsigned short h = f2bf_rne(r);
    planes[at + (size_t)p * 1024] = h;
    r -= bf2f(h);
  }
}

// K (row-major, the caller's) -> Kt (MFMA operand order, zero-padded to Np).
// One thread per 16-byte operand slot, in Kt order: a wavefront writes 1 KiB
// of contiguous memory and reads 64 bytes from each of 16 rows of K.
__global__ __launch_bounds__(256) void dense_tile_k_kernel(const unsigned short* __restrict__ K, int N, int Np,
                                                           bf16x8* __restrict__ Kt) {
  const size_t c = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= (size_t)Np * (Np / 8)) return;
  const int lane = (int)(c & 63), t = (int)((c >> 6) & 3);
  const size_t tile = c >> 8;                       // rb * (Np / 32) + ct
  const int ct = (int)(tile % (size_t)(Np / 32)), rb = (int)(tile / (size_t)(Np / 32));
  const int row = 64 * rb + 16 * t + (lane & 15), col = 32 * ct + 8 * (lane >> 4);
  bf16x8 v;
  if ((N & 7) == 0 && row < N && col < N) {
    v = *reinterpret_cast<const bf16x8*>(K + (size_t)row * N + col);
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const unsigned short x = (row < N && col + e < N) ? K[(size_t)row * N + col + e] : (unsigned short)0;
      v[e] = __builtin_bit_cast(__bf16, x);
    }
  }
  Kt[c] = v;
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
    store_planes<NS>(planes, l, i, q);
    const float t = wave_sum_dpp(q);
    if (lane == 0) a.t_out[((size_t)b * a.NRB + rb) * kLP + l] = t;
  }
}

// One workgroup: the 64-row block rb against the j slice ks.  Each of the
// kStepWaves wavefronts holds the whole 64 x 32 tile (four 16-row MFMA
// tiles) and takes every kStepWaves-th 32-column step of the slice, so a Q
// operand it loads meets four K operands and no two wavefronts load the
// same Q columns.  The per-wavefront tiles are added through LDS in
// wavefront order.
constexpr int kPSt = kLP + 1;    // LDS row stride of the per-wavefront tiles
constexpr int kStepWaves = 8;    // wavefronts per workgroup of the MFMA kernel (8 measured
                                 // faster than 4: one load trip per wavefront)

template <int NS>
__global__ __launch_bounds__(64 * kStepWaves) void dense_step_kernel(DenseStepArgs a) {
  constexpr int NW = kStepWaves, NT = 64 * NW;
  __shared__ float part[NW * kRB * kPSt];
  const int b = blockIdx.y;
  const int rb = blockIdx.x / a.KS, ks = blockIdx.x - (blockIdx.x / a.KS) * a.KS;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int Np = a.Np;
  const int c0 = ks * (a.jchunk / 32);                           // first 32-column chunk of the slice
  const int nst = (min((ks + 1) * a.jchunk, Np) - ks * a.jchunk) / 32;
  const bf16x8* __restrict__ Kb = reinterpret_cast<const bf16x8*>(a.Kt) + ((size_t)rb * (Np / 32) + c0) * 256 + lane;
  const bf16x8* __restrict__ Qb =
      reinterpret_cast<const bf16x8*>(a.q_in + (size_t)b * NS * kLP * Np) + (size_t)c0 * NS * 128 + lane;
  auto load_k = [&](int st_, int t) { return Kb[((size_t)st_ * 4 + t) * 64]; };
  auto load_q = [&](int st_, int p, int half) { return Qb[((size_t)st_ * NS * 2 + p * 2 + half) * 64]; };
  f32x4 acc[4][2];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t][0] = acc[t][1] = f32x4{0.f, 0.f, 0.f, 0.f};

  // two of the wavefront's steps per trip: all their loads before their MFMAs
  constexpr int U = 2;
  int st = wave;
  for (; st + NW * (U - 1) < nst; st += NW * U) {
    bf16x8 av[U][4], bq[U][NS][2];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int t = 0; t < 4; ++t) av[u][t] = load_k(st + NW * u, t);
#pragma unroll
      for (int p = 0; p < NS; ++p) {
        bq[u][p][0] = load_q(st + NW * u, p, 0);
        bq[u][p][1] = load_q(st + NW * u, p, 1);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int p = 0; p < NS; ++p)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          acc[t][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[u][t], bq[u][p][0], acc[t][0], 0, 0, 0);
          acc[t][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[u][t], bq[u][p][1], acc[t][1], 0, 0, 0);
        }
  }
  for (; st < nst; st += NW) {
    bf16x8 av[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) av[t] = load_k(st, t);
#pragma unroll
    for (int p = 0; p < NS; ++p) {
      const bf16x8 b0 = load_q(st, p, 0), b1 = load_q(st, p, 1);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        acc[t][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[t], b0, acc[t][0], 0, 0, 0);
        acc[t][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[t], b1, acc[t][1], 0, 0, 0);
      }
    }
  }
  // lane holds rows 16 t + 4 (lane / 16) + i, labels lane % 16 and 16 + lane % 16
  float* pw = part + wave * kRB * kPSt;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 16 * t + 4 * (lane >> 4) + i;
      pw[r * kPSt + (lane & 15)] = acc[t][0][i];
      pw[r * kPSt + 16 + (lane & 15)] = acc[t][1][i];
    }
  __syncthreads();
  float* sp = a.s_part + (((size_t)b * a.KS + ks) * Np + (size_t)rb * kRB) * kLP;
#pragma unroll
  for (int r = 0; r < kRB * kLP / NT; ++r) {
    const int f = tid + NT * r, o = (f / kLP) * kPSt + (f % kLP);
    float v = part[o];                   // wavefront order
#pragma unroll
    for (int w = 1; w < NW; ++w) v += part[w * kRB * kPSt + o];
    sp[f] = v;
  }
}

// The per-node step of one 64-row block: the KS partial sums of S in a fixed
// order, the message, the step, the next Q planes and the block's column
// sums of q.  kEpiGroups wavefronts: lane = node of the block, wavefront
// w = label group (labels w + kEpiGroups j).  The partials arrive node-major and are
// transposed through LDS (coalesced loads); the terms that mix labels
// (Theta S, the co-occurrence product, the per-node max and sum) read the
// node's other labels from LDS.  LC > 0 fixes L at compile time so the
// label loops unroll; every global load is issued before the first wait.
constexpr int kEpiGroups = 8;                 // label groups (wavefronts) per 64-node block:
                                              // 8 measured faster than 4 (shorter per-thread chains)
constexpr int kEpiThreads = 64 * kEpiGroups;
constexpr int kSt = kLP + 1;          // LDS row stride of the node x label tiles
constexpr int kTParts = kEpiThreads / kLP;

template <int NS, int COMPAT, bool COOC, int LC>
__global__ __launch_bounds__(kEpiThreads) void dense_epilogue_kernel(DenseStepArgs a, float one_minus_alpha) {
  const int rb = blockIdx.x, b = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // label group, uniform in the wavefront
  const int L = LC > 0 ? LC : a.L, N = a.N, Np = a.Np;
  __shared__ float Th[kLP * kLP];      // Theta (general), rows of stride 32
  __shared__ float Cc[kLP * kLP];      // co-occurrence
  __shared__ float St[kRB * kSt];      // S[node][label]
  __shared__ float Qt[kRB * kSt];      // q[node][label] (co-occurrence)
  __shared__ float red[kEpiGroups * kRB];   // per-node partials of the label groups
  __shared__ float Tp[kEpiThreads];    // partial column sums of q at the previous step
  __shared__ float Ts[kLP];

  const int i = rb * kRB + lane;
  const bool inside = i < N;
  const size_t base = (size_t)b * L * N + (inside ? i : 0);
  constexpr int NG = kEpiGroups, J = kLP / NG;
  // per-node total over the label groups, in one fixed order
  auto group_sum = [&]() {
    float v = red[lane];
#pragma unroll
    for (int g = 1; g < NG; ++g) v += red[g * kRB + lane];
    return v;
  };
  float ell[J], un[J], z[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int l = w + NG * j;
    const bool on = inside && l < L;
    ell[j] = on ? a.state_in[base + (size_t)l * N] : 0.f;
    un[j] = on ? a.unary[base + (size_t)l * N] : 0.f;
  }
  if (COMPAT != MF_COMPAT_POTTS)
    for (int f = tid; f < L * L; f += kEpiThreads) Th[(f / L) * kLP + f % L] = a.theta[f];
  if (COOC)
    for (int f = tid; f < L * L; f += kEpiThreads) Cc[(f / L) * kLP + f % L] = a.cooc[f];
  if (COOC) {
    // column sums: label tid % 32, blocks tid / 32 + 8 k in order
    const int l = tid % kLP;
    float t = 0.f;
#pragma unroll 8
    for (int k = tid / kLP; k < a.NRB; k += kTParts) t += a.t_in[((size_t)b * a.NRB + k) * kLP + l];
    Tp[tid] = t;
  }
  // S = sum over the KS slices, element by element in slice order
  {
    const float* sp = a.s_part + ((size_t)b * a.KS * Np + (size_t)rb * kRB) * kLP;
    float acc[kRB * kLP / kEpiThreads];
#pragma unroll
    for (int r = 0; r < kRB * kLP / kEpiThreads; ++r) acc[r] = 0.f;
#pragma unroll 8
    for (int k = 0; k < a.KS; ++k) {
#pragma unroll
      for (int r = 0; r < kRB * kLP / kEpiThreads; ++r) acc[r] += sp[(size_t)k * Np * kLP + tid + r * kEpiThreads];
    }
#pragma unroll
    for (int r = 0; r < kRB * kLP / kEpiThreads; ++r) {
      const int f = tid + r * kEpiThreads;
      St[(f / kLP) * kSt + (f % kLP)] = acc[r];
    }
  }
  if (COOC) {
#pragma unroll
    for (int j = 0; j < J; ++j) Qt[lane * kSt + w + NG * j] = (inside && w + NG * j < L) ? __expf(ell[j]) : 0.f;
  }
  __syncthreads();
  if (COOC && tid < kLP) {
    float t = 0.f;
#pragma unroll
    for (int p = 0; p < kTParts; ++p) t += Tp[p * kLP + tid];
    Ts[tid] = t;
  }

  float tot = 0.f;
  if (COMPAT == MF_COMPAT_POTTS) {
    float part = 0.f;
#pragma unroll
    for (int j = 0; j < J; ++j) part += (w + NG * j < L) ? St[lane * kSt + w + NG * j] : 0.f;
    red[w * kRB + lane] = part;
  }
  __syncthreads();
  if (COMPAT == MF_COMPAT_POTTS) tot = group_sum();
  // the node's S and q rows, read once
  float srow[kLP], qrow[kLP];
  if (COMPAT != MF_COMPAT_POTTS) {
#pragma unroll
    for (int k = 0; k < kLP; ++k) srow[k] = (LC == 0 || k < L) ? St[lane * kSt + k] : 0.f;
  }
  if (COOC) {
#pragma unroll
    for (int k = 0; k < kLP; ++k) qrow[k] = (LC == 0 || k < L) ? Ts[k] - Qt[lane * kSt + k] : 0.f;
  }
  float mx = -INFINITY;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int l = w + NG * j;
    z[j] = -INFINITY;
    if (l < L) {
      float m = un[j];
      if (COMPAT == MF_COMPAT_POTTS) {
        m += a.potts_w * (tot - St[lane * kSt + l]);
      } else {
        float acc = 0.f;
        if constexpr (LC > 0) {
#pragma unroll
          for (int k = 0; k < LC; ++k) acc = fmaf(Th[l * kLP + k], srow[k], acc);
        } else {
          for (int k = 0; k < L; ++k) acc = fmaf(Th[l * kLP + k], St[lane * kSt + k], acc);
        }
        m += acc;
      }
      if (COOC) {
        float c = 0.f;
        if constexpr (LC > 0) {
#pragma unroll
          for (int k = 0; k < LC; ++k) c = fmaf(Cc[l * kLP + k], qrow[k], c);
        } else {
          for (int k = 0; k < L; ++k) c = fmaf(Cc[l * kLP + k], Ts[k] - Qt[lane * kSt + k], c);
        }
        m += c * a.inv_n;
      }
      z[j] = one_minus_alpha * ell[j] - a.alpha * m;
      mx = fmaxf(mx, z[j]);
    }
  }
  // per-node max and sum over the label groups, fixed order
  __syncthreads();
  red[w * kRB + lane] = mx;
  __syncthreads();
  mx = red[lane];
#pragma unroll
  for (int g = 1; g < NG; ++g) mx = fmaxf(mx, red[g * kRB + lane]);
  __syncthreads();
  float e[J];
  float se = 0.f;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    e[j] = (w + NG * j < L) ? __expf(z[j] - mx) : 0.f;
    se += e[j];
  }
  red[w * kRB + lane] = se;
  __syncthreads();
  se = group_sum();
  const float lse = mx + __logf(se);
  const float inv = 1.0f / se;
  unsigned short* planes = a.q_out + (size_t)b * NS * kLP * Np;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int l = w + NG * j;
    const float q = inside ? e[j] * inv : 0.f;
    if (inside && l < L) a.state_out[base + (size_t)l * N] = z[j] - lse;
    store_planes<NS>(planes, l, i, q);
    if (COOC) {
      const float t = wave_sum_dpp(q);
      if (lane == 0) a.t_out[((size_t)b * a.NRB + rb) * kLP + l] = t;
    }
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

template <int NS, int LC>
hipError_t epilogue_lc(const DenseStepArgs& a, int compat, float om, hipStream_t s) {
  const dim3 grid(a.NRB, a.B);
  const bool cooc = a.cooc != nullptr;
  if (compat == MF_COMPAT_POTTS) {
    if (cooc) hipLaunchKernelGGL((dense_epilogue_kernel<NS, MF_COMPAT_POTTS, true, LC>), grid, dim3(kEpiThreads), 0, s, a, om);
    else hipLaunchKernelGGL((dense_epilogue_kernel<NS, MF_COMPAT_POTTS, false, LC>), grid, dim3(kEpiThreads), 0, s, a, om);
  } else {
    if (cooc) hipLaunchKernelGGL((dense_epilogue_kernel<NS, MF_COMPAT_GENERAL, true, LC>), grid, dim3(kEpiThreads), 0, s, a, om);
    else hipLaunchKernelGGL((dense_epilogue_kernel<NS, MF_COMPAT_GENERAL, false, LC>), grid, dim3(kEpiThreads), 0, s, a, om);
  }
  return hipGetLastError();
}

template <int NS>
hipError_t step_ns(const DenseStepArgs& a, int compat, hipStream_t s) {
  hipLaunchKernelGGL((dense_step_kernel<NS>), dim3(a.NRB * a.KS, a.B), dim3(64 * kStepWaves), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const float om = (float)(1.0 - (double)a.alpha);
  return a.L == 21 ? epilogue_lc<NS, 21>(a, compat, om, s) : epilogue_lc<NS, 0>(a, compat, om, s);
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

hipError_t launch_dense_tile_k(const DenseStepArgs& a, hipStream_t s) {
  const size_t chunks = (size_t)a.Np * (a.Np / 8);
  hipLaunchKernelGGL(dense_tile_k_kernel, dim3((unsigned)((chunks + 255) / 256)), dim3(256), 0, s, a.K, a.N, a.Np,
                     reinterpret_cast<bf16x8*>(a.Kt));
  return hipGetLastError();
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
