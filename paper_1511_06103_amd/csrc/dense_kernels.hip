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
// workgroup per 16 nodes, adds the KS partials in a fixed order and runs
// the per-node step, so the result is deterministic; it also writes the
// next Q planes and the block's column sums of q, which the co-occurrence
// term of the next step reduces in a fixed order.  The
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

// The per-node kernels (q^0 planes, and the step after the product) take
// kEB = 16 nodes per workgroup: wavefront w holds nodes 2w and 2w + 1 of the
// block, lane x node 2w + x / 32 and label slot x % 32.  A node's labels
// are then one half-wave, so its max and sum reduce with an xor butterfly
// of shuffles (the two lanes of a pair add the same operands, so every lane
// gets a bitwise-identical total), and N = 4096 gives 256 workgroups.
constexpr int kEB = 16;                  // nodes per workgroup
constexpr int kNT = 64 * kEB / 2;        // threads: eight wavefronts of two nodes
constexpr int kQSt = kLP + 1;            // LDS row stride (conflict-free across the label lanes)

// Column sums of q over the block's 16 nodes in node order: each wavefront's
// pair first, then the wavefronts in order.  Every thread calls it.
__device__ inline void block_col_sums(float q, float* __restrict__ red, float* __restrict__ t_row, int tid) {
  const int wave = tid >> 6, lane = tid & 63;
  const float pair = q + __shfl_xor(q, 32);
  if (lane < kLP) red[wave * kLP + lane] = pair;
  __syncthreads();
  if (tid < kLP) {
    float t = red[tid];
#pragma unroll
    for (int w = 1; w < kNT / 64; ++w) t += red[w * kLP + tid];
    t_row[tid] = t;
  }
}

// q^0 planes and the blocks' column sums from the initial state.
template <int NS>
__global__ __launch_bounds__(kNT) void dense_prepare_kernel(DenseStepArgs a) {
  __shared__ float red[kNT / 64 * kLP];
  const int eb = blockIdx.x, b = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, l = lane & 31;
  const int i = eb * kEB + 2 * (tid >> 6) + (lane >> 5);
  const int L = a.L, N = a.N;
  float q = 0.f;
  if (i < N && l < L) q = __expf(a.state_in[((size_t)b * L + l) * N + i]);
  store_planes<NS>(a.q_out + (size_t)b * NS * kLP * a.Np, l, i, q);
  block_col_sums(q, red, a.t_out + ((size_t)b * a.NEB + eb) * kLP, tid);
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

// The per-node step of 16 nodes (mapping as for dense_prepare_kernel): the
// KS partial sums of S in slice order (node-major, so a wavefront's loads
// are 256 contiguous bytes), the message, the step, the next Q planes and
// the block's column sums of q.  The terms that mix labels (Theta S, the
// co-occurrence product) read the node's S and q rows from LDS; Theta and C
// are staged there too.  LC > 0 fixes L at compile time so the label loops
// unroll.
template <int NS, int COMPAT, bool COOC, int LC>
__global__ __launch_bounds__(kNT) void dense_epilogue_kernel(DenseStepArgs a, float one_minus_alpha) {
  constexpr bool GEN = COMPAT != MF_COMPAT_POTTS;
  __shared__ float Th[GEN ? kLP * kQSt : 1];        // Theta (general)
  __shared__ float Cc[COOC ? kLP * kQSt : 1];       // co-occurrence
  __shared__ float Sr[kEB * kQSt];                  // S rows of the block's nodes
  __shared__ float Qr[COOC ? kEB * kQSt : 1];       // q rows (co-occurrence)
  __shared__ float Tp[COOC ? kNT : 1];              // partial column sums of q at the previous step
  __shared__ float Ts[kLP];
  __shared__ float red[kNT / 64 * kLP];
  const int eb = blockIdx.x, b = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, l = lane & 31;
  const int nl = 2 * (tid >> 6) + (lane >> 5);      // node within the block
  const int i = eb * kEB + nl;
  const int L = LC > 0 ? LC : a.L, N = a.N, Np = a.Np;
  const bool valid = i < N && l < L;
  // every global load is issued before the first wait; addresses are clamped
  const size_t at = ((size_t)b * L + (l < L ? l : L - 1)) * N + (i < N ? i : N - 1);
  const float ell = a.state_in[at];
  const float un = a.unary[at];
  if (GEN)
    for (int f = tid; f < L * L; f += kNT) Th[(f / L) * kQSt + f % L] = a.theta[f];
  if (COOC) {
    for (int f = tid; f < L * L; f += kNT) Cc[(f / L) * kQSt + f % L] = a.cooc[f];
    // column sums: label tid % 32, blocks tid / 32 + 16 k in order
    const int lt = tid % kLP;
    float t = 0.f;
    // 16 loads per trip: one round trip for the 256 blocks of 4096 nodes
#pragma unroll 16
    for (int k = tid / kLP; k < a.NEB; k += kNT / kLP) t += a.t_in[((size_t)b * a.NEB + k) * kLP + lt];
    Tp[tid] = t;
  }
  float S = 0.f;
  {
    const float* sp = a.s_part + ((size_t)b * a.KS * Np + i) * kLP + l;
#pragma unroll 8
    for (int k = 0; k < a.KS; ++k) S += sp[(size_t)k * Np * kLP];
  }
  Sr[nl * kQSt + l] = S;
  if (COOC) Qr[nl * kQSt + l] = valid ? __expf(ell) : 0.f;
  __syncthreads();
  if (COOC && tid < kLP) {
    float t = 0.f;
#pragma unroll
    for (int p = 0; p < kNT / kLP; ++p) t += Tp[p * kLP + tid];
    Ts[tid] = t;
  }
  if (COOC) __syncthreads();

  const float* srow = Sr + nl * kQSt;
  float m = un;
  if (!GEN) {
    float tot = 0.f;
    if constexpr (LC > 0) {
#pragma unroll
      for (int k = 0; k < LC; ++k) tot += srow[k];
    } else {
      for (int k = 0; k < L; ++k) tot += srow[k];
    }
    m += a.potts_w * (tot - S);
  } else if (l < L) {
    const float* th = Th + l * kQSt;
    float acc = 0.f;
    if constexpr (LC > 0) {
#pragma unroll
      for (int k = 0; k < LC; ++k) acc = fmaf(th[k], srow[k], acc);
    } else {
      for (int k = 0; k < L; ++k) acc = fmaf(th[k], srow[k], acc);
    }
    m += acc;
  }
  if (COOC && l < L) {
    const float* cr = Cc + l * kQSt;
    const float* qrow = Qr + nl * kQSt;
    float c = 0.f;
    if constexpr (LC > 0) {
#pragma unroll
      for (int k = 0; k < LC; ++k) c = fmaf(cr[k], Ts[k] - qrow[k], c);
    } else {
      for (int k = 0; k < L; ++k) c = fmaf(cr[k], Ts[k] - qrow[k], c);
    }
    m += c * a.inv_n;
  }
  const float z = valid ? one_minus_alpha * ell - a.alpha * m : -INFINITY;
  // per-node max and sum over the node's half-wave
  float mx = z;
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 32));
  const float e = valid ? __expf(z - mx) : 0.f;
  float se = e;
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) se += __shfl_xor(se, off, 32);
  const float lse = mx + __logf(se);
  const float q = valid ? e * (1.0f / se) : 0.f;
  if (valid) a.state_out[at] = z - lse;
  store_planes<NS>(a.q_out + (size_t)b * NS * kLP * Np, l, i, q);
  if (COOC) block_col_sums(q, red, a.t_out + ((size_t)b * a.NEB + eb) * kLP, tid);
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
  const dim3 grid(a.NEB, a.B);
  const bool cooc = a.cooc != nullptr;
  if (compat == MF_COMPAT_POTTS) {
    if (cooc) hipLaunchKernelGGL((dense_epilogue_kernel<NS, MF_COMPAT_POTTS, true, LC>), grid, dim3(kNT), 0, s, a, om);
    else hipLaunchKernelGGL((dense_epilogue_kernel<NS, MF_COMPAT_POTTS, false, LC>), grid, dim3(kNT), 0, s, a, om);
  } else {
    if (cooc) hipLaunchKernelGGL((dense_epilogue_kernel<NS, MF_COMPAT_GENERAL, true, LC>), grid, dim3(kNT), 0, s, a, om);
    else hipLaunchKernelGGL((dense_epilogue_kernel<NS, MF_COMPAT_GENERAL, false, LC>), grid, dim3(kNT), 0, s, a, om);
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
  g.NEB = g.Np / kEB;
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
  dim3 grid(a.NEB, a.B);
  switch (NS) {
    case 3: hipLaunchKernelGGL(dense_prepare_kernel<3>, grid, dim3(kNT), 0, s, a); break;
    case 2: hipLaunchKernelGGL(dense_prepare_kernel<2>, grid, dim3(kNT), 0, s, a); break;
    default: hipLaunchKernelGGL(dense_prepare_kernel<1>, grid, dim3(kNT), 0, s, a); break;
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
