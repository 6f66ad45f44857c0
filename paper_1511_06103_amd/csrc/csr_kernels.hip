// General sparse graphs (CSR): the parallel proximal step with a gathered
// neighbour aggregation, its initialisation, the FP64 free energy and a
// device-side check of the CSR arrays.
//
// S_i = sum_{e in row i} w_e q_{col[e]}   (neighbour aggregation, Sec. 2.2.2)
// m_i = u_i + Theta S_i;  z_i = (1 - alpha) log q_i - alpha m_i;
// log q_i <- z_i - logsumexp(z_i)          (Eq. 15 with Eq. 16)
//
// The gather reads a node-major copy of q ([B][N][LQ], LQ = L rounded up to
// a multiple of 4, padding zero) so each neighbour costs LQ / 4 contiguous
// 16-byte loads instead of L scattered 4-byte loads from the label-major
// state.  The step writes the next node-major q itself (q' = exp(z - max) /
// sum, taken from the log-sum-exp), so no separate transpose pass runs.
#include <hip/hip_runtime.h>

#include "mf_internal.h"

namespace mf {
namespace {

constexpr int kCsrThreads = 256;

// Flags (workspace int32 word 0): bit 0 non-finite input, bit 1 malformed CSR.
__global__ __launch_bounds__(kCsrThreads) void csr_check_kernel(const int* __restrict__ row_ptr,
                                                                const int* __restrict__ col, int N,
                                                                long long nnz, int* __restrict__ flags) {
  const int i = blockIdx.x * kCsrThreads + threadIdx.x;
  if (i > N) return;
  bool bad = false;
  const int r = row_ptr[i];
  if (i == 0 && r != 0) bad = true;
  if (i == N && (long long)r != nnz) bad = true;
  if (i < N) {
    const int r1 = row_ptr[i + 1];
    if (r1 < r || r < 0 || (long long)r1 > nnz) {
      bad = true;
    } else {
      for (int e = r; e < r1; ++e) {
        const int j = col[e];
        if (j < 0 || j >= N) bad = true;
      }
    }
  }
  if (bad) atomicOr(flags, 2);
}

// Node-major q from the label-major log q (after initialisation).
template <int LQ>
__global__ __launch_bounds__(kCsrThreads) void csr_q_from_state_kernel(const float* __restrict__ state,
                                                                       float* __restrict__ qn, int L, int N) {
  const int i = blockIdx.x * kCsrThreads + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= N) return;
  const float* s = state + (size_t)b * L * N + i;
  float v[LQ];
#pragma unroll
  for (int l = 0; l < LQ; ++l) v[l] = (l < L) ? expf(s[(size_t)l * N]) : 0.f;
  float4* dst = reinterpret_cast<float4*>(qn + ((size_t)b * N + i) * LQ);
#pragma unroll
  for (int k = 0; k < LQ / 4; ++k) dst[k] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
}

template <int LQ, bool EXACT, int COMPAT>
__global__ __launch_bounds__(kCsrThreads) void csr_step_kernel(CsrStepArgs a, float one_minus_alpha) {
  const int L = EXACT ? LQ : a.L;
  const int N = a.N;
  const int i = blockIdx.x * kCsrThreads + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= N) return;
  const size_t base = (size_t)b * L * N;
  const float* __restrict__ li = a.state_in + base + i;
  const float* __restrict__ ui = a.unary + base + i;

  float ell[LQ], uu[LQ];
#pragma unroll
  for (int l = 0; l < LQ; ++l) {
    ell[l] = (l < L) ? li[(size_t)l * N] : 0.f;
    uu[l] = (l < L) ? ui[(size_t)l * N] : 0.f;
  }

  float S[LQ];
#pragma unroll
  for (int l = 0; l < LQ; ++l) S[l] = 0.f;
  const float4* __restrict__ qb = reinterpret_cast<const float4*>(a.q_in + (size_t)b * N * LQ);
  // Clamp the row to [0, nnz) and skip out-of-range columns: a malformed CSR
  // (reported through the flags by csr_check_kernel) never reads out of bounds.
  long long e0 = a.row_ptr[i], e1 = a.row_ptr[i + 1];
  e0 = e0 < 0 ? 0 : e0;
  e1 = e1 > a.nnz ? a.nnz : e1;
  for (long long e = e0; e < e1; ++e) {
    const int j = a.col[e];
    if (j < 0 || j >= N) continue;
    const float w = a.w ? a.w[e] : 1.f;
    const float4* qj = qb + (size_t)j * (LQ / 4);
#pragma unroll
    for (int k = 0; k < LQ / 4; ++k) {
      const float4 v = qj[k];
      S[4 * k] = fmaf(w, v.x, S[4 * k]);
      S[4 * k + 1] = fmaf(w, v.y, S[4 * k + 1]);
      S[4 * k + 2] = fmaf(w, v.z, S[4 * k + 2]);
      S[4 * k + 3] = fmaf(w, v.w, S[4 * k + 3]);
    }
  }

  float z[LQ];
  if (COMPAT == MF_COMPAT_POTTS) {
    float tot = 0.f;
#pragma unroll
    for (int l = 0; l < LQ; ++l) tot += S[l];
#pragma unroll
    for (int l = 0; l < LQ; ++l) z[l] = one_minus_alpha * ell[l] - a.alpha * (uu[l] + a.potts_w * (tot - S[l]));
  } else {
    const float* __restrict__ th = a.theta;
#pragma unroll
    for (int l = 0; l < LQ; ++l) {
      float acc = 0.f;
      if (l < L) {
#pragma unroll
        for (int k = 0; k < LQ; ++k)
          if (k < L) acc = fmaf(th[l * L + k], S[k], acc);
      }
      z[l] = one_minus_alpha * ell[l] - a.alpha * (uu[l] + acc);
    }
  }
  float mx = -INFINITY;
#pragma unroll
  for (int l = 0; l < LQ; ++l)
    if (l < L) mx = fmaxf(mx, z[l]);
  float e[LQ];
  float se = 0.f;
#pragma unroll
  for (int l = 0; l < LQ; ++l) {
    e[l] = (l < L) ? __expf(z[l] - mx) : 0.f;
    se += e[l];
  }
  const float lse = mx + __logf(se);
  const float inv = 1.0f / se;
  float* __restrict__ out = a.state_out + base + i;
#pragma unroll
  for (int l = 0; l < LQ; ++l)
    if (l < L) out[(size_t)l * N] = z[l] - lse;
  float4* qo = reinterpret_cast<float4*>(a.q_out + ((size_t)b * N + i) * LQ);
#pragma unroll
  for (int k = 0; k < LQ / 4; ++k)
    qo[k] = make_float4(e[4 * k] * inv, e[4 * k + 1] * inv, e[4 * k + 2] * inv, e[4 * k + 3] * inv);
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double block_sum_d(double v) {
  __shared__ double red[kCsrThreads / 64];
  v = wave_sum_d(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kCsrThreads / 64; ++k) t += red[k];
  return t;
}

// Per-node free energy in FP64: sum_l q_l (u_l + log q_l) + 1/2 q . (Theta S).
template <int COMPAT>
__global__ __launch_bounds__(kCsrThreads) void csr_fe_kernel(CsrFreeEnergyArgs a) {
  const int L = a.L, N = a.N;
  const int b = blockIdx.y;
  const int i = blockIdx.x * kCsrThreads + threadIdx.x;
  double f = 0.0;
  if (i < N) {
    const size_t base = (size_t)b * L * N;
    const float* st = a.state + base;
    double S[MF_MAX_LABELS];
#pragma unroll
    for (int l = 0; l < MF_MAX_LABELS; ++l) S[l] = 0.0;
    long long e0 = a.row_ptr[i], e1 = a.row_ptr[i + 1];
    e0 = e0 < 0 ? 0 : e0;
    e1 = e1 > a.nnz ? a.nnz : e1;
    for (long long e = e0; e < e1; ++e) {
      const int j = a.col[e];
      if (j < 0 || j >= N) continue;
      const double w = a.w ? (double)a.w[e] : 1.0;
#pragma unroll
      for (int l = 0; l < MF_MAX_LABELS; ++l)
        if (l < L) S[l] += w * exp((double)st[(size_t)l * N + j]);
    }
    double tot = 0.0;
#pragma unroll
    for (int l = 0; l < MF_MAX_LABELS; ++l) tot += S[l];
#pragma unroll
    for (int l = 0; l < MF_MAX_LABELS; ++l) {
      if (l >= L) continue;
      const double lq = (double)st[(size_t)l * N + i];
      const double q = exp(lq);
      double pm;
      if (COMPAT == MF_COMPAT_POTTS) {
        pm = (double)a.potts_w * (tot - S[l]);
      } else {
        pm = 0.0;
#pragma unroll
        for (int k = 0; k < MF_MAX_LABELS; ++k)
          if (k < L) pm += (double)a.theta[l * L + k] * S[k];
      }
      f += q * ((double)a.unary[base + (size_t)l * N + i] + lq + 0.5 * pm);
    }
  }
  const double t = block_sum_d(f);
  if (threadIdx.x == 0) a.partials[(size_t)b * a.n_blocks + blockIdx.x] = t;
}

template <int LQ, bool EXACT>
hipError_t csr_step_lq(const CsrStepArgs& a, int compat, hipStream_t s) {
  dim3 grid((a.N + kCsrThreads - 1) / kCsrThreads, a.B);
  const float om = (float)(1.0 - (double)a.alpha);
  if (compat == MF_COMPAT_POTTS)
    hipLaunchKernelGGL((csr_step_kernel<LQ, EXACT, MF_COMPAT_POTTS>), grid, dim3(kCsrThreads), 0, s, a, om);
  else
    hipLaunchKernelGGL((csr_step_kernel<LQ, EXACT, MF_COMPAT_GENERAL>), grid, dim3(kCsrThreads), 0, s, a, om);
  return hipGetLastError();
}

template <int LQ>
hipError_t csr_q_lq(const float* state, float* qn, int B, int L, int N, hipStream_t s) {
  dim3 grid((N + kCsrThreads - 1) / kCsrThreads, B);
  hipLaunchKernelGGL((csr_q_from_state_kernel<LQ>), grid, dim3(kCsrThreads), 0, s, state, qn, L, N);
  return hipGetLastError();
}

}  // namespace

int csr_label_stride(int L) { return (L + 3) & ~3; }

hipError_t launch_csr_check(const int* row_ptr, const int* col, int N, long long nnz, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(csr_check_kernel, dim3((N + 1 + kCsrThreads - 1) / kCsrThreads), dim3(kCsrThreads), 0, s,
                     row_ptr, col, N, nnz, flags);
  return hipGetLastError();
}

hipError_t launch_csr_q_from_state(const float* state, float* qn, int B, int L, int N, hipStream_t s) {
  switch (csr_label_stride(L)) {
    case 4: return csr_q_lq<4>(state, qn, B, L, N, s);
    case 8: return csr_q_lq<8>(state, qn, B, L, N, s);
    case 12: return csr_q_lq<12>(state, qn, B, L, N, s);
    case 16: return csr_q_lq<16>(state, qn, B, L, N, s);
    case 20: return csr_q_lq<20>(state, qn, B, L, N, s);
    case 24: return csr_q_lq<24>(state, qn, B, L, N, s);
    case 28: return csr_q_lq<28>(state, qn, B, L, N, s);
    default: return csr_q_lq<32>(state, qn, B, L, N, s);
  }
}

hipError_t launch_csr_step(const CsrStepArgs& a, int compat, hipStream_t s) {
  switch (csr_label_stride(a.L)) {
    case 4: return a.L == 4 ? csr_step_lq<4, true>(a, compat, s) : csr_step_lq<4, false>(a, compat, s);
    case 8: return a.L == 8 ? csr_step_lq<8, true>(a, compat, s) : csr_step_lq<8, false>(a, compat, s);
    case 12: return csr_step_lq<12, false>(a, compat, s);
    case 16: return csr_step_lq<16, false>(a, compat, s);
    case 20: return csr_step_lq<20, false>(a, compat, s);
    case 24: return csr_step_lq<24, false>(a, compat, s);
    case 28: return csr_step_lq<28, false>(a, compat, s);
    default: return csr_step_lq<32, false>(a, compat, s);
  }
}

hipError_t launch_csr_free_energy(const CsrFreeEnergyArgs& a, int compat, hipStream_t s) {
  dim3 grid(a.n_blocks, a.B);
  if (compat == MF_COMPAT_POTTS)
    hipLaunchKernelGGL((csr_fe_kernel<MF_COMPAT_POTTS>), grid, dim3(kCsrThreads), 0, s, a);
  else
    hipLaunchKernelGGL((csr_fe_kernel<MF_COMPAT_GENERAL>), grid, dim3(kCsrThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace mf
