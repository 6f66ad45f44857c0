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
#include "msg_codec.h"

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

typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));
typedef unsigned int v2u32 __attribute__((ext_vector_type(2)));

// A raw buffer resource over bytes [0, bytes) of p (dword 3: the 32-bit
// data format of CDNA raw buffers).
__device__ inline __amdgpu_buffer_rsrc_t csr_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ inline float rd32(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0u, 0));
}

// Four consecutive labels of a node-major q row: one 16-byte load in FP32,
// one 8-byte load of 16-bit values in the BF16 / FP16 message modes (the
// operand rounding of the neighbour aggregation, as on grids).
template <int PREC>
struct Q4 {
  using M = MsgT<PREC>;
  using C = typename std::conditional<PREC == P_F32, float4, uint2>::type;
  __device__ static unsigned short bits(typename M::T h) {
    if constexpr (PREC == P_F16) return __builtin_bit_cast(unsigned short, h);
    else return (unsigned short)h;
  }
  __device__ static float dec16(unsigned int b) {
    if constexpr (PREC == P_F16) return M::dec(__builtin_bit_cast(_Float16, (unsigned short)b));
    else return M::dec((unsigned short)b);
  }
  __device__ static void dec(const C& c, float (&v)[4]) {
    if constexpr (PREC == P_F32) {
      v[0] = c.x; v[1] = c.y; v[2] = c.z; v[3] = c.w;
    } else {
      v[0] = dec16(c.x & 0xFFFFu); v[1] = dec16(c.x >> 16);
      v[2] = dec16(c.y & 0xFFFFu); v[3] = dec16(c.y >> 16);
    }
  }
  // four labels of a row through a buffer resource
  __device__ static C load(__amdgpu_buffer_rsrc_t r, unsigned off) {
    if constexpr (PREC == P_F32) {
      return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0u, 0));
    } else {
      return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0u, 0));
    }
  }
  __device__ static void store(const C& c, __amdgpu_buffer_rsrc_t r, unsigned off) {
    if constexpr (PREC == P_F32) {
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4u32, c), r, off, 0u, 0);
    } else {
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u32, c), r, off, 0u, 0);
    }
  }
  __device__ static C enc(float a, float b, float c, float d) {
    if constexpr (PREC == P_F32) {
      return make_float4(a, b, c, d);
    } else {
      C r;
      r.x = (unsigned int)bits(M::enc(a)) | ((unsigned int)bits(M::enc(b)) << 16);
      r.y = (unsigned int)bits(M::enc(c)) | ((unsigned int)bits(M::enc(d)) << 16);
      return r;
    }
  }
};

// Node-major q from the label-major log q (after initialisation).
template <int LQ, int PREC>
__global__ __launch_bounds__(kCsrThreads) void csr_q_from_state_kernel(const float* __restrict__ state,
                                                                       void* __restrict__ qn, int L, int N) {
  using Q = Q4<PREC>;
  const int i = blockIdx.x * kCsrThreads + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= N) return;
  const float* s = state + (size_t)b * L * N + i;
  float v[LQ];
#pragma unroll
  for (int l = 0; l < LQ; ++l) v[l] = (l < L) ? expf(s[(size_t)l * N]) : 0.f;
  typename Q::C* dst = reinterpret_cast<typename Q::C*>(qn) + ((size_t)b * N + i) * (LQ / 4);
#pragma unroll
  for (int k = 0; k < LQ / 4; ++k) dst[k] = Q::enc(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
}

// Partner lane of a node (P = 2): lanes 2n and 2n + 1 swap a value (DPP
// quad permutation 1, 0, 3, 2).
__device__ inline float partner(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}

// P lanes per node (P = 1 or 2): lane h of a node holds labels
// [h LH, h LH + LH), LH = LQ / P, and gathers that part of each neighbour's
// q row; the halves of S, the max and the sum are exchanged with the partner
// lane in a fixed order, so both lanes hold bitwise the same values.  Two
// lanes per node double the wavefronts in flight, which hides the latency of
// the dependent row_ptr -> col -> q loads.  LC > 0: L == LC at compile
// time.  Theta is staged in LDS zero-padded to LQ x LQ, so the message needs
// no per-label test for any L; padded labels carry z = -inf (q = 0).
template <int LQ, int LC, int COMPAT, int P, int PREC>
__global__ __launch_bounds__(kCsrThreads) void csr_step_kernel(CsrStepArgs a, float one_minus_alpha) {
  using Q = Q4<PREC>;
  using C = typename Q::C;
  constexpr int LH = LQ / P;
  static_assert(LH % 4 == 0, "each lane gathers whole four-label slices");
  __shared__ float Th[COMPAT == MF_COMPAT_GENERAL ? LQ * LQ : 1];
  const int L = LC > 0 ? LC : a.L;
  const int N = a.N;
  const int t = blockIdx.x * kCsrThreads + threadIdx.x;
  const int i = t / P, h = P == 1 ? 0 : (t & 1);
  const int b = blockIdx.y;
  if (COMPAT == MF_COMPAT_GENERAL) {
    for (int f = threadIdx.x; f < LQ * LQ; f += kCsrThreads) {
      const int l = f / LQ, k = f - (f / LQ) * LQ;
      Th[f] = (l < L && k < L) ? a.theta[l * L + k] : 0.f;
    }
    __syncthreads();
  }
  if (i >= N) return;   // both lanes of a node leave together
  // Buffer resources over this problem's arrays: every access below is a
  // 32-bit byte offset (L N < 2^30, N LQ 4 < 2^32 and nnz < 2^31 are
  // checked at creation), no 64-bit address arithmetic per lane.
  const size_t base = (size_t)b * L * N;
  const unsigned pbytes = (unsigned)L * (unsigned)N * 4u;
  const __amdgpu_buffer_rsrc_t rl = csr_rsrc(a.state_in + base, pbytes);
  const __amdgpu_buffer_rsrc_t ru = csr_rsrc(a.unary + base, pbytes);
  const int l0 = h * LH;

  // log q and u of the node's labels: loaded before the gather in FP32 (their
  // latency hides under it), after it with 16-bit rows, where the registers
  // freed during the gather keep more wavefronts resident (60 against 87).
  float ell[LH], uu[LH];
  auto load_state = [&]() {
#pragma unroll
    for (int u = 0; u < LH; ++u) {
      const int l = l0 + u;
      const unsigned at = ((unsigned)(l < L ? l : L - 1) * (unsigned)N + (unsigned)i) * 4u;   // clamped: no branch
      const float x = rd32(rl, at), y = rd32(ru, at);
      ell[u] = l < L ? x : 0.f;
      uu[u] = l < L ? y : 0.f;
    }
  };
  if constexpr (PREC == P_F32) load_state();

  float S[LH];
#pragma unroll
  for (int u = 0; u < LH; ++u) S[u] = 0.f;
  constexpr unsigned kRow = (LQ / 4) * sizeof(C);         // bytes of one node-major q row
  const __amdgpu_buffer_rsrc_t rq =
      csr_rsrc(reinterpret_cast<const C*>(a.q_in) + (size_t)b * N * (LQ / 4), (unsigned)N * kRow);
  const unsigned hoff = (unsigned)(h * (LH / 4)) * (unsigned)sizeof(C);
  const int nnz = (int)a.nnz;
  const __amdgpu_buffer_rsrc_t rc = csr_rsrc(a.col, (unsigned)nnz * 4u);
  const __amdgpu_buffer_rsrc_t rw = csr_rsrc(a.w, a.w ? (unsigned)nnz * 4u : 0u);
  // Clamp the row to [0, nnz) and skip out-of-range columns: a malformed CSR
  // (reported through the flags by csr_check_kernel) never reads out of bounds.
  int e0 = a.row_ptr[i], e1 = a.row_ptr[i + 1];
  e0 = e0 < 0 ? 0 : e0;
  e1 = e1 > nnz ? nnz : e1;
  // EB edges per trip: their column indices, then their q rows, are loaded
  // together, and the next trip's column indices and weights are in flight
  // with this trip's q rows (one round trip per trip after the first).
  // Edges past the row end (and out-of-range columns) get weight 0 and a
  // valid address; the products are added in edge order.
  constexpr int EB = 4;
  int jn[EB];
  float wn[EB];
  auto load_cols = [&](int e) {
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const bool on = e + u < e1;
      const unsigned ec = (unsigned)(on ? e + u : e0) * 4u;   // called only when e0 < e1
      jn[u] = (int)__builtin_amdgcn_raw_buffer_load_b32(rc, ec, 0u, 0);
      wn[u] = on ? (a.w ? rd32(rw, ec) : 1.f) : 0.f;
    }
  };
  if (e0 < e1) load_cols(e0);
  for (int e = e0; e < e1; e += EB) {
    int j[EB];
    float w[EB];
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const bool ok = e + u < e1 && jn[u] >= 0 && jn[u] < N;
      j[u] = ok ? jn[u] : 0;
      w[u] = ok ? wn[u] : 0.f;
    }
    if (e + EB < e1) load_cols(e + EB);
    C v[EB][LH / 4];
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const unsigned qo = (unsigned)j[u] * kRow + hoff;
#pragma unroll
      for (int k = 0; k < LH / 4; ++k) v[u][k] = Q::load(rq, qo + (unsigned)(k * sizeof(C)));
    }
#pragma unroll
    for (int u = 0; u < EB; ++u) {
#pragma unroll
      for (int k = 0; k < LH / 4; ++k) {
        float f[4];
        Q::dec(v[u][k], f);
#pragma unroll
        for (int c = 0; c < 4; ++c) S[4 * k + c] = fmaf(w[u], f[c], S[4 * k + c]);
      }
    }
  }

  if constexpr (PREC != P_F32) load_state();

  // S of all LQ labels in label order: own half and the partner's
  float Sa[LQ];
#pragma unroll
  for (int u = 0; u < LH; ++u) {
    if constexpr (P == 1) {
      Sa[u] = S[u];
    } else {
      const float o = partner(S[u]);
      Sa[u] = h == 0 ? S[u] : o;
      Sa[LH + u] = h == 0 ? o : S[u];
    }
  }
  float z[LH];
  if (COMPAT == MF_COMPAT_POTTS) {
    float tot = 0.f;
#pragma unroll
    for (int k = 0; k < LQ; ++k) tot += Sa[k];
#pragma unroll
    for (int u = 0; u < LH; ++u) z[u] = one_minus_alpha * ell[u] - a.alpha * (uu[u] + a.potts_w * (tot - S[u]));
  } else {
#pragma unroll
    for (int u = 0; u < LH; ++u) {
      float acc = 0.f;
      // with L compiled in, the columns past L (zero in Th) are left out
#pragma unroll
      for (int k = 0; k < (LC > 0 ? LC : LQ); ++k) acc = fmaf(Th[(l0 + u) * LQ + k], Sa[k], acc);
      z[u] = one_minus_alpha * ell[u] - a.alpha * (uu[u] + acc);
    }
  }
#pragma unroll
  for (int u = 0; u < LH; ++u) z[u] = l0 + u < L ? z[u] : -INFINITY;
  float mx = z[0];
#pragma unroll
  for (int u = 1; u < LH; ++u) mx = fmaxf(mx, z[u]);
  if constexpr (P == 2) mx = fmaxf(mx, partner(mx));
  float e[LH];
  float se = 0.f;
#pragma unroll
  for (int u = 0; u < LH; ++u) {
    e[u] = __expf(z[u] - mx);
    se += e[u];
  }
  if constexpr (P == 2) {
    const float o = partner(se);
    se = h == 0 ? se + o : o + se;   // the lower half first in both lanes
  }
  const float lse = mx + __logf(se);
  const float inv = 1.0f / se;
  const __amdgpu_buffer_rsrc_t ro = csr_rsrc(a.state_out + base, pbytes);
#pragma unroll
  for (int u = 0; u < LH; ++u)
    if (l0 + u < L)
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(z[u] - lse), ro,
                                            ((unsigned)(l0 + u) * (unsigned)N + (unsigned)i) * 4u, 0u, 0);
  const __amdgpu_buffer_rsrc_t rqo =
      csr_rsrc(reinterpret_cast<const C*>(a.q_out) + (size_t)b * N * (LQ / 4), (unsigned)N * kRow);
#pragma unroll
  for (int k = 0; k < LH / 4; ++k)
    Q::store(Q::enc(e[4 * k] * inv, e[4 * k + 1] * inv, e[4 * k + 2] * inv, e[4 * k + 3] * inv), rqo,
             (unsigned)i * kRow + hoff + (unsigned)(k * sizeof(C)));
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
    double S[kSmallLabels];
#pragma unroll
    for (int l = 0; l < kSmallLabels; ++l) S[l] = 0.0;
    long long e0 = a.row_ptr[i], e1 = a.row_ptr[i + 1];
    e0 = e0 < 0 ? 0 : e0;
    e1 = e1 > a.nnz ? a.nnz : e1;
    for (long long e = e0; e < e1; ++e) {
      const int j = a.col[e];
      if (j < 0 || j >= N) continue;
      const double w = a.w ? (double)a.w[e] : 1.0;
#pragma unroll
      for (int l = 0; l < kSmallLabels; ++l)
        if (l < L) S[l] += w * exp((double)st[(size_t)l * N + j]);
    }
    double tot = 0.0;
#pragma unroll
    for (int l = 0; l < kSmallLabels; ++l) tot += S[l];
#pragma unroll
    for (int l = 0; l < kSmallLabels; ++l) {
      if (l >= L) continue;
      const double lq = (double)st[(size_t)l * N + i];
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
      f += q * ((double)a.unary[base + (size_t)l * N + i] + lq + 0.5 * pm);
    }
  }
  const double t = block_sum_d(f);
  if (threadIdx.x == 0) a.partials[(size_t)b * a.n_blocks + blockIdx.x] = t;
}

template <int LQ, int LC, int PREC, int P>
hipError_t csr_step_lanes(const CsrStepArgs& a, int compat, hipStream_t s) {
  dim3 grid((unsigned)(((size_t)a.N * P + kCsrThreads - 1) / kCsrThreads), a.B);
  const float om = (float)(1.0 - (double)a.alpha);
  if (compat == MF_COMPAT_POTTS)
    hipLaunchKernelGGL((csr_step_kernel<LQ, LC, MF_COMPAT_POTTS, P, PREC>), grid, dim3(kCsrThreads), 0, s, a, om);
  else
    hipLaunchKernelGGL((csr_step_kernel<LQ, LC, MF_COMPAT_GENERAL, P, PREC>), grid, dim3(kCsrThreads), 0, s, a, om);
  return hipGetLastError();
}

// Two lanes per node above 12 labels unless the descriptor asks for one
// (mf_desc.csr_lanes = 1).
template <int LQ, int LC, int PREC>
hipError_t csr_step_prec(const CsrStepArgs& a, int compat, hipStream_t s) {
  if constexpr (LQ >= 16) {
    if (a.lanes != 1) return csr_step_lanes<LQ, LC, PREC, 2>(a, compat, s);
  }
  return csr_step_lanes<LQ, LC, PREC, 1>(a, compat, s);
}

template <int LQ, int LC>
hipError_t csr_step_lq(const CsrStepArgs& a, int compat, int prec, hipStream_t s) {
  switch (prec) {
    case MF_P_F32: return csr_step_prec<LQ, LC, P_F32>(a, compat, s);
    case MF_P_BF16MSG: return csr_step_prec<LQ, LC, P_BF16>(a, compat, s);
    default: return csr_step_prec<LQ, LC, P_F16>(a, compat, s);
  }
}

template <int LQ>
hipError_t csr_q_lq(const float* state, void* qn, int B, int L, int N, int prec, hipStream_t s) {
  dim3 grid((N + kCsrThreads - 1) / kCsrThreads, B);
  if (prec == MF_P_F32)
    hipLaunchKernelGGL((csr_q_from_state_kernel<LQ, P_F32>), grid, dim3(kCsrThreads), 0, s, state, qn, L, N);
  else if (prec == MF_P_BF16MSG)
    hipLaunchKernelGGL((csr_q_from_state_kernel<LQ, P_BF16>), grid, dim3(kCsrThreads), 0, s, state, qn, L, N);
  else
    hipLaunchKernelGGL((csr_q_from_state_kernel<LQ, P_F16>), grid, dim3(kCsrThreads), 0, s, state, qn, L, N);
  return hipGetLastError();
}

}  // namespace

// Node-major q row length: L rounded up to 4 (L <= 12) or to 8 (two lanes
// per node, each gathering whole float4 slices).
int csr_label_stride(int L) { return L <= 12 ? (L + 3) & ~3 : (L + 7) & ~7; }

hipError_t launch_csr_check(const int* row_ptr, const int* col, int N, long long nnz, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(csr_check_kernel, dim3((N + 1 + kCsrThreads - 1) / kCsrThreads), dim3(kCsrThreads), 0, s,
                     row_ptr, col, N, nnz, flags);
  return hipGetLastError();
}

int csr_q_bytes(int precision) { return precision == MF_P_F32 ? 4 : 2; }

hipError_t launch_csr_q_from_state(const float* state, void* qn, int B, int L, int N, int precision,
                                   hipStream_t s) {
  switch (csr_label_stride(L)) {
    case 4: return csr_q_lq<4>(state, qn, B, L, N, precision, s);
    case 8: return csr_q_lq<8>(state, qn, B, L, N, precision, s);
    case 12: return csr_q_lq<12>(state, qn, B, L, N, precision, s);
    case 16: return csr_q_lq<16>(state, qn, B, L, N, precision, s);
    case 24: return csr_q_lq<24>(state, qn, B, L, N, precision, s);
    default: return csr_q_lq<32>(state, qn, B, L, N, precision, s);
  }
}

hipError_t launch_csr_step(const CsrStepArgs& a, int compat, int precision, hipStream_t s) {
  switch (csr_label_stride(a.L)) {
    case 4: return a.L == 4 ? csr_step_lq<4, 4>(a, compat, precision, s) : csr_step_lq<4, 0>(a, compat, precision, s);
    case 8: return a.L == 8 ? csr_step_lq<8, 8>(a, compat, precision, s) : csr_step_lq<8, 0>(a, compat, precision, s);
    case 12: return csr_step_lq<12, 0>(a, compat, precision, s);
    case 16: return csr_step_lq<16, 0>(a, compat, precision, s);
    case 24:
      return a.L == 21 ? csr_step_lq<24, 21>(a, compat, precision, s) : csr_step_lq<24, 0>(a, compat, precision, s);
    default: return csr_step_lq<32, 0>(a, compat, precision, s);
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
