// One proximal step on a grid with many labels (32 < L <= 128): the
// compatibility product Theta S on the matrix cores.
//
// Step (Eq. 15 with the fixed step of Eq. 16, Sec. 3.1-3.2), per node i:
//   S_i = sum of q_j over the 4 / 8 grid neighbours (free boundary)
//   m_i = u_i + Theta S_i
//   z_i = (1 - alpha) log q_i - alpha m_i;   log q_i <- z_i - lse(z_i)
//
// At these label counts m = u + Theta S costs 2 L flops per node-label
// against 12 bytes of state and unaries, a real dense contraction
// [L x L] x [L x nodes]: it runs on MFMA, the rest of the step on the VALU.
//
// A workgroup (four wavefronts) owns a tile of 64 consecutive nodes of one
// grid row.  The labels are taken in chunks of 32: for each chunk the
// workgroup stages q = exp(log q) of the tile's three rows (the row and
// its neighbours above and below, 66 nodes each, off-grid q = 0) in LDS,
// forms the chunk of S for its 64 nodes in LDS, and every wavefront
// multiplies that S chunk by the matching columns of Theta into its
// accumulators.  Wavefront w owns the output label blocks w, w + 4 (16
// labels each) for all 64 nodes; its rows of Theta stay in registers for
// the whole launch.  The per-node log-sum-exp runs over the accumulators
// of the four wavefronts: a max and a sum inside each (lanes x, x ^ 16,
// x ^ 32, x ^ 48 with the gfx950 row-swap permutes), combined across
// wavefronts through LDS.
//
// Products.  FP32 messages: v_mfma_f32_16x16x4f32 on FP32 Theta and S, so
// the step keeps FP32 accuracy.  BF16 / FP16 messages: q is rounded to the
// 16-bit type where it is staged in LDS (as in the other grid kernels) and
// S accumulates in FP32; S and Theta are then each split into two BF16
// parts (hi = bf16(x), lo = bf16(x - hi)) and Theta S is formed as
// hi.hi + hi.lo + lo.hi with v_mfma_f32_16x16x32_bf16 and FP32
// accumulation.  The dropped lo.lo term and the roundings of the parts
// leave a relative error of about 2^-16, well below the 2^-9 (BF16) and
// 2^-11 (FP16) rounding of q itself, so the 16-bit modes round only q, as
// they do on the other graphs.
#include <hip/hip_runtime.h>

#include "grid_temporal.h"
#include "mf_internal.h"
#include "msg_codec.h"

namespace mf {
namespace large {

constexpr int kTN = 64;             // nodes per tile (one row segment)
constexpr int kNT = 256;            // threads per workgroup
constexpr int kKC = 32;             // labels per chunk
constexpr int kRW = kTN + 2;        // region row: the tile and one node either side
constexpr int kRP = 3 * kRW;        // region nodes per label plane (three rows)
constexpr int kRegion = kKC * kRP;  // staged q values per chunk
constexpr int kLoads = (kRegion + kNT - 1) / kNT;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// Row stride (floats) of the S chunk [32 labels][64 nodes] in LDS.  The
// FP32 product reads rows 4 kb + g (g = lane / 16) at 16 consecutive
// nodes: a stride of 16 mod 64 words puts the four row groups on disjoint
// banks.  The BF16 product reads rows 8 g + e: a stride of 66 puts 8 g on
// 16 g mod 64 words.
template <int PREC>
constexpr int s_stride() { return PREC == P_F32 ? 80 : 66; }

__device__ inline unsigned short bf16_bits(float x) { return MsgT<P_BF16>::enc(x); }
__device__ inline float bf16_val(unsigned short b) { return MsgT<P_BF16>::dec(b); }

// hi = bf16(x), lo = bf16(x - hi): x = hi + lo to about 2^-16 relative.
__device__ inline void split8(const float (&x)[8], bf16x8& hi, bf16x8& lo) {
  u16x8 h, l;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const unsigned short hb = bf16_bits(x[e]);
    h[e] = hb;
    l[e] = bf16_bits(x[e] - bf16_val(hb));
  }
  hi = __builtin_bit_cast(bf16x8, h);
  lo = __builtin_bit_cast(bf16x8, l);
}

template <int LP, int CONN, int PREC, bool STREAM>
__global__ __launch_bounds__(kNT) void large_step_kernel(StepArgs a, float one_minus_alpha, int potts) {
  using M = MsgT<PREC>;
  using T = typename M::T;
  constexpr bool F32 = PREC == P_F32;
  constexpr int NOB = LP / 64;       // output blocks of 16 labels per wavefront
  constexpr int NC = LP / kKC;       // label chunks
  constexpr int NNB = kTN / 16;      // node blocks of 16 per tile
  constexpr int SST = s_stride<PREC>();
  __shared__ T qs[kRegion];
  __shared__ float ss[kKC * SST];
  __shared__ float red_m[4][kTN], red_s[4][kTN];

  const int L = a.L;
  const unsigned N = (unsigned)a.N;
  const int H = a.H, W = a.W;
  const int tiles_x = (W + kTN - 1) / kTN;
  const int tile = lanes::xcd_tile(blockIdx.x, tiles_x * H * a.B);
  const int b = tile / (tiles_x * H);
  const int tr = tile - b * (tiles_x * H);
  const int y = tr / tiles_x;
  const int x0 = (tr - y * tiles_x) * kTN;
  const size_t base = (size_t)b * L * N;
  const float* __restrict__ lin = a.state_in + base;
  const float* __restrict__ ug = a.unary + base;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = lane & 15, g = lane >> 4;

  // Theta rows of this wavefront's output blocks (label 16 (wave + 4 ob) + c),
  // zero outside L x L; Potts builds w (1 1^T - I).
  auto theta_at = [&](int row, int col) -> float {
    if (row >= L || col >= L) return 0.f;
    if (potts) return row == col ? 0.f : a.potts_w;
    return a.theta[row * L + col];
  };
  float tha[F32 ? NOB : 1][F32 ? LP / 4 : 1];
  bf16x8 thh[F32 ? 1 : NOB][F32 ? 1 : NC], thl[F32 ? 1 : NOB][F32 ? 1 : NC];
#pragma unroll
  for (int ob = 0; ob < NOB; ++ob) {
    const int row = 16 * (wave + 4 * ob) + c;
    if constexpr (F32) {
      // A of k-step kb: Theta[row][4 kb + g]
#pragma unroll
      for (int kb = 0; kb < LP / 4; ++kb) tha[ob][kb] = theta_at(row, 4 * kb + g);
    } else {
      // A of chunk kc: Theta[row][32 kc + 8 g + e], e < 8
#pragma unroll
      for (int kc = 0; kc < NC; ++kc) {
        float t[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = theta_at(row, kKC * kc + 8 * g + e);
        split8(t, thh[ob][kc], thl[ob][kc]);
      }
    }
  }

  f32x4 acc[NOB][NNB];
#pragma unroll
  for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
    for (int nb = 0; nb < NNB; ++nb) acc[ob][nb] = f32x4{0.f, 0.f, 0.f, 0.f};

#pragma unroll
  for (int kc = 0; kc < NC; ++kc) {
    // q of the chunk's 32 labels on the three rows y - 1, y, y + 1, nodes
    // x0 - 1 .. x0 + 64; off-grid nodes and labels >= L hold q = 0
    float v[kLoads];
#pragma unroll
    for (int r = 0; r < kLoads; ++r) {
      const int f = tid + r * kNT;
      const int kk = f / kRP;
      const int rem = f - kk * kRP;
      const int row = rem / kRW;
      const int col = rem - row * kRW;
      const int l = kKC * kc + kk;
      const int gy = y + row - 1, gx = x0 + col - 1;
      const bool ok = f < kRegion && l < L && gy >= 0 && gy < H && gx >= 0 && gx < W;
      const float x = lin[ok ? (unsigned)l * N + (unsigned)(gy * W + gx) : 0u];
      v[r] = ok ? x : -INFINITY;
    }
#pragma unroll
    for (int r = 0; r < kLoads; ++r) {
      const int f = tid + r * kNT;
      if (f < kRegion) qs[f] = M::enc(__expf(v[r]));   // exp(-inf) = 0
    }
    __syncthreads();   // q staged; every wavefront is past the previous chunk's products

    // S chunk: wavefront w forms labels w + 4 j of the chunk, lane = node
#pragma unroll
    for (int j = 0; j < kKC / 4; ++j) {
      const int kk = wave + 4 * j;
      const T* q = qs + kk * kRP + lane + 1;           // row y - 1 at node lane
      float s = M::dec(q[0]) + M::dec(q[2 * kRW]) + M::dec(q[kRW - 1]) + M::dec(q[kRW + 1]);
      if (CONN == 8) s += (M::dec(q[-1]) + M::dec(q[1])) + (M::dec(q[2 * kRW - 1]) + M::dec(q[2 * kRW + 1]));
      ss[kk * SST + lane] = s;
    }
    __syncthreads();   // S chunk complete

    if constexpr (F32) {
#pragma unroll
      for (int nb = 0; nb < NNB; ++nb) {
#pragma unroll
        for (int kb = 0; kb < kKC / 4; ++kb) {
          const float bv = ss[(4 * kb + g) * SST + 16 * nb + c];
#pragma unroll
          for (int ob = 0; ob < NOB; ++ob)
            acc[ob][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(tha[ob][(kKC / 4) * kc + kb], bv, acc[ob][nb], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int nb = 0; nb < NNB; ++nb) {
        float sv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) sv[e] = ss[(8 * g + e) * SST + 16 * nb + c];
        bf16x8 sh, sl;
        split8(sv, sh, sl);
#pragma unroll
        for (int ob = 0; ob < NOB; ++ob) {
          acc[ob][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(thh[ob][kc], sh, acc[ob][nb], 0, 0, 0);
          acc[ob][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(thh[ob][kc], sl, acc[ob][nb], 0, 0, 0);
          acc[ob][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(thl[ob][kc], sh, acc[ob][nb], 0, 0, 0);
        }
      }
    }
  }

  // Epilogue.  Accumulator i of (ob, nb) is label 16 (wave + 4 ob) + 4 g + i
  // at node x0 + 16 nb + c.
  const unsigned row_n = (unsigned)(y * W);
  float z[NOB][NNB][4];
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb) {
    const int x = x0 + 16 * nb + c;
    const unsigned n = row_n + (unsigned)(x < W ? x : W - 1);
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int l = 16 * (wave + 4 * ob) + 4 * g + i;
        const unsigned o = (unsigned)(l < L ? l : L - 1) * N + n;
        const float e = lin[o];
        const float u = STREAM ? __builtin_nontemporal_load(&ug[o]) : ug[o];
        const float zz = one_minus_alpha * e - a.alpha * (u + acc[ob][nb][i]);
        z[ob][nb][i] = l < L ? zz : -INFINITY;
      }
    }
  }
  float mx[NNB], se[NNB];
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb) {
    float m = z[0][nb][0];
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
      for (int i = 0; i < 4; ++i) m = fmaxf(m, z[ob][nb][i]);
    m = temporal::rows_max(m);
    // a wavefront whose labels all lie past L has m = -inf and contributes 0
    const float mref = m == -INFINITY ? 0.f : m;
    float s = 0.f;
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
      for (int i = 0; i < 4; ++i) s += __expf(z[ob][nb][i] - mref);
    s = temporal::rows_sum(s);
    mx[nb] = m;
    se[nb] = s;
    if (g == 0) {
      red_m[wave][16 * nb + c] = m;
      red_s[wave][16 * nb + c] = s;
    }
  }
  __syncthreads();
  float* __restrict__ out = a.state_out + base;
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb) {
    const int p = 16 * nb + c;
    float M = red_m[0][p];
#pragma unroll
    for (int w = 1; w < 4; ++w) M = fmaxf(M, red_m[w][p]);
    float tot = 0.f;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const float mw = red_m[w][p];
      tot += mw == -INFINITY ? 0.f : red_s[w][p] * __expf(mw - M);
    }
    const float lse = M + __logf(tot);
    const int x = x0 + p;
    if (x < W) {
      const unsigned n = row_n + (unsigned)x;
#pragma unroll
      for (int ob = 0; ob < NOB; ++ob) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int l = 16 * (wave + 4 * ob) + 4 * g + i;
          if (l < L) {
            if constexpr (STREAM) __builtin_nontemporal_store(z[ob][nb][i] - lse, &out[(unsigned)l * N + n]);
            else out[(unsigned)l * N + n] = z[ob][nb][i] - lse;
          }
        }
      }
    }
  }
  (void)mx;
  (void)se;
}

template <int LP, int PREC, bool STREAM>
hipError_t go(const StepArgs& a, int conn, int compat, hipStream_t s) {
  const dim3 grid((unsigned)(((a.W + kTN - 1) / kTN) * a.H * a.B)), block(kNT);
  const float om = (float)(1.0 - (double)a.alpha);
  const int potts = compat == MF_COMPAT_POTTS;
  if (conn == 4) hipLaunchKernelGGL((large_step_kernel<LP, 4, PREC, STREAM>), grid, block, 0, s, a, om, potts);
  else hipLaunchKernelGGL((large_step_kernel<LP, 8, PREC, STREAM>), grid, block, 0, s, a, om, potts);
  return hipGetLastError();
}

template <int PREC>
hipError_t by_size(const StepArgs& a, int conn, int compat, hipStream_t s) {
  const bool stream = lanes::streams_past_cache(a);
  if (a.L <= 64) return stream ? go<64, PREC, true>(a, conn, compat, s) : go<64, PREC, false>(a, conn, compat, s);
  return stream ? go<128, PREC, true>(a, conn, compat, s) : go<128, PREC, false>(a, conn, compat, s);
}

}  // namespace large

hipError_t launch_grid_step_large(const StepArgs& a, int conn, int compat, int prec, hipStream_t s) {
  switch (prec) {
    case MF_P_F32: return large::by_size<P_F32>(a, conn, compat, s);
    case MF_P_BF16MSG: return large::by_size<P_BF16>(a, conn, compat, s);
    default: return large::by_size<P_F16>(a, conn, compat, s);
  }
}

}  // namespace mf
