// Small grids in one workgroup: the whole problem (N <= 1024 nodes, L <= 8
// labels) lives in LDS, one thread per node, and every requested step runs
// in the same launch, a barrier between steps.  This is the parallel
// proximal step of Eq. 15 with the fixed step of Eq. 16 with the same
// per-node formulas as the tile kernels (neighbour sums with a free
// boundary, Theta S or the Potts form, the damped step and the per-node
// log-sum-exp).  The results agree with the tile kernels to FP32 rounding,
// not bitwise: the next step's q operand here is exp(z - max) / sum, taken
// from the log-sum-exp, where the single-step tile kernel re-exponentiates
// the stored log q.  A launch of the tile kernels
// costs a few microseconds however small the grid, so a 32 x 32 problem is
// bound by launches, not by the step.
//
// One workgroup per batch item.  LDS holds q of every node twice (this
// step's and the next), in the message precision; log q and the unaries
// stay in the node's registers.  A solve can run as one launch: the first
// launch may take the initialisation (init >= 0, the mf_init_mode) and the
// last may write q = exp(log q), each with the arithmetic and the order of
// the separate kernels (the label groups of the initialisation's sums, expf
// for the write-out), so the results are those of init, steps and
// write-out launched one by one.
#include <hip/hip_runtime.h>

#include "mf_internal.h"
#include "msg_codec.h"

namespace mf {
namespace {

constexpr int kWholeThreads = 1024;

template <int LP, int CONN, int COMPAT, int PREC>
__global__ __launch_bounds__(kWholeThreads) void whole_grid_kernel(StepArgs a, float one_minus_alpha, int ks,
                                                                   int init, int* __restrict__ flags,
                                                                   float* __restrict__ q_out) {
  using M = MsgT<PREC>;
  using T = typename M::T;
  __shared__ T qs[2][LP * kWholeThreads];
  __shared__ float th[COMPAT == MF_COMPAT_GENERAL ? LP * LP : 1];
  const int b = blockIdx.x;
  const int n = threadIdx.x;
  const int L = a.L, N = a.N, H = a.H, W = a.W;
  const bool on = n < N;
  const size_t base = (size_t)b * L * N;
  const int y = on ? n / W : 0, x = on ? n - (n / W) * W : 0;

  float ell[LP], uu[LP];
#pragma unroll
  for (int l = 0; l < LP; ++l) {
    const bool v = on && l < L;
    const size_t at = base + (size_t)(l < L ? l : L - 1) * N + (on ? n : 0);   // clamped
    const float e_ = a.state_in[at], u_ = a.unary[at];
    ell[l] = v ? e_ : 0.f;
    uu[l] = v ? u_ : 0.f;
  }
  if (init >= 0) {
    // log q^0 as the initialisation kernel forms it: its label groups are
    // one thread of LG labels (L <= 4) or two of four (L <= 8), each with its
    // own max and sum, the two combined afterwards
    constexpr int GL = LP <= 4 ? LP : 4, NG = LP / GL;
    bool bad = false;
    if (on) {
#pragma unroll
      for (int l = 0; l < LP; ++l) {
        if (l < L) bad |= !isfinite(uu[l]);
        if (init == MF_INIT_STATE && l < L) bad |= !isfinite(ell[l]);
      }
      if (init == MF_INIT_UNARY) {
        float v[LP], gm[NG], gs[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          gm[g] = -INFINITY;
#pragma unroll
          for (int j = 0; j < GL; ++j) {
            const int l = g * GL + j;
            v[l] = l < L ? -uu[l] : -INFINITY;
            gm[g] = fmaxf(gm[g], v[l]);
          }
        }
        const float mx = NG == 1 ? gm[0] : fmaxf(gm[0], gm[NG - 1]);
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          gs[g] = 0.f;
#pragma unroll
          for (int j = 0; j < GL; ++j) gs[g] += g * GL + j < L ? expf(v[g * GL + j] - mx) : 0.f;
        }
        const float se = NG == 1 ? gs[0] : gs[0] + gs[NG - 1];
        const float lse = mx + logf(se);
#pragma unroll
        for (int l = 0; l < LP; ++l) ell[l] = l < L ? v[l] - lse : 0.f;
      } else if (init == MF_INIT_UNIFORM) {
        const float u0 = -logf((float)L);
#pragma unroll
        for (int l = 0; l < LP; ++l) ell[l] = l < L ? u0 : 0.f;
      }
    }
    if (bad) atomicOr(flags, 1);
  }
  if (COMPAT == MF_COMPAT_GENERAL)
    for (int f = n; f < LP * LP; f += kWholeThreads) {
      const int l = f / LP, k = f - (f / LP) * LP;
      th[f] = (l < L && k < L) ? a.theta[l * L + k] : 0.f;
    }
#pragma unroll
  for (int l = 0; l < LP; ++l) qs[0][l * kWholeThreads + n] = M::enc(on && l < L ? __expf(ell[l]) : 0.f);

  // neighbours on the grid (free boundary); off-grid ones read slot n, weight 0
  constexpr int NB = CONN == 8 ? 8 : 4;
  int nb[NB];
  bool ok[NB];
  {
    const bool up = y > 0, dn = y < H - 1, lf = x > 0, rt = x < W - 1;
    nb[0] = n - W; ok[0] = up;
    nb[1] = n - 1; ok[1] = lf;
    nb[2] = n + 1; ok[2] = rt;
    nb[3] = n + W; ok[3] = dn;
    if constexpr (CONN == 8) {
      nb[4] = n - W - 1; ok[4] = up && lf;
      nb[5] = n - W + 1; ok[5] = up && rt;
      nb[6] = n + W - 1; ok[6] = dn && lf;
      nb[7] = n + W + 1; ok[7] = dn && rt;
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      ok[k] = ok[k] && on;
      nb[k] = ok[k] ? nb[k] : n;
    }
  }
  __syncthreads();

  int cur = 0;
  for (int s = 0; s < ks; ++s) {
    if (on) {
      const T* q = qs[cur];
      float S[LP];
#pragma unroll
      for (int l = 0; l < LP; ++l) {
        const T* ql = q + l * kWholeThreads;
        float v[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) v[k] = ok[k] ? M::dec(ql[nb[k]]) : 0.f;
        float t = (v[0] + v[1]) + (v[2] + v[3]);
        if constexpr (CONN == 8) t += (v[4] + v[5]) + (v[6] + v[7]);
        S[l] = t;
      }
      float z[LP];
      float mx = -INFINITY;
      if (COMPAT == MF_COMPAT_POTTS) {
        float tot = 0.f;
#pragma unroll
        for (int l = 0; l < LP; ++l) tot += S[l];
#pragma unroll
        for (int l = 0; l < LP; ++l) {
          const float m = uu[l] + a.potts_w * (tot - S[l]);
          z[l] = l < L ? one_minus_alpha * ell[l] - a.alpha * m : -INFINITY;
          mx = fmaxf(mx, z[l]);
        }
      } else {
#pragma unroll
        for (int l = 0; l < LP; ++l) {
          float acc = 0.f;
#pragma unroll
          for (int k = 0; k < LP; ++k) acc = fmaf(th[l * LP + k], S[k], acc);
          z[l] = l < L ? one_minus_alpha * ell[l] - a.alpha * (uu[l] + acc) : -INFINITY;
          mx = fmaxf(mx, z[l]);
        }
      }
      float e[LP];
      float se = 0.f;
#pragma unroll
      for (int l = 0; l < LP; ++l) {
        e[l] = __expf(z[l] - mx);   // exp(-inf) = 0 for padding slots
        se += e[l];
      }
      const float lse = mx + __logf(se);
      const float inv = 1.0f / se;
      T* qn = qs[cur ^ 1];
#pragma unroll
      for (int l = 0; l < LP; ++l) {
        ell[l] = l < L ? z[l] - lse : 0.f;
        qn[l * kWholeThreads + n] = M::enc(e[l] * inv);
      }
    }
    __syncthreads();
    cur ^= 1;
  }
  if (on) {
#pragma unroll
    for (int l = 0; l < LP; ++l) {
      if (l < L) {
        a.state_out[base + (size_t)l * N + n] = ell[l];
        if (q_out) q_out[base + (size_t)l * N + n] = expf(ell[l]);
      }
    }
  }
}

struct WholeExtra {
  int init;        // mf_init_mode, or -1: the state is already initialised
  int* flags;
  float* q_out;    // nullptr: no write-out
};

template <int LP, int PREC>
hipError_t whole_lp(const StepArgs& a, int conn, int compat, int ks, const WholeExtra& x, hipStream_t s) {
  const float om = (float)(1.0 - (double)a.alpha);
  const dim3 grid(a.B), block(kWholeThreads);
  if (conn == 4) {
    if (compat == MF_COMPAT_POTTS)
      hipLaunchKernelGGL((whole_grid_kernel<LP, 4, MF_COMPAT_POTTS, PREC>), grid, block, 0, s, a, om, ks, x.init,
                         x.flags, x.q_out);
    else
      hipLaunchKernelGGL((whole_grid_kernel<LP, 4, MF_COMPAT_GENERAL, PREC>), grid, block, 0, s, a, om, ks, x.init,
                         x.flags, x.q_out);
  } else {
    if (compat == MF_COMPAT_POTTS)
      hipLaunchKernelGGL((whole_grid_kernel<LP, 8, MF_COMPAT_POTTS, PREC>), grid, block, 0, s, a, om, ks, x.init,
                         x.flags, x.q_out);
    else
      hipLaunchKernelGGL((whole_grid_kernel<LP, 8, MF_COMPAT_GENERAL, PREC>), grid, block, 0, s, a, om, ks, x.init,
                         x.flags, x.q_out);
  }
  return hipGetLastError();
}

template <int PREC>
hipError_t whole_prec(const StepArgs& a, int conn, int compat, int ks, const WholeExtra& x, hipStream_t s) {
  if (a.L <= 2) return whole_lp<2, PREC>(a, conn, compat, ks, x, s);
  if (a.L <= 4) return whole_lp<4, PREC>(a, conn, compat, ks, x, s);
  return whole_lp<8, PREC>(a, conn, compat, ks, x, s);
}

}  // namespace

bool grid_whole_fits(int L, int N) { return L >= 1 && L <= kWholeMaxLabels && N >= 1 && N <= kWholeThreads; }

hipError_t launch_grid_whole(const StepArgs& a, int conn, int compat, int precision, int ks, int init, int* flags,
                             float* q_out, hipStream_t s) {
  if (!grid_whole_fits(a.L, a.N) || ks < 1 || (init >= 0 && !flags)) return hipErrorInvalidValue;
  const WholeExtra x{init, flags, q_out};
  switch (precision) {
    case MF_P_F32: return whole_prec<P_F32>(a, conn, compat, ks, x, s);
    case MF_P_BF16MSG: return whole_prec<P_BF16>(a, conn, compat, ks, x, s);
    default: return whole_prec<P_F16>(a, conn, compat, ks, x, s);
  }
}

}  // namespace mf
