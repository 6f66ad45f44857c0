// Several parallel proximal steps per launch on a grid (temporal blocking).
//
// A workgroup owns a TX x TY output tile and loads the tile plus a K-node
// halo into LDS: log q and q = exp(log q) of (TX + 2K) x (TY + 2K) nodes.
// Sub-step s recomputes the region shrunk by s nodes on each side, so after
// K sub-steps the output tile holds iteration t + K exactly as K separate
// Jacobi steps would (each node still reads its neighbours at iteration
// t + s - 1).  The halo nodes are recomputed redundantly by neighbouring
// workgroups; in exchange the state crosses HBM once per K steps and the
// launch overhead is paid once per K steps, which is what bounds small
// grids whose whole state fits in the last-level cache.
//
// q for the next sub-step comes out of the log-sum-exp for free:
// q'_l = exp(z_l - max) / sum_k exp(z_k - max), so no second exponential
// is taken per node-label inside the launch.
#pragma once
#include <hip/hip_runtime.h>

#include "mf_internal.h"

namespace mf {
namespace temporal {

enum { P_F32 = 0, P_BF16 = 1, P_F16 = 2 };

template <int PREC> struct MsgT;
template <> struct MsgT<P_F32> {
  using T = float;
  __device__ static T enc(float x) { return x; }
  __device__ static float dec(T x) { return x; }
};
template <> struct MsgT<P_BF16> {
  using T = unsigned short;
  __device__ static T enc(float x) {   // round to nearest even; x finite, >= 0
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

constexpr int kTThreads = 256;

template <int LP, bool EXACT, int CONN, int COMPAT, int PREC, int TX, int TY, int K>
__global__ __launch_bounds__(kTThreads) void grid_multi_step_kernel(StepArgs a, float one_minus_alpha,
                                                                    int ks) {
  using M = MsgT<PREC>;
  using T = typename M::T;
  constexpr int RX = TX + 2 * K, RY = TY + 2 * K, RN = RX * RY;
  constexpr int LOADS = (LP * RN + kTThreads - 1) / kTThreads;
  __shared__ T qs[2][LP * RN];
  __shared__ float ls[LP * RN];

  const int L = EXACT ? LP : a.L;
  const int N = a.N, H = a.H, W = a.W;
  const int b = blockIdx.z;
  const int gx0 = blockIdx.x * TX - K, gy0 = blockIdx.y * TY - K;
  const size_t base = (size_t)b * L * N;
  const float* __restrict__ lin = a.state_in + base;
  const float* __restrict__ ug = a.unary + base;
  const int tid = threadIdx.x;

  // Load log q of the tile and its K-halo; nodes off the grid get q = 0.
#pragma unroll
  for (int r = 0; r < LOADS; ++r) {
    const int f = tid + r * kTThreads;
    if (f < L * RN) {
      const int l = f / RN;
      const int c = f - l * RN;
      const int ry = c / RX, rx = c - (c / RX) * RX;
      const int gy = gy0 + ry, gx = gx0 + rx;
      float v = -INFINITY;
      if (gy >= 0 && gy < H && gx >= 0 && gx < W) v = lin[(size_t)l * N + gy * W + gx];
      ls[f] = v;
      const T e = M::enc(__expf(v));
      qs[0][f] = e;
      qs[1][f] = e;
    }
  }
  __syncthreads();

  int cur = 0;
  for (int s = 1; s <= ks; ++s) {
    const int m0 = K - ks + s;                 // margin of the region updated in this sub-step
    const int AX = RX - 2 * m0, AY = RY - 2 * m0;
    const int A = AX * AY;
    const T* __restrict__ qc = qs[cur];
    T* __restrict__ qn = qs[cur ^ 1];
    for (int i = tid; i < A; i += kTThreads) {
      const int ry = m0 + i / AX, rx = m0 + (i - (i / AX) * AX);
      const int gy = gy0 + ry, gx = gx0 + rx;
      if (gy < 0 || gy >= H || gx < 0 || gx >= W) continue;
      const int c = ry * RX + rx;
      const int n = gy * W + gx;

      float uu[LP];
#pragma unroll
      for (int l = 0; l < LP; ++l) uu[l] = (l < L) ? ug[(size_t)l * N + n] : 0.f;

      float S[LP];
#pragma unroll
      for (int l = 0; l < LP; ++l) {
        S[l] = 0.f;
        if (l < L) {
          const T* q = qc + l * RN + c;
          float sum = M::dec(q[-RX]) + M::dec(q[-1]) + M::dec(q[1]) + M::dec(q[RX]);
          if (CONN == 8) sum += (M::dec(q[-RX - 1]) + M::dec(q[-RX + 1])) + (M::dec(q[RX - 1]) + M::dec(q[RX + 1]));
          S[l] = sum;
        }
      }

      float z[LP];
      if (COMPAT == MF_COMPAT_POTTS) {
        float tot = 0.f;
#pragma unroll
        for (int l = 0; l < LP; ++l) tot += S[l];
#pragma unroll
        for (int l = 0; l < LP; ++l) {
          z[l] = -INFINITY;
          if (l < L) {
            const float m = uu[l] + a.potts_w * (tot - S[l]);
            z[l] = one_minus_alpha * ls[l * RN + c] - a.alpha * m;
          }
        }
      } else {
        const float* __restrict__ th = a.theta;
#pragma unroll
        for (int l = 0; l < LP; ++l) {
          z[l] = -INFINITY;
          if (l < L) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < LP; ++k)
              if (k < L) acc = fmaf(th[l * L + k], S[k], acc);
            const float m = uu[l] + acc;
            z[l] = one_minus_alpha * ls[l * RN + c] - a.alpha * m;
          }
        }
      }

      float mx = -INFINITY;
#pragma unroll
      for (int l = 0; l < LP; ++l)
        if (l < L) mx = fmaxf(mx, z[l]);
      float e[LP];
      float se = 0.f;
#pragma unroll
      for (int l = 0; l < LP; ++l) {
        e[l] = 0.f;
        if (l < L) {
          e[l] = __expf(z[l] - mx);
          se += e[l];
        }
      }
      const float lse = mx + __logf(se);
      const float inv = 1.0f / se;
#pragma unroll
      for (int l = 0; l < LP; ++l) {
        if (l < L) {
          ls[l * RN + c] = z[l] - lse;
          qn[l * RN + c] = M::enc(e[l] * inv);
        }
      }
    }
    __syncthreads();
    cur ^= 1;
  }

  // Write the TX x TY output tile (iteration t + ks).
  float* __restrict__ out = a.state_out + base;
  for (int f = tid; f < L * TX * TY; f += kTThreads) {
    const int l = f / (TX * TY);
    const int o = f - l * (TX * TY);
    const int oy = o / TX, ox = o - (o / TX) * TX;
    const int gy = gy0 + K + oy, gx = gx0 + K + ox;
    if (gy < H && gx < W) out[(size_t)l * N + gy * W + gx] = ls[l * RN + (K + oy) * RX + (K + ox)];
  }
}

template <int LP, bool EXACT, int CONN, int COMPAT, int PREC, int TX, int TY, int K>
hipError_t multi_launch(const StepArgs& a, int ks, hipStream_t s) {
  dim3 grid((a.W + TX - 1) / TX, (a.H + TY - 1) / TY, a.B);
  const float om = (float)(1.0 - (double)a.alpha);
  hipLaunchKernelGGL((grid_multi_step_kernel<LP, EXACT, CONN, COMPAT, PREC, TX, TY, K>), grid,
                     dim3(kTThreads), 0, s, a, om, ks);
  return hipGetLastError();
}

// LDS bytes of one workgroup: two q buffers of the message type plus log q.
template <int LP, int PREC, int RN>
constexpr size_t lds_bytes() {
  return (size_t)LP * RN * (2 * (PREC == P_F32 ? 4 : 2) + 4);
}

template <int LP, bool EXACT, int CONN, int COMPAT, int PREC>
hipError_t multi_k(const StepArgs& a, int K, int ks, hipStream_t s) {
  constexpr size_t kMax = 160 * 1024;
  if (K >= 4 && lds_bytes<LP, PREC, 24 * 24>() <= kMax)
    return multi_launch<LP, EXACT, CONN, COMPAT, PREC, 16, 16, (lds_bytes<LP, PREC, 24 * 24>() <= kMax ? 4 : 1)>(a, ks, s);
  if (K >= 3 && lds_bytes<LP, PREC, 22 * 22>() <= kMax)
    return multi_launch<LP, EXACT, CONN, COMPAT, PREC, 16, 16, (lds_bytes<LP, PREC, 22 * 22>() <= kMax ? 3 : 1)>(a, ks, s);
  return multi_launch<LP, EXACT, CONN, COMPAT, PREC, 16, 16, 2>(a, ks, s);
}

template <int PREC>
struct ForPrec {
  template <int LP, bool EXACT>
  static hipError_t lp(const StepArgs& a, int conn, int compat, int K, int ks, hipStream_t s) {
    if (conn == 4) {
      return compat == MF_COMPAT_POTTS ? multi_k<LP, EXACT, 4, MF_COMPAT_POTTS, PREC>(a, K, ks, s)
                                       : multi_k<LP, EXACT, 4, MF_COMPAT_GENERAL, PREC>(a, K, ks, s);
    }
    return compat == MF_COMPAT_POTTS ? multi_k<LP, EXACT, 8, MF_COMPAT_POTTS, PREC>(a, K, ks, s)
                                     : multi_k<LP, EXACT, 8, MF_COMPAT_GENERAL, PREC>(a, K, ks, s);
  }
  static hipError_t launch(const StepArgs& a, int conn, int compat, int K, int ks, hipStream_t s) {
    const int L = a.L;
    if (L == 2) return lp<2, true>(a, conn, compat, K, ks, s);
    if (L == 21) return lp<21, true>(a, conn, compat, K, ks, s);
    if (L <= 4) return lp<4, false>(a, conn, compat, K, ks, s);
    if (L <= 8) return lp<8, false>(a, conn, compat, K, ks, s);
    if (L <= 16) return lp<16, false>(a, conn, compat, K, ks, s);
    return lp<32, false>(a, conn, compat, K, ks, s);
  }
};

hipError_t launch_f32(const StepArgs& a, int conn, int compat, int K, int ks, hipStream_t s);
hipError_t launch_bf16(const StepArgs& a, int conn, int compat, int K, int ks, hipStream_t s);
hipError_t launch_f16(const StepArgs& a, int conn, int compat, int K, int ks, hipStream_t s);

}  // namespace temporal
}  // namespace mf
