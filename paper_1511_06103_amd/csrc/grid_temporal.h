// Several parallel proximal steps per launch on a grid (temporal blocking),
// with the labels of a node split over LPN lanes.
//
// A workgroup owns a TX x TY output tile and loads the tile plus a K-node
// halo into LDS: log q and q = exp(log q) of (TX + 2K) x (TY + 2K) nodes.
// Sub-step s recomputes the region shrunk by s nodes on each side, so after
// K sub-steps the output tile holds iteration t + K exactly as K separate
// Jacobi steps would (each node still reads its neighbours at iteration
// t + s - 1).  The halo nodes are recomputed redundantly by neighbouring
// workgroups; in exchange the state crosses memory once per K steps and the
// launch is paid once per K steps, which is what bounds grids whose whole
// state fits in the last-level cache.
//
// Inside a sub-step each node of the active region is one task for a group
// of LPN lanes (LG labels per lane, as in grid_lanes.h): neighbour sums of
// the lane's labels, quad-permute DPP broadcasts to assemble the node's S,
// the lane's rows of Theta S, and a log-sum-exp reduced across the group.
// q for the next sub-step comes out of the log-sum-exp for free:
// q'_l = exp(z_l - max) / sum_k exp(z_k - max).
#pragma once
#include <hip/hip_runtime.h>

#include "grid_lanes.h"
#include "mf_internal.h"
#include "msg_codec.h"

namespace mf {
namespace temporal {

using lanes::group_bcast;
using lanes::group_max;
using lanes::group_sum;

constexpr size_t kLdsMax = 160 * 1024;

template <int LG, int LPN, int LC, int PREC, int TX, int TY, int K>
struct TGeom {
  static constexpr int NT = TX * TY * LPN;            // threads per workgroup
  static constexpr int LP = LG * LPN;                 // label slots per node
  static constexpr int NPL = LC > 0 ? LC : LP;        // label planes held in LDS
  static constexpr int RX = TX + 2 * K, RY = TY + 2 * K, RN = RX * RY;
  static constexpr int TS = (NPL + 3) & ~3;           // Theta row stride in LDS
  static constexpr size_t lds = (size_t)NPL * RN * (2 * sizeof(typename MsgT<PREC>::T) + 4) +
                                (size_t)NPL * TS * 4;
};


template <int LG, int LPN, int LC, int CONN, int COMPAT, int PREC, int TX, int TY, int K>
__global__ __launch_bounds__((TGeom<LG, LPN, LC, PREC, TX, TY, K>::NT)) void multi_step_kernel(
    StepArgs a, float one_minus_alpha, int ks) {
  using G = TGeom<LG, LPN, LC, PREC, TX, TY, K>;
  using M = MsgT<PREC>;
  using T = typename M::T;
  constexpr int NT = G::NT, LP = G::LP, NPL = G::NPL, RX = G::RX, RN = G::RN, TS = G::TS;
  constexpr int LOADS = (NPL * RN + NT - 1) / NT;
  constexpr int KMAX = LC > 0 ? LC : LP;
  __shared__ T qs[2][NPL * RN];
  __shared__ float ls[NPL * RN];
  __shared__ float ths[NPL * TS];

  const int L = LC > 0 ? LC : a.L;
  const unsigned N = (unsigned)a.N;
  const int H = a.H, W = a.W;
  const int b = blockIdx.z;
  const int gx0 = blockIdx.x * TX - K, gy0 = blockIdx.y * TY - K;
  const size_t base = (size_t)b * L * N;
  const float* __restrict__ lin = a.state_in + base;
  const float* __restrict__ ug = a.unary + base;
  const int tid = threadIdx.x;

  // Region load: log q and q of the tile and its K-halo; off-grid q = 0.
  float v[LOADS];
#pragma unroll
  for (int r = 0; r < LOADS; ++r) {
    const int f = tid + r * NT;
    const int l = f / RN;
    const int c = f - l * RN;
    const int ry = c / RX, rx = c - (c / RX) * RX;
    const int gy = gy0 + ry, gx = gx0 + rx;
    const bool ok = f < NPL * RN && l < L && gy >= 0 && gy < H && gx >= 0 && gx < W;
    const float x = lin[ok ? (unsigned)l * N + (unsigned)(gy * W + gx) : 0u];
    v[r] = ok ? x : -INFINITY;
  }
  if (COMPAT == MF_COMPAT_GENERAL) {
    for (int f = tid; f < NPL * TS; f += NT) {
      const int l = f / TS, k = f - (f / TS) * TS;
      ths[f] = (l < L && k < L) ? a.theta[l * L + k] : 0.f;
    }
  }
#pragma unroll
  for (int r = 0; r < LOADS; ++r) {
    const int f = tid + r * NT;
    if (f < NPL * RN) {
      ls[f] = v[r];
      const T e = M::enc(__expf(v[r]));
      qs[0][f] = e;
      qs[1][f] = e;
    }
  }
  __syncthreads();

  int cur = 0;
  for (int s = 1; s <= ks; ++s) {
    const int m0 = K - ks + s;                 // margin of the region updated in this sub-step
    const int AX = RX - 2 * m0, AY = G::RY - 2 * m0;
    const int tasks = AX * AY * LPN;
    const T* __restrict__ qc = qs[cur];
    T* __restrict__ qn = qs[cur ^ 1];
    for (int i = tid; i < tasks; i += NT) {
      const int node = i / LPN, sub = i - (i / LPN) * LPN;
      const int ry = m0 + node / AX, rx = m0 + (node - (node / AX) * AX);
      const int gy = gy0 + ry, gx = gx0 + rx;
      if (gy < 0 || gy >= H || gx < 0 || gx >= W) continue;   // the whole group skips together
      const int c = ry * RX + rx;
      const unsigned n = (unsigned)(gy * W + gx);

      bool valid[LG];
      int pl[LG];
      float uu[LG];
#pragma unroll
      for (int j = 0; j < LG; ++j) {
        const int l = sub * LG + j;
        valid[j] = l < L;
        pl[j] = l < L ? l : L - 1;
        uu[j] = ug[(unsigned)pl[j] * N + n];
      }
      float S[LG], ell[LG];
#pragma unroll
      for (int j = 0; j < LG; ++j) {
        const T* q = qc + pl[j] * RN + c;
        float sum = M::dec(q[-RX]) + M::dec(q[-1]) + M::dec(q[1]) + M::dec(q[RX]);
        if (CONN == 8) sum += (M::dec(q[-RX - 1]) + M::dec(q[-RX + 1])) + (M::dec(q[RX - 1]) + M::dec(q[RX + 1]));
        S[j] = valid[j] ? sum : 0.f;
        ell[j] = ls[pl[j] * RN + c];
      }

      float z[LG];
      if (COMPAT == MF_COMPAT_POTTS) {
        float tot = 0.f;
#pragma unroll
        for (int j = 0; j < LG; ++j) tot += S[j];
        tot = group_sum<LPN>(tot);
#pragma unroll
        for (int j = 0; j < LG; ++j) {
          const float m = uu[j] + a.potts_w * (tot - S[j]);
          z[j] = valid[j] ? one_minus_alpha * ell[j] - a.alpha * m : -INFINITY;
        }
      } else {
        float Sa[LP];
#pragma unroll
        for (int j = 0; j < LG; ++j) {
          Sa[0 * LG + j] = group_bcast<LPN, 0>(S[j]);
          if constexpr (LPN >= 2) Sa[1 * LG + j] = group_bcast<LPN, 1>(S[j]);
          if constexpr (LPN >= 4) {
            Sa[2 * LG + j] = group_bcast<LPN, 2>(S[j]);
            Sa[3 * LG + j] = group_bcast<LPN, 3>(S[j]);
          }
        }
#pragma unroll
        for (int j = 0; j < LG; ++j) {
          const float* th = ths + pl[j] * TS;
          float acc = 0.f;
#pragma unroll
          for (int k = 0; k < KMAX; ++k) acc = fmaf(th[k], Sa[k], acc);
          const float zz = one_minus_alpha * ell[j] - a.alpha * (uu[j] + acc);
          z[j] = valid[j] ? zz : -INFINITY;
        }
      }

      float mx = z[0];
#pragma unroll
      for (int j = 1; j < LG; ++j) mx = fmaxf(mx, z[j]);
      mx = group_max<LPN>(mx);
      float e[LG];
      float se = 0.f;
#pragma unroll
      for (int j = 0; j < LG; ++j) {
        e[j] = __expf(z[j] - mx);            // exp(-inf) = 0 for empty slots
        se += e[j];
      }
      se = group_sum<LPN>(se);
      const float lse = mx + __logf(se);
      const float inv = 1.0f / se;
#pragma unroll
      for (int j = 0; j < LG; ++j) {
        if (valid[j]) {
          ls[pl[j] * RN + c] = z[j] - lse;
          qn[pl[j] * RN + c] = M::enc(e[j] * inv);
        }
      }
    }
    __syncthreads();
    cur ^= 1;
  }

  // Write the TX x TY output tile (iteration t + ks).
  float* __restrict__ out = a.state_out + base;
  for (int f = tid; f < L * TX * TY; f += NT) {
    const int l = f / (TX * TY);
    const int o = f - l * (TX * TY);
    const int oy = o / TX, ox = o - (o / TX) * TX;
    const int gy = gy0 + K + oy, gx = gx0 + K + ox;
    if (gy < H && gx < W) out[(unsigned)l * N + (unsigned)(gy * W + gx)] = ls[l * RN + (K + oy) * RX + (K + ox)];
  }
}

// Largest K in {4, 3, 2} whose LDS footprint fits, for a label split.
template <int LG, int LPN, int LC, int PREC>
constexpr int kmax_for() {
  if (TGeom<LG, LPN, LC, PREC, 16, 16, 4>::lds <= kLdsMax) return 4;
  if (TGeom<LG, LPN, LC, PREC, 16, 16, 3>::lds <= kLdsMax) return 3;
  return 2;
}

template <int PREC>
struct ForPrec {
  template <int LG, int LPN, int LC, int CONN, int COMPAT, int K>
  static hipError_t go(const StepArgs& a, int ks, hipStream_t s) {
    dim3 grid((a.W + 15) / 16, (a.H + 15) / 16, a.B);
    const float om = (float)(1.0 - (double)a.alpha);
    hipLaunchKernelGGL((multi_step_kernel<LG, LPN, LC, CONN, COMPAT, PREC, 16, 16, K>), grid,
                       dim3(TGeom<LG, LPN, LC, PREC, 16, 16, K>::NT),
                       0, s, a, om, ks);
    return hipGetLastError();
  }
  template <int LG, int LPN, int LC, int CONN, int COMPAT>
  static hipError_t k(const StepArgs& a, int K, int ks, hipStream_t s) {
    constexpr int KM = kmax_for<LG, LPN, LC, PREC>();
    if (K >= 4 && KM >= 4) return go<LG, LPN, LC, CONN, COMPAT, (KM >= 4 ? 4 : 2)>(a, ks, s);
    if (K >= 3 && KM >= 3) return go<LG, LPN, LC, CONN, COMPAT, (KM >= 3 ? 3 : 2)>(a, ks, s);
    return go<LG, LPN, LC, CONN, COMPAT, 2>(a, ks, s);
  }
  template <int LG, int LPN, int LC>
  static hipError_t split(const StepArgs& a, int conn, int compat, int K, int ks, hipStream_t s) {
    if (conn == 4) {
      return compat == MF_COMPAT_POTTS ? k<LG, LPN, LC, 4, MF_COMPAT_POTTS>(a, K, ks, s)
                                       : k<LG, LPN, LC, 4, MF_COMPAT_GENERAL>(a, K, ks, s);
    }
    return compat == MF_COMPAT_POTTS ? k<LG, LPN, LC, 8, MF_COMPAT_POTTS>(a, K, ks, s)
                                     : k<LG, LPN, LC, 8, MF_COMPAT_GENERAL>(a, K, ks, s);
  }
  // Same label splits as the single-step kernels.
  static hipError_t launch(const StepArgs& a, int conn, int compat, int K, int ks, hipStream_t s) {
    const int L = a.L;
    if (L == 2) return split<2, 1, 2>(a, conn, compat, K, ks, s);
    if (L <= 2) return split<2, 1, 0>(a, conn, compat, K, ks, s);
    if (L <= 4) return split<4, 1, 0>(a, conn, compat, K, ks, s);
    if (L <= 8) return split<4, 2, 0>(a, conn, compat, K, ks, s);
    if (L <= 16) return split<4, 4, 0>(a, conn, compat, K, ks, s);
    if (L == 21) return split<6, 4, 21>(a, conn, compat, K, ks, s);
    if (L <= 24) return split<6, 4, 0>(a, conn, compat, K, ks, s);
    return split<8, 4, 0>(a, conn, compat, K, ks, s);
  }
  static int kmax(int L) {
    if (L == 2) return kmax_for<2, 1, 2, PREC>();
    if (L <= 2) return kmax_for<2, 1, 0, PREC>();
    if (L <= 4) return kmax_for<4, 1, 0, PREC>();
    if (L <= 8) return kmax_for<4, 2, 0, PREC>();
    if (L <= 16) return kmax_for<4, 4, 0, PREC>();
    if (L == 21) return kmax_for<6, 4, 21, PREC>();
    if (L <= 24) return kmax_for<6, 4, 0, PREC>();
    return kmax_for<8, 4, 0, PREC>();
  }
};

hipError_t launch_f32(const StepArgs& a, int conn, int compat, int K, int ks, hipStream_t s);
hipError_t launch_bf16(const StepArgs& a, int conn, int compat, int K, int ks, hipStream_t s);
hipError_t launch_f16(const StepArgs& a, int conn, int compat, int K, int ks, hipStream_t s);

}  // namespace temporal
}  // namespace mf
