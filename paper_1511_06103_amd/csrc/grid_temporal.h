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

#include <type_traits>

#include "grid_lanes.h"
#include "mf_internal.h"
#include "msg_codec.h"

namespace mf {
namespace temporal {

using lanes::group_bcast;
using lanes::group_max;
using lanes::group_sum;

constexpr size_t kLdsMax = 160 * 1024;

// Store and load of a q value in either LDS layout (identity in FP32).
template <class QT, class M>
__device__ inline QT q_put(float v) {
  if constexpr (std::is_same<QT, float>::value) return M::dec(M::enc(v));
  else return M::enc(v);
}
template <class QT, class M>
__device__ inline float q_get(QT v) {
  if constexpr (std::is_same<QT, float>::value) return v;
  else return M::dec(v);
}

template <int LG, int LPN, int LC, int PREC, int TX, int TY, int K>
struct TGeom {
  static constexpr int NT = TX * TY * LPN;            // threads per workgroup
  static constexpr int LP = LG * LPN;                 // label slots per node
  static constexpr int NPL = LC > 0 ? LC : LP;        // label planes held in LDS
  static constexpr int RX = TX + 2 * K, RY = TY + 2 * K;
  // plane stride: at least RX * RY, padded so that the LPN lanes of a node
  // (reading planes LG apart at the same position) hit different LDS banks
  static constexpr int RN = lanes::plane_stride<LG, LPN>(RX * RY);
  static constexpr int TS = (NPL + 3) & ~3;           // Theta row stride in LDS
  static constexpr size_t lds_with(size_t qbytes) {
    return (size_t)NPL * RN * (2 * qbytes + 4) + (size_t)NPL * TS * 4;
  }
  // q in LDS as FP32 values of the message type whenever both buffers fit
  // that way (as in MGeom below)
  static constexpr bool QF = PREC == P_F32 || lds_with(4) <= kLdsMax;
  using QT = typename std::conditional<QF, float, typename MsgT<PREC>::T>::type;
  static constexpr size_t lds = lds_with(sizeof(QT));
};


template <int LG, int LPN, int LC, int CONN, int COMPAT, int PREC, int TX, int TY, int K>
__global__ __launch_bounds__((TGeom<LG, LPN, LC, PREC, TX, TY, K>::NT)) void multi_step_kernel(
    StepArgs a, float one_minus_alpha, int ks) {
  using G = TGeom<LG, LPN, LC, PREC, TX, TY, K>;
  using M = MsgT<PREC>;
  using T = typename G::QT;                 // q's word in LDS
  constexpr int NT = G::NT, LP = G::LP, NPL = G::NPL, RX = G::RX, RN = G::RN, TS = G::TS;
  constexpr int RA = RX * G::RY;                       // region nodes (RN >= RA is the padded stride)
  constexpr int LOADS = (NPL * RA + NT - 1) / NT;
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
    const int l = f / RA;
    const int c = f - l * RA;
    const int ry = c / RX, rx = c - (c / RX) * RX;
    const int gy = gy0 + ry, gx = gx0 + rx;
    const bool ok = f < NPL * RA && l < L && gy >= 0 && gy < H && gx >= 0 && gx < W;
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
    if (f < NPL * RA) {
      const int l = f / RA;
      const int o = l * RN + (f - l * RA);
      ls[o] = v[r];
      const T e = q_put<T, M>(__expf(v[r]));
      qs[0][o] = e;
      qs[1][o] = e;
    }
  }
  __syncthreads();

  int cur = 0;
  for (int s = 1; s <= ks; ++s) {
    const int m0 = K - ks + s;                 // margin of the region updated in this sub-step
    const int AX = RX - 2 * m0, AY = G::RY - 2 * m0;
    const int tasks = AX * AY * LPN;
    // node / AX through a float reciprocal: node < 2^12 and AX <= 64, so the
    // rounded quotient is off by at most one and is corrected below
    const float inv_ax = 1.0f / (float)AX;
    const T* __restrict__ qc = qs[cur];
    T* __restrict__ qn = qs[cur ^ 1];
    for (int i = tid; i < tasks; i += NT) {
      const int node = i / LPN, sub = i - (i / LPN) * LPN;
      int qy = (int)((float)node * inv_ax);
      int qx = node - qy * AX;
      if (qx < 0) { qy -= 1; qx += AX; }
      if (qx >= AX) { qy += 1; qx -= AX; }
      const int ry = m0 + qy, rx = m0 + qx;
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
        float sum = q_get<T, M>(q[-RX]) + q_get<T, M>(q[-1]) + q_get<T, M>(q[1]) + q_get<T, M>(q[RX]);
        if (CONN == 8)
          sum += (q_get<T, M>(q[-RX - 1]) + q_get<T, M>(q[-RX + 1])) + (q_get<T, M>(q[RX - 1]) + q_get<T, M>(q[RX + 1]));
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
          qn[pl[j] * RN + c] = q_put<T, M>(e[j] * inv);
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

// ---------------------------------------------------------------------------
// The same fused steps with Theta S on the FP32 matrix cores (general Theta,
// 8 < L <= 32).
//
// v_mfma_f32_16x16x4f32 computes D(16x16) += A(16x4) B(4x16); lane x of the
// wavefront holds A[x % 16][x / 16], B[x / 16][x % 16] and rows
// 4 (x / 16) + i, column x % 16 of D in accumulator register i.  A task is
// 16 nodes (column c = x % 16) and lane group g = x / 16 owns label slots
// g + 4 j, j < LG.  B for k-block j is then exactly the lane's own
// neighbour sum S[g + 4 j] -- no exchange of S between lanes -- and
// D rows are numbered so that register i of output block ob lands on slot
// g + 4 (4 ob + i) of the same lane: the lane receives Theta S for the
// labels it owns.  A is Theta under these two numberings, a constant
// 2 x LG registers per lane.  The per-node log-sum-exp reduces over the four
// lanes x, x ^ 16, x ^ 32, x ^ 48 with the gfx950 row-swap permutes.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Reductions over the four lanes x, x ^ 16, x ^ 32, x ^ 48 (one node's label
// slots), in the VALU.  v_permlane16_swap with both operands equal to v
// leaves rows (0, 0, 2, 2) of v in the first result and rows (1, 1, 3, 3) in
// the second, so op(first, second) combines rows 0 with 1 and 2 with 3 in
// every lane; v_permlane32_swap does the same for the two half-waves.  The
// operation is commutative, so all four lanes hold bitwise the same result.
__device__ inline float max_sel(float a, float b) { return a > b ? a : b; }   // no NaN quieting

__device__ inline float rows_max(float v) {
  const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = max_sel(__uint_as_float(p[0]), __uint_as_float(p[1]));
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return max_sel(__uint_as_float(r[0]), __uint_as_float(r[1]));
}

// LDS byte address of a __shared__ object, and an LDS pointer from one.
template <class T>
__device__ inline unsigned lds_addr(const T* p) {
  return (unsigned)(size_t)(const __attribute__((address_space(3))) T*)p;
}
template <class T>
__device__ inline const T* lds_ptr(unsigned byte_addr) {
  return (const T*)(const __attribute__((address_space(3))) T*)(size_t)byte_addr;
}

// An integer the compiler must treat as unknown (an empty register-to-
// register asm, no memory access): loads addressed from it keep it as their
// base instead of being re-paired onto freshly computed bases.
__device__ inline unsigned opaque(unsigned x) {
  asm volatile("" : "+v"(x));
  return x;
}

__device__ inline float rows_sum(float v) {
  const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = __uint_as_float(p[0]) + __uint_as_float(p[1]);
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Plane stride for the MFMA layout: lanes x and x + 16 read planes one apart
// at the same position, so a stride of 16 mod 64 words puts the four lane
// groups of a wavefront on disjoint LDS banks.
constexpr int mfma_plane_stride(int ra) { return ra + ((16 - ra % 64) + 64) % 64; }

template <int LG, int LC, int PREC, int TX, int TY, int K>
struct MGeom {
  static constexpr int NT = TX * TY * 4;              // 4 lanes per node
  static constexpr int LP = 4 * LG;                   // label slots = q planes in LDS
  static constexpr int NPL = LC > 0 ? LC : LP;        // log q planes in LDS
  static constexpr int NOB = (LG + 3) / 4;            // output blocks of 16 rows
  static constexpr int RX = TX + 2 * K, RY = TY + 2 * K, RA = RX * RY;
  static constexpr int RN = mfma_plane_stride(RA);
  static constexpr size_t lds_with(size_t qbytes) { return (size_t)RN * (2 * LP * qbytes + NPL * 4); }
  // q in LDS as FP32 values of the message type (16-bit messages rounded
  // where q is written) whenever both buffers fit that way; 16-bit words
  // otherwise, where FP32 words would force a shallower launch.  The
  // stencil reads whole words without a decode in the FP32 layout.
  static constexpr bool QF = PREC == P_F32 || lds_with(4) <= kLdsMax;
  using QT = typename std::conditional<QF, float, typename MsgT<PREC>::T>::type;
  static constexpr size_t lds = lds_with(sizeof(QT));
};

// Global load at a 32-bit byte offset from a wavefront-uniform base (the
// saddr + voffset form: no per-lane 64-bit address arithmetic).
__device__ inline float load_at(const float* base, unsigned byte_off) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + byte_off);
}

template <int LG, int LC, int CONN, int PREC, int TX, int TY, int K>
__global__ __launch_bounds__((MGeom<LG, LC, PREC, TX, TY, K>::NT)) void multi_step_mfma_kernel(
    StepArgs a, float one_minus_alpha, int ks) {
  using G = MGeom<LG, LC, PREC, TX, TY, K>;
  using M = MsgT<PREC>;
  using T = typename G::QT;                 // q's word in LDS
  constexpr int NT = G::NT, NW = NT / 64, LP = G::LP, NPL = G::NPL, NOB = G::NOB;
  constexpr int RX = G::RX, RA = G::RA, RN = G::RN;
  constexpr int LOADS = (LP * RA + NT - 1) / NT;
  __shared__ T qs[2][LP * RN];
  __shared__ float ls[NPL * RN];

  const int L = LC > 0 ? LC : a.L;
  const unsigned N = (unsigned)a.N;
  const int H = a.H, W = a.W;
  // tiles dealt XCD by XCD (see lanes::xcd_tile): adjacent tiles, whose
  // K-halo regions overlap, share an L2
  const int tiles_x = (a.W + TX - 1) / TX, tiles_y = (a.H + TY - 1) / TY;
  const int tile = lanes::xcd_tile(blockIdx.x, tiles_x * tiles_y * a.B);
  const int b = tile / (tiles_x * tiles_y);
  const int tr = tile - b * (tiles_x * tiles_y);
  const int tyi = tr / tiles_x, txi = tr - tyi * tiles_x;
  const int gx0 = txi * TX - K, gy0 = tyi * TY - K;
  const size_t base = (size_t)b * L * N;
  const float* __restrict__ lin = a.state_in + base;
  const float* __restrict__ ug = a.unary + base;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col = lane & 15, g = lane >> 4;

  // A operands: Theta[out slot of row col][in slot g + 4 kb], zero outside L x L.
  float tha[NOB][LG];
#pragma unroll
  for (int ob = 0; ob < NOB; ++ob) {
    const int jo = 4 * ob + (col & 3);
    const int so = (col >> 2) + 4 * jo;
#pragma unroll
    for (int kb = 0; kb < LG; ++kb) {
      const int si = g + 4 * kb;
      const bool ok = jo < LG && so < L && si < L;
      const float t = a.theta[ok ? so * L + si : 0];
      tha[ob][kb] = ok ? t : 0.f;
    }
  }

  // Region load: log q and q of the tile and its K-halo; off-grid q = 0 and
  // the q planes of padding slots (L <= slot < LP) are 0.
  float v[LOADS];
#pragma unroll
  for (int r = 0; r < LOADS; ++r) {
    const int f = tid + r * NT;
    const int l = f / RA;
    const int c = f - l * RA;
    const int ry = c / RX, rx = c - (c / RX) * RX;
    const int gy = gy0 + ry, gx = gx0 + rx;
    const bool ok = f < LP * RA && l < L && gy >= 0 && gy < H && gx >= 0 && gx < W;
    const float x = lin[ok ? (unsigned)l * N + (unsigned)(gy * W + gx) : 0u];
    v[r] = ok ? x : -INFINITY;
  }
#pragma unroll
  for (int r = 0; r < LOADS; ++r) {
    const int f = tid + r * NT;
    if (f < LP * RA) {
      const int l = f / RA;
      const int o = l * RN + (f - l * RA);
      if (l < NPL) ls[o] = v[r];
      const T e = q_put<T, M>(__expf(v[r]));
      qs[0][o] = e;
      qs[1][o] = e;
    }
  }

  // Slot g + 4 j of this lane.  With the label count known at compile time,
  // every slot of j <= (L - 4) / 4 is a label for all four lane groups.
  bool valid[LG];
#pragma unroll
  for (int j = 0; j < LG; ++j) valid[j] = (LC > 0 && 4 * j + 3 < LC) || g + 4 * j < L;
  const unsigned gN4 = (unsigned)g * N * 4u;
  // A workgroup whose whole region lies on the grid skips the per-node
  // boundary tests (a uniform branch: most workgroups of a large grid).
  const bool interior = gx0 >= 0 && gy0 >= 0 && gx0 + RX <= W && gy0 + G::RY <= H;

  // Geometry of sub-step s: the region shrunk by a margin m0 on each side.
  struct Geo {
    int m0, AX, AY, nodes, wtasks, dy, dx, dc, dn, c_last;
  };
  auto geo = [&](int s) {
    Geo q;
    q.m0 = K - ks + s;
    q.AX = RX - 2 * q.m0;
    q.AY = G::RY - 2 * q.m0;
    q.nodes = q.AX * q.AY;
    q.wtasks = (q.nodes + 15) >> 4;
    q.dy = (NW * 16) / q.AX;
    q.dx = NW * 16 - q.dy * q.AX;
    q.dc = q.dy * RX + q.dx;
    q.dn = q.dy * W + q.dx;
    q.c_last = (q.m0 + q.AY - 1) * RX + q.m0 + q.AX - 1;
    return q;
  };
  // A lane's node: index in the active region, column qx, region offset c,
  // grid position (gy, gx) and grid index n.  Tasks of a wavefront step by
  // NW * 16 nodes.
  struct Pos {
    int node, qx, c, gy, gx, n;
  };
  auto first_pos = [&](const Geo& q) {
    Pos p;
    p.node = wave * 16 + col;
    // node < 2^12 and AX <= 64: the float-reciprocal quotient is off by at
    // most one, corrected below
    int qy = (int)((float)p.node * (1.0f / (float)q.AX));
    p.qx = p.node - qy * q.AX;
    if (p.qx < 0) { qy -= 1; p.qx += q.AX; }
    if (p.qx >= q.AX) { qy += 1; p.qx -= q.AX; }
    p.c = (q.m0 + qy) * RX + q.m0 + p.qx;
    p.gy = gy0 + q.m0 + qy;
    p.gx = gx0 + q.m0 + p.qx;
    p.n = p.gy * W + p.gx;
    return p;
  };
  auto next_pos = [&](Pos p, const Geo& q) {
    p.node += NW * 16;
    p.qx += q.dx;
    p.c += q.dc;
    p.n += q.dn;
    p.gy += q.dy;
    p.gx += q.dx;
    if (p.qx >= q.AX) {
      p.qx -= q.AX;
      p.c += RX - q.AX;
      p.n += W - q.AX;
      p.gy += 1;
      p.gx -= q.AX;
    }
    return p;
  };

  auto sub_steps = [&](auto interior_tag) {
    constexpr bool INTERIOR = decltype(interior_tag)::value;
    auto active = [&](const Pos& p, const Geo& q) {
      const bool on_grid = INTERIOR || (p.gy >= 0 && p.gy < H && p.gx >= 0 && p.gx < W);
      return p.node < q.nodes && on_grid;
    };
    auto load_u = [&](const Pos& p, const Geo& q, float (&u)[LG]) {
      const unsigned nn = active(p, q) ? (unsigned)p.n : 0u;
      const unsigned ub = gN4 + nn * 4u;
#pragma unroll
      for (int j = 0; j < LG; ++j) {
        // a padding slot reads the unary of label L - 1 (unused)
        const unsigned off = valid[j] ? ub + (unsigned)(16 * j) * N : ((unsigned)(L - 1) * N + nn) * 4u;
        u[j] = load_at(ug, off);
      }
    };

    __syncthreads();                           // region load complete
    int cur = 0;
    for (int s = 1; s <= ks; ++s) {
      const Geo qg = geo(s);
      Pos p = first_pos(qg);
      // LDS byte address of plane g at region offset - RX - 1 of this buffer
      const unsigned qc_base = lds_addr(qs[cur]) + (unsigned)(g * RN - RX - 1) * (unsigned)sizeof(T);
      T* __restrict__ qn = qs[cur ^ 1];
      // The loop bound is uniform over the wavefront, so every lane reaches
      // the matrix instructions; nodes past the region or off the grid
      // compute on clamped positions and store nothing.
      for (int t = wave; t < qg.wtasks; t += NW) {
        const Pos pc = p;
        p = next_pos(p, qg);
        float uu[LG];
        load_u(pc, qg, uu);
        const bool in_region = pc.node < qg.nodes;
        const bool act = active(pc, qg);
        const int cc = in_region ? pc.c : qg.c_last;
        const int cb = g * RN + cc;             // plane g at this node
        const unsigned qb = qc_base + (unsigned)cc * (unsigned)sizeof(T);

        float S[LG], ell[LG];
#pragma unroll
        for (int j = 0; j < LG; ++j) {
          // one base per label plane, the eight neighbours at small constant
          // offsets from it (the opaque copy keeps the compiler from
          // re-deriving a base for each pair of reads)
          const T* qp = lds_ptr<T>(opaque(qb + (unsigned)(4 * j * RN) * (unsigned)sizeof(T)));
          const float n0 = q_get<T, M>(qp[1]), w0 = q_get<T, M>(qp[RX]), e0 = q_get<T, M>(qp[RX + 2]),
                      s0 = q_get<T, M>(qp[2 * RX + 1]);
          float tot = (n0 + w0) + (e0 + s0);
          if (CONN == 8)
            tot += (q_get<T, M>(qp[0]) + q_get<T, M>(qp[2])) + (q_get<T, M>(qp[2 * RX]) + q_get<T, M>(qp[2 * RX + 2]));
          S[j] = valid[j] ? tot : 0.f;
          // log q of a padding slot is never used; its plane exists only when NPL == LP
          const int eo = (NPL == LP || valid[j]) ? cb + 4 * j * RN : cc;
          ell[j] = ls[eo];
        }

        f32x4 acc[NOB];
#pragma unroll
        for (int ob = 0; ob < NOB; ++ob) acc[ob] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < LG; ++kb) {
#pragma unroll
          for (int ob = 0; ob < NOB; ++ob)
            acc[ob] = __builtin_amdgcn_mfma_f32_16x16x4f32(tha[ob][kb], S[kb], acc[ob], 0, 0, 0);
        }

        float z[LG];
#pragma unroll
        for (int j = 0; j < LG; ++j) {
          const float zz = one_minus_alpha * ell[j] - a.alpha * (uu[j] + acc[j >> 2][j & 3]);
          z[j] = valid[j] ? zz : -INFINITY;
        }
        float mx = z[0];
#pragma unroll
        for (int j = 1; j < LG; ++j) mx = fmaxf(mx, z[j]);
        mx = rows_max(mx);
        float e[LG];
#pragma unroll
        for (int j = 0; j < LG; ++j) e[j] = __expf(z[j] - mx);   // exp(-inf) = 0 for empty slots
        float se = e[0];
#pragma unroll
        for (int j = 1; j < LG; ++j) se += e[j];
        se = rows_sum(se);
        const float lse = mx + __logf(se);
        const float inv = __builtin_amdgcn_rcpf(se);   // 1 ulp; se >= 1 (the max term is exp(0))
        if (act) {
#pragma unroll
          for (int j = 0; j < LG; ++j) {
            if (valid[j]) {
              ls[cb + 4 * j * RN] = z[j] - lse;
              qn[cb + 4 * j * RN] = q_put<T, M>(e[j] * inv);
            }
          }
        }
      }
      __syncthreads();
      cur ^= 1;
    }
  };
  if (interior) {
    sub_steps(std::true_type{});
  } else {
    sub_steps(std::false_type{});
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

template <int LG, int LC, int PREC>
constexpr int kmax_mfma() {
  if (MGeom<LG, LC, PREC, 16, 16, 4>::lds <= kLdsMax) return 4;
  if (MGeom<LG, LC, PREC, 16, 16, 3>::lds <= kLdsMax) return 3;
  return 2;
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
  template <int LG, int LC, int CONN, int K>
  static hipError_t go_mfma(const StepArgs& a, int ks, hipStream_t s) {
    dim3 grid(((a.W + 15) / 16) * ((a.H + 15) / 16) * a.B);
    const float om = (float)(1.0 - (double)a.alpha);
    hipLaunchKernelGGL((multi_step_mfma_kernel<LG, LC, CONN, PREC, 16, 16, K>), grid,
                       dim3(MGeom<LG, LC, PREC, 16, 16, K>::NT), 0, s, a, om, ks);
    return hipGetLastError();
  }
  template <int LG, int LC, int CONN>
  static hipError_t k_mfma(const StepArgs& a, int K, int ks, hipStream_t s) {
    constexpr int KM = kmax_mfma<LG, LC, PREC>();
    if (K >= 4 && KM >= 4) return go_mfma<LG, LC, CONN, (KM >= 4 ? 4 : 2)>(a, ks, s);
    if (K >= 3 && KM >= 3) return go_mfma<LG, LC, CONN, (KM >= 3 ? 3 : 2)>(a, ks, s);
    return go_mfma<LG, LC, CONN, 2>(a, ks, s);
  }
  template <int LG, int LC>
  static hipError_t mfma(const StepArgs& a, int conn, int K, int ks, hipStream_t s) {
    return conn == 4 ? k_mfma<LG, LC, 4>(a, K, ks, s) : k_mfma<LG, LC, 8>(a, K, ks, s);
  }
  // General Theta with 8 < L <= 32 takes Theta S on the matrix cores.
  static bool uses_mfma(int L, int compat) { return compat == MF_COMPAT_GENERAL && L > 8 && L <= 32; }

  // Same label splits as the single-step kernels.
  static hipError_t launch(const StepArgs& a, int conn, int compat, int K, int ks, hipStream_t s) {
    const int L = a.L;
    if (uses_mfma(L, compat)) {
      if (L <= 16) return mfma<4, 0>(a, conn, K, ks, s);
      if (L == 21) return mfma<6, 21>(a, conn, K, ks, s);
      if (L <= 24) return mfma<6, 0>(a, conn, K, ks, s);
      return mfma<8, 0>(a, conn, K, ks, s);
    }
    if (L == 2) return split<2, 1, 2>(a, conn, compat, K, ks, s);
    if (L <= 2) return split<2, 1, 0>(a, conn, compat, K, ks, s);
    if (L <= 4) return split<4, 1, 0>(a, conn, compat, K, ks, s);
    if (L <= 8) return split<4, 2, 0>(a, conn, compat, K, ks, s);
    if (L <= 16) return split<4, 4, 0>(a, conn, compat, K, ks, s);
    if (L == 21) return split<6, 4, 21>(a, conn, compat, K, ks, s);
    if (L <= 24) return split<6, 4, 0>(a, conn, compat, K, ks, s);
    return split<8, 4, 0>(a, conn, compat, K, ks, s);
  }
  static int kmax(int L, int compat) {
    if (uses_mfma(L, compat)) {
      if (L <= 16) return kmax_mfma<4, 0, PREC>();
      if (L == 21) return kmax_mfma<6, 21, PREC>();
      if (L <= 24) return kmax_mfma<6, 0, PREC>();
      return kmax_mfma<8, 0, PREC>();
    }
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
