// One proximal step on a grid with LPN lanes per node (label-parallel).
//
// Each node's labels are split over a group of LPN adjacent lanes, LG labels
// per lane (LP = LG * LPN >= L slots).  A lane stages q for its own labels,
// sums the neighbours for them, then receives the other lanes' neighbour
// sums through quad-permute DPP broadcasts so that it can form its LG rows
// of Theta S; the per-node log-sum-exp is a max and a sum reduced across
// the LPN lanes with DPP butterflies.  Splitting a node over lanes
// multiplies the wavefront count by LPN: a 256 x 256 grid then keeps
// several wavefronts per SIMD instead of one, so memory and LDS latency are
// covered by other wavefronts instead of stalling the only one.
//
// Step (Eq. 15 with the fixed step of Eq. 16), per node i:
//   S_i = sum of q_j over the 4/8 grid neighbours (free boundary)
//   m_i = u_i + Theta S_i          (Potts: w (sum(S_i) 1 - S_i))
//   z_i = (1 - alpha) log q_i - alpha m_i;   log q_i <- z_i - lse(z_i)
//
// The tile body is shared by the single-problem kernel and the
// many-problem (continuous batching) kernel, so a problem gets bitwise the
// same iterates whichever of the two advances it.
#pragma once
#include <hip/hip_runtime.h>

#include "mf_internal.h"
#include "msg_codec.h"

namespace mf {
namespace lanes {

// Quad-permute DPP: lane i of every group of four reads lane ((CTRL >> 2i) & 3).
template <int CTRL>
__device__ inline float qperm(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Value of lane S of this node's group of LPN lanes.
template <int LPN, int S>
__device__ inline float group_bcast(float v) {
  if constexpr (LPN == 1) {
    return v;
  } else if constexpr (LPN == 2) {
    return qperm<S | (S << 2) | ((2 + S) << 4) | ((2 + S) << 6)>(v);
  } else {
    return qperm<S | (S << 2) | (S << 4) | (S << 6)>(v);
  }
}

template <int LPN>
__device__ inline float group_max(float v) {
  if constexpr (LPN >= 2) v = fmaxf(v, qperm<0xB1>(v));   // xor 1
  if constexpr (LPN >= 4) v = fmaxf(v, qperm<0x4E>(v));   // xor 2
  return v;
}

template <int LPN>
__device__ inline float group_sum(float v) {
  if constexpr (LPN >= 2) v += qperm<0xB1>(v);
  if constexpr (LPN >= 4) v += qperm<0x4E>(v);
  return v;
}

// Plane stride of the q tile in LDS: at least HN, chosen so that the LPN
// lanes of a node (reading LPN different label planes at the same position)
// fall into different LDS banks.
template <int LG, int LPN>
constexpr int plane_stride(int hn) {
  if (LPN == 1) return hn;
  const int want = 64 / LPN;                      // bank offset between sub-lanes
  for (int ps = hn; ps < hn + 64; ++ps)
    if ((LG * ps) % 64 == want) return ps;
  return hn;
}

template <int LG, int LPN, int TX, int TY>
struct Geometry {
  static constexpr int NT = TX * TY * LPN;           // threads per workgroup
  static constexpr int LP = LG * LPN;                // label slots
  static constexpr int HX = TX + 2, HY = TY + 2, HN = HX * HY;
  static constexpr int PS = plane_stride<LG, LPN>(HN);
  static constexpr int LS = (LP + 3) & ~3;           // Theta row stride in LDS
  static constexpr int HALO = 2 * HX + 2 * TY;       // halo ring nodes
};

template <int TX, int TY>
__device__ inline int halo_pos(int h) {
  constexpr int HX = TX + 2, HY = TY + 2;
  if (h < HX) return h;                                   // top row
  if (h < 2 * HX) return (HY - 1) * HX + (h - HX);        // bottom row
  const int k = h - 2 * HX;                               // sides, rows 1..TY
  return (1 + (k >> 1)) * HX + ((k & 1) ? HX - 1 : 0);
}

template <int LG, int LPN, int TX, int TY, int PREC>
struct Smem {
  using G = Geometry<LG, LPN, TX, TY>;
  // q as FP32 values of the message type (16-bit messages rounded where
  // they are written): the stencil reads whole words in every precision
  float q[G::LP * G::PS];
  float theta[G::LP * G::LS];
};

// One problem's [L][N] planes as a raw buffer resource (range = their byte
// extent, dword 3 = the 32-bit data format of CDNA raw buffers).  Loads and
// stores through it take a 32-bit per-lane byte offset plus a wavefront-
// uniform scalar one: no 64-bit address arithmetic per lane and access.
// Byte offsets fit in 32 bits because L N < 2^30 is checked at creation.
__device__ inline __amdgpu_buffer_rsrc_t planes_rsrc(const float* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), (short)0, (int)bytes, 0x00020000);
}
// aux bit 1: non-temporal (the nt bit of the access)
constexpr int kBufNt = 2;
template <int AUX>
__device__ inline float buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
}
template <int AUX>
__device__ inline void buf_store(float v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, AUX);
}

// Normalise z over the valid slots and store z - lse(z) as log q'.
template <int LG>
__device__ inline void store_normalised(float* __restrict__ out, const bool (&valid)[LG], const float (&z)[LG],
                                        unsigned N, unsigned n) {
  float mx = z[0];
#pragma unroll
  for (int j = 1; j < LG; ++j) mx = fmaxf(mx, z[j]);
  float se = 0.f;
#pragma unroll
  for (int j = 0; j < LG; ++j) se += __expf(z[j] - mx);    // exp(-inf) = 0 for empty slots
  const float lse = mx + __logf(se);
#pragma unroll
  for (int j = 0; j < LG; ++j)
    if (valid[j]) out[(unsigned)j * N + n] = z[j] - lse;
}

// The update of the non-fixed step rules from the messages mm at one node
// (one lane per node: slot j is label j).  z holds the fixed-step value.
template <int LG, int CONN, int RULE>
__device__ inline void rule_epilogue(const StepArgs& a, const RuleArgs& rx, const bool (&valid)[LG],
                                     const float (&ell)[LG], const float (&mm)[LG], float (&z)[LG], size_t base,
                                     unsigned N, unsigned n, int x, int y, int L) {
  float* __restrict__ out = a.state_out + base;
  if constexpr (RULE == MF_RULE_ADAPTIVE) {
    // Eq. 19: d_i = q_i0 q_i1 d, alpha_i = 1 / (1 + d_i) (L = 2)
    const float qq = __expf(ell[0]) * __expf(ell[1]);
    const float eta = 1.0f / (1.0f + qq * rx.d);
#pragma unroll
    for (int j = 0; j < LG; ++j) z[j] = valid[j] ? (1.0f - eta) * ell[j] - eta * mm[j] : -INFINITY;
    store_normalised<LG>(out, valid, z, N, n);
  } else if constexpr (RULE == MF_RULE_ADHOC) {
    // Eq. 9: q' = (1 - eta) q + eta softmax(-m), eta = alpha
    float zs[LG];
#pragma unroll
    for (int j = 0; j < LG; ++j) zs[j] = valid[j] ? -mm[j] : -INFINITY;
    float mx = zs[0];
#pragma unroll
    for (int j = 1; j < LG; ++j) mx = fmaxf(mx, zs[j]);
    float se = 0.f;
#pragma unroll
    for (int j = 0; j < LG; ++j) se += __expf(zs[j] - mx);
    const float lse = mx + __logf(se);
    const float eta = a.alpha;
#pragma unroll
    for (int j = 0; j < LG; ++j) {
      if (valid[j]) {
        const float qn = (1.0f - eta) * __expf(ell[j]) + eta * __expf(zs[j] - lse);
        out[(unsigned)j * N + n] = __logf(qn);
      }
    }
  } else if constexpr (RULE == MF_RULE_SWEEP) {
    // colour class of the node; the others are copied unchanged
    // neighbours always differ in colour: (x + y) mod 2 with 4 neighbours,
    // (x mod 2) + 2 (y mod 2) with 8
    const int colour = CONN == 4 ? ((x + y) & 1) : ((x & 1) + 2 * (y & 1));
    if (colour == rx.colour) {
#pragma unroll
      for (int j = 0; j < LG; ++j) z[j] = valid[j] ? -mm[j] : -INFINITY;
      store_normalised<LG>(out, valid, z, N, n);
    } else {
#pragma unroll
      for (int j = 0; j < LG; ++j)
        if (valid[j]) out[(unsigned)j * N + n] = ell[j];
    }
  } else {
    static_assert(RULE == MF_RULE_MOMENTUM || RULE == MF_RULE_ADAM, "unknown step rule");
    float* __restrict__ mom = rx.mom + base;
    if (rx.init) {
      // mom^0 = m(q^0), v^0 = v0; log q is left as it is
#pragma unroll
      for (int j = 0; j < LG; ++j) {
        if (valid[j]) {
          mom[(unsigned)j * N + n] = mm[j];
          if constexpr (RULE == MF_RULE_ADAM) rx.sq[base + (unsigned)j * N + n] = rx.v0;
        }
      }
      return;
    }
    float mo[LG];
#pragma unroll
    for (int j = 0; j < LG; ++j) {
      const unsigned o = (unsigned)(j < L ? j : L - 1) * N + n;
      mo[j] = rx.gamma1 * mom[o] + (1.0f - rx.gamma1) * mm[j];
    }
    if constexpr (RULE == MF_RULE_MOMENTUM) {
      const float om = 1.0f - a.alpha;
#pragma unroll
      for (int j = 0; j < LG; ++j) z[j] = valid[j] ? om * ell[j] - a.alpha * mo[j] : -INFINITY;
    } else {
      // natural gradient g = m + log q, centred over the labels
      float* __restrict__ sq = rx.sq + base;
      float g[LG];
      float gbar = 0.f;
#pragma unroll
      for (int j = 0; j < LG; ++j) {
        g[j] = mm[j] + ell[j];
        if (valid[j]) gbar += g[j];
      }
      gbar /= (float)L;
#pragma unroll
      for (int j = 0; j < LG; ++j) {
        const unsigned o = (unsigned)(j < L ? j : L - 1) * N + n;
        const float gc = g[j] - gbar;
        const float v = rx.gamma2 * sq[o] + (1.0f - rx.gamma2) * gc * gc;
        const float dt = fmaxf(sqrtf(v) * rx.d + rx.eps - 1.0f, 1e-6f);
        const float eta = 1.0f / (1.0f + dt);
        z[j] = valid[j] ? (1.0f - eta) * ell[j] - eta * mo[j] : -INFINITY;
        if (valid[j]) sq[o] = v;
      }
    }
#pragma unroll
    for (int j = 0; j < LG; ++j)
      if (valid[j]) mom[(unsigned)j * N + n] = mo[j];
    store_normalised<LG>(out, valid, z, N, n);
  }
}

// Branch-free tile body.  LC is the label count when it is known at compile
// time (0: runtime a.L); slots l >= L are carried with q = 0 and a zero row
// and column of Theta, so every lane runs the same straight-line code and
// only the final store is masked.
//
// RULE selects the update made from the messages m (mf_rule); every rule but
// MF_RULE_FIXED runs one lane per node and takes its extra state and
// constants from rx.
//
// STREAM marks the unaries and the new state as streams (non-temporal load and
// store): on grids whose arrays cannot stay in the last-level cache between
// steps they are read or written once per step, and keeping them out of the
// cache leaves it to the halo rows that neighbouring tiles share.
template <int LG, int LPN, int LC, int CONN, int COMPAT, int PREC, int TX, int TY, int RULE = MF_RULE_FIXED,
          bool STREAM = false>
__device__ inline void tile_step(const StepArgs& a, float one_minus_alpha, int b, int x0, int y0,
                                 Smem<LG, LPN, TX, TY, PREC>& sm, const RuleArgs* rx = nullptr) {
  static_assert(RULE == MF_RULE_FIXED || LPN == 1, "step rules run one lane per node");
  using G = Geometry<LG, LPN, TX, TY>;
  using M = MsgT<PREC>;
  constexpr int LP = G::LP, PS = G::PS, LS = G::LS, HX = G::HX, NT = G::NT, HALO = G::HALO;
  constexpr int HREG = (LP * HALO + NT - 1) / NT;
  constexpr int TREG = (COMPAT == MF_COMPAT_GENERAL) ? (LP * LS + NT - 1) / NT : 0;
  constexpr int KMAX = LC > 0 ? LC : LP;      // Theta columns that can be nonzero
  const int L = LC > 0 ? LC : a.L;
  const unsigned N = (unsigned)a.N;
  const int H = a.H, W = a.W;
  const size_t base = (size_t)b * L * N;
  const float* __restrict__ lin = a.state_in + base;
  const float* __restrict__ ug = a.unary + base;
  const int tid = threadIdx.x;
  const int sub = tid % LPN, nl = tid / LPN;
  const int tx = nl % TX, ty = nl / TX;
  const int x = x0 + tx, y = y0 + ty;
  const bool inside = x < W && y < H;
  const unsigned n = inside ? (unsigned)(y * W + x) : 0u;

  // All global loads first: own labels, this thread's share of the halo, Theta.
  // Addresses are clamped into range and the value is selected afterwards, so
  // no load is skipped by a branch.  With one lane per node the label
  // plane's offset is the same in every lane (the scalar offset).
  const unsigned pbytes = (unsigned)L * N * 4u;
  const __amdgpu_buffer_rsrc_t rl = planes_rsrc(lin, pbytes), ru = planes_rsrc(ug, pbytes);
  constexpr int kUAux = STREAM ? kBufNt : 0;
  bool valid[LG];
  float ell[LG], uu[LG];
#pragma unroll
  for (int j = 0; j < LG; ++j) {
    const int l = sub * LG + j;
    valid[j] = l < L;
    if constexpr (LPN == 1) {
      const unsigned so = (unsigned)(j < L ? j : L - 1) * N * 4u;
      ell[j] = buf_load<0>(rl, n * 4u, so);
      uu[j] = buf_load<kUAux>(ru, n * 4u, so);
    } else {
      const unsigned vo = ((unsigned)(l < L ? l : L - 1) * N + n) * 4u;
      ell[j] = buf_load<0>(rl, vo, 0u);
      uu[j] = buf_load<kUAux>(ru, vo, 0u);
    }
  }
  float hv[HREG];
#pragma unroll
  for (int r = 0; r < HREG; ++r) {
    const int f = tid + r * NT;
    const int l = f / HALO;
    const int pos = halo_pos<TX, TY>(f - l * HALO);
    const int hy = pos / HX, hx = pos - (pos / HX) * HX;
    const int gy = y0 + hy - 1, gx = x0 + hx - 1;
    const bool ok = f < LP * HALO && l < L && gy >= 0 && gy < H && gx >= 0 && gx < W;
    const unsigned off = ok ? (unsigned)l * N + (unsigned)(gy * W + gx) : 0u;
    const float v = buf_load<0>(rl, off * 4u, 0u);
    hv[r] = ok ? v : -INFINITY;
  }
  float tv[TREG > 0 ? TREG : 1];
#pragma unroll
  for (int r = 0; r < TREG; ++r) {
    const int f = tid + r * NT;
    const int l = f / LS, k = f - (f / LS) * LS;
    const bool ok = l < L && k < L;
    const float v = a.theta[ok ? l * L + k : 0];
    tv[r] = ok ? v : 0.f;
  }

  const int p = (ty + 1) * HX + (tx + 1);
#pragma unroll
  for (int j = 0; j < LG; ++j) {
    const int l = sub * LG + j;
    sm.q[l * PS + p] = M::dec(M::enc((inside && valid[j]) ? __expf(ell[j]) : 0.f));
  }
#pragma unroll
  for (int r = 0; r < HREG; ++r) {
    const int f = tid + r * NT;
    if (f < LP * HALO) {
      const int l = f / HALO;
      sm.q[l * PS + halo_pos<TX, TY>(f - l * HALO)] = M::dec(M::enc(__expf(hv[r])));   // exp(-inf) = 0
    }
  }
#pragma unroll
  for (int r = 0; r < TREG; ++r) {
    const int f = tid + r * NT;
    if (f < LP * LS) sm.theta[f] = tv[r];
  }
  __syncthreads();
  if (!inside) return;     // whole groups leave together: the LPN lanes share the node

  // Neighbour sums of this lane's labels.
  float S[LG];
#pragma unroll
  for (int j = 0; j < LG; ++j) {
    const float* q = sm.q + (sub * LG + j) * PS + p;
    float s = q[-HX] + q[-1] + q[1] + q[HX];
    if (CONN == 8) s += (q[-HX - 1] + q[-HX + 1]) + (q[HX - 1] + q[HX + 1]);
    S[j] = s;
  }

  // m = u + Theta S (Potts: u + w (sum(S) 1 - S)) and the fixed-step z
  float mm[LG], z[LG];
  if (COMPAT == MF_COMPAT_POTTS) {
    float tot = 0.f;
#pragma unroll
    for (int j = 0; j < LG; ++j) tot += S[j];
    tot = group_sum<LPN>(tot);
#pragma unroll
    for (int j = 0; j < LG; ++j) {
      const float m = uu[j] + a.potts_w * (tot - S[j]);
      mm[j] = m;
      z[j] = valid[j] ? one_minus_alpha * ell[j] - a.alpha * m : -INFINITY;
    }
  } else {
    // every lane needs the whole S of its node
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
      const float* th = sm.theta + (sub * LG + j) * LS;
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < KMAX; ++k) acc = fmaf(th[k], Sa[k], acc);
      const float m = uu[j] + acc;
      mm[j] = m;
      const float zz = one_minus_alpha * ell[j] - a.alpha * m;
      z[j] = valid[j] ? zz : -INFINITY;
    }
  }
  if constexpr (RULE != MF_RULE_FIXED) {
    rule_epilogue<LG, CONN, RULE>(a, *rx, valid, ell, mm, z, base, N, n, x, y, L);
    return;
  }

  float mx = z[0];
#pragma unroll
  for (int j = 1; j < LG; ++j) mx = fmaxf(mx, z[j]);
  mx = group_max<LPN>(mx);
  float se = 0.f;
#pragma unroll
  for (int j = 0; j < LG; ++j) se += __expf(z[j] - mx);   // exp(-inf) = 0 for empty slots
  se = group_sum<LPN>(se);
  const float lse = mx + __logf(se);
  const __amdgpu_buffer_rsrc_t ro = planes_rsrc(a.state_out + base, pbytes);
#pragma unroll
  for (int j = 0; j < LG; ++j) {
    const int l = sub * LG + j;
    if (valid[j]) {
      if constexpr (LPN == 1) buf_store<kUAux>(z[j] - lse, ro, n * 4u, (unsigned)j * N * 4u);
      else buf_store<kUAux>(z[j] - lse, ro, ((unsigned)l * N + n) * 4u, 0u);
    }
  }
}

// Workgroups are dealt to the eight XCDs round-robin (workgroup w runs on
// XCD w mod 8), and each XCD has its own L2.  Tile t = (x, y, b) in
// row-major order is given to workgroup w so that XCD k takes the k-th
// contiguous run of tiles: horizontally and vertically adjacent tiles then
// share an L2, and the halo rows and the cache lines of the side halo
// columns that a tile reads are the lines its neighbours read.
constexpr int kXcds = 8;

__device__ inline int xcd_tile(int w, int total) {
  const int q = total / kXcds, r = total - q * kXcds;
  const int x = w % kXcds;
  return x * q + (x < r ? x : r) + w / kXcds;
}

template <int LG, int LPN, int LC, int CONN, int COMPAT, int PREC, int TX, int TY, bool STREAM>
__global__ __launch_bounds__(TX * TY * LPN) void step_kernel(StepArgs a, float one_minus_alpha) {
  __shared__ Smem<LG, LPN, TX, TY, PREC> sm;
  const int tiles_x = (a.W + TX - 1) / TX, tiles_y = (a.H + TY - 1) / TY;
  const int t = xcd_tile(blockIdx.x, tiles_x * tiles_y * a.B);
  const int per_item = tiles_x * tiles_y;
  const int b = t / per_item;
  const int r = t - b * per_item;
  const int ty = r / tiles_x, tx = r - ty * tiles_x;
  tile_step<LG, LPN, LC, CONN, COMPAT, PREC, TX, TY, MF_RULE_FIXED, STREAM>(a, one_minus_alpha, b, tx * TX, ty * TY,
                                                                            sm);
}

// Many independent problems in one launch: slot k owns tiles
// [tile_begin[k], tile_begin[k + 1]).  Tiles are dealt to workgroups XCD by
// XCD as in step_kernel (adjacent tiles of a problem share an L2), and the
// slot of a tile is found by binary search over tile_begin.
template <int LG, int LPN, int LC, int CONN, int COMPAT, int PREC, int TX, int TY>
__global__ __launch_bounds__(TX * TY * LPN) void step_many_kernel(ManyArgs m) {
  __shared__ Smem<LG, LPN, TX, TY, PREC> sm;
  const int blk = xcd_tile(blockIdx.x, m.tile_begin[m.count]);
  int k = 0, hi = m.count - 1;            // the last slot with tile_begin <= blk
  while (k < hi) {
    const int mid = (k + hi + 1) >> 1;
    if (m.tile_begin[mid] <= blk) k = mid;
    else hi = mid - 1;
  }
  const int t = blk - m.tile_begin[k];
  const int tiles_x = (m.slot[k].W + TX - 1) / TX;
  const int tiles_per_item = tiles_x * ((m.slot[k].H + TY - 1) / TY);
  const int b = t / tiles_per_item;
  const int r = t - b * tiles_per_item;
  const int ty = r / tiles_x, tx = r - (r / tiles_x) * tiles_x;
  tile_step<LG, LPN, LC, CONN, COMPAT, PREC, TX, TY>(m.slot[k], m.one_minus_alpha[k], b, tx * TX, ty * TY, sm);
}

// Single-step kernels run one lane per node (LPN = 1), the launch helpers
// below taking 64 x 4 as the base tile (see ForPrec::one for the shapes
// launched): of the label splits measured on the 256 x 256, L = 21 grid (1, 2 and 4 lanes
// per node, 64 x 4 / 32 x 4 / 16 x 4 / 16 x 8 tiles) all took 10-13 us per
// step there, while on the 2048 x 2048 grid one lane per node streamed
// fastest (277 us per step against 346-508 us).  The label-parallel split
// pays off in the fused multi-step kernel (grid_temporal.h) instead.  Grids
// whose arrays stream past the cache take 64 x 12 tiles: on 2048 x 2048,
// L = 21 they ran at 208 us per step against 222 us for 64 x 4 (64 x 8:
// 215, 32 x 8: 218, 128 x 4: 243, 64 x 16: 275; shapes whose wavefront
// count is not a multiple of the four SIMDs, 64 x 5 and 64 x 10, 258 and
// 320 us).  Cache-resident grids take 64 x 8 tiles: on the 16 x 128 x 128,
// L = 21 batch 18.9 us per step against 19.9 us for 64 x 4 (BF16 messages
// 17.9 against 19.4), the same on 256 x 256; the batched kernel's step
// kernels in the 512-request serving replay 0.167 s against 0.175 s.
inline int slots_for(int L) {
  return L == 2 ? 2 : L == 21 ? 21 : L <= 4 ? 4 : L <= 8 ? 8 : L <= 16 ? 16 : 32;
}

// The unaries and both state planes of one step (12 B per node-label) exceed
// the 256 MB last-level cache: nothing of them survives to the next step, so
// the step kernel streams the unaries and the new state past the cache.
constexpr size_t kLastLevelCacheBytes = (size_t)256 << 20;
inline bool streams_past_cache(const StepArgs& a) {
  return (size_t)12 * a.B * a.L * a.N > kLastLevelCacheBytes;
}

inline int tiles(int B, int H, int W, int L) {
  (void)L;
  return B * ((W + 63) / 64) * ((H + 7) / 8);
}

hipError_t launch_f32(const StepArgs& a, int conn, int compat, hipStream_t s);
hipError_t launch_bf16(const StepArgs& a, int conn, int compat, hipStream_t s);
hipError_t launch_f16(const StepArgs& a, int conn, int compat, hipStream_t s);
hipError_t launch_many_f32(const ManyArgs& m, int L, int conn, int compat, hipStream_t s);
hipError_t launch_many_bf16(const ManyArgs& m, int L, int conn, int compat, hipStream_t s);
hipError_t launch_many_f16(const ManyArgs& m, int L, int conn, int compat, hipStream_t s);

// Instantiation helper used by the per-precision translation units.
template <int PREC>
struct ForPrec {
  template <int LG, int LPN, int LC, int TX, int TY, bool STREAM>
  static hipError_t one_s(const StepArgs& a, int conn, int compat, hipStream_t s) {
    // one-dimensional grid: step_kernel maps workgroups to tiles XCD by XCD
    dim3 grid(((a.W + TX - 1) / TX) * ((a.H + TY - 1) / TY) * a.B);
    dim3 block(TX * TY * LPN);
    const float om = (float)(1.0 - (double)a.alpha);
    if (conn == 4) {
      if (compat == MF_COMPAT_POTTS)
        hipLaunchKernelGGL((step_kernel<LG, LPN, LC, 4, MF_COMPAT_POTTS, PREC, TX, TY, STREAM>), grid, block, 0, s, a, om);
      else
        hipLaunchKernelGGL((step_kernel<LG, LPN, LC, 4, MF_COMPAT_GENERAL, PREC, TX, TY, STREAM>), grid, block, 0, s, a,
                           om);
    } else {
      if (compat == MF_COMPAT_POTTS)
        hipLaunchKernelGGL((step_kernel<LG, LPN, LC, 8, MF_COMPAT_POTTS, PREC, TX, TY, STREAM>), grid, block, 0, s, a, om);
      else
        hipLaunchKernelGGL((step_kernel<LG, LPN, LC, 8, MF_COMPAT_GENERAL, PREC, TX, TY, STREAM>), grid, block, 0, s, a,
                           om);
    }
    return hipGetLastError();
  }
  // Single-step launches take 64 x 12 tiles when streaming (twelve
  // wavefronts, two workgroups and six wavefronts per SIMD at L = 21 where
  // 64 x 4 fits four and four), 64 x 8 otherwise (half the halo rows per node
  // of 64 x 4 at the same occupancy), as the batched kernel does.
  template <int LG, int LPN, int LC, int TX, int TY>
  static hipError_t one(const StepArgs& a, int conn, int compat, hipStream_t s) {
    return streams_past_cache(a) ? one_s<LG, LPN, LC, TX, 3 * TY, true>(a, conn, compat, s)
                                 : one_s<LG, LPN, LC, TX, 2 * TY, false>(a, conn, compat, s);
  }
  template <int LG, int LPN, int LC, int TX, int TY>
  static hipError_t many(const ManyArgs& m, int conn, int compat, hipStream_t s) {
    const int total = m.tile_begin[m.count];
    if (total <= 0) return hipSuccess;
    dim3 block(TX * TY * LPN);
    if (conn == 4) {
      if (compat == MF_COMPAT_POTTS)
        hipLaunchKernelGGL((step_many_kernel<LG, LPN, LC, 4, MF_COMPAT_POTTS, PREC, TX, TY>), dim3(total), block, 0, s, m);
      else
        hipLaunchKernelGGL((step_many_kernel<LG, LPN, LC, 4, MF_COMPAT_GENERAL, PREC, TX, TY>), dim3(total), block, 0, s, m);
    } else {
      if (compat == MF_COMPAT_POTTS)
        hipLaunchKernelGGL((step_many_kernel<LG, LPN, LC, 8, MF_COMPAT_POTTS, PREC, TX, TY>), dim3(total), block, 0, s, m);
      else
        hipLaunchKernelGGL((step_many_kernel<LG, LPN, LC, 8, MF_COMPAT_GENERAL, PREC, TX, TY>), dim3(total), block, 0, s, m);
    }
    return hipGetLastError();
  }
  // L = 2 and L = 21 (the label counts of the benchmark workloads) are
  // compiled for their exact count; other counts use the next slot size.
  static hipError_t launch(const StepArgs& a, int conn, int compat, hipStream_t s) {
    switch (slots_for(a.L)) {
      case 2: return a.L == 2 ? one<2, 1, 2, 64, 4>(a, conn, compat, s) : one<2, 1, 0, 64, 4>(a, conn, compat, s);
      case 21: return one<21, 1, 21, 64, 4>(a, conn, compat, s);
      case 4: return one<4, 1, 0, 64, 4>(a, conn, compat, s);
      case 8: return one<8, 1, 0, 64, 4>(a, conn, compat, s);
      case 16: return one<16, 1, 0, 64, 4>(a, conn, compat, s);
      default: return one<32, 1, 0, 64, 4>(a, conn, compat, s);
    }
  }
  static hipError_t launch_many(const ManyArgs& m, int L, int conn, int compat, hipStream_t s) {
    switch (slots_for(L)) {
      case 2: return L == 2 ? many<2, 1, 2, 64, 8>(m, conn, compat, s) : many<2, 1, 0, 64, 8>(m, conn, compat, s);
      case 21: return many<21, 1, 21, 64, 8>(m, conn, compat, s);
      case 4: return many<4, 1, 0, 64, 8>(m, conn, compat, s);
      case 8: return many<8, 1, 0, 64, 8>(m, conn, compat, s);
      case 16: return many<16, 1, 0, 64, 8>(m, conn, compat, s);
      default: return many<32, 1, 0, 64, 8>(m, conn, compat, s);
    }
  }
};

}  // namespace lanes
}  // namespace mf
