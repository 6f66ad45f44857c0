// Every step of a solve in one launch on a small grid: one resident
// workgroup per 16 x 16 tile, the one-node halo exchanged through global
// memory after each step.
//
// Step (Eq. 15 with the fixed step of Eq. 16, Sec. 3.1-3.2), per node i:
//   S_i = sum of q_j over the 4 / 8 grid neighbours (free boundary)
//   m_i = u_i + Theta S_i
//   z_i = (1 - alpha) log q_i - alpha m_i;   log q_i <- z_i - lse(z_i)
// The Jacobi update of Sec. 2.2.2: every node reads its neighbours at the
// previous iterate.
//
// A workgroup of 16 wavefronts owns one tile for the whole launch.  Its
// log q and unaries stay in registers (wavefront w always updates the same
// 16 nodes, four lanes per node, Theta S on the FP32 matrix cores with the
// lane layout of the fused multi-step kernel), q of the tile and of its
// one-node halo sits in LDS, double-buffered.  Wavefronts 0-3 own the 60
// nodes of the tile's boundary ring (15 each, the four sides taken as
// quarter turns of the top row) plus one inner node; wavefronts 4-15 own
// the other 192 inner nodes, which read only the tile itself and never
// wait.
//
// Halo exchange.  After each step the ring wavefronts publish q of their
// ring nodes, one 64-bit word per node-label: the step's tag in the high
// half, the value in the low half, written with an agent-scope atomic store
// into one of two slots per tile (by step parity).  Before the next step a
// ring wavefront reads, with agent-scope atomic loads, exactly the halo
// cells its own nodes' stencils need and re-reads those whose tag is not yet
// the expected one.  A word is written and read whole, so a matching tag
// carries its own value: no fence, flag or cache maintenance.  The need is
// mutual (a halo cell's node has this tile's node in its own stencil), so a
// producer cannot publish step t + 2 into a slot before every reader of
// step t in that slot has read it.  Tags are per launch (a base the host
// advances past every tag it has used), so no word of an earlier launch
// matches.  Every wait is bounded (20 ms of the constant 100 MHz clock;
// the environment variable MF_PERSIST_WAIT_US sets another bound): a
// wavefront that gives up sets bit 2 of the handle's flags and stops
// waiting for the rest of the launch, so every workgroup finishes.
// Persistent launches of one process on one device are serialised across
// streams (an event recorded after each), so two never share the compute
// units.  The
// host launches it only when the occupancy query says every tile's
// workgroup fits on the device at once (at 256 tiles: one per compute
// unit).  Workgroups of kernels running beside it on other streams can
// still hold compute units for a while; a tile that starts late only delays
// its neighbours, unless it starts more than 20 ms late: then the waits give
// up and the flag reports it.  (A cooperative launch, which would have the
// runtime guarantee residency, measured 20 us slower per launch.)
//
// Arithmetic per node is that of the fused kernel, so with the same launch
// boundaries the iterates match the fused kernel's bitwise (neighbours' q
// arrive as the exact values their owners computed).  A launch may also
// take the initialisation and the write-out of q, with the arithmetic of
// the separate kernels, so that a solve is one launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdlib>
#include <mutex>

#include "grid_temporal.h"
#include "mf_internal.h"
#include "msg_codec.h"

namespace mf {
namespace persist {

constexpr int kT = 16;                    // tile side
constexpr int kR = kT + 2;                // region side: the tile and one node either side
constexpr int kRA = kR * kR;              // region nodes
constexpr int kRingW = 64;                // exchange words per label plane, slot and tile (60 ring nodes)
constexpr int kNT = 1024;                 // 16 wavefronts, one 16-node task each
constexpr long long kWaitUs = 20000;     // default bound of one halo wait (20 ms)

struct ExchangeArgs {
  uint64_t* xch;       // [tiles][2][L][kRingW] tagged words
  unsigned tag0;       // tag of q^0 in this launch; step s publishes tag0 + s
  int ks;              // steps in this launch
  int* flags;          // bit 0: a non-finite input (with init >= 0); bit 2: a halo wait gave up
  int init;            // mf_init_mode applied to the state first, or -1 (the state is initialised)
  float* q_out;        // [B][L][N] q = exp(log q) of the last step, or nullptr
  long long wait_ticks;  // bound of one halo wait, ticks of the 100 MHz constant clock
};

// k quarter turns clockwise inside the tile: (y, x) -> (x, 15 - y); also
// for the halo coordinates -1 and 16.
__device__ inline void rot(int k, int& y, int& x) {
  for (int i = 0; i < k; ++i) {
    const int t = y;
    y = x;
    x = kT - 1 - t;
  }
}

// Position of a ring node in its tile's exchange plane: the top row
// (x < 15), the right column (y < 15), the bottom row (x > 0), the left
// column (y > 0), each 15 nodes in the order of the ring wavefront's lanes.
__device__ inline int ring_index(int y, int x) {
  if (y == 0 && x < kT - 1) return x;
  if (x == kT - 1 && y < kT - 1) return 15 + y;
  if (y == kT - 1 && x > 0) return 30 + (kT - 1 - x);
  return 45 + (kT - 1 - y);
}

template <int LG, int LC, int CONN, int PREC>
__global__ __launch_bounds__(kNT) void persist_kernel(StepArgs a, ExchangeArgs x, float one_minus_alpha) {
  using M = MsgT<PREC>;
  constexpr int LP = 4 * LG;
  constexpr int NOB = (LG + 3) / 4;
  constexpr int RN = temporal::mfma_plane_stride(kRA);
  constexpr int NH = CONN == 8 ? 19 : 16;           // halo cells a ring wavefront reads
  constexpr int NF = (NH * LP + 63) / 64;           // (cell, label) pairs per lane
  // q in LDS as FP32 values of the message type (16-bit messages decoded on
  // write): the stencil reads full dwords whatever the message precision
  __shared__ float qs[2][LP * RN];

  const int L = LC > 0 ? LC : a.L;
  const unsigned N = (unsigned)a.N;
  const int H = a.H, W = a.W;
  const int tiles_x = (W + kT - 1) / kT, tiles_y = (H + kT - 1) / kT;
  const int tile = lanes::xcd_tile(blockIdx.x, tiles_x * tiles_y * a.B);
  const int b = tile / (tiles_x * tiles_y);
  const int tr = tile - b * (tiles_x * tiles_y);
  const int tyi = tr / tiles_x, txi = tr - tyi * tiles_x;
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

  // This lane's node: ring wavefronts take the ring (lanes 0-14) and one of
  // the four last inner nodes (lane 15); the others take 16 inner nodes.
  int ny = 0, nx = col;
  if (wave < 4 && col < 15) {
    rot(wave, ny, nx);
  } else {
    const int i = wave < 4 ? 192 + wave : (wave - 4) * 16 + col;
    ny = 1 + i / 14;
    nx = 1 + i % 14;
  }
  const int gy = tyi * kT + ny, gx = txi * kT + nx;
  const bool act = gy < H && gx < W;
  const bool ring = wave < 4 && col < 15 && act;
  const unsigned n = act ? (unsigned)(gy * W + gx) : 0u;
  const int cc = (ny + 1) * kR + nx + 1;
  const int cb = g * RN + cc;                       // plane g at this node
  bool valid[LG];
#pragma unroll
  for (int j = 0; j < LG; ++j) valid[j] = (LC > 0 && 4 * j + 3 < LC) || g + 4 * j < L;
  // this tile's exchange area (both slots); a ring lane's node sits at
  // position 15 wave + col of each label plane
  uint64_t* __restrict__ my_x = x.xch + (size_t)tile * 2 * L * kRingW;
  const unsigned rpos = ring ? (unsigned)(15 * wave + col) : 0u;

  // The node's log q and unaries (loads first: the LDS clear runs under them)
  float ell[LG], uu[LG];
#pragma unroll
  for (int j = 0; j < LG; ++j) {
    const unsigned off = ((unsigned)(valid[j] ? g + 4 * j : L - 1) * N + n) * 4u;
    ell[j] = temporal::load_at(lin, off);
    uu[j] = temporal::load_at(ug, off);
  }
  // with the initialisation from the unaries: this lane's group of LG
  // consecutive labels g LG .. g LG + LG - 1
  float ug4[LG];
  if (x.init == MF_INIT_UNARY) {
#pragma unroll
    for (int j = 0; j < LG; ++j) {
      const int l = g * LG + j;
      ug4[j] = temporal::load_at(ug, ((unsigned)(l < L ? l : 0) * N + n) * 4u);
    }
  }

  // Both q buffers start at zero: off-grid halo cells, nodes past the
  // grid's edge and padding label slots stay q = 0.
  for (int f = tid; f < 2 * LP * RN; f += kNT) (&qs[0][0])[f] = 0.f;

  if (x.init >= 0) {
    // log q^0 as the initialisation kernel forms it (Eq. 6 reading
    // q^0 = softmax(-u), or uniform, or the given state): four label groups
    // of LG consecutive labels, one per lane of the node, each with its own
    // max and its own sum in label order; the maxima combined, the sums as
    // (s0 + s2) + (s1 + s3), the same bits in every lane of the node
    bool bad = false;
#pragma unroll
    for (int j = 0; j < LG; ++j) {
      if (valid[j]) bad |= !isfinite(uu[j]);
      if (valid[j] && x.init == MF_INIT_STATE) bad |= !isfinite(ell[j]);
    }
    if (x.init == MF_INIT_UNARY) {
      float mx = -INFINITY;
#pragma unroll
      for (int j = 0; j < LG; ++j) mx = fmaxf(mx, g * LG + j < L ? -ug4[j] : -INFINITY);
      mx = temporal::rows_max(mx);
      float sg = 0.f;
#pragma unroll
      for (int j = 0; j < LG; ++j) sg += g * LG + j < L ? expf(-ug4[j] - mx) : 0.f;
      // rows g and g ^ 2 first (the two half-waves), then the two pairs
      const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(sg), __float_as_uint(sg), false, false);
      sg = __uint_as_float(r[0]) + __uint_as_float(r[1]);
      const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(sg), __float_as_uint(sg), false, false);
      sg = __uint_as_float(p[0]) + __uint_as_float(p[1]);
      const float lse = mx + logf(sg);
#pragma unroll
      for (int j = 0; j < LG; ++j) ell[j] = -uu[j] - lse;
    } else if (x.init == MF_INIT_UNIFORM) {
      const float u0 = -logf((float)a.L);   // the run-time count: the initialisation kernel's device logf
#pragma unroll
      for (int j = 0; j < LG; ++j) ell[j] = u0;
    }
    if (act && bad) atomicOr(x.flags, 1);
  }
  __syncthreads();                                  // buffers cleared
  if (act) {
#pragma unroll
    for (int j = 0; j < LG; ++j) {
      if (valid[j]) {
        const float e = M::dec(M::enc(__expf(ell[j])));
        qs[0][cb + 4 * j * RN] = e;
        if (ring) {
          const uint64_t w = ((uint64_t)x.tag0 << 32) | __float_as_uint(e);
          __hip_atomic_store(my_x + (unsigned)((g + 4 * j) * kRingW) + rpos, w, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  }

  // Halo pairs of a ring wavefront: pair p = lane + 64 it is cell p % NH of
  // label p / NH.  Cells are quarter turns of the top row's list:
  // 8 neighbours: (-1, -1 .. 15), (0, -1), (1, -1); 4 neighbours:
  // (-1, 0 .. 14), (0, -1).  Off-grid cells are not read (q = 0).
  unsigned woff[NF], loff[NF];
  unsigned fetch = 0;
  if (wave < 4) {
#pragma unroll
    for (int it = 0; it < NF; ++it) {
      const int p = lane + 64 * it;
      const int c = p % NH, l = p / NH;
      int hy, hx;
      if (CONN == 8) {
        hy = c < 17 ? -1 : c - 17;
        hx = c < 17 ? c - 1 : -1;
      } else {
        hy = c < 15 ? -1 : 0;
        hx = c < 15 ? c : -1;
      }
      rot(wave, hy, hx);
      const int ghy = tyi * kT + hy, ghx = txi * kT + hx;
      const bool on = l < L && ghy >= 0 && ghy < H && ghx >= 0 && ghx < W;
      const int ptile = on ? (b * tiles_y + (ghy >> 4)) * tiles_x + (ghx >> 4) : 0;
      const int r = on ? ring_index(ghy & (kT - 1), ghx & (kT - 1)) : 0;
      woff[it] = ((unsigned)ptile * 2u * (unsigned)L + (unsigned)(on ? l : 0)) * kRingW + (unsigned)r;
      loff[it] = (unsigned)((on ? l : 0) * RN + (hy + 1) * kR + hx + 1);
      fetch |= on ? 1u << it : 0u;
    }
  }
  __syncthreads();                                  // q^0 of the tile in LDS

  bool aborted = false;
  for (int s = 0; s < x.ks; ++s) {
    const int cur = s & 1;
    float* __restrict__ qc = qs[cur];
    float* __restrict__ qn = qs[cur ^ 1];
    if (wave < 4) {
      // the halo of step s: words of slot s % 2 tagged tag0 + s
      const unsigned expect = x.tag0 + (unsigned)s;
      const unsigned slot = (unsigned)(cur * L * kRingW);
      unsigned pend = fetch;
      const long long t0 = wall_clock64();
      while (true) {
        uint64_t w[NF];
#pragma unroll
        for (int it = 0; it < NF; ++it)
          if ((pend >> it) & 1u)
            w[it] = __hip_atomic_load(x.xch + woff[it] + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int it = 0; it < NF; ++it) {
          if (((pend >> it) & 1u) && (unsigned)(w[it] >> 32) == expect) {
            qc[loff[it]] = __uint_as_float((unsigned)w[it]);
            pend &= ~(1u << it);
          }
        }
        if (!__any(pend != 0u)) break;
        if (aborted || wall_clock64() - t0 > x.wait_ticks) {
          if (!aborted && lane == 0) atomicOr(x.flags, 4);
          aborted = true;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      // this wavefront's LDS writes above come before its reads below
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }

    // LDS byte address of plane g at region offset - kR - 1 of this node
    const unsigned qb = temporal::lds_addr(qc) + (unsigned)(cb - kR - 1) * 4u;
    float S[LG];
#pragma unroll
    for (int j = 0; j < LG; ++j) {
      const float* qp = temporal::lds_ptr<float>(temporal::opaque(qb + (unsigned)(4 * j * RN) * 4u));
      const float n0 = qp[1], w0 = qp[kR], e0 = qp[kR + 2], s0 = qp[2 * kR + 1];
      float tot = (n0 + w0) + (e0 + s0);
      if (CONN == 8) tot += (qp[0] + qp[2]) + (qp[2 * kR] + qp[2 * kR + 2]);
      S[j] = valid[j] ? tot : 0.f;
    }

    temporal::f32x4 acc[NOB];
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob) acc[ob] = temporal::f32x4{0.f, 0.f, 0.f, 0.f};
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
    mx = temporal::rows_max(mx);
    float e[LG];
#pragma unroll
    for (int j = 0; j < LG; ++j) e[j] = __expf(z[j] - mx);   // exp(-inf) = 0 for empty slots
    float se = e[0];
#pragma unroll
    for (int j = 1; j < LG; ++j) se += e[j];
    se = temporal::rows_sum(se);
    const float lse = mx + __logf(se);
    const float inv = __builtin_amdgcn_rcpf(se);   // 1 ulp; se >= 1 (the max term is exp(0))
    const unsigned tag = x.tag0 + (unsigned)s + 1u;
    const unsigned nslot = (unsigned)((cur ^ 1) * L * kRingW);
#pragma unroll
    for (int j = 0; j < LG; ++j) {
      ell[j] = z[j] - lse;
      if (act && valid[j]) {
        const float qv = M::dec(M::enc(e[j] * inv));
        qn[cb + 4 * j * RN] = qv;
        if (ring) {
          const uint64_t w = ((uint64_t)tag << 32) | __float_as_uint(qv);
          __hip_atomic_store(my_x + nslot + (unsigned)((g + 4 * j) * kRingW) + rpos, w, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    __syncthreads();
  }

  // log q of the last step, and q as the separate write-out forms it
  float* __restrict__ out = a.state_out + base;
  if (act) {
#pragma unroll
    for (int j = 0; j < LG; ++j) {
      if (valid[j]) {
        out[(unsigned)(g + 4 * j) * N + n] = ell[j];
        if (x.q_out) x.q_out[base + (size_t)(g + 4 * j) * N + n] = expf(ell[j]);
      }
    }
  }
}

// Workgroups of one instantiation resident per compute unit (queried once
// per device).
template <int LG, int LC, int CONN, int PREC>
int resident_per_cu() {
  static int cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (!cached[dev]) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, persist_kernel<LG, LC, CONN, PREC>, kNT, 0) != hipSuccess)
      n = 0;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
    cached[dev] = n * cus;
    if (cached[dev] == 0) cached[dev] = -1;
  }
  return cached[dev] > 0 ? cached[dev] : 0;
}

template <int LG, int LC, int CONN, int PREC>
hipError_t go(const StepArgs& a, const ExchangeArgs& x, hipStream_t s, bool query, int* capacity) {
  if (query) {
    *capacity = resident_per_cu<LG, LC, CONN, PREC>();
    return hipSuccess;
  }
  const int tiles = ((a.W + kT - 1) / kT) * ((a.H + kT - 1) / kT) * a.B;
  const float om = (float)(1.0 - (double)a.alpha);
  hipLaunchKernelGGL((persist_kernel<LG, LC, CONN, PREC>), dim3(tiles), dim3(kNT), 0, s, a, x, om);
  return hipGetLastError();
}

template <int PREC>
hipError_t by_labels(const StepArgs& a, int conn, const ExchangeArgs& x, hipStream_t s, bool query, int* cap) {
  const int L = a.L;
  if (conn == 4) {
    if (L <= 16) return go<4, 0, 4, PREC>(a, x, s, query, cap);
    if (L == 21) return go<6, 21, 4, PREC>(a, x, s, query, cap);
    if (L <= 24) return go<6, 0, 4, PREC>(a, x, s, query, cap);
    return go<8, 0, 4, PREC>(a, x, s, query, cap);
  }
  if (L <= 16) return go<4, 0, 8, PREC>(a, x, s, query, cap);
  if (L == 21) return go<6, 21, 8, PREC>(a, x, s, query, cap);
  if (L <= 24) return go<6, 0, 8, PREC>(a, x, s, query, cap);
  return go<8, 0, 8, PREC>(a, x, s, query, cap);
}

hipError_t dispatch(const StepArgs& a, int conn, int precision, const ExchangeArgs& x, hipStream_t s, bool query,
                    int* cap) {
  switch (precision) {
    case MF_P_F32: return by_labels<P_F32>(a, conn, x, s, query, cap);
    case MF_P_BF16MSG: return by_labels<P_BF16>(a, conn, x, s, query, cap);
    default: return by_labels<P_F16>(a, conn, x, s, query, cap);
  }
}

}  // namespace persist

bool grid_persist_eligible(int L, int compat) { return compat == MF_COMPAT_GENERAL && L > 8 && L <= 32; }

size_t grid_persist_exchange_bytes(int B, int H, int W, int L) {
  const size_t tiles = (size_t)B * ((W + persist::kT - 1) / persist::kT) * ((H + persist::kT - 1) / persist::kT);
  return tiles * 2 * (size_t)L * persist::kRingW * sizeof(uint64_t);
}

int grid_persist_capacity(int L, int conn, int precision) {
  StepArgs a{};
  a.L = L;
  persist::ExchangeArgs x{};
  int cap = 0;
  if (persist::dispatch(a, conn, precision, x, nullptr, true, &cap) != hipSuccess) return 0;
  return cap;
}

hipError_t launch_grid_persist(const StepArgs& a, int conn, int precision, uint64_t* xch, unsigned tag0, int ks,
                               int* flags, int init, float* q_out, hipStream_t s) {
  persist::ExchangeArgs x;
  x.xch = xch;
  x.tag0 = tag0;
  x.ks = ks;
  x.flags = flags;
  x.init = init;
  x.q_out = q_out;
  // MF_PERSIST_WAIT_US overrides the bound of one halo wait (diagnostics:
  // 0 makes every wait that finds a tag not yet written give up)
  long long us = persist::kWaitUs;
  if (const char* v = std::getenv("MF_PERSIST_WAIT_US")) {
    char* end = nullptr;
    const long long w = std::strtoll(v, &end, 10);
    if (end != v && w >= 0) us = w;
  }
  x.wait_ticks = us * 100;
  // Persistent launches of this process on one device run one after
  // another, whatever their streams: two of them sharing the compute units
  // would each wait for tiles the other keeps from starting.
  static std::mutex mu;
  static hipEvent_t last_ev[64] = {};
  static hipStream_t last_stream[64] = {};
  static bool have[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  // (A stream under graph capture takes no part: the graph's own order applies.)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &cs);
  if (e != hipSuccess) return e;
  int cap = 0;
  if (cs != hipStreamCaptureStatusNone) return persist::dispatch(a, conn, precision, x, s, false, &cap);
  std::lock_guard<std::mutex> lock(mu);
  if (!last_ev[dev]) e = hipEventCreateWithFlags(&last_ev[dev], hipEventDisableTiming);
  if (e == hipSuccess && have[dev] && last_stream[dev] != s) e = hipStreamWaitEvent(s, last_ev[dev], 0);
  if (e == hipSuccess) e = persist::dispatch(a, conn, precision, x, s, false, &cap);
  if (e == hipSuccess) e = hipEventRecord(last_ev[dev], s);
  if (e == hipSuccess) {
    have[dev] = true;
    last_stream[dev] = s;
  }
  return e;
}

}  // namespace mf
