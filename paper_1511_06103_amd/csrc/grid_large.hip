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
// A tile is 64 consecutive nodes of one grid row.  A workgroup has one
// wavefront per block of 16 output labels (L rounded up to 64 or 128) and
// half tile, 8 or 16 wavefronts, stays resident for the whole launch and
// works through its tiles one after another; each wavefront keeps its 16
// rows of Theta in registers throughout.  The labels of a tile are taken in
// chunks of 32, one pipeline stage per chunk: a stage multiplies the S chunk
// formed in the stage before by the matching columns of the wavefronts'
// Theta rows into their accumulators, forms the next chunk's S (sums over
// the neighbours of q = exp(log q) staged in LDS for the tile's three rows,
// the row and its neighbours above and below, 66 nodes each, off-grid
// q = 0), and stages the q of the chunk after that from registers loaded
// one or two stages earlier.  S, staged q and the tile's own log q (the
// middle row, kept for the step's epilogue) are double-buffered in LDS, so
// a stage needs one barrier.  The last stage of a tile also runs the
// epilogue: the per-node log-sum-exp over the accumulators of all
// wavefronts, a max and a sum inside each (lanes x, x ^ 16, x ^ 32, x ^ 48
// with the gfx950 row-swap permutes), combined across wavefronts through
// LDS.
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
constexpr int kKC = 32;             // labels per chunk
constexpr int kRW = kTN + 2;        // region row: the tile and one node either side
constexpr int kRP = 3 * kRW;        // region nodes per label plane (three rows)
constexpr int kRegion = kKC * kRP;  // staged q values per chunk

constexpr int kSegs = kKC * 3;     // (label, row) segments of a chunk's region

// Wavefronts: one per block of 16 output labels and half tile (32 nodes),
// 2 LP / 16 in all; one workgroup per compute unit.
template <int LP>
struct Geo {
  static constexpr int NOB = LP / 16;        // output label blocks
  static constexpr int NW = 2 * NOB;         // wavefronts per workgroup
  static constexpr int NT = 64 * NW;
  static constexpr int SEGS = kSegs / NW;    // region segments staged per wavefront
  static constexpr int WAVES_PER_SIMD = NW / 4;
  // stages between issuing a chunk's loads and staging it: two where the
  // registers allow (LP = 64, two waves per SIMD), one at LP = 128
  static constexpr int AHEAD = LP == 64 ? 2 : 1;
};

// One chunk's region in registers: the 64 tile columns of SEGS segments
// (lane = column) and one of the 2 x 96 edge columns (threads < 192).
template <int LP>
struct Region {
  float v[Geo<LP>::SEGS];
  float edge;
};

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

// The work of a workgroup is a sequence of stages, one per (tile, chunk)
// pair: stage k is chunk k % NC of the workgroup's tile k / NC.  Stage k
// multiplies the S chunk of stage k (ss[k % 2]) into the accumulators, forms
// the S chunk of stage k + 1 from its staged q (qs[(k + 1) % 2]), stages the
// q of stage k + 2 (qs[k % 2]) from registers loaded one stage earlier, and
// issues the loads of stage k + 3; the last stage of a tile also runs the
// step's epilogue.  The buffers that a stage writes are the ones no other
// wavefront reads in that stage, so one barrier per stage orders it all.
template <int LP, int CONN, int PREC, bool STREAM>
__global__ __launch_bounds__(Geo<LP>::NT)
__attribute__((amdgpu_waves_per_eu(Geo<LP>::WAVES_PER_SIMD, Geo<LP>::WAVES_PER_SIMD)))
void large_step_kernel(StepArgs a, float one_minus_alpha, int potts) {
  using M = MsgT<PREC>;
  using T = typename M::T;
  constexpr bool F32 = PREC == P_F32;
  constexpr int NOB = Geo<LP>::NOB, NW = Geo<LP>::NW, SEGS = Geo<LP>::SEGS;
  constexpr int NC = LP / kKC;       // label chunks (stages) per tile: 2 or 4
  constexpr int NNB = 2;             // node blocks of 16 per wavefront (half a tile)
  constexpr int SST = s_stride<PREC>();
  constexpr int LS = kTN + 4;        // row stride of the own-row log q: rows 4 g + i on disjoint banks
  constexpr int D = Geo<LP>::AHEAD;  // stages of load prefetch
  static_assert(NC % 2 == 0, "stage parity follows the chunk index");
  __shared__ T qs[2][kRegion];
  __shared__ float ss[2][kKC * SST];
  __shared__ float ls[2][LP * LS];
  __shared__ float red_m[NOB][kTN], red_s[NOB][kTN];

  const int L = a.L;
  const unsigned N = (unsigned)a.N;
  const int H = a.H, W = a.W;
  const int tiles_x = (W + kTN - 1) / kTN;
  const int total = tiles_x * H * a.B;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ob = wave % NOB;         // output labels 16 ob .. 16 ob + 15
  const int half = wave / NOB;       // tile nodes 32 half .. 32 half + 31
  const int c = lane & 15, g = lane >> 4;
  if ((int)blockIdx.x >= total) return;
  // tiles of this workgroup: blockIdx.x + j gridDim.x, j < n_tiles
  const int n_tiles = (total - (int)blockIdx.x + (int)gridDim.x - 1) / (int)gridDim.x;

  // Theta rows of this wavefront's output block (label 16 ob + c), held for
  // every tile of the launch; zero outside L x L; Potts builds w (1 1^T - I).
  // Every lane loads (no divergent branch around the loads); with Potts
  // (theta may be NULL) the load reads the unaries' first element instead.
  const int trow = 16 * ob + c;
  const float* thp = potts ? a.unary : a.theta;
  auto theta_at = [&](int col) -> float {
    const bool ok = trow < L && col < L;
    const float t = thp[(ok && !potts) ? trow * L + col : 0];
    return !ok ? 0.f : potts ? (trow == col ? 0.f : a.potts_w) : t;
  };
  float tha[F32 ? LP / 4 : 1];
  bf16x8 thh[F32 ? 1 : NC], thl[F32 ? 1 : NC];
  if constexpr (F32) {
    // A of k-step kb: Theta[row][4 kb + g]
#pragma unroll
    for (int kb = 0; kb < LP / 4; ++kb) tha[kb] = theta_at(4 * kb + g);
  } else {
    // A of chunk kc: Theta[row][32 kc + 8 g + e], e < 8
#pragma unroll
    for (int kc = 0; kc < NC; ++kc) {
      float t[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) t[e] = theta_at(kKC * kc + 8 * g + e);
      split8(t, thh[kc], thl[kc]);
    }
  }

  // Tile j of this workgroup: tiles are dealt XCD by XCD (lanes::xcd_tile);
  // the grid is a multiple of 8 workgroups, so a workgroup stays on the XCD
  // range it starts in.
  struct Tile {
    int y, x0;
    const float* lin;
    const float* ug;
    float* out;
    unsigned row_n;
  };
  auto tile_of = [&](int j) {
    Tile t;
    const int tile = lanes::xcd_tile((int)blockIdx.x + j * (int)gridDim.x, total);
    const int b = tile / (tiles_x * H);
    const int tr = tile - b * (tiles_x * H);
    t.y = tr / tiles_x;
    t.x0 = (tr - t.y * tiles_x) * kTN;
    const size_t base = (size_t)b * L * N;
    t.lin = a.state_in + base;
    t.ug = a.unary + base;
    t.out = a.state_out + base;
    t.row_n = (unsigned)(t.y * W);
    return t;
  };

  // log q of chunk kc's 32 labels on the three rows y - 1, y, y + 1, nodes
  // x0 - 1 .. x0 + 64; off-grid nodes and labels >= L read as -inf (q = 0).
  // Segment s = (label kk = s / 3, row = s % 3) of the chunk goes to
  // wavefront s % NW: its (label, row) is uniform, its lanes are the 64
  // tile columns; the two edge columns of every segment go to threads
  // 0 .. 191.  Loads at 32-bit byte offsets from the tile's uniform base.
  auto load_region = [&](const Tile& t, int kc, Region<LP>& rg) {
    const int gx = t.x0 + lane;
    const bool col_ok = gx < W;
#pragma unroll
    for (int j = 0; j < SEGS; ++j) {
      const int seg = wave + NW * j;
      const int kk = seg / 3, row = seg - 3 * (seg / 3);
      const int l = kKC * kc + kk, gy = t.y + row - 1;
      const bool ok = col_ok && l < L && gy >= 0 && gy < H;
      const unsigned off = ok ? ((unsigned)l * N + (unsigned)(gy * W + gx)) * 4u : 0u;
      const float x = temporal::load_at(t.lin, off);
      rg.v[j] = ok ? x : -INFINITY;
    }
    const int e = (int)temporal::opaque((unsigned)tid);
    const int seg = e >> 1;
    const int kk = seg / 3, row = seg - 3 * (seg / 3);
    const int l = kKC * kc + kk, gy = t.y + row - 1, ex = (e & 1) ? t.x0 + kTN : t.x0 - 1;
    const bool ok = e < 2 * kSegs && l < L && gy >= 0 && gy < H && ex >= 0 && ex < W;
    const unsigned off = ok ? ((unsigned)l * N + (unsigned)(gy * W + ex)) * 4u : 0u;
    const float x = temporal::load_at(t.lin, off);
    rg.edge = ok ? x : -INFINITY;
  };
  // q to staging buffer qb, and the tile's own log q (the middle row) to lsb
  auto store_region = [&](int kc, const Region<LP>& rg, T* __restrict__ qb, float* __restrict__ lsb) {
#pragma unroll
    for (int j = 0; j < SEGS; ++j) {
      const int seg = wave + NW * j;
      const int kk = seg / 3, row = seg - 3 * (seg / 3);
      qb[kk * kRP + row * kRW + 1 + lane] = M::enc(__expf(rg.v[j]));   // exp(-inf) = 0
      if (row == 1) lsb[(kKC * kc + kk) * LS + lane] = rg.v[j];
    }
    const int e = tid;
    if (e < 2 * kSegs) {
      const int seg = e >> 1;
      const int kk = seg / 3, row = seg - 3 * (seg / 3);
      qb[kk * kRP + row * kRW + ((e & 1) ? kRW - 1 : 0)] = M::enc(__expf(rg.edge));
    }
  };
  // S of one chunk from staged q: wavefront w forms labels w + NW j, lane = node
  auto form_s = [&](const T* __restrict__ qb, float* __restrict__ sb) {
#pragma unroll
    for (int j = 0; j < kKC / NW; ++j) {
      const int kk = wave + NW * j;
      const T* q = qb + kk * kRP + lane + 1;           // row y - 1 at node lane
      float sv = M::dec(q[0]) + M::dec(q[2 * kRW]) + M::dec(q[kRW - 1]) + M::dec(q[kRW + 1]);
      if (CONN == 8) sv += (M::dec(q[-1]) + M::dec(q[1])) + (M::dec(q[2 * kRW - 1]) + M::dec(q[2 * kRW + 1]));
      sb[kk * SST + lane] = sv;
    }
  };
  // accumulator i of node block nb is label 16 ob + 4 g + i at node
  // x0 + 16 (2 half + nb) + c (clamped into the grid; masked at the store)
  auto unary_at = [&](const Tile& t, int nb, int i) -> const float* {
    const int x = t.x0 + 16 * (2 * half + nb) + c;
    const int l = 16 * ob + 4 * g + i;
    const unsigned off = ((unsigned)(l < L ? l : L - 1) * N + t.row_n + (unsigned)(x < W ? x : W - 1)) * 4u;
    return reinterpret_cast<const float*>(reinterpret_cast<const char*>(t.ug) + off);
  };

  // Prologue: q of stages 0 and 1 staged, S of stage 0 formed, and with two
  // stages of prefetch the loads of stage 2 in flight.  The loads of stage s
  // go to rv[s % D] (D divides NC, so s % D = its chunk index % D).
  Tile cur = tile_of(0);
  const bool one_tile = n_tiles == 1;
  Region<LP> rv[D];
  {
    Region<LP> t;
    load_region(cur, 0, t);
    store_region(0, t, qs[0], ls[0]);
    load_region(cur, 1, t);
    store_region(1, t, qs[1], ls[0]);
  }
  if (D == 2) {
    if (NC > 2) load_region(cur, 2, rv[0]);
    else if (!one_tile) load_region(tile_of(1), 0, rv[0]);
  }
  __syncthreads();
  form_s(qs[0], ss[0]);
  __syncthreads();

  for (int jt = 0; jt < n_tiles; ++jt) {
    const bool has_next = jt + 1 < n_tiles;
    const Tile nxt = tile_of(has_next ? jt + 1 : jt);
    const bool has_next2 = jt + 2 < n_tiles;
    f32x4 acc[NNB];
#pragma unroll
    for (int nb = 0; nb < NNB; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    float uu[NNB][4];

#pragma unroll
    for (int kc = 0; kc < NC; ++kc) {
      // stage k = jt NC + kc issues the loads of stage k + 1 + D: a later
      // chunk of this tile, or a chunk of the next tile (or, with D = 2 and
      // NC = 2, of the tile after it)
      {
        const int kl = kc + 1 + D;
        Region<LP>& dst = rv[kl % D];
        if (kl < NC) {
          load_region(cur, kl, dst);
        } else if (kl < 2 * NC) {
          if (has_next) load_region(nxt, kl - NC, dst);
        } else if (has_next2) {
          load_region(tile_of(jt + 2), kl - 2 * NC, dst);
        }
      }
      if (kc == NC - D) {
        // the unaries of this tile's epilogue, D - 1 stages ahead
#pragma unroll
        for (int nb = 0; nb < NNB; ++nb)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float* pu = unary_at(cur, nb, j);
            uu[nb][j] = STREAM ? __builtin_nontemporal_load(pu) : *pu;
          }
      }

      // products of this stage's S chunk
      const float* sb = ss[kc & 1];
      if constexpr (F32) {
#pragma unroll
        for (int nb = 0; nb < NNB; ++nb) {
#pragma unroll
          for (int kb = 0; kb < kKC / 4; ++kb) {
            const float bv = sb[(4 * kb + g) * SST + 16 * (2 * half + nb) + c];
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(tha[(kKC / 4) * kc + kb], bv, acc[nb], 0, 0, 0);
          }
        }
      } else {
#pragma unroll
        for (int nb = 0; nb < NNB; ++nb) {
          float sv[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) sv[e] = sb[(8 * g + e) * SST + 16 * (2 * half + nb) + c];
          bf16x8 sh, sl;
          split8(sv, sh, sl);
          acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(thh[kc], sh, acc[nb], 0, 0, 0);
          acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(thh[kc], sl, acc[nb], 0, 0, 0);
          acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(thl[kc], sh, acc[nb], 0, 0, 0);
        }
      }

      // S of stage k + 1 (the next chunk, or chunk 0 of the next tile)
      if (kc + 1 < NC || has_next) form_s(qs[(kc + 1) & 1], ss[(kc + 1) & 1]);
      // stage the q of stage k + 2 over the buffer of stage k
      {
        const int k2 = kc + 2;
        if (k2 < NC) store_region(k2, rv[k2 % D], qs[kc & 1], ls[jt & 1]);
        else if (has_next) store_region(k2 - NC, rv[k2 % D], qs[kc & 1], ls[(jt + 1) & 1]);
      }

      if (kc == NC - 1) {
        // Epilogue: the damped step, then the per-node log-sum-exp over the
        // NOB output blocks of the node's half.
        const float* lsb = ls[jt & 1];
        float z[NNB][4];
#pragma unroll
        for (int nb = 0; nb < NNB; ++nb) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int l = 16 * ob + 4 * g + j;
            const float e = lsb[(l < LP ? l : LP - 1) * LS + 16 * (2 * half + nb) + c];
            const float zz = one_minus_alpha * e - a.alpha * (uu[nb][j] + acc[nb][j]);
            z[nb][j] = l < L ? zz : -INFINITY;
          }
        }
#pragma unroll
        for (int nb = 0; nb < NNB; ++nb) {
          float m = z[nb][0];
#pragma unroll
          for (int j = 1; j < 4; ++j) m = fmaxf(m, z[nb][j]);
          m = temporal::rows_max(m);
          // a block whose labels all lie past L (or a node past the grid's
          // edge) has m = -inf and contributes 0
          const float mref = m == -INFINITY ? 0.f : m;
          float sm = 0.f;
#pragma unroll
          for (int j = 0; j < 4; ++j) sm += __expf(z[nb][j] - mref);
          sm = temporal::rows_sum(sm);
          if (g == 0) {
            red_m[ob][16 * (2 * half + nb) + c] = m;
            red_s[ob][16 * (2 * half + nb) + c] = sm;
          }
        }
        __syncthreads();   // the stage's barrier: S, staging and the partial sums done
#pragma unroll
        for (int nb = 0; nb < NNB; ++nb) {
          const int p = 16 * (2 * half + nb) + c;
          float Mx = red_m[0][p];
#pragma unroll
          for (int w = 1; w < NOB; ++w) Mx = fmaxf(Mx, red_m[w][p]);
          float tot = 0.f;
#pragma unroll
          for (int w = 0; w < NOB; ++w) {
            const float mw = red_m[w][p];
            tot += mw == -INFINITY ? 0.f : red_s[w][p] * __expf(mw - Mx);
          }
          const float lse = Mx + __logf(tot);
          const int x = cur.x0 + p;
          if (x < W) {
            const unsigned n = cur.row_n + (unsigned)x;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int l = 16 * ob + 4 * g + j;
              if (l < L) {
                if constexpr (STREAM) __builtin_nontemporal_store(z[nb][j] - lse, &cur.out[(unsigned)l * N + n]);
                else cur.out[(unsigned)l * N + n] = z[nb][j] - lse;
              }
            }
          }
        }
      } else {
        __syncthreads();   // the stage's barrier
      }
    }
    cur = nxt;
  }
}

// Compute units of the current device (queried once per device).
inline int compute_units() {
  static int cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    cached[dev] = cus;
  }
  return cached[dev];
}

// Workgroups of one kernel resident per compute unit (from its registers
// and LDS; queried once per device).
template <typename K>
int resident_per_cu(K kernel, int threads) {
  static int cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 1;
  if (!cached[dev]) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0) != hipSuccess || n <= 0) n = 1;
    cached[dev] = n;
  }
  return cached[dev];
}

template <int LP, int CONN, int PREC, bool STREAM>
hipError_t go(const StepArgs& a, int compat, hipStream_t s) {
  const auto kernel = large_step_kernel<LP, CONN, PREC, STREAM>;
  const long long tiles = (long long)((a.W + kTN - 1) / kTN) * a.H * a.B;
  // resident workgroups for the whole launch, a multiple of 8 so that each
  // stays on one XCD's tile range, at most one per tile
  long long wgs = (long long)resident_per_cu(kernel, Geo<LP>::NT) * compute_units();
  if (tiles <= wgs) wgs = tiles;
  else wgs -= wgs % lanes::kXcds;
  const dim3 grid((unsigned)wgs), block(Geo<LP>::NT);
  const float om = (float)(1.0 - (double)a.alpha);
  const int potts = compat == MF_COMPAT_POTTS;
  hipLaunchKernelGGL(kernel, grid, block, 0, s, a, om, potts);
  return hipGetLastError();
}

template <int LP, int PREC>
hipError_t by_stream(const StepArgs& a, int conn, int compat, hipStream_t s) {
  const bool stream = lanes::streams_past_cache(a);
  if (conn == 4) return stream ? go<LP, 4, PREC, true>(a, compat, s) : go<LP, 4, PREC, false>(a, compat, s);
  return stream ? go<LP, 8, PREC, true>(a, compat, s) : go<LP, 8, PREC, false>(a, compat, s);
}

template <int PREC>
hipError_t by_size(const StepArgs& a, int conn, int compat, hipStream_t s) {
  if (a.L <= 64) return by_stream<64, PREC>(a, conn, compat, s);
  return by_stream<128, PREC>(a, conn, compat, s);
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
