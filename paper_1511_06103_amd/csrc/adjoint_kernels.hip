// Reverse pass of T unrolled proximal steps on a grid (hand-written adjoint).
//
// Forward step (Eq. 15 with the fixed step of Eq. 16):
//   S = A q,  m = u + Theta S,  z = (1 - a) ell - a m,  ell' = z - lse(z)
// Given g = dLoss/d ell', one reverse step computes
//   zb   = g - q' (sum_l g_l)                 (through the normalisation)
//   mb   = -a zb;   ub += mb;   Thetab += sum_i mb_i S_i^T
//   Sb   = Theta^T mb;   qb = A Sb            (A symmetric on a grid)
//   g    <- (1 - a) zb + q (.) qb            (dLoss / d ell)
// Kernel A does everything up to Sb for one 64 x 4 tile (S needs the q halo),
// kernel B the transposed stencil over Sb (needs the Sb halo) and the new g.
// Theta_bar partials are per tile: mb and S of the tile's nodes are staged in
// LDS (over the q halo, which is dead by then) and the L x L block product is
// formed there on the FP32 matrix cores, then added to the tile's own FP64
// accumulator (each workgroup owns its slot, so there is no race).  After the last step the tile accumulators
// are reduced in a fixed order: the sum runs over steps within a tile, then
// over tiles, and is deterministic.
#include <hip/hip_runtime.h>

#include "grid_lanes.h"
#include "mf_internal.h"

namespace mf {
namespace {

// Tile of this workgroup, dealt XCD by XCD as in the forward step kernel so
// that neighbouring tiles (which read each other's halo) share an L2.
struct AdjTile {
  int t, b, x0, y0;
};
__device__ inline AdjTile adj_tile(const AdjointArgs& a) {
  const int tx = (a.W + kTileX - 1) / kTileX, ty = (a.H + kTileY - 1) / kTileY;
  AdjTile r;
  r.t = lanes::xcd_tile(blockIdx.x, tx * ty * a.B);
  r.b = r.t / (tx * ty);
  const int q = r.t - r.b * (tx * ty);
  r.y0 = (q / tx) * kTileY;
  r.x0 = (q - (q / tx) * tx) * kTileX;
  return r;
}

constexpr int AX = kTileX + 2;
constexpr int AY = kTileY + 2;
constexpr int AN = AX * AY;
// Tile partials of Theta_bar summed per stage-1 block.
constexpr int kThetaChunk = 32;

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Stage the L label planes of a (64 + 2) x (4 + 2) halo region into LDS,
// optionally through exp.  The trip count is fixed by LP, so every load of
// a thread is issued before the first is used.
template <int LP, bool EXP>
__device__ __forceinline__ void load_halo(const float* __restrict__ src, float* __restrict__ dst, int L, int N, int H, int W,
                                 int x0, int y0, int tid) {
  constexpr int IT = (LP * AN + kThreads - 1) / kThreads;
  float v[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = tid + it * kThreads;
    const int l = idx / AN;
    const int r = idx - l * AN;
    const int hy = r / AX, hx = r - (r / AX) * AX;
    const int gy = y0 + hy - 1, gx = x0 + hx - 1;
    const bool on = l < L && gy >= 0 && gy < H && gx >= 0 && gx < W;
    // clamped address: the load is unconditional, the value selected
    const int lc = l < L ? l : L - 1;
    const int gyc = gy < 0 ? 0 : (gy < H ? gy : H - 1), gxc = gx < 0 ? 0 : (gx < W ? gx : W - 1);
    const float t = src[(size_t)lc * N + gyc * W + gxc];
    v[it] = on ? t : (EXP ? -INFINITY : 0.f);
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = tid + it * kThreads;
    if (idx < L * AN) dst[idx] = EXP ? __expf(v[it]) : v[it];
  }
}

// At L = 21 the kernel fits 122 VGPRs and 35 KB of LDS: asking for four
// waves per SIMD keeps the MFMA accumulator out of AGPRs, so four
// workgroups share a CU (one wave of workgroups on the 16 x 128 x 128
// batch).  Other label counts keep the compiler's choice.
template <int LP, bool EXACT, int CONN, int COMPAT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(LP == 21 ? 4 : 1))) void adj_a_kernel(
    AdjointArgs a) {
  constexpr int NB = (LP + 15) / 16;       // 16-label blocks of Theta_bar
  constexpr int NOB = NB * NB, WPB = 4 / NOB, KJ = kThreads / WPB;
  // mb and S are staged in HS passes of HN nodes, so that the staging fits
  // in the space of the q halo; the row stride is 4 words past HN, so the 16
  // label rows a wavefront reads at once fall on distinct banks.
  constexpr int HS = WPB == 1 ? 2 : 1;
  constexpr int HN = kThreads / HS;
  constexpr int RH = HN + 4;
  constexpr int kU = LP * AN > 2 * LP * RH ? LP * AN : 2 * LP * RH;
  __shared__ float lds_u[kU];
  float* qs = lds_u;                       // q halo, then the staging
  float* mbs = lds_u;
  float* Ss = lds_u + LP * RH;
  // Theta transposed, rows padded to 4: Theta^T mb reads contiguous rows
  constexpr int TS = (LP + 3) & ~3;
  __shared__ float ths[COMPAT == MF_COMPAT_GENERAL ? LP * TS : 1];
  __shared__ float red[NB == 1 ? 4 * 256 : 1];
  const int L = EXACT ? LP : a.L;
  const int N = a.N, H = a.H, W = a.W;
  const AdjTile tile = adj_tile(a);
  const int b = tile.b, x0 = tile.x0, y0 = tile.y0;
  const size_t base = (size_t)b * L * N;
  const int tid = threadIdx.x;
  const int tx = tid % kTileX, ty = tid / kTileX;
  const int x = x0 + tx, y = y0 + ty;
  const bool inside = x < W && y < H;
  const int n = inside ? y * W + x : 0;
  const int p = (ty + 1) * AX + (tx + 1);

  // every load of the node is issued before any store: the output planes may
  // alias nothing the kernel reads, but the compiler cannot know that
  float g[LP], q1[LP], ub[LP];
#pragma unroll
  for (int l = 0; l < LP; ++l) {
    const bool on = inside && l < L;
    const size_t at = base + (size_t)(l < L ? l : L - 1) * N + n;
    const float g_ = a.g_in[at], q_ = a.ell_t1[at], u_ = a.u_bar[at];
    g[l] = on ? g_ : 0.f;
    q1[l] = on ? q_ : 0.f;
    ub[l] = on ? u_ : 0.f;
  }
  load_halo<LP, true>(a.ell_t + base, qs, L, N, H, W, x0, y0, tid);
  if (COMPAT == MF_COMPAT_GENERAL) {
#pragma unroll
    for (int f = tid; f < LP * TS; f += kThreads) {
      const int k = f / TS, l = f - (f / TS) * TS;
      ths[f] = (l < L && k < L) ? a.theta[l * L + k] : 0.f;
    }
  }
  __syncthreads();

  float mb[LP], S[LP];
#pragma unroll
  for (int l = 0; l < LP; ++l) {
    mb[l] = 0.f;
    S[l] = 0.f;
  }
  if (inside) {
    float sg = 0.f;
#pragma unroll
    for (int l = 0; l < LP; ++l) sg += g[l];
#pragma unroll
    for (int l = 0; l < LP; ++l) {
      if (l < L) {
        mb[l] = -a.alpha * (g[l] - __expf(q1[l]) * sg);
        a.u_bar[base + (size_t)l * N + n] = ub[l] + mb[l];
        const float* q = qs + l * AN + p;
        float s = q[-AX] + q[-1] + q[1] + q[AX];
        if (CONN == 8) s += (q[-AX - 1] + q[-AX + 1]) + (q[AX - 1] + q[AX + 1]);
        S[l] = s;
      }
    }
    // Sb = Theta^T mb
#pragma unroll
    for (int k = 0; k < LP; ++k) {
      if (k < L) {
        float acc = 0.f;
        if (COMPAT == MF_COMPAT_POTTS) {
          float tot = 0.f;
#pragma unroll
          for (int l = 0; l < LP; ++l) tot += mb[l];
          acc = a.potts_w * (tot - mb[k]);
        } else {
#pragma unroll
          for (int l = 0; l < LP; ++l) acc = fmaf(ths[k * TS + l], mb[l], acc);
        }
        a.s_bar[base + (size_t)k * N + n] = acc;
      }
    }
  }
  // Theta_bar partial of this tile, P[l][k] = sum_n mb[l][n] S[k][n]: an
  // (L x 256) (256 x L) product on v_mfma_f32_16x16x4f32 with L padded to
  // 16 NB.  Lane x of a wavefront reads A[x % 16][x / 16] = mb[row][node]
  // and B[x / 16][x % 16] = S[col][node] and holds rows 4 (x / 16) + i,
  // column x % 16 of the output block.  With NB = 2 each of the four
  // wavefronts owns one 16 x 16 output block and runs over the nodes in two
  // staged passes (the same accumulation order as one pass); with NB = 1
  // they split the 256 nodes and their sums are added in a fixed order.
  {
    const int wave = tid >> 6, lane = tid & 63;
    const int ob = wave / WPB, kpart = wave - ob * WPB;
    const int rb = ob / NB, cb = ob - rb * NB;
    const int la = 16 * rb + (lane & 15), kc = 16 * cb + (lane & 15);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const int j0 = kpart * KJ + (lane >> 4);
    for (int h = 0; h < HS; ++h) {
      __syncthreads();   // h = 0: the q halo is dead; h = 1: the first pass is read
      if (tid / HN == h) {
#pragma unroll
        for (int l = 0; l < LP; ++l) {
          mbs[l * RH + tid - h * HN] = mb[l];
          Ss[l * RH + tid - h * HN] = S[l];
        }
      }
      __syncthreads();
#pragma unroll 8
      for (int kb = 0; kb < KJ / 4 / HS; ++kb) {
        const int j = j0 + 4 * kb;
        const float av = la < LP ? mbs[la * RH + j] : 0.f;
        const float bv = kc < LP ? Ss[kc * RH + j] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
      }
    }
    const size_t part = (size_t)tile.t;
    double* out = a.theta_tile + part * L * L;
    if constexpr (WPB == 1) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int l = 16 * rb + 4 * (lane >> 4) + i;
        if (l < L && kc < L) out[l * L + kc] += (double)acc[i];
      }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) red[wave * 256 + lane * 4 + i] = acc[i];
      __syncthreads();
      if (wave == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float v = ((red[lane * 4 + i] + red[256 + lane * 4 + i]) + red[512 + lane * 4 + i]) +
                          red[768 + lane * 4 + i];
          const int l = 4 * (lane >> 4) + i;
          if (l < L && kc < L) out[l * L + kc] += (double)v;
        }
      }
    }
  }
}

template <int LP, bool EXACT, int CONN>
__global__ __launch_bounds__(kThreads) void adj_b_kernel(AdjointArgs a) {
  __shared__ float sb[LP * AN];
  const int L = EXACT ? LP : a.L;
  const int N = a.N, H = a.H, W = a.W;
  const AdjTile tile = adj_tile(a);
  const int b = tile.b, x0 = tile.x0, y0 = tile.y0;
  const size_t base = (size_t)b * L * N;
  const int tid = threadIdx.x;
  const int tx = tid % kTileX, ty = tid / kTileX;
  const int x = x0 + tx, y = y0 + ty;
  const bool inside = x < W && y < H;
  const int n = inside ? y * W + x : 0;
  const int p = (ty + 1) * AX + (tx + 1);
  load_halo<LP, false>(a.s_bar + base, sb, L, N, H, W, x0, y0, tid);
  __syncthreads();
  if (!inside) return;
  // the node's loads first, then the stores
  float g[LP], l1[LP], l0[LP];
#pragma unroll
  for (int l = 0; l < LP; ++l) {
    const size_t at = base + (size_t)(l < L ? l : L - 1) * N + n;
    g[l] = a.g_in[at];
    l1[l] = a.ell_t1[at];
    l0[l] = a.ell_t[at];
    if (l >= L) g[l] = 0.f;
  }
  float sg = 0.f;
#pragma unroll
  for (int l = 0; l < LP; ++l) sg += g[l];
  const float om = 1.f - a.alpha;
#pragma unroll
  for (int l = 0; l < LP; ++l) {
    if (l < L) {
      const float zb = g[l] - __expf(l1[l]) * sg;
      const float* s = sb + l * AN + p;
      float qb = s[-AX] + s[-1] + s[1] + s[AX];
      if (CONN == 8) qb += (s[-AX - 1] + s[-AX + 1]) + (s[AX - 1] + s[AX + 1]);
      a.g_out[base + (size_t)l * N + n] = om * zb + __expf(l0[l]) * qb;
    }
  }
}

// theta_acc[e] = sum over tiles of theta_tile[tile][e] in FP64, in a fixed
// order: stage 1, block c sums tiles [32 c, 32 c + 32) (loads coalesced over
// e); stage 2 adds the stage-1 sums in block order.
__global__ __launch_bounds__(256) void adj_theta_stage(const double* __restrict__ part, int n_parts, int LL,
                                                       double* __restrict__ stage) {
  const int c = blockIdx.x;
  const int k0 = c * kThetaChunk;
  const int k1 = k0 + kThetaChunk < n_parts ? k0 + kThetaChunk : n_parts;
  for (int e = threadIdx.x; e < LL; e += 256) {
    // fixed order; the loads of the chunk are issued before the adds
    double v[kThetaChunk];
#pragma unroll
    for (int k = 0; k < kThetaChunk; ++k) {
      const double t = part[(size_t)(k0 + k < k1 ? k0 + k : k1 - 1) * LL + e];   // clamped: no branch
      v[k] = k0 + k < k1 ? t : 0.0;
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kThetaChunk; ++k) s += v[k];
    stage[(size_t)c * LL + e] = s;
  }
}

__global__ __launch_bounds__(256) void adj_theta_finish(const double* __restrict__ stage, int n_stage, int LL,
                                                        double* __restrict__ acc) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= LL) return;
  double s = 0.0;
#pragma unroll 16
  for (int c = 0; c < n_stage; ++c) s += stage[(size_t)c * LL + e];
  acc[e] = s;
}

// Through the initialisation log q0 = -u - lse(-u): ub += -(g0 - q0 sum g0).
__global__ __launch_bounds__(256) void adj_init_kernel(const float* __restrict__ g0, const float* __restrict__ ell0,
                                                       float* __restrict__ u_bar, int L, int N) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  const int b = blockIdx.y;
  if (n >= N) return;
  const size_t base = (size_t)b * L * N + n;
  float sg = 0.f;
  for (int l = 0; l < L; ++l) sg += g0[base + (size_t)l * N];
  for (int l = 0; l < L; ++l) {
    const float q0 = __expf(ell0[base + (size_t)l * N]);
    u_bar[base + (size_t)l * N] -= g0[base + (size_t)l * N] - q0 * sg;
  }
}

__global__ __launch_bounds__(256) void fill_f32(float* __restrict__ p, size_t n, float v) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void fill_f64(double* __restrict__ p, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

__global__ __launch_bounds__(256) void copy_f32(const float* __restrict__ s, float* __restrict__ d, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) d[i] = s[i];
}

__global__ __launch_bounds__(256) void f64_to_f32(const double* __restrict__ s, float* __restrict__ d, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) d[i] = (float)s[i];
}

template <int LP, bool EXACT>
hipError_t adj_lp(const AdjointArgs& a, int conn, int compat, hipStream_t s) {
  const dim3 grid((unsigned)adjoint_theta_parts(a.B, a.H, a.W));
  if (conn == 4) {
    if (compat == MF_COMPAT_POTTS) hipLaunchKernelGGL((adj_a_kernel<LP, EXACT, 4, MF_COMPAT_POTTS>), grid, dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL((adj_a_kernel<LP, EXACT, 4, MF_COMPAT_GENERAL>), grid, dim3(kThreads), 0, s, a);
  } else {
    if (compat == MF_COMPAT_POTTS) hipLaunchKernelGGL((adj_a_kernel<LP, EXACT, 8, MF_COMPAT_POTTS>), grid, dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL((adj_a_kernel<LP, EXACT, 8, MF_COMPAT_GENERAL>), grid, dim3(kThreads), 0, s, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (conn == 4) hipLaunchKernelGGL((adj_b_kernel<LP, EXACT, 4>), grid, dim3(kThreads), 0, s, a);
  else hipLaunchKernelGGL((adj_b_kernel<LP, EXACT, 8>), grid, dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace

size_t adjoint_theta_parts(int B, int H, int W) {
  return (size_t)B * ((H + kTileY - 1) / kTileY) * ((W + kTileX - 1) / kTileX);
}

size_t adjoint_theta_stages(int B, int H, int W) {
  return (adjoint_theta_parts(B, H, W) + kThetaChunk - 1) / kThetaChunk;
}

hipError_t launch_adjoint_step(const AdjointArgs& a, int conn, int compat, hipStream_t s) {
  const int L = a.L;
  if (L == 2) return adj_lp<2, true>(a, conn, compat, s);
  if (L == 21) return adj_lp<21, true>(a, conn, compat, s);
  if (L <= 4) return adj_lp<4, false>(a, conn, compat, s);
  if (L <= 8) return adj_lp<8, false>(a, conn, compat, s);
  if (L <= 16) return adj_lp<16, false>(a, conn, compat, s);
  return adj_lp<32, false>(a, conn, compat, s);
}

hipError_t launch_adjoint_theta_reduce(const AdjointArgs& a, hipStream_t s) {
  const int n_parts = (int)adjoint_theta_parts(a.B, a.H, a.W);
  const int LL = a.L * a.L;
  const int n_stage = (n_parts + kThetaChunk - 1) / kThetaChunk;
  hipLaunchKernelGGL(adj_theta_stage, dim3(n_stage), dim3(256), 0, s, a.theta_tile, n_parts, LL, a.theta_stage);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adj_theta_finish, dim3((LL + 255) / 256), dim3(256), 0, s, a.theta_stage, n_stage, LL,
                     a.theta_acc);
  return hipGetLastError();
}

hipError_t launch_adjoint_init(const float* g0, const float* ell0, float* u_bar, int B, int L, int N, hipStream_t s) {
  hipLaunchKernelGGL(adj_init_kernel, dim3((N + 255) / 256, B), dim3(256), 0, s, g0, ell0, u_bar, L, N);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_copy_f32(const float* src, float* dst, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_f64_to_f32(const double* src, float* dst, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(f64_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace mf
