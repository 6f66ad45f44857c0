// Power method for the Lipschitz constant of the gradient of the expected
// energy on the tangent space of the product of simplices (Sec. 3.2).
//
// The pairwise part of E(q) is quadratic, so its gradient (the message
// minus the unary, theta* of Eq. 15) is linear in q and applying it to a
// direction v is the Hessian-vector product:
//   (H v)_i = Theta S_i(v) [+ C (T(v) - v_i) / N],  S_i(v) = sum_j w_ij v_j,
// with T(v) = sum_j v_j for the co-occurrence term.  P subtracts each node's
// mean over labels (the tangent space of the simplex).  One iteration is
//   hvp:    w = P H P v + shift v, with v = scale * (previous w); per-block
//           FP64 partial sums of w.w, v.w, v.v (and of w per label for the
//           co-occurrence column sums)
//   reduce: one workgroup sums the partials in a fixed order and sets the
//           scale of the next iterate (1 / |w|) and the estimates
// so no host round trip sits between iterations.  Arithmetic on v is FP32,
// every sum FP64.
#include <hip/hip_runtime.h>

#include "grid_lanes.h"
#include "mf_internal.h"

namespace mf {
namespace {

constexpr int kLipThreads = 256;
constexpr int kLipWaves = kLipThreads / 64;
constexpr int kSparseThreads = 256;

// Block sum of NV doubles per thread into part[0..NV) (the first NV threads
// write); WAVES wavefronts per block.
template <int NV, int WAVES = kLipWaves>
__device__ inline void block_sum_store(double (&x)[NV], double* red, double* part) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double v = x[i];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((tid & 63) == 0) red[(tid >> 6) * NV + i] = v;
  }
  __syncthreads();
  if (tid < NV) {
    double s = 0.0;
    for (int w = 0; w < WAVES; ++w) s += red[w * NV + tid];
    part[tid] = s;
  }
}

// Centre, shift and accumulate for one node: h is H v at the node (FP32),
// vo the node's v.  Writes w and adds to the three partial sums.
__device__ inline void finish_node(float (&h)[kSmallLabels], const float (&vo)[kSmallLabels], int L,
                                   unsigned N, unsigned n, float shift, float* __restrict__ w, double& ww,
                                   double& vw, double& vv) {
  float mean = 0.f;
#pragma unroll
  for (int l = 0; l < kSmallLabels; ++l)
    if (l < L) mean += h[l];
  mean /= (float)L;
#pragma unroll
  for (int l = 0; l < kSmallLabels; ++l) {
    if (l < L) {
      const float wl = (h[l] - mean) + shift * vo[l];
      w[(unsigned)l * N + n] = wl;
      ww += (double)wl * wl;
      vw += (double)vo[l] * wl;
      vv += (double)vo[l] * vo[l];
      h[l] = wl;
    }
  }
}

__device__ inline void compat_product(const LipArgs& a, const float (&S)[kSmallLabels], float (&h)[kSmallLabels]) {
  const int L = a.L;
  if (a.compat == MF_COMPAT_POTTS) {
    float tot = 0.f;
#pragma unroll
    for (int k = 0; k < kSmallLabels; ++k)
      if (k < L) tot += S[k];
#pragma unroll
    for (int l = 0; l < kSmallLabels; ++l) h[l] = l < L ? a.potts_w * (tot - S[l]) : 0.f;
  } else {
#pragma unroll
    for (int l = 0; l < kSmallLabels; ++l) {
      float acc = 0.f;
      if (l < L) {
#pragma unroll
        for (int k = 0; k < kSmallLabels; ++k)
          if (k < L) acc = fmaf(a.theta[l * L + k], S[k], acc);
      }
      h[l] = acc;
    }
  }
}

// Shared tail of the sparse products: Theta S (or Potts), centring, the
// shift term, the write of w and the three partial sums.
template <int LC>
__device__ inline void hvp_finish(const LipArgs& a, const float* th, const float (&S)[LC], const float (&vo)[LC],
                                  float scale, float shift, unsigned n, double (&x)[3]) {
  const int L = a.L;
  const unsigned N = (unsigned)a.N;
  float h[LC];
  if (a.compat == MF_COMPAT_POTTS) {
    float tot = 0.f;
#pragma unroll
    for (int k = 0; k < LC; ++k) tot += S[k];
#pragma unroll
    for (int l = 0; l < LC; ++l) h[l] = l < L ? a.potts_w * scale * (tot - S[l]) : 0.f;
  } else {
#pragma unroll
    for (int l = 0; l < LC; ++l) {
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < LC; ++k) acc = fmaf(th[l * LC + k], S[k], acc);
      h[l] = acc * scale;
    }
  }
  float mean = 0.f;
#pragma unroll
  for (int l = 0; l < LC; ++l) mean += h[l];
  mean /= (float)L;
#pragma unroll
  for (int l = 0; l < LC; ++l) {
    if (l < L) {
      const float wl = (h[l] - mean) + shift * vo[l];
      a.w[(unsigned)l * N + n] = wl;
      x[0] += (double)wl * wl;
      x[1] += (double)vo[l] * wl;
      x[2] += (double)vo[l] * vo[l];
    }
  }
}

template <int LC>
__device__ inline void stage_theta(const LipArgs& a, float* th, int nthreads) {
  if (a.compat == MF_COMPAT_GENERAL) {
    for (int f = threadIdx.x; f < LC * LC; f += nthreads) {
      const int l = f / LC, k = f - (f / LC) * LC;
      th[f] = (l < a.L && k < a.L) ? a.theta[l * a.L + k] : 0.f;
    }
  }
}

// Grids: a 16 x 16 tile of nodes per workgroup with its 1-node halo of v in
// LDS (off-grid entries 0: free boundary, unit weights).  LC label slots
// (the label count rounded up to 2, 4, 8, 16, 21 or 32; slots >= L stay
// zero) so the label loops unroll exactly; Theta is staged in LDS.
constexpr int kGT = 16, kGH = kGT + 2;
template <int LC>
__global__ __launch_bounds__(kGT * kGT) void lip_hvp_grid_kernel(LipArgs a) {
  __shared__ double red[kGT * kGT / 64 * 3];
  __shared__ float th[LC * LC];
  __shared__ float tile[LC * kGH * kGH];
  const unsigned N = (unsigned)a.N;
  const int L = a.L, H = a.H, W = a.W;
  // tiles dealt XCD by XCD (neighbouring tiles share an L2); the partial
  // sums are indexed by the tile, so their order is fixed
  const int tiles_x = (W + kGT - 1) / kGT;
  const int tid_t = lanes::xcd_tile(blockIdx.x, tiles_x * ((H + kGT - 1) / kGT));
  const int x0 = (tid_t - (tid_t / tiles_x) * tiles_x) * kGT - 1, y0 = (tid_t / tiles_x) * kGT - 1;
  stage_theta<LC>(a, th, kGT * kGT);
  for (int f = threadIdx.x; f < LC * kGH * kGH; f += kGT * kGT) {
    const int l = f / (kGH * kGH), c = f - l * (kGH * kGH);
    const int gy = y0 + c / kGH, gx = x0 + (c - (c / kGH) * kGH);
    const bool ok = l < L && gy >= 0 && gy < H && gx >= 0 && gx < W;
    const float v = a.v[ok ? (unsigned)l * N + (unsigned)(gy * W + gx) : 0u];
    tile[f] = ok ? v : 0.f;
  }
  __syncthreads();
  const float scale = (float)a.sc[0];
  const float shift = (float)a.sc[1];
  const int tx = threadIdx.x % kGT, ty = threadIdx.x / kGT;
  const int gx = x0 + 1 + tx, gy = y0 + 1 + ty;
  double x[3] = {0.0, 0.0, 0.0};
  if (gx < W && gy < H) {
    const unsigned n = (unsigned)(gy * W + gx);
    const int c = (ty + 1) * kGH + (tx + 1);
    float S[LC], vo[LC];
#pragma unroll
    for (int l = 0; l < LC; ++l) {
      const float* t = tile + l * kGH * kGH + c;
      float sum = (t[-kGH] + t[-1]) + (t[1] + t[kGH]);
      if (a.graph == MF_GRID8) sum += (t[-kGH - 1] + t[-kGH + 1]) + (t[kGH - 1] + t[kGH + 1]);
      S[l] = sum;
      vo[l] = scale * t[0];
    }
    hvp_finish<LC>(a, th, S, vo, scale, shift, n, x);
  }
  block_sum_store<3>(x, red, a.part + (size_t)tid_t * a.np);
}

// CSR: one thread per node gathering its row.
template <int LC>
__global__ __launch_bounds__(kSparseThreads) void lip_hvp_csr_kernel(LipArgs a) {
  __shared__ double red[kSparseThreads / 64 * 3];
  __shared__ float th[LC * LC];
  const unsigned N = (unsigned)a.N;
  const int L = a.L;
  const unsigned n = blockIdx.x * kSparseThreads + threadIdx.x;
  stage_theta<LC>(a, th, kSparseThreads);
  __syncthreads();
  const float scale = (float)a.sc[0];
  const float shift = (float)a.sc[1];
  double x[3] = {0.0, 0.0, 0.0};
  if (n < N) {
    float S[LC], vo[LC];
#pragma unroll
    for (int l = 0; l < LC; ++l) {
      S[l] = 0.f;
      vo[l] = l < L ? scale * a.v[(unsigned)l * N + n] : 0.f;
    }
    // rows clamped to [0, nnz) and out-of-range columns skipped, as in the
    // step kernel: a malformed CSR never reads out of bounds
    long long e0 = a.row_ptr[n], e1 = a.row_ptr[n + 1];
    e0 = e0 < 0 ? 0 : e0;
    e1 = e1 > a.nnz ? a.nnz : e1;
    for (long long e = e0; e < e1; ++e) {
      const int jc = a.col[e];
      if (jc < 0 || jc >= (int)N) continue;
      const unsigned j = (unsigned)jc;
      const float we = a.csr_w ? a.csr_w[e] : 1.f;
#pragma unroll
      for (int l = 0; l < LC; ++l)
        if (l < L) S[l] = fmaf(we, a.v[(unsigned)l * N + j], S[l]);
    }
    hvp_finish<LC>(a, th, S, vo, scale, shift, n, x);
  }
  block_sum_store<3>(x, red, a.part + (size_t)blockIdx.x * a.np);
}

// Dense graph: one wavefront per row i, lanes over the columns j of the
// BF16 kernel row; then the compatibility product, the co-occurrence term
// C (T - v_i) / N with T the (scaled) column sums of v, and the per-label
// column sums of w for the next iteration.
__global__ __launch_bounds__(kLipThreads) void lip_hvp_dense_kernel(LipArgs a) {
  __shared__ double red[kLipWaves * (3 + kSmallLabels)];
  __shared__ float rows_w[kLipWaves][kSmallLabels];
  const unsigned N = (unsigned)a.N;
  const int L = a.L;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned i = blockIdx.x * kLipWaves + wave;
  const float scale = (float)a.sc[0];
  const float shift = (float)a.sc[1];
  double x[3] = {0.0, 0.0, 0.0};
  float S[kSmallLabels];
#pragma unroll
  for (int l = 0; l < kSmallLabels; ++l) S[l] = 0.f;
  if (i < N) {
    const uint16_t* Ki = a.K + (size_t)i * N;
    for (unsigned j = lane; j < N; j += 64) {
      const float k = __uint_as_float((unsigned)Ki[j] << 16);
#pragma unroll
      for (int l = 0; l < kSmallLabels; ++l)
        if (l < L) S[l] = fmaf(k, a.v[(unsigned)l * N + j], S[l]);
    }
  }
#pragma unroll
  for (int l = 0; l < kSmallLabels; ++l) {
    float s = S[l];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    S[l] = s * scale;
  }
  float wrow[kSmallLabels];
#pragma unroll
  for (int l = 0; l < kSmallLabels; ++l) wrow[l] = 0.f;
  if (i < N && lane == 0) {
    float vo[kSmallLabels], h[kSmallLabels];
#pragma unroll
    for (int l = 0; l < kSmallLabels; ++l) vo[l] = l < L ? scale * a.v[(unsigned)l * N + i] : 0.f;
    compat_product(a, S, h);
    if (a.cooc) {
      // C (T - v_i) / N in FP64 (T is kept in FP64 by the reduction)
#pragma unroll
      for (int l = 0; l < kSmallLabels; ++l) {
        if (l < L) {
          double c = 0.0;
#pragma unroll
          for (int k = 0; k < kSmallLabels; ++k)
            if (k < L) c += (double)a.cooc[l * L + k] * (a.sc[2 + k] - (double)vo[k]);
          h[l] += (float)(c / (double)N);
        }
      }
    }
    finish_node(h, vo, L, N, i, shift, a.w, x[0], x[1], x[2]);
#pragma unroll
    for (int l = 0; l < kSmallLabels; ++l) wrow[l] = h[l];
  }
  // per-label column sums of w over the block's rows (lane 0 of each wave holds its row)
  if (lane == 0) {
#pragma unroll
    for (int l = 0; l < kSmallLabels; ++l) rows_w[wave][l] = wrow[l];
  }
  double xs[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) xs[t] = lane == 0 ? x[t] : 0.0;
  block_sum_store<3>(xs, red, a.part + (size_t)blockIdx.x * a.np);
  if (threadIdx.x < kSmallLabels) {
    double s = 0.0;
    for (int w = 0; w < kLipWaves; ++w) s += (double)rows_w[w][threadIdx.x];
    a.part[(size_t)blockIdx.x * a.np + 3 + threadIdx.x] = s;
  }
}

// v = v0 - mean over labels (per node) into a.w, with the partial sums of
// v.v (slot 2) and, for the co-occurrence term, of v per label.
__global__ __launch_bounds__(kLipThreads) void lip_center_kernel(LipArgs a, const float* __restrict__ v0) {
  __shared__ double red[kLipWaves * (3 + kSmallLabels)];
  const unsigned N = (unsigned)a.N;
  const int L = a.L;
  const unsigned n = blockIdx.x * kLipThreads + threadIdx.x;
  double x[3 + kSmallLabels];
#pragma unroll
  for (int t = 0; t < 3 + kSmallLabels; ++t) x[t] = 0.0;
  if (n < N) {
    float mean = 0.f;
#pragma unroll
    for (int l = 0; l < kSmallLabels; ++l)
      if (l < L) mean += v0[(unsigned)l * N + n];
    mean /= (float)L;
#pragma unroll
    for (int l = 0; l < kSmallLabels; ++l) {
      if (l < L) {
        const float c = v0[(unsigned)l * N + n] - mean;
        a.w[(unsigned)l * N + n] = c;
        x[2] += (double)c * c;
        x[3 + l] = c;
      }
    }
  }
  if (a.np > 3) {
    block_sum_store<3 + kSmallLabels>(x, red, a.part + (size_t)blockIdx.x * a.np);
  } else {
    double y[3] = {x[0], x[1], x[2]};
    block_sum_store<3>(y, red, a.part + (size_t)blockIdx.x * a.np);
  }
}

// Sum the partials of n_blocks blocks (fixed order) and update the scalars.
//   mode 0: after centring, run 1 (scale 1: the first ratio uses the raw start)
//   mode 1: after centring, run 2 (scale 1 / |v|; shift = rho of run 1)
//   mode 2: after an hvp of run 1: rho = |w| / |v| until |w| = 0
//   mode 3: after an hvp of run 2: lam = v.w / v.v until |w| = 0
// sc: [0] scale of the next v, [1] shift, [2..2+L) T of the next v,
// res: [0] rho, [1] lam, [2] run-1 stopped, [3] run-2 stopped.
__global__ __launch_bounds__(kLipThreads) void lip_reduce_kernel(LipArgs a, int n_blocks, int mode) {
  __shared__ double red[kLipThreads];
  __shared__ double tot[3 + kSmallLabels];
  const int tid = threadIdx.x;
  for (int c = 0; c < a.np; ++c) {
    double s = 0.0;
    for (int b = tid; b < n_blocks; b += kLipThreads) s += a.part[(size_t)b * a.np + c];
    red[tid] = s;
    __syncthreads();
    for (int o = kLipThreads / 2; o > 0; o >>= 1) {
      if (tid < o) red[tid] += red[tid + o];
      __syncthreads();
    }
    if (tid == 0) tot[c] = red[0];
    __syncthreads();
  }
  if (tid == 0) {
    double* sc = a.sc;
    double* res = a.res;
    const double ww = tot[0], vw = tot[1], vv = tot[2];
    double scale;
    if (mode == 0 || mode == 1) {
      // ww slot holds nothing here; vv is |v0 - mean|^2
      scale = mode == 0 ? 1.0 : (vv > 0.0 ? 1.0 / sqrt(vv) : 0.0);
      sc[1] = mode == 0 ? 0.0 : res[0];
      if (mode == 1) res[3] = vv > 0.0 ? 0.0 : 1.0;
      if (mode == 0) {
        res[0] = 0.0;
        res[1] = 0.0;
        res[2] = 0.0;
      }
    } else {
      const double nw = sqrt(ww);
      const int stop_slot = mode == 2 ? 2 : 3;
      if (res[stop_slot] == 0.0) {
        if (nw == 0.0) {
          res[stop_slot] = 1.0;
          if (mode == 3) res[1] = 0.0;
        } else if (mode == 2) {
          res[0] = nw / sqrt(vv);
        } else {
          res[1] = vw / vv;
        }
      }
      scale = nw > 0.0 ? 1.0 / nw : 0.0;
    }
    sc[0] = scale;
    if (a.np > 3) {
      for (int l = 0; l < a.L; ++l) sc[2 + l] = tot[3 + l] * scale;
    }
  }
}

}  // namespace

hipError_t launch_lip_center(const LipArgs& a, const float* v0, hipStream_t s) {
  const unsigned blocks = (unsigned)((a.N + kLipThreads - 1) / kLipThreads);
  hipLaunchKernelGGL(lip_center_kernel, dim3(blocks), dim3(kLipThreads), 0, s, a, v0);
  return hipGetLastError();
}

hipError_t launch_lip_hvp(const LipArgs& a, hipStream_t s) {
  if (a.graph == MF_DENSE) {
    const unsigned blocks = (unsigned)((a.N + kLipWaves - 1) / kLipWaves);
    hipLaunchKernelGGL(lip_hvp_dense_kernel, dim3(blocks), dim3(kLipThreads), 0, s, a);
  } else {
    const int L = a.L;
    if (a.graph == MF_CSR) {
      const dim3 grid((unsigned)((a.N + kSparseThreads - 1) / kSparseThreads)), block(kSparseThreads);
      if (L <= 2) hipLaunchKernelGGL(lip_hvp_csr_kernel<2>, grid, block, 0, s, a);
      else if (L <= 4) hipLaunchKernelGGL(lip_hvp_csr_kernel<4>, grid, block, 0, s, a);
      else if (L <= 8) hipLaunchKernelGGL(lip_hvp_csr_kernel<8>, grid, block, 0, s, a);
      else if (L <= 16) hipLaunchKernelGGL(lip_hvp_csr_kernel<16>, grid, block, 0, s, a);
      else if (L == 21) hipLaunchKernelGGL(lip_hvp_csr_kernel<21>, grid, block, 0, s, a);
      else hipLaunchKernelGGL(lip_hvp_csr_kernel<32>, grid, block, 0, s, a);
    } else {
      const dim3 grid((unsigned)(((a.W + kGT - 1) / kGT) * ((a.H + kGT - 1) / kGT))), block(kGT * kGT);
      if (L <= 2) hipLaunchKernelGGL(lip_hvp_grid_kernel<2>, grid, block, 0, s, a);
      else if (L <= 4) hipLaunchKernelGGL(lip_hvp_grid_kernel<4>, grid, block, 0, s, a);
      else if (L <= 8) hipLaunchKernelGGL(lip_hvp_grid_kernel<8>, grid, block, 0, s, a);
      else if (L <= 16) hipLaunchKernelGGL(lip_hvp_grid_kernel<16>, grid, block, 0, s, a);
      else if (L == 21) hipLaunchKernelGGL(lip_hvp_grid_kernel<21>, grid, block, 0, s, a);
      else hipLaunchKernelGGL(lip_hvp_grid_kernel<32>, grid, block, 0, s, a);
    }
  }
  return hipGetLastError();
}

hipError_t launch_lip_reduce(const LipArgs& a, int n_blocks, int mode, hipStream_t s) {
  hipLaunchKernelGGL(lip_reduce_kernel, dim3(1), dim3(kLipThreads), 0, s, a, n_blocks, mode);
  return hipGetLastError();
}

int lip_blocks(int graph, int N, int H, int W) {
  if (graph == MF_DENSE) return (N + kLipWaves - 1) / kLipWaves;
  if (graph == MF_CSR) return (N + kSparseThreads - 1) / kSparseThreads;
  return ((W + kGT - 1) / kGT) * ((H + kGT - 1) / kGT);
}

}  // namespace mf
