// Storage codecs of the neighbour-message operand q (in LDS on grids, the
// node-major copy in HBM on general graphs), one per precision mode: FP32,
// BF16 (round to nearest even) or FP16.
#pragma once
#include <hip/hip_runtime.h>

namespace mf {

enum { P_F32 = 0, P_BF16 = 1, P_F16 = 2 };

template <int PREC> struct MsgT;
template <> struct MsgT<P_F32> {
  using T = float;
  __device__ static T enc(float x) { return x; }
  __device__ static float dec(T x) { return x; }
};
template <> struct MsgT<P_BF16> {
  using T = unsigned short;
  // q is finite and non-negative: add half an ulp of the kept part, ties to even
  __device__ static T enc(float x) {
    unsigned int u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (T)(u >> 16);
  }
  __device__ static float dec(T x) { return __uint_as_float(((unsigned int)x) << 16); }
};
template <> struct MsgT<P_F16> {
  using T = _Float16;
  // The FP32 value is rounded to FP16: the empty asm keeps the compiler from
  // folding the product that formed x into one mixed-precision FMA rounded
  // once to FP16, which it would do at some call sites and not at others,
  // so every kernel stores the same bits for the same x.
  __device__ static T enc(float x) {
    asm("" : "+v"(x));
    return (T)x;
  }
  __device__ static float dec(T x) { return (float)x; }
};

}  // namespace mf
