// Device code of the learned index's model, shared by the single-table
// learned search, the error bound and the plan kernels: parameter layout,
// model input, the compiled forward pass, predicted index and the verified
// window search.
#pragma once

#include "ss_device.h"
#include "../../include/searchsorted.h"

namespace ss {

constexpr int kH = 32;
constexpr int kOffW1 = 0, kOffB1 = 32, kOffW2 = 64, kOffB2 = 64 + kH * kH, kOffW3 = kOffB2 + kH,
              kOffB3 = kOffW3 + kH, kNP = kOffB3 + 1;
static_assert(kNP == SS_MLP_PARAMS, "parameter layout");
constexpr int kTrainThreads = 256;  // also the batch size

// Model input: z = (log2 x - u0) * inv, in FP32 from x rounded to FP32.
__device__ __forceinline__ float model_input(double x, float u0, float inv) {
  return (__log2f((float)x) - u0) * inv;
}

// The forward pass as the search evaluates it.  With one input, layer 1
// followed by layer 2's pre-activation is piecewise linear in z: unit j of
// layer 1 switches at its breakpoint t_j = -b1_j / w1_j, and between two
// consecutive breakpoints the set of active units is fixed, so for z in
// segment s
//   g_k(z) = b2_k + sum_{j active in s} W2_kj (w1_j z + b1_j) = P_sk z + Q_sk.
// The model is compiled once (compile_model) into an image holding the at
// most 32 breakpoints sorted ascending, one row (P_sk, Q_sk) for k < 32 per
// segment (33 segments) and the output layer, and a query costs a 6-step
// bisection over the breakpoints, 32 fused multiply-adds for g, 32 ReLUs and
// the 32-term output sum: the same function as the 1088 multiply-adds of the
// layered form, in another order of rounding.
//
// Image layout (floats; identical in global memory and LDS):
//   [0, 32)    breakpoints, ascending, padded with +inf
//   [32, 64)   w3
//   64         b3 (65..67 unused)
//   [68, ...)  33 rows of pitch 68: row s holds P_s0, Q_s0, P_s1, Q_s1, ...
//              (the pitch puts consecutive rows' 16-byte reads on
//              different LDS banks)
constexpr int kIT = 0, kIW3 = 32, kIB3 = 64, kIRows = 68, kIRowPitch = 68, kISegments = kH + 1;
constexpr int kImageFloats = kIRows + kISegments * kIRowPitch;
constexpr int kImageBytes = kImageFloats * 4;
static_assert(kImageBytes % 16 == 0, "16-byte copies");

// Copies a compiled image into LDS with 16-byte loads; called by every
// thread of the workgroup, followed by a barrier before use.
__device__ __forceinline__ void stage_image(float* m, const float* __restrict__ img) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const f4* src = reinterpret_cast<const f4*>(img);
  f4* dst = reinterpret_cast<f4*>(m);
  for (int i = threadIdx.x; i < kImageFloats / 4; i += blockDim.x) dst[i] = src[i];
}

// max(v, 0) as one integer max on the encoding: non-negative floats are
// non-negative integers and negative floats negative ones, so the result is
// v for v >= +0 and +0 for v < 0 (and for -0).
__device__ __forceinline__ float relu_bits(float v) {
  return __int_as_float(max(__float_as_int(v), 0));
}

typedef float v4f __attribute__((ext_vector_type(4)));

// The output layer of a staged model: the same for every lane, so it is read
// once per staging and kept in scalar registers (the 32 weights would
// otherwise take 32 vector registers per lane).  The whole workgroup calls
// it after the barrier that follows stage_image.
struct OutLayer {
  float w3[kH];
  float b3;
};

__device__ __forceinline__ float lane0_f(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ OutLayer load_out_layer(const float* m) {
  OutLayer o;
#pragma unroll
  for (int k = 0; k < kH; ++k) o.w3[k] = lane0_f(m[kIW3 + k]);
  o.b3 = lane0_f(m[kIB3]);
  return o;
}

// The model's output p(z) from a compiled image in LDS and its output
// layer.  The segment is s = #{i : t_i < z} (0..32; NaN gives 0).  Lanes
// are independent: no wavefront-wide operation.
__device__ __forceinline__ float mlp_eval(const float* m, const OutLayer& o, float z) {
  int s = 0;
#pragma unroll
  for (int step = 16; step >= 1; step >>= 1) s = (m[kIT + s + step - 1] < z) ? s + step : s;
  s += (m[kIT + s] < z) ? 1 : 0;
  const v4f* row = reinterpret_cast<const v4f*>(m + kIRows + kIRowPitch * s);
  float acc0 = o.b3, acc1 = 0.0f;
#pragma unroll
  for (int c = 0; c < kH / 4; ++c) {
    const v4f a = row[2 * c], b = row[2 * c + 1];
    acc0 = fmaf(o.w3[4 * c], relu_bits(fmaf(a[0], z, a[1])), acc0);
    acc1 = fmaf(o.w3[4 * c + 1], relu_bits(fmaf(a[2], z, a[3])), acc1);
    acc0 = fmaf(o.w3[4 * c + 2], relu_bits(fmaf(b[0], z, b[1])), acc0);
    acc1 = fmaf(o.w3[4 * c + 3], relu_bits(fmaf(b[2], z, b[3])), acc1);
  }
  return acc0 + acc1;
}

// Predicted index g = floor(p (n-1)) clamped to [-1, n-1].  Any p, even NaN
// or inf, yields a valid index (fmaxf/fminf return the bound for NaN).
__device__ __forceinline__ int predicted_index(float p, int n) {
  const float g = floorf(p * (float)(n - 1));
  return (int)fminf(fmaxf(g, -1.0f), (float)(n - 1));
}

// The verified window search for Q targets per lane.  m is the model's
// compiled image in LDS, o its output layer.
template <int Q>
__device__ __forceinline__ void search_learned(const double* __restrict__ sa, int n,
                                               const float* m, const OutLayer& o, int E,
                                               float u0, float inv, const double (&x)[Q],
                                               int (&r)[Q], int (&fell_back)[Q]) {
  float p[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) p[q] = mlp_eval(m, o, model_input(x[q], u0, inv));
  int step = 1;
  while (step * 2 <= 2 * E + 1) step *= 2;  // >= half the window length
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int g = predicted_index(p[q], n);
    const int L = max(g - E, -1), R = min(g + E, n - 1);
    const bool lo_ok = L < 0 || sa[max(L, 0)] < x[q];
    const bool hi_ok = R >= n - 1 || x[q] <= sa[min(R + 1, n - 1)];
    fell_back[q] = !(lo_ok && hi_ok);
    if (lo_ok && hi_ok) {
      // pos = #{a < x} lies in [L+1, R+1]: every entry up to a[L] is below
      // x and every entry from a[R+1] on is not, so the steps need no upper
      // bound (a read at or past R+1 never advances pos; reads past the
      // table are clamped to its +inf sentinel a[n]).  2 step - 1 >= 2E
      // covers the window.
      int pos = L + 1;
      for (int s = step; s >= 1; s >>= 1) pos = (sa[min(pos + s - 1, n)] < x[q]) ? pos + s : pos;
      r[q] = pos - 1;
    } else {
      int base = 0, len = n;
      while (len > 1) {
        const int half = len >> 1;
        base = (sa[base + half] < x[q]) ? base + half : base;
        len -= half;
      }
      r[q] = base + (sa[base] < x[q] ? 1 : 0) - 1;
    }
  }
}

}  // namespace ss
