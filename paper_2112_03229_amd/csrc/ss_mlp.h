// Device code of the learned index's model, shared by the single-table
// learned search, the error bound and the plan kernels: parameter layout,
// model input, the matrix-core forward pass, predicted index and the
// verified window search.
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

// LDS image of one model for the matrix-core forward pass: the vectors w1,
// b1, b2, w3, b3, then W2 with its rows padded to 36 floats (16-byte aligned
// rows that start on different banks).
constexpr int kMW1 = 0, kMB1 = 32, kMB2 = 64, kMW3 = 96, kMB3 = 128, kMW2 = 132, kW2Pitch = 36;
constexpr int kModelFloats = kMW2 + kH * kW2Pitch;
constexpr int kModelBytes = kModelFloats * 4;

// Copies the 1153 parameters (standard layout) into the LDS image; called
// by every thread of the workgroup, followed by a barrier before use.
__device__ __forceinline__ void stage_model(float* m, const float* __restrict__ P) {
  for (int i = threadIdx.x; i < kNP; i += blockDim.x) {
    int d;
    if (i < kOffW2) d = i;                                        // w1, b1
    else if (i < kOffB2) d = kMW2 + kW2Pitch * ((i - kOffW2) / kH) + (i - kOffW2) % kH;
    else if (i < kOffW3) d = kMB2 + (i - kOffB2);
    else if (i < kOffB3) d = kMW3 + (i - kOffW3);
    else d = kMB3;
    m[d] = P[i];
  }
}

// max(v, 0) as one integer max on the encoding: non-negative floats are
// non-negative integers and negative floats negative ones, so the result is
// v for v >= +0 and +0 for v < 0 (and for -0).
__device__ __forceinline__ float relu_bits(float v) {
  return __int_as_float(max(__float_as_int(v), 0));
}

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v32f __attribute__((ext_vector_type(32)));

// Forward pass of one input per lane, 64 inputs per call: every lane of the
// wavefront must call it (uniform control flow).  Layer 1 and the output
// layer run on the vector ALUs; layer 2 (1024 of the 1088 multiply-adds) is
// a 32 x 32 x 32 product per 32 inputs on the matrix cores:
//   H2^T (unit k x input q) = W2 (k x j) . H1^T (j x q)
// as 32 rank-1 steps of v_mfma_f32_32x32x1f32, whose two 32 x 32 blocks
// hold the inputs of lanes 0-31 and of lanes 32-63.  At step j lane l gives
// the A operand W2[l mod 32][j] and the B operand h1_j of its own input.
// Block b's result column c (input of lane 32b + c) is spread over lanes c
// and c + 32, 16 units each: accumulator register r of lane l holds unit
// 8 (r / 4) + 4 (l / 32) + r mod 4.  Each lane sums the output layer over
// its 16 units for both blocks and swaps the other block's partial sum with
// lane l xor 32.
__device__ __forceinline__ float mlp_eval_wave(const float* m0, float z) {
  // The model is re-read from LDS on every call: an opaque zero offset keeps
  // the compiler from holding all of it in registers across calls, which
  // would halve the wavefronts per SIMD that keep the matrix cores fed.
  int opaque = 0;
  asm volatile("" : "+s"(opaque));
  const float* m = m0 + opaque;
  const int lane = threadIdx.x & 63;
  const int row = lane & 31, hi = lane >> 5;
  const v4f* b2v = reinterpret_cast<const v4f*>(m + kMB2);
  const v4f* w3v = reinterpret_cast<const v4f*>(m + kMW3);
  const v4f* w1v = reinterpret_cast<const v4f*>(m + kMW1);
  const v4f* b1v = reinterpret_cast<const v4f*>(m + kMB1);
  const v4f* w2v = reinterpret_cast<const v4f*>(m + kMW2 + kW2Pitch * row);
  v32f acc;
#pragma unroll
  for (int t = 0; t < 4; ++t) {  // start from the bias of the units held
    const v4f b = b2v[2 * t + hi];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc[4 * t + u] = b[u];
      acc[16 + 4 * t + u] = b[u];
    }
  }
#pragma unroll
  for (int j4 = 0; j4 < kH / 4; ++j4) {
    const v4f w2 = w2v[j4], w1 = w1v[j4], b1 = b1v[j4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float h = fmaxf(fmaf(w1[u], z, b1[u]), 0.0f);
      acc = __builtin_amdgcn_mfma_f32_32x32x1f32(w2[u], h, acc, 0, 0, 0);
    }
  }
  float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const v4f w = w3v[2 * t + hi];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      s0 = fmaf(w[u], relu_bits(acc[4 * t + u]), s0);
      s1 = fmaf(w[u], relu_bits(acc[16 + 4 * t + u]), s1);
    }
  }
  const float own = hi ? s1 : s0, other = hi ? s0 : s1;
  return own + __shfl_xor(other, 32) + m[kMB3];
}

// Predicted index g = floor(p (n-1)) clamped to [-1, n-1].  Any p, even NaN
// or inf, yields a valid index (fmaxf/fminf return the bound for NaN).
__device__ __forceinline__ int predicted_index(float p, int n) {
  const float g = floorf(p * (float)(n - 1));
  return (int)fminf(fmaxf(g, -1.0f), (float)(n - 1));
}

// The verified window search for Q targets per lane (every lane of the
// wavefront calls it).  m is the model's LDS image.
template <int Q>
__device__ __forceinline__ void search_learned(const double* __restrict__ sa, int n,
                                               const float* m, int E, float u0, float inv,
                                               const double (&x)[Q], int (&r)[Q],
                                               int (&fell_back)[Q]) {
  float p[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) p[q] = mlp_eval_wave(m, model_input(x[q], u0, inv));
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
      // largest pos in [L+1, R+1] with a[pos-1] < x (all of a[..L] are < x)
      int pos = L + 1;
      for (int s = step; s >= 1; s >>= 1) {
        const int cand = pos + s;
        const int ridx = max(min(cand, R + 1) - 1, 0);
        pos = ((cand <= R + 1) & (sa[ridx] < x[q])) ? cand : pos;
      }
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
