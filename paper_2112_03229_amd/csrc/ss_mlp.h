// Device code of the learned index's model, shared by the single-table
// learned search and the plan kernels: parameter layout, model input,
// forward pass, predicted index and the verified window search.
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

// Forward pass for Q inputs at once (the search's and the bound's code).
// P points to the 1153 parameters in any address space; the search passes a
// constant-address-space pointer so that they are read with scalar loads.
template <int Q, typename PT>
__device__ __forceinline__ void mlp_eval(PT P, const float (&z)[Q], float (&out)[Q]) {
  float h1[Q][kH];
#pragma unroll
  for (int j = 0; j < kH; ++j) {
    const float w = P[kOffW1 + j], b = P[kOffB1 + j];
#pragma unroll
    for (int q = 0; q < Q; ++q) h1[q][j] = fmaxf(fmaf(w, z[q], b), 0.0f);
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) out[q] = P[kOffB3];
  // one row of layer-2 weights per iteration (rolled loop): only 32
  // parameters are live in SGPRs at a time
#pragma nounroll
  for (int k = 0; k < kH; ++k) {
    float acc[Q];
    const float b2 = P[kOffB2 + k];
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] = b2;
#pragma unroll
    for (int j = 0; j < kH; ++j) {
      const float w = P[kOffW2 + kH * k + j];
#pragma unroll
      for (int q = 0; q < Q; ++q) acc[q] = fmaf(w, h1[q][j], acc[q]);
    }
    const float w3 = P[kOffW3 + k];
#pragma unroll
    for (int q = 0; q < Q; ++q) out[q] = fmaf(w3, fmaxf(acc[q], 0.0f), out[q]);
  }
}

// Predicted index g = floor(p (n-1)) clamped to [-1, n-1].  Any p, even NaN
// or inf, yields a valid index (fmaxf/fminf return the bound for NaN).
__device__ __forceinline__ int predicted_index(float p, int n) {
  const float g = floorf(p * (float)(n - 1));
  return (int)fminf(fmaxf(g, -1.0f), (float)(n - 1));
}

typedef const __attribute__((address_space(4))) float* ConstFloatPtr;

template <int Q>
__device__ __forceinline__ void search_learned(const double* __restrict__ sa, int n,
                                               ConstFloatPtr P, int E, float u0,
                                               float inv, const double (&x)[Q], int (&r)[Q],
                                               int (&fell_back)[Q]) {
  float z[Q], p[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) z[q] = model_input(x[q], u0, inv);
  mlp_eval<Q>(P, z, p);
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
