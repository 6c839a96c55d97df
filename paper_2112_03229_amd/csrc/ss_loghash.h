// Logarithm hash (paper Sec. 3.4, Eq. 1-3) on the device.
//
// Eq. 1 chooses the base b so that |H| bins of width log_b 1 span the table:
// log2 b = (log2 Xmax - log2 Xmin) / |H|.  Eq. 2's key is
//   hash(x) = floor(log_b x) - floor(log_b Xmin) = floor(u(x) S + phi)
// with u(x) = log2 x - log2 Xmin, S = 1 / log2 b and phi = frac(log_b Xmin).
// u is formed in FP32 from the exact binary exponent and the FP32 log2 of
// the mantissa in [1, 2):  u = (e(x) - e(Xmin)) + (log2 m(x) - log2 m(Xmin)),
// accurate to about 1e-7 whatever the magnitude of x (a plain log2f of x
// would carry the absolute error of a number near log2 x, up to ~1e3).
// Keys are clamped to [0, |H| - 1] (Eq. 1 puts Xmax itself at |H|); x <= 0
// and subnormal x take bin 0.
//
// Every rounding step (double to float, the sums, the fused multiply-add,
// floor) is monotone, so the key is non-decreasing in x as long as the
// hardware log2 is; the search verifies its bracket anyway and falls back to
// bisection, so a non-monotone log2 could cost time but never correctness.
// The bin table is Eq. 3 in prefix-count form, C[i] = #{j : key(a_j) < i},
// built by the same gap filling as the exponent hash's.
#pragma once

#include "ss_device.h"

namespace ss {

struct LogHashParams {
  int ok;     // 1 if the table admits the log hash (0 < a[0] normal, a[0] < a[n-1] < inf)
  int nb;     // |H|
  int K;      // most entries in one bin (set by build_log_bins)
  int e0;     // biased exponent of Xmin
  float lm0;  // log2 of Xmin's mantissa
  float S;    // |H| / u(Xmax) = 1 / log2 b
  float phi;  // frac(log_b Xmin)
};

__device__ __forceinline__ float log_u(double x, int e0, float lm0) {
  const int hi = hi_word(x);
  const int e = (hi >> 20) & 0x7ff;
  const double m = __hiloint2double((hi & 0x000fffff) | 0x3ff00000, __double2loint(x));
  return (float)(e - e0) + (__log2f((float)m) - lm0);
}

__device__ __forceinline__ int log_key(double x, const LogHashParams& p) {
  const int hi = hi_word(x);
  const int e = (hi >> 20) & 0x7ff;
  float t = floorf(fmaf(log_u(x, p.e0, p.lm0), p.S, p.phi));
  t = fminf(fmaxf(t, 0.0f), (float)(p.nb - 1));  // NaN -> 0
  return (hi < 0 || e == 0) ? 0 : (int)t;
}

__device__ __forceinline__ float uniform_f(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Parameters for |H| = nb bins; uniform across the workgroup.  `a` may point
// to LDS or global memory.
__device__ __forceinline__ LogHashParams choose_loghash(const double* a, int n, int nb) {
  LogHashParams p{0, 0, 0, 0, 0.0f, 0.0f, 0.0f};
  if (n < 2 || nb < 1 || nb > 65535) return p;
  const double x0 = a[0], x1 = a[n - 1];
  if (!(x0 >= 0x1p-1022) || !(x1 > x0) || __builtin_isinf(x1)) return p;
  const int e0 = (hi_word(x0) >> 20) & 0x7ff;
  const double m0 = __hiloint2double((hi_word(x0) & 0x000fffff) | 0x3ff00000, __double2loint(x0));
  const float lm0 = __log2f((float)m0);
  const float u1 = log_u(x1, e0, lm0);
  if (!(u1 > 0.0f)) return p;
  const float S = (float)nb / u1;
  // log_b Xmin = log2 Xmin * S, in double; any phi in [0, 1) gives valid
  // bins as long as the build and the search use the same one
  const double lb0 = ((double)(e0 - 1023) + (double)lm0) * (double)S;
  float phi = (float)(lb0 - floor(lb0));
  phi = fminf(fmaxf(phi, 0.0f), 0x1.fffffep-1f);
  p.ok = 1;
  p.nb = __builtin_amdgcn_readfirstlane(nb);
  p.e0 = __builtin_amdgcn_readfirstlane(e0);
  p.lm0 = uniform_f(lm0);
  p.S = uniform_f(S);
  p.phi = uniform_f(phi);
  return p;
}

// C[0..nb] by gap filling (see build_bins) with the log key, one key
// evaluation per entry and one for its predecessor; then K, the most
// entries in one bin, from the finished table (max of C[b+1] - C[b], capped
// at SS_SCAN_MAX + 1).  `scratch` is one int; the whole workgroup calls.
template <typename CT>
__device__ __forceinline__ void build_log_bins(const double* __restrict__ sa, int n,
                                               LogHashParams& p, CT* __restrict__ C,
                                               int* scratch) {
  const int nt = blockDim.x, tid = threadIdx.x;
  if (tid == 0) *scratch = 0;
  for (int i = tid; i < n; i += nt) {
    const int kb = log_key(sa[i], p);
    const int kp = i == 0 ? -1 : log_key(sa[i - 1], p);
    for (int b = kp + 1; b <= kb; ++b) C[SS_IN(b, 0, p.nb + 1)] = (CT)i;
  }
  // bins past the last entry's key (the clamp keeps a[n-1] in nb - 1, so
  // only a table whose keys are not ordered leaves any) hold n
  if (tid == 0) C[p.nb] = (CT)n;
  __syncthreads();
  int run_max = 0;
  for (int b = tid; b < p.nb; b += nt)
    run_max = max(run_max, min((int)C[b + 1], n) - min((int)C[b], n));
  run_max = min(run_max, SS_SCAN_MAX + 1);
  for (int o = 32; o > 0; o >>= 1) run_max = max(run_max, __shfl_xor(run_max, o));
  if ((tid & 63) == 0) atomicMax(scratch, run_max);
  __syncthreads();
  p.K = __builtin_amdgcn_readfirstlane(*scratch);
}

// The search: key, C[key], then the count of entries below x inside the
// window that holds the key's bin -- a fixed K-step scan from C[key], or,
// for bins longer than SS_SCAN_MAX, a bisection inside [C[b], C[b+1]).  The
// count is idx(x) exactly when every entry before the window is below x and
// the entry after it is not; those two reads do not depend on the scan, and
// where either check fails (only possible if the hardware log2 were not
// monotone) a full bisection gives the answer.  NaN gives -1.
template <int Q>
__device__ __forceinline__ void search_loghash(const double* __restrict__ sa,
                                               const uint16_t* __restrict__ C, int n,
                                               const LogHashParams& p, const double (&x)[Q],
                                               int (&r)[Q]) {
  int b[Q], j0[Q], j1[Q];
  bool ok[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    b[q] = log_key(x[q], p);
    j0[q] = min((int)C[SS_IN(b[q], 0, p.nb + 1)], n);
  }
  if (p.K <= SS_SCAN_MAX) {
    int cnt[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      cnt[q] = 0;
      j1[q] = min(j0[q] + p.K, n);  // a[n] is the +inf sentinel
      ok[q] = (j0[q] == 0 || sa[max(j0[q] - 1, 0)] < x[q]) &&
              x[q] <= sa[SS_IN(j1[q], 0, n + SS_PAD)];
    }
#pragma nounroll
    for (int k = 0; k < p.K; ++k) {
#pragma unroll
      for (int q = 0; q < Q; ++q) cnt[q] += (sa[SS_IN(j0[q] + k, 0, n + SS_PAD)] < x[q]) ? 1 : 0;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) r[q] = j0[q] + cnt[q] - 1;
  } else {
    int pos[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      j1[q] = min(max((int)C[SS_IN(b[q] + 1, 0, p.nb + 1)], j0[q]), n);
      pos[q] = j0[q];
      ok[q] = (j0[q] == 0 || sa[max(j0[q] - 1, 0)] < x[q]) && x[q] <= sa[j1[q]];
    }
    int step = 1;
    while (step * 2 <= n) step *= 2;
    for (; step >= 1; step >>= 1) {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int cand = pos[q] + step;
        const int ridx = max(min(cand, j1[q]) - 1, 0);
        pos[q] = ((cand <= j1[q]) & (sa[SS_IN(ridx, 0, n + SS_PAD)] < x[q])) ? cand : pos[q];
      }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) r[q] = pos[q] - 1;
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (!ok[q] && x[q] == x[q]) {
      int base = 0, len = n;
      while (len > 1) {
        const int half = len >> 1;
        base = (sa[SS_IN(base + half, 0, n + SS_PAD)] < x[q]) ? base + half : base;
        len -= half;
      }
      r[q] = base + (sa[SS_IN(base, 0, n + SS_PAD)] < x[q] ? 1 : 0) - 1;
    }
    if (x[q] != x[q]) r[q] = -1;
  }
}

}  // namespace ss
