// Device code of the learned index's model, shared by the single-table
// learned search, the error bound and the plan kernels: parameter layout,
// model input, the compiled (piecewise-linear) forward pass, predicted index
// and the verified window search.
#pragma once

#include "ss_device.h"
#include "../../include/searchsorted.h"

namespace ss {

constexpr int kH = 32;
constexpr int kOffW1 = 0, kOffB1 = 32, kOffW2 = 64, kOffB2 = 64 + kH * kH, kOffW3 = kOffB2 + kH,
              kOffB3 = kOffW3 + kH, kNP = kOffB3 + 1;
static_assert(kNP == SS_MLP_PARAMS, "parameter layout");
constexpr int kTrainThreads = 256;  // also the batch size

typedef float v4f __attribute__((ext_vector_type(4)));  // matrix-core accumulator (training)

// Model input: z = (log2 x - u0) * inv, in FP32 from x rounded to FP32.
__device__ __forceinline__ float model_input(double x, float u0, float inv) {
  return (__log2f((float)x) - u0) * inv;
}

// The forward pass as the search evaluates it.  With one input z the
// network is a piecewise-linear function of z, and it is evaluated in that
// form.  Unit j of layer 1 switches at its breakpoint t_j = -b1_j / w1_j;
// between two consecutive breakpoints the set of active layer-1 units is
// fixed, so layer 2's pre-activations are linear there, g_k(z) = P_k z +
// Q_k, and each switches at most once inside the segment (at -Q_k / P_k).
// Between consecutive switching points of either layer the active sets of
// both layers are fixed and the output is one line,
//   p(z) = b3 + sum_{k active} w3_k (P_k z + Q_k) = slope z + intercept.
// compile_model lists these pieces once per model (at most 33 segments of
// at most 33 pieces): the sorted boundaries and one (slope, intercept) per
// piece, formed in float64 and rounded once.  A query then finds its piece,
// i = #{boundaries < z}, and costs one fused multiply-add: the same
// function as the 1088 multiply-adds of the layered form, up to FP32
// rounding.  The piece is found through a table of G equal cells over the
// boundaries' range (the idea of the logarithm hash, applied to z):
// C[c] counts the boundaries in cells before c, so i = C[cell(z)] plus a
// scan of at most K boundaries from there.  cell() is monotone and the
// same FP32 expression for boundaries and queries, so every boundary in an
// earlier cell is below z and every one in a later cell is not.  A model
// whose fullest cell holds more than kCellScan boundaries has no table
// (G = 0) and is searched by bisection over the boundaries.
//
// Image layout (floats; identical in global memory and LDS):
//   [0] nbp   boundary slots: a power of two >= nb + kCellScan (int bits)
//   [1] np    pieces; nb = np - 1 real boundaries (int bits)
//   [2] G     cells (0: none) (int bits)
//   [3] K     most boundaries in one cell, <= kCellScan (int bits)
//   [4] z0, [5] cinv   cell(z) = clamp((z - z0) * cinv, 0, G - 1), truncated
//   [6] coff  first float of the cell table (int bits)
//   [8, 8 + nbp)          boundaries, ascending, padded with +inf
//   [8 + nbp, + 2 np)     np pairs (slope, intercept)
//   [coff, ...)           G + 1 uint16 prefix counts C[0..G]
constexpr int kIHead = 8;
constexpr int kISegments = kH + 1;  // layer-1 segments: at most 32 breakpoints
constexpr int kIMaxPieces = (kH + 1) * (kH + 1);
constexpr int kCellScan = 8;        // longest in-cell scan; fuller tables bisect
constexpr int kIMaxBounds = 2048;   // a power of two >= kIMaxPieces - 1 + kCellScan
constexpr int kIMaxCells = 2048;
constexpr int kImageFloats =
    (kIHead + kIMaxBounds + 2 * kIMaxPieces + (kIMaxCells + 2) / 2 + 3) / 4 * 4;
constexpr int kImageBytes = kImageFloats * 4;
static_assert(kImageBytes % 16 == 0, "16-byte copies");
static_assert(kIMaxPieces - 1 + kCellScan <= kIMaxBounds, "boundary slots");

// Floats in use of an image (a multiple of 4, for 16-byte staging).
__host__ __device__ constexpr int image_used_floats(int nbp, int np, int G) {
  return (kIHead + nbp + 2 * np + (G > 0 ? (G + 2) / 2 : 0) + 3) / 4 * 4;
}

// The first four header words (nbp, np, G, K) of a compiled image, as the
// host reads them back: true if they describe an image that fits the slot.
inline bool image_header_valid(const int* head) {
  const int nbp = head[0], np = head[1], G = head[2], K = head[3];
  const bool pow2_nbp = nbp >= 2 && nbp <= kIMaxBounds && (nbp & (nbp - 1)) == 0;
  const bool cells_ok = G == 0 ? K == 0 : (G >= 2 && G <= kIMaxCells && (G & (G - 1)) == 0 &&
                                           K >= 1 && K <= kCellScan);
  return pow2_nbp && np >= 1 && np <= kIMaxPieces && np - 1 + kCellScan <= nbp && cells_ok;
}

__device__ __forceinline__ int image_floats(const float* img) {
  return image_used_floats(__float_as_int(img[0]), __float_as_int(img[1]),
                           __float_as_int(img[2]));
}

// Copies the used part of a compiled image into LDS with 16-byte loads;
// called by every thread of the workgroup, followed by a barrier before use.
__device__ __forceinline__ void stage_image(float* m, const float* __restrict__ img) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const int count = __builtin_amdgcn_readfirstlane(image_floats(img)) / 4;
  const f4* src = reinterpret_cast<const f4*>(img);
  f4* dst = reinterpret_cast<f4*>(m);
  for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = src[i];
}

// The header of a staged image, uniform across the workgroup (read after
// the barrier that follows stage_image).
struct ImageHead {
  int nbp, G, K, coff;
  float z0, cinv;
};

__device__ __forceinline__ ImageHead image_head(const float* m) {
  ImageHead h;
  h.nbp = __builtin_amdgcn_readfirstlane(__float_as_int(m[0]));
  h.G = __builtin_amdgcn_readfirstlane(__float_as_int(m[2]));
  h.K = __builtin_amdgcn_readfirstlane(__float_as_int(m[3]));
  h.z0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(m[4])));
  h.cinv = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(m[5])));
  h.coff = __builtin_amdgcn_readfirstlane(__float_as_int(m[6]));
  return h;
}

// Cell of a boundary or an input (G > 0): monotone non-decreasing in v, NaN
// to cell 0.  Compilation and search must evaluate exactly this expression.
__device__ __forceinline__ int cell_of(float v, float z0, float cinv, int G) {
  float t = (v - z0) * cinv;
  t = fminf(fmaxf(t, 0.0f), (float)(G - 1));
  return (int)t;
}

// The model's outputs p(z) for Q inputs per lane from a compiled image in
// LDS: piece i = #{boundaries < z} (0 for NaN), then one fused
// multiply-add.  Both lookups (the cell scan, or the bisection over the
// nbp slots) have uniform trip counts and issue the Q lanes' reads of each
// step together.  Lanes are independent.
template <int Q>
__device__ __forceinline__ void mlp_eval_q(const float* m, const ImageHead& h,
                                           const float (&z)[Q], float (&p)[Q]) {
  const float* b = m + kIHead;
  int i[Q];
  if (h.G > 0) {
    const uint16_t* C = reinterpret_cast<const uint16_t*>(m + h.coff);
    int base[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      base[q] = C[SS_IN(cell_of(z[q], h.z0, h.cinv, h.G), 0, h.G + 1)];
      i[q] = base[q];
    }
    // base + k < nb + kCellScan <= nbp: reads past the cell's boundaries
    // meet later cells' boundaries (not below z) or the +inf padding
    if (h.K <= 2) {  // uniform: both boundaries from one two-word read
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int k = SS_IN(base[q], 0, h.nbp - 1);
        i[q] += (b[k] < z[q] ? 1 : 0) + (b[k + 1] < z[q] ? 1 : 0);
      }
    } else {
      for (int k = 0; k < h.K; ++k) {
#pragma unroll
        for (int q = 0; q < Q; ++q) i[q] += (b[SS_IN(base[q] + k, 0, h.nbp)] < z[q]) ? 1 : 0;
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) i[q] = 0;
    for (int step = h.nbp >> 1; step >= 1; step >>= 1) {
#pragma unroll
      for (int q = 0; q < Q; ++q)
        i[q] = (b[SS_IN(i[q] + step - 1, 0, h.nbp)] < z[q]) ? i[q] + step : i[q];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) i[q] += (b[SS_IN(i[q], 0, h.nbp)] < z[q]) ? 1 : 0;
  }
  typedef float f2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const f2 sq = *reinterpret_cast<const f2*>(m + kIHead + h.nbp + 2 * SS_IN(i[q], 0, h.nbp));
    p[q] = fmaf(sq.x, z[q], sq.y);
  }
}

__device__ __forceinline__ float mlp_eval(const float* m, const ImageHead& h, float z) {
  const float zq[1] = {z};
  float p[1];
  mlp_eval_q<1>(m, h, zq, p);
  return p[0];
}

// Predicted index g = floor(p (n-1)) clamped to [-1, n-1].  Any p, even NaN
// or inf, yields a valid index (fmaxf/fminf return the bound for NaN).
__device__ __forceinline__ int predicted_index(float p, int n) {
  const float g = floorf(p * (float)(n - 1));
  return (int)fminf(fmaxf(g, -1.0f), (float)(n - 1));
}

// How search_learned may read the table sa:
//   kWinGlobal : in place in global memory, no sentinels: every read is
//                clamped into [0, n);
//   kWinPadded : staged in LDS with SS_PAD +inf entries from a[n] on (plans);
//   kWinBounded: staged with window_front(E) -inf entries before a[0] and
//                window_tail(E) +inf entries from a[n] on, so that the
//                window's end checks and steps need no clamps or branches.
constexpr int kWinGlobal = 0, kWinPadded = 1, kWinBounded = 2;

// The window bisection's first step for a bound E: the largest power of
// two <= 2E + 1, so that its 2 step positions cover the 2E + 1 of [g - E,
// g + E].
__host__ __device__ constexpr int window_step(int E) {
  int s = 1;
  while (s * 2 <= 2 * E + 1) s *= 2;
  return s;
}

// A kWinBounded window is [L, L + 2 step - 1], L = g - E for a predicted g
// in [-1, n - 1], read without clamping: its lower check reads a[L] >=
// a[-E - 1], its upper check a[L + 2 step] <= a[n - 1 - E + 2 step].  The
// steps read from a[L] at most one step ahead of an entry below the target
// (or of a[L]): step s <= 2E + 1 at first, s <= E after that, and every
// entry below a non-NaN target lies at or before a[n - 1], so no step
// reads past a[n - 1 + 2 step - E] either.
__host__ __device__ constexpr int window_front(int E) { return E + 1; }
__host__ __device__ constexpr int window_tail(int E) {
  return 2 * window_step(E) - E > SS_PAD ? 2 * window_step(E) - E : SS_PAD;
}
// Bytes before a[0] of a bounded region: the front, rounded up to 16.
__host__ __device__ constexpr int window_lead(int E) { return (window_front(E) * 8 + 15) / 16 * 16; }

// The verified window search for Q targets per lane.  m is the model's
// compiled image in LDS, h its header, sa the table read as MODE says.
// fell[q] is the wave's mask of lanes whose target q took the fallback;
// called by every lane of the wave.
template <int Q, int MODE = kWinPadded>
__device__ __forceinline__ void search_learned(const double* __restrict__ sa, int n,
                                               const float* m, const ImageHead& h, int E,
                                               float u0, float inv, const double (&x)[Q],
                                               int (&r)[Q], uint64_t (&fell)[Q]) {
  float z[Q], p[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) z[q] = model_input(x[q], u0, inv);
  mlp_eval_q<Q>(m, h, z, p);
  const int step = window_step(E);  // >= half the window length
  unsigned ok = 0;  // bit q: target q's window was verified
  // Window search, all Q together.  If the window is verified, pos = #{a <
  // x} lies in [L+1, R+1]: every entry up to a[L] is below x and every
  // entry from a[R+1] on is not, so the steps need no upper bound (a read
  // at or past R+1 never advances pos; a read past the table counts as
  // +inf: the sentinel a[n], or an explicit test without one).
  // 2 step - 1 >= R - L covers the window (R = g + E, or L + 2 step - 1 for
  // a bounded table).  Lanes whose window failed run the same steps
  // harmlessly and are redone below.
  // The steps track r = pos - 1 as a byte offset into the table, which
  // saves the index arithmetic of each step (the kernel is vector-bound);
  // with the bounded table as the entry's 32-bit LDS address itself, one
  // add per step.
  const char* sb = reinterpret_cast<const char*>(sa);
  if constexpr (MODE == kWinBounded) {
    typedef const char __attribute__((address_space(3))) lds_char;
    typedef const double __attribute__((address_space(3))) lds_double;
    lds_char* const lb = (lds_char*)sb;
    lds_char* const lw = lb - 8 * E;  // &a[g - E] for g = 0
    const int span = 16 * step;  // from a[L] to a[R + 1], R + 1 = L + 2 step
    lds_char* pb[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      pb[q] = lw + 8 * predicted_index(p[q], n);  // &a[L], L = g - E >= -E - 1
      SS_ASSERT(pb[q] >= lb - 8 * window_front(E) && pb[q] + span < lb + 8 * (n + window_tail(E)));
      const bool lo_ok = *(lds_double*)pb[q] < x[q];
      const bool hi_ok = x[q] <= *(lds_double*)(pb[q] + span);
      ok |= (lo_ok && hi_ok) ? 1u << q : 0u;
      fell[q] = __builtin_amdgcn_ballot_w64(!(lo_ok && hi_ok));
    }
    for (int s8 = step * 8; s8 >= 8; s8 >>= 1) {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        lds_char* kp = pb[q] + s8;  // &a[k]: inside the staged front and tail
        SS_ASSERT(kp >= lb - 8 * window_front(E) && kp < lb + 8 * (n + window_tail(E)));
        pb[q] = *(lds_double*)kp < x[q] ? kp : pb[q];
      }
    }
    // a verified window ends on the last entry below x: a[-1] (-inf) at the
    // lowest
#pragma unroll
    for (int q = 0; q < Q; ++q) r[q] = (int)(pb[q] - lb) >> 3;
  } else {
    int rb[Q];
    const int n8 = n * 8;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int g = predicted_index(p[q], n);
      const int L = max(g - E, -1), R = min(g + E, n - 1);
      const bool lo_ok = L < 0 || sa[SS_IN(max(L, 0), 0, n)] < x[q];
      const bool hi_ok = R >= n - 1 || x[q] <= sa[SS_IN(min(R + 1, n - 1), 0, n)];
      ok |= (lo_ok && hi_ok) ? 1u << q : 0u;
      fell[q] = __builtin_amdgcn_ballot_w64(!(lo_ok && hi_ok));
      rb[q] = L * 8;  // (pos - 1) * 8, pos = L + 1
    }
    for (int s8 = step * 8; s8 >= 8; s8 >>= 1) {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int kb = rb[q] + s8;  // a[k], k = pos + s - 1 >= 0
        bool lt;
        if constexpr (MODE == kWinPadded) {
          SS_ASSERT(kb >= 0);  // min(kb, n8) reads a[0..n], a[n] the sentinel
          lt = *reinterpret_cast<const double*>(sb + min(kb, n8)) < x[q];
        } else {
          SS_ASSERT(kb >= 0);  // min(kb, n8 - 8) reads a[0..n-1]
          lt = kb < n8 && *reinterpret_cast<const double*>(sb + min(kb, n8 - 8)) < x[q];
        }
        rb[q] = lt ? kb : rb[q];
      }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) r[q] = rb[q] >> 3;
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (!((ok >> q) & 1u)) {  // fallback: bisection over the whole table
      int base = 0, len = n;
      while (len > 1) {
        const int half = len >> 1;
        base = (sa[SS_IN(base + half, 0, n)] < x[q]) ? base + half : base;
        len -= half;
      }
      r[q] = base + (sa[SS_IN(base, 0, n)] < x[q] ? 1 : 0) - 1;
    }
  }
}

}  // namespace ss
