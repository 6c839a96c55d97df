// Learned index: an FP32 1-32-32-1 ReLU position model per table, trained on
// the device on the table's CDF, with a device-measured error bound and a
// verified bounded search (exact by construction; bisection is the fallback).
//
// Kernels:
//   train_kernel   one workgroup per table: full-batch Adam, points in
//                  batches of 256 (one per lane); per batch, phase A stores
//                  each point's activations and back-propagated errors in
//                  LDS, phase B sums every parameter's gradient over the
//                  batch in a fixed order (deterministic): the 1024 W2
//                  gradients as a 32 x 256 x 32 product on the matrix
//                  cores, the other 129 one thread each.
//   compile_kernel the trained model as the search evaluates it: the
//                  network is piecewise linear in its one input, so it is
//                  listed as its pieces (sorted boundaries and one slope
//                  and intercept each, formed in float64, rounded once).
//   bound_kernel   E = 1 + max |g(x) - idx(x)| over the probes, with the
//                  compiled model.
//   learned_kernel the search: table and compiled model in LDS, Q targets
//                  per lane.
//   predict_kernel the model's fractional position for inspection.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ss_device.h"
#include "ss_host.h"
#include "ss_mlp.h"
#include "ss_learned.h"

namespace ss {

// ---------------------------------------------------------------------------
// Training.
// ---------------------------------------------------------------------------

struct TrainArgs {
  const double* table;   // the table's first entry
  int n;
  int steps;       // 0 with grad_out set: one gradient only
  float lr;
  uint64_t seed;
  float u0, inv;
  float* params;   // [kNP] in: initial values unless init_from_seed; out: trained
  int init_from_seed;
  float* grad_out; // [kNP] or null
  float* loss_out; // [1]: final loss (mean squared error)
};

__device__ __forceinline__ float uhash(uint64_t seed, uint64_t i) {
  uint64_t z = seed * 0x9e3779b97f4a7c15ULL + (i + 1) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  z ^= z >> 31;
  return (float)(z >> 40) * 0x1.0p-24f;  // [0, 1)
}

// Rows of the per-point arrays are padded to 33 floats: a lane writing its
// own row then hits a different bank from its neighbours.
constexpr int kRow = kH + 1;

struct TrainLds {
  float P[kNP];
  float m[kNP];
  float v[kNP];
  float h1[kTrainThreads][kRow];
  float h2[kTrainThreads][kRow];
  float d2[kTrainThreads][kRow];   // dLoss / d(pre-activation of layer 2)
  float d1[kTrainThreads][kRow];   // dLoss / d(pre-activation of layer 1)
  float z[kTrainThreads];
  float g[kTrainThreads];          // dLoss / dp
  float red[kTrainThreads];
};

// Trains (or, with steps == 0, differentiates) one table's model; called by
// a whole workgroup of kTrainThreads lanes.
__device__ void train_body(TrainLds& L, const TrainArgs& a) {
  const int tid = threadIdx.x;
  const int n = a.n;
  for (int i = tid; i < kNP; i += kTrainThreads) {
    float val;
    if (a.init_from_seed) {
      const float u = uhash(a.seed, (uint64_t)i);
      if (i < kOffB1) {                 // slopes: +-(0.5 .. 4.5)
        const float sgn = uhash(a.seed ^ 0x5bd1e995ULL, (uint64_t)i) < 0.5f ? -1.0f : 1.0f;
        val = sgn * (0.5f + 4.0f * u);
      } else if (i < kOffW2) {          // ReLU kinks spread over z in [0, 1]
        const int j = i - kOffB1;
        const float sgn = uhash(a.seed ^ 0x5bd1e995ULL, (uint64_t)j) < 0.5f ? -1.0f : 1.0f;
        const float w = sgn * (0.5f + 4.0f * uhash(a.seed, (uint64_t)j));
        val = -w * u;
      } else if (i < kOffB2) {
        val = (2.0f * u - 1.0f) * 0.4330127f;  // sqrt(6 / 32)
      } else if (i < kOffW3) {
        val = 0.1f;
      } else if (i < kOffB3) {
        val = (2.0f * u - 1.0f) * 0.4330127f;
      } else {
        val = 0.5f;
      }
    } else {
      val = a.params[i];
    }
    L.P[i] = val;
    L.m[i] = 0.0f;
    L.v[i] = 0.0f;
  }
  __syncthreads();
  const float inv_n = 1.0f / (float)n;
  const float inv_nm1 = 1.0f / (float)(n - 1);
  const int nbatch = (n + kTrainThreads - 1) / kTrainThreads;
  const int total_steps = a.steps > 0 ? a.steps : 1;
  // Gradient ownership: wave w holds the W2 gradients of the 16 x 16
  // quadrant (units k in [16 (w / 2), +16), inputs j in [16 (w mod 2), +16))
  // in the accumulator of a v_mfma_f32_16x16x4f32 chain, lane l's register r
  // being entry (k0 + 4 (l / 16) + r, j0 + l mod 16); threads 0..128 hold
  // the other 129 parameters' gradients (w1, b1, b2, w3, b3).
  static_assert(kTrainThreads == 256, "four wavefronts, one W2 quadrant each");
  const int wave = tid >> 6, lane = tid & 63;
  const int k0 = (wave >> 1) * 16, j0 = (wave & 1) * 16;
  const int small_pi = tid < 64 ? tid : tid < 96 ? kOffB2 + (tid - 64)
                     : tid < 128 ? kOffW3 + (tid - 96) : kOffB3;
  for (int step = 1; step <= total_steps; ++step) {
    v4f gw2 = {0.0f, 0.0f, 0.0f, 0.0f};
    float gsmall = 0.0f;
    float sq = 0.0f;
    for (int bt = 0; bt < nbatch; ++bt) {
      // phase A: one point per lane.  Loops over units are rolled so that
      // only h1 and the back-propagated sums live in registers; the rest of
      // each point's activations goes straight to its LDS row.
      const int i = bt * kTrainThreads + tid;
      float* h1row = L.h1[tid];
      float* h2row = L.h2[tid];
      float* d1row = L.d1[tid];
      float* d2row = L.d2[tid];
      if (i < n) {
        const float zi = model_input(a.table[i], a.u0, a.inv);
        float h1[kH];
#pragma unroll
        for (int j = 0; j < kH; ++j) {
          h1[j] = fmaxf(fmaf(L.P[kOffW1 + j], zi, L.P[kOffB1 + j]), 0.0f);
          h1row[j] = h1[j];
        }
        float p = L.P[kOffB3];
#pragma nounroll
        for (int k = 0; k < kH; ++k) {
          float acc = L.P[kOffB2 + k];
#pragma unroll
          for (int j = 0; j < kH; ++j) acc = fmaf(L.P[kOffW2 + kH * k + j], h1[j], acc);
          const float h2k = fmaxf(acc, 0.0f);
          h2row[k] = h2k;
          p = fmaf(L.P[kOffW3 + k], h2k, p);
        }
        const float err = p - (float)i * inv_nm1;
        sq = fmaf(err, err, sq);
        const float gi = 2.0f * err * inv_n;
        float s[kH];
#pragma unroll
        for (int j = 0; j < kH; ++j) s[j] = 0.0f;
#pragma nounroll
        for (int k = 0; k < kH; ++k) {
          const float d2k = h2row[k] > 0.0f ? gi * L.P[kOffW3 + k] : 0.0f;
          d2row[k] = d2k;
#pragma unroll
          for (int j = 0; j < kH; ++j) s[j] = fmaf(L.P[kOffW2 + kH * k + j], d2k, s[j]);
        }
#pragma unroll
        for (int j = 0; j < kH; ++j) d1row[j] = h1[j] > 0.0f ? s[j] : 0.0f;
        L.z[tid] = zi;
        L.g[tid] = gi;
      } else {
#pragma unroll
        for (int j = 0; j < kH; ++j) {
          h1row[j] = 0.0f;
          h2row[j] = 0.0f;
          d1row[j] = 0.0f;
          d2row[j] = 0.0f;
        }
        L.z[tid] = 0.0f;
        L.g[tid] = 0.0f;
      }
      __syncthreads();
      // phase B: gradients summed over the batch in a fixed order.  W2 (1024
      // entries): G[k][j] += sum_t d2[t][k] h1[t][j] as rank-4 MFMA steps
      // over the batch's rows (rows past the table's end hold zeros).
      const int rows = min(kTrainThreads, n - bt * kTrainThreads);
      for (int t4 = 0; t4 < rows; t4 += 4) {
        const int t = t4 + (lane >> 4);
        gw2 = __builtin_amdgcn_mfma_f32_16x16x4f32(L.d2[t][k0 + (lane & 15)],
                                                   L.h1[t][j0 + (lane & 15)], gw2, 0, 0, 0);
      }
      if (tid <= 128) {
        float s = 0.0f;
        if (tid < 32) {
          for (int t = 0; t < rows; ++t) s = fmaf(L.d1[t][tid], L.z[t], s);
        } else if (tid < 64) {
          for (int t = 0; t < rows; ++t) s += L.d1[t][tid - 32];
        } else if (tid < 96) {
          for (int t = 0; t < rows; ++t) s += L.d2[t][tid - 64];
        } else if (tid < 128) {
          for (int t = 0; t < rows; ++t) s = fmaf(L.g[t], L.h2[t][tid - 96], s);
        } else {
          for (int t = 0; t < rows; ++t) s += L.g[t];
        }
        gsmall += s;
      }
      __syncthreads();
    }
    if (a.steps <= 0 || step == total_steps) {
      // loss: fixed-order tree reduction of the lanes' sums
      L.red[tid] = sq;
      __syncthreads();
      for (int o = kTrainThreads / 2; o > 0; o >>= 1) {
        if (tid < o) L.red[tid] += L.red[tid + o];
        __syncthreads();
      }
      if (tid == 0 && a.loss_out) a.loss_out[0] = L.red[0] * inv_n;
      __syncthreads();
    }
    if (a.steps <= 0) {
      if (a.grad_out) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          a.grad_out[kOffW2 + kH * (k0 + 4 * (lane >> 4) + r) + j0 + (lane & 15)] = gw2[r];
        if (tid <= 128) a.grad_out[small_pi] = gsmall;
      }
      break;
    }
    // Adam with bias correction and a cosine-decayed rate, each parameter
    // updated by the thread that holds its gradient
    const float lr_t = a.lr * 0.5f * (1.0f + cosf(3.14159265f * (float)(step - 1) / (float)total_steps));
    const float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
    auto adam = [&](int pi, float gr) {
      const float mm = 0.9f * L.m[pi] + 0.1f * gr;
      const float vv = 0.999f * L.v[pi] + 0.001f * gr * gr;
      L.m[pi] = mm;
      L.v[pi] = vv;
      L.P[pi] -= lr_t * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
    };
#pragma unroll
    for (int r = 0; r < 4; ++r)
      adam(kOffW2 + kH * (k0 + 4 * (lane >> 4) + r) + j0 + (lane & 15), gw2[r]);
    if (tid <= 128) adam(small_pi, gsmall);
    __syncthreads();
  }
  for (int i = tid; i < kNP; i += kTrainThreads) a.params[i] = L.P[i];
}


__global__ __launch_bounds__(kTrainThreads) void train_kernel(TrainArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  train_body(*reinterpret_cast<TrainLds*>(lds_raw), a);
}

// One workgroup per slot (table) of a plan: trains every model at once.
__global__ __launch_bounds__(kTrainThreads) void train_many_kernel(
    const double* tables_a, const double* tables_b, const LearnedSlot* slots, float* params,
    int steps, float lr, uint64_t seed) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const LearnedSlot sl = slots[blockIdx.x];
  TrainArgs a{(sl.which ? tables_b : tables_a) + sl.tab_off, sl.n, steps, lr,
              seed ^ (0x9e3779b97f4a7c15ULL * (uint64_t)(blockIdx.x + 1)), sl.u0, sl.inv,
              params + (int64_t)blockIdx.x * kNP, 1, nullptr, nullptr};
  train_body(*reinterpret_cast<TrainLds*>(lds_raw), a);
}

// ---------------------------------------------------------------------------
// Compilation of a trained model into the image the search evaluates (the
// piecewise-linear form, the cell table and the layout are described with
// mlp_eval_q).
// ---------------------------------------------------------------------------

// Midpoint of (lo, hi) with infinite ends: a point inside the interval
// (either end may be +-inf; an interval with both ends infinite gives 0).
__device__ __forceinline__ double inside(double lo, double hi) {
  const double inf = __builtin_inf();
  if (lo == -inf && hi == inf) return 0.0;
  if (lo == -inf) return hi - fmax(1.0, fabs(hi));
  if (hi == inf) return lo + fmax(1.0, fabs(lo));
  return 0.5 * lo + 0.5 * hi;
}

// One workgroup (at least 64 threads) compiles one model: P holds the kNP
// parameters in the standard layout, img receives the image described with
// mlp_eval.  Everything is formed in float64 and rounded once:
//   1. layer 1's breakpoints t_j = -b1_j / w1_j, sorted; a unit without one
//      (w1_j = 0, or a NaN) is active exactly when b1_j > 0;
//   2. per segment s between consecutive breakpoints (at most 33), the
//      active layer-1 units at a point inside it and layer 2's lines
//      g_k = P_sk z + Q_sk;
//   3. per segment, the points -Q_sk / P_sk strictly inside it where a
//      layer-2 unit switches, sorted;
//   4. the pieces, segment by segment: boundaries in order (each segment's
//      switching points, then the segment's right breakpoint), and per
//      piece the active layer-2 units at a point inside it, giving
//      slope = sum w3_k P_sk and intercept = b3 + sum w3_k Q_sk;
//   5. the cell table: G (a power of two >= 2 nb, at most kIMaxCells,
//      the smallest that gives the shortest scan)
//      equal cells over the boundaries' range less its outermost few, each
//      boundary's cell from the FP32 expression the search uses, the prefix
//      counts by gap filling, and K, the fullest cell (no table if
//      K > kCellScan).
// Breakpoints beyond the FP32 range round to +-inf, which leaves the piece
// of every FP32 input unchanged.
__device__ void compile_model(const float* __restrict__ P, float* __restrict__ img) {
  constexpr int S = kISegments;
  __shared__ double bp[kH], ts[kH];
  __shared__ unsigned act[S];
  __shared__ double ps[S][kH], qs[S][kH], cr[S][kH], crs[S][kH];
  __shared__ int ncr[S], poff[S + 1], m_s, nbp_s;
  __shared__ float bnd[kIMaxBounds];
  __shared__ int cells[kIMaxCells + 1];
  __shared__ int G_s, K_s;
  __shared__ float z0_s, cinv_s;
  const int tid = threadIdx.x, nt = blockDim.x;
  const double inf = __builtin_inf();
  if (tid < kH) {
    const double w = P[kOffW1 + tid], b = P[kOffB1 + tid];
    const double t = -b / w;
    bp[tid] = (w != 0.0 && t == t) ? t : inf;
  }
  __syncthreads();
  if (tid < kH) {  // rank by (breakpoint, unit): a permutation of 0..31
    const double t = bp[tid];
    int rank = 0;
    for (int i = 0; i < kH; ++i) rank += (bp[i] < t || (bp[i] == t && i < tid)) ? 1 : 0;
    ts[rank] = t;
  }
  if (tid == 0) {
    int c = 0;
    for (int i = 0; i < kH; ++i) c += bp[i] < inf ? 1 : 0;
    m_s = c;
  }
  __syncthreads();
  const int m = m_s;
  // 2. active layer-1 units and layer 2's lines per segment
  if (tid < S) {
    const double z = inside(tid == 0 || m == 0 ? -inf : ts[min(tid, m) - 1],
                            tid >= m ? inf : ts[tid]);
    unsigned mask = 0;
    for (int j = 0; j < kH; ++j) {
      const double w = P[kOffW1 + j], b = P[kOffB1 + j];
      const bool on = bp[j] < inf ? w * z + b > 0.0 : b > 0.0;
      mask |= on ? 1u << j : 0u;
    }
    act[tid] = mask;
  }
  __syncthreads();
  for (int i = tid; i < S * kH; i += nt) {
    const int seg = i / kH, k = i % kH;
    const unsigned mask = act[seg];
    double pk = 0.0, qk = P[kOffB2 + k];
    for (int j = 0; j < kH; ++j) {
      if ((mask >> j) & 1u) {
        const double w2 = P[kOffW2 + k * kH + j];
        pk += w2 * (double)P[kOffW1 + j];
        qk += w2 * (double)P[kOffB1 + j];
      }
    }
    ps[seg][k] = pk;
    qs[seg][k] = qk;
    // 3. where unit k switches strictly inside the segment (+inf if not)
    const double lo = seg == 0 || m == 0 ? -inf : ts[min(seg, m) - 1];
    const double hi = seg >= m ? inf : ts[seg];
    const double c = -qk / pk;
    cr[seg][k] = (seg <= m && pk != 0.0 && c > lo && c < hi) ? c : inf;
  }
  __syncthreads();
  for (int i = tid; i < S * kH; i += nt) {  // sort each segment's points
    const int seg = i / kH, k = i % kH;
    const double c = cr[seg][k];
    int rank = 0;
    for (int j = 0; j < kH; ++j) rank += (cr[seg][j] < c || (cr[seg][j] == c && j < k)) ? 1 : 0;
    crs[seg][rank] = c;
  }
  if (tid < S) {
    int c = 0;
    for (int j = 0; j < kH; ++j) c += cr[tid][j] < inf ? 1 : 0;
    ncr[tid] = c;
  }
  __syncthreads();
  if (tid == 0) {  // pieces of segment s start at poff[s]
    poff[0] = 0;
    for (int seg = 0; seg < S; ++seg) poff[seg + 1] = poff[seg] + (seg <= m ? ncr[seg] + 1 : 0);
    const int nb = poff[S] - 1;
    int nbp = 2;
    while (nbp < nb + kCellScan) nbp <<= 1;  // the cell scan may read kCellScan - 1 past
    nbp_s = nbp;
  }
  __syncthreads();
  const int np = poff[S], nbp = nbp_s;
  // 4. boundaries, padding and pieces
  for (int i = tid; i < nbp; i += nt) {
    float v = __builtin_inff();
    if (i < np - 1) {
      int seg = 0;
      while (poff[seg + 1] <= i) ++seg;
      const int j = i - poff[seg];
      v = (float)(j < ncr[seg] ? crs[seg][j] : ts[seg]);
    }
    img[kIHead + i] = v;
    bnd[i] = v;
  }
  for (int p = tid; p < np; p += nt) {
    int seg = 0;
    while (poff[seg + 1] <= p) ++seg;
    const int j = p - poff[seg];
    const double slo = seg == 0 ? -inf : ts[seg - 1], shi = seg >= m ? inf : ts[seg];  // seg <= m
    const double z = inside(j == 0 ? slo : crs[seg][j - 1], j == ncr[seg] ? shi : crs[seg][j]);
    double slope = 0.0, icpt = P[kOffB3];
    for (int k = 0; k < kH; ++k) {
      const double pk = ps[seg][k], qk = qs[seg][k];
      if (pk != 0.0 ? pk * z + qk > 0.0 : qk > 0.0) {
        slope += (double)P[kOffW3 + k] * pk;
        icpt += (double)P[kOffW3 + k] * qk;
      }
    }
    img[kIHead + nbp + 2 * p] = (float)slope;
    img[kIHead + nbp + 2 * p + 1] = (float)icpt;
  }
  // 5. the cell table.  Cells span [bnd[s], bnd[nb-1-s]]: trimming the s
  // outermost boundaries on each side (layer-1 breakpoints far outside the
  // table's range) keeps them from stretching the cells; they then share
  // the end cells.  Thread 0 tries s = 0..kCellScan and keeps the fullest
  // cell's smallest count K (the longest run of equal cells along the
  // sorted boundaries).
  __syncthreads();
  const int nb = np - 1;
  if (tid == 0) {
    const float inff = __builtin_inff();
    int bestK = kIMaxBounds + 1, bestG = 0;
    float bz0 = 0.0f, bcinv = 0.0f;
    if (nb > 0) {
      int G0 = 2;
      while (G0 < 2 * nb && G0 < kIMaxCells) G0 <<= 1;
      const int smax = min(kCellScan, (nb - 1) / 2);
      // finer tables shorten the scan (one LDS step per boundary of the
      // fullest cell) at 2 bytes per cell: the smallest K wins, then the
      // fewest cells
      for (int G = G0; G <= kIMaxCells; G <<= 1) {
        for (int t = 0; t <= smax; ++t) {
          const float lo = bnd[t], span = bnd[nb - 1 - t] - lo;
          if (!(lo > -inff) || !(span > 0.0f && span < inff)) continue;
          const float cinv = (float)G / span;
          int K = 0, run = 0, prev = -1;
          for (int k = 0; k < nb; ++k) {
            const int c = cell_of(bnd[k], lo, cinv, G);
            run = c == prev ? run + 1 : 1;
            prev = c;
            K = max(K, run);
          }
          if (K < bestK) {
            bestK = K;
            bestG = G;
            bz0 = lo;
            bcinv = cinv;
          }
        }
        if (bestK <= 1) break;
      }
    }
    const bool use = bestG > 0 && bestK <= kCellScan;
    G_s = use ? bestG : 0;
    K_s = use ? bestK : 0;
    z0_s = use ? bz0 : 0.0f;
    cinv_s = use ? bcinv : 0.0f;
  }
  __syncthreads();
  const int G = G_s, K = K_s;
  const float z0 = z0_s, cinv = cinv_s;
  if (G > 0) {
    // boundary k opens the cells after its predecessor's, up to its own
    for (int k = tid; k < nb; k += nt) {
      const int ck = cell_of(bnd[k], z0, cinv, G);
      const int cp = k == 0 ? -1 : cell_of(bnd[k - 1], z0, cinv, G);
      for (int c = cp + 1; c <= ck; ++c) cells[c] = k;
    }
    const int clast = cell_of(bnd[nb - 1], z0, cinv, G);
    for (int c = clast + 1 + tid; c <= G; c += nt) cells[c] = nb;
  }
  __syncthreads();
  const int Gw = G;
  const int coff = kIHead + nbp + 2 * np;
  if (Gw > 0) {
    uint16_t* C = reinterpret_cast<uint16_t*>(img + coff);
    for (int c = tid; c <= Gw; c += nt) C[c] = (uint16_t)cells[c];
  }
  if (tid == 0) {
    img[0] = __int_as_float(nbp);
    img[1] = __int_as_float(np);
    img[2] = __int_as_float(Gw);
    img[3] = __int_as_float(K);
    img[4] = z0;
    img[5] = cinv;
    img[6] = __int_as_float(coff);
    img[7] = 0.0f;
  }
}

__global__ __launch_bounds__(256) void compile_kernel(const float* __restrict__ P,
                                                      float* __restrict__ img) {
  compile_model(P, img);
}

// One workgroup per slot of a plan.
__global__ __launch_bounds__(256) void compile_many_kernel(const LearnedSlot* slots,
                                                           const float* __restrict__ params,
                                                           float* __restrict__ images) {
  compile_model(params + (int64_t)blockIdx.x * kNP, images + slots[blockIdx.x].i_off);
}

// ---------------------------------------------------------------------------
// Error bound over probes: every entry, its upward neighbour, and the
// log-midpoint to the next entry.  The true index comes from bisection.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int exact_index(const double* __restrict__ a, int n, double x) {
  int base = 0, len = n;
  while (len > 1) {
    const int half = len >> 1;
    base = (a[base + half] < x) ? base + half : base;
    len -= half;
  }
  return base + (a[base] < x ? 1 : 0) - 1;
}

// Largest |g(x) - idx(x)| over the three probes of entry i, with the
// search's own forward pass (so every lane of the wavefront calls it; lanes
// without an entry pass valid = false and get 0).
__device__ __forceinline__ int probe_error(const double* __restrict__ a, int n, const float* m,
                                           const ImageHead& hd, float u0, float inv, int i,
                                           bool valid) {
  const int e = valid ? i : 0;
  double probe[3];
  probe[0] = a[e];
  probe[1] = nextafter(a[e], __builtin_inf());
  probe[2] = e + 1 < n ? sqrt(a[e]) * sqrt(a[e + 1]) : a[e];
  int worst = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float p = mlp_eval(m, hd, model_input(probe[c], u0, inv));
    const int g = predicted_index(p, n);
    worst = max(worst, abs(g - exact_index(a, n, probe[c])));
  }
  return valid ? worst : 0;
}

__global__ __launch_bounds__(256) void bound_kernel(const double* __restrict__ a, int n,
                                                    const float* __restrict__ img, float u0,
                                                    float inv, int* worst) {
  __shared__ __align__(16) float model[kImageFloats];
  stage_image(model, img);
  __syncthreads();
  const ImageHead hd = image_head(model);
  int local = 0;
  const int stride = gridDim.x * blockDim.x;
  // the loop bound is uniform across the workgroup: every lane takes part
  // in every forward pass
  for (int base = blockIdx.x * blockDim.x; base < n; base += stride) {
    const int i = base + threadIdx.x;
    local = max(local, probe_error(a, n, model, hd, u0, inv, i, i < n));
  }
  for (int o = 32; o > 0; o >>= 1) local = max(local, __shfl_xor(local, o));
  if ((threadIdx.x & 63) == 0) atomicMax(worst, local);
}

// Per-slot versions for plans: normalisation (one lane per slot) and the
// error bound (one workgroup per slot).
__global__ void norm_many_kernel(const double* tables_a, const double* tables_b,
                                 LearnedSlot* slots, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const LearnedSlot sl = slots[i];
  const double* a = (sl.which ? tables_b : tables_a) + sl.tab_off;
  const float l0 = __log2f((float)a[0]);
  const float l1 = __log2f((float)a[sl.n - 1]);
  slots[i].u0 = l0;
  slots[i].inv = l1 > l0 ? 1.0f / (l1 - l0) : 1.0f;
}

__global__ __launch_bounds__(256) void bound_many_kernel(const double* tables_a,
                                                         const double* tables_b,
                                                         LearnedSlot* slots,
                                                         const float* images) {
  __shared__ int worst;
  __shared__ __align__(16) float model[kImageFloats];
  const LearnedSlot sl = slots[blockIdx.x];
  const double* a = (sl.which ? tables_b : tables_a) + sl.tab_off;
  stage_image(model, images + sl.i_off);
  if (threadIdx.x == 0) worst = 0;
  __syncthreads();
  const ImageHead hd = image_head(model);
  int local = 0;
  for (int base = 0; base < sl.n; base += blockDim.x) {
    const int i = base + threadIdx.x;
    local = max(local, probe_error(a, sl.n, model, hd, sl.u0, sl.inv, i, i < sl.n));
  }
  for (int o = 32; o > 0; o >>= 1) local = max(local, __shfl_xor(local, o));
  if ((threadIdx.x & 63) == 0) atomicMax(&worst, local);
  __syncthreads();
  if (threadIdx.x == 0) {
    slots[blockIdx.x].E = worst + 1;
    for (int k = 0; k < 4; ++k) slots[blockIdx.x].head[k] = __float_as_int(model[k]);
  }
}

// ---------------------------------------------------------------------------
// Search.
// ---------------------------------------------------------------------------

struct LearnedArgs {
  const double* table;
  const float* img;     // compiled model
  const double* x;
  int32_t* out;
  unsigned long long* fallbacks;
  int64_t m;
  int n;
  int E;
  float u0, inv;
  int model_off;  // byte offset of the model's LDS image (after the table; 0 if not staged)
  int lead;       // byte offset of a[0] in LDS (window_lead(E); staged only)
  int tail;       // +inf entries staged after the table (window_tail(E))
};


// GLOBAL = 1: the table is too large to stage and is read in place from
// global memory (L2-resident after the first reads); only the model is
// staged.
template <int Q, int CONV, int GLOBAL>
__global__ __launch_bounds__(256) void learned_kernel(LearnedArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  // staged: the -inf front, then the table (16-byte aligned)
  const double* sa = GLOBAL ? a.table : reinterpret_cast<const double*>(lds + a.lead);
  const int nt = blockDim.x;
  const int64_t per_tile = (int64_t)nt * Q;
  const int64_t ntiles = (a.m + per_tile - 1) / per_tile;
  float* model = reinterpret_cast<float*>(lds + a.model_off);
  int64_t t = blockIdx.x;
  double cur[Q];
  if (t < ntiles) load_tile<Q>(a.x, a.m, t * per_tile + threadIdx.x, nt, (t + 1) * per_tile <= a.m, cur);
  if constexpr (!GLOBAL)
    stage_table_bounded(reinterpret_cast<double*>(lds + a.lead), a.table, a.n,
                        window_front(a.E), a.tail);
  stage_image(model, a.img);
  __syncthreads();
  const ImageHead hd = image_head(model);
  uint64_t fb = 0;  // the wave's fallbacks (uniform: counted from ballots)
  for (; t < ntiles; t += gridDim.x) {
    const int64_t tn = t + gridDim.x;
    double nxt[Q];
    if (tn < ntiles) load_tile<Q>(a.x, a.m, tn * per_tile + threadIdx.x, nt, (tn + 1) * per_tile <= a.m, nxt);
    int r[Q];
    uint64_t fell[Q];
    if constexpr (CONV) {
      double xs[Q];
      convention_in<Q>(cur, xs);
      search_learned<Q, GLOBAL ? kWinGlobal : kWinBounded>(sa, a.n, model, hd, a.E, a.u0,
                                                             a.inv, xs, r, fell);
      convention_out<Q>(a.n, cur, r);
    } else {
      search_learned<Q, GLOBAL ? kWinGlobal : kWinBounded>(sa, a.n, model, hd, a.E, a.u0,
                                                             a.inv, cur, r, fell);
    }
    const int64_t base = t * per_tile + threadIdx.x;
    const bool full = (t + 1) * per_tile <= a.m;
    // lanes past the end of the ragged last tile searched a stand-in
    if (full) {
#pragma unroll
      for (int q = 0; q < Q; ++q) fb += __builtin_popcountll(fell[q]);
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q)
        fb += __builtin_popcountll(fell[q] & __builtin_amdgcn_ballot_w64(base + (int64_t)q * nt < a.m));
    }
    store_tile<Q>(a.out, a.m, base, nt, full, r);
    for (int q = 0; q < Q; ++q) cur[q] = nxt[q];
  }
  // one atomic per wavefront
  if ((threadIdx.x & 63) == 0 && fb) atomicAdd(a.fallbacks, (unsigned long long)fb);
}

__global__ void clear_counter_kernel(unsigned long long* c) { *c = 0ull; }

__global__ __launch_bounds__(256) void predict_kernel(const float* __restrict__ img,
                                                      const double* __restrict__ x, int64_t m,
                                                      float* __restrict__ out, float u0,
                                                      float inv, int n) {
  __shared__ __align__(16) float model[kImageFloats];
  stage_image(model, img);
  __syncthreads();
  const ImageHead hd = image_head(model);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < m; base += stride) {
    const int64_t i = base + threadIdx.x;
    const float p = mlp_eval(model, hd, model_input(x[i < m ? i : 0], u0, inv));
    if (i < m) out[i] = p * (float)(n - 1);
  }
}

}  // namespace ss

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------

struct ss_learned {
  const double* table = nullptr;
  int n = 0;
  float u0 = 0, inv = 0;
  int E = 0;
  int steps = 0;
  double loss = 0;
  int device = -1;
  float* d_params = nullptr;
  float* d_image = nullptr;  // the compiled model the search evaluates
  int image_floats = 0;      // its floats in use (a multiple of 4)
  int pieces = 0, bound_slots = 0;  // its pieces and padded boundary slots
  int cells = 0, cell_scan = 0;     // its cell table (0: none) and fullest cell
  unsigned long long* d_fallbacks = nullptr;
  std::vector<float> params;
  ~ss_learned() {
    if (d_params) (void)hipFree(d_params);
    if (d_image) (void)hipFree(d_image);
    if (d_fallbacks) (void)hipFree(d_fallbacks);
  }
};

namespace ss {
namespace {

constexpr int kLearnedQ = 4;  // measured best of 1, 2, 4, 6, 8 on a 2000-entry table
constexpr int kLearnedBlock = 256;
constexpr size_t kLearnedStageLimit = 65536;  // LDS bytes: table + model, if staged

int check_learned_table(const double* table, int64_t n, std::vector<double>* host) {
  if (n < 2 || n > 65535) return fail(SS_ERR_INVALID_ARG, "n must be in 2..65535");
  int rc = check_span(table, n, sizeof(double), alignof(double), "table");
  if (rc != SS_OK) return rc;
  if ((rc = check_device_ptr(table, "table")) != SS_OK) return rc;
  host->resize(n);
  hipStream_t st = current_stream();
  SS_TRY_HIP(hipMemcpyAsync(host->data(), table, 8 * n, hipMemcpyDeviceToHost, st));
  SS_TRY_HIP(hipStreamSynchronize(st));
  const double a0 = (*host)[0], a1 = (*host)[n - 1];
  if (!(a0 > 0) || !std::isfinite(a1) || !(a1 > a0))
    return fail(SS_ERR_INVALID_ARG, "learned index needs 0 < a[0] < a[n-1] < inf");
  return SS_OK;
}

// u0 / inv are computed on the device with the model's own log2 so that
// table entries map to exactly 0 and (nearly) 1.
__global__ void norm_kernel(const double* a, int n, float* out) {
  const float l0 = __log2f((float)a[0]);
  const float l1 = __log2f((float)a[n - 1]);
  out[0] = l0;
  out[1] = l1 > l0 ? 1.0f / (l1 - l0) : 1.0f;
}

int make_handle(const double* table, int64_t n, ss_learned** h) {
  ss_learned* p = new (std::nothrow) ss_learned();
  if (!p) return fail(SS_ERR_OOM, "learned handle");
  p->table = table;
  p->n = (int)n;
  *h = p;
  return SS_OK;
}

int measure_bound(ss_learned* h) {
  hipStream_t st = current_stream();
  int* d_worst = nullptr;
  SS_TRY_HIP(hipMalloc(&d_worst, sizeof(int)));
  int worst = 0;
  hipError_t e = hipMemcpyAsync(d_worst, &worst, sizeof(int), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    const int blocks = std::min(1024, (h->n + 255) / 256);
    hipLaunchKernelGGL(bound_kernel, dim3(blocks), dim3(256), 0, st, h->table, h->n, h->d_image,
                       h->u0, h->inv, d_worst);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&worst, d_worst, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d_worst);
  if (e != hipSuccess) return hip_fail(e, "error bound");
  h->E = worst + 1;
  return SS_OK;
}

int setup_norm(ss_learned* h) {
  hipStream_t st = current_stream();
  float* d = nullptr;
  SS_TRY_HIP(hipMalloc(&d, 2 * sizeof(float)));
  float hv[2] = {0, 0};
  hipLaunchKernelGGL(norm_kernel, dim3(1), dim3(1), 0, st, h->table, h->n, d);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(hv, d, sizeof(hv), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d);
  if (e != hipSuccess) return hip_fail(e, "normalisation");
  h->u0 = hv[0];
  h->inv = hv[1];
  return SS_OK;
}

int run_train(const double* table, int n, float u0, float inv, float* d_params, int steps,
              float lr, uint64_t seed, int init_from_seed, float* d_grad, double* loss) {
  hipStream_t st = current_stream();
  float* d_loss = nullptr;
  SS_TRY_HIP(hipMalloc(&d_loss, sizeof(float)));
  TrainArgs a{table, n, steps, lr, seed, u0, inv, d_params, init_from_seed, d_grad, d_loss};
  const size_t lds = sizeof(TrainLds);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&train_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) {
    (void)hipFree(d_loss);
    return hip_fail(e, "training kernel LDS size");
  }
  hipLaunchKernelGGL(train_kernel, dim3(1), dim3(kTrainThreads), lds, st, a);
  e = hipGetLastError();
  float lv = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&lv, d_loss, sizeof(float), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d_loss);
  if (e != hipSuccess) return hip_fail(e, "training");
  if (loss) *loss = lv;
  return SS_OK;
}

int finish_learned(ss_learned* h) {
  SS_TRY_HIP(hipMalloc(&h->d_fallbacks, sizeof(unsigned long long)));
  SS_TRY_HIP(hipMemset(h->d_fallbacks, 0, sizeof(unsigned long long)));
  SS_TRY_HIP(hipMalloc(&h->d_image, sizeof(float) * kImageFloats));
  hipLaunchKernelGGL(compile_kernel, dim3(1), dim3(256), 0, current_stream(), h->d_params,
                     h->d_image);
  SS_TRY_HIP(hipGetLastError());
  h->params.resize(kNP);
  SS_TRY_HIP(hipMemcpy(h->params.data(), h->d_params, sizeof(float) * kNP, hipMemcpyDeviceToHost));
  int dev = 0;
  (void)hipGetDevice(&dev);
  h->device = dev;
  int rc = measure_bound(h);  // (synchronises the stream after the compile)
  if (rc != SS_OK) return rc;
  int head[4] = {0, 0, 0, 0};
  SS_TRY_HIP(hipMemcpy(head, h->d_image, sizeof(head), hipMemcpyDeviceToHost));
  if (!image_header_valid(head)) return fail(SS_ERR_UNSUPPORTED, "compiled model is malformed");
  h->image_floats = image_used_floats(head[0], head[1], head[2]);
  h->bound_slots = head[0];
  h->pieces = head[1];
  h->cells = head[2];
  h->cell_scan = head[3];
  return SS_OK;
}

}  // namespace

bool learned_eligible(const double* a, int64_t n) {
  return n >= 2 && n <= 65535 && a[0] > 0 && std::isfinite(a[n - 1]) && a[n - 1] > a[0];
}

int learned_train_slots(const double* tables_a, const double* tables_b,
                        std::vector<LearnedSlot>& slots, float* d_images, int steps, float lr,
                        uint64_t seed, const float* weights_in, std::vector<float>* weights_out) {
  if (slots.empty()) return SS_OK;
  hipStream_t st = current_stream();
  const int count = (int)slots.size();
  LearnedSlot* d_slots = nullptr;
  float* d_params = nullptr;
  SS_TRY_HIP(hipMalloc(&d_slots, sizeof(LearnedSlot) * count));
  const size_t lds = sizeof(TrainLds);
  hipError_t e = hipMalloc(&d_params, sizeof(float) * kNP * count);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_slots, slots.data(), sizeof(LearnedSlot) * count,
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(norm_many_kernel, dim3((count + 255) / 256), dim3(256), 0, st, tables_a,
                       tables_b, d_slots, count);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&train_many_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess && weights_in) {
    e = hipMemcpyAsync(d_params, weights_in, sizeof(float) * kNP * count,
                       hipMemcpyHostToDevice, st);
  } else if (e == hipSuccess) {
    hipLaunchKernelGGL(train_many_kernel, dim3(count), dim3(kTrainThreads), lds, st, tables_a,
                       tables_b, d_slots, d_params, steps, lr, seed);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(compile_many_kernel, dim3(count), dim3(256), 0, st, d_slots, d_params,
                       d_images);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(bound_many_kernel, dim3(count), dim3(256), 0, st, tables_a, tables_b,
                       d_slots, d_images);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(slots.data(), d_slots, sizeof(LearnedSlot) * count,
                       hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && weights_out) {
    weights_out->resize((size_t)kNP * count);
    e = hipMemcpyAsync(weights_out->data(), d_params, sizeof(float) * kNP * count,
                       hipMemcpyDeviceToHost, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d_slots);
  if (d_params) (void)hipFree(d_params);
  if (e != hipSuccess) return hip_fail(e, "training plan models");
  return SS_OK;
}

}  // namespace ss

using namespace ss;

extern "C" {

int ss_learned_build(const double* table, int64_t n, const ss_mlp_opts* opts, ss_learned** out) {
  clear_error();
  if (!out) return fail(SS_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  ss_mlp_opts o{3000, 0.01f, 1};
  if (opts) o = *opts;
  if (o.steps < 0 || o.steps > 1000000) return fail(SS_ERR_INVALID_ARG, "steps: 0..1e6");
  if (!(o.lr > 0) || !std::isfinite(o.lr)) return fail(SS_ERR_INVALID_ARG, "lr must be > 0");
  std::vector<double> host;
  int rc = check_learned_table(table, n, &host);
  if (rc != SS_OK) return rc;
  ss_learned* h = nullptr;
  if ((rc = make_handle(table, n, &h)) != SS_OK) return rc;
  h->steps = o.steps;
  rc = setup_norm(h);
  if (rc == SS_OK) {
    hipError_t e = hipMalloc(&h->d_params, sizeof(float) * kNP);
    rc = e == hipSuccess ? SS_OK : hip_fail(e, "hipMalloc(params)");
  }
  if (rc == SS_OK)
    rc = run_train(table, h->n, h->u0, h->inv, h->d_params, o.steps, o.lr, o.seed, 1, nullptr,
                   &h->loss);
  if (rc == SS_OK) rc = finish_learned(h);
  if (rc != SS_OK) {
    delete h;
    return rc;
  }
  log_line("learned model: n %d, %d Adam steps, loss %.3g, error bound E = %d", h->n, o.steps,
           h->loss, h->E);
  *out = h;
  return SS_OK;
}

int ss_learned_from_weights(const double* table, int64_t n, const float* weights,
                            ss_learned** out) {
  clear_error();
  if (!out || !weights) return fail(SS_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  std::vector<double> host;
  int rc = check_learned_table(table, n, &host);
  if (rc != SS_OK) return rc;
  ss_learned* h = nullptr;
  if ((rc = make_handle(table, n, &h)) != SS_OK) return rc;
  rc = setup_norm(h);
  if (rc == SS_OK) {
    hipError_t e = hipMalloc(&h->d_params, sizeof(float) * kNP);
    if (e == hipSuccess)
      e = hipMemcpy(h->d_params, weights, sizeof(float) * kNP, hipMemcpyHostToDevice);
    rc = e == hipSuccess ? SS_OK : hip_fail(e, "parameters");
  }
  if (rc == SS_OK) rc = finish_learned(h);
  if (rc != SS_OK) {
    delete h;
    return rc;
  }
  *out = h;
  return SS_OK;
}

int ss_learned_save(const ss_learned* h, const char* path) {
  clear_error();
  if (!h || !path) return fail(SS_ERR_INVALID_ARG, "null argument");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(SS_ERR_INVALID_ARG, std::string("cannot write ") + path);
  std::fprintf(f, "{\n \"format\": \"searchsorted-learned-1\",\n \"n\": %d,\n \"E\": %d,\n"
                  " \"steps\": %d,\n \"loss\": %.17g,\n \"u0\": %.9g,\n \"inv\": %.9g,\n"
                  " \"weights\": [",
               h->n, h->E, h->steps, h->loss, (double)h->u0, (double)h->inv);
  for (int i = 0; i < kNP; ++i)
    std::fprintf(f, "%s%.9g", i ? ", " : "", (double)h->params[i]);
  std::fprintf(f, "]\n}\n");
  const bool ok = std::fclose(f) == 0;
  return ok ? SS_OK : fail(SS_ERR_INVALID_ARG, std::string("cannot write ") + path);
}

namespace {

// Finds "key": in a saved model and returns a pointer just past the colon.
const char* find_key(const std::string& text, const char* key) {
  const std::string k = std::string("\"") + key + "\"";
  const size_t at = text.find(k);
  if (at == std::string::npos) return nullptr;
  const size_t colon = text.find(':', at + k.size());
  return colon == std::string::npos ? nullptr : text.c_str() + colon + 1;
}

}  // namespace

int ss_learned_load(const double* table, int64_t n, const char* path, ss_learned** out) {
  clear_error();
  if (!out || !path) return fail(SS_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(SS_ERR_INVALID_ARG, std::string("cannot read ") + path);
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  std::fclose(f);
  if (text.find("\"searchsorted-learned-1\"") == std::string::npos)
    return fail(SS_ERR_INVALID_ARG, "not a saved learned model");
  const char* pn = find_key(text, "n");
  const char* pw = find_key(text, "weights");
  const char* ps = find_key(text, "steps");
  const char* pl = find_key(text, "loss");
  if (!pn || !pw) return fail(SS_ERR_INVALID_ARG, "saved model lacks n or weights");
  if (std::strtoll(pn, nullptr, 10) != n)
    return fail(SS_ERR_INVALID_ARG, "saved model was trained on a table of another size");
  std::vector<float> w(kNP);
  const char* c = std::strchr(pw, '[');
  if (!c) return fail(SS_ERR_INVALID_ARG, "malformed weights");
  ++c;
  for (int i = 0; i < kNP; ++i) {
    char* end = nullptr;
    w[i] = std::strtof(c, &end);
    if (end == c) return fail(SS_ERR_INVALID_ARG, "malformed weights");
    c = end;
    while (*c == ' ' || *c == ',' || *c == '\n') ++c;
  }
  if (*c != ']') return fail(SS_ERR_INVALID_ARG, "weights: expected 1153 values");
  int rc = ss_learned_from_weights(table, n, w.data(), out);
  if (rc != SS_OK) return rc;
  if (ps) (*out)->steps = (int)std::strtol(ps, nullptr, 10);
  if (pl) (*out)->loss = std::strtod(pl, nullptr);
  return SS_OK;
}

int ss_learned_search(ss_learned* h, const double* targets, int64_t m, int32_t* out_idx) {
  clear_error();
  if (!h) return fail(SS_ERR_INVALID_ARG, "handle is null");
  int rc = check_span(targets, m, 8, 8, "targets");
  if (rc == SS_OK) rc = check_span(out_idx, m, 4, 4, "out_idx");
  if (rc != SS_OK) return rc;
  hipStream_t st = current_stream();
  hipLaunchKernelGGL(clear_counter_kernel, dim3(1), dim3(1), 0, st, h->d_fallbacks);
  SS_TRY_HIP(hipGetLastError());
  if (m == 0) return SS_OK;
  if (overlaps(out_idx, (size_t)m * 4, targets, (size_t)m * 8))
    return fail(SS_ERR_INVALID_ARG, "out_idx overlaps targets");
  if ((rc = check_device_ptr(targets, "targets")) != SS_OK ||
      (rc = check_device_ptr(out_idx, "out_idx")) != SS_OK)
    return rc;
  DeviceInfo di;
  if ((rc = device_info(&di)) != SS_OK) return rc;
  // the table is staged with the model when both fit (window_front -inf
  // entries, the table, window_tail +inf entries), else read in place
  const int tail = window_tail(h->E), lead = window_lead(h->E);
  size_t tab = (size_t)lead + ((size_t)(h->n + tail) * 8 + 15) / 16 * 16;
  const bool staged = tab + (size_t)h->image_floats * 4 <= kLearnedStageLimit;
  if (!staged) tab = 0;
  const size_t lds = tab + (size_t)h->image_floats * 4;
  const bool conv = option(SS_OPT_CONVENTION) != 0;
  const void* kern =
      staged ? (conv ? reinterpret_cast<const void*>(&learned_kernel<kLearnedQ, 1, 0>)
                     : reinterpret_cast<const void*>(&learned_kernel<kLearnedQ, 0, 0>))
             : (conv ? reinterpret_cast<const void*>(&learned_kernel<kLearnedQ, 1, 1>)
                     : reinterpret_cast<const void*>(&learned_kernel<kLearnedQ, 0, 1>));
  const int64_t per_tile = (int64_t)kLearnedBlock * kLearnedQ;
  const int64_t ntiles = (m + per_tile - 1) / per_tile;
  int64_t grid = (int64_t)blocks_per_cu(kern, kLearnedBlock, lds) * di.num_cus * 4;
  grid = std::max<int64_t>(1, std::min<int64_t>(grid, ntiles));
  LearnedArgs a{h->table, h->d_image, targets, out_idx, h->d_fallbacks, m, h->n, h->E, h->u0,
                h->inv, (int)tab, lead, tail};
  void* args[] = {&a};
  SS_TRY_HIP(hipLaunchKernel(kern, dim3((unsigned)grid), dim3(kLearnedBlock), args, lds, st));
  return SS_OK;
}

int ss_learned_predict(ss_learned* h, const double* x, int64_t m, float* out_pos) {
  clear_error();
  if (!h) return fail(SS_ERR_INVALID_ARG, "handle is null");
  int rc = check_span(x, m, 8, 8, "x");
  if (rc == SS_OK) rc = check_span(out_pos, m, 4, 4, "out_pos");
  if (rc != SS_OK || m == 0) return rc;
  if ((rc = check_device_ptr(x, "x")) != SS_OK || (rc = check_device_ptr(out_pos, "out_pos")) != SS_OK)
    return rc;
  const int64_t blocks = std::min<int64_t>((m + 255) / 256, 8192);
  hipLaunchKernelGGL(predict_kernel, dim3((unsigned)blocks), dim3(256), 0, current_stream(),
                     h->d_image, x, m, out_pos, h->u0, h->inv, h->n);
  SS_TRY_HIP(hipGetLastError());
  return SS_OK;
}

int ss_learned_info(const ss_learned* h, double* info, int count) {
  clear_error();
  if (!h || !info || count < 6) return fail(SS_ERR_INVALID_ARG, "need a handle and 6 slots");
  info[0] = h->E;
  info[1] = h->n;
  info[2] = h->steps;
  info[3] = h->loss;
  info[4] = h->u0;
  info[5] = h->inv;
  if (count >= 8) {
    info[6] = h->pieces;
    info[7] = h->bound_slots;
  }
  if (count >= 10) {
    info[8] = h->cells;
    info[9] = h->cell_scan;
  }
  return SS_OK;
}

int ss_learned_fallbacks(ss_learned* h, int64_t* count) {
  clear_error();
  if (!h || !count) return fail(SS_ERR_INVALID_ARG, "null argument");
  unsigned long long v = 0;
  hipStream_t st = current_stream();
  SS_TRY_HIP(hipMemcpyAsync(&v, h->d_fallbacks, sizeof(v), hipMemcpyDeviceToHost, st));
  SS_TRY_HIP(hipStreamSynchronize(st));
  *count = (int64_t)v;
  return SS_OK;
}

int ss_learned_error_bound(const ss_learned* h, int32_t* E) {
  clear_error();
  if (!h || !E) return fail(SS_ERR_INVALID_ARG, "null argument");
  *E = h->E;
  return SS_OK;
}

int ss_learned_set_error_bound(ss_learned* h, int32_t E) {
  clear_error();
  if (!h) return fail(SS_ERR_INVALID_ARG, "null handle");
  if (E < 0 || E > 65535) return fail(SS_ERR_INVALID_ARG, "E must be in 0..65535");
  h->E = E;
  return SS_OK;
}

int ss_learned_stats(ss_learned* h, int64_t* fallbacks) {
  return ss_learned_fallbacks(h, fallbacks);
}

int ss_learned_weights(const ss_learned* h, float* out, int64_t cap) {
  clear_error();
  if (!h || !out || cap < kNP) return fail(SS_ERR_INVALID_ARG, "need a handle and 1153 slots");
  std::memcpy(out, h->params.data(), sizeof(float) * kNP);
  return SS_OK;
}

int ss_mlp_gradient(const double* table, int64_t n, const float* weights, float* grad_out,
                    double* loss_out) {
  clear_error();
  if (!weights || !grad_out) return fail(SS_ERR_INVALID_ARG, "null argument");
  std::vector<double> host;
  int rc = check_learned_table(table, n, &host);
  if (rc != SS_OK) return rc;
  ss_learned tmp;
  tmp.table = table;
  tmp.n = (int)n;
  if ((rc = setup_norm(&tmp)) != SS_OK) return rc;
  float *d_p = nullptr, *d_g = nullptr;
  SS_TRY_HIP(hipMalloc(&d_p, sizeof(float) * kNP));
  hipError_t e = hipMalloc(&d_g, sizeof(float) * kNP);
  if (e == hipSuccess) e = hipMemcpy(d_p, weights, sizeof(float) * kNP, hipMemcpyHostToDevice);
  double loss = 0;
  if (e == hipSuccess) rc = run_train(table, tmp.n, tmp.u0, tmp.inv, d_p, 0, 1.0f, 0, 0, d_g, &loss);
  else rc = hip_fail(e, "gradient buffers");
  if (rc == SS_OK) {
    e = hipMemcpy(grad_out, d_g, sizeof(float) * kNP, hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = hip_fail(e, "gradient copy");
  }
  (void)hipFree(d_p);
  if (d_g) (void)hipFree(d_g);
  if (rc == SS_OK && loss_out) *loss_out = loss;
  return rc;
}

int ss_learned_destroy(ss_learned* h) {
  clear_error();
  delete h;
  return SS_OK;
}

}  // extern "C"

namespace ss {
int learned_export(const ss_learned* h, LearnedExport* out) {
  if (!h || !out || !h->d_image) return fail(SS_ERR_INVALID_ARG, "learned handle is null");
  out->table = h->table;
  out->n = h->n;
  out->device = h->device;
  out->E = h->E;
  out->u0 = h->u0;
  out->inv = h->inv;
  out->image = h->d_image;
  out->image_floats = h->image_floats;
  out->params = h->params.data();
  return SS_OK;
}
}  // namespace ss

namespace ss {
int violations_learned(unsigned long long* out) { return read_violations(out); }
}  // namespace ss
