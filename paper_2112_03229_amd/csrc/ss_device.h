// Device building blocks of the sorted search (gfx950 / CDNA4, wave64).
//
// Every search routine here returns idx(x) = #{i : a[i] < x} - 1 for a table
// a[0..n) that has been staged in LDS as `sa`, followed by SS_PAD copies of
// +inf (so a read up to SS_PAD entries past the end is defined and never
// counts).  Queries are processed Q at a time per lane (one query per lane
// per slot, Q independent slots) so that LDS latency is hidden by ILP.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/searchsorted.h"

#define SS_PAD 8            // +inf sentinels after the staged table
#define SS_SCAN_MAX SS_PAD  // longest fixed in-bin scan; longer bins bisect
#define SS_MAX_BITS 20      // bin bits that fit in the high word of a double

namespace ss {

// ---------------------------------------------------------------------------
// Device bounds checks.  In a checked build (compiled with
// -DSS_DEVICE_CHECKS=1) SS_IN(i, lo, hi) tests lo <= i < hi for an index
// about to be used in an access to a region of hi entries; a violation is
// counted in this module's device counter and i is clamped into the
// region, so the checked kernels report an indexing mistake instead of
// reading or writing outside it.  SS_ASSERT(c) counts a violated condition.
// In normal builds both compile to nothing.  read_violations (host) returns
// and clears the module's count.
// ---------------------------------------------------------------------------
#if SS_DEVICE_CHECKS
static __device__ unsigned long long g_ss_violations = 0;

__device__ __forceinline__ int checked_index(int i, int lo, int hi) {
  if (i < lo || i >= hi) {
    atomicAdd(&g_ss_violations, 1ull);
    i = i < lo ? lo : hi - 1;
  }
  return i;
}
#define SS_IN(i, lo, hi) ::ss::checked_index((i), (lo), (hi))
#define SS_ASSERT(c)                                     \
  do {                                                   \
    if (!(c)) atomicAdd(&::ss::g_ss_violations, 1ull);   \
  } while (0)

static inline int read_violations(unsigned long long* out) {
  unsigned long long zero = 0;
  if (hipMemcpyFromSymbol(out, HIP_SYMBOL(g_ss_violations), sizeof(*out)) != hipSuccess ||
      hipMemcpyToSymbol(HIP_SYMBOL(g_ss_violations), &zero, sizeof(zero)) != hipSuccess) {
    (void)hipGetLastError();
    return SS_ERR_HIP;
  }
  return SS_OK;
}
#else
#define SS_IN(i, lo, hi) (i)
#define SS_ASSERT(c) ((void)0)
static inline int read_violations(unsigned long long* out) {
  *out = 0;
  return SS_ERR_UNSUPPORTED;  // not a checked build
}
#endif

// High 32 bits of the IEEE-754 encoding, as a signed integer: sign bit,
// 11-bit biased exponent, 20 leading fraction bits.
__device__ __forceinline__ int hi_word(double v) { return __double2hiint(v); }

// Exponent-hash key with s leading fraction bits (paper Sec. 3.5 for s = 0).
// For v with a clear sign bit the key is non-decreasing in v; v with the
// sign bit set (negative values, -0.0, -NaN) maps below every such key.
__device__ __forceinline__ int hash_key(double v, int shift /* 20 - s */) {
  return hi_word(v) >> shift;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// ---------------------------------------------------------------------------
// Staging (a1): coalesced copy of the table into LDS plus +inf padding.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void stage_table(double* __restrict__ sa,
                                            const double* __restrict__ table, int n) {
  const int nt = blockDim.x;
  for (int i = threadIdx.x; i < n + SS_PAD; i += nt)
    sa[i] = i < n ? table[i] : __builtin_inf();
}

// The bounded form for the learned search's window (see window_front and
// window_tail): a[-front..n + tail) at sa = front copies of -inf, the
// table, tail copies of +inf.  sa must have front entries of its region
// before it.
__device__ __forceinline__ void stage_table_bounded(double* __restrict__ sa,
                                                    const double* __restrict__ table, int n,
                                                    int front, int tail) {
  for (int i = (int)threadIdx.x - front; i < n + tail; i += blockDim.x)
    sa[i] = i < 0 ? -__builtin_inf() : i < n ? table[i] : __builtin_inf();
}

// ---------------------------------------------------------------------------
// Exponent-hash bins (a2): parameters and the prefix-count table in LDS.
//   key(v) = hi_word(v) >> (20 - s),  kmin = key(a[0]),  nb = key(a[n-1]) - kmin + 1
//   C[b]   = #{ i : key(a[i]) - kmin < b },  b = 0..nb        (Eq. 3, prefix form)
// ---------------------------------------------------------------------------
struct HashParams {
  int ok;      // 1 if the exponent hash applies to this table
  int shift;   // 20 - s
  int kmin;    // key of a[0]
  int kmaxc;   // kmin + nb - 1 (upper clamp of target keys)
  int nb;      // number of bins
  int K;       // most entries in one bin (set by build_bins)
};

// Chooses s: the forced value if bits >= 0, else the largest s in [0, 20]
// whose bin count fits `cap`.  Uniform across the workgroup (depends only on
// a[0], a[n-1], bits and cap).  Not applicable when n == 0, when a[0] has its
// sign bit set, when the keys are not ordered, or when no s fits.  `a` may
// point to LDS or global memory.
__device__ __forceinline__ HashParams choose_hash(const double* a, int n, int bits, int cap) {
  HashParams hp{0, SS_MAX_BITS, 0, 0, 0, 0};
  if (n < 1 || n > 65535) return hp;
  const int h0 = __builtin_amdgcn_readfirstlane(hi_word(a[0]));
  const int h1 = __builtin_amdgcn_readfirstlane(hi_word(a[n - 1]));
  if (h0 < 0 || h1 < h0) return hp;
  int s = bits >= 0 ? min(bits, SS_MAX_BITS) : SS_MAX_BITS;
  for (;;) {
    const int sh = SS_MAX_BITS - s;
    const int nb = (h1 >> sh) - (h0 >> sh) + 1;
    if (nb <= cap) {
      hp.ok = 1;
      hp.shift = __builtin_amdgcn_readfirstlane(sh);
      hp.kmin = __builtin_amdgcn_readfirstlane(h0 >> sh);
      hp.kmaxc = __builtin_amdgcn_readfirstlane(h1 >> sh);
      hp.nb = __builtin_amdgcn_readfirstlane(nb);
      return hp;
    }
    if (bits >= 0 || s == 0) return hp;
    --s;
  }
}

// Builds C[0..nb] by gap filling: entry i writes C[b] = i for every bin b it
// opens, i.e. b in (key bin of a[i-1], key bin of a[i]], and C[nb] = n.  For
// a sorted table every b is written exactly once (no atomics, no clearing
// pass).  K, the most entries sharing one bin, is the longest run of equal
// keys, measured per entry by looking back at most SS_SCAN_MAX entries
// (K = SS_SCAN_MAX + 1 stands for "longer").  `scratch` is one int; the whole
// workgroup must call.  A table that violates the sort precondition can
// leave bins unwritten: readers clamp C values to [0, n].
template <typename CT>
__device__ __forceinline__ void build_bins(const double* __restrict__ sa, int n, HashParams& hp,
                                           CT* __restrict__ C, int* scratch) {
  const int nt = blockDim.x, tid = threadIdx.x;
  if (tid == 0) *scratch = 0;
  __syncthreads();  // (callers stage the table before; one barrier suffices)
  int run_max = 0;
  for (int i = tid; i < n; i += nt) {
    const int kb = clampi(hash_key(sa[i], hp.shift), hp.kmin, hp.kmaxc) - hp.kmin;
    const int kp =
        i == 0 ? -1 : clampi(hash_key(sa[i - 1], hp.shift), hp.kmin, hp.kmaxc) - hp.kmin;
    for (int b = kp + 1; b <= kb; ++b) C[SS_IN(b, 0, hp.nb + 1)] = (CT)i;
    int run = 1;
    if (kp == kb) {
      run = 2;
      while (run <= SS_SCAN_MAX && i - run >= 0 &&
             clampi(hash_key(sa[i - run], hp.shift), hp.kmin, hp.kmaxc) - hp.kmin == kb)
        ++run;
    }
    run_max = max(run_max, run);
  }
  if (tid == 0) C[hp.nb] = (CT)n;
  for (int o = 32; o > 0; o >>= 1) run_max = max(run_max, __shfl_xor(run_max, o));
  if ((tid & 63) == 0) atomicMax(scratch, run_max);
  __syncthreads();
  hp.K = __builtin_amdgcn_readfirstlane(*scratch);
}

// ---------------------------------------------------------------------------
// K1: branchless bisection (Sec. 3.2).  Fixed trip count ceil(log2 n) that
// depends only on n, so the loop is wavefront-uniform; each step is one LDS
// read, one compare and one select.  count = #{a < x}; NaN counts 0.
// ---------------------------------------------------------------------------
template <int Q>
__device__ __forceinline__ void search_binary(const double* __restrict__ sa, int n,
                                              const double (&x)[Q], int (&r)[Q]) {
  int base[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) base[q] = 0;
  int len = n;
  while (len > 1) {
    const int half = len >> 1;
#pragma unroll
    for (int q = 0; q < Q; ++q)
      base[q] = (sa[SS_IN(base[q] + half, 0, n + SS_PAD)] < x[q]) ? base[q] + half : base[q];
    len -= half;
  }
  // n == 0: sa[0] is the +inf sentinel, so the count is 0.
#pragma unroll
  for (int q = 0; q < Q; ++q) r[q] = base[q] + (sa[SS_IN(base[q], 0, n + SS_PAD)] < x[q] ? 1 : 0) - 1;
}

// Global-memory variant for tables too large to stage (same arithmetic).
template <int Q>
__device__ __forceinline__ void search_binary_global(const double* __restrict__ a, int n,
                                                     const double (&x)[Q], int (&r)[Q]) {
  int base[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) base[q] = 0;
  int len = n;
  while (len > 1) {
    const int half = len >> 1;
#pragma unroll
    for (int q = 0; q < Q; ++q) base[q] = (a[base[q] + half] < x[q]) ? base[q] + half : base[q];
    len -= half;
  }
#pragma unroll
  for (int q = 0; q < Q; ++q)
    r[q] = (n > 0 ? base[q] + (a[base[q]] < x[q] ? 1 : 0) : 0) - 1;
}

// ---------------------------------------------------------------------------
// K3: exponent hash (Sec. 3.5).  Integer key from the high word, clamp to the
// table's key range, C[b] gives the number of entries in earlier bins, then a
// linear scan (Sec. 3.4's interior search) of the bin.  Entries after the bin
// have larger keys, hence larger values, so a fixed-length scan of K entries
// (K = largest bin) counts exactly the bin's entries below x.  Bins longer
// than SS_SCAN_MAX are searched by bisection inside [C[b], C[b+1]).  C values
// are clamped to [0, n] so that even a table violating the sort precondition
// reads only the staged table and its padding.
// NaN targets need the one select: their key lands in the last bin.
// ---------------------------------------------------------------------------
template <int Q>
__device__ __forceinline__ void search_exphash(const double* __restrict__ sa,
                                               const uint16_t* __restrict__ C, int n,
                                               const HashParams& hp, const double (&x)[Q],
                                               int (&r)[Q]) {
  int b[Q], j0[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    b[q] = clampi(hash_key(x[q], hp.shift), hp.kmin, hp.kmaxc) - hp.kmin;
    j0[q] = min((int)C[SS_IN(b[q], 0, hp.nb + 1)], n);
  }
  if (hp.K <= SS_SCAN_MAX) {
    int cnt[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) cnt[q] = 0;
#pragma nounroll
    for (int k = 0; k < hp.K; ++k) {
#pragma unroll
      for (int q = 0; q < Q; ++q) cnt[q] += (sa[SS_IN(j0[q] + k, 0, n + SS_PAD)] < x[q]) ? 1 : 0;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) r[q] = (x[q] != x[q]) ? -1 : j0[q] + cnt[q] - 1;
  } else {
    // long bins: bisection inside [C[b], C[b+1]) -- the largest pos in
    // [lo, hi] with a[pos-1] < x, by binary lifting with steps P, P/2, .., 1
    // where P is the largest power of two <= n (>= every bin length)
    int hi[Q], pos[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      hi[q] = min(max((int)C[SS_IN(b[q] + 1, 0, hp.nb + 1)], j0[q]), n);
      pos[q] = j0[q];
    }
    int step = 1;
    while (step * 2 <= n) step *= 2;
    for (; step >= 1; step >>= 1) {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int cand = pos[q] + step;
        const int ridx = max(min(cand, hi[q]) - 1, 0);
        const bool lt = sa[SS_IN(ridx, 0, n + SS_PAD)] < x[q];
        pos[q] = ((cand <= hi[q]) & lt) ? cand : pos[q];
      }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) r[q] = (x[q] != x[q]) ? -1 : pos[q] - 1;
  }
}

// ---------------------------------------------------------------------------
// K2: linear scan (Sec. 2.1) restricted to the wavefront's bracket.  The
// smallest and largest target of the wavefront (NaN ignored) bound every
// lane's answer; their counts come from ballots over the table held 64
// entries per step, one per lane.  Each lane then scans only [lo, hi).
// Cheap when a wavefront's targets are close together (sorted streams),
// a full scan when they are spread over the table.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

template <int Q>
__device__ __forceinline__ void search_ballot(const double* __restrict__ sa, int n,
                                              const double (&x)[Q], int (&r)[Q]) {
  const int lane = threadIdx.x & 63;
  double lmin = x[0], lmax = x[0];
#pragma unroll
  for (int q = 1; q < Q; ++q) {
    lmin = fmin(lmin, x[q]);
    lmax = fmax(lmax, x[q]);
  }
  const double wmin = wave_min(lmin);
  const double wmax = wave_max(lmax);
  int lo = 0, hi = 0;
  for (int c = 0; c < n; c += 64) {
    const double e = sa[SS_IN(min(c + lane, n), 0, n + SS_PAD)];  // index n is the +inf sentinel
    lo += __popcll(__ballot(e < wmin));
    hi += __popcll(__ballot(e < wmax));
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  hi = __builtin_amdgcn_readfirstlane(hi);
  int cnt[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) cnt[q] = 0;
  for (int j = lo; j < hi; ++j) {
    const double aj = sa[SS_IN(j, 0, n + SS_PAD)];
#pragma unroll
    for (int q = 0; q < Q; ++q) cnt[q] += (aj < x[q]) ? 1 : 0;
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) r[q] = (x[q] != x[q]) ? -1 : lo + cnt[q] - 1;
}

// ---------------------------------------------------------------------------
// The paper's convention (Sec. 3): the last index with a[i] <= x, 0 when
// there is none, n - 1 above the table, i.e. min(max(#{a <= x} - 1, 0), n-1).
// Every search above counts a < x; a <= x counts the same as a < up(x), with
// up(x) the next double above x, for every x except +inf (whose count is n,
// since tables hold no NaN).  A NaN target stays NaN, counts 0 and gives 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double next_up(double x) {
  const long long i = __double_as_longlong(x);
  const double up = __longlong_as_double(i >= 0 ? i + 1 : i - 1);
  return x == 0.0 ? 0x1p-1074 : up;  // -0.0 and +0.0 step to the smallest subnormal
}

template <int Q>
__device__ __forceinline__ void convention_in(const double (&x)[Q], double (&xs)[Q]) {
#pragma unroll
  for (int q = 0; q < Q; ++q) xs[q] = x[q] == __builtin_inf() ? x[q] : next_up(x[q]);
}

template <int Q>
__device__ __forceinline__ void convention_out(int n, const double (&x)[Q], int (&r)[Q]) {
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int v = x[q] == __builtin_inf() ? n - 1 : r[q];
    r[q] = n > 0 ? min(max(v, 0), n - 1) : -1;
  }
}

// ---------------------------------------------------------------------------
// Streaming targets (a3) and indices (a6).
// ---------------------------------------------------------------------------
// Loads one tile slot set: slot q of lane t is target base + q*nt.  A full
// tile uses plain non-temporal loads; the ragged last tile clamps the index
// (so every load stays in bounds and none is predicated) and turns the
// missing targets into NaN, which every search handles.
template <int Q>
__device__ __forceinline__ void load_tile(const double* __restrict__ x, int64_t m, int64_t base,
                                          int nt, bool full, double (&xv)[Q]) {
  SS_ASSERT(base >= 0 && (!full || base + (int64_t)(Q - 1) * nt < m));
  if (full) {
#pragma unroll
    for (int q = 0; q < Q; ++q) xv[q] = __builtin_nontemporal_load(x + base + (int64_t)q * nt);
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t k = base + (int64_t)q * nt;
      const double v = x[k < m ? k : m - 1];
      xv[q] = k < m ? v : __builtin_nan("");
    }
  }
}

template <int Q>
__device__ __forceinline__ void store_tile(int32_t* __restrict__ out, int64_t m, int64_t base,
                                           int nt, bool full, const int (&r)[Q]) {
  SS_ASSERT(base >= 0 && (!full || base + (int64_t)(Q - 1) * nt < m));
  if (full) {
#pragma unroll
    for (int q = 0; q < Q; ++q) __builtin_nontemporal_store(r[q], out + base + (int64_t)q * nt);
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t k = base + (int64_t)q * nt;
      if (k < m) out[k] = r[q];
    }
  }
}

// Streams the tiles t = blockIdx.x, blockIdx.x + gridDim.x, ... through
// `search`, software-pipelined: the next tile's targets are in flight while
// the current tile is searched and stored.
}  // namespace ss
