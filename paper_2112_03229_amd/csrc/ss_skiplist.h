// Skiplist search (paper Sec. 3.3) as a two-level LDS search.
//
// The skip table holds every 8th entry, sk[i] = a[8 i] for i < ceil(n/8),
// contiguous in LDS (the paper gives each index its own cache line; on the
// GPU a separate compact array keeps the first level's reads on distinct
// banks, where a stride-8 view of the table would put them all on two).
// Level 1 bisects the skip table: j = #{i : sk[i] < x} - 1, the last block
// whose first entry is below x.  Every entry before block j is then below
// x and every entry from block j+1 on is not, so
//   idx(x) = 8 j + #{k < 8 : a[8 j + k] < x} - 1    (j >= 0),   -1 if j < 0.
// Level 2 reads the block's 8 doubles with four independent 16-byte LDS
// reads (the staged table's +inf padding covers a short last block).
#pragma once

#include "ss_device.h"

namespace ss {

constexpr int kSkip = 8;  // entries per skip-table block

__device__ __forceinline__ int skip_count(int n) { return (n + kSkip - 1) / kSkip; }

// sk[i] = sa[8 i] for i < ceil(n/8), then SS_PAD +inf sentinels.  The whole
// workgroup calls, after the table is staged; a barrier must follow.
__device__ __forceinline__ void build_skip_table(const double* __restrict__ sa, int n,
                                                 double* __restrict__ sk) {
  const int ns = skip_count(n);
  for (int i = threadIdx.x; i < ns + SS_PAD; i += blockDim.x)
    sk[i] = i < ns ? sa[kSkip * i] : __builtin_inf();
}

template <int Q>
__device__ __forceinline__ void search_skiplist(const double* __restrict__ sa,
                                                const double* __restrict__ sk, int n,
                                                const double (&x)[Q], int (&r)[Q]) {
  const int ns = skip_count(n);
  int base[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) base[q] = 0;
  int len = ns;
  while (len > 1) {
    const int half = len >> 1;
#pragma unroll
    for (int q = 0; q < Q; ++q)
      base[q] = (sk[SS_IN(base[q] + half, 0, ns + SS_PAD)] < x[q]) ? base[q] + half : base[q];
    len -= half;
  }
  typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    // n == 0: sk[0] is a sentinel, j = -1
    const int j = base[q] + (sk[SS_IN(base[q], 0, ns + SS_PAD)] < x[q] ? 1 : 0) - 1;
    SS_ASSERT(kSkip * max(j, 0) + kSkip <= n + SS_PAD);
    const d2* blk = reinterpret_cast<const d2*>(sa + kSkip * max(j, 0));
    int cnt = 0;
#pragma unroll
    for (int h = 0; h < kSkip / 2; ++h) {
      const d2 v = blk[h];
      cnt += (v.x < x[q] ? 1 : 0) + (v.y < x[q] ? 1 : 0);
    }
    r[q] = j < 0 ? -1 : kSkip * j + cnt - 1;
  }
}

}  // namespace ss
