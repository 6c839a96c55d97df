// Single-table search: kernels K1 (bisection), K2 (ballot-bracketed linear
// scan), K3 (exponent hash), the logarithm hash, the two-level skiplist and
// the global-memory bisection, plus the C ABI entry points search_sorted_batch, ss_search_with,
// ss_validate_table, ss_exphash_bins and ss_loghash_bins.
//
// Launch shape: at least enough workgroups to fill every CU at the occupancy
// the LDS footprint allows, and a few tiles per workgroup (more for larger
// tables and for the hashes, whose setup costs more).  Each workgroup stages
// the table once (K3 also builds its bin table in LDS) and then streams tiles
// of blockDim.x * Q targets: slot q of lane t reads target base + q*blockDim.x + t,
// so every load and store instruction of a wavefront covers one contiguous
// run (512 B of targets, 256 B of indices).  Targets are read and indices
// written with non-temporal hints: each byte is touched once.
#include <algorithm>
#include <string>

#include "ss_device.h"
#include "ss_host.h"
#include "ss_loghash.h"
#include "ss_skiplist.h"

namespace ss {

constexpr int kDefaultQ = 8;          // targets per lane per tile
constexpr int kDefaultBlock = 512;    // threads per workgroup
// Tiles per workgroup of the default grid (see tiles_per_workgroup).  A
// grid several times larger than the resident workgroup count lets the
// dispatcher balance CUs that run at different speeds (a strictly
// persistent grid loses ~10% to its slowest workgroups).
constexpr int kTilesPerBlockHash = 6;
constexpr int kTilesPerBlockOther = 3;
constexpr size_t kStageLimit = 65536; // LDS bytes a single-table launch may use

struct SingleArgs {
  const double* table;
  const double* x;
  int32_t* out;
  int64_t m;
  int n;
  int bits;     // exponent-hash bits, -1 = automatic
  int cap;      // exponent-hash bin cap; logarithm hash: its bin count |H|
  int c_off;    // byte offset of the bin table in LDS
  int scr_off;  // byte offset of one int of LDS scratch
};

// The caller issues the first tile's loads (first_tile) before its own setup
// (table staging, bin build) so that their latency overlaps that setup.
template <int Q>
__device__ __forceinline__ void first_tile(const double* __restrict__ x, int64_t m,
                                           double (&cur)[Q]) {
  const int nt = blockDim.x;
  const int64_t per_tile = (int64_t)nt * Q;
  const int64_t t = blockIdx.x;
  if (t * per_tile < m) load_tile<Q>(x, m, t * per_tile + threadIdx.x, nt, (t + 1) * per_tile <= m, cur);
}

// CONV = 1 answers in the paper's convention (convention_in/_out around the
// search); n is the table size.
template <int Q, int CONV, typename Search>
__device__ __forceinline__ void stream_tiles(const double* __restrict__ x, int64_t m,
                                             int32_t* __restrict__ out, double (&cur)[Q], int n,
                                             Search&& search) {
  const int nt = blockDim.x;
  const int64_t per_tile = (int64_t)nt * Q;
  const int64_t ntiles = (m + per_tile - 1) / per_tile;
  int64_t t = blockIdx.x;
  if (t >= ntiles) return;
  double nxt[Q];
  for (;;) {
    const int64_t tn = t + gridDim.x;
    const bool has_next = tn < ntiles;
    if (has_next) load_tile<Q>(x, m, tn * per_tile + threadIdx.x, nt, (tn + 1) * per_tile <= m, nxt);
    int r[Q];
    if constexpr (CONV) {
      double xs[Q];
      convention_in<Q>(cur, xs);
      search(xs, r);
      convention_out<Q>(n, cur, r);
    } else {
      search(cur, r);
    }
    store_tile<Q>(out, m, t * per_tile + threadIdx.x, nt, (t + 1) * per_tile <= m, r);
    if (!has_next) break;
    for (int q = 0; q < Q; ++q) cur[q] = nxt[q];
    t = tn;
  }
}

template <int ALGO, int Q, int CONV>
__global__ __launch_bounds__(1024) void single_kernel(SingleArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  double cur[Q];
  first_tile<Q>(a.x, a.m, cur);
  if constexpr (ALGO == SS_ALGO_BINARY_GLOBAL) {
    const double* __restrict__ tab = a.table;
    const int n = a.n;
    stream_tiles<Q, CONV>(a.x, a.m, a.out, cur, a.n, [&](const double(&xv)[Q], int(&r)[Q]) {
      search_binary_global<Q>(tab, n, xv, r);
    });
    return;
  } else {
    double* sa = reinterpret_cast<double*>(lds);
    const int n = a.n;
    stage_table(sa, a.table, n);
    __syncthreads();
    if constexpr (ALGO == SS_ALGO_EXPHASH) {
      uint16_t* C = reinterpret_cast<uint16_t*>(lds + a.c_off);
      int* scratch = reinterpret_cast<int*>(lds + a.scr_off);
      HashParams hp = choose_hash(sa, n, a.bits, a.cap);
      if (hp.ok) {
        build_bins(sa, n, hp, C, scratch);
        stream_tiles<Q, CONV>(a.x, a.m, a.out, cur, a.n, [&](const double(&xv)[Q], int(&r)[Q]) {
          search_exphash<Q>(sa, C, n, hp, xv, r);
        });
        return;
      }
      // not applicable (negative entries, unordered keys): bisection below
    }
    if constexpr (ALGO == SS_ALGO_LOGHASH) {
      uint16_t* C = reinterpret_cast<uint16_t*>(lds + a.c_off);
      int* scratch = reinterpret_cast<int*>(lds + a.scr_off);
      LogHashParams lp = choose_loghash(sa, n, a.cap);
      if (lp.ok) {
        build_log_bins(sa, n, lp, C, scratch);
        stream_tiles<Q, CONV>(a.x, a.m, a.out, cur, a.n, [&](const double(&xv)[Q], int(&r)[Q]) {
          search_loghash<Q>(sa, C, n, lp, xv, r);
        });
        return;
      }
      // not applicable (a[0] <= 0 or subnormal, a single value): bisection
    }
    if constexpr (ALGO == SS_ALGO_SKIPLIST) {
      double* sk = reinterpret_cast<double*>(lds + a.c_off);
      build_skip_table(sa, n, sk);
      __syncthreads();
      stream_tiles<Q, CONV>(a.x, a.m, a.out, cur, a.n, [&](const double(&xv)[Q], int(&r)[Q]) {
        search_skiplist<Q>(sa, sk, n, xv, r);
      });
      return;
    }
    if constexpr (ALGO == SS_ALGO_BALLOT) {
      stream_tiles<Q, CONV>(a.x, a.m, a.out, cur, a.n, [&](const double(&xv)[Q], int(&r)[Q]) {
        search_ballot<Q>(sa, n, xv, r);
      });
      return;
    }
    stream_tiles<Q, CONV>(a.x, a.m, a.out, cur, a.n, [&](const double(&xv)[Q], int(&r)[Q]) {
      search_binary<Q>(sa, n, xv, r);
    });
  }
}

// ---------------------------------------------------------------------------

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

static int auto_cap(int64_t n) {
  int64_t c = 64;
  while (c < 4 * n && c < 16384) c <<= 1;
  return (int)c;
}

struct SinglePlan {
  int algo;
  int cap;
  size_t lds;
  int c_off, scr_off;
};

// Chooses the kernel and its LDS layout.  Returns SS_OK or an error for a
// forced kernel that cannot run on this table size.
//
// The automatic choice is the staged bisection whenever the table fits in
// LDS.  Measured on MI355X with 1e8 i.i.d. log-uniform targets, each kernel
// at its best tiles per workgroup: n = 100, bisection 545 Gq/s against 512
// for the exponent hash; n = 1000, 522 against 500; n = 2000, 497 against
// 481; n = 4000, 474 against 444.  Small m gives the same order
// (64 graph-replayed calls of 1e2..1e4 targets: n = 110, 3.7 against 5.4
// us per call; n = 4000, 5.6 against 11.3 us).  With the table in LDS the
// search is bound by HBM either way, and each workgroup's bin build (gap
// fill, two barriers, the longest-bin reduction) costs more than the few
// LDS probes it saves.  Plans, whose bin tables are built once per table
// and only copied by each workgroup, are where the hash wins (their tuner
// chooses per table).
static int plan_single(int64_t n, int algo, int cap_opt, SinglePlan* p) {
  const size_t tab_bytes = align_up((size_t)(n + SS_PAD) * sizeof(double), 16);
  const bool stageable = tab_bytes <= kStageLimit;
  if (algo == SS_ALGO_AUTO) algo = stageable ? SS_ALGO_BINARY : SS_ALGO_BINARY_GLOBAL;
  // an empty table is answered by the staged bisection (its +inf sentinel
  // makes every count 0) so that no kernel reads a zero-length table
  if (n == 0) algo = SS_ALGO_BINARY;
  p->algo = algo;
  p->cap = 0;
  p->c_off = p->scr_off = 0;
  if (algo == SS_ALGO_BINARY_GLOBAL) {
    p->lds = 0;
    return SS_OK;
  }
  if (!stageable)
    return fail(SS_ERR_UNSUPPORTED, "table too large to stage in LDS for the forced kernel");
  p->lds = tab_bytes;
  if (algo == SS_ALGO_SKIPLIST) {
    p->c_off = (int)tab_bytes;
    p->lds = tab_bytes + align_up((size_t)((n + 7) / 8 + SS_PAD) * sizeof(double), 16);
    if (p->lds > kStageLimit)
      return fail(SS_ERR_UNSUPPORTED, "table too large to stage in LDS for the skiplist");
    return SS_OK;
  }
  if (algo == SS_ALGO_EXPHASH || algo == SS_ALGO_LOGHASH) {
    int cap = cap_opt > 0 ? cap_opt : auto_cap(n);
    // shrink the bin cap until table + bins + scratch fit
    while (cap > 16 && tab_bytes + align_up((size_t)(cap + 1) * 2, 16) + 16 > kStageLimit) cap >>= 1;
    p->cap = cap;
    p->c_off = (int)tab_bytes;
    p->scr_off = (int)(tab_bytes + align_up((size_t)(cap + 1) * 2, 16));
    p->lds = (size_t)p->scr_off + 16;
    if (p->lds > kStageLimit) {
      p->algo = SS_ALGO_BINARY;
      p->lds = tab_bytes;
    }
  }
  return SS_OK;
}

// Tiles each workgroup of the default grid streams.  The staged bisection
// pays one table copy per workgroup, so small tables take the finest grid:
// measured on MI355X (512 x 8 targets per tile, 1e8 targets, Gq/s at 1 / 2
// / 3 / 4 / 6 tiles): n = 100, 545 / 533 / 517 / 508 / 486; n = 1000, 457 /
// 522 / 517 / 505 / 482; n = 2000, 415 / 493 / 497 / 495 / 483; n = 4000,
// 349 / 445 / 471 / 472 / 474.  The hashes also amortise their bin build.
static int tiles_per_workgroup(int algo, int64_t n) {
  if (algo == SS_ALGO_BINARY) return n <= 128 ? 1 : n <= 1024 ? 2 : n <= 2048 ? 3 : 4;
  if (algo == SS_ALGO_EXPHASH || algo == SS_ALGO_LOGHASH) return kTilesPerBlockHash;
  return kTilesPerBlockOther;
}

template <int Q, int CONV>
static const void* single_kernel_ptr(int algo) {
  switch (algo) {
    case SS_ALGO_BINARY: return reinterpret_cast<const void*>(&single_kernel<SS_ALGO_BINARY, Q, CONV>);
    case SS_ALGO_BALLOT: return reinterpret_cast<const void*>(&single_kernel<SS_ALGO_BALLOT, Q, CONV>);
    case SS_ALGO_EXPHASH: return reinterpret_cast<const void*>(&single_kernel<SS_ALGO_EXPHASH, Q, CONV>);
    case SS_ALGO_BINARY_GLOBAL:
      return reinterpret_cast<const void*>(&single_kernel<SS_ALGO_BINARY_GLOBAL, Q, CONV>);
    case SS_ALGO_LOGHASH:
      return reinterpret_cast<const void*>(&single_kernel<SS_ALGO_LOGHASH, Q, CONV>);
    case SS_ALGO_SKIPLIST:
      return reinterpret_cast<const void*>(&single_kernel<SS_ALGO_SKIPLIST, Q, CONV>);
    default: return nullptr;
  }
}

static int check_single_args(const double* table, int64_t n, const double* x, int64_t m,
                             const int32_t* out) {
  if (n < 0 || m < 0) return fail(SS_ERR_INVALID_ARG, "negative size");
  if (n > INT32_MAX) return fail(SS_ERR_INVALID_ARG, "n exceeds INT32_MAX");
  if (m == 0) return SS_OK;
  int rc;
  if ((rc = check_span(table, n, sizeof(double), alignof(double), "table")) != SS_OK) return rc;
  if ((rc = check_span(x, m, sizeof(double), alignof(double), "targets")) != SS_OK) return rc;
  if ((rc = check_span(out, m, sizeof(int32_t), alignof(int32_t), "out_idx")) != SS_OK) return rc;
  if (overlaps(out, (size_t)m * 4, x, (size_t)m * 8) ||
      overlaps(out, (size_t)m * 4, table, (size_t)n * 8))
    return fail(SS_ERR_INVALID_ARG, "out_idx overlaps an input");
  if (n > 0 && (rc = check_device_ptr(table, "table")) != SS_OK) return rc;
  if ((rc = check_device_ptr(x, "targets")) != SS_OK) return rc;
  if ((rc = check_device_ptr(out, "out_idx")) != SS_OK) return rc;
  return SS_OK;
}

int launch_single(const double* table, int64_t n, const double* x, int64_t m, int32_t* out,
                  int algo, int bits) {
  if (algo < SS_ALGO_AUTO || algo > SS_ALGO_SKIPLIST || algo == SS_ALGO_LEARNED)
    return fail(SS_ERR_INVALID_ARG, "unknown single-table algorithm");
  if (bits < -1 || bits > SS_MAX_BITS) return fail(SS_ERR_INVALID_ARG, "bucket_bits: -1..20");
  int rc = check_single_args(table, n, x, m, out);
  if (rc != SS_OK || m == 0) return rc;
  DeviceInfo di;
  if ((rc = device_info(&di)) != SS_OK) return rc;
  SinglePlan p;
  if ((rc = plan_single(n, algo, (int)option(SS_OPT_BUCKET_CAP), &p)) != SS_OK) return rc;
  int nt = (int)option(SS_OPT_BLOCK_SIZE);
  if (nt == 0) nt = kDefaultBlock;
  int q = (int)option(SS_OPT_TARGETS_PER_LANE);
  int64_t grid = option(SS_OPT_GRID_BLOCKS);
  const bool conv = option(SS_OPT_CONVENTION) != 0;
  auto kernel_for = [&](int qq) {
    return qq == 4 ? (conv ? single_kernel_ptr<4, 1>(p.algo) : single_kernel_ptr<4, 0>(p.algo))
                   : (conv ? single_kernel_ptr<8, 1>(p.algo) : single_kernel_ptr<8, 0>(p.algo));
  };
  // A small call (at most three passes of the resident workgroups at the
  // default shape) takes four targets per lane and a grid of one pass, each
  // workgroup looping over its tiles: no partly filled last pass.  Measured
  // per call on a 110-entry table: 1e6 targets 5.07 -> 4.76 us, 5e6
  // 13.65 -> 12.26, 1e7 22.4 -> 21.8; at 2e7 (4.8 passes) the default shape
  // was faster, 40.0 against 42.0.
  bool small = false;
  if (q == 0 && grid <= 0) {
    const int64_t tiles8 = (m + (int64_t)nt * kDefaultQ - 1) / ((int64_t)nt * kDefaultQ);
    const int64_t resident8 =
        (int64_t)blocks_per_cu(kernel_for(kDefaultQ), nt, p.lds) * di.num_cus;
    small = tiles8 <= 3 * resident8;
  }
  if (q == 0) q = small ? 4 : kDefaultQ;
  const void* kern = kernel_for(q);
  const int64_t per_tile = (int64_t)nt * q;
  const int64_t ntiles = (m + per_tile - 1) / per_tile;
  if (grid <= 0) {
    const int64_t resident = (int64_t)blocks_per_cu(kern, nt, p.lds) * di.num_cus;
    grid = small ? resident : std::max<int64_t>(resident, ntiles / tiles_per_workgroup(p.algo, n));
  }
  grid = std::max<int64_t>(1, std::min<int64_t>(grid, ntiles));
  SingleArgs a{table, x, out, m, (int)n, bits, p.cap, p.c_off, p.scr_off};
  void* args[] = {&a};
  hipError_t e = hipLaunchKernel(kern, dim3((unsigned)grid), dim3(nt), args, p.lds,
                                 current_stream());
  if (e != hipSuccess) return hip_fail(e, "hipLaunchKernel(single)");
  return SS_OK;
}

// ---------------------------------------------------------------------------
// Table validation: smallest i with a[i] NaN or a[i] > a[i+1].

__global__ void validate_kernel(const double* __restrict__ a, int64_t n,
                                unsigned long long* __restrict__ bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double v = a[i];
    const bool broken = (v != v) || (i + 1 < n && v > a[i + 1]);
    if (broken) atomicMin(bad, (unsigned long long)i);
  }
}

// Bin table of one table into global memory (one workgroup).  info receives
// {s, kmin, nb, K} or s = -1 if the exponent hash does not apply.
__global__ __launch_bounds__(1024) void bins_kernel(const double* __restrict__ a, int n, int bits,
                                                    int cap, int32_t* __restrict__ counts,
                                                    int64_t* __restrict__ info) {
  __shared__ int scratch;
  HashParams hp = choose_hash(a, n, bits, cap);
  if (!hp.ok) {
    if (threadIdx.x == 0) info[0] = -1;
    return;
  }
  build_bins(a, n, hp, counts, &scratch);
  if (threadIdx.x == 0) {
    info[0] = SS_MAX_BITS - hp.shift;
    info[1] = hp.kmin;
    info[2] = hp.nb;
    info[3] = hp.K;
  }
}

// Log-hash bin table of one table into global memory (one workgroup).
// info receives {nb, K, e0, lm0, S, phi}, or nb = -1 if not applicable.
__global__ __launch_bounds__(1024) void log_bins_kernel(const double* __restrict__ a, int n,
                                                        int nb, int32_t* __restrict__ counts,
                                                        double* __restrict__ info) {
  __shared__ int scratch;
  LogHashParams p = choose_loghash(a, n, nb);
  if (!p.ok) {
    if (threadIdx.x == 0) info[0] = -1;
    return;
  }
  build_log_bins(a, n, p, counts, &scratch);
  if (threadIdx.x == 0) {
    info[0] = p.nb;
    info[1] = p.K;
    info[2] = p.e0;
    info[3] = p.lm0;
    info[4] = p.S;
    info[5] = p.phi;
  }
}

}  // namespace ss

extern "C" {

int search_sorted_batch(const double* table, int64_t n, const double* targets, int64_t m,
                        int32_t* out_idx) {
  ss::clear_error();
  return ss::launch_single(table, n, targets, m, out_idx,
                           (int)ss::option(SS_OPT_FORCE_ALGO),
                           (int)ss::option(SS_OPT_BUCKET_BITS));
}

int ss_search_with(const double* table, int64_t n, const double* targets, int64_t m,
                   int32_t* out_idx, int algo, int bucket_bits) {
  ss::clear_error();
  return ss::launch_single(table, n, targets, m, out_idx, algo, bucket_bits);
}

int ss_validate_table(const double* table, int64_t n, int64_t* bad_index_out) {
  ss::clear_error();
  if (!bad_index_out) return ss::fail(SS_ERR_INVALID_ARG, "bad_index_out is null");
  if (n < 0 || n > INT32_MAX) return ss::fail(SS_ERR_INVALID_ARG, "n out of range");
  int rc = ss::check_span(table, n, sizeof(double), alignof(double), "table");
  if (rc != SS_OK) return rc;
  *bad_index_out = -1;
  if (n == 0) return SS_OK;
  if ((rc = ss::check_device_ptr(table, "table")) != SS_OK) return rc;
  unsigned long long* d_bad = nullptr;
  SS_TRY_HIP(hipMalloc(&d_bad, sizeof(unsigned long long)));
  const unsigned long long init = ~0ULL;
  hipStream_t st = ss::current_stream();
  unsigned long long host_bad = init;
  hipError_t e = hipMemcpyAsync(d_bad, &init, sizeof(init), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(ss::validate_kernel, dim3((unsigned)blocks), dim3(256), 0, st, table, n,
                       d_bad);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&host_bad, d_bad, sizeof(host_bad), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d_bad);
  if (e != hipSuccess) return ss::hip_fail(e, "ss_validate_table");
  *bad_index_out = host_bad == init ? -1 : (int64_t)host_bad;
  return SS_OK;
}

int ss_exphash_bins(const double* table, int64_t n, int bucket_bits, int32_t* counts,
                    int64_t cap, int64_t* info_out) {
  ss::clear_error();
  if (!info_out) return ss::fail(SS_ERR_INVALID_ARG, "info_out is null");
  if (n < 1 || n > 65535) return ss::fail(SS_ERR_INVALID_ARG, "n must be in 1..65535");
  if (bucket_bits < -1 || bucket_bits > SS_MAX_BITS)
    return ss::fail(SS_ERR_INVALID_ARG, "bucket_bits: -1..20");
  if (cap < 2 || cap > (1 << 24)) return ss::fail(SS_ERR_INVALID_ARG, "cap must be in 2..2^24");
  int rc = ss::check_span(table, n, sizeof(double), alignof(double), "table");
  if (rc == SS_OK) rc = ss::check_span(counts, cap, sizeof(int32_t), alignof(int32_t), "counts");
  if (rc != SS_OK) return rc;
  if ((rc = ss::check_device_ptr(table, "table")) != SS_OK) return rc;
  if ((rc = ss::check_device_ptr(counts, "counts")) != SS_OK) return rc;
  int64_t* d_info = nullptr;
  SS_TRY_HIP(hipMalloc(&d_info, 4 * sizeof(int64_t)));
  hipStream_t st = ss::current_stream();
  int64_t h_info[4] = {-1, 0, 0, 0};
  hipError_t e = hipMemcpyAsync(d_info, h_info, sizeof(h_info), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(ss::bins_kernel, dim3(1), dim3(1024), 0, st, table, (int)n, bucket_bits,
                       (int)(cap - 1), counts, d_info);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h_info, d_info, sizeof(h_info), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d_info);
  if (e != hipSuccess) return ss::hip_fail(e, "ss_exphash_bins");
  if (h_info[0] < 0)
    return ss::fail(SS_ERR_INVALID_ARG,
                    "exponent hash not applicable (sign bit of a[0], unordered keys or cap)");
  for (int i = 0; i < 4; ++i) info_out[i] = h_info[i];
  return SS_OK;
}

int ss_loghash_bins(const double* table, int64_t n, int64_t nb, int32_t* counts,
                    double* info_out) {
  ss::clear_error();
  if (!info_out) return ss::fail(SS_ERR_INVALID_ARG, "info_out is null");
  if (n < 2 || n > 65535) return ss::fail(SS_ERR_INVALID_ARG, "n must be in 2..65535");
  if (nb < 1 || nb > 65535) return ss::fail(SS_ERR_INVALID_ARG, "nb must be in 1..65535");
  int rc = ss::check_span(table, n, sizeof(double), alignof(double), "table");
  if (rc == SS_OK) rc = ss::check_span(counts, nb + 1, sizeof(int32_t), alignof(int32_t), "counts");
  if (rc != SS_OK) return rc;
  if ((rc = ss::check_device_ptr(table, "table")) != SS_OK) return rc;
  if ((rc = ss::check_device_ptr(counts, "counts")) != SS_OK) return rc;
  double* d_info = nullptr;
  SS_TRY_HIP(hipMalloc(&d_info, 6 * sizeof(double)));
  hipStream_t st = ss::current_stream();
  double h_info[6] = {-1, 0, 0, 0, 0, 0};
  hipError_t e = hipMemcpyAsync(d_info, h_info, sizeof(h_info), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(ss::log_bins_kernel, dim3(1), dim3(1024), 0, st, table, (int)n, (int)nb,
                       counts, d_info);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h_info, d_info, sizeof(h_info), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d_info);
  if (e != hipSuccess) return ss::hip_fail(e, "ss_loghash_bins");
  if (h_info[0] < 0)
    return ss::fail(SS_ERR_INVALID_ARG,
                    "log hash not applicable (needs a normal 0 < a[0] < a[n-1] < inf)");
  for (int i = 0; i < 6; ++i) info_out[i] = h_info[i];
  return SS_OK;
}

}  // extern "C"

namespace ss {
#if SS_DEVICE_CHECKS
namespace {
// Stores an index of 5 clamped into a region of 3: one counted violation
// and out[0] = 2; no access leaves the one-int buffer.
__global__ void checks_selftest_kernel(int* out) { out[0] = SS_IN(5, 0, 3); }
}  // namespace
#endif

int violations_single(unsigned long long* out) { return read_violations(out); }

int checks_selftest() {
#if SS_DEVICE_CHECKS
  int* d = nullptr;
  SS_TRY_HIP(hipMalloc(&d, sizeof(int)));
  hipLaunchKernelGGL(checks_selftest_kernel, dim3(1), dim3(1), 0, current_stream(), d);
  hipError_t e = hipGetLastError();
  int v = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&v, d, sizeof(int), hipMemcpyDeviceToHost,
                                          current_stream());
  if (e == hipSuccess) e = hipStreamSynchronize(current_stream());
  (void)hipFree(d);
  if (e != hipSuccess) return hip_fail(e, "bounds-check self-test");
  return v == 2 ? SS_OK : fail(SS_ERR_HIP, "bounds-check self-test stored an unclamped index");
#else
  return fail(SS_ERR_UNSUPPORTED, "not a device-checked build");
#endif
}
}  // namespace ss
