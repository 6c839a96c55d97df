// Batched search with no plan and no allocation: ss_multi_search_noalloc.
//
// ss_multi_search runs over device buffers that plan creation allocates
// (descriptors, tile offsets, workgroup records).  This entry point serves the
// same batched operation to callers that cannot allocate device memory (code
// under HIP graph capture, serving loops that forbid hipMalloc).  Its only
// device memory beyond the caller's inputs and outputs is the file-scope array
// `scratch` below: every GPU the library runs on holds one copy of it until the
// process ends, and every call on that GPU shares it.
//
// Two launches on the caller's stream:
//   1. na_offsets_kernel (one workgroup) reads the caller's device CSR target
//      offsets, clamps them into [0, m] and makes them non-decreasing (a
//      running maximum), then numbers every segment's target tiles back to back
//      (a prefix sum); both arrays go to `scratch`.  Every entry the search
//      reads is rewritten by each call, so nothing needs clearing.
//   2. na_search_kernel: workgroups take ranges of consecutive tiles in a
//      grid-stride loop (every workgroup leaves once the ranges are exhausted),
//      stage each segment's table in LDS once per range and search it by
//      bisection.  Tables longer than the LDS budget are searched in place in
//      global memory.  Tiles are cut at absolute multiples of blockDim.x * Q
//      target positions, as in the plans, so inner tiles cover whole lines.
#include <algorithm>
#include <mutex>
#include <string>

#include "ss_device.h"
#include "ss_host.h"

namespace ss {
namespace {
constexpr int kNaMaxTables = 65536;  // tables per call (bounded by the scratch size)
constexpr int kNaBlock = 512;
constexpr int kNaQ = 8;
constexpr int kNaRange = 4;          // consecutive tiles per workgroup range
constexpr int kNaScanThreads = 1024;
constexpr int kNaMaxStaged = 6136;   // entries staged in LDS (48 KB with the +inf padding)
constexpr size_t kNaLds = (size_t)(kNaMaxStaged + SS_PAD) * sizeof(double);
}  // namespace
}  // namespace ss

// Per GPU: [0, kNaMaxTables] the normalised target offsets of the segments,
// [kNaMaxTables + 1, 2 kNaMaxTables + 1] the first tile of every segment
// (entry T holds the tile count).  1 MiB.  In host code this name is only a
// handle for hipGetSymbolAddress; kernels receive the device address.
static __device__ __align__(256) int64_t scratch[2 * (ss::kNaMaxTables + 1)];

namespace ss {
namespace {

// Block-wide inclusive scan of one value per thread (kNaScanThreads
// threads), with op = sum or max; sh holds kNaScanThreads values.
template <bool MAX>
__device__ int64_t block_inclusive_scan(int64_t v, int64_t* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < kNaScanThreads; off <<= 1) {
    const int64_t o = tid >= off ? sh[tid - off] : (MAX ? INT64_MIN : 0);
    __syncthreads();
    v = MAX ? max(v, o) : v + o;
    sh[tid] = v;
    __syncthreads();
  }
  return v;
}

__global__ __launch_bounds__(kNaScanThreads) void na_offsets_kernel(
    const int64_t* __restrict__ query_off, int T, int64_t m, int64_t per_tile,
    int64_t* __restrict__ qs, int64_t* __restrict__ first) {
  __shared__ int64_t sh[kNaScanThreads];
  const int tid = threadIdx.x;
  // offsets 0..T in contiguous chunks of `per` entries per thread
  const int per = (T + 1 + kNaScanThreads - 1) / kNaScanThreads;
  const int c0 = min(tid * per, T + 1), c1 = min(c0 + per, T + 1);
  // running maximum of the clamped offsets
  int64_t run = INT64_MIN;
  for (int i = c0; i < c1; ++i) run = max(run, min(max(query_off[i], (int64_t)0), m));
  block_inclusive_scan<true>(run, sh);
  int64_t before = tid > 0 ? sh[tid - 1] : INT64_MIN;
  __syncthreads();
  for (int i = c0; i < c1; ++i) {
    before = max(before, min(max(query_off[i], (int64_t)0), m));
    qs[i] = before;
  }
  __syncthreads();  // qs is read across chunks below
  // tiles of segments c0..min(c1, T)-1, then their first tiles
  int64_t cnt = 0;
  for (int s = c0; s < min(c1, T); ++s) {
    const int64_t q0 = qs[s], q1 = qs[s + 1];
    cnt += q1 > q0 ? (q1 - 1) / per_tile - q0 / per_tile + 1 : 0;
  }
  block_inclusive_scan<false>(cnt, sh);
  int64_t f = tid > 0 ? sh[tid - 1] : 0;
  for (int s = c0; s < min(c1, T); ++s) {
    first[s] = f;
    const int64_t q0 = qs[s], q1 = qs[s + 1];
    f += q1 > q0 ? (q1 - 1) / per_tile - q0 / per_tile + 1 : 0;
  }
  if (tid == kNaScanThreads - 1) first[T] = sh[kNaScanThreads - 1];
}

struct NaArgs {
  const double* tables;
  int64_t total_n;
  const int64_t* table_off;
  const int64_t* qs;
  const int64_t* first;
  const double* x;
  int32_t* out;
  int T;
};

template <int CONV>
__global__ __launch_bounds__(kNaBlock) void na_search_kernel(NaArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  double* sa = reinterpret_cast<double*>(lds);
  const int nt = blockDim.x;
  const int64_t per_tile = (int64_t)nt * kNaQ;
  const int64_t total = a.first[a.T];
  const int64_t ranges = (total + kNaRange - 1) / kNaRange;
  int staged = -1;  // segment whose table is in LDS
  const double* gtab = nullptr;
  int n = 0;
  bool in_lds = true;
  for (int64_t rg = blockIdx.x; rg < ranges; rg += gridDim.x) {
    const int64_t j0 = rg * kNaRange, j1 = min(j0 + kNaRange, total);
    // the segment holding tile j0: the largest s with first[s] <= j0
    int lo = 0, hi = a.T;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (a.first[mid] <= j0) lo = mid;
      else hi = mid;
    }
    int s = lo;
    for (int64_t j = j0; j < j1; ++j) {
      while (j >= a.first[s + 1]) ++s;
      if (s != staged) {
        const int64_t t0 = min(max(a.table_off[s], (int64_t)0), a.total_n);
        const int64_t t1 = min(max(a.table_off[s + 1], t0), a.total_n);
        n = (int)min(t1 - t0, (int64_t)INT32_MAX);
        gtab = a.tables + t0;
        in_lds = n <= kNaMaxStaged;
        __syncthreads();  // every lane is done with the previous table
        if (in_lds) stage_table(sa, gtab, n);
        __syncthreads();
        staged = s;
      }
      const int64_t q0 = a.qs[s], q1 = a.qs[s + 1];
      const int64_t b = q0 / per_tile + (j - a.first[s]);
      const int64_t lo_q = max(q0, b * per_tile), hi_q = min((b + 1) * per_tile, q1);
      const bool full = lo_q + per_tile == hi_q;
      double x[kNaQ];
      load_tile<kNaQ>(a.x, hi_q, lo_q + threadIdx.x, nt, full, x);
      int r[kNaQ];
      auto search = [&](const double(&xq)[kNaQ]) {
        if (in_lds) search_binary<kNaQ>(sa, n, xq, r);
        else search_binary_global<kNaQ>(gtab, n, xq, r);
      };
      if constexpr (CONV) {
        double xs[kNaQ];
        convention_in<kNaQ>(x, xs);
        search(xs);
        convention_out<kNaQ>(n, x, r);
      } else {
        search(x);
      }
      store_tile<kNaQ>(a.out, hi_q, lo_q + threadIdx.x, nt, full, r);
    }
  }
}

// Device address of `scratch` on each device, looked up on the first call
// made with that device current.
std::mutex g_na_mu;
void* g_na_scratch[64] = {nullptr};

int scratch_address(int dev, int64_t** out) {
  if (dev < 0 || dev >= 64) return fail(SS_ERR_UNSUPPORTED, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (!g_na_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(SS_ERR_HIP, "hipGetSymbolAddress(scratch) returned null");
    g_na_scratch[dev] = p;
  }
  *out = static_cast<int64_t*>(g_na_scratch[dev]);
  return SS_OK;
}

}  // namespace
}  // namespace ss

extern "C" {

int ss_multi_search_noalloc(const double* tables, int64_t total_n, const int64_t* table_off,
                            int32_t T, const int64_t* query_off, const double* targets, int64_t m,
                            int32_t* out_idx) {
  using namespace ss;
  clear_error();
  if (T < 1 || T > kNaMaxTables)
    return fail(SS_ERR_INVALID_ARG, "T must be in 1..65536 (the size of the device scratch)");
  if (total_n < 0 || m < 0) return fail(SS_ERR_INVALID_ARG, "negative size");
  int rc = check_span(tables, total_n, 8, 8, "tables");
  if (rc == SS_OK) rc = check_span(table_off, (int64_t)T + 1, 8, 8, "table_off");
  if (rc == SS_OK) rc = check_span(query_off, (int64_t)T + 1, 8, 8, "query_off");
  if (rc == SS_OK) rc = check_span(targets, m, 8, 8, "targets");
  if (rc == SS_OK) rc = check_span(out_idx, m, 4, 4, "out_idx");
  if (rc != SS_OK) return rc;
  if (m == 0) return SS_OK;
  const size_t ob = (size_t)m * 4, offb = ((size_t)T + 1) * 8;
  if (overlaps(out_idx, ob, targets, (size_t)m * 8) ||
      overlaps(out_idx, ob, tables, (size_t)total_n * 8) ||
      overlaps(out_idx, ob, table_off, offb) || overlaps(out_idx, ob, query_off, offb))
    return fail(SS_ERR_INVALID_ARG, "out_idx overlaps an input");
  if ((total_n > 0 && (rc = check_device_ptr(tables, "tables")) != SS_OK) ||
      (rc = check_device_ptr(table_off, "table_off")) != SS_OK ||
      (rc = check_device_ptr(query_off, "query_off")) != SS_OK ||
      (rc = check_device_ptr(targets, "targets")) != SS_OK ||
      (rc = check_device_ptr(out_idx, "out_idx")) != SS_OK)
    return rc;
  DeviceInfo di;
  if ((rc = device_info(&di)) != SS_OK) return rc;
  int64_t* scr = nullptr;
  if ((rc = scratch_address(di.device, &scr)) != SS_OK) return rc;
  int64_t* qs = scr;
  int64_t* first = scr + kNaMaxTables + 1;
  const int64_t per_tile = (int64_t)kNaBlock * kNaQ;
  hipStream_t st = current_stream();
  hipLaunchKernelGGL(na_offsets_kernel, dim3(1), dim3(kNaScanThreads), 0, st, query_off, (int)T,
                     m, per_tile, qs, first);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "hipLaunchKernel(offsets)");
  const bool conv = option(SS_OPT_CONVENTION) != 0;
  const void* kern = conv ? reinterpret_cast<const void*>(&na_search_kernel<1>)
                          : reinterpret_cast<const void*>(&na_search_kernel<0>);
  // at most m / per_tile + 2 T tiles: a segment adds at most two partial ones
  const int64_t max_ranges = (m / per_tile + 2 * (int64_t)T + kNaRange) / kNaRange;
  const int64_t resident = (int64_t)blocks_per_cu(kern, kNaBlock, kNaLds) * di.num_cus;
  const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(4 * resident, max_ranges));
  NaArgs a{tables, total_n, table_off, qs, first, targets, out_idx, (int)T};
  void* args[] = {&a};
  e = hipLaunchKernel(kern, dim3((unsigned)grid), dim3(kNaBlock), args, kNaLds, st);
  if (e != hipSuccess) return hip_fail(e, "hipLaunchKernel(search)");
  return SS_OK;
}

}  // extern "C"

namespace ss {
int violations_noalloc(unsigned long long* out) { return read_violations(out); }
}  // namespace ss
