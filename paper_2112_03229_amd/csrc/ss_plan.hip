// Many tables in one launch: plans, the autotuner's per-table choices, the
// device-built exponent-hash bin tables, the persistent work-queue kernel
// (batched and paired forms) and the HIP graph that launches it.
//
// A plan splits every table's targets into chunks (the tile shape the tuner
// picks), orders the chunks longest first, and runs one persistent grid in
// which each workgroup pops chunks from an atomic counter.  On popping a
// chunk of a table it has not staged, the workgroup copies that table and
// its precomputed bin table from global memory into LDS (a table change is
// the only restaging); the first tile's targets are requested before the
// copy so their latency overlaps it.  Inside a chunk, tiles are streamed
// sequentially with the next tile prefetched, exactly as in the
// single-table kernels.  The counter is zeroed by a one-thread kernel node
// that precedes the search node in the plan's graph.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "ss_device.h"
#include "ss_host.h"
#include "ss_tuner.h"

namespace ss {

struct TableDesc {
  int64_t tab_off;   // first entry in the tables array
  int64_t bins_off;  // first entry in the bin pool (exponent hash), else 0
  int n;
  int algo;          // SS_ALGO_BINARY or SS_ALGO_EXPHASH
  int shift, kmin, kmaxc, nb, K;
  int pad_;
};

struct Chunk {
  int32_t table;     // table (batched) or material (paired) index
  int32_t pad_;
  int64_t q0, q1;    // target positions [q0, q1)
};

struct MultiArgs {
  const double* tables_a;
  const double* tables_b;
  const TableDesc* desc;     // [T] batched; [2M] paired (density, then temperature)
  const uint16_t* bins;
  const Chunk* chunks;
  unsigned int* counter;
  const double* xa;
  int32_t* oa;
  const double* xb;
  int32_t* ob;
  int nchunks;
  int pair_base;             // index of the first temperature descriptor (paired)
  int lds_bins_a, lds_tab_b, lds_bins_b;  // byte offsets in LDS
};

__global__ void reset_counter_kernel(unsigned int* counter) { *counter = 0u; }

// Copies one table (+inf padded) and, for the exponent hash, its bin table
// into LDS.  Returns the search parameters.
__device__ __forceinline__ HashParams stage_desc(const TableDesc& d, const double* __restrict__ tables,
                                                 const uint16_t* __restrict__ bins, double* sa,
                                                 uint16_t* C) {
  stage_table(sa, tables + d.tab_off, d.n);
  HashParams hp{0, d.shift, d.kmin, d.kmaxc, d.nb, d.K};
  if (d.algo == SS_ALGO_EXPHASH) {
    hp.ok = 1;
    const uint16_t* src = bins + d.bins_off;
    for (int b = threadIdx.x; b <= d.nb; b += blockDim.x) C[b] = src[b];
  }
  return hp;
}

template <int Q>
__device__ __forceinline__ void search_desc(const HashParams& hp, const double* sa,
                                            const uint16_t* C, int n, const double (&x)[Q],
                                            int (&r)[Q]) {
  if (hp.ok) search_exphash<Q>(sa, C, n, hp, x, r);
  else search_binary<Q>(sa, n, x, r);
}

template <int Q>
__device__ __forceinline__ void load_range_tile(const double* __restrict__ x, int64_t q0, int64_t q1,
                                                int64_t t, double (&v)[Q]) {
  const int nt = blockDim.x;
  const int64_t per_tile = (int64_t)nt * Q;
  const int64_t base = q0 + t * per_tile;
  load_tile<Q>(x, q1, base + threadIdx.x, nt, base + per_tile <= q1, v);
}

template <int PAIRED, int Q>
__global__ __launch_bounds__(1024) void multi_kernel(MultiArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ int s_chunk;
  double* sa = reinterpret_cast<double*>(lds);
  uint16_t* Ca = reinterpret_cast<uint16_t*>(lds + a.lds_bins_a);
  double* sb = reinterpret_cast<double*>(lds + a.lds_tab_b);
  uint16_t* Cb = reinterpret_cast<uint16_t*>(lds + a.lds_bins_b);
  const int nt = blockDim.x;
  const int64_t per_tile = (int64_t)nt * Q;
  int staged = -1;
  HashParams hpa{}, hpb{};
  int na = 0, nb_ = 0;
  for (;;) {
    if (threadIdx.x == 0) s_chunk = (int)atomicAdd(a.counter, 1u);
    __syncthreads();
    const int c = s_chunk;
    __syncthreads();  // every lane has read s_chunk before it is written again
    if (c >= a.nchunks) break;
    const Chunk ch = a.chunks[c];
    const int64_t mq = ch.q1 - ch.q0;
    const int64_t ntiles = (mq + per_tile - 1) / per_tile;
    double ca[Q], cb[Q];
    load_range_tile<Q>(a.xa, ch.q0, ch.q1, 0, ca);
    if constexpr (PAIRED) load_range_tile<Q>(a.xb, ch.q0, ch.q1, 0, cb);
    if (ch.table != staged) {
      const TableDesc da = a.desc[ch.table];
      hpa = stage_desc(da, a.tables_a, a.bins, sa, Ca);
      na = da.n;
      if constexpr (PAIRED) {
        const TableDesc db = a.desc[a.pair_base + ch.table];
        hpb = stage_desc(db, a.tables_b, a.bins, sb, Cb);
        nb_ = db.n;
      }
      staged = ch.table;
      __syncthreads();
    }
    for (int64_t t = 0;; ++t) {
      const bool has_next = t + 1 < ntiles;
      double xa_n[Q], xb_n[Q];
      if (has_next) {
        load_range_tile<Q>(a.xa, ch.q0, ch.q1, t + 1, xa_n);
        if constexpr (PAIRED) load_range_tile<Q>(a.xb, ch.q0, ch.q1, t + 1, xb_n);
      }
      const int64_t base = ch.q0 + t * per_tile;
      const bool full = base + per_tile <= ch.q1;
      int r[Q];
      search_desc<Q>(hpa, sa, Ca, na, ca, r);
      store_tile<Q>(a.oa, ch.q1, base + threadIdx.x, nt, full, r);
      if constexpr (PAIRED) {
        search_desc<Q>(hpb, sb, Cb, nb_, cb, r);
        store_tile<Q>(a.ob, ch.q1, base + threadIdx.x, nt, full, r);
      }
      if (!has_next) break;
      for (int q = 0; q < Q; ++q) {
        ca[q] = xa_n[q];
        if constexpr (PAIRED) cb[q] = xb_n[q];
      }
    }
  }
}

// Builds every exponent-hash table's bins into the pool (one workgroup per
// table) with the same routine the single-table kernels run in LDS, and
// reports the longest bin it measured.
__global__ __launch_bounds__(256) void plan_bins_kernel(const double* __restrict__ tables_a,
                                                        const double* __restrict__ tables_b,
                                                        int pair_base, const TableDesc* desc,
                                                        uint16_t* pool, int* k_out) {
  __shared__ int scratch;
  const int t = blockIdx.x;
  const TableDesc d = desc[t];
  if (d.algo != SS_ALGO_EXPHASH) {
    if (threadIdx.x == 0) k_out[t] = 0;
    return;
  }
  const double* tab = (pair_base > 0 && t >= pair_base ? tables_b : tables_a) + d.tab_off;
  HashParams hp{1, d.shift, d.kmin, d.kmaxc, d.nb, 0};
  build_bins(tab, d.n, hp, pool + d.bins_off, &scratch);
  if (threadIdx.x == 0) k_out[t] = hp.K;
}

}  // namespace ss

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------

struct ss_plan {
  int paired = 0;
  int32_t T = 0;                 // descriptors (batched: tables; paired: 2 * materials)
  int32_t M = 0;                 // materials (paired)
  int64_t total_queries = 0;
  int device = -1;
  std::vector<int64_t> query_off;
  std::vector<ss::TableDesc> desc;
  std::vector<ss::TunedTable> tuned;
  ss::TableDesc* d_desc = nullptr;
  uint16_t* d_bins = nullptr;
  ss::Chunk* d_chunks = nullptr;
  unsigned int* d_counter = nullptr;
  int* d_k = nullptr;
  int nchunks = 0;
  int64_t chunk_targets = 0;
  int grid = 0, block = 0, q = 0;
  size_t lds = 0;
  int max_k = 0;
  ss::MultiArgs args{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t search_node = nullptr;
  int64_t graph_uses = 0;
  const void* kernel = nullptr;

  ~ss_plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (d_desc) (void)hipFree(d_desc);
    if (d_bins) (void)hipFree(d_bins);
    if (d_chunks) (void)hipFree(d_chunks);
    if (d_counter) (void)hipFree(d_counter);
    if (d_k) (void)hipFree(d_k);
  }
};

namespace ss {

namespace {

constexpr int kPlanBlock = 512;
constexpr int kPlanQ = 8;
constexpr int kPairQ = 4;
// LDS a plan's workgroup may use (tables + bin tables): three 512-thread
// workgroups per CU fit in 160 KB.
constexpr size_t kPlanLdsBudget = 48 * 1024;
constexpr int kWorkgroupsPerCuEstimate = 3;

int check_offsets(const int64_t* off, int32_t T, const char* name, int64_t max_len) {
  if (!off) return fail(SS_ERR_INVALID_ARG, std::string(name) + " is null");
  if (off[0] != 0) return fail(SS_ERR_INVALID_ARG, std::string(name) + "[0] must be 0");
  for (int32_t t = 0; t < T; ++t) {
    const int64_t len = off[t + 1] - off[t];
    if (len < 0) return fail(SS_ERR_INVALID_ARG, std::string(name) + " must be non-decreasing");
    if (len > max_len)
      return fail(SS_ERR_INVALID_ARG, std::string(name) + ": segment " + std::to_string(t) +
                                          " longer than " + std::to_string(max_len));
  }
  return SS_OK;
}

// Fills desc[i] from a tuned choice; bin pool offsets are assigned in order.
void describe(const TunedTable& tt, int64_t tab_off, TableDesc* d, int64_t* pool_len) {
  d->tab_off = tab_off;
  d->n = tt.n;
  d->algo = tt.algo;
  d->shift = tt.algo == SS_ALGO_EXPHASH ? SS_MAX_BITS - tt.bits : 0;
  d->kmin = tt.kmin;
  d->kmaxc = tt.kmaxc;
  d->nb = tt.nb;
  d->K = tt.K;
  d->bins_off = 0;
  if (tt.algo == SS_ALGO_EXPHASH) {
    d->bins_off = *pool_len;
    *pool_len += tt.nb + 1;
    *pool_len = (*pool_len + 7) / 8 * 8;  // 16-byte aligned starts
  }
}

size_t align16(size_t v) { return (v + 15) / 16 * 16; }

int fail_delete(ss_plan* p, const char* msg, int code = SS_ERR_INVALID_ARG) {
  delete p;
  return msg ? fail(code, msg) : code;
}

int finish_plan(ss_plan* p, const double* tables_a, const double* tables_b, int64_t pool_len,
                size_t lds_tab_a, size_t lds_bins_a, size_t lds_tab_b, size_t lds_bins_b) {
  hipStream_t st = current_stream();
  const int T = p->T;
  SS_TRY_HIP(hipMalloc(&p->d_desc, sizeof(TableDesc) * T));
  SS_TRY_HIP(hipMalloc(&p->d_bins, sizeof(uint16_t) * std::max<int64_t>(pool_len, 8)));
  SS_TRY_HIP(hipMalloc(&p->d_counter, sizeof(unsigned int)));
  SS_TRY_HIP(hipMalloc(&p->d_k, sizeof(int) * T));
  SS_TRY_HIP(hipMemcpyAsync(p->d_desc, p->desc.data(), sizeof(TableDesc) * T,
                            hipMemcpyHostToDevice, st));
  SS_TRY_HIP(hipMemsetAsync(p->d_counter, 0, sizeof(unsigned int), st));
  hipLaunchKernelGGL(plan_bins_kernel, dim3(T), dim3(256), 0, st, tables_a, tables_b,
                     p->paired ? p->M : 0, p->d_desc, p->d_bins, p->d_k);
  SS_TRY_HIP(hipGetLastError());
  std::vector<int> k(T);
  SS_TRY_HIP(hipMemcpyAsync(k.data(), p->d_k, sizeof(int) * T, hipMemcpyDeviceToHost, st));
  SS_TRY_HIP(hipStreamSynchronize(st));
  // the device's measured longest bin must match the tuner's (same table bytes)
  for (int t = 0; t < T; ++t) {
    if (p->desc[t].algo != SS_ALGO_EXPHASH) continue;
    const int want = std::min(p->desc[t].K, SS_SCAN_MAX + 1);
    if (k[t] != want)
      return fail(SS_ERR_INVALID_ARG, "table " + std::to_string(t) +
                                          " changed during plan creation or is not sorted");
    p->max_k = std::max(p->max_k, k[t]);
  }

  // chunks: each segment split into chunk_targets pieces, longest first
  std::vector<Chunk> chunks;
  const int nsegs = p->paired ? p->M : p->T;
  for (int s = 0; s < nsegs; ++s) {
    for (int64_t q0 = p->query_off[s]; q0 < p->query_off[s + 1]; q0 += p->chunk_targets) {
      Chunk c;
      c.table = s;
      c.pad_ = 0;
      c.q0 = q0;
      c.q1 = std::min(q0 + p->chunk_targets, p->query_off[s + 1]);
      chunks.push_back(c);
    }
  }
  std::stable_sort(chunks.begin(), chunks.end(), [](const Chunk& x, const Chunk& y) {
    return (x.q1 - x.q0) > (y.q1 - y.q0);
  });
  if (chunks.size() > (size_t)INT32_MAX) return fail(SS_ERR_INVALID_ARG, "too many chunks");
  p->nchunks = (int)chunks.size();
  if (p->nchunks > 0) {
    SS_TRY_HIP(hipMalloc(&p->d_chunks, sizeof(Chunk) * chunks.size()));
    SS_TRY_HIP(hipMemcpy(p->d_chunks, chunks.data(), sizeof(Chunk) * chunks.size(),
                         hipMemcpyHostToDevice));
  }

  p->lds = lds_tab_a + lds_bins_a + lds_tab_b + lds_bins_b;
  p->block = kPlanBlock;
  p->q = p->paired ? kPairQ : kPlanQ;
  p->kernel = p->paired ? reinterpret_cast<const void*>(&multi_kernel<1, kPairQ>)
                        : reinterpret_cast<const void*>(&multi_kernel<0, kPlanQ>);
  DeviceInfo di;
  int rc = device_info(&di);
  if (rc != SS_OK) return rc;
  p->device = di.device;
  const int resident = blocks_per_cu(p->kernel, p->block, p->lds) * di.num_cus;
  p->grid = std::max(1, std::min(resident, std::max(p->nchunks, 1)));

  MultiArgs& a = p->args;
  a.tables_a = tables_a;
  a.tables_b = tables_b;
  a.desc = p->d_desc;
  a.bins = p->d_bins;
  a.chunks = p->d_chunks;
  a.counter = p->d_counter;
  a.nchunks = p->nchunks;
  a.pair_base = p->paired ? p->M : 0;
  a.lds_bins_a = (int)lds_tab_a;
  a.lds_tab_b = (int)(lds_tab_a + lds_bins_a);
  a.lds_bins_b = (int)(lds_tab_a + lds_bins_a + lds_tab_b);

  // graph: counter reset -> persistent search
  SS_TRY_HIP(hipGraphCreate(&p->graph, 0));
  hipGraphNode_t reset_node;
  hipKernelNodeParams rp{};
  void* rargs[] = {&p->d_counter};
  rp.func = reinterpret_cast<void*>(&reset_counter_kernel);
  rp.gridDim = dim3(1);
  rp.blockDim = dim3(1);
  rp.sharedMemBytes = 0;
  rp.kernelParams = rargs;
  rp.extra = nullptr;
  SS_TRY_HIP(hipGraphAddKernelNode(&reset_node, p->graph, nullptr, 0, &rp));
  hipKernelNodeParams kp{};
  void* kargs[] = {&p->args};
  kp.func = const_cast<void*>(p->kernel);
  kp.gridDim = dim3(p->grid);
  kp.blockDim = dim3(p->block);
  kp.sharedMemBytes = (unsigned)p->lds;
  kp.kernelParams = kargs;
  kp.extra = nullptr;
  SS_TRY_HIP(hipGraphAddKernelNode(&p->search_node, p->graph, &reset_node, 1, &kp));
  SS_TRY_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
  return SS_OK;
}

int run_plan(ss_plan* p, const double* xa, int32_t* oa, const double* xb, int32_t* ob) {
  if (p->total_queries == 0 || p->nchunks == 0) return SS_OK;
  int dev = -1;
  SS_TRY_HIP(hipGetDevice(&dev));
  if (dev != p->device) return fail(SS_ERR_INVALID_ARG, "plan was built on another device");
  if (xa != p->args.xa || oa != p->args.oa || xb != p->args.xb || ob != p->args.ob) {
    p->args.xa = xa;
    p->args.oa = oa;
    p->args.xb = xb;
    p->args.ob = ob;
    hipKernelNodeParams kp{};
    void* kargs[] = {&p->args};
    kp.func = const_cast<void*>(p->kernel);
    kp.gridDim = dim3(p->grid);
    kp.blockDim = dim3(p->block);
    kp.sharedMemBytes = (unsigned)p->lds;
    kp.kernelParams = kargs;
    kp.extra = nullptr;
    SS_TRY_HIP(hipGraphExecKernelNodeSetParams(p->exec, p->search_node, &kp));
  }
  SS_TRY_HIP(hipGraphLaunch(p->exec, current_stream()));
  ++p->graph_uses;
  return SS_OK;
}

}  // namespace

}  // namespace ss

using namespace ss;

extern "C" {

int ss_multi_plan_create(const double* tables, const int64_t* table_off, int32_t T,
                         const int64_t* query_off, ss_plan** out) {
  clear_error();
  if (!out) return fail(SS_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  if (T < 1 || T > (1 << 20)) return fail(SS_ERR_INVALID_ARG, "T must be in 1..2^20");
  int rc = check_offsets(table_off, T, "table_off", 65535);
  if (rc == SS_OK) rc = check_offsets(query_off, T, "query_off", INT64_MAX);
  if (rc != SS_OK) return rc;
  const int64_t total_n = table_off[T];
  if ((rc = check_span(tables, total_n, sizeof(double), alignof(double), "tables")) != SS_OK)
    return rc;
  if (total_n > 0 && (rc = check_device_ptr(tables, "tables")) != SS_OK) return rc;

  std::vector<double> host(total_n);
  if (total_n > 0) {
    SS_TRY_HIP(hipMemcpyAsync(host.data(), tables, sizeof(double) * total_n,
                              hipMemcpyDeviceToHost, current_stream()));
    SS_TRY_HIP(hipStreamSynchronize(current_stream()));
  }
  ss_plan* p = new (std::nothrow) ss_plan();
  if (!p) return fail(SS_ERR_OOM, "plan");
  p->T = T;
  p->query_off.assign(query_off, query_off + T + 1);
  p->total_queries = query_off[T];
  const TunerModel& model = tuner_model();
  p->desc.resize(T);
  p->tuned.resize(T);
  size_t max_tab = 16, max_bins = 0;
  for (int t = 0; t < T; ++t)
    max_tab = std::max(max_tab, align16((size_t)(table_off[t + 1] - table_off[t] + SS_PAD) * 8));
  if (max_tab > kPlanLdsBudget) return fail_delete(p, "tables too large for LDS");
  int64_t pool = 0;
  for (int t = 0; t < T; ++t) {
    const int n = (int)(table_off[t + 1] - table_off[t]);
    p->tuned[t] = tune_table(model, host.data() + table_off[t], n, kPlanLdsBudget - max_tab);
    describe(p->tuned[t], table_off[t], &p->desc[t], &pool);
    if (p->tuned[t].algo == SS_ALGO_EXPHASH)
      max_bins = std::max(max_bins, align16((size_t)(p->tuned[t].nb + 1) * 2));
  }
  DeviceInfo di;
  if ((rc = device_info(&di)) != SS_OK) return fail_delete(p, nullptr, rc);
  p->chunk_targets = choose_chunk_targets(model, p->total_queries, kPlanBlock * kPlanQ,
                                          max_tab + max_bins,
                                          di.num_cus * kWorkgroupsPerCuEstimate);
  rc = finish_plan(p, tables, nullptr, pool, max_tab, max_bins, 0, 0);
  if (rc != SS_OK) {
    delete p;
    return rc;
  }
  *out = p;
  return SS_OK;
}

int ss_multi_search(ss_plan* p, const double* targets, int32_t* out_idx) {
  clear_error();
  if (!p) return fail(SS_ERR_INVALID_ARG, "plan is null");
  if (p->paired) return fail(SS_ERR_INVALID_ARG, "paired plan: use ss_pair_search");
  const int64_t m = p->total_queries;
  int rc = check_span(targets, m, sizeof(double), alignof(double), "targets");
  if (rc == SS_OK) rc = check_span(out_idx, m, sizeof(int32_t), alignof(int32_t), "out_idx");
  if (rc != SS_OK) return rc;
  if (m > 0 && overlaps(out_idx, (size_t)m * 4, targets, (size_t)m * 8))
    return fail(SS_ERR_INVALID_ARG, "out_idx overlaps targets");
  if (m > 0 && ((rc = check_device_ptr(targets, "targets")) != SS_OK ||
                (rc = check_device_ptr(out_idx, "out_idx")) != SS_OK))
    return rc;
  return run_plan(p, targets, out_idx, nullptr, nullptr);
}

int ss_pair_plan_create(const double* rho_tables, const int64_t* rho_off, const double* t_tables,
                        const int64_t* t_off, int32_t M, const int64_t* pair_off, ss_plan** out) {
  clear_error();
  if (!out) return fail(SS_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  if (M < 1 || M > (1 << 20)) return fail(SS_ERR_INVALID_ARG, "M must be in 1..2^20");
  int rc = check_offsets(rho_off, M, "rho_off", 65535);
  if (rc == SS_OK) rc = check_offsets(t_off, M, "t_off", 65535);
  if (rc == SS_OK) rc = check_offsets(pair_off, M, "pair_off", INT64_MAX);
  if (rc != SS_OK) return rc;
  const int64_t nr = rho_off[M], ntt = t_off[M];
  if ((rc = check_span(rho_tables, nr, 8, 8, "rho_tables")) != SS_OK) return rc;
  if ((rc = check_span(t_tables, ntt, 8, 8, "t_tables")) != SS_OK) return rc;
  if (nr > 0 && (rc = check_device_ptr(rho_tables, "rho_tables")) != SS_OK) return rc;
  if (ntt > 0 && (rc = check_device_ptr(t_tables, "t_tables")) != SS_OK) return rc;
  std::vector<double> hr(nr), ht(ntt);
  hipStream_t st = current_stream();
  if (nr > 0) SS_TRY_HIP(hipMemcpyAsync(hr.data(), rho_tables, 8 * nr, hipMemcpyDeviceToHost, st));
  if (ntt > 0) SS_TRY_HIP(hipMemcpyAsync(ht.data(), t_tables, 8 * ntt, hipMemcpyDeviceToHost, st));
  SS_TRY_HIP(hipStreamSynchronize(st));
  ss_plan* p = new (std::nothrow) ss_plan();
  if (!p) return fail(SS_ERR_OOM, "plan");
  p->paired = 1;
  p->M = M;
  p->T = 2 * M;
  p->query_off.assign(pair_off, pair_off + M + 1);
  p->total_queries = pair_off[M];
  const TunerModel& model = tuner_model();
  p->desc.resize(2 * M);
  p->tuned.resize(2 * M);
  size_t tab_a = 16, bins_a = 0, tab_b = 16, bins_b = 0;
  for (int j = 0; j < M; ++j) {
    tab_a = std::max(tab_a, align16((size_t)(rho_off[j + 1] - rho_off[j] + SS_PAD) * 8));
    tab_b = std::max(tab_b, align16((size_t)(t_off[j + 1] - t_off[j] + SS_PAD) * 8));
  }
  if (tab_a + tab_b > kPlanLdsBudget) return fail_delete(p, "tables too large for LDS");
  // the bin budget is split in proportion to the two axes' largest tables
  const size_t bins_total = kPlanLdsBudget - tab_a - tab_b;
  const size_t budget_a = bins_total * tab_a / (tab_a + tab_b);
  const size_t budget_b = bins_total - budget_a;
  int64_t pool = 0;
  for (int j = 0; j < M; ++j) {
    const int n = (int)(rho_off[j + 1] - rho_off[j]);
    p->tuned[j] = tune_table(model, hr.data() + rho_off[j], n, budget_a);
    describe(p->tuned[j], rho_off[j], &p->desc[j], &pool);
    if (p->tuned[j].algo == SS_ALGO_EXPHASH)
      bins_a = std::max(bins_a, align16((size_t)(p->tuned[j].nb + 1) * 2));
  }
  for (int j = 0; j < M; ++j) {
    const int n = (int)(t_off[j + 1] - t_off[j]);
    p->tuned[M + j] = tune_table(model, ht.data() + t_off[j], n, budget_b);
    describe(p->tuned[M + j], t_off[j], &p->desc[M + j], &pool);
    if (p->tuned[M + j].algo == SS_ALGO_EXPHASH)
      bins_b = std::max(bins_b, align16((size_t)(p->tuned[M + j].nb + 1) * 2));
  }
  DeviceInfo di;
  if ((rc = device_info(&di)) != SS_OK) return fail_delete(p, nullptr, rc);
  p->chunk_targets = choose_chunk_targets(model, p->total_queries, kPlanBlock * kPairQ,
                                          tab_a + bins_a + tab_b + bins_b,
                                          di.num_cus * kWorkgroupsPerCuEstimate);
  rc = finish_plan(p, rho_tables, t_tables, pool, tab_a, bins_a, tab_b, bins_b);
  if (rc != SS_OK) {
    delete p;
    return rc;
  }
  *out = p;
  return SS_OK;
}

int ss_pair_search(ss_plan* p, const double* rho, const double* temp, int32_t* out_rho,
                   int32_t* out_t) {
  clear_error();
  if (!p) return fail(SS_ERR_INVALID_ARG, "plan is null");
  if (!p->paired) return fail(SS_ERR_INVALID_ARG, "batched plan: use ss_multi_search");
  const int64_t m = p->total_queries;
  int rc = check_span(rho, m, 8, 8, "rho");
  if (rc == SS_OK) rc = check_span(temp, m, 8, 8, "temp");
  if (rc == SS_OK) rc = check_span(out_rho, m, 4, 4, "out_rho");
  if (rc == SS_OK) rc = check_span(out_t, m, 4, 4, "out_t");
  if (rc != SS_OK) return rc;
  if (m > 0) {
    const size_t ob = (size_t)m * 4, ib = (size_t)m * 8;
    if (overlaps(out_rho, ob, rho, ib) || overlaps(out_rho, ob, temp, ib) ||
        overlaps(out_t, ob, rho, ib) || overlaps(out_t, ob, temp, ib) ||
        overlaps(out_rho, ob, out_t, ob))
      return fail(SS_ERR_INVALID_ARG, "outputs overlap inputs or each other");
    if ((rc = check_device_ptr(rho, "rho")) != SS_OK ||
        (rc = check_device_ptr(temp, "temp")) != SS_OK ||
        (rc = check_device_ptr(out_rho, "out_rho")) != SS_OK ||
        (rc = check_device_ptr(out_t, "out_t")) != SS_OK)
      return rc;
  }
  return run_plan(p, rho, out_rho, temp, out_t);
}

int ss_plan_destroy(ss_plan* p) {
  clear_error();
  delete p;
  return SS_OK;
}

int ss_plan_info(const ss_plan* p, int what, void* out, int64_t cap) {
  clear_error();
  if (!p || !out) return fail(SS_ERR_INVALID_ARG, "null argument");
  switch (what) {
    case SS_PLAN_ALGOS:
    case SS_PLAN_BITS: {
      if (cap < p->T) return fail(SS_ERR_INVALID_ARG, "cap smaller than the table count");
      int32_t* o = static_cast<int32_t*>(out);
      for (int t = 0; t < p->T; ++t)
        o[t] = what == SS_PLAN_ALGOS ? p->tuned[t].algo
                                     : (p->tuned[t].algo == SS_ALGO_EXPHASH ? p->tuned[t].bits : -1);
      return SS_OK;
    }
    case SS_PLAN_SUMMARY: {
      if (cap < 8) return fail(SS_ERR_INVALID_ARG, "cap must be >= 8");
      int64_t* o = static_cast<int64_t*>(out);
      o[0] = p->T;
      o[1] = p->nchunks;
      o[2] = p->chunk_targets;
      o[3] = p->grid;
      o[4] = p->block;
      o[5] = (int64_t)p->lds;
      o[6] = p->max_k;
      o[7] = p->graph_uses;
      return SS_OK;
    }
    default:
      return fail(SS_ERR_INVALID_ARG, "unknown query");
  }
}

}  // extern "C"
