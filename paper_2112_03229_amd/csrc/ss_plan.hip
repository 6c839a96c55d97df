// Many tables in one launch: plans, the autotuner's per-table choices, the
// device-built exponent-hash bin tables, the search kernel (batched and
// paired forms) and the HIP graph that launches it.
//
// Every table's targets are cut into tiles at absolute multiples of
// blockDim.x * Q target positions (so a table's first and last tiles may be
// short and every other tile is aligned: its loads and stores cover whole
// cache lines).  Each segment's tiles (a table's, or one axis of a
// material's) go to workgroups of at most k tiles (k is the tile shape the
// tuner picks), either as contiguous ranges or strided so that the
// segment's workgroups sweep it side by side (SS_OPT_PLAN_ORDER); a
// workgroup never leaves its segment.  The grid is several times the
// resident workgroup count and the hardware dispatcher balances it, exactly
// like the single-table launch.  A workgroup requests its first two tiles'
// targets, stages its segment's table (copying the table and its
// precomputed bin table from global memory into LDS) once, and streams its
// tiles with the next two prefetched.  No atomics, no work queue: a plan is
// one kernel node in its graph.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <cstdio>
#include <sstream>
#include <string>
#include <vector>

#include "ss_device.h"
#include "ss_host.h"
#include "ss_learned.h"
#include "ss_mlp.h"
#include "ss_tuner.h"

namespace ss {

struct TableDesc {
  int64_t tab_off;   // first entry in the tables array
  int64_t bins_off;  // first entry in the bin pool (exponent hash), else 0
  int64_t p_off;     // first float of its compiled model in the image pool (learned), else 0
  int n;
  int algo;          // SS_ALGO_BINARY, SS_ALGO_EXPHASH, SS_ALGO_BALLOT or SS_ALGO_LEARNED
  int shift, kmin, kmaxc, nb, K;
  int E;             // learned: error bound
  float u0, inv;     // learned: input normalisation
  int tail;          // learned, bounded staging: +inf entries after the table
  int pad_;
};

// Everything a workgroup needs to issue its first target loads, in one
// 32-byte record: its segment's target range and tile count, and which of
// the segment's tiles it searches.  Workgroup ranges are cut at segment
// boundaries (the last workgroup of a segment may take fewer tiles), so a
// workgroup stages one table once and never restages mid-range.
struct WgStart {
  int64_t seg_q0;    // the segment's first target
  int64_t seg_q1;    // end of the segment's targets
  int32_t seg;       // segment (table or material)
  int32_t first;     // index of the workgroup's first tile within the segment
  int32_t seg_tiles; // tiles of the segment
  int32_t count;     // tiles of this workgroup
};

// Launch forms of the plan kernel.
enum PlanMode {
  kBatched = 0,    // one target array, one table per segment
  kPairJoint = 1,  // paired: a workgroup searches a tile of both axes (both tables staged)
  kPairSplit = 2,  // paired: the density searches and the temperature searches are
                   // 2M segments of one launch, one table staged per workgroup
  kPairInterp = 3, // paired as kPairJoint, then bilinear interpolation of the
                   // material's value grid at each pair
};

struct MultiArgs {
  const double* tables_a;
  const double* tables_b;
  const TableDesc* desc;     // [T] batched; [2M] paired (density, then temperature)
  const uint16_t* bins;
  const int64_t* tile_off;   // [S+1] first tile of each segment (table or material)
  const int64_t* query_off;  // [S+1] first target of each segment
  const struct WgStart* wg_start;  // [num_wg] where each workgroup starts
  const float* params;       // model pool (plans with learned tables)
  unsigned long long* fallbacks;  // learned window misses of the last search
  const double* xa;
  int32_t* oa;
  const double* xb;
  int32_t* ob;
  int64_t total_tiles;
  int tiles_per_wg;
  int strided;               // 1: a segment's workgroups take every stride-th tile
  int num_wg;                // workgroups with work (the grid may be padded)
  int xcd_groups;            // > 1: workgroup ids remapped per XCD (see below)
  int xcd_chunk;             // consecutive workgroups an XCD takes per turn
  int pair_base;             // index of the first temperature descriptor (paired)
  int64_t split;             // kPairSplit: temperature segments' targets start here in
                             // the segment offsets (targets of segment s >= pair_base
                             // are xb[query_off[s] - split ...])
  int lds_bins_a, lds_tab_b, lds_bins_b;  // byte offsets in LDS
  int lds_model_a, lds_model_b;           // learned models' LDS images
  int lead;          // bounded learned staging: bytes of every table region before a[0]
  // kPairInterp: value grids (material j's grid at value_off[j], row-major
  // over (density, temperature)), the interpolated output and whether the
  // index outputs oa / ob are written
  const double* values;
  const int64_t* value_off;
  double* of;
  int store_idx;
  int lds_grid;      // byte offset of the staged value grid in LDS
  int grid_cap;      // grids of at most this many values are staged in LDS
};

// What a workgroup keeps about the table it has staged.
struct Staged {
  HashParams hp;   // exponent hash (hp.ok) ...
  int learned;     // ... or learned model (its image staged in LDS) ...
  int n;           // ... or bisection ...
  int E;
  float u0, inv;
  int ballot;      // ... or the ballot scan
};

// Copies one table (+inf padded) and, for the exponent hash, its bin table
// into LDS with 16-byte loads (the pool's bin tables start 16-byte aligned;
// tables are 8-byte aligned, so they are copied in 8-byte words); for a
// learned table, its model's LDS image.
template <bool BOUNDED>
__device__ __forceinline__ Staged stage_desc(const TableDesc& d, const double* __restrict__ tables,
                                             const uint16_t* __restrict__ bins,
                                             const float* __restrict__ params, double* sa,
                                             uint16_t* C, float* model) {
  if (BOUNDED && d.algo == SS_ALGO_LEARNED)
    stage_table_bounded(sa, tables + d.tab_off, d.n, window_front(d.E), d.tail);
  else
    stage_table(sa, tables + d.tab_off, d.n);
  Staged st{{0, d.shift, d.kmin, d.kmaxc, d.nb, d.K}, d.algo == SS_ALGO_LEARNED, d.n, d.E,
            d.u0, d.inv, d.algo == SS_ALGO_BALLOT};
  if (d.algo == SS_ALGO_LEARNED) stage_image(model, params + d.p_off);
  if (d.algo == SS_ALGO_EXPHASH) {
    st.hp.ok = 1;
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4* src = reinterpret_cast<const u32x4*>(bins + d.bins_off);
    u32x4* dst = reinterpret_cast<u32x4*>(C);
    const int words = (d.nb + 1 + 7) / 8;  // the pool pads every table to 8 entries
    for (int w = threadIdx.x; w < words; w += blockDim.x) dst[w] = src[w];
  }
  return st;
}

template <int Q, int LEARN>
__device__ __forceinline__ void search_staged(const Staged& st, const double* sa,
                                              const uint16_t* C, const float* model,
                                              const ImageHead& hd, const double (&x)[Q],
                                              int (&r)[Q], uint64_t (&fell)[Q]) {
#pragma unroll
  for (int q = 0; q < Q; ++q) fell[q] = 0;
  if constexpr (LEARN) {
    if (st.learned) {  // uniform across the workgroup
      search_learned<Q, LEARN == 2 ? kWinBounded : kWinPadded>(sa, st.n, model, hd, st.E, st.u0,
                                                               st.inv, x, r, fell);
      return;
    }
  }
  if (st.hp.ok) search_exphash<Q>(sa, C, st.n, st.hp, x, r);
  else if (st.ballot) search_ballot<Q>(sa, st.n, x, r);  // every lane of the wave takes it
  else search_binary<Q>(sa, st.n, x, r);
}

struct TileRange {
  int64_t q0, q1;
};

// Adds a tile's learned window misses (the wave's masks) to the wave's
// count; lanes past the end of a short tile searched a stand-in and are not
// counted.  full is uniform, so a whole tile takes the short path.
template <int Q>
__device__ __forceinline__ void count_fallbacks(bool full, TileRange cur, int nt,
                                                const uint64_t (&fell)[Q], uint64_t& count) {
  if (full) {
#pragma unroll
    for (int q = 0; q < Q; ++q) count += __builtin_popcountll(fell[q]);
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q)
      count += __builtin_popcountll(
          fell[q] & __builtin_amdgcn_ballot_w64(cur.q0 + threadIdx.x + (int64_t)q * nt < cur.q1));
  }
}

template <int Q>
__device__ __forceinline__ void load_range(const double* __restrict__ x, TileRange r,
                                           double (&v)[Q]) {
  const int nt = blockDim.x;
  load_tile<Q>(x, r.q1, r.q0 + threadIdx.x, nt, r.q0 + (int64_t)nt * Q <= r.q1, v);
}

template <int Q>
__device__ __forceinline__ void store_tile_f64(double* __restrict__ out, int64_t m, int64_t base,
                                               int nt, bool full, const double (&v)[Q]) {
  if (full) {
#pragma unroll
    for (int q = 0; q < Q; ++q) __builtin_nontemporal_store(v[q], out + base + (int64_t)q * nt);
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t k = base + (int64_t)q * nt;
      if (k < m) out[k] = v[q];
    }
  }
}

// Searches one tile of targets against a staged table, in the strict
// convention or (CONV = 1) the paper's.
template <int Q, int LEARN, int CONV>
__device__ __forceinline__ void search_tile(const Staged& st, const double* sa, const uint16_t* C,
                                            const float* model, const ImageHead& hd,
                                            const double (&x)[Q], int (&r)[Q], uint64_t (&fell)[Q]) {
  if constexpr (CONV) {
    double xs[Q];
    convention_in<Q>(x, xs);
    search_staged<Q, LEARN>(st, sa, C, model, hd, xs, r, fell);
    convention_out<Q>(st.n, x, r);
  } else {
    search_staged<Q, LEARN>(st, sa, C, model, hd, x, r, fell);
  }
}

// Bilinear interpolation of one material's grid at Q pairs whose cells the
// two searches found (ra over the staged density axis sa, rb over the
// temperature axis sb): the strict index clamped to the edge cells, the
// fractional positions u and v (linear extension outside the axes), and
// the four corner values F read from the grid (LDS or global memory).  The
// value is formed as two interpolations along the density axis followed by
// one along the temperature axis, g0 = u f10 + (1 - u) f00, g1 = u f11 +
// (1 - u) f01, f = v g1 + (1 - v) g0, each a product and a fused
// multiply-add: the same four terms w_ij F_ij as the four-weight form
// (weights from the same rounded u, 1 - u, v, 1 - v), summed in another
// order, so within a few units of rounding of sum |w_ij F_ij| of it, in
// fewer float64 operations, and exact at the grid nodes (u and v in {0, 1};
// a target equal to a node lands in the cell below it with u = 1).
template <int Q>
__device__ __forceinline__ void interpolate(const double* sa, int na, const double* sb, int nb,
                                            const double* __restrict__ F, const double (&r)[Q],
                                            const double (&t)[Q], const int (&ra)[Q],
                                            const int (&rb)[Q], double (&f)[Q]) {
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = min(max(ra[q], 0), na - 2), k = min(max(rb[q], 0), nb - 2);
    const double u = (r[q] - sa[i]) / (sa[i + 1] - sa[i]);
    const double v = (t[q] - sb[k]) / (sb[k + 1] - sb[k]);
    const double* row0 = F + (int64_t)i * nb + k;
    const double* row1 = row0 + nb;
    const double f00 = row0[0], f01 = row0[1], f10 = row1[0], f11 = row1[1];
    const double u1 = 1.0 - u, v1 = 1.0 - v;
    const double g0 = fma(u, f10, u1 * f00), g1 = fma(u, f11, u1 * f01);
    f[q] = fma(v, g1, v1 * g0);
  }
}

// Where a material's value grid is read from: staged in LDS when it fits
// (each workgroup copies it once; the corner reads then cost LDS bandwidth
// instead of two L2 lines per pair), else from global memory.
struct Grid {
  const double* g;   // global grid
  const double* l;   // LDS copy, or null
};

__device__ __forceinline__ Grid stage_grid(const MultiArgs& a, int seg, int nr, int nt,
                                           double* lds_grid) {
  const double* g = a.values + a.value_off[seg];
  const int count = nr * nt;
  if (count > a.grid_cap) return {g, nullptr};
  for (int i = threadIdx.x; i < count; i += blockDim.x) lds_grid[i] = g[i];
  return {g, lds_grid};
}

template <int MODE, int Q, int LEARN, int CONV>
__global__ __launch_bounds__(1024) void multi_kernel(MultiArgs a) {
  constexpr bool INTERP = MODE == kPairInterp;
  constexpr bool PAIRED = MODE == kPairJoint || INTERP;
  constexpr bool SPLIT = MODE == kPairSplit;
  // LEARN = 2: learned tables are staged bounded (the -inf front before the
  // table, the +inf tail after it), so every table region starts a.lead
  // bytes in
  constexpr bool BOUNDED = LEARN == 2;
  const int lead = BOUNDED ? a.lead : 0;
  extern __shared__ __align__(16) unsigned char lds[];
  double* sa = reinterpret_cast<double*>(lds + lead);
  uint16_t* Ca = reinterpret_cast<uint16_t*>(lds + a.lds_bins_a);
  double* sb = reinterpret_cast<double*>(lds + a.lds_tab_b + lead);
  uint16_t* Cb = reinterpret_cast<uint16_t*>(lds + a.lds_bins_b);
  float* Ma = reinterpret_cast<float*>(lds + a.lds_model_a);
  float* Mb = reinterpret_cast<float*>(lds + a.lds_model_b);
  const int nt = blockDim.x;
  const int64_t per_tile = (int64_t)nt * Q;
  // Workgroup b runs on XCD b mod X (the dispatcher's round robin) as that
  // XCD's i-th workgroup, i = b / X.  With X = xcd_groups > 1 (the grid
  // padded to a multiple of X) the workgroup ranges are dealt to the XCDs in
  // chunks of C = xcd_chunk consecutive ranges: XCD x takes chunks x, x + X,
  // x + 2X, ..., so neighbouring ranges, which mostly share a table, run on
  // one XCD and find it in that XCD's L2, while every XCD still receives an
  // even mix of the whole plan (large and small tables alike).  The slots
  // past the last whole chunk keep dispatch order.  A bijection on
  // [0, grid): chunk slots map onto [0, X * full), the rest onto
  // [X * full, grid).
  int wid = blockIdx.x;
  if (a.xcd_groups > 1) {
    const int X = a.xcd_groups, C = a.xcd_chunk;
    const int x = blockIdx.x % X, i = blockIdx.x / X;
    const int full = gridDim.x / X / C * C;
    wid = i < full ? ((i / C) * X + x) * C + i % C : X * full + (i - full) * X + x;
  }
  if (wid >= a.num_wg) return;
  const WgStart ws = a.wg_start[wid];
  if (ws.count <= 0) return;
  // A workgroup works inside one segment: tiles first, first + stride, ...
  // (count of them) of the segment, whose targets are [q0, q1) of its own
  // target array.  Tile k of a segment is the part of the aligned block
  // q0 / per_tile + k that lies in [q0, q1).  stride is 1 (a contiguous
  // range of tiles) or the segment's workgroup count (its workgroups sweep
  // it side by side, see wg_order).
  const bool part = SPLIT && ws.seg >= a.pair_base;
  const double* __restrict__ xa = part ? a.xb : a.xa;
  int32_t* __restrict__ oa_ = part ? a.ob : a.oa;
  const int64_t q0 = ws.seg_q0, q1 = ws.seg_q1;
  const int64_t b0 = q0 / per_tile + ws.first;
  const int64_t stride =
      a.strided ? (ws.seg_tiles + a.tiles_per_wg - 1) / a.tiles_per_wg : 1;
  auto tile = [&](int k) -> TileRange {
    const int64_t b = b0 + (int64_t)k * stride;
    return {max(q0, b * per_tile), min((b + 1) * per_tile, q1)};
  };
  const int count = ws.count;
  // Tiles k, k+1 and k+2 are in flight at once: the targets of the two
  // tiles after the one being searched are already being loaded.
  TileRange cur = tile(0), nx1{0, 0};
  double ca[Q], cb[Q], ca1[Q], cb1[Q];
  load_range<Q>(xa, cur, ca);
  if constexpr (PAIRED) load_range<Q>(a.xb, cur, cb);
  if (count > 1) {
    nx1 = tile(1);
    load_range<Q>(xa, nx1, ca1);
    if constexpr (PAIRED) load_range<Q>(a.xb, nx1, cb1);
  }

  Staged sta, stb{};
  Grid grid{nullptr, nullptr};
  double* lds_grid = reinterpret_cast<double*>(lds + a.lds_grid);
  sta = stage_desc<BOUNDED>(a.desc[ws.seg], part ? a.tables_b : a.tables_a, a.bins, a.params, sa,
                           Ca, Ma);
  if constexpr (PAIRED)
    stb = stage_desc<BOUNDED>(a.desc[a.pair_base + ws.seg], a.tables_b, a.bins, a.params, sb, Cb,
                              Mb);
  if constexpr (INTERP) grid = stage_grid(a, ws.seg, sta.n, stb.n, lds_grid);
#if SS_DEVICE_CHECKS
  // the host's LDS layout holds what was staged (learned images are
  // checked by their lookups)
  SS_ASSERT(lead + (sta.n + (BOUNDED && sta.learned ? a.desc[ws.seg].tail : SS_PAD)) * 8 <=
            a.lds_bins_a);
  SS_ASSERT(!(BOUNDED && sta.learned) || window_front(sta.E) * 8 <= lead);
  SS_ASSERT(!sta.hp.ok || a.lds_bins_a + (sta.hp.nb + 1) * 2 <= a.lds_tab_b);
  if constexpr (PAIRED) {
    SS_ASSERT(a.lds_tab_b + lead +
                  (stb.n + (BOUNDED && stb.learned ? a.desc[a.pair_base + ws.seg].tail : SS_PAD)) *
                      8 <=
              a.lds_bins_b);
    SS_ASSERT(!(BOUNDED && stb.learned) || window_front(stb.E) * 8 <= lead);
    SS_ASSERT(!stb.hp.ok ||
              a.lds_bins_b + (stb.hp.nb + 1) * 2 <= (INTERP ? a.lds_grid : a.lds_model_a));
  }
  if constexpr (INTERP) SS_ASSERT(!grid.l || sta.n * stb.n <= a.grid_cap);
#endif
  __syncthreads();
  // headers of staged learned models (unused for other tables)
  ImageHead oa{}, ob{};
  if constexpr (LEARN) {
    oa = image_head(Ma);
    if constexpr (PAIRED) ob = image_head(Mb);
  }
  uint64_t fallbacks = 0;  // the wave's learned window misses (uniform)
  for (int k = 0; k < count; ++k) {
    double ca2[Q], cb2[Q];
    TileRange nx2{0, 0};
    if (k + 2 < count) {
      nx2 = tile(k + 2);
      load_range<Q>(xa, nx2, ca2);
      if constexpr (PAIRED) load_range<Q>(a.xb, nx2, cb2);
    }
    const bool full = cur.q0 + per_tile == cur.q1;
    SS_ASSERT(cur.q0 >= q0 && cur.q1 <= q1 && cur.q0 < cur.q1 && cur.q1 - cur.q0 <= per_tile);
    int r[Q];
    uint64_t fell[Q];
    search_tile<Q, LEARN, CONV>(sta, sa, Ca, Ma, oa, ca, r, fell);
    if constexpr (!INTERP)
      store_tile<Q>(oa_, cur.q1, cur.q0 + threadIdx.x, nt, full, r);
    if constexpr (LEARN) count_fallbacks<Q>(full, cur, nt, fell, fallbacks);
    if constexpr (INTERP) {
      int rt[Q];
      search_tile<Q, LEARN, CONV>(stb, sb, Cb, Mb, ob, cb, rt, fell);
      double f[Q];
      if (grid.l)  // uniform: the grid of the workgroup's material
        interpolate<Q>(sa, sta.n, sb, stb.n, grid.l, ca, cb, r, rt, f);
      else
        interpolate<Q>(sa, sta.n, sb, stb.n, grid.g, ca, cb, r, rt, f);
      store_tile_f64<Q>(a.of, cur.q1, cur.q0 + threadIdx.x, nt, full, f);
      if (a.store_idx) {
        store_tile<Q>(a.oa, cur.q1, cur.q0 + threadIdx.x, nt, full, r);
        store_tile<Q>(a.ob, cur.q1, cur.q0 + threadIdx.x, nt, full, rt);
      }
    } else if constexpr (PAIRED) {
      search_tile<Q, LEARN, CONV>(stb, sb, Cb, Mb, ob, cb, r, fell);
      store_tile<Q>(a.ob, cur.q1, cur.q0 + threadIdx.x, nt, full, r);
      if constexpr (LEARN) count_fallbacks<Q>(full, cur, nt, fell, fallbacks);
    }
    cur = nx1;
    nx1 = nx2;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      ca[q] = ca1[q];
      ca1[q] = ca2[q];
      if constexpr (PAIRED) {
        cb[q] = cb1[q];
        cb1[q] = cb2[q];
      }
    }
  }
  if constexpr (LEARN) {
    if ((threadIdx.x & 63) == 0 && fallbacks) atomicAdd(a.fallbacks, (unsigned long long)fallbacks);
  }
}

__global__ void plan_clear_kernel(unsigned long long* c) { *c = 0ull; }

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

// One table's searches as a sample for the ballot scan's cost: the table
// (device), its target array and the targets [q0, q1) searched in it.
struct BracketJob {
  const double* tab;
  const double* x;
  int64_t q0, q1;
  int n;
  int pad_;
};

// The ballot scan's work per wave on sample targets: for each job (one
// workgroup), `samples` wave footprints spread evenly over its tiles.  The
// footprint of wave slot w of tile b is what one wave of the plan kernel
// searches together: targets b * per_tile + w * 64 + lane + j * nt, j < Q,
// inside [q0, q1).  Its bracket is #{a < max} - #{a < min} over those
// targets (NaN ignored), the entries each lane then scans.  Writes the mean
// bracket per job, -1 for a job without targets.
__global__ __launch_bounds__(256) void plan_bracket_kernel(const BracketJob* jobs, int nt, int Q,
                                                           int64_t per_tile, int samples,
                                                           double* mean_out) {
  __shared__ double sum;
  __shared__ int count;
  const BracketJob jb = jobs[blockIdx.x];
  if (threadIdx.x == 0) {
    sum = 0;
    count = 0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
  const int slots = max(nt / 64, 1);
  if (jb.q1 > jb.q0) {
    const int64_t b0 = jb.q0 / per_tile, b1 = (jb.q1 - 1) / per_tile;
    const int64_t tiles = b1 - b0 + 1;
    for (int f = wave; f < samples; f += waves) {
      const int64_t b = b0 + (int64_t)f * tiles / samples;
      const int64_t base = b * per_tile + (int64_t)(f % slots) * 64 + lane;
      double lo = __builtin_nan(""), hi = __builtin_nan("");
      for (int j = 0; j < Q; ++j) {
        const int64_t k = base + (int64_t)j * nt;
        if (k >= jb.q0 && k < jb.q1) {
          const double v = jb.x[k];
          lo = fmin(lo, v);
          hi = fmax(hi, v);
        }
      }
      const double wmin = wave_min(lo), wmax = wave_max(hi);
      if (lane == 0 && wmin == wmin) {  // some target of the footprint is a number
        int c[2];
        const double v[2] = {wmin, wmax};
        for (int e = 0; e < 2; ++e) {  // #{a < v} by bisection over the table
          int first = 0, len = jb.n;
          while (len > 0) {
            const int half = len >> 1;
            if (jb.tab[first + half] < v[e]) {
              first += half + 1;
              len -= half + 1;
            } else {
              len = half;
            }
          }
          c[e] = first;
        }
        atomicAdd(&sum, (double)(c[1] - c[0]));
        atomicAdd(&count, 1);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) mean_out[blockIdx.x] = count > 0 ? sum / count : -1.0;
}

}  // namespace ss

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------

struct ss_plan {
  int paired = 0;
  int mode = 0;                  // ss::PlanMode
  int64_t split = 0;             // kPairSplit: offset of the temperature segments' targets
  bool convention = false;       // the paper's convention (SS_OPT_CONVENTION at creation)
  int64_t* d_value_off = nullptr;  // kPairInterp: first value of each material's grid
  int grid_cap = 0;                // kPairInterp: largest grid (values) staged in LDS
  int32_t T = 0;                 // descriptors (batched: tables; paired: 2 * materials)
  int32_t M = 0;                 // materials (paired)
  int32_t S = 0;                 // segments: tables (batched), materials (joint paired) or
                                 // 2 * materials (split paired)
  int64_t total_queries = 0;
  int device = -1;
  std::vector<int64_t> query_off;
  std::vector<ss::TableDesc> desc;
  std::vector<ss::TunedTable> tuned;
  ss::TableDesc* d_desc = nullptr;
  uint16_t* d_bins = nullptr;
  int64_t* d_tile_off = nullptr;
  int64_t* d_query_off = nullptr;
  ss::WgStart* d_wg_start = nullptr;
  int* d_k = nullptr;
  float* d_pool = nullptr;                 // learned models, compiled (kImageFloats each)
  size_t image_bytes = 0;                  // largest compiled model in use (16-byte multiple)
  unsigned long long* d_fallbacks = nullptr;
  int learned_tables = 0;
  int64_t total_tiles = 0;
  int tiles_per_wg = 0;
  bool strided = false;
  std::vector<std::vector<float>> weights;  // per descriptor: a learned table's parameters
  std::vector<double> brackets;             // per descriptor: mean ballot bracket on the
                                            // sample targets (-1: not sampled)
  int preset_tiles = 0;                     // from a saved plan: tiles per workgroup,
  int preset_order = -1;                    // tile order (SS_OPT_PLAN_ORDER value) and
  int preset_conv = -1;                     // convention, else -1 / 0 (options decide)
  int num_wg = 0, xcd_groups = 1, xcd_chunk = 1;
  int grid = 0, block = 0, q = 0;
  int learn = 0;  // plan kernel's learned form: 0 none, 1 clamped window, 2 bounded staging
  int lead = 0;   // learn = 2: bytes of every table region before a[0]
  size_t lds = 0;
  int max_k = 0;
  ss::MultiArgs args{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t search_node = nullptr;
  hipGraphNode_t clear_node = nullptr;
  int64_t graph_uses = 0;
  const void* kernel = nullptr;

  ~ss_plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (void* ptr : {(void*)d_desc, (void*)d_bins, (void*)d_tile_off, (void*)d_query_off,
                      (void*)d_wg_start, (void*)d_k, (void*)d_pool, (void*)d_fallbacks,
                      (void*)d_value_off})
      if (ptr) (void)hipFree(ptr);
  }
};

namespace ss {

namespace {

constexpr int kPlanBlock = 512;
constexpr int kPlanQ = 8;
constexpr int kPairQ = 4;
// Batched and split plans whose learned tables carry at least this share of
// the targets take 4 targets per lane (the learned search at 8 holds 121
// VGPRs, 4 waves per SIMD; at 4, 65 and 7).  Measured: every table learned,
// the 512-table batch 374-376 Gq/s at 8 against 423-425 at 4, the paired
// workload 353 against 404-405; one learned table among 512 (the others
// exponent hash), 506 at 8 against 493 at 4.  The per-target costs those
// imply break even at a learned share of about 15%.
constexpr double kLearnedQ4Share = 0.15;
// Set by the tuner's calibration: learned plans take kPlanQ whatever their
// share (the cost a learned table has in a plan of few of them).
thread_local bool t_learned_q_fixed = false;
constexpr int kDefaultPlanLearnedSteps = 500;
constexpr int kXcds = 8;                  // accelerator complex dies of an MI355X
// Workgroup ranges per XCD turn for plans with long segments.  Measured on
// MI355X (strided tile order, 5 tiles per workgroup, mean of three runs):
// the 512-table batch (segments of ~350 tiles) 1.468 ms in dispatch order
// against 1.447 ms in chunks of 8; the 4096-material paired workload
// (segments of ~60 tiles) 3.984 against 4.003 ms.  Plans whose segments
// average under 64 tiles therefore keep dispatch order.  Earlier, with
// contiguous tile ranges: chunks of 1 / 8 / 64 / one contiguous part per
// XCD gave 5.97 / 6.03 / 5.90 / 5.89 TB/s on the batch; a contiguous part
// per XCD gives the dies unequal work (the paired plan's density segments,
// with the larger tables, come first).
constexpr int kXcdChunk = 8;
constexpr int kShortSegmentTiles = 64;  // in tiles of 4096 targets
// LDS a plan's workgroup may use (tables + bin tables): three 512-thread
// workgroups per CU fit in 160 KB.
constexpr size_t kPlanLdsBudget = 48 * 1024;
// Interpolation plans stage a material's value grid in LDS when it has at
// most this many float64 values (120 KB: with the axes, one workgroup per
// CU).  Measured on 1024 materials (grids of 1000 to 14850 values, 1e9
// pairs): grids up to 9216 values staged (72 KB, two 512-thread workgroups
// per CU; the other 15% of the pairs read their corners from L2) 5.51-5.66
// ms; up to 5632 values (three workgroups per CU) 6.84-7.07 ms; every grid
// staged, one 1024-thread workgroup per CU, 5.08-5.11 ms.
constexpr int64_t kInterpGridLdsValues = 15360;
// A staged grid above this size leaves its CU to one workgroup.
constexpr size_t kInterpGridShared = 72 * 1024;

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
  d->p_off = 0;
  d->E = 0;
  d->u0 = d->inv = 0.0f;
  d->tail = 0;
  d->pad_ = 0;
  if (tt.algo == SS_ALGO_EXPHASH) {
    d->bins_off = *pool_len;
    *pool_len += tt.nb + 1;
    *pool_len = (*pool_len + 7) / 8 * 8;  // 16-byte aligned starts
  }
}

size_t align16(size_t v) { return (v + 15) / 16 * 16; }

// Learned models of plans built now (SS_OPT_PLAN_LEARNED, overridden by a
// forced plan kernel).
enum LearnedMode { kLearnedTuner = 0, kLearnedAll = 1, kLearnedNone = 2 };
// Tile order of a segment's workgroups (SS_OPT_PLAN_ORDER).
enum TileOrder { kOrderDefault = 0, kOrderContiguous = 1, kOrderStrided = 2 };

// A saved plan's choices (ss_plan_save / ss_*_plan_load): per descriptor its
// size, kernel, bin bits and, for a learned table, the model's parameters.
struct PlanPreset {
  int mode = 0;
  int descriptors = 0, materials = 0;
  int tiles_per_wg = 0, strided = 1, convention = 0;
  std::vector<int> n, algo, bits;
  std::vector<std::vector<float>> weights;
};

// Block size and targets per lane of a plan of this form.  An
// interpolation plan whose staged grids leave each CU to one workgroup
// takes the largest workgroup (1024 threads: 5.61 ms against 5.99 at 512 on
// the 1024-material workload, every grid staged).
int plan_block(int mode = kBatched, size_t grid_bytes = 0) {
  if (option(SS_OPT_BLOCK_SIZE) > 0) return (int)option(SS_OPT_BLOCK_SIZE);
  return mode == kPairInterp && grid_bytes > kInterpGridShared ? 1024 : kPlanBlock;
}
int plan_q(int mode, double learned_share = 0.0) {
  if (mode == kPairJoint || mode == kPairInterp) return kPairQ;
  return learned_share >= kLearnedQ4Share ? kPairQ : kPlanQ;
}

// Wave footprints sampled per table for the ballot scan's bracket.
constexpr int kBracketSamples = 32;

// Mean ballot bracket of every job on its sample targets, with the tile
// shape of a plan of this form (-1 for a job without targets).
// SYNCHRONOUS on the current stream.
int sample_brackets(const std::vector<BracketJob>& jobs, int mode, std::vector<double>* mean) {
  mean->assign(jobs.size(), -1.0);
  if (jobs.empty()) return SS_OK;
  hipStream_t st = current_stream();
  void* dj = nullptr;
  void* dm = nullptr;
  hipError_t e = hipMalloc(&dj, sizeof(BracketJob) * jobs.size());
  if (e == hipSuccess) e = hipMalloc(&dm, sizeof(double) * jobs.size());
  if (e == hipSuccess)
    e = hipMemcpyAsync(dj, jobs.data(), sizeof(BracketJob) * jobs.size(), hipMemcpyHostToDevice,
                       st);
  if (e == hipSuccess) {
    const int nt = plan_block(), Q = plan_q(mode);
    hipLaunchKernelGGL(plan_bracket_kernel, dim3((unsigned)jobs.size()), dim3(256), 0, st,
                       static_cast<const BracketJob*>(dj), nt, Q, (int64_t)nt * Q,
                       kBracketSamples, static_cast<double*>(dm));
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(mean->data(), dm, sizeof(double) * jobs.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (dj) (void)hipFree(dj);
  if (dm) (void)hipFree(dm);
  return e == hipSuccess ? SS_OK : hip_fail(e, "ballot bracket sampling");
}

// Turns a tuned choice into the ballot scan, at its modelled cost for the
// sampled bracket (unknown, -1: a full scan of the table).
void make_ballot(const TunerModel& model, double bracket, TunedTable* t) {
  t->algo = SS_ALGO_BALLOT;
  t->bits = -1;
  t->kmin = t->kmaxc = t->nb = t->K = 0;
  t->est_ns = ballot_cost_ns(model, bracket >= 0 ? bracket : (double)t->n, t->n);
}

// The per-table choice with sampled targets: SS_OPT_PLAN_ALGO forcing the
// ballot scan takes it everywhere; the tuner weighs it against the
// bisection only, where its modelled cost for the sampled bracket is lower.
// Against the exponent hash it never won in a plan: measured on MI355X with
// 256 tables of 16 / 48 / 128 / 400 entries and 2.8e6 sorted targets each
// (brackets of 0.02 to 0.5 entries), the hash took 1.370 / 1.370 / 1.383 /
// 1.384 ms, the ballot scan 1.419 / 1.421 / 1.413 / 1.389 and the bisection
// 1.404 / 1.377 / 1.375 / 1.435.  Both searches are far below the memory
// time there; the ballot scan's two wave-wide reductions per tile add
// latency that the hash does not have.  With i.i.d. targets the ballot scan
// took 1.55 / 2.72 / 6.17 / 18.2 ms.
void consider_ballot(const TunerModel& model, double bracket, int force, TunedTable* t) {
  if (t->n < 1) return;
  if (force == SS_ALGO_BALLOT) {
    make_ballot(model, bracket, t);
    return;
  }
  if (force != SS_ALGO_AUTO || !(bracket >= 0) || t->algo != SS_ALGO_BINARY) return;
  if (ballot_cost_ns(model, bracket, t->n) < t->est_ns * (1.0 - 1e-9)) make_ballot(model, bracket, t);
}

// The saved choice for one table, re-derived from the table as it is now:
// the exponent hash at the saved bits if it still applies within the LDS
// budget (its bin parameters and longest bin recomputed from the entries),
// else the tuner's choice; a learned table keeps its plain fallback choice
// here and gets its model afterwards.
TunedTable preset_table(const TunerModel& model, const double* a, int n, size_t budget,
                        int algo, int bits) {
  if (algo == SS_ALGO_BINARY) return tune_table(model, a, n, budget, SS_ALGO_BINARY);
  if (algo == SS_ALGO_BALLOT && n >= 1) {
    TunedTable t = tune_table(model, a, n, budget, SS_ALGO_BINARY);
    make_ballot(model, -1.0, &t);
    return t;
  }
  if (algo == SS_ALGO_EXPHASH && bits >= 0 && bits <= SS_MAX_BITS && n >= 1 && n <= 65535) {
    TunedTable t = tune_table(model, a, n, budget, SS_ALGO_EXPHASH);
    if (t.algo == SS_ALGO_EXPHASH && t.bits == bits) return t;
    uint64_t u0, u1;
    std::memcpy(&u0, &a[0], 8);
    std::memcpy(&u1, &a[n - 1], 8);
    const int h0 = (int)(int32_t)(uint32_t)(u0 >> 32), h1 = (int)(int32_t)(uint32_t)(u1 >> 32);
    const int sh = SS_MAX_BITS - bits;
    const int64_t nb = (int64_t)(h1 >> sh) - (h0 >> sh) + 1;
    if (h0 >= 0 && h1 >= h0 && nb <= 65535 && (size_t)(nb + 1) * 2 + 16 <= budget) {
      t.algo = SS_ALGO_EXPHASH;
      t.bits = bits;
      t.kmin = h0 >> sh;
      t.kmaxc = h1 >> sh;
      t.nb = (int)nb;
      t.K = host_longest_bin(a, n, bits);
      t.est_ns = t.K <= SS_SCAN_MAX ? model.hash_base_ns + model.hash_per_k_ns * t.K
                                    : model.hash_base_ns + model.bin_per_step_ns * 17;
      return t;
    }
  }
  return tune_table(model, a, n, budget);
}
int learned_mode() {
  if (option(SS_OPT_PLAN_ALGO) != SS_ALGO_AUTO) return kLearnedNone;
  return (int)option(SS_OPT_PLAN_LEARNED);
}

int fail_delete(ss_plan* p, const char* msg, int code = SS_ERR_INVALID_ARG) {
  delete p;
  return msg ? fail(code, msg) : code;
}

// Learned models for a plan's tables, trained on the device in one launch.
// kLearnedAll: every eligible table gets one.  kLearnedTuner: only tables
// whose modelled learned cost at the best possible bound (E = 1, a one-step
// cell lookup) undercuts their tuned plain kernel are trained, and a model
// is kept where its cost with the measured E and lookup still does.
// host_a / host_b are host copies of the two tables arrays.
int apply_learned(ss_plan* p, const double* tables_a, const double* tables_b,
                  const std::vector<double>& host_a, const std::vector<double>& host_b,
                  int mode, const PlanPreset* preset = nullptr) {
  const TunerModel model = tuner_model();
  constexpr int kBestLookup = 3;  // cell read, one boundary, piece read
  std::vector<LearnedSlot> slots;
  std::vector<int> slot_desc;
  std::vector<float> given;  // a saved plan's parameters, one model per slot
  for (int t = 0; t < p->T; ++t) {
    TableDesc& d = p->desc[t];
    const int which = (p->paired && t >= p->M) ? 1 : 0;
    const double* h = (which ? host_b.data() : host_a.data()) + d.tab_off;
    if (!learned_eligible(h, d.n)) continue;
    if (preset) {
      if (preset->weights[t].empty()) continue;
      given.insert(given.end(), preset->weights[t].begin(), preset->weights[t].end());
    } else if (mode == kLearnedTuner &&
               !(learned_cost_ns(model, 1, kBestLookup) < p->tuned[t].est_ns)) {
      continue;
    }
    LearnedSlot sl{};
    sl.tab_off = d.tab_off;
    sl.i_off = (int64_t)slots.size() * kImageFloats;
    sl.n = d.n;
    sl.which = which;
    slots.push_back(sl);
    slot_desc.push_back(t);
  }
  if (slots.empty()) return SS_OK;
  SS_TRY_HIP(hipMalloc(&p->d_pool, sizeof(float) * kImageFloats * slots.size()));
  SS_TRY_HIP(hipMalloc(&p->d_fallbacks, sizeof(unsigned long long)));
  SS_TRY_HIP(hipMemset(p->d_fallbacks, 0, sizeof(unsigned long long)));
  int steps = (int)option(SS_OPT_LEARNED_STEPS);
  if (steps <= 0) steps = kDefaultPlanLearnedSteps;
  std::vector<float> trained;
  int rc = learned_train_slots(tables_a, tables_b, slots, p->d_pool, steps, 0.01f, 1,
                               preset ? given.data() : nullptr, &trained);
  if (rc != SS_OK) return rc;
  // every image's (boundaries, pieces, cells, fullest cell) header, as the
  // bound kernel staged it: LDS is reserved for the largest kept image
  p->image_bytes = 0;
  int kept = 0;
  for (size_t i = 0; i < slots.size(); ++i) {
    const int* hd = slots[i].head;
    if (!image_header_valid(hd))
      return fail(SS_ERR_UNSUPPORTED,
                  "compiled model " + std::to_string(i) + " (table " +
                      std::to_string(slot_desc[i]) + ", n " + std::to_string(slots[i].n) +
                      ") is malformed: boundary slots " + std::to_string(hd[0]) + ", pieces " +
                      std::to_string(hd[1]) + ", cells " + std::to_string(hd[2]) +
                      ", fullest cell " + std::to_string(hd[3]));
    const int t = slot_desc[i];
    int lookup = 2 + hd[3];  // cell read, scan of the fullest cell, piece read
    if (hd[2] == 0) {        // no cell table: bisection over the boundary slots
      lookup = 2;
      for (int v = 1; v < hd[0]; v <<= 1) ++lookup;
    }
    p->tuned[t].learned_ns = learned_cost_ns(model, slots[i].E, lookup);
    if (!preset && mode == kLearnedTuner && !(p->tuned[t].learned_ns < p->tuned[t].est_ns)) {
      slot_desc[i] = -1;  // trained, but its plain kernel is cheaper
      continue;
    }
    ++kept;
    p->image_bytes =
        std::max(p->image_bytes, (size_t)image_used_floats(hd[0], hd[1], hd[2]) * 4);
  }
  for (size_t i = 0; i < slots.size(); ++i) {
    const int t = slot_desc[i];
    if (t < 0) continue;
    TableDesc& d = p->desc[t];
    d.algo = SS_ALGO_LEARNED;
    d.bins_off = 0;
    d.nb = d.K = 0;
    d.p_off = slots[i].i_off;
    d.E = slots[i].E;
    d.u0 = slots[i].u0;
    d.inv = slots[i].inv;
    p->tuned[t].algo = SS_ALGO_LEARNED;
    p->tuned[t].bits = -1;
    p->weights[t].assign(trained.begin() + (int64_t)i * SS_MLP_PARAMS,
                         trained.begin() + (int64_t)(i + 1) * SS_MLP_PARAMS);
  }
  p->learned_tables = kept;
  return SS_OK;
}

// Attaches given learned handles to a batched plan (models[t], or null for
// the tuner's choice): each handle must have been built on table t's own
// memory.  Its compiled model is copied into the plan's pool, so the plan
// does not depend on the handle afterwards.
int attach_learned(ss_plan* p, const double* tables, const int64_t* table_off,
                   ss_learned* const* models) {
  int dev = 0;
  SS_TRY_HIP(hipGetDevice(&dev));
  std::vector<int> with;
  std::vector<LearnedExport> ex;
  for (int t = 0; t < p->T; ++t) {
    if (!models[t]) continue;
    LearnedExport e{};
    const int rc = learned_export(models[t], &e);
    if (rc != SS_OK) return rc;
    if (e.table != tables + table_off[t] || e.n != table_off[t + 1] - table_off[t])
      return fail(SS_ERR_INVALID_ARG,
                  "model " + std::to_string(t) + " was not built on table " + std::to_string(t));
    if (e.device != dev)
      return fail(SS_ERR_INVALID_ARG, "model " + std::to_string(t) + " is on another device");
    with.push_back(t);
    ex.push_back(e);
  }
  if (ex.empty()) return SS_OK;
  SS_TRY_HIP(hipMalloc(&p->d_pool, sizeof(float) * kImageFloats * ex.size()));
  SS_TRY_HIP(hipMalloc(&p->d_fallbacks, sizeof(unsigned long long)));
  SS_TRY_HIP(hipMemset(p->d_fallbacks, 0, sizeof(unsigned long long)));
  p->image_bytes = 0;
  for (size_t i = 0; i < ex.size(); ++i) {
    SS_TRY_HIP(hipMemcpy(p->d_pool + i * kImageFloats, ex[i].image,
                         sizeof(float) * ex[i].image_floats, hipMemcpyDeviceToDevice));
    p->image_bytes = std::max(p->image_bytes, (size_t)ex[i].image_floats * 4);
    const int t = with[i];
    if (ex[i].params) p->weights[t].assign(ex[i].params, ex[i].params + SS_MLP_PARAMS);
    TableDesc& d = p->desc[t];
    d.algo = SS_ALGO_LEARNED;
    d.bins_off = 0;
    d.nb = d.K = 0;
    d.p_off = (int64_t)i * kImageFloats;
    d.E = ex[i].E;
    d.u0 = ex[i].u0;
    d.inv = ex[i].inv;
    p->tuned[t].algo = SS_ALGO_LEARNED;
    p->tuned[t].bits = -1;
  }
  p->learned_tables = (int)ex.size();
  return SS_OK;
}

template <int MODE, int Q, int LEARN>
const void* plan_kernel_conv(bool conv) {
  return conv ? reinterpret_cast<const void*>(&multi_kernel<MODE, Q, LEARN, 1>)
              : reinterpret_cast<const void*>(&multi_kernel<MODE, Q, LEARN, 0>);
}

// learn: 0 no learned tables; 1 learned, clamped window; 2 learned, bounded staging
template <int MODE, int Q>
const void* plan_kernel_learn(int learn, bool conv) {
  return learn == 2   ? plan_kernel_conv<MODE, Q, 2>(conv)
         : learn == 1 ? plan_kernel_conv<MODE, Q, 1>(conv)
                      : plan_kernel_conv<MODE, Q, 0>(conv);
}

// Batched and split plans: kPlanQ targets per lane, or kPairQ for plans of
// mostly learned targets (which always have learned tables).
template <int MODE>
const void* plan_kernel_q(int q, int learn, bool conv) {
  if (q == kPairQ && learn > 0)
    return learn == 2 ? plan_kernel_conv<MODE, kPairQ, 2>(conv)
                      : plan_kernel_conv<MODE, kPairQ, 1>(conv);
  return plan_kernel_learn<MODE, kPlanQ>(learn, conv);
}

const void* plan_kernel(int mode, int q, int learn, bool conv) {
  switch (mode) {
    case kPairInterp:
      return reinterpret_cast<const void*>(&multi_kernel<kPairInterp, kPairQ, 0, 0>);
    case kPairJoint: return plan_kernel_learn<kPairJoint, kPairQ>(learn, conv);
    case kPairSplit: return plan_kernel_q<kPairSplit>(q, learn, conv);
    default: return plan_kernel_q<kBatched>(q, learn, conv);
  }
}

hipKernelNodeParams search_node_params(ss_plan* p, void** kargs) {
  hipKernelNodeParams kp{};
  kp.func = const_cast<void*>(p->kernel);
  kp.gridDim = dim3(p->grid);
  kp.blockDim = dim3(p->block);
  kp.sharedMemBytes = (unsigned)p->lds;
  kp.kernelParams = kargs;
  kp.extra = nullptr;
  return kp;
}

int finish_plan(ss_plan* p, const double* tables_a, const double* tables_b, int64_t pool_len,
                size_t lds_tab_a, size_t lds_bins_a, size_t lds_tab_b, size_t lds_bins_b) {
  hipStream_t st = current_stream();
  const int T = p->T;
  // Learned tables are staged bounded (window_front -inf entries before,
  // window_tail +inf entries after) when every region still fits the
  // staging budget that way; the window's checks and steps then need no
  // clamps.  Every table region then starts `lead` bytes in, the largest
  // front of the plan's learned tables.  Otherwise the clamped form.
  p->learn = p->learned_tables > 0 ? 1 : 0;
  p->lead = 0;
  if (p->learned_tables > 0) {
    const bool two = p->mode == kPairJoint || p->mode == kPairInterp;
    size_t lead = 16;
    for (int t = 0; t < T; ++t)
      if (p->desc[t].algo == SS_ALGO_LEARNED)
        lead = std::max(lead, (size_t)window_lead(p->desc[t].E));
    size_t need_a = lead, need_b = two ? lead : 0;
    for (int t = 0; t < T; ++t) {
      const TableDesc& d = p->desc[t];
      const int rows = d.n + (d.algo == SS_ALGO_LEARNED ? window_tail(d.E) : SS_PAD);
      const size_t need = lead + align16((size_t)rows * 8);
      if (two && t >= p->M) need_b = std::max(need_b, need);
      else need_a = std::max(need_a, need);
    }
    if (!two) need_a = std::max(need_a, lds_tab_a);
    if (need_a + lds_bins_a + need_b + lds_bins_b <= kPlanLdsBudget + 16 * 1024) {
      p->learn = 2;
      p->lead = (int)lead;
      lds_tab_a = std::max(lds_tab_a, need_a);
      if (two) lds_tab_b = std::max(lds_tab_b, need_b);
      for (int t = 0; t < T; ++t)
        if (p->desc[t].algo == SS_ALGO_LEARNED)
          p->desc[t].tail = window_tail(p->desc[t].E);
    }
  }
  SS_TRY_HIP(hipMalloc(&p->d_desc, sizeof(TableDesc) * T));
  SS_TRY_HIP(hipMalloc(&p->d_bins, sizeof(uint16_t) * std::max<int64_t>(pool_len, 8)));
  SS_TRY_HIP(hipMalloc(&p->d_k, sizeof(int) * T));
  SS_TRY_HIP(hipMemcpyAsync(p->d_desc, p->desc.data(), sizeof(TableDesc) * T,
                            hipMemcpyHostToDevice, st));
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

  p->block = plan_block(p->mode, p->mode == kPairInterp ? (size_t)p->grid_cap * 8 : 0);
  // targets per lane: the form's, or fewer for a plan of mostly learned
  // targets (segment s searches descriptor s in the batched and split forms)
  double learned_share = 0.0;
  if (p->learned_tables > 0 && !t_learned_q_fixed &&
      (p->mode == kBatched || p->mode == kPairSplit)) {
    int64_t lq = 0;
    for (int s = 0; s < p->S; ++s)
      if (p->desc[s].algo == SS_ALGO_LEARNED) lq += p->query_off[s + 1] - p->query_off[s];
    const int64_t all = p->query_off[p->S] - p->query_off[0];
    learned_share = all > 0 ? (double)lq / (double)all : 0.0;
  }
  p->q = plan_q(p->mode, learned_share);
  const int64_t per_tile = (int64_t)p->block * p->q;
  // tiles of every segment, numbered back to back; a segment's positions are
  // taken relative to the start of its own target array
  const int S = p->S;
  auto seg_base = [&](int s) -> int64_t {
    return p->mode == kPairSplit && s >= p->M ? p->split : 0;
  };
  std::vector<int64_t> tile_off(S + 1, 0);
  for (int s = 0; s < S; ++s) {
    const int64_t q0 = p->query_off[s] - seg_base(s), q1 = p->query_off[s + 1] - seg_base(s);
    tile_off[s + 1] = tile_off[s] + (q1 > q0 ? (q1 - 1) / per_tile - q0 / per_tile + 1 : 0);
  }
  p->total_tiles = tile_off[S];

  p->lds = lds_tab_a + lds_bins_a + lds_tab_b + lds_bins_b;
  const bool learned = p->learned_tables > 0;
  if (p->mode == kPairInterp && p->grid_cap > 0) {
    p->args.lds_grid = (int)p->lds;
    p->args.grid_cap = p->grid_cap;
    p->lds += (size_t)p->grid_cap * sizeof(double);
  }
  int model_a = (int)p->lds, model_b = (int)p->lds;
  if (learned) {  // one model image per staged table
    p->lds += p->image_bytes;
    if (p->mode == kPairJoint || p->mode == kPairInterp) {
      model_b = (int)p->lds;
      p->lds += p->image_bytes;
    }
  }
  // interpolation locates cells with the strict index (its own definition)
  p->convention = p->mode != kPairInterp &&
                  (p->preset_conv >= 0 ? p->preset_conv : option(SS_OPT_CONVENTION)) != 0;
  p->kernel = plan_kernel(p->mode, p->q, p->learn, p->convention);
  DeviceInfo di;
  int rc = device_info(&di);
  if (rc != SS_OK) return rc;
  p->device = di.device;
  // staged grids and learned models can take a workgroup past the 64 KB a
  // launch gets without asking
  if (p->lds > di.lds_per_block)
    return fail(SS_ERR_UNSUPPORTED, "plan needs " + std::to_string(p->lds) +
                                        " bytes of LDS per workgroup; the device has " +
                                        std::to_string(di.lds_per_block));
  if (p->lds > 65536)
    SS_TRY_HIP(hipFuncSetAttribute(p->kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)p->lds));
  const int per_cu = blocks_per_cu(p->kernel, p->block, p->lds);
  const int resident = per_cu * di.num_cus;
  p->tiles_per_wg = choose_tiles_per_workgroup(tuner_model(), p->total_tiles, resident, S,
                                               per_tile);
  // An interpolation workgroup alone on its CU stages its grid with no
  // other workgroup's work to overlap: four times the tiles (5 / 20 / 40
  // tiles of 4096 pairs per workgroup: 5.61 / 5.11 / 5.09 ms on the
  // 1024-material workload), while that leaves six workgroups per slot.
  if (p->mode == kPairInterp && per_cu == 1)
    p->tiles_per_wg = (int)std::max<int64_t>(
        p->tiles_per_wg,
        std::min<int64_t>(4LL * p->tiles_per_wg, p->total_tiles / (6LL * resident)));
  if (option(SS_OPT_PLAN_TILES) > 0) p->tiles_per_wg = (int)option(SS_OPT_PLAN_TILES);
  if (p->preset_tiles > 0) p->tiles_per_wg = p->preset_tiles;
  // Each segment's tiles go to ceil(tiles / k) workgroups of at most k
  // tiles each (k = tiles_per_wg), never across a segment boundary: either
  // as contiguous ranges (workgroup i takes tiles i k .. i k + k - 1) or
  // strided (workgroup i of W takes tiles i, i + W, i + 2W, ...).
  // Strided is the default: measured on the 4096-material paired workload
  // (1e9 pairs) at 4 / 6 tiles per workgroup, contiguous 4.070 / 4.089 ms,
  // strided 4.029 / 4.016 ms; the 512-table batch 1.460 / 1.490 against
  // 1.459 / 1.464 ms.  A segment's workgroups are dispatched together, and
  // strided they read one advancing window of the segment's targets rather
  // than W separate streams.
  const int64_t order = p->preset_order >= 0 ? p->preset_order : option(SS_OPT_PLAN_ORDER);
  p->strided = order != kOrderContiguous;
  std::vector<WgStart> wg_start;
  for (int s = 0; s < S; ++s) {
    const int64_t tiles = tile_off[s + 1] - tile_off[s];
    const int64_t W = (tiles + p->tiles_per_wg - 1) / p->tiles_per_wg;
    for (int64_t i = 0; i < W; ++i) {
      WgStart st;
      st.seg = s;
      st.seg_q0 = p->query_off[s] - seg_base(s);
      st.seg_q1 = p->query_off[s + 1] - seg_base(s);
      st.seg_tiles = (int32_t)tiles;
      if (p->strided) {
        st.first = (int32_t)i;
        st.count = (int32_t)((tiles - i + W - 1) / W);
      } else {
        st.first = (int32_t)(i * p->tiles_per_wg);
        st.count = (int32_t)std::min<int64_t>(p->tiles_per_wg, tiles - st.first);
      }
      wg_start.push_back(st);
    }
  }
  if (wg_start.empty()) {  // no targets: one idle record keeps the launch valid
    WgStart st{0, 0, 0, 0, 0, 0};
    wg_start.push_back(st);
  }
  const int64_t num_wg = (int64_t)wg_start.size();
  const int64_t xcd = option(SS_OPT_PLAN_XCD);
  const int64_t tile_scale = std::max<int64_t>(1, 4096 / per_tile);
  const bool short_segments =
      p->total_tiles / std::max(S, 1) / tile_scale < kShortSegmentTiles;
  const int64_t chunk = xcd >= 2 ? xcd : (xcd == 1 || short_segments) ? 1 : kXcdChunk;
  const int groups = chunk == 1 ? 1 : kXcds;
  const int64_t grid = (num_wg + groups - 1) / groups * groups;
  if (grid > INT32_MAX) return fail(SS_ERR_INVALID_ARG, "too many tiles for one launch");
  p->grid = (int)grid;
  p->num_wg = (int)num_wg;
  p->xcd_groups = groups;
  p->xcd_chunk = (int)std::max<int64_t>(1, std::min<int64_t>(chunk, grid / groups));
  SS_TRY_HIP(hipMalloc(&p->d_tile_off, sizeof(int64_t) * (S + 1)));
  SS_TRY_HIP(hipMalloc(&p->d_query_off, sizeof(int64_t) * (S + 1)));
  SS_TRY_HIP(hipMalloc(&p->d_wg_start, sizeof(WgStart) * p->num_wg));
  SS_TRY_HIP(hipMemcpy(p->d_tile_off, tile_off.data(), sizeof(int64_t) * (S + 1),
                       hipMemcpyHostToDevice));
  SS_TRY_HIP(hipMemcpy(p->d_query_off, p->query_off.data(), sizeof(int64_t) * (S + 1),
                       hipMemcpyHostToDevice));
  SS_TRY_HIP(hipMemcpy(p->d_wg_start, wg_start.data(), sizeof(WgStart) * p->num_wg,
                       hipMemcpyHostToDevice));

  MultiArgs& a = p->args;
  a.tables_a = tables_a;
  a.tables_b = tables_b;
  a.desc = p->d_desc;
  a.bins = p->d_bins;
  a.tile_off = p->d_tile_off;
  a.query_off = p->d_query_off;
  a.wg_start = p->d_wg_start;
  a.params = p->d_pool;
  a.fallbacks = p->d_fallbacks;
  a.total_tiles = p->total_tiles;
  a.tiles_per_wg = p->tiles_per_wg;
  a.strided = p->strided ? 1 : 0;
  a.num_wg = p->num_wg;
  a.xcd_groups = p->xcd_groups;
  a.xcd_chunk = p->xcd_chunk;
  a.pair_base = p->paired ? p->M : 0;
  a.split = p->split;
  a.lds_bins_a = (int)lds_tab_a;
  a.lds_tab_b = (int)(lds_tab_a + lds_bins_a);
  a.lds_bins_b = (int)(lds_tab_a + lds_bins_a + lds_tab_b);
  a.lds_model_a = model_a;
  a.lds_model_b = model_b;
  a.lead = p->lead;

  // the graph holds the one search launch (preceded, with learned tables, by
  // a one-thread node clearing the fallback counter); pointers are updated
  // in place
  SS_TRY_HIP(hipGraphCreate(&p->graph, 0));
  void* kargs[] = {&p->args};
  hipKernelNodeParams kp = search_node_params(p, kargs);
  if (p->learned_tables > 0) {
    hipKernelNodeParams cp{};
    void* cargs[] = {&p->d_fallbacks};
    cp.func = reinterpret_cast<void*>(&plan_clear_kernel);
    cp.gridDim = dim3(1);
    cp.blockDim = dim3(1);
    cp.sharedMemBytes = 0;
    cp.kernelParams = cargs;
    cp.extra = nullptr;
    SS_TRY_HIP(hipGraphAddKernelNode(&p->clear_node, p->graph, nullptr, 0, &cp));
    SS_TRY_HIP(hipGraphAddKernelNode(&p->search_node, p->graph, &p->clear_node, 1, &kp));
  } else {
    SS_TRY_HIP(hipGraphAddKernelNode(&p->search_node, p->graph, nullptr, 0, &kp));
  }
  SS_TRY_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
  if (log_enabled()) {
    int count[8] = {0};
    double br_sum = 0;
    int br_n = 0;
    for (int t = 0; t < p->T; ++t) {
      ++count[std::min(std::max(p->tuned[t].algo, 0), 7)];
      if (t < (int)p->brackets.size() && p->brackets[t] >= 0) {
        br_sum += p->brackets[t];
        ++br_n;
      }
    }
    static const char* kForm[] = {"batched", "paired-joint", "paired-split", "interpolation"};
    log_line("plan %s: %d tables (exphash %d, bisection %d, ballot %d, learned %d), %lld "
             "targets, %lld tiles of %d, %d per workgroup %s, grid %d x %d, LDS %zu B, XCD "
             "chunk %d%s",
             kForm[p->mode], p->T, count[SS_ALGO_EXPHASH], count[SS_ALGO_BINARY],
             count[SS_ALGO_BALLOT], count[SS_ALGO_LEARNED], (long long)p->total_queries,
             (long long)p->total_tiles, p->block * p->q, p->tiles_per_wg,
             p->strided ? "strided" : "contiguous", p->grid, p->block, p->lds,
             p->xcd_groups > 1 ? p->xcd_chunk : 1, p->convention ? ", paper convention" : "");
    if (br_n > 0)
      log_line("plan sample: mean ballot bracket %.2f entries over %d tables", br_sum / br_n,
               br_n);
  }
  return SS_OK;
}

int run_plan(ss_plan* p, const double* xa, int32_t* oa, const double* xb, int32_t* ob,
             double* of = nullptr) {
  if (p->total_queries == 0 || p->total_tiles == 0) return SS_OK;
  int dev = -1;
  SS_TRY_HIP(hipGetDevice(&dev));
  if (dev != p->device) return fail(SS_ERR_INVALID_ARG, "plan was built on another device");
  if (xa != p->args.xa || oa != p->args.oa || xb != p->args.xb || ob != p->args.ob ||
      of != p->args.of) {
    p->args.xa = xa;
    p->args.oa = oa;
    p->args.xb = xb;
    p->args.ob = ob;
    p->args.of = of;
    p->args.store_idx = oa != nullptr && ob != nullptr;
    void* kargs[] = {&p->args};
    hipKernelNodeParams kp = search_node_params(p, kargs);
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

// Batched plan creation; models (T handles, entries may be null) attaches
// learned models, else SS_OPT_PLAN_LEARNED may train them.
static int create_batched(const double* tables, const int64_t* table_off, int32_t T,
                          const int64_t* query_off, ss_learned* const* models, ss_plan** out,
                          const PlanPreset* preset = nullptr, const double* sample = nullptr) {
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
  if (sample && query_off[T] > 0 &&
      ((rc = check_span(sample, query_off[T], 8, 8, "sample")) != SS_OK ||
       (rc = check_device_ptr(sample, "sample")) != SS_OK))
    return rc;

  std::vector<double> host(total_n);
  if (total_n > 0) {
    SS_TRY_HIP(hipMemcpyAsync(host.data(), tables, sizeof(double) * total_n,
                              hipMemcpyDeviceToHost, current_stream()));
    SS_TRY_HIP(hipStreamSynchronize(current_stream()));
  }
  ss_plan* p = new (std::nothrow) ss_plan();
  if (!p) return fail(SS_ERR_OOM, "plan");
  p->T = T;
  p->S = T;
  p->query_off.assign(query_off, query_off + T + 1);
  p->total_queries = query_off[T];
  const TunerModel& model = tuner_model();
  p->desc.resize(T);
  p->tuned.resize(T);
  p->weights.resize(T);
  if (preset) {
    if (preset->mode != kBatched || preset->descriptors != T)
      return fail_delete(p, "the saved plan is not a batched plan of this many tables");
    for (int t = 0; t < T; ++t)
      if (preset->n[t] != table_off[t + 1] - table_off[t])
        return fail_delete(p, ("table " + std::to_string(t) + " differs in size from the saved "
                               "plan's").c_str());
    p->preset_tiles = preset->tiles_per_wg;
    p->preset_order = preset->strided ? kOrderStrided : kOrderContiguous;
    p->preset_conv = preset->convention;
  }
  size_t max_tab = 16, max_bins = 0;
  for (int t = 0; t < T; ++t)
    max_tab = std::max(max_tab, align16((size_t)(table_off[t + 1] - table_off[t] + SS_PAD) * 8));
  if (max_tab > kPlanLdsBudget)
    return fail_delete(p, "a table exceeds the 48 KB LDS staging budget (6136 entries)",
                       SS_ERR_UNSUPPORTED);
  const int force = (int)option(SS_OPT_PLAN_ALGO);
  p->brackets.assign(T, -1.0);
  if (sample && !preset) {
    std::vector<BracketJob> jobs(T);
    for (int t = 0; t < T; ++t)
      jobs[t] = {tables + table_off[t], sample, query_off[t], query_off[t + 1],
                 (int)(table_off[t + 1] - table_off[t]), 0};
    if ((rc = sample_brackets(jobs, kBatched, &p->brackets)) != SS_OK)
      return fail_delete(p, nullptr, rc);
  }
  int64_t pool = 0;
  for (int t = 0; t < T; ++t) {
    const int n = (int)(table_off[t + 1] - table_off[t]);
    if (preset) {
      p->tuned[t] = preset_table(model, host.data() + table_off[t], n, kPlanLdsBudget - max_tab,
                                 preset->algo[t], preset->bits[t]);
    } else {
      p->tuned[t] = tune_table(model, host.data() + table_off[t], n, kPlanLdsBudget - max_tab,
                               force);
      consider_ballot(model, p->brackets[t], force, &p->tuned[t]);
    }
    describe(p->tuned[t], table_off[t], &p->desc[t], &pool);
    if (p->tuned[t].algo == SS_ALGO_EXPHASH)
      max_bins = std::max(max_bins, align16((size_t)(p->tuned[t].nb + 1) * 2));
  }
  if (models || preset || learned_mode() != kLearnedNone) {
    rc = models ? attach_learned(p, tables, table_off, models)
                : apply_learned(p, tables, nullptr, host, host, learned_mode(), preset);
    if (rc != SS_OK) return fail_delete(p, nullptr, rc);
    max_bins = 0;
    for (int t = 0; t < T; ++t)
      if (p->desc[t].algo == SS_ALGO_EXPHASH)
        max_bins = std::max(max_bins, align16((size_t)(p->desc[t].nb + 1) * 2));
  }
  rc = finish_plan(p, tables, nullptr, pool, max_tab, max_bins, 0, 0);
  if (rc != SS_OK) {
    delete p;
    return rc;
  }
  *out = p;
  return SS_OK;
}

int ss_multi_plan_create(const double* tables, const int64_t* table_off, int32_t T,
                         const int64_t* query_off, ss_plan** out) {
  return create_batched(tables, table_off, T, query_off, nullptr, out);
}

int ss_multi_plan_create_sampled(const double* tables, const int64_t* table_off, int32_t T,
                                 const int64_t* query_off, const double* sample,
                                 ss_plan** out) {
  if (!sample) {
    clear_error();
    return fail(SS_ERR_INVALID_ARG, "sample is null");
  }
  return create_batched(tables, table_off, T, query_off, nullptr, out, nullptr, sample);
}

int ss_multi_plan_create_learned(const double* tables, const int64_t* table_off, int32_t T,
                                 const int64_t* query_off, ss_learned* const* models,
                                 ss_plan** out) {
  if (!models) {
    clear_error();
    return fail(SS_ERR_INVALID_ARG, "models is null");
  }
  return create_batched(tables, table_off, T, query_off, models, out);
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

}  // extern "C"

namespace ss {
namespace {

// Paired plans of every form (mode kPairSplit, kPairJoint or kPairInterp;
// values: the interpolation form's value grids, else null).
int create_paired(const double* rho_tables, const int64_t* rho_off, const double* t_tables,
                  const int64_t* t_off, int32_t M, const int64_t* pair_off, int mode,
                  const double* values, ss_plan** out, const PlanPreset* preset = nullptr,
                  const double* sample_rho = nullptr, const double* sample_t = nullptr) {
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
  if (sample_rho && pair_off[M] > 0 &&
      ((rc = check_span(sample_rho, pair_off[M], 8, 8, "sample_rho")) != SS_OK ||
       (rc = check_span(sample_t, pair_off[M], 8, 8, "sample_temp")) != SS_OK ||
       (rc = check_device_ptr(sample_rho, "sample_rho")) != SS_OK ||
       (rc = check_device_ptr(sample_t, "sample_temp")) != SS_OK))
    return rc;
  std::vector<double> hr(nr), ht(ntt);
  hipStream_t st = current_stream();
  if (nr > 0) SS_TRY_HIP(hipMemcpyAsync(hr.data(), rho_tables, 8 * nr, hipMemcpyDeviceToHost, st));
  if (ntt > 0) SS_TRY_HIP(hipMemcpyAsync(ht.data(), t_tables, 8 * ntt, hipMemcpyDeviceToHost, st));
  SS_TRY_HIP(hipStreamSynchronize(st));
  int64_t nvalues = 0, grid_cap_needed = 0;
  std::vector<int64_t> value_off;
  if (mode == kPairInterp) {
    // every axis needs a cell: at least 2 strictly increasing finite entries
    value_off.assign(M + 1, 0);
    for (int j = 0; j < M; ++j) {
      const double* axes[2] = {hr.data() + rho_off[j], ht.data() + t_off[j]};
      const int64_t len[2] = {rho_off[j + 1] - rho_off[j], t_off[j + 1] - t_off[j]};
      for (int ax = 0; ax < 2; ++ax) {
        if (len[ax] < 2)
          return fail(SS_ERR_INVALID_ARG, "interpolation needs 2 or more entries per axis");
        for (int64_t i = 0; i < len[ax]; ++i)
          if (!std::isfinite(axes[ax][i]) || (i > 0 && !(axes[ax][i] > axes[ax][i - 1])))
            return fail(SS_ERR_INVALID_ARG, "material " + std::to_string(j) +
                                                ": axes must be finite and strictly increasing");
      }
      value_off[j + 1] = value_off[j] + len[0] * len[1];
    }
    nvalues = value_off[M];
    for (int j = 0; j < M; ++j) {
      const int64_t count = value_off[j + 1] - value_off[j];
      if (count <= kInterpGridLdsValues) grid_cap_needed = std::max(grid_cap_needed, count);
    }
    if ((rc = check_span(values, nvalues, 8, 8, "values")) != SS_OK) return rc;
    if ((rc = check_device_ptr(values, "values")) != SS_OK) return rc;
  }
  ss_plan* p = new (std::nothrow) ss_plan();
  if (!p) return fail(SS_ERR_OOM, "plan");
  p->paired = 1;
  p->mode = mode;
  p->grid_cap = (int)grid_cap_needed;
  p->M = M;
  p->T = 2 * M;
  p->total_queries = pair_off[M];
  if (p->mode == kPairJoint || p->mode == kPairInterp) {
    p->S = M;
    p->query_off.assign(pair_off, pair_off + M + 1);
  } else {
    // segments 0..M-1: density axis; M..2M-1: temperature axis, whose
    // offsets continue after the last pair
    p->S = 2 * M;
    p->split = pair_off[M];
    p->query_off.assign(pair_off, pair_off + M + 1);
    for (int j = 1; j <= M; ++j) p->query_off.push_back(p->split + pair_off[j]);
  }
  const TunerModel& model = tuner_model();
  p->desc.resize(2 * M);
  p->tuned.resize(2 * M);
  p->weights.resize(2 * M);
  if (preset) {
    if (preset->mode != mode || preset->descriptors != 2 * M)
      return fail_delete(p, "the saved plan is not a paired plan of this form and size");
    for (int j = 0; j < M; ++j)
      if (preset->n[j] != rho_off[j + 1] - rho_off[j] ||
          preset->n[M + j] != t_off[j + 1] - t_off[j])
        return fail_delete(p, ("material " + std::to_string(j) + " differs in size from the "
                               "saved plan's").c_str());
    p->preset_tiles = preset->tiles_per_wg;
    p->preset_order = preset->strided ? kOrderStrided : kOrderContiguous;
    p->preset_conv = preset->convention;
  }
  size_t tab_a = 16, bins_a = 0, tab_b = 16, bins_b = 0;
  for (int j = 0; j < M; ++j) {
    tab_a = std::max(tab_a, align16((size_t)(rho_off[j + 1] - rho_off[j] + SS_PAD) * 8));
    tab_b = std::max(tab_b, align16((size_t)(t_off[j + 1] - t_off[j] + SS_PAD) * 8));
  }
  size_t budget_a, budget_b;
  if (p->mode == kPairJoint || p->mode == kPairInterp) {
    if (tab_a + tab_b > kPlanLdsBudget)
      return fail_delete(p,
                         "the largest density and temperature tables together exceed the "
                         "48 KB LDS staging budget (6128 entries)",
                         SS_ERR_UNSUPPORTED);
    // the bin budget is split in proportion to the two axes' largest tables
    const size_t bins_total = kPlanLdsBudget - tab_a - tab_b;
    budget_a = bins_total * tab_a / (tab_a + tab_b);
    budget_b = bins_total - budget_a;
  } else {
    // one table at a time: either axis may use what the largest table leaves
    tab_a = tab_b = std::max(tab_a, tab_b);
    if (tab_a > kPlanLdsBudget)
      return fail_delete(p, "a table exceeds the 48 KB LDS staging budget (6136 entries)",
                         SS_ERR_UNSUPPORTED);
    budget_a = budget_b = kPlanLdsBudget - tab_a;
  }
  int64_t pool = 0;
  const int force = (int)option(SS_OPT_PLAN_ALGO);
  // both axes' searches of material j cover the pairs [pair_off[j], pair_off[j + 1])
  p->brackets.assign(2 * M, -1.0);
  if (sample_rho && !preset) {
    std::vector<BracketJob> jobs(2 * M);
    for (int j = 0; j < M; ++j) {
      jobs[j] = {rho_tables + rho_off[j], sample_rho, pair_off[j], pair_off[j + 1],
                 (int)(rho_off[j + 1] - rho_off[j]), 0};
      jobs[M + j] = {t_tables + t_off[j], sample_t, pair_off[j], pair_off[j + 1],
                     (int)(t_off[j + 1] - t_off[j]), 0};
    }
    if ((rc = sample_brackets(jobs, mode, &p->brackets)) != SS_OK)
      return fail_delete(p, nullptr, rc);
  }
  for (int j = 0; j < M; ++j) {
    const int n = (int)(rho_off[j + 1] - rho_off[j]);
    if (preset) {
      p->tuned[j] = preset_table(model, hr.data() + rho_off[j], n, budget_a, preset->algo[j],
                                 preset->bits[j]);
    } else {
      p->tuned[j] = tune_table(model, hr.data() + rho_off[j], n, budget_a, force);
      consider_ballot(model, p->brackets[j], force, &p->tuned[j]);
    }
    describe(p->tuned[j], rho_off[j], &p->desc[j], &pool);
    if (p->tuned[j].algo == SS_ALGO_EXPHASH)
      bins_a = std::max(bins_a, align16((size_t)(p->tuned[j].nb + 1) * 2));
  }
  for (int j = 0; j < M; ++j) {
    const int n = (int)(t_off[j + 1] - t_off[j]);
    if (preset) {
      p->tuned[M + j] = preset_table(model, ht.data() + t_off[j], n, budget_b,
                                     preset->algo[M + j], preset->bits[M + j]);
    } else {
      p->tuned[M + j] = tune_table(model, ht.data() + t_off[j], n, budget_b, force);
      consider_ballot(model, p->brackets[M + j], force, &p->tuned[M + j]);
    }
    describe(p->tuned[M + j], t_off[j], &p->desc[M + j], &pool);
    if (p->tuned[M + j].algo == SS_ALGO_EXPHASH)
      bins_b = std::max(bins_b, align16((size_t)(p->tuned[M + j].nb + 1) * 2));
  }
  if ((preset || learned_mode() != kLearnedNone) && p->mode != kPairInterp) {
    if ((rc = apply_learned(p, rho_tables, t_tables, hr, ht, learned_mode(), preset)) != SS_OK)
      return fail_delete(p, nullptr, rc);
    bins_a = bins_b = 0;
    for (int j = 0; j < M; ++j) {
      if (p->desc[j].algo == SS_ALGO_EXPHASH)
        bins_a = std::max(bins_a, align16((size_t)(p->desc[j].nb + 1) * 2));
      if (p->desc[M + j].algo == SS_ALGO_EXPHASH)
        bins_b = std::max(bins_b, align16((size_t)(p->desc[M + j].nb + 1) * 2));
    }
  }
  if (p->mode == kPairInterp) {
    hipError_t e = hipMalloc(&p->d_value_off, sizeof(int64_t) * (M + 1));
    if (e == hipSuccess)
      e = hipMemcpy(p->d_value_off, value_off.data(), sizeof(int64_t) * (M + 1),
                    hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      delete p;
      return hip_fail(e, "interpolation value offsets");
    }
    p->args.values = values;
    p->args.value_off = p->d_value_off;
  }
  if (p->mode == kPairJoint || p->mode == kPairInterp)
    rc = finish_plan(p, rho_tables, t_tables, pool, tab_a, bins_a, tab_b, bins_b);
  else
    rc = finish_plan(p, rho_tables, t_tables, pool, tab_a, std::max(bins_a, bins_b), 0, 0);
  if (rc != SS_OK) {
    delete p;
    return rc;
  }
  *out = p;
  return SS_OK;
}

}  // namespace
}  // namespace ss

extern "C" {

int ss_pair_plan_create(const double* rho_tables, const int64_t* rho_off, const double* t_tables,
                        const int64_t* t_off, int32_t M, const int64_t* pair_off, ss_plan** out) {
  clear_error();
  return create_paired(rho_tables, rho_off, t_tables, t_off, M, pair_off,
                       option(SS_OPT_PAIR_JOINT) ? kPairJoint : kPairSplit, nullptr, out);
}

int ss_pair_plan_create_sampled(const double* rho_tables, const int64_t* rho_off,
                                const double* t_tables, const int64_t* t_off, int32_t M,
                                const int64_t* pair_off, const double* sample_rho,
                                const double* sample_temp, ss_plan** out) {
  clear_error();
  if (!sample_rho || !sample_temp) return fail(SS_ERR_INVALID_ARG, "a sample array is null");
  return create_paired(rho_tables, rho_off, t_tables, t_off, M, pair_off,
                       option(SS_OPT_PAIR_JOINT) ? kPairJoint : kPairSplit, nullptr, out,
                       nullptr, sample_rho, sample_temp);
}

int ss_interp_plan_create(const double* rho_tables, const int64_t* rho_off,
                          const double* t_tables, const int64_t* t_off, int32_t M,
                          const int64_t* pair_off, const double* values, ss_plan** out) {
  clear_error();
  return create_paired(rho_tables, rho_off, t_tables, t_off, M, pair_off, kPairInterp, values,
                       out);
}

int ss_interp_search(ss_plan* p, const double* rho, const double* temp, double* out_f,
                     int32_t* out_rho, int32_t* out_t) {
  clear_error();
  if (!p) return fail(SS_ERR_INVALID_ARG, "plan is null");
  if (p->mode != kPairInterp) return fail(SS_ERR_INVALID_ARG, "not an interpolation plan");
  if ((out_rho == nullptr) != (out_t == nullptr))
    return fail(SS_ERR_INVALID_ARG, "out_rho and out_t: both or neither");
  const int64_t m = p->total_queries;
  int rc = check_span(rho, m, 8, 8, "rho");
  if (rc == SS_OK) rc = check_span(temp, m, 8, 8, "temp");
  if (rc == SS_OK) rc = check_span(out_f, m, 8, 8, "out_f");
  if (rc == SS_OK && out_rho) rc = check_span(out_rho, m, 4, 4, "out_rho");
  if (rc == SS_OK && out_t) rc = check_span(out_t, m, 4, 4, "out_t");
  if (rc != SS_OK) return rc;
  if (m > 0) {
    const size_t ib = (size_t)m * 8, ob = (size_t)m * 4;
    if (overlaps(out_f, ib, rho, ib) || overlaps(out_f, ib, temp, ib) ||
        (out_rho && (overlaps(out_rho, ob, rho, ib) || overlaps(out_rho, ob, temp, ib) ||
                     overlaps(out_rho, ob, out_f, ib) || overlaps(out_t, ob, rho, ib) ||
                     overlaps(out_t, ob, temp, ib) || overlaps(out_t, ob, out_f, ib) ||
                     overlaps(out_rho, ob, out_t, ob))))
      return fail(SS_ERR_INVALID_ARG, "outputs overlap inputs or each other");
    if ((rc = check_device_ptr(rho, "rho")) != SS_OK ||
        (rc = check_device_ptr(temp, "temp")) != SS_OK ||
        (rc = check_device_ptr(out_f, "out_f")) != SS_OK ||
        (out_rho && (rc = check_device_ptr(out_rho, "out_rho")) != SS_OK) ||
        (out_t && (rc = check_device_ptr(out_t, "out_t")) != SS_OK))
      return rc;
  }
  return run_plan(p, rho, out_rho, temp, out_t, out_f);
}

int ss_pair_search(ss_plan* p, const double* rho, const double* temp, int32_t* out_rho,
                   int32_t* out_t) {
  clear_error();
  if (!p) return fail(SS_ERR_INVALID_ARG, "plan is null");
  if (!p->paired) return fail(SS_ERR_INVALID_ARG, "batched plan: use ss_multi_search");
  if (p->mode == kPairInterp) return fail(SS_ERR_INVALID_ARG, "interpolation plan: use ss_interp_search");
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

// Saved plans: a text file of the plan's choices, "ss_plan 1" then
//   mode M descriptors T materials M tiles K strided 0|1 convention 0|1
//   table t n N algo A bits S          (one line per descriptor)
//   weights t w0 ... w1152             (one line per learned table)
//   end
// Parameters are printed with 9 significant digits, which read back into
// the same FP32 values.
int ss_plan_save(const ss_plan* p, const char* path) {
  clear_error();
  if (!p || !path) return fail(SS_ERR_INVALID_ARG, "null argument");
  if (p->mode == kPairInterp)
    return fail(SS_ERR_UNSUPPORTED, "interpolation plans are not saved (no learned tables)");
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(SS_ERR_INVALID_ARG, std::string("cannot write ") + path);
  std::fprintf(f, "ss_plan 1\nmode %d descriptors %d materials %d tiles %d strided %d convention %d\n",
               p->mode, p->T, p->M, p->tiles_per_wg, p->strided ? 1 : 0, p->convention ? 1 : 0);
  for (int t = 0; t < p->T; ++t)
    std::fprintf(f, "table %d n %d algo %d bits %d\n", t, p->desc[t].n, p->tuned[t].algo,
                 p->tuned[t].algo == SS_ALGO_EXPHASH ? p->tuned[t].bits : -1);
  for (int t = 0; t < p->T; ++t) {
    if (p->weights[t].empty()) continue;
    std::fprintf(f, "weights %d", t);
    for (float w : p->weights[t]) std::fprintf(f, " %.9g", (double)w);
    std::fprintf(f, "\n");
  }
  std::fprintf(f, "end\n");
  return std::fclose(f) == 0 ? SS_OK : fail(SS_ERR_INVALID_ARG, std::string("cannot write ") + path);
}

}  // extern "C"

namespace ss {
namespace {

int read_preset(const char* path, PlanPreset* pr) {
  if (!path) return fail(SS_ERR_INVALID_ARG, "path is null");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(SS_ERR_INVALID_ARG, std::string("cannot open ") + path);
  std::string text;
  char buf[1 << 16];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  std::fclose(f);
  std::istringstream in(text);
  const std::string bad = std::string("malformed saved plan ") + path;
  auto expect = [&](const char* word) {
    std::string w;
    return (in >> w) && w == word;
  };
  int version = 0;
  if (!expect("ss_plan") || !(in >> version) || version != 1) return fail(SS_ERR_INVALID_ARG, bad);
  if (!expect("mode") || !(in >> pr->mode) || !expect("descriptors") || !(in >> pr->descriptors) ||
      !expect("materials") || !(in >> pr->materials) || !expect("tiles") ||
      !(in >> pr->tiles_per_wg) || !expect("strided") || !(in >> pr->strided) ||
      !expect("convention") || !(in >> pr->convention))
    return fail(SS_ERR_INVALID_ARG, bad);
  if (pr->mode < kBatched || pr->mode > kPairSplit || pr->descriptors < 1 ||
      pr->descriptors > (2 << 20) || pr->tiles_per_wg < 1 || pr->tiles_per_wg > 4096)
    return fail(SS_ERR_INVALID_ARG, bad);
  const int T = pr->descriptors;
  pr->n.assign(T, -1);
  pr->algo.assign(T, 0);
  pr->bits.assign(T, -1);
  pr->weights.assign(T, {});
  for (int t = 0; t < T; ++t) {
    int idx = -1;
    if (!expect("table") || !(in >> idx) || idx != t || !expect("n") || !(in >> pr->n[t]) ||
        !expect("algo") || !(in >> pr->algo[t]) || !expect("bits") || !(in >> pr->bits[t]))
      return fail(SS_ERR_INVALID_ARG, bad);
  }
  std::string w;
  while (in >> w && w == "weights") {
    int t = -1;
    if (!(in >> t) || t < 0 || t >= T || !pr->weights[t].empty())
      return fail(SS_ERR_INVALID_ARG, bad);
    pr->weights[t].resize(SS_MLP_PARAMS);
    for (int i = 0; i < SS_MLP_PARAMS; ++i) {
      std::string v;
      if (!(in >> v)) return fail(SS_ERR_INVALID_ARG, bad);
      char* end = nullptr;
      pr->weights[t][i] = std::strtof(v.c_str(), &end);
      if (end == v.c_str() || *end) return fail(SS_ERR_INVALID_ARG, bad);
    }
  }
  if (w != "end") return fail(SS_ERR_INVALID_ARG, bad);
  return SS_OK;
}

}  // namespace
}  // namespace ss

extern "C" {

int ss_multi_plan_load(const char* path, const double* tables, const int64_t* table_off,
                       int32_t T, const int64_t* query_off, ss_plan** out) {
  clear_error();
  if (!out) return fail(SS_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  PlanPreset pr;
  const int rc = read_preset(path, &pr);
  if (rc != SS_OK) return rc;
  return create_batched(tables, table_off, T, query_off, nullptr, out, &pr);
}

int ss_pair_plan_load(const char* path, const double* rho_tables, const int64_t* rho_off,
                      const double* t_tables, const int64_t* t_off, int32_t M,
                      const int64_t* pair_off, ss_plan** out) {
  clear_error();
  if (!out) return fail(SS_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  PlanPreset pr;
  const int rc = read_preset(path, &pr);
  if (rc != SS_OK) return rc;
  if (pr.mode != kPairSplit && pr.mode != kPairJoint)
    return fail(SS_ERR_INVALID_ARG, "the saved plan is not a paired plan");
  return create_paired(rho_tables, rho_off, t_tables, t_off, M, pair_off, pr.mode, nullptr, out,
                       &pr);
}

int ss_plan_destroy(ss_plan* p) {
  clear_error();
  delete p;
  return SS_OK;
}

int ss_plan_fallbacks(ss_plan* p, int64_t* count) {
  clear_error();
  if (!p || !count) return fail(SS_ERR_INVALID_ARG, "null argument");
  *count = 0;
  if (!p->d_fallbacks) return SS_OK;
  unsigned long long v = 0;
  hipStream_t st = current_stream();
  SS_TRY_HIP(hipMemcpyAsync(&v, p->d_fallbacks, sizeof(v), hipMemcpyDeviceToHost, st));
  SS_TRY_HIP(hipStreamSynchronize(st));
  *count = (int64_t)v;
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
    case SS_PLAN_BRACKETS: {
      if (cap < p->T) return fail(SS_ERR_INVALID_ARG, "cap smaller than the table count");
      double* o = static_cast<double*>(out);
      for (int t = 0; t < p->T; ++t) o[t] = t < (int)p->brackets.size() ? p->brackets[t] : -1.0;
      return SS_OK;
    }
    case SS_PLAN_COSTS: {
      if (cap < 2 * (int64_t)p->T) return fail(SS_ERR_INVALID_ARG, "cap smaller than 2 T");
      double* o = static_cast<double*>(out);
      for (int t = 0; t < p->T; ++t) {
        o[2 * t] = p->tuned[t].est_ns;
        o[2 * t + 1] = p->tuned[t].learned_ns;
      }
      return SS_OK;
    }
    case SS_PLAN_SUMMARY: {
      if (cap < 8) return fail(SS_ERR_INVALID_ARG, "cap must be >= 8");
      int64_t* o = static_cast<int64_t*>(out);
      o[0] = p->T;
      o[1] = p->total_tiles;
      o[2] = p->tiles_per_wg;
      o[3] = p->grid;
      o[4] = p->block;
      o[5] = (int64_t)p->lds;
      o[6] = p->max_k;
      o[7] = p->graph_uses;
      if (cap >= 10) {
        o[8] = p->q;
        o[9] = p->learn;
      }
      return SS_OK;
    }
    default:
      return fail(SS_ERR_INVALID_ARG, "unknown query");
  }
}

}  // extern "C"

namespace ss {
int violations_plan(unsigned long long* out) { return read_violations(out); }
void plan_learned_q_fixed(bool fixed) { t_learned_q_fixed = fixed; }
}  // namespace ss
