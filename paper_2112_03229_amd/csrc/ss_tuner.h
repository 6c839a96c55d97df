// Autotuner: a cost model of the search kernels, calibrated by device
// microbenchmarks, that picks each table's kernel, exponent-hash bin bits
// and how many consecutive target tiles a plan's workgroup searches.
#pragma once

#include <stdint.h>
#include <stddef.h>

namespace ss {

// Device-wide costs in nanoseconds per query at full occupancy.  A query's
// time is max(memory, compute): memory = 12 bytes / stream bandwidth,
// compute from the per-kernel terms below.
struct TunerModel {
  // Defaults: the values calibrate() measures on an MI355X (rounded).
  double stream_gbs = 6600.0;        // sustained bytes/ns of a 12 B/query stream
  double hash_base_ns = 3.3e-3;      // exponent hash: key, bin read, select
  double hash_per_k_ns = 0.4e-3;     // per entry of the fixed in-bin scan
  double bin_base_ns = 0.0;          // bisection: final compare and select
  double bin_per_step_ns = 1.05e-3;  // per bisection step
  double learned_base_ns = 0.0;      // learned index: input, prediction and
                                     // the window's verification
  double learned_per_step_ns = 1.05e-3;  // per LDS step of its model lookup and
                                         // window bisection
  double bins_per_entry = 4.0;       // most exponent-hash bins per table entry
                                     // (each workgroup copies its bins)
  double tiles_short = 5;            // target tiles (of 4096) per plan workgroup
  double tiles_long = 5;             // for segments averaging under / over 64 tiles
  double ballot_base_ns = 2.0e-3;    // ballot scan: wave bracket and select
  double ballot_per_entry_ns = 0.5e-3;  // per iteration of its bracket scan or
                                        // of its 64-entry ballot pass
  int calibrated = 0;                // 1 once measured on this device
};

// Modelled compute cost (ns per query) of the ballot scan on a table of n
// entries whose waves' targets span `bracket` entries on average (the
// per-lane scan) after ceil((n + 1) / 64) ballot steps.
double ballot_cost_ns(const TunerModel& model, double bracket, int n);

// Modelled compute cost (ns per query) of the learned index with error bound
// E and a model whose piece lookup takes `lookup_steps` LDS steps.
double learned_cost_ns(const TunerModel& model, int E, int lookup_steps);

// Window steps of the learned search for error bound E (the bisection over
// 2E + 1 candidate positions plus the two checks of its ends).
int learned_window_steps(int E);

struct TunedTable {
  int n = 0;
  int algo = 1;        // SS_ALGO_BINARY, SS_ALGO_EXPHASH, SS_ALGO_BALLOT or SS_ALGO_LEARNED
  int bits = -1;       // s for the exponent hash
  int kmin = 0, kmaxc = 0, nb = 0;
  int K = 0;           // longest bin (exact)
  double est_ns = 0;   // modelled ns per query of the plain choice (compute part)
  double learned_ns = -1;  // modelled ns per query of its trained learned model
                           // (-1: none trained)
};

// The process-wide model (defaults until calibrated or loaded).
TunerModel tuner_model();

// Chooses the kernel and bin bits for one table of n entries; the bin table
// may take at most `bins_budget` bytes of LDS.  force = SS_ALGO_AUTO picks
// the cheapest; SS_ALGO_BINARY the bisection; SS_ALGO_EXPHASH the cheapest
// bin bits of the exponent hash wherever it applies (else the bisection).
TunedTable tune_table(const TunerModel& model, const double* a, int n, size_t bins_budget,
                      int force = 0);

// Consecutive tiles per workgroup of a plan launch with `total_tiles`
// tiles of `per_tile` targets in `segments` segments and `resident`
// workgroups resident at once.
int choose_tiles_per_workgroup(const TunerModel& model, int64_t total_tiles, int resident,
                               int segments, int64_t per_tile);

// While set (on this thread), plans with learned tables keep the plain
// targets per lane whatever their learned share: the calibration prices a
// learned table as it runs in a plan of few of them (ss_plan.hip).
void plan_learned_q_fixed(bool fixed);

// Longest run of equal exponent-hash keys (the largest bin) at bits s.
int host_longest_bin(const double* a, int n, int s);

}  // namespace ss
