// Host-side interface for training learned-index models of many tables at
// once (used by plans).  Internal to the library.
#pragma once

#include <stdint.h>

#include <vector>

#include "../../include/searchsorted.h"

namespace ss {

struct LearnedSlot {
  int64_t tab_off;  // first entry in its tables array
  int64_t i_off;    // first float of its compiled image in the image pool
  int n;            // entries (>= 2, 0 < a[0] < a[n-1] < inf)
  int which;        // 0: first tables array, 1: second (paired plans)
  float u0, inv;    // model input normalisation (computed on the device)
  int E;            // error bound (measured on the device)
  int head[4];      // its compiled image's header: boundary slots, pieces,
                    // cells, fullest cell (copied by the bound kernel)
  int pad_;
};

// Trains one model per slot (one workgroup per slot), compiles each into
// d_images (kImageFloats floats per slot at i_off) and measures each slot's
// error bound with the compiled forward pass; fills u0, inv and E of every
// slot.  With weights_in (host, SS_MLP_PARAMS floats per slot) the given
// parameters replace training; weights_out (if not null) receives every
// slot's parameters.  SYNCHRONOUS on the current stream.
int learned_train_slots(const double* tables_a, const double* tables_b,
                        std::vector<LearnedSlot>& slots, float* d_images, int steps, float lr,
                        uint64_t seed, const float* weights_in = nullptr,
                        std::vector<float>* weights_out = nullptr);

// True if a table (host copy) can have a learned model.
bool learned_eligible(const double* a, int64_t n);

// What a plan needs of a learned handle to search its table with it.
struct LearnedExport {
  const double* table;   // the device table the model was built on
  int n;
  int device;
  int E;
  float u0, inv;
  const float* image;    // compiled model (device)
  int image_floats;      // its floats in use
  const float* params;   // its SS_MLP_PARAMS parameters (host)
};
int learned_export(const ss_learned* h, LearnedExport* out);

}  // namespace ss
