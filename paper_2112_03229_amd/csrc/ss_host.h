// Host-side internals shared by the library's translation units: status and
// error reporting, the per-thread stream, process-wide options, device
// properties and argument checks.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/searchsorted.h"

namespace ss {

// Records `msg` as the calling thread's last error and returns `code`.
int fail(int code, const std::string& msg);
// Maps a HIP error to SS_ERR_HIP (or SS_ERR_OOM) with context; SS_OK if ok.
int hip_fail(hipError_t e, const char* what);
void clear_error();

hipStream_t current_stream();

int64_t option(int opt);

// SS_LOG: 1 or more writes one line per library decision to stderr.
bool log_enabled();
// printf-style line on stderr, prefixed "[ss] ", when SS_LOG is set.
void log_line(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

struct DeviceInfo {
  int device = -1;
  int num_cus = 0;
  size_t lds_per_block = 0;  // max dynamic + static LDS per workgroup
  int arch_ok = 0;           // 1 for gfx950
  char arch[64] = {0};
};
// Properties of the current device (cached per device).  Returns SS_OK or an
// error code (no device, HIP failure).
int device_info(DeviceInfo* out);

// Argument checks shared by the entry points.
int check_span(const void* p, int64_t count, size_t elem, size_t align, const char* name);
int check_device_ptr(const void* p, const char* name);
bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes);

// Device bounds-check violations counted by each module's kernels since
// the last read, then cleared (checked builds; SS_ERR_UNSUPPORTED
// otherwise).  One per translation unit: each holds its own counter.
int violations_single(unsigned long long* out);
int violations_plan(unsigned long long* out);
int violations_learned(unsigned long long* out);
int violations_noalloc(unsigned long long* out);
// Checked builds: one clamped out-of-range index in a one-thread kernel.
int checks_selftest();

// Workgroups of `kernel` that fit on one CU with `threads` threads and
// `lds` bytes of dynamic LDS (cached).
int blocks_per_cu(const void* kernel, int threads, size_t lds);

}  // namespace ss

#define SS_TRY_HIP(expr)                                   \
  do {                                                     \
    hipError_t _e = (expr);                                \
    if (_e != hipSuccess) return ::ss::hip_fail(_e, #expr); \
  } while (0)
