// Library runtime: error state, stream selection, options, device queries
// and argument checks behind the C ABI.
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "ss_host.h"

namespace ss {

namespace {
thread_local std::string t_last_error;
thread_local hipStream_t t_stream = nullptr;

std::atomic<int64_t> g_force_algo{SS_ALGO_AUTO};
std::atomic<int64_t> g_bucket_bits{-1};
std::atomic<int64_t> g_bucket_cap{0};
std::atomic<int64_t> g_block_size{0};
std::atomic<int64_t> g_grid_blocks{0};
std::atomic<int64_t> g_check_pointers{1};
std::atomic<int64_t> g_targets_per_lane{0};
std::atomic<int64_t> g_plan_tiles{0};
std::atomic<int64_t> g_plan_learned{0};
std::atomic<int64_t> g_learned_steps{0};
std::atomic<int64_t> g_plan_xcd{0};
std::atomic<int64_t> g_pair_joint{0};
std::atomic<int64_t> g_convention{0};
std::atomic<int64_t> g_plan_algo{SS_ALGO_AUTO};
std::atomic<int64_t> g_plan_order{0};

std::mutex g_dev_mu;
std::map<int, DeviceInfo> g_dev_cache;
std::map<std::tuple<const void*, int, size_t, int>, int> g_occ_cache;
}  // namespace

int fail(int code, const std::string& msg) {
  t_last_error = msg;
  return code;
}

void clear_error() { t_last_error.clear(); }

int hip_fail(hipError_t e, const char* what) {
  (void)hipGetLastError();  // do not leave the error for an unrelated call
  std::string msg = std::string(what) + ": " + hipGetErrorString(e);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return fail(SS_ERR_OOM, msg);
  if (e == hipErrorNoDevice || e == hipErrorInvalidDevice) return fail(SS_ERR_NO_DEVICE, msg);
  return fail(SS_ERR_HIP, msg);
}

hipStream_t current_stream() { return t_stream; }

int64_t option(int opt) {
  switch (opt) {
    case SS_OPT_FORCE_ALGO: return g_force_algo.load();
    case SS_OPT_BUCKET_BITS: return g_bucket_bits.load();
    case SS_OPT_BUCKET_CAP: return g_bucket_cap.load();
    case SS_OPT_BLOCK_SIZE: return g_block_size.load();
    case SS_OPT_GRID_BLOCKS: return g_grid_blocks.load();
    case SS_OPT_CHECK_POINTERS: return g_check_pointers.load();
    case SS_OPT_TARGETS_PER_LANE: return g_targets_per_lane.load();
    case SS_OPT_PLAN_TILES: return g_plan_tiles.load();
    case SS_OPT_PLAN_LEARNED: return g_plan_learned.load();
    case SS_OPT_LEARNED_STEPS: return g_learned_steps.load();
    case SS_OPT_PLAN_XCD: return g_plan_xcd.load();
    case SS_OPT_PAIR_JOINT: return g_pair_joint.load();
    case SS_OPT_CONVENTION: return g_convention.load();
    case SS_OPT_PLAN_ALGO: return g_plan_algo.load();
    case SS_OPT_PLAN_ORDER: return g_plan_order.load();
    default: return 0;
  }
}

int device_info(DeviceInfo* out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_dev_cache.find(dev);
    if (it != g_dev_cache.end()) {
      *out = it->second;
      return SS_OK;
    }
  }
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  DeviceInfo d;
  d.device = dev;
  d.num_cus = prop.multiProcessorCount;
  d.lds_per_block = prop.sharedMemPerBlock;
  snprintf(d.arch, sizeof(d.arch), "%s", prop.gcnArchName);
  d.arch_ok = std::string(prop.gcnArchName).rfind("gfx950", 0) == 0;
  std::lock_guard<std::mutex> lk(g_dev_mu);
  g_dev_cache[dev] = d;
  *out = d;
  return SS_OK;
}

int check_span(const void* p, int64_t count, size_t elem, size_t align, const char* name) {
  if (count < 0) return fail(SS_ERR_INVALID_ARG, std::string(name) + ": negative size");
  if (count == 0) return SS_OK;
  if (p == nullptr) return fail(SS_ERR_INVALID_ARG, std::string(name) + ": null pointer");
  if (reinterpret_cast<uintptr_t>(p) % align != 0)
    return fail(SS_ERR_INVALID_ARG, std::string(name) + ": misaligned pointer");
  if ((uint64_t)count > (uint64_t)INT64_MAX / elem)
    return fail(SS_ERR_INVALID_ARG, std::string(name) + ": size overflow");
  return SS_OK;
}

int check_device_ptr(const void* p, const char* name) {
  if (p == nullptr || !g_check_pointers.load()) return SS_OK;
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(SS_ERR_NOT_DEVICE_PTR, std::string(name) + ": not a device pointer");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(SS_ERR_NOT_DEVICE_PTR, std::string(name) + ": not device memory");
  return SS_OK;
}

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  if (!a || !b || abytes == 0 || bbytes == 0) return false;
  uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
  return a0 < b0 + bbytes && b0 < a0 + abytes;
}

int blocks_per_cu(const void* kernel, int threads, size_t lds) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  auto key = std::make_tuple(kernel, threads, lds, dev);
  {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_occ_cache.find(key);
    if (it != g_occ_cache.end()) return it->second;
  }
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, threads, lds) != hipSuccess) {
    (void)hipGetLastError();
    blocks = 1;
  }
  if (blocks < 1) blocks = 1;
  std::lock_guard<std::mutex> lk(g_dev_mu);
  g_occ_cache[key] = blocks;
  return blocks;
}

namespace {
std::atomic<int> g_log{0};
}  // namespace

bool log_enabled() { return g_log.load(std::memory_order_relaxed) > 0; }

void log_line(const char* fmt, ...) {
  if (!log_enabled()) return;
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "[ss] %s\n", buf);
}

}  // namespace ss

extern "C" int ss_set_option(int opt, int64_t v);

namespace ss {
namespace {

// Options from the environment, applied once when the library is loaded:
// SS_<NAME>=<value> for the option SS_OPT_<NAME>, an integer or (for the
// two algorithm options) an algorithm name.  Values the option refuses are
// reported on stderr and ignored.
struct EnvOption {
  const char* name;
  int opt;
  bool algo;
};
constexpr EnvOption kEnvOptions[] = {
    {"SS_FORCE_ALGO", SS_OPT_FORCE_ALGO, true},
    {"SS_BUCKET_BITS", SS_OPT_BUCKET_BITS, false},
    {"SS_BUCKET_CAP", SS_OPT_BUCKET_CAP, false},
    {"SS_BLOCK_SIZE", SS_OPT_BLOCK_SIZE, false},
    {"SS_GRID_BLOCKS", SS_OPT_GRID_BLOCKS, false},
    {"SS_CHECK_POINTERS", SS_OPT_CHECK_POINTERS, false},
    {"SS_TARGETS_PER_LANE", SS_OPT_TARGETS_PER_LANE, false},
    {"SS_PLAN_TILES", SS_OPT_PLAN_TILES, false},
    {"SS_PLAN_LEARNED", SS_OPT_PLAN_LEARNED, false},
    {"SS_LEARNED_STEPS", SS_OPT_LEARNED_STEPS, false},
    {"SS_PLAN_XCD", SS_OPT_PLAN_XCD, false},
    {"SS_PAIR_JOINT", SS_OPT_PAIR_JOINT, false},
    {"SS_CONVENTION", SS_OPT_CONVENTION, false},
    {"SS_PLAN_ALGO", SS_OPT_PLAN_ALGO, true},
    {"SS_PLAN_ORDER", SS_OPT_PLAN_ORDER, false},
};

constexpr const char* kAlgoNames[] = {"auto",          "binary",  "ballot",  "exphash",
                                      "binary_global", "learned", "loghash", "skiplist"};

// Parses a whole decimal integer (or, if algo, an algorithm name).
bool parse_value(const char* text, bool algo, int64_t* v) {
  if (algo)
    for (int i = 0; i < (int)(sizeof(kAlgoNames) / sizeof(kAlgoNames[0])); ++i)
      if (std::strcmp(text, kAlgoNames[i]) == 0) {
        *v = i;
        return true;
      }
  char* end = nullptr;
  const long long x = std::strtoll(text, &end, 10);
  if (end == text || *end) return false;
  *v = x;
  return true;
}

struct EnvInit {
  EnvInit() {
    const char* lv = std::getenv("SS_LOG");
    int64_t level = 0;
    if (lv && *lv) {
      if (parse_value(lv, false, &level) && level >= 0)
        g_log = (int)std::min<int64_t>(level, 9);
      else
        std::fprintf(stderr, "[ss] ignoring SS_LOG=%s: expected a non-negative integer\n", lv);
    }
    for (const EnvOption& e : kEnvOptions) {
      const char* text = std::getenv(e.name);
      if (!text || !*text) continue;
      int64_t v = 0;
      if (!parse_value(text, e.algo, &v)) {
        std::fprintf(stderr, "[ss] ignoring %s=%s: not %s\n", e.name, text,
                     e.algo ? "an integer or algorithm name" : "an integer");
        continue;
      }
      if (ss_set_option(e.opt, v) != SS_OK) {
        std::fprintf(stderr, "[ss] ignoring %s=%s: %s\n", e.name, text, t_last_error.c_str());
        t_last_error.clear();
        continue;
      }
      log_line("option %s = %lld (environment)", e.name, (long long)v);
    }
  }
};
const EnvInit g_env_init;

}  // namespace
}  // namespace ss

extern "C" {

const char* ss_last_error(void) { return ss::t_last_error.c_str(); }

int ss_version(void) { return 100; }

int ss_set_stream(void* hip_stream) {
  ss::t_stream = reinterpret_cast<hipStream_t>(hip_stream);
  return SS_OK;
}

int ss_set_option(int opt, int64_t v) {
  switch (opt) {
    case SS_OPT_FORCE_ALGO:
      if (v < SS_ALGO_AUTO || v > SS_ALGO_SKIPLIST || v == SS_ALGO_LEARNED)
        return ss::fail(SS_ERR_INVALID_ARG,
                        "SS_OPT_FORCE_ALGO: unknown single-table algorithm");
      ss::g_force_algo = v;
      return SS_OK;
    case SS_OPT_BUCKET_BITS:
      if (v < -1 || v > 20)
        return ss::fail(SS_ERR_INVALID_ARG, "SS_OPT_BUCKET_BITS: expected -1..20");
      ss::g_bucket_bits = v;
      return SS_OK;
    case SS_OPT_BUCKET_CAP:
      if (v < 0 || v > 65535)
        return ss::fail(SS_ERR_INVALID_ARG, "SS_OPT_BUCKET_CAP: expected 0..65535");
      ss::g_bucket_cap = v;
      return SS_OK;
    case SS_OPT_BLOCK_SIZE:
      if (v != 0 && v != 256 && v != 512 && v != 1024)
        return ss::fail(SS_ERR_INVALID_ARG, "SS_OPT_BLOCK_SIZE: expected 0, 256, 512 or 1024");
      ss::g_block_size = v;
      return SS_OK;
    case SS_OPT_GRID_BLOCKS:
      if (v < 0 || v > (1 << 20))
        return ss::fail(SS_ERR_INVALID_ARG, "SS_OPT_GRID_BLOCKS: expected 0..2^20");
      ss::g_grid_blocks = v;
      return SS_OK;
    case SS_OPT_CHECK_POINTERS:
      if (v != 0 && v != 1) return ss::fail(SS_ERR_INVALID_ARG, "SS_OPT_CHECK_POINTERS: 0 or 1");
      ss::g_check_pointers = v;
      return SS_OK;
    case SS_OPT_TARGETS_PER_LANE:
      if (v != 0 && v != 4 && v != 8)
        return ss::fail(SS_ERR_INVALID_ARG, "SS_OPT_TARGETS_PER_LANE: expected 0, 4 or 8");
      ss::g_targets_per_lane = v;
      return SS_OK;
    case SS_OPT_PLAN_TILES:
      if (v < 0 || v > 4096)
        return ss::fail(SS_ERR_INVALID_ARG, "SS_OPT_PLAN_TILES: expected 0..4096");
      ss::g_plan_tiles = v;
      return SS_OK;
    case SS_OPT_PLAN_LEARNED:
      if (v < 0 || v > 2) return ss::fail(SS_ERR_INVALID_ARG, "SS_OPT_PLAN_LEARNED: 0, 1 or 2");
      ss::g_plan_learned = v;
      return SS_OK;
    case SS_OPT_LEARNED_STEPS:
      if (v < 0 || v > 1000000)
        return ss::fail(SS_ERR_INVALID_ARG, "SS_OPT_LEARNED_STEPS: expected 0..1e6");
      ss::g_learned_steps = v;
      return SS_OK;
    case SS_OPT_PLAN_XCD:
      if (v < 0 || v > (int64_t(1) << 24))
        return ss::fail(SS_ERR_INVALID_ARG, "SS_OPT_PLAN_XCD: expected 0..2^24");
      ss::g_plan_xcd = v;
      return SS_OK;
    case SS_OPT_PAIR_JOINT:
      if (v != 0 && v != 1) return ss::fail(SS_ERR_INVALID_ARG, "SS_OPT_PAIR_JOINT: 0 or 1");
      ss::g_pair_joint = v;
      return SS_OK;
    case SS_OPT_CONVENTION:
      if (v != 0 && v != 1) return ss::fail(SS_ERR_INVALID_ARG, "SS_OPT_CONVENTION: 0 or 1");
      ss::g_convention = v;
      return SS_OK;
    case SS_OPT_PLAN_ALGO:
      if (v != SS_ALGO_AUTO && v != SS_ALGO_BINARY && v != SS_ALGO_EXPHASH &&
          v != SS_ALGO_BALLOT)
        return ss::fail(SS_ERR_INVALID_ARG,
                        "SS_OPT_PLAN_ALGO: SS_ALGO_AUTO, SS_ALGO_BINARY, SS_ALGO_EXPHASH or "
                        "SS_ALGO_BALLOT");
      ss::g_plan_algo = v;
      return SS_OK;
    case SS_OPT_PLAN_ORDER:
      if (v < 0 || v > 2) return ss::fail(SS_ERR_INVALID_ARG, "SS_OPT_PLAN_ORDER: 0, 1 or 2");
      ss::g_plan_order = v;
      return SS_OK;
    default:
      return ss::fail(SS_ERR_INVALID_ARG, "unknown option");
  }
}

int ss_debug_violations(int64_t* count) {
  ss::clear_error();
  if (!count) return ss::fail(SS_ERR_INVALID_ARG, "count is null");
  *count = 0;
  int (*readers[])(unsigned long long*) = {ss::violations_single, ss::violations_plan,
                                           ss::violations_learned, ss::violations_noalloc};
  for (auto rd : readers) {
    unsigned long long v = 0;
    const int rc = rd(&v);
    if (rc == SS_ERR_UNSUPPORTED) return ss::fail(rc, "not a device-checked build");
    if (rc != SS_OK) return ss::fail(rc, "reading the bounds-check counters");
    *count += (int64_t)v;
  }
  return SS_OK;
}

int ss_debug_selftest(void) {
  ss::clear_error();
  return ss::checks_selftest();
}

int ss_get_option(int opt, int64_t* value_out) {
  if (!value_out) return ss::fail(SS_ERR_INVALID_ARG, "value_out is null");
  switch (opt) {
    case SS_OPT_FORCE_ALGO:
    case SS_OPT_BUCKET_BITS:
    case SS_OPT_BUCKET_CAP:
    case SS_OPT_BLOCK_SIZE:
    case SS_OPT_GRID_BLOCKS:
    case SS_OPT_CHECK_POINTERS:
    case SS_OPT_TARGETS_PER_LANE:
    case SS_OPT_PLAN_TILES:
    case SS_OPT_PLAN_LEARNED:
    case SS_OPT_LEARNED_STEPS:
    case SS_OPT_PLAN_XCD:
    case SS_OPT_PAIR_JOINT:
    case SS_OPT_CONVENTION:
    case SS_OPT_PLAN_ALGO:
    case SS_OPT_PLAN_ORDER:
      *value_out = ss::option(opt);
      return SS_OK;
    default:
      return ss::fail(SS_ERR_INVALID_ARG, "unknown option");
  }
}

}  // extern "C"
