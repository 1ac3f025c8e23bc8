// hk_runtime.hip -- error text and reduction scratch of libhk.
#include <map>
#include <mutex>
#include <utility>

#include "hk_internal.hpp"

namespace hk {

static thread_local std::string g_error;

void set_error_text(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
}

const char* error_text() { return g_error.c_str(); }

int reduce_scratch(hipStream_t s, size_t bytes, ReduceScratch** out) {
  static std::mutex mu;
  static std::map<std::pair<int, hipStream_t>, ReduceScratch> pool;
  int dev = 0;
  HK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  ReduceScratch& r = pool[{dev, s}];
  if (r.bytes < bytes) {
    if (r.partials) {
      HK_HIP(hipStreamSynchronize(s));
      HK_HIP(hipFree(r.partials));
      r.partials = nullptr;
      r.bytes = 0;
    }
    size_t want = bytes < (1u << 16) ? (1u << 16) : bytes;
    if (hipMalloc(&r.partials, want) != hipSuccess)
      HK_FAIL(HK_ENOMEM, "reduction scratch: hipMalloc(%zu) failed", want);
    r.bytes = want;
  }
  *out = &r;
  return HK_OK;
}

}  // namespace hk

extern "C" const char* hk_last_error(void) { return hk::error_text(); }
